// The constant-potential MD loop around the electrostatics (appendix:
// velocity Verlet with a 2 fs step, Nose-Hoover thermostat on the
// electrolyte, one per sub-cell of the doubled cell, rigid three-site cations
// by SHAKE, Lennard-Jones within 1.6 nm, electrode charges re-solved every
// fifth step).
//
// Per step (positions x, velocities v, forces f known):
//   thermostat half step; v += dt/2 f/m; x' = x + dt v; SHAKE; v = (x' - x)/dt
//   f = f_LJ(x') + f_Coulomb(x')            (charges re-solved every k-th step)
//   v += dt/2 f/m; RATTLE; thermostat half step
// thermostat half step per group (Q = N_f k T tau^2, K2 = sum m v^2):
//   xi += dt/4 (K2 - N_f kT)/Q; eta += dt/2 xi; v *= exp(-xi dt/2);
//   K2 *= exp(-xi dt); xi += dt/4 (K2 - N_f kT)/Q
//
// SHAKE and RATTLE solve a molecule's three constraints together (Newton
// steps on the multipliers; a 3 x 3 linear solve for the velocities): the
// same constrained positions and velocities as one constraint at a time.
//
// k_lj: one workgroup per site over all sites and graphene atoms (minimum
// image, pairs of one molecule excluded, energy shifted to zero at the
// cutoff; Lorentz-Berthelot mixing from the stored square roots of epsilon).  k_md_integrate: one 1024-thread workgroup for the whole
// electrolyte (a thread per molecule, its sites in registers), since the
// thermostat needs the groups' kinetic energies between the two halves of
// the update; one launch joins the end of one step and the start of the
// next.
#include "common.h"

namespace cpm {

constexpr double KB_KJ = 0.0083144626;      // kJ/mol/K
constexpr double EV_KJ = 96.48533212;       // kJ/mol per eV

__global__ __launch_bounds__(256) void k_lj(MDArgs a) {
  // one workgroup per site: its 256 threads share the partners, so that a
  // site's sum is spread over four wavefronts and every CU holds many sites
  __shared__ double red[4][4];
  const int i = blockIdx.x;
  const double xi = a.x[i], yi = a.x[a.n_site + i], zi = a.x[2 * a.n_site + i];
  const double si = a.sigma[i], qi = a.sqeps[i];
  const int mi = a.mol_of[i];
  const double rc2 = a.lj_cut * a.lj_cut;
  double fx = 0.0, fy = 0.0, fz = 0.0, u = 0.0, uw = 0.5;   // a site-site pair's energy is shared by its sites
  auto pair = [&](double dx, double dy, double dz, double sig, double eps) {
    dx -= a.box[0] * rint(dx * a.inv_box[0]);
    dy -= a.box[1] * rint(dy * a.inv_box[1]);
    dz -= a.box[2] * rint(dz * a.inv_box[2]);
    const double r2 = dx * dx + dy * dy + dz * dz;
    if (r2 < rc2 && r2 > 0.0) {
      const double ir2 = 1.0 / r2;
      const double t = sig * sig * ir2, s6 = t * t * t;
      const double tc = sig * sig / rc2, c6 = tc * tc * tc;
      const double fr = 24.0 * eps * (2.0 * s6 * s6 - s6) * ir2;
      fx += fr * dx; fy += fr * dy; fz += fr * dz;
      u += uw * (4.0 * eps * (s6 * s6 - s6) - 4.0 * eps * (c6 * c6 - c6));
    }
  };
  for (int j = threadIdx.x; j < a.n_site; j += blockDim.x) {
    if (a.mol_of[j] == mi) continue;
    pair(xi - a.x[j], yi - a.x[a.n_site + j], zi - a.x[2 * a.n_site + j], 0.5 * (si + a.sigma[j]), qi * a.sqeps[j]);
  }
  uw = 1.0;
  const double sc = 0.5 * (si + a.carbon_sigma), ec = qi * a.carbon_sqeps;
  for (int j = threadIdx.x; j < a.n_lj_elec; j += blockDim.x)
    pair(xi - a.cx[j], yi - a.cx[a.n_lj_elec + j], zi - a.cx[2 * a.n_lj_elec + j], sc, ec);
  fx = wave_sum(fx); fy = wave_sum(fy); fz = wave_sum(fz); u = wave_sum(u);
  const int w = threadIdx.x / WAVE;
  if ((threadIdx.x & (WAVE - 1)) == 0) { red[w][0] = fx; red[w][1] = fy; red[w][2] = fz; red[w][3] = u; }
  __syncthreads();
  if (threadIdx.x < 4) {
    const double t = (red[0][threadIdx.x] + red[1][threadIdx.x]) + (red[2][threadIdx.x] + red[3][threadIdx.x]);
    if (threadIdx.x < 3) a.f_lj[threadIdx.x * a.n_site + i] = t;
    else a.u_lj[i] = t;
  }
}

// minimum-image difference of two sites' coordinates along axis d
__device__ __forceinline__ double md_diff(const MDArgs& a, double p, double q, int d) {
  const double r = p - q;
  return r - a.box[d] * rint(r * a.inv_box[d]);
}

// Constraint solves of one rigid three-site molecule, in registers.  The
// three constraints c = (0,1), (0,2), (1,2) are taken together: site s moves
// by g_c sigma_sc v_c / m_s for each c (sigma = +1 on the constraint's first
// site, -1 on its second, v_c the constraint's vector), so the bond vector
// of constraint a changes by sum_b K_ab g_b v_b with
// K_ab = sigma(i_a, b) / m(i_a) - sigma(j_a, b) / m(j_a).

__device__ __forceinline__ double md_kab(int a, int b, const double m[3]) {
  const int ci[3] = {0, 0, 1}, cj[3] = {1, 2, 2};
  auto sig = [&](int s, int c) { return s == ci[c] ? 1.0 : (s == cj[c] ? -1.0 : 0.0); };
  return sig(ci[a], b) / m[ci[a]] - sig(cj[a], b) / m[cj[a]];
}

// x = M^-1 y for a 3 x 3 matrix (Cramer's rule; M is well conditioned here:
// the three bond vectors of the triangle are independent)
__device__ __forceinline__ void solve3(const double M[3][3], const double y[3], double x[3]) {
  const double c00 = M[1][1] * M[2][2] - M[1][2] * M[2][1];
  const double c01 = M[1][2] * M[2][0] - M[1][0] * M[2][2];
  const double c02 = M[1][0] * M[2][1] - M[1][1] * M[2][0];
  const double det = M[0][0] * c00 + M[0][1] * c01 + M[0][2] * c02;
  const double id = 1.0 / det;
  x[0] = id * (y[0] * c00 + y[1] * (M[0][2] * M[2][1] - M[0][1] * M[2][2]) + y[2] * (M[0][1] * M[1][2] - M[0][2] * M[1][1]));
  x[1] = id * (y[0] * c01 + y[1] * (M[0][0] * M[2][2] - M[0][2] * M[2][0]) + y[2] * (M[0][2] * M[1][0] - M[0][0] * M[1][2]));
  x[2] = id * (y[0] * c02 + y[1] * (M[0][1] * M[2][0] - M[0][0] * M[2][1]) + y[2] * (M[0][0] * M[1][1] - M[0][1] * M[1][0]));
}

// SHAKE: move the new positions p along the old bond vectors (from o) until
// |p_i - p_j| = d for all three constraints, by Newton steps on the three
// multipliers together (the same fixed point as one constraint at a time,
// reached in a few steps)
__device__ void shake3(const MDArgs& a, double p[3][3], const double o[3][3], const double m[3]) {
  const int ci[3] = {0, 0, 1}, cj[3] = {1, 2, 2};
  const double d[3] = {a.bond, a.bond, a.bond * 1.7320508075688772};
  double ro[3][3];                                     // [constraint][axis], fixed during the solve
  _Pragma("unroll") for (int c = 0; c < 3; ++c)
    _Pragma("unroll") for (int k = 0; k < 3; ++k) ro[c][k] = md_diff(a, o[k][ci[c]], o[k][cj[c]], k);
  double K[3][3];
  _Pragma("unroll") for (int x = 0; x < 3; ++x)
    _Pragma("unroll") for (int y = 0; y < 3; ++y) K[x][y] = md_kab(x, y, m);
  for (int it = 0; it < MD_MAX_ITER; ++it) {
    double r[3][3], f[3];
    bool done = true;
    _Pragma("unroll") for (int c = 0; c < 3; ++c) {
      _Pragma("unroll") for (int k = 0; k < 3; ++k) r[c][k] = md_diff(a, p[k][ci[c]], p[k][cj[c]], k);
      f[c] = r[c][0] * r[c][0] + r[c][1] * r[c][1] + r[c][2] * r[c][2] - d[c] * d[c];
      done = done && fabs(f[c]) <= MD_TOL * d[c] * d[c];
    }
    if (done) return;
    double J[3][3], g[3];
    _Pragma("unroll") for (int x = 0; x < 3; ++x)
      _Pragma("unroll") for (int y = 0; y < 3; ++y)
        J[x][y] = 2.0 * K[x][y] * (r[x][0] * ro[y][0] + r[x][1] * ro[y][1] + r[x][2] * ro[y][2]);
    solve3(J, f, g);
    _Pragma("unroll") for (int c = 0; c < 3; ++c)
      _Pragma("unroll") for (int k = 0; k < 3; ++k) {
        p[k][ci[c]] -= g[c] * ro[c][k] / m[ci[c]];
        p[k][cj[c]] += g[c] * ro[c][k] / m[cj[c]];
      }
  }
}

// RATTLE: remove the velocity components along the three constraints, a
// linear 3 x 3 system for the multipliers solved at once
__device__ void rattle3(const MDArgs& a, double v[3][3], const double p[3][3], const double m[3]) {
  const int ci[3] = {0, 0, 1}, cj[3] = {1, 2, 2};
  double r[3][3], vr[3];
  _Pragma("unroll") for (int c = 0; c < 3; ++c) {
    _Pragma("unroll") for (int k = 0; k < 3; ++k) r[c][k] = md_diff(a, p[k][ci[c]], p[k][cj[c]], k);
    vr[c] = (v[0][ci[c]] - v[0][cj[c]]) * r[c][0] + (v[1][ci[c]] - v[1][cj[c]]) * r[c][1] +
            (v[2][ci[c]] - v[2][cj[c]]) * r[c][2];
  }
  double M[3][3], kk[3];
  _Pragma("unroll") for (int x = 0; x < 3; ++x)
    _Pragma("unroll") for (int y = 0; y < 3; ++y)
      M[x][y] = md_kab(x, y, m) * (r[x][0] * r[y][0] + r[x][1] * r[y][1] + r[x][2] * r[y][2]);
  solve3(M, vr, kk);
  _Pragma("unroll") for (int c = 0; c < 3; ++c)
    _Pragma("unroll") for (int k = 0; k < 3; ++k) {
      v[k][ci[c]] -= kk[c] * r[c][k] / m[ci[c]];
      v[k][cj[c]] += kk[c] * r[c][k] / m[cj[c]];
    }
}

// per-group totals of a per-thread partial (every thread gets the totals)
__device__ void group_sums(int n_groups, const double* part, double* out, double* red) {
  const int nw = blockDim.x / WAVE, w = threadIdx.x / WAVE;
  for (int g = 0; g < n_groups; ++g) {
    const double s = wave_sum(part[g]);
    if ((threadIdx.x & (WAVE - 1)) == 0) red[g * nw + w] = s;
  }
  __syncthreads();
  for (int g = 0; g < n_groups; ++g) {
    double t = 0.0;
    for (int k = 0; k < nw; ++k) t += red[g * nw + k];
    out[g] = t;
  }
  __syncthreads();
}

// one molecule's sites (up to 3) between global memory and registers
struct MolRegs {
  int s0, n, g;
  double p[3][3], v[3][3], m[3];
};

__device__ __forceinline__ void mol_load(const MDArgs& a, int mol, MolRegs& r) {
  r.s0 = a.mol_start[mol]; r.n = a.mol_size[mol]; r.g = a.mol_group[mol];
  _Pragma("unroll") for (int s = 0; s < 3; ++s) if (s < r.n) {
    r.m[s] = a.mass[r.s0 + s];
    _Pragma("unroll") for (int k = 0; k < 3; ++k) {
      r.p[k][s] = a.x[k * a.n_site + r.s0 + s];
      r.v[k][s] = a.v[k * a.n_site + r.s0 + s];
    }
  }
}

__device__ __forceinline__ double mol_force(const MDArgs& a, const MolRegs& r, int k, int s) {
  const size_t o = (size_t)k * a.n_site + r.s0 + s;
  return a.f_lj[o] + EV_KJ * a.f_c[o];
}

// one thermostat half step: the groups' sum m v^2 from the velocities in
// memory, xi and eta advanced identically in every thread, velocities scaled
__device__ void thermostat_half(const MDArgs& a, double* xi, double* eta, double* red) {
  double part[MD_MAX_GROUPS] = {};
  for (int mol = threadIdx.x; mol < a.n_mol; mol += blockDim.x) {
    const int s0 = a.mol_start[mol], n = a.mol_size[mol], g = a.mol_group[mol];
    for (int s = 0; s < n; ++s) {
      double vv = 0.0;
      _Pragma("unroll") for (int k = 0; k < 3; ++k) { const double c = a.v[k * a.n_site + s0 + s]; vv += c * c; }
      part[g] += a.mass[s0 + s] * vv;
    }
  }
  double k2[MD_MAX_GROUPS], scale[MD_MAX_GROUPS];
  group_sums(a.n_groups, part, k2, red);
  for (int g = 0; g < a.n_groups; ++g) {
    xi[g] += 0.25 * a.dt * (k2[g] - a.nf[g] * a.kt) / a.Q[g];
    eta[g] += 0.5 * a.dt * xi[g];
    scale[g] = exp(-0.5 * a.dt * xi[g]);
    k2[g] *= scale[g] * scale[g];
    xi[g] += 0.25 * a.dt * (k2[g] - a.nf[g] * a.kt) / a.Q[g];
  }
  for (int mol = threadIdx.x; mol < a.n_mol; mol += blockDim.x) {
    const int s0 = a.mol_start[mol], n = a.mol_size[mol], g = a.mol_group[mol];
    for (int s = 0; s < n; ++s)
      _Pragma("unroll") for (int k = 0; k < 3; ++k) a.v[k * a.n_site + s0 + s] *= scale[g];
  }
}

// mode bit 4: RATTLE of the initial velocities; bit 1: end of a step (kick
// with the new forces, RATTLE, thermostat half step, record rec_step); bit 2:
// start of a step (thermostat half step, kick, drift, SHAKE).  Every thread
// handles molecules threadIdx.x + k blockDim.x in every phase, so it only
// re-reads what it wrote itself; the group sums go through LDS.
__global__ __launch_bounds__(MD_THREADS) void k_md_integrate(MDArgs a, int mode, int rec_step) {
  __shared__ double red[MD_MAX_GROUPS * (MD_THREADS / WAVE)];
  double xi[MD_MAX_GROUPS], eta[MD_MAX_GROUPS];
  for (int g = 0; g < a.n_groups; ++g) { xi[g] = a.xi[g]; eta[g] = a.eta[g]; }
  if (mode & 4) {
    for (int mol = threadIdx.x; mol < a.n_mol; mol += blockDim.x) {
      MolRegs r;
      mol_load(a, mol, r);
      if (r.n != 3) continue;
      rattle3(a, r.v, r.p, r.m);
      _Pragma("unroll") for (int s = 0; s < 3; ++s)
        _Pragma("unroll") for (int k = 0; k < 3; ++k) a.v[k * a.n_site + r.s0 + s] = r.v[k][s];
    }
  }
  if (mode & 1) {
    for (int mol = threadIdx.x; mol < a.n_mol; mol += blockDim.x) {
      MolRegs r;
      mol_load(a, mol, r);
      _Pragma("unroll") for (int s = 0; s < 3; ++s) if (s < r.n)
        _Pragma("unroll") for (int k = 0; k < 3; ++k) r.v[k][s] += 0.5 * a.dt * mol_force(a, r, k, s) / r.m[s];
      if (r.n == 3) rattle3(a, r.v, r.p, r.m);
      _Pragma("unroll") for (int s = 0; s < 3; ++s) if (s < r.n)
        _Pragma("unroll") for (int k = 0; k < 3; ++k) a.v[k * a.n_site + r.s0 + s] = r.v[k][s];
    }
    if (a.thermostat) thermostat_half(a, xi, eta, red);
    if (a.thermo_out) {
      double part[MD_MAX_GROUPS] = {}, tot[MD_MAX_GROUPS];
      for (int mol = threadIdx.x; mol < a.n_mol; mol += blockDim.x) {
        MolRegs r;
        mol_load(a, mol, r);
        _Pragma("unroll") for (int s = 0; s < 3; ++s) if (s < r.n)
          part[0] += 0.5 * r.m[s] * (r.v[0][s] * r.v[0][s] + r.v[1][s] * r.v[1][s] + r.v[2][s] * r.v[2][s]);
      }
      group_sums(1, part, tot, red);
      const double ke = tot[0];
      part[0] = 0.0;
      for (int i = threadIdx.x; i < a.n_site; i += blockDim.x) part[0] += a.u_lj[i];
      group_sums(1, part, tot, red);
      if (threadIdx.x == 0) {
        double th = 0.0;
        for (int g = 0; g < a.n_groups; ++g) th += 0.5 * a.Q[g] * xi[g] * xi[g] + a.nf[g] * a.kt * eta[g];
        double* o = a.thermo_out + (size_t)rec_step * MD_THERMO;
        o[0] = ke;
        o[1] = tot[0];
        o[2] = EV_KJ * a.energy[1];
        o[3] = th;
      }
    }
  }
  if (mode & 2) {
    if (a.thermostat) thermostat_half(a, xi, eta, red);
    for (int mol = threadIdx.x; mol < a.n_mol; mol += blockDim.x) {
      MolRegs r;
      mol_load(a, mol, r);
      double o[3][3];
      _Pragma("unroll") for (int s = 0; s < 3; ++s) if (s < r.n)
        _Pragma("unroll") for (int k = 0; k < 3; ++k) {
          o[k][s] = r.p[k][s];
          r.v[k][s] += 0.5 * a.dt * mol_force(a, r, k, s) / r.m[s];
          r.p[k][s] += a.dt * r.v[k][s];
        }
      if (r.n == 3) shake3(a, r.p, o, r.m);
      _Pragma("unroll") for (int s = 0; s < 3; ++s) if (s < r.n)
        _Pragma("unroll") for (int k = 0; k < 3; ++k) {
          a.x[k * a.n_site + r.s0 + s] = r.p[k][s];
          a.v[k * a.n_site + r.s0 + s] = (r.p[k][s] - o[k][s]) / a.dt;
        }
    }
  }
  if (threadIdx.x == 0)
    for (int g = 0; g < a.n_groups; ++g) { a.xi[g] = xi[g]; a.eta[g] = eta[g]; }
}

void launch_lj(hipStream_t s, const MDArgs& a) {
  hipLaunchKernelGGL(k_lj, dim3(a.n_site), dim3(256), 0, s, a);
}
void launch_md_integrate(hipStream_t s, const MDArgs& a, int mode, int rec_step) {
  hipLaunchKernelGGL(k_md_integrate, dim3(1), dim3(MD_THREADS), 0, s, a, mode, rec_step);
}

}  // namespace cpm
