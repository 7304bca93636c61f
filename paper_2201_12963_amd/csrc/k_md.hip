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
// k_lj: one workgroup per site over the sites and graphene atoms of the z
// layers within the cutoff (the layers of the electrostatic cell grid, whose
// binning of the same positions runs first; minimum image, pairs of one
// molecule excluded, energy shifted to zero at the cutoff; Lorentz-Berthelot
// mixing from the stored square roots of epsilon).  k_md_end / k_md_start:
// the update, a thread per molecule with its sites in registers; one pair of
// launches joins the end of one step and the start of the next.
#include "common.h"
#include "lj.h"

namespace cpm {

constexpr double KB_KJ = 0.0083144626;      // kJ/mol/K
constexpr double EV_KJ = 96.48533212;       // kJ/mol per eV

template <int NW>
__global__ __launch_bounds__(NW * WAVE) void k_lj(MDArgs a) {
  lj_site<NW>(a, blockIdx.x);
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

// the value of a per-group register array at a run-time group index
__device__ __forceinline__ double group_pick(const double* v, int g) {
  double r = v[0];
  _Pragma("unroll") for (int k = 1; k < MD_MAX_GROUPS; ++k) if (g == k) r = v[k];
  return r;
}

// one Nose-Hoover half step of group g from its sum k2 = sum m v^2 (k2 is
// left at the scaled velocities' value); returns the velocity scale
__device__ __forceinline__ double nh_half(const MDArgs& a, int g, double& k2, double& xi, double& eta) {
  xi += 0.25 * a.dt * (k2 - a.nf[g] * a.kt) / a.Q[g];
  eta += 0.5 * a.dt * xi;
  const double scale = exp(-0.5 * a.dt * xi);
  k2 *= scale * scale;
  xi += 0.25 * a.dt * (k2 - a.nf[g] * a.kt) / a.Q[g];
  return scale;
}

// mode bit 4: RATTLE of the initial velocities; bit 1: end of a step (kick
// with the new forces, RATTLE, thermostat half step, record rec_step); bit 2:
// start of a step (thermostat half step, kick, drift, SHAKE).  The thermostat
// needs every group's sum of m v^2 between the kick and the scaling, so an
// update is two launches of one wavefront per 64 molecules (a thread per
// molecule): k_md_end does the end-of-step kick and RATTLE and leaves one
// partial sum per workgroup; k_md_start totals the partials (the same order
// in every workgroup, so every workgroup holds the same thermostat state),
// scales, and does the start-of-step kick, drift and SHAKE.  A scaling
// multiplies sum m v^2 by the square of the scale, so both half steps of a
// joined end and start come from the one sum.
__global__ __launch_bounds__(WAVE) void k_md_end(MDArgs a, int mode) {
  const int mol = blockIdx.x * WAVE + threadIdx.x;
  // the Lennard-Jones energies first (independent of the molecule's loads)
  double ul = 0.0;
  if ((mode & 1) && a.thermo_out)
    for (int i = mol; i < a.n_site; i += gridDim.x * WAVE) ul += a.u_lj[i];
  double part[MD_MAX_GROUPS] = {};
  if (mol < a.n_mol) {
    MolRegs r;
    mol_load(a, mol, r);
    if (mode & 1)
      _Pragma("unroll") for (int s = 0; s < 3; ++s) if (s < r.n)
        _Pragma("unroll") for (int k = 0; k < 3; ++k) r.v[k][s] += 0.5 * a.dt * mol_force(a, r, k, s) / r.m[s];
    if ((mode & 5) && r.n == 3) rattle3(a, r.v, r.p, r.m);
    if (mode & 5)
      _Pragma("unroll") for (int s = 0; s < 3; ++s) if (s < r.n)
        _Pragma("unroll") for (int k = 0; k < 3; ++k) a.v[k * a.n_site + r.s0 + s] = r.v[k][s];
    double mv2 = 0.0;
    _Pragma("unroll") for (int s = 0; s < 3; ++s) if (s < r.n)
      mv2 += r.m[s] * (r.v[0][s] * r.v[0][s] + r.v[1][s] * r.v[1][s] + r.v[2][s] * r.v[2][s]);
    _Pragma("unroll") for (int g = 0; g < MD_MAX_GROUPS; ++g) if (g == r.g) part[g] = mv2;
  }
  _Pragma("unroll") for (int g = 0; g < MD_MAX_GROUPS; ++g) part[g] = wave_sum(part[g]);
  ul = wave_sum(ul);
  if (threadIdx.x == 0) {
    double* o = a.md_part + (size_t)blockIdx.x * MD_PART;
    _Pragma("unroll") for (int g = 0; g < MD_MAX_GROUPS; ++g) o[g] = part[g];
    o[MD_MAX_GROUPS] = ul;
    // the thermostat state that k_md_start reads (it writes a.xi, a.eta)
    if (blockIdx.x == 0)
      _Pragma("unroll") for (int g = 0; g < MD_MAX_GROUPS; ++g) {
        a.nh_in[g] = a.xi[g];
        a.nh_in[MD_MAX_GROUPS + g] = a.eta[g];
      }
  }
}

__global__ __launch_bounds__(WAVE) void k_md_start(MDArgs a, int mode, int rec_step, int n_part) {
  // the molecule and its forces first: their loads do not wait for the
  // partial sums, so the two latencies overlap
  const int mol = blockIdx.x * WAVE + threadIdx.x;
  const bool live = mol < a.n_mol;
  MolRegs r;
  double fm[3][3];
  if (live) {
    mol_load(a, mol, r);
    if (mode & 2)
      _Pragma("unroll") for (int s = 0; s < 3; ++s) if (s < r.n)
        _Pragma("unroll") for (int k = 0; k < 3; ++k) fm[k][s] = mol_force(a, r, k, s);
  }
  double k2[MD_MAX_GROUPS] = {}, ul = 0.0;
  for (int b = threadIdx.x; b < n_part; b += WAVE) {
    const double* o = a.md_part + (size_t)b * MD_PART;
    _Pragma("unroll") for (int g = 0; g < MD_MAX_GROUPS; ++g) k2[g] += o[g];
    ul += o[MD_MAX_GROUPS];
  }
  _Pragma("unroll") for (int g = 0; g < MD_MAX_GROUPS; ++g) k2[g] = wave_sum(k2[g]);
  ul = wave_sum(ul);
  double xi[MD_MAX_GROUPS], eta[MD_MAX_GROUPS], s1[MD_MAX_GROUPS], s2[MD_MAX_GROUPS];
  _Pragma("unroll") for (int g = 0; g < MD_MAX_GROUPS; ++g) {
    xi[g] = a.nh_in[g]; eta[g] = a.nh_in[MD_MAX_GROUPS + g];
    s1[g] = 1.0; s2[g] = 1.0;
  }
  const bool nh = a.thermostat != 0;
  if (mode & 1) {
    if (nh)
      _Pragma("unroll") for (int g = 0; g < MD_MAX_GROUPS; ++g)
        if (g < a.n_groups) s1[g] = nh_half(a, g, k2[g], xi[g], eta[g]);
    if (a.thermo_out && blockIdx.x == 0 && threadIdx.x == 0) {
      double ke = 0.0, th = 0.0;
      for (int g = 0; g < a.n_groups; ++g) {
        ke += 0.5 * k2[g];
        th += 0.5 * a.Q[g] * xi[g] * xi[g] + a.nf[g] * a.kt * eta[g];
      }
      double* o = a.thermo_out + (size_t)rec_step * MD_THERMO;
      o[0] = ke;
      o[1] = ul;
      o[2] = EV_KJ * a.energy[1];
      o[3] = th;
    }
  }
  if ((mode & 2) && nh)
    _Pragma("unroll") for (int g = 0; g < MD_MAX_GROUPS; ++g)
      if (g < a.n_groups) s2[g] = nh_half(a, g, k2[g], xi[g], eta[g]);
  if (live) {
    const double c1 = group_pick(s1, r.g), c2 = group_pick(s2, r.g);
    _Pragma("unroll") for (int s = 0; s < 3; ++s) if (s < r.n)
      _Pragma("unroll") for (int k = 0; k < 3; ++k) {
        if ((mode & 1) && nh) r.v[k][s] *= c1;
        if ((mode & 2) && nh) r.v[k][s] *= c2;
      }
    if (mode & 2) {
      double o[3][3];
      _Pragma("unroll") for (int s = 0; s < 3; ++s) if (s < r.n)
        _Pragma("unroll") for (int k = 0; k < 3; ++k) {
          o[k][s] = r.p[k][s];
          r.v[k][s] += 0.5 * a.dt * fm[k][s] / r.m[s];
          r.p[k][s] += a.dt * r.v[k][s];
        }
      if (r.n == 3) shake3(a, r.p, o, r.m);
      _Pragma("unroll") for (int s = 0; s < 3; ++s) if (s < r.n)
        _Pragma("unroll") for (int k = 0; k < 3; ++k) {
          a.x[k * a.n_site + r.s0 + s] = r.p[k][s];
          a.v[k * a.n_site + r.s0 + s] = (r.p[k][s] - o[k][s]) / a.dt;
        }
    } else {
      _Pragma("unroll") for (int s = 0; s < 3; ++s) if (s < r.n)
        _Pragma("unroll") for (int k = 0; k < 3; ++k) a.v[k * a.n_site + r.s0 + s] = r.v[k][s];
    }
  }
  if (blockIdx.x == 0 && threadIdx.x == 0)
    for (int g = 0; g < a.n_groups; ++g) { a.xi[g] = xi[g]; a.eta[g] = eta[g]; }
}

constexpr int LJ_WAVES = 4;
void launch_lj(hipStream_t s, const MDArgs& a) {
  hipLaunchKernelGGL(k_lj<LJ_WAVES>, dim3(a.n_site), dim3(LJ_WAVES * WAVE), 0, s, a);
}
void launch_md_integrate(hipStream_t s, const MDArgs& a, int mode, int rec_step) {
  const int nb = md_workgroups(a.n_mol);
  hipLaunchKernelGGL(k_md_end, dim3(nb), dim3(WAVE), 0, s, a, mode);
  if (mode & 3) hipLaunchKernelGGL(k_md_start, dim3(nb), dim3(WAVE), 0, s, a, mode, rec_step, nb);
}

}  // namespace cpm
