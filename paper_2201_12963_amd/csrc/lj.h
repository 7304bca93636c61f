// Lennard-Jones forces and energy share of one electrolyte site, by one
// workgroup of NW wavefronts whose threads share the partners: the sites and
// graphene atoms of the z layers within the cutoff (the layers of the
// electrostatic cell grid, whose binning of the same positions has run),
// minimum image, pairs of one molecule excluded, energy shifted to zero at
// the cutoff, Lorentz-Berthelot mixing from the stored square roots of
// epsilon.  A kernel of its own (k_lj) or extra workgroups of the MD loop's
// field z pass.
#pragma once
#include "common.h"
#include "bin.h"

namespace cpm {

template <int NW>
__device__ __forceinline__ void lj_site(const MDArgs& a, int i) {
  __shared__ double red[NW][4];
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
  // the z layer of the site, by the binning's arithmetic on the same
  // coordinate, and the sorted-site ranges of the layers within lj_reach
  int cz;
  wrap_and_cell(zi, a.Lz, a.nc_z, cz);
  const int* cs = a.cell_start;
  int lo0 = 0, hi0 = a.n_site, lo1 = 0, hi1 = 0;
  if (2 * a.lj_reach + 1 < a.nc_z) {
    const int la = cz - a.lj_reach, lb = cz + a.lj_reach;
    if (la < 0) { lo0 = cs[(la + a.nc_z) * a.nxy]; hi1 = cs[(lb + 1) * a.nxy]; }
    else if (lb >= a.nc_z) { lo0 = cs[la * a.nxy]; hi1 = cs[(lb + 1 - a.nc_z) * a.nxy]; }
    else { lo0 = cs[la * a.nxy]; hi0 = cs[(lb + 1) * a.nxy]; }
  }
  auto site = [&](int s) {
    const int j = a.order[s];
    if (a.mol_of[j] == mi) return;
    pair(xi - a.x[j], yi - a.x[a.n_site + j], zi - a.x[2 * a.n_site + j], 0.5 * (si + a.sigma[j]), qi * a.sqeps[j]);
  };
  for (int s = lo0 + threadIdx.x; s < hi0; s += blockDim.x) site(s);
  for (int s = lo1 + threadIdx.x; s < hi1; s += blockDim.x) site(s);
  uw = 1.0;
  const double sc = 0.5 * (si + a.carbon_sigma), ec = qi * a.carbon_sqeps;
  const int* cr = a.carbon_run + 4 * cz;
#pragma unroll
  for (int h = 0; h < 2; ++h)
    for (int j = cr[2 * h] + threadIdx.x; j < cr[2 * h + 1]; j += blockDim.x)
      pair(xi - a.cx[j], yi - a.cx[a.n_lj_elec + j], zi - a.cx[2 * a.n_lj_elec + j], sc, ec);
  fx = wave_sum(fx); fy = wave_sum(fy); fz = wave_sum(fz); u = wave_sum(u);
  const int w = threadIdx.x / WAVE;
  if ((threadIdx.x & (WAVE - 1)) == 0) { red[w][0] = fx; red[w][1] = fy; red[w][2] = fz; red[w][3] = u; }
  __syncthreads();
  if (threadIdx.x < 4) {
    double t = red[0][threadIdx.x];
#pragma unroll
    for (int k = 1; k < NW; ++k) t += red[k][threadIdx.x];
    if (threadIdx.x < 3) a.f_lj[threadIdx.x * a.n_site + i] = t;
    else a.u_lj[i] = t;
  }
}

}  // namespace cpm
