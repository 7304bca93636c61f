// Energies of the step (Eq. 3 and its constant-potential counterpart), as
// one workgroup per frame (any whole number of wavefronts up to 1024 threads): ten sums over the electrodes, the
// sites and the k-space parts, reduced together, then U_coul and E_cp for
// every dV of the frame.
#pragma once
#include "common.h"

namespace cpm {

__device__ __forceinline__ void energy_block(const EnergyArgs& ea, int frame) {
  // ten partial sums reduced together: 8 dot products over the electrodes,
  // the site real-space energies and the k-space energy parts
  __shared__ double red[16][10];
  const size_t fe = (size_t)frame * ea.n_elec;
  double s[10] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
  for (int i = threadIdx.x; i < ea.n_elec; i += blockDim.x) {
    double Q = ea.Q0[fe + i], bb = ea.b[fe + i], sc = ea.Sc[i], c = ea.c[i], d = ea.d[i], z = ea.ze[i];
    s[0] += Q * bb; s[1] += sc * bb; s[2] += Q * c; s[3] += sc * c;
    s[4] += d * Q; s[5] += d * sc; s[6] += z * Q; s[7] += z * sc;
  }
  for (int j = threadIdx.x; j < ea.n_site; j += blockDim.x) s[8] += ea.u_site[(size_t)frame * ea.n_site + j];
  for (int j = threadIdx.x; j < ea.n_ek; j += blockDim.x) s[9] += ea.ek[(size_t)frame * ea.n_ek + j];
  const double v0[8] = {s[0], s[1], s[2], s[3], s[4], s[5], s[6], s[7]};
  const double v1[8] = {s[8], s[9], 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  const double t0 = wave_sum8(v0), t1 = wave_sum8(v1);     // lane 8k: total of value k
  const int lane = threadIdx.x & 63;
  if ((lane & 7) == 0) {
    red[threadIdx.x >> 6][lane >> 3] = t0;
    if (lane < 16) red[threadIdx.x >> 6][8 + (lane >> 3)] = t1;
  }
  __syncthreads();
  double S[10];
  const int nw = blockDim.x >> 6;
  for (int t = 0; t < 10; ++t) {
    S[t] = red[0][t];
    for (int w = 1; w < nw; ++w) S[t] += red[w][t];
  }
  double zdip = ea.zdip ? ea.zdip[frame] : 0.0;
  // slab geometry: the electrolyte block of the dipole correction
  double u_elyt = S[8] + S[9] - ea.self_energy + 0.5 * ea.slab_kappa * zdip * zdip;
  for (int v = threadIdx.x; v < ea.n_dv; v += blockDim.x) {
    double dv = ea.dv ? ea.dv[v] : ea.dv_single;
    double qb = S[0] + dv * S[1];
    double qv = S[0] + dv * (S[2] + S[1]) + dv * dv * S[3];
    double dq = S[4] + dv * S[5];
    double zq = S[6] + dv * S[7];
    double uc = u_elyt - qb + 0.5 * qv;
    double ecp = uc - dv * dq;
    if (ea.ff) ecp += dv / ea.Lz * (zq + zdip);
    double* o = ea.out + ((size_t)frame * ea.n_dv + v) * 2;
    o[0] = uc;
    o[1] = ecp;
  }
}

}  // namespace cpm
