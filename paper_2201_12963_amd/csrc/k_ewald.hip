// Explicit Ewald reciprocal sums over a list of half-space wavevectors
// (k and -k contribute complex conjugates, so each listed k carries the
// doubled weight ew = 2 k_e w(k), w(k) = (4 pi/V) exp(-k^2/4 alpha^2)/k^2).
// Used for small cells, where a k-sphere of ~10^3 vectors is cheaper and
// more accurate than a mesh.
//   structure factor   rho(k) = sum_j Q_j e^{i k.R_j}       (one wave per k)
//   potential at the electrodes  sum_k ew Re(e^{-i k.r_i} rho(k))  (one wave per atom)
//   all-charge factor  rho_all(k) = rho(k) + sum_i q_i e^{i k.r_i}
//   field at the sites E_j = -sum_k ew k Im(e^{-i k.R_j} rho_all(k))
// The electrode phases e^{i k.r_i} are a fixed table [k][atom].
#include "common.h"

namespace cpm {

__global__ __launch_bounds__(256) void k_ewald_sf(int nk, const double* __restrict__ kv, const double* __restrict__ ew,
                                                  SiteSet<double> st, double2* __restrict__ rho_all,
                                                  double* __restrict__ ek_all) {
  const int lane = threadIdx.x & (WAVE - 1);
  const int k = blockIdx.x * (blockDim.x / WAVE) + (threadIdx.x >> 6);
  const int frame = blockIdx.y;
  if (k >= nk) return;
  const size_t fo = (size_t)frame * st.n;
  const double kx = kv[k], ky = kv[nk + k], kz = kv[2 * nk + k];
  double re = 0.0, im = 0.0;
  for (int j = lane; j < st.n; j += WAVE) {
    double s, c;
    sincos(kx * st.x[fo + j] + ky * st.y[fo + j] + kz * st.z[fo + j], &s, &c);
    re += st.q[fo + j] * c;
    im += st.q[fo + j] * s;
  }
  re = wave_sum(re);
  im = wave_sum(im);
  if (lane == 0) {
    rho_all[(size_t)frame * nk + k] = double2{re, im};
    if (ek_all) ek_all[(size_t)frame * nk + k] = 0.5 * ew[k] * (re * re + im * im);
  }
}

__global__ __launch_bounds__(256) void k_ewald_phi(int nk, int n_elec, const double* __restrict__ ew,
                                                   const double2* __restrict__ eph, const double2* __restrict__ rho_all,
                                                   const double* __restrict__ phi_real_all, double* __restrict__ b_all,
                                                   SlabTerms sl) {
  const int lane = threadIdx.x & (WAVE - 1);
  const int i = blockIdx.x * (blockDim.x / WAVE) + (threadIdx.x >> 6);
  const int frame = blockIdx.y;
  if (i >= n_elec) return;
  const double2* rho = rho_all + (size_t)frame * nk;
  double acc = 0.0;
  for (int k = lane; k < nk; k += WAVE) {
    double2 e = eph[(size_t)k * n_elec + i];
    double2 r = rho[k];
    acc += ew[k] * (e.x * r.x + e.y * r.y);       // Re(conj(e) rho)
  }
  acc = wave_sum(acc);
  if (lane == 0) {
    size_t o = (size_t)frame * n_elec + i;
    b_all[o] = -(phi_real_all[o] + acc) - slab_b_term(sl, i, frame);
  }
}

__global__ __launch_bounds__(256) void k_ewald_rho_all(int nk, int n_elec, const double2* __restrict__ eph,
                                                       const double* __restrict__ q_all, size_t q_stride,
                                                       const double2* __restrict__ rho_all,
                                                       double2* __restrict__ out_all) {
  const int lane = threadIdx.x & (WAVE - 1);
  const int k = blockIdx.x * (blockDim.x / WAVE) + (threadIdx.x >> 6);
  const int frame = blockIdx.y;
  if (k >= nk) return;
  const double* q = q_all + (size_t)frame * q_stride;
  double re = 0.0, im = 0.0;
  for (int i = lane; i < n_elec; i += WAVE) {
    double2 e = eph[(size_t)k * n_elec + i];
    re += q[i] * e.x;
    im += q[i] * e.y;
  }
  re = wave_sum(re);
  im = wave_sum(im);
  if (lane == 0) {
    double2 r = rho_all ? rho_all[(size_t)frame * nk + k] : double2{0.0, 0.0};
    out_all[(size_t)frame * nk + k] = double2{r.x + re, r.y + im};
  }
}

__global__ __launch_bounds__(256) void k_ewald_field(int nk, const double* __restrict__ kv, const double* __restrict__ ew,
                                                     SiteSet<double> st, const double2* __restrict__ rho_all,
                                                     double* __restrict__ E_all) {
  const int lane = threadIdx.x & (WAVE - 1);
  const int j = blockIdx.x * (blockDim.x / WAVE) + (threadIdx.x >> 6);
  const int frame = blockIdx.y;
  if (j >= st.n) return;
  const size_t fo = (size_t)frame * st.n;
  const double x = st.x[fo + j], y = st.y[fo + j], z = st.z[fo + j];
  const double2* rho = rho_all + (size_t)frame * nk;
  double e0 = 0.0, e1 = 0.0, e2 = 0.0;
  for (int k = lane; k < nk; k += WAVE) {
    double kx = kv[k], ky = kv[nk + k], kz = kv[2 * nk + k];
    double s, c;
    sincos(kx * x + ky * y + kz * z, &s, &c);
    double2 r = rho[k];
    double im = c * r.y - s * r.x;                 // Im(e^{-i k.R} rho)
    double a = -ew[k] * im;
    e0 += a * kx; e1 += a * ky; e2 += a * kz;
  }
  e0 = wave_sum(e0); e1 = wave_sum(e1); e2 = wave_sum(e2);
  if (lane == 0) {
    double* E = E_all + (size_t)frame * 3 * st.n;
    E[j] = e0; E[st.n + j] = e1; E[2 * st.n + j] = e2;
  }
}

void launch_ewald_sf(hipStream_t s, int n_frames, int nk, const double* kv, const double* ew,
                     const SiteSet<double>& st, double2* rho, double* ek) {
  hipLaunchKernelGGL(k_ewald_sf, dim3((nk + 3) / 4, n_frames), dim3(256), 0, s, nk, kv, ew, st, rho, ek);
}
void launch_ewald_phi(hipStream_t s, int n_frames, int nk, int n_elec, const double* ew, const double2* eph,
                      const double2* rho, const double* phi_real, double* b, const SlabTerms& sl) {
  hipLaunchKernelGGL(k_ewald_phi, dim3((n_elec + 3) / 4, n_frames), dim3(256), 0, s, nk, n_elec, ew, eph, rho,
                     phi_real, b, sl);
}
void launch_ewald_rho_all(hipStream_t s, int n_frames, int nk, int n_elec, const double2* eph, const double* q,
                          size_t q_stride, const double2* rho, double2* out) {
  hipLaunchKernelGGL(k_ewald_rho_all, dim3((nk + 3) / 4, n_frames), dim3(256), 0, s, nk, n_elec, eph, q,
                     q_stride, rho, out);
}
void launch_ewald_field(hipStream_t s, int n_frames, int nk, const double* kv, const double* ew,
                        const SiteSet<double>& st, const double2* rho, double* E) {
  hipLaunchKernelGGL(k_ewald_field, dim3((st.n + 3) / 4, n_frames), dim3(256), 0, s, nk, kv, ew, st, rho, E);
}

}  // namespace cpm
