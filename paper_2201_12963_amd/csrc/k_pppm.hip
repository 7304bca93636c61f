// Particle-mesh steps of PPPM (Hockney-Eastwood, as used by the paper for
// the long-range electrostatics): B-spline charge assignment of the
// electrolyte sites and of the electrode charges, and interpolation of the
// mesh potential at the electrode atoms, which gives the k-space part of b.
//
// (The electrolyte sites are spread plane by plane inside the forward x-y
// transform, k_fft_xy_spread.)
// Electrode spreading and gathering: the electrodes never move, so their
// stencils (mesh index and weight of every (atom, point) pair) are tables
// built once; the spread is then a deterministic sparse gather per touched
// mesh point (16 lanes each), and the potential at an atom is one
// wavefront-reduced dot product over its P^3 points.
#include <type_traits>

#include "common.h"

namespace cpm {

// rho[touch[t]] = sum_k val[k] q[col[k]] over rowptr[t] <= k < rowptr[t+1];
// 16 lanes per touched mesh point, reduced with shuffles
__global__ __launch_bounds__(256) void k_spread_elec(int n_touch, const int* __restrict__ touch,
                                                     const int* __restrict__ rowptr,
                                                     const int* __restrict__ col,
                                                     const double* __restrict__ val_d,
                                                     const float* __restrict__ val_f,
                                                     const double* __restrict__ q_all, size_t q_stride,
                                                     double* __restrict__ rho_d, float* __restrict__ rho_f, int M,
                                                     SlabTerms sl, double* __restrict__ slab_field) {
  const int sub = threadIdx.x & 15;
  const int t = blockIdx.x * (blockDim.x / 16) + (threadIdx.x >> 4);
  const int frame = blockIdx.y;
  const double* q = q_all + (size_t)frame * q_stride;
  if (slab_field && blockIdx.x == gridDim.x - 1) {   // the frame's slab field, one extra workgroup
    slab_field_block(sl, q, slab_field, frame);
    return;
  }
  const bool ok = t < n_touch;
  double acc = 0.0;
  if (ok) {
    const int k1 = rowptr[t + 1];
    for (int k = rowptr[t] + sub; k < k1; k += 16) acc += (val_d ? val_d[k] : (double)val_f[k]) * q[col[k]];
  }
#pragma unroll
  for (int off = 8; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 16);
  if (ok && sub == 0) {
    if (rho_d) rho_d[(size_t)frame * M + touch[t]] = acc;
    else rho_f[(size_t)frame * M + touch[t]] = (float)acc;
  }
}

// b_i = -(phi_real_i + sum_t gw[i][t] phi[gidx[i][t]]): one wavefront per atom
template <typename T>
__global__ __launch_bounds__(256) void k_gather_b(int n_elec, int P3, const int* __restrict__ gidx,
                                                  const T* __restrict__ gw, const T* __restrict__ phi_all,
                                                  int M, const T* __restrict__ phi_real_all,
                                                  double* __restrict__ b_all, SlabTerms sl) {
  const int lane = threadIdx.x & (WAVE - 1);
  const int i = blockIdx.x * (blockDim.x / WAVE) + (threadIdx.x >> 6);
  const int frame = blockIdx.y;
  if (i >= n_elec) return;
  const T* phi = phi_all + (size_t)frame * M;
  T acc = 0;
  for (int t = lane; t < P3; t += WAVE) acc += gw[(size_t)i * P3 + t] * phi[gidx[(size_t)i * P3 + t]];
  acc = wave_sum(acc);
  if (lane == 0) {
    size_t o = (size_t)frame * n_elec + i;
    b_all[o] = -((double)phi_real_all[o] + (double)acc) - slab_b_term(sl, i, frame);
  }
}

// The same with 16 lanes per atom, four atoms per wavefront (many frames:
// four times fewer wavefronts for the same loads)
template <typename T>
__global__ __launch_bounds__(256) void k_gather_b16(int n_elec, int P3, const int* __restrict__ gidx,
                                                    const T* __restrict__ gw, const T* __restrict__ phi_all,
                                                    int M, const T* __restrict__ phi_real_all,
                                                    double* __restrict__ b_all, SlabTerms sl) {
  const int sub = threadIdx.x & 15;
  const int i = blockIdx.x * (blockDim.x / 16) + (threadIdx.x >> 4);
  const int frame = blockIdx.y;
  const bool live = i < n_elec;
  const int ii = live ? i : n_elec - 1;
  const T* phi = phi_all + (size_t)frame * M;
  T acc = 0;
  for (int t = sub; t < P3; t += 16) acc += gw[(size_t)ii * P3 + t] * phi[gidx[(size_t)ii * P3 + t]];
#pragma unroll
  for (int off = 8; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 16);
  if (live && sub == 0) {
    size_t o = (size_t)frame * n_elec + i;
    b_all[o] = -((double)phi_real_all[o] + (double)acc) - slab_b_term(sl, i, frame);
  }
}

template <typename T>
void launch_spread_elec_t(hipStream_t s, int n_frames, int n_touch, const int* touch, const int* rowptr,
                          const int* col, const T* val, const double* q, size_t q_stride, T* rho, int M,
                          const SlabTerms& sl, double* slab_field) {
  dim3 grid((n_touch + 15) / 16 + (slab_field ? 1 : 0), n_frames);
  const bool dbl = std::is_same<T, double>::value;
  hipLaunchKernelGGL(k_spread_elec, grid, dim3(256), 0, s, n_touch, touch, rowptr, col,
                     dbl ? (const double*)val : nullptr, dbl ? nullptr : (const float*)val, q, q_stride,
                     dbl ? (double*)rho : nullptr, dbl ? nullptr : (float*)rho, M, sl, slab_field);
}

__global__ __launch_bounds__(256) void k_slab_field(SlabTerms sl, const double* __restrict__ q_all, size_t q_stride,
                                                    double* __restrict__ field) {
  slab_field_block(sl, q_all + (size_t)blockIdx.x * q_stride, field, blockIdx.x);
}

void launch_slab_field(hipStream_t s, int n_frames, const SlabTerms& sl, const double* q, size_t q_stride,
                       double* field) {
  hipLaunchKernelGGL(k_slab_field, dim3(n_frames), dim3(256), 0, s, sl, q, q_stride, field);
}

template <typename T>
void launch_gather_b_t(hipStream_t s, int n_frames, int n_elec, int P3, const int* gidx, const T* gw,
                       const T* phi, int M, const T* phi_real, double* b, const SlabTerms& sl) {
  if (n_frames == 1) {
    dim3 grid((n_elec + 3) / 4, 1);
    hipLaunchKernelGGL(k_gather_b<T>, grid, dim3(256), 0, s, n_elec, P3, gidx, gw, phi, M, phi_real, b, sl);
  } else {
    dim3 grid((n_elec + 15) / 16, n_frames);
    hipLaunchKernelGGL(k_gather_b16<T>, grid, dim3(256), 0, s, n_elec, P3, gidx, gw, phi, M, phi_real, b, sl);
  }
}

template void launch_spread_elec_t<double>(hipStream_t, int, int, const int*, const int*, const int*,
                                           const double*, const double*, size_t, double*, int, const SlabTerms&,
                                           double*);
template void launch_spread_elec_t<float>(hipStream_t, int, int, const int*, const int*, const int*,
                                          const float*, const double*, size_t, float*, int, const SlabTerms&,
                                          double*);
template void launch_gather_b_t<double>(hipStream_t, int, int, int, const int*, const double*, const double*,
                                        int, const double*, double*, const SlabTerms&);
template void launch_gather_b_t<float>(hipStream_t, int, int, int, const int*, const float*, const float*,
                                       int, const float*, double*, const SlabTerms&);

}  // namespace cpm
