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
// mesh point, and the potential at an atom one reduced dot product over its
// P^3 points.  Many frames share each table read: the spread stages the
// charges of up to 8 frames in LDS, the gather gives every lane 8 frames.
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

// The same sums for many frames: a workgroup takes F frames (their charges
// staged in LDS) and a chunk of the touched points, a thread one (point,
// frame) pair, whose row it walks alone; the F threads of a point read the
// same table entries, so the table is read once per F frames instead of
// once per frame
constexpr int SPREAD_FRAMES_THREADS = 512;
constexpr int SPREAD_FRAMES_LDS = 64 * 1024;     // staged charges of 8 frames at most, bytes
constexpr int SPREAD_FRAMES_LDS_MAX = 128 * 1024;  // of 4 or 2 frames (one workgroup per CU)
constexpr int SPREAD_FRAMES_CHUNKS = 4;          // point chunks (workgroups per frame group)

template <typename T, int F>
__global__ __launch_bounds__(SPREAD_FRAMES_THREADS) void k_spread_elec_frames(
    int n_touch, const int* __restrict__ touch, const int* __restrict__ rowptr, const int* __restrict__ col,
    const T* __restrict__ val, const double* __restrict__ q_all, size_t q_stride, int n_elec, int n_frames,
    T* __restrict__ rho, int M) {
  extern __shared__ double qs[];                 // [F][n_elec]
  const int f0 = blockIdx.y * F;
  const int nfr = min(F, n_frames - f0);
  for (int i = threadIdx.x; i < F * n_elec; i += SPREAD_FRAMES_THREADS) {
    const int f = i / n_elec;
    qs[i] = f < nfr ? q_all[(size_t)(f0 + f) * q_stride + (i - f * n_elec)] : 0.0;
  }
  __syncthreads();
  const int f = threadIdx.x % F;
  if (f >= nfr) return;                          // (no barrier below)
  const int per = (n_touch + gridDim.x - 1) / gridDim.x;
  const int t_lo = blockIdx.x * per, t_hi = min(n_touch, t_lo + per);
  const double* qf = qs + f * n_elec;
  T* out = rho + (size_t)(f0 + f) * M;
  for (int t = t_lo + (int)threadIdx.x / F; t < t_hi; t += SPREAD_FRAMES_THREADS / F) {
    const int k1 = rowptr[t + 1];
    double acc = 0.0;
#pragma unroll 4
    for (int k = rowptr[t]; k < k1; ++k) acc += (double)val[k] * qf[col[k]];
    out[touch[t]] = (T)acc;
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

// The same for many frames: 16 lanes per atom, four atoms per wavefront,
// and GATHER_FRAMES frames per lane, so that every table entry a lane reads
// serves that many frames (one table read per GATHER_FRAMES frames instead
// of one per frame).  The sums are FP64 in either precision.
constexpr int GATHER_FRAMES = 8;

template <typename T>
__global__ __launch_bounds__(256) void k_gather_b_frames(int n_elec, int P3, const int* __restrict__ gidx,
                                                         const T* __restrict__ gw, const T* __restrict__ phi_all,
                                                         int M, const T* __restrict__ phi_real_all,
                                                         double* __restrict__ b_all, SlabTerms sl, int n_frames) {
  constexpr int F = GATHER_FRAMES;
  const int sub = threadIdx.x & 15;
  const int i = blockIdx.x * (blockDim.x / 16) + (threadIdx.x >> 4);
  const int f0 = blockIdx.y * F;
  const int nfr = min(F, n_frames - f0);
  const bool live = i < n_elec;
  const int ii = live ? i : n_elec - 1;
  const T* phi = phi_all + (size_t)f0 * M;
  double acc[F];
#pragma unroll
  for (int f = 0; f < F; ++f) acc[f] = 0.0;
  for (int t = sub; t < P3; t += 16) {
    const double w = (double)gw[(size_t)ii * P3 + t];
    const int g = gidx[(size_t)ii * P3 + t];
#pragma unroll
    for (int f = 0; f < F; ++f)
      if (f < nfr) acc[f] += w * (double)phi[(size_t)f * M + g];
  }
#pragma unroll
  for (int f = 0; f < F; ++f)
#pragma unroll
    for (int off = 8; off > 0; off >>= 1) acc[f] += __shfl_xor(acc[f], off, 16);
  if (live && sub == 0) {
#pragma unroll
    for (int f = 0; f < F; ++f) {
      if (f < nfr) {
        const size_t o = (size_t)(f0 + f) * n_elec + i;
        b_all[o] = -((double)phi_real_all[o] + acc[f]) - slab_b_term(sl, i, f0 + f);
      }
    }
  }
}

template <typename T>
void launch_spread_elec_t(hipStream_t s, int n_frames, int n_touch, const int* touch, const int* rowptr,
                          const int* col, const T* val, const double* q, size_t q_stride, T* rho, int M,
                          const SlabTerms& sl, double* slab_field, int n_elec) {
  // many frames: 8 per workgroup where their charges fit in 64 KiB, else 4
  // or 2 within 128 KiB (8 frames in 112 KiB, one workgroup per CU, measured
  // slower than 4 in 56 KiB; a single frame per workgroup slower than the
  // per-frame kernel below, which then serves)
  const size_t row = (size_t)n_elec * sizeof(double);
  const int F = n_frames <= 1 || n_elec <= 0            ? 0
                : 8 * row <= (size_t)SPREAD_FRAMES_LDS     ? 8
                : 4 * row <= (size_t)SPREAD_FRAMES_LDS_MAX ? 4
                : 2 * row <= (size_t)SPREAD_FRAMES_LDS_MAX ? 2
                                                           : 0;
  if (F > 0) {
    const dim3 grid(SPREAD_FRAMES_CHUNKS, (n_frames + F - 1) / F);
    const size_t lds = (size_t)F * n_elec * sizeof(double);
    auto go = [&](auto kern) {
      hipLaunchKernelGGL(kern, grid, dim3(SPREAD_FRAMES_THREADS), lds, s, n_touch, touch, rowptr, col, val, q,
                         q_stride, n_elec, n_frames, rho, M);
    };
    if (F == 8) go(k_spread_elec_frames<T, 8>);
    else if (F == 4) go(k_spread_elec_frames<T, 4>);
    else go(k_spread_elec_frames<T, 2>);
    if (slab_field) launch_slab_field(s, n_frames, sl, q, q_stride, slab_field);
    return;
  }
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
    dim3 grid((n_elec + 15) / 16, (n_frames + GATHER_FRAMES - 1) / GATHER_FRAMES);
    hipLaunchKernelGGL(k_gather_b_frames<T>, grid, dim3(256), 0, s, n_elec, P3, gidx, gw, phi, M, phi_real, b, sl,
                       n_frames);
  }
}

template void launch_spread_elec_t<double>(hipStream_t, int, int, const int*, const int*, const int*,
                                           const double*, const double*, size_t, double*, int, const SlabTerms&,
                                           double*, int);
template void launch_spread_elec_t<float>(hipStream_t, int, int, const int*, const int*, const int*,
                                          const float*, const double*, size_t, float*, int, const SlabTerms&,
                                          double*, int);
template void launch_gather_b_t<double>(hipStream_t, int, int, int, const int*, const double*, const double*,
                                        int, const double*, double*, const SlabTerms&);
template void launch_gather_b_t<float>(hipStream_t, int, int, int, const int*, const float*, const float*,
                                       int, const float*, double*, const SlabTerms&);

}  // namespace cpm
