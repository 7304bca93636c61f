// Mixed-precision charge solve.
//
// Single frame: q = S (b - mean(b)) with S stored in FP32 and FP32
// accumulation (S e = 0, so centring b changes nothing exactly and removes
// the large common offset of b before rounding), then an FP64 re-projection
// onto the neutral subspace (per sub-cell for the doubled cell).
//
// Batch: Q = S B as a split-precision GEMM on the bf16 matrix cores
// (k_gemm.hip).  Each operand is written here as three bf16 terms
// x = x0 + x1 + x2 (x0 = bf16(x), x1 = bf16(x - x0), x2 = bf16(x - x0 - x1),
// about 2^-25 relative left over) and S B ~ sum of the six products x_a y_b
// with a + b <= 2, accumulated in FP32.  Two terms (three products) are not
// enough here: the rows of S sum to zero, so |q_i| is a small fraction of
// sum_j |S_ij b_j| and a 2^-17 relative product error shows up as ~1e-5 e.
#include "common.h"

namespace cpm {

// bf16 bits by round-to-nearest-even (finite inputs)
__device__ __forceinline__ unsigned short bf16_rne(float x) {
  unsigned int u = __float_as_uint(x);
  unsigned int lsb = (u >> 16) & 1u;
  u += 0x7fffu + lsb;
  return (unsigned short)(u >> 16);
}
__device__ __forceinline__ float bf16_to_f(unsigned short h) { return __uint_as_float(((unsigned int)h) << 16); }

// S (n x n, double) -> FP32 copy (n x n) and bf16 hi/lo split with rows padded to n_pad
// three-term bf16 split of v: t[0] + t[1] + t[2]
__device__ __forceinline__ void split3(double v, unsigned short* t) {
  t[0] = bf16_rne((float)v);
  double r = v - (double)bf16_to_f(t[0]);
  t[1] = bf16_rne((float)r);
  r -= (double)bf16_to_f(t[1]);
  t[2] = bf16_rne((float)r);
}

// S (n x n, double) -> FP32 copy (n x n) and three bf16 terms with rows padded
// to n_pad: term k at split[k * n * n_pad + row * n_pad + col]
__global__ __launch_bounds__(256) void k_split_matrix(int n, int n_pad, const double* __restrict__ S,
                                                      float* __restrict__ Sf, unsigned short* __restrict__ split) {
  const int col = blockIdx.x * blockDim.x + threadIdx.x;
  const int row = blockIdx.y;
  if (col >= n_pad) return;
  double v = col < n ? S[(size_t)row * n + col] : 0.0;
  if (Sf && col < n) Sf[(size_t)row * n + col] = (float)v;
  unsigned short t[3];
  split3(v, t);
  const size_t plane = (size_t)n * n_pad;
  for (int k = 0; k < 3; ++k) split[k * plane + (size_t)row * n_pad + col] = t[k];
}


// mean-centred b of each frame, split into three bf16 terms, rows [frame][n_pad]
// (term k at split[k * n_frames * n_pad + ...])
__global__ __launch_bounds__(256) void k_split_b(int n, int n_pad, const double* __restrict__ b_all,
                                                 unsigned short* __restrict__ split) {
  __shared__ double red[4];
  const int f = blockIdx.x;
  const double* b = b_all + (size_t)f * n;
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) s += b[i];
  s = wave_sum(s);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  const double mean = (red[0] + red[1] + red[2] + red[3]) / n;
  const size_t plane = (size_t)gridDim.x * n_pad;
  for (int i = threadIdx.x; i < n_pad; i += blockDim.x) {
    unsigned short t[3];
    split3(i < n ? b[i] - mean : 0.0, t);
    for (int k = 0; k < 3; ++k) split[k * plane + (size_t)f * n_pad + i] = t[k];
  }
}

// Column sums of the FP32 copy of S over each neutrality group (group 1: the
// first sub-cell of the doubled cell, group 0: the rest; one group for the
// finite field and slab), in FP64: colsum[g][j] = sum_{i in g} Sf[i][j].
// One thread per column (rows read in turn, coalesced across the columns).
__global__ __launch_bounds__(256) void k_colsum(int n, const float* __restrict__ Sf,
                                                const unsigned char* __restrict__ sub1, double* __restrict__ colsum) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  double s0 = 0.0, s1 = 0.0;
  for (int i = 0; i < n; ++i) {
    const double v = (double)Sf[(size_t)i * n + j];
    if (sub1 && sub1[i]) s1 += v; else s0 += v;
  }
  colsum[j] = s0;
  colsum[n + j] = s1;
}

// One-frame mixed charge step in one launch: q = Sf b - m_g + dV S c with S
// stored in FP32 (half the bytes the FP64 GEMV streams) but products and sums
// in FP64, and m_g = colsum_g . b / n_g the mean of (Sf b) over the atom's
// neutrality group: sum_{i in g} (Sf b)_i = colsum_g . b, so subtracting m_g
// re-projects onto the neutral subspace exactly as a pass over the finished
// charges would, without that pass.  Every workgroup forms the two means
// from the cached colsum and b; a wavefront per row of S.
__global__ __launch_bounds__(256) void k_charges_mixed(int n, const float* __restrict__ Sf,
                                                       const double* __restrict__ colsum,
                                                       const unsigned char* __restrict__ sub1, double inv_n0,
                                                       double inv_n1, const double* __restrict__ b_all,
                                                       const double* __restrict__ Sc, double dv,
                                                       double* __restrict__ Q0_all, double* __restrict__ q_all,
                                                       const int* __restrict__ epos, double* __restrict__ qs_all) {
  __shared__ double red[2][4];
  const int lane = threadIdx.x & (WAVE - 1);
  const int frame = blockIdx.y;
  const double* b = b_all + (size_t)frame * n;
  double m0 = 0.0, m1 = 0.0;
  for (int j = threadIdx.x; j < n; j += blockDim.x) {
    const double bj = b[j];
    m0 = fma(colsum[j], bj, m0);
    m1 = fma(colsum[n + j], bj, m1);
  }
  m0 = wave_sum(m0);
  m1 = wave_sum(m1);
  if (lane == 0) { red[0][threadIdx.x >> 6] = m0; red[1][threadIdx.x >> 6] = m1; }
  __syncthreads();
  const double mean0 = ((red[0][0] + red[0][1]) + (red[0][2] + red[0][3])) * inv_n0;
  const double mean1 = ((red[1][0] + red[1][1]) + (red[1][2] + red[1][3])) * inv_n1;
  const int i = blockIdx.x * (blockDim.x / WAVE) + (threadIdx.x >> 6);
  if (i >= n) return;
  const int ep = qs_all ? epos[i] : 0;
  double a0 = 0.0, a1 = 0.0;
  if ((n & 3) == 0) {       // rows 16-byte aligned: four FP32 values per load
    const float4* row = reinterpret_cast<const float4*>(Sf + (size_t)i * n);
    const double2* b2 = reinterpret_cast<const double2*>(b);
    const int n4 = n >> 2;
    for (int j = lane; j < n4; j += WAVE) {
      const float4 sv = row[j];
      const double2 v0 = b2[2 * j], v1 = b2[2 * j + 1];
      a0 = fma((double)sv.x, v0.x, fma((double)sv.y, v0.y, a0));
      a1 = fma((double)sv.z, v1.x, fma((double)sv.w, v1.y, a1));
    }
  } else {
    const float* row = Sf + (size_t)i * n;
    for (int j = lane; j < n; j += WAVE) a0 = fma((double)row[j], b[j], a0);
  }
  const double acc = wave_sum(a0 + a1) - ((sub1 && sub1[i]) ? mean1 : mean0);
  if (lane == 0) {
    const size_t o = (size_t)frame * n + i;
    const double qv = acc + dv * Sc[i];
    if (Q0_all) Q0_all[o] = acc;
    if (q_all) q_all[o] = qv;
    if (qs_all) qs_all[(size_t)frame * n + ep] = qv;
  }
}

// FP64 re-projection onto the neutral subspace: Q0 -= mean over each sub-cell
// (one sub-cell for the finite field); one workgroup per frame
__global__ __launch_bounds__(256) void k_reproject(int n, const unsigned char* __restrict__ sub1, double* __restrict__ Q0_all) {
  __shared__ double red[4];
  double* Q = Q0_all + (size_t)blockIdx.x * n;
  double s0 = 0.0, s1 = 0.0;
  int n1 = 0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    bool in1 = sub1 && sub1[i];
    (in1 ? s1 : s0) += Q[i];
    n1 += in1;
  }
  double S0 = block_sum_d(s0, red), S1 = block_sum_d(s1, red), N1 = block_sum_d((double)n1, red);
  const double m0 = S0 / (n - N1), m1 = N1 > 0 ? S1 / N1 : 0.0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) Q[i] -= (sub1 && sub1[i]) ? m1 : m0;
}

// ------------------------------------------------------------ launchers

void launch_split_matrix(hipStream_t s, int n, int n_pad, const double* S, float* Sf, unsigned short* split) {
  hipLaunchKernelGGL(k_split_matrix, dim3((n_pad + 255) / 256, n), dim3(256), 0, s, n, n_pad, S, Sf, split);
}
void launch_split_b(hipStream_t s, int n_frames, int n, int n_pad, const double* b, unsigned short* split) {
  hipLaunchKernelGGL(k_split_b, dim3(n_frames), dim3(256), 0, s, n, n_pad, b, split);
}
void launch_colsum(hipStream_t s, int n, const float* Sf, const unsigned char* sub1, double* colsum) {
  hipLaunchKernelGGL(k_colsum, dim3((n + 255) / 256), dim3(256), 0, s, n, Sf, sub1, colsum);
}
void launch_charges_mixed(hipStream_t s, int n_frames, int n, const float* Sf, const double* colsum,
                          const unsigned char* sub1, double inv_n0, double inv_n1, const double* b, const double* Sc,
                          double dv, double* Q0, double* q, const int* epos, double* qs) {
  hipLaunchKernelGGL(k_charges_mixed, dim3((n + 3) / 4, n_frames), dim3(256), 0, s, n, Sf, colsum, sub1, inv_n0, inv_n1,
                     b, Sc, dv, Q0, q, epos, qs);
}
void launch_reproject(hipStream_t s, int n_frames, int n, const unsigned char* sub1, double* Q0) {
  hipLaunchKernelGGL(k_reproject, dim3(n_frames), dim3(256), 0, s, n, sub1, Q0);
}
}  // namespace cpm
