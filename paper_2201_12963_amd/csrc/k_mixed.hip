// Mixed-precision charge solve.
//
// Single frame: q = S (b - mean(b)) with S stored in FP32 and FP32
// accumulation (S e = 0, so centring b changes nothing exactly and removes
// the large common offset of b before rounding), then an FP64 re-projection
// onto the neutral subspace (per sub-cell for the doubled cell).
//
// Batch: Q = S B as a split-precision GEMM on the bf16 matrix cores.  Each
// operand is written as three bf16 terms x = x0 + x1 + x2 (x0 = bf16(x),
// x1 = bf16(x - x0), x2 = bf16(x - x0 - x1), about 2^-25 relative left over)
// and S B ~ sum of the six products x_a y_b with a + b <= 2, accumulated in
// FP32 by v_mfma_f32_16x16x16 bf16.  Two terms (three products) are not
// enough here: the rows of S sum to zero, so |q_i| is a small fraction of
// sum_j |S_ij b_j| and a 2^-17 relative product error shows up as ~1e-5 e.
// A 256-thread workgroup owns a 64 x 64 output tile, each wavefront a
// 32 x 32 quarter (2 x 2 MFMA blocks); operand slabs of 64 x 16 pass through
// LDS.
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

// out = x + a y (and its cell-sorted copy out_s[epos[i]], if given)
__global__ __launch_bounds__(256) void k_axpy(int n, const double* __restrict__ x, const double* __restrict__ y,
                                              double a, double* __restrict__ out, const int* __restrict__ epos,
                                              double* __restrict__ out_s) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) {
    const double v = x[i] + a * y[i];
    out[i] = v;
    if (out_s) out_s[epos[i]] = v;
  }
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

// Q0[f][i] = sum_j Sf[i][j] (b[f][j] - mean_f b), FP32 accumulation; one wavefront per row
__global__ __launch_bounds__(256) void k_charges_f32(int n, const float* __restrict__ Sf, const double* __restrict__ b_all,
                                                     double* __restrict__ Q0_all) {
  __shared__ float bc[4096];
  __shared__ double red[4];
  const int lane = threadIdx.x & (WAVE - 1);
  const int frame = blockIdx.y;
  const double* b = b_all + (size_t)frame * n;
  double s = 0.0;
  for (int j = threadIdx.x; j < n; j += blockDim.x) s += b[j];
  s = wave_sum(s);
  if (lane == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  const double mean = (red[0] + red[1] + red[2] + red[3]) / n;
  for (int j = threadIdx.x; j < n; j += blockDim.x) bc[j] = (float)(b[j] - mean);
  __syncthreads();
  const int i = blockIdx.x * (blockDim.x / WAVE) + (threadIdx.x >> 6);
  if (i >= n) return;
  const float* row = Sf + (size_t)i * n;
  float acc = 0.0f;
  for (int j = lane; j < n; j += WAVE) acc = fmaf(row[j], bc[j], acc);
  acc = wave_sum(acc);
  if (lane == 0) Q0_all[(size_t)frame * n + i] = (double)acc;
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

// D[f][i] = sum_k A[f][k] B[i][k]; A and B given as three bf16 terms of rows
// of length K (K a multiple of 16; rows beyond M or N read as zero).
typedef short short4_t __attribute__((ext_vector_type(4)));
typedef float float4_t __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(256) void k_gemm_bf16x6(int M, int N, int K, const unsigned short* __restrict__ A,
                                                     size_t a_plane, const unsigned short* __restrict__ B,
                                                     size_t b_plane, double* __restrict__ D, int ldd) {
  __shared__ unsigned short sA[3][64][16 + 4], sB[3][64][16 + 4];
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int m0 = blockIdx.y * 64, n0 = blockIdx.x * 64;
  const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
  float4_t acc[2][2];
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b) acc[a][b] = float4_t{0.f, 0.f, 0.f, 0.f};
  // MFMA operand layout (16 x 16 x 16, bf16): lane l feeds row/column l % 16
  // with k = 4 (l / 16) .. 4 (l / 16) + 3
  const int r = lane & 15, kg = (lane >> 4) * 4;
  const int lrow = threadIdx.x >> 2, lk = (threadIdx.x & 3) * 4;
  for (int k0 = 0; k0 < K; k0 += 16) {
    const int ga = m0 + lrow, gb = n0 + lrow;
    for (int p = 0; p < 3; ++p)
      for (int t = 0; t < 4; ++t) {
        sA[p][lrow][lk + t] = ga < M ? A[p * a_plane + (size_t)ga * K + k0 + lk + t] : 0;
        sB[p][lrow][lk + t] = gb < N ? B[p * b_plane + (size_t)gb * K + k0 + lk + t] : 0;
      }
    __syncthreads();
    short4_t av[3][2], bv[3][2];
    for (int p = 0; p < 3; ++p)
      for (int a = 0; a < 2; ++a)
        for (int t = 0; t < 4; ++t) {
          av[p][a][t] = (short)sA[p][wm + 16 * a + r][kg + t];
          bv[p][a][t] = (short)sB[p][wn + 16 * a + r][kg + t];
        }
    for (int a = 0; a < 2; ++a)
      for (int b = 0; b < 2; ++b) {
        // smallest terms first
        acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av[1][a], bv[1][b], acc[a][b], 0, 0, 0);
        acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av[2][a], bv[0][b], acc[a][b], 0, 0, 0);
        acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av[0][a], bv[2][b], acc[a][b], 0, 0, 0);
        acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av[1][a], bv[0][b], acc[a][b], 0, 0, 0);
        acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av[0][a], bv[1][b], acc[a][b], 0, 0, 0);
        acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av[0][a], bv[0][b], acc[a][b], 0, 0, 0);
      }
    __syncthreads();
  }
  // D block layout: lane holds rows 4 (lane / 16) + t of column lane % 16
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b)
      for (int t = 0; t < 4; ++t) {
        int gm = m0 + wm + 16 * a + (lane >> 4) * 4 + t;
        int gn = n0 + wn + 16 * b + (lane & 15);
        if (gm < M && gn < N) D[(size_t)gm * ldd + gn] = (double)acc[a][b][t];
      }
}

// ------------------------------------------------------------ launchers

void launch_split_matrix(hipStream_t s, int n, int n_pad, const double* S, float* Sf, unsigned short* split) {
  hipLaunchKernelGGL(k_split_matrix, dim3((n_pad + 255) / 256, n), dim3(256), 0, s, n, n_pad, S, Sf, split);
}
void launch_axpy(hipStream_t s, int n, const double* x, const double* y, double a, double* out, const int* epos,
                 double* out_s) {
  hipLaunchKernelGGL(k_axpy, dim3((n + 255) / 256), dim3(256), 0, s, n, x, y, a, out, epos, out_s);
}
void launch_split_b(hipStream_t s, int n_frames, int n, int n_pad, const double* b, unsigned short* split) {
  hipLaunchKernelGGL(k_split_b, dim3(n_frames), dim3(256), 0, s, n, n_pad, b, split);
}
void launch_charges_f32(hipStream_t s, int n_frames, int n, const float* Sf, const double* b, double* Q0) {
  hipLaunchKernelGGL(k_charges_f32, dim3((n + 3) / 4, n_frames), dim3(256), 0, s, n, Sf, b, Q0);
}
void launch_reproject(hipStream_t s, int n_frames, int n, const unsigned char* sub1, double* Q0) {
  hipLaunchKernelGGL(k_reproject, dim3(n_frames), dim3(256), 0, s, n, sub1, Q0);
}
void launch_gemm_bf16x6(hipStream_t s, int M, int N, int K, const unsigned short* A, size_t a_plane,
                        const unsigned short* B, size_t b_plane, double* D, int ldd) {
  hipLaunchKernelGGL(k_gemm_bf16x6, dim3((N + 63) / 64, (M + 63) / 64), dim3(256), 0, s, M, N, K, A, a_plane, B,
                     b_plane, D, ldd);
}

}  // namespace cpm
