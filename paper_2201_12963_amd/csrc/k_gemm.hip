// Dense contractions on the matrix cores (gfx950).
//
// Both GEMMs here are "NT": D[m][n] = sum_k A[m][k] B[n][k], both operands
// with k contiguous, which is how the batched charge step Q0 = B S^T (frames
// x atoms times the symmetric atoms x atoms S) and the k-space part of the
// elastance, 2 C C^T, are stored.
//
// FP64: v_mfma_f64_16x16x4 (the path's FP64 arithmetic, unchanged).  A
// 256-thread workgroup owns a 64 x 64 tile of D, each wavefront a 32 x 32
// quarter as 2 x 2 MFMA blocks; operand slabs of 64 rows x 16 k go through
// LDS with two buffers, the next slab's global loads in flight while the
// current one is multiplied (one barrier per slab).
//
// Mixed form: the three-term bf16 split of both operands (x = x0 + x1 + x2,
// six products x_a y_b with a + b <= 2, FP32 accumulation), on
// v_mfma_f32_16x16x32_bf16: slabs of 64 rows x 32 k per split term, 16-byte
// global and LDS accesses, the same tiling and double buffering.
//
// MFMA lane layouts (16 x 16 blocks): operand lane l carries row (or column)
// l % 16 and the k values (l / 16) * kw .. (l / 16) * kw + kw - 1 (kw = 1 for
// f64 x4, 8 for bf16 x32).  Result lane l holds column l % 16 in four
// values t = 0..3: rows 4 t + l / 16 for f64 (interleaved), rows
// 4 (l / 16) + t for the f32 results of the bf16 products (measured with a
// one-wavefront probe of each builtin).
#include "common.h"

namespace cpm {

typedef double double4_t __attribute__((ext_vector_type(4)));
typedef float float4_t __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));

constexpr int G64_TILE = 64, G64_K = 16, G64_LD = G64_K + 1;   // LDS rows padded against bank conflicts

__global__ __launch_bounds__(256) void k_gemm_f64_mfma(int M, int N, int K, double alpha, const double* __restrict__ A,
                                                       int lda, const double* __restrict__ B, int ldb, double beta,
                                                       double* __restrict__ D, int ldd) {
  __shared__ double sA[2][G64_TILE * G64_LD], sB[2][G64_TILE * G64_LD];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int m0 = blockIdx.y * G64_TILE, n0 = blockIdx.x * G64_TILE;
  const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
  // loader: thread t moves 4 consecutive k of row t / 4 of each operand
  const int lrow = threadIdx.x >> 2, lk = (threadIdx.x & 3) * 4;
  const int ga = m0 + lrow, gb = n0 + lrow;
  const bool vec = ((lda | ldb) & 1) == 0 && ((reinterpret_cast<uintptr_t>(A) | reinterpret_cast<uintptr_t>(B)) & 15) == 0;
  double ra[4], rb[4];
  auto load = [&](int k0) {
    const int k = k0 + lk;
    if (vec && k + 3 < K) {
      if (ga < M) {
        const double2 v0 = *reinterpret_cast<const double2*>(A + (size_t)ga * lda + k);
        const double2 v1 = *reinterpret_cast<const double2*>(A + (size_t)ga * lda + k + 2);
        ra[0] = v0.x; ra[1] = v0.y; ra[2] = v1.x; ra[3] = v1.y;
      } else {
        ra[0] = ra[1] = ra[2] = ra[3] = 0.0;
      }
      if (gb < N) {
        const double2 v0 = *reinterpret_cast<const double2*>(B + (size_t)gb * ldb + k);
        const double2 v1 = *reinterpret_cast<const double2*>(B + (size_t)gb * ldb + k + 2);
        rb[0] = v0.x; rb[1] = v0.y; rb[2] = v1.x; rb[3] = v1.y;
      } else {
        rb[0] = rb[1] = rb[2] = rb[3] = 0.0;
      }
    } else {
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        ra[t] = (ga < M && k + t < K) ? A[(size_t)ga * lda + k + t] : 0.0;
        rb[t] = (gb < N && k + t < K) ? B[(size_t)gb * ldb + k + t] : 0.0;
      }
    }
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      sA[buf][lrow * G64_LD + lk + t] = ra[t];
      sB[buf][lrow * G64_LD + lk + t] = rb[t];
    }
  };
  double4_t acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = double4_t{0.0, 0.0, 0.0, 0.0};
  const int r = lane & 15, kq = lane >> 4;
  const int n_slabs = (K + G64_K - 1) / G64_K;
  load(0);
  store(0);
  __syncthreads();
  for (int s = 0; s < n_slabs; ++s) {
    const int buf = s & 1;
    if (s + 1 < n_slabs) load((s + 1) * G64_K);
    const double* pa = sA[buf];
    const double* pb = sB[buf];
#pragma unroll
    for (int kk = 0; kk < G64_K; kk += 4) {
      double av[2], bv[2];
#pragma unroll
      for (int a = 0; a < 2; ++a) av[a] = pa[(wm + 16 * a + r) * G64_LD + kk + kq];
#pragma unroll
      for (int b = 0; b < 2; ++b) bv[b] = pb[(wn + 16 * b + r) * G64_LD + kk + kq];
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[a], bv[b], acc[a][b], 0, 0, 0);
    }
    if (s + 1 < n_slabs) store(buf ^ 1);
    __syncthreads();
  }
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int gm = m0 + wm + 16 * a + 4 * t + kq, gn = n0 + wn + 16 * b + r;
        if (gm < M && gn < N) {
          double* d = D + (size_t)gm * ldd + gn;
          *d = (beta == 0.0 ? 0.0 : beta * *d) + alpha * acc[a][b][t];
        }
      }
}

// ---------------------------------------------------------- bf16 x 6 products

constexpr int GB_TILE = 64, GB_K = 32, GB_LD = GB_K + 8;   // rows of 40 bf16 (80 B): 16-byte aligned, skewed banks

__global__ __launch_bounds__(256) void k_gemm_bf16x6_mfma(int M, int N, int K, const unsigned short* __restrict__ A,
                                                          size_t a_plane, const unsigned short* __restrict__ B,
                                                          size_t b_plane, double* __restrict__ D, int ldd) {
  // [buffer][term][row * GB_LD + k]
  __shared__ __align__(16) unsigned short sA[2][3][GB_TILE * GB_LD], sB[2][3][GB_TILE * GB_LD];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int m0 = blockIdx.y * GB_TILE, n0 = blockIdx.x * GB_TILE;
  const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
  // loader: thread t moves 8 consecutive k (16 bytes) of row t / 4 of each term of each operand
  const int lrow = threadIdx.x >> 2, lk = (threadIdx.x & 3) * 8;
  const int ga = m0 + lrow, gb = n0 + lrow;
  uint4 ra[3], rb[3];
  auto load = [&](int k0) {
#pragma unroll
    for (int p = 0; p < 3; ++p) {
      ra[p] = ga < M ? *reinterpret_cast<const uint4*>(A + p * a_plane + (size_t)ga * K + k0 + lk) : uint4{0, 0, 0, 0};
      rb[p] = gb < N ? *reinterpret_cast<const uint4*>(B + p * b_plane + (size_t)gb * K + k0 + lk) : uint4{0, 0, 0, 0};
    }
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int p = 0; p < 3; ++p) {
      *reinterpret_cast<uint4*>(&sA[buf][p][lrow * GB_LD + lk]) = ra[p];
      *reinterpret_cast<uint4*>(&sB[buf][p][lrow * GB_LD + lk]) = rb[p];
    }
  };
  float4_t acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = float4_t{0.f, 0.f, 0.f, 0.f};
  const int r = lane & 15, kq = (lane >> 4) * 8;
  const int n_slabs = K / GB_K;
  load(0);
  store(0);
  __syncthreads();
  for (int s = 0; s < n_slabs; ++s) {
    const int buf = s & 1;
    if (s + 1 < n_slabs) load((s + 1) * GB_K);
    bf16x8_t av[3][2], bv[3][2];
#pragma unroll
    for (int p = 0; p < 3; ++p) {
#pragma unroll
      for (int a = 0; a < 2; ++a)
        av[p][a] = *reinterpret_cast<const bf16x8_t*>(&sA[buf][p][(wm + 16 * a + r) * GB_LD + kq]);
#pragma unroll
      for (int b = 0; b < 2; ++b)
        bv[p][b] = *reinterpret_cast<const bf16x8_t*>(&sB[buf][p][(wn + 16 * b + r) * GB_LD + kq]);
    }
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        // smallest products first
        acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[1][a], bv[1][b], acc[a][b], 0, 0, 0);
        acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[2][a], bv[0][b], acc[a][b], 0, 0, 0);
        acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[0][a], bv[2][b], acc[a][b], 0, 0, 0);
        acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[1][a], bv[0][b], acc[a][b], 0, 0, 0);
        acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[0][a], bv[1][b], acc[a][b], 0, 0, 0);
        acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[0][a], bv[0][b], acc[a][b], 0, 0, 0);
      }
    if (s + 1 < n_slabs) store(buf ^ 1);
    __syncthreads();
  }
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int gm = m0 + wm + 16 * a + 4 * (lane >> 4) + t, gn = n0 + wn + 16 * b + r;
        if (gm < M && gn < N) D[(size_t)gm * ldd + gn] = (double)acc[a][b][t];
      }
}

void launch_gemm_nt(hipStream_t s, int M, int N, int K, double alpha, const double* A, int lda, const double* B,
                    int ldb, double beta, double* D, int ldd) {
  if (M <= 0 || N <= 0) return;
  hipLaunchKernelGGL(k_gemm_f64_mfma, dim3((N + G64_TILE - 1) / G64_TILE, (M + G64_TILE - 1) / G64_TILE), dim3(256), 0,
                     s, M, N, K, alpha, A, lda, B, ldb, beta, D, ldd);
}

void launch_gemm_bf16x6(hipStream_t s, int M, int N, int K, const unsigned short* A, size_t a_plane,
                        const unsigned short* B, size_t b_plane, double* D, int ldd) {
  if (M <= 0 || N <= 0) return;
  hipLaunchKernelGGL(k_gemm_bf16x6_mfma, dim3((N + GB_TILE - 1) / GB_TILE, (M + GB_TILE - 1) / GB_TILE), dim3(256), 0,
                     s, M, N, K, A, a_plane, B, b_plane, D, ldd);
}

}  // namespace cpm
