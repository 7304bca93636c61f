// Dense linear algebra of the constant-potential solve, all FP64:
//   * elastance matrix A (paper Eq. 3): Gaussian-Gaussian real-space pairs,
//     k-space as 2 k_e C C^T from the cos/sin factor matrix, self term;
//   * its inverse by blocked Gauss-Jordan elimination without pivoting (A is
//     symmetric positive definite for alpha < eta/sqrt2, so every pivot block
//     is too; a non-positive pivot reports CPM_ENOTSPD);
//   * the projections S = A^-1 - u u^T/(e.u), u = A^-1 e (Eq. 8-9), and for
//     the doubled cell S <- S - w w^T/(e1.w), w = S e1 (Eq. 14-15);
//   * the per-step charge solve q = S b + dV S c (one wavefront per row,
//     streaming S once) and the energy reductions.
#include "common.h"

namespace cpm {

// ------------------------------------------------------------ elastance

__global__ __launch_bounds__(256) void k_elastance_real(int n, const double* __restrict__ ex,
                                                        const double* __restrict__ ey, const double* __restrict__ ez,
                                                        Cell cell, double alpha, double eta, double rc2,
                                                        double self_term, double* __restrict__ A) {
  const int j = blockIdx.x * 16 + (threadIdx.x & 15);
  const int i = blockIdx.y * 16 + (threadIdx.x >> 4);
  if (i >= n || j >= n) return;
  const double eta2 = eta * 0.70710678118654752;   // eta / sqrt(2)
  double dx0 = min_image(ex[i] - ex[j], cell.L[0], cell.invL[0]);
  double dy0 = min_image(ey[i] - ey[j], cell.L[1], cell.invL[1]);
  double dz0 = min_image(ez[i] - ez[j], cell.L[2], cell.invL[2]);
  double acc = 0.0;
  for (int a = -cell.img[0]; a <= cell.img[0]; ++a)
    for (int b = -cell.img[1]; b <= cell.img[1]; ++b)
      for (int c = -cell.img[2]; c <= cell.img[2]; ++c) {
        if (i == j && a == 0 && b == 0 && c == 0) continue;
        double dx = dx0 + a * cell.L[0], dy = dy0 + b * cell.L[1], dz = dz0 + c * cell.L[2];
        double r2 = dx * dx + dy * dy + dz * dz;
        if (r2 < rc2) {
          double r = sqrt(r2);
          acc += (erfc(alpha * r) - erfc(eta2 * r)) / r;
        }
      }
  if (i == j) acc += self_term;
  A[(size_t)i * n + j] = KE * acc;
}

// C[i][c] for the k-vectors k0 .. k0+nkc-1: c < nkc -> s_k cos(k.r_i),
// c >= nkc -> s_k sin(k.r_i), s_k = sqrt(2 k_e w(k)); row-major n x 2 nkc
__global__ __launch_bounds__(256) void k_phase_matrix(int n, int nkc, int k0, int nk, const double* __restrict__ kv,
                                                      const double* __restrict__ sk, const double* __restrict__ ex,
                                                      const double* __restrict__ ey, const double* __restrict__ ez,
                                                      double* __restrict__ C) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  const int i = blockIdx.y;
  if (c >= nkc) return;
  const int k = k0 + c;
  double s, co;
  sincos(kv[k] * ex[i] + kv[nk + k] * ey[i] + kv[2 * nk + k] * ez[i], &s, &co);
  C[(size_t)i * 2 * nkc + c] = sk[k] * co;
  C[(size_t)i * 2 * nkc + nkc + c] = sk[k] * s;
}

__global__ void k_symmetrize(int n, double* __restrict__ A) {
  const int j = blockIdx.x * 16 + (threadIdx.x & 15);
  const int i = blockIdx.y * 16 + (threadIdx.x >> 4);
  if (i >= n || j >= n || j <= i) return;
  double a = A[(size_t)i * n + j], b = A[(size_t)j * n + i];
  double m = 0.5 * (a + b);
  A[(size_t)i * n + j] = m;
  A[(size_t)j * n + i] = m;
}

// ---------------------------------------------------- Gauss-Jordan inverse

constexpr int GJ_NB = GJ_BLOCK;

// Invert the nb x nb diagonal block at k0 in LDS (Gauss-Jordan, no
// pivoting); Dinv -> dinv; flag on a non-positive or non-finite pivot.
__global__ __launch_bounds__(256) void k_gj_pivot(int n, int k0, int nb, const double* __restrict__ A,
                                                  double* __restrict__ dinv, int* __restrict__ flag) {
  __shared__ double D[GJ_NB][GJ_NB + 1];
  __shared__ double prow[GJ_NB], pcol[GJ_NB];
  __shared__ double piv;
  for (int t = threadIdx.x; t < nb * nb; t += blockDim.x) {
    int r = t / nb, c = t % nb;
    D[r][c] = A[(size_t)(k0 + r) * n + k0 + c];
  }
  __syncthreads();
  for (int p = 0; p < nb; ++p) {
    if (threadIdx.x == 0) {
      piv = D[p][p];
      if (!(piv > 0.0) || !isfinite(piv)) { atomicOr(flag, 1); piv = 1.0; }
    }
    __syncthreads();
    double ip = 1.0 / piv;
    for (int t = threadIdx.x; t < nb; t += blockDim.x) { prow[t] = D[p][t]; pcol[t] = D[t][p]; }
    __syncthreads();
    for (int t = threadIdx.x; t < nb * nb; t += blockDim.x) {
      int r = t / nb, c = t % nb;
      double v;
      if (r == p && c == p) v = ip;
      else if (r == p) v = prow[c] * ip;
      else if (c == p) v = -pcol[r] * ip;
      else v = D[r][c] - pcol[r] * prow[c] * ip;
      D[r][c] = v;
    }
    __syncthreads();
  }
  for (int t = threadIdx.x; t < nb * nb; t += blockDim.x) {
    int r = t / nb, c = t % nb;
    dinv[r * nb + c] = D[r][c];
  }
}

// Panels: pc[i][t] = A[i][k0+t] (column block, i outside the pivot rows is
// what the update needs) and rx[t][j] = (Dinv A[k0.., j]) for j outside the
// block, Dinv[t][j-k0] inside it.
__global__ __launch_bounds__(256) void k_gj_panels(int n, int k0, int nb, const double* __restrict__ A,
                                                   const double* __restrict__ dinv, double* __restrict__ pc,
                                                   double* __restrict__ rx) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  for (int t = 0; t < nb; ++t) pc[(size_t)j * nb + t] = A[(size_t)j * n + k0 + t];
  if (j >= k0 && j < k0 + nb) {
    for (int t = 0; t < nb; ++t) rx[(size_t)t * n + j] = dinv[t * nb + (j - k0)];
  } else {
    double col[GJ_NB];
    for (int t = 0; t < nb; ++t) col[t] = A[(size_t)(k0 + t) * n + j];
    for (int t = 0; t < nb; ++t) {
      double s = 0.0;
      for (int u = 0; u < nb; ++u) s += dinv[t * nb + u] * col[u];
      rx[(size_t)t * n + j] = s;
    }
  }
}

// A[i][j] = rx[i-k0][j] for i in the block, else (j in block ? 0 : A[i][j]) - sum_t pc[i][t] rx[t][j]
__global__ __launch_bounds__(256) void k_gj_update(int n, int k0, int nb, double* __restrict__ A,
                                                   const double* __restrict__ pc, const double* __restrict__ rx) {
  __shared__ double Ps[64][GJ_NB + 1];
  __shared__ double Rs[GJ_NB][64 + 1];
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  const int i0 = blockIdx.y * 64, j0 = blockIdx.x * 64;
  for (int t = threadIdx.x; t < 64 * nb; t += 256) {
    int r = t / nb, c = t % nb;
    Ps[r][c] = (i0 + r < n) ? pc[(size_t)(i0 + r) * nb + c] : 0.0;
  }
  for (int t = threadIdx.x; t < nb * 64; t += 256) {
    int r = t / 64, c = t % 64;
    Rs[r][c] = (j0 + c < n) ? rx[(size_t)r * n + j0 + c] : 0.0;
  }
  __syncthreads();
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      int li = ty + 16 * u, lj = tx + 16 * v;
      int gi = i0 + li, gj = j0 + lj;
      if (gi >= n || gj >= n) continue;
      double* a = A + (size_t)gi * n + gj;
      if (gi >= k0 && gi < k0 + nb) {
        *a = Rs[gi - k0][lj];
      } else {
        double s = 0.0;
        for (int t = 0; t < nb; ++t) s = fma(Ps[li][t], Rs[t][lj], s);
        double base = (gj >= k0 && gj < k0 + nb) ? 0.0 : *a;
        *a = base - s;
      }
    }
}

// ------------------------------------------------------------ projections

// y[i] = sum_j M[i][j] x[j] (x == nullptr: x = 1); one wavefront per row
__global__ __launch_bounds__(256) void k_matvec(int n, const double* __restrict__ Mx, const double* __restrict__ x,
                                                double* __restrict__ y) {
  const int lane = threadIdx.x & (WAVE - 1);
  const int i = blockIdx.x * (blockDim.x / WAVE) + (threadIdx.x >> 6);
  if (i >= n) return;
  const double* row = Mx + (size_t)i * n;
  double acc = 0.0;
  for (int j = lane; j < n; j += WAVE) acc += row[j] * (x ? x[j] : 1.0);
  acc = wave_sum(acc);
  if (lane == 0) y[i] = acc;
}

// out[0] = sum_i a[i] * (b ? b[i] : 1)  (one workgroup)
__global__ __launch_bounds__(256) void k_dot(int n, const double* __restrict__ a, const double* __restrict__ b,
                                             double* __restrict__ out) {
  __shared__ double red[4];
  double acc = 0.0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) acc += a[i] * (b ? b[i] : 1.0);
  acc = wave_sum(acc);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) out[0] = red[0] + red[1] + red[2] + red[3];
}

// S[i][j] -= u_i u_j / s
__global__ void k_rank1(int n, double* __restrict__ S, const double* __restrict__ u, const double* __restrict__ s) {
  const int j = blockIdx.x * 16 + (threadIdx.x & 15);
  const int i = blockIdx.y * 16 + (threadIdx.x >> 4);
  if (i >= n || j >= n) return;
  S[(size_t)i * n + j] -= u[i] * u[j] / s[0];
}

// ------------------------------------------------------------ charge solve

// Q0 = S b (per frame), q = Q0 + dv Sc; one wavefront per row, four
// independent accumulators so that four row loads per lane are in flight
__global__ __launch_bounds__(256) void k_charges(int n, const double* __restrict__ S, const double* __restrict__ b_all,
                                                 const double* __restrict__ Sc, double dv,
                                                 double* __restrict__ Q0_all, double* __restrict__ q_all,
                                                 const int* __restrict__ epos, double* __restrict__ qs_all) {
  const int lane = threadIdx.x & (WAVE - 1);
  const int i = blockIdx.x * (blockDim.x / WAVE) + (threadIdx.x >> 6);
  const int frame = blockIdx.y;
  if (i >= n) return;
  const double* b = b_all + (size_t)frame * n;
  const int ep = qs_all ? epos[i] : 0;      // read now, used at the end
  double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
  if ((n & 1) == 0) {       // rows are 16-byte aligned: stream them as double2
    const double2* row = reinterpret_cast<const double2*>(S + (size_t)i * n);
    const double2* b2 = reinterpret_cast<const double2*>(b);
    const int n2 = n >> 1;
    int j = lane;
    for (; j + 3 * WAVE < n2; j += 4 * WAVE) {
      const double2 s0 = row[j], s1 = row[j + WAVE], s2 = row[j + 2 * WAVE], s3 = row[j + 3 * WAVE];
      const double2 v0 = b2[j], v1 = b2[j + WAVE], v2 = b2[j + 2 * WAVE], v3 = b2[j + 3 * WAVE];
      a0 = fma(s0.x, v0.x, fma(s0.y, v0.y, a0));
      a1 = fma(s1.x, v1.x, fma(s1.y, v1.y, a1));
      a2 = fma(s2.x, v2.x, fma(s2.y, v2.y, a2));
      a3 = fma(s3.x, v3.x, fma(s3.y, v3.y, a3));
    }
    for (; j < n2; j += WAVE) {
      const double2 s0 = row[j], v0 = b2[j];
      a0 = fma(s0.x, v0.x, fma(s0.y, v0.y, a0));
    }
  } else {
    const double* row = S + (size_t)i * n;
    for (int j = lane; j < n; j += WAVE) a0 = fma(row[j], b[j], a0);
  }
  const double acc = wave_sum((a0 + a1) + (a2 + a3));
  if (lane == 0) {
    const size_t o = (size_t)frame * n + i;
    const double qv = acc + dv * Sc[i];
    if (Q0_all) Q0_all[o] = acc;
    if (q_all) q_all[o] = qv;
    if (qs_all) qs_all[(size_t)frame * n + ep] = qv;      // cell-sorted copy
  }
}

// dst[f][epos[i]] = src[f][i]: charges of every frame in the electrodes'
// cell-sorted order (what the pair walkers stream)
__global__ __launch_bounds__(256) void k_permute(int n, const int* __restrict__ epos, const double* __restrict__ src,
                                                 double* __restrict__ dst) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const size_t f = blockIdx.y;
  if (i < n) dst[f * n + epos[i]] = src[f * n + i];
}

// ------------------------------------------------------------ energies

__device__ double block_sum(double v, double* red) {
  v = wave_sum(v);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double s = 0.0;
  for (int w = 0; w < (int)(blockDim.x >> 6); ++w) s += red[w];
  return s;
}


// q[f][v][i] = Q0[f][i] + dv[v] Sc[i]
__global__ __launch_bounds__(256) void k_expand_charges(int n_elec, int n_dv, const double* __restrict__ dv,
                                                        const double* __restrict__ Q0, const double* __restrict__ Sc,
                                                        double* __restrict__ q) {
  // a thread takes atom i of frame f over the whole sweep (its two inputs
  // read once, every store a run of consecutive atoms)
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int f = blockIdx.y;
  if (i >= n_elec) return;
  const double a = Q0[(size_t)f * n_elec + i], b = Sc[i];
  double* o = q + (size_t)f * n_dv * n_elec + i;
  for (int v = 0; v < n_dv; ++v) o[(size_t)v * n_elec] = a + dv[v] * b;
}

// out[f][v][k] = comp[f][0][k] + dv[v] comp[f][1][k], k < n3: the forces are
// affine in dV, so the sweep is written from two vectors per frame, every
// store a full run of consecutive values
__global__ __launch_bounds__(256) void k_expand_forces(int n3, int n_dv, const double* __restrict__ dv,
                                                       const double* __restrict__ comp, double* __restrict__ out) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  const int f = blockIdx.y;
  if (k >= n3) return;
  const double a = comp[(size_t)f * 2 * n3 + k];
  const double b = comp[(size_t)f * 2 * n3 + n3 + k];
  double* o = out + (size_t)f * n_dv * n3 + k;
  for (int v = 0; v < n_dv; ++v) o[(size_t)v * n3] = a + dv[v] * b;
}

// ------------------------------------------------------------ adjoint

// g = 2 (q - t) + dv c   (the right-hand side of lambda = S g)
__global__ __launch_bounds__(256) void k_adjoint_rhs(int n, const double* __restrict__ q, const double* __restrict__ t,
                                                     const double* __restrict__ c, double dv, double* __restrict__ g) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) g[i] = 2.0 * (q[i] - t[i]) + dv * c[i];
}

// qa = q - lambda  (electrode charges of the adjoint force pass)
// (and its cell-sorted copy out_s[epos[i]])
__global__ __launch_bounds__(256) void k_sub(int n, const double* __restrict__ a, const double* __restrict__ b,
                                             double* __restrict__ out, const int* __restrict__ epos,
                                             double* __restrict__ out_s) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) {
    const double v = a[i] - b[i];
    out[i] = v;
    if (out_s) out_s[epos[i]] = v;
  }
}

// loss = sum (q - t)^2 + U_coul;  dL/ddV = lambda . c   (one workgroup)
__global__ __launch_bounds__(256) void k_grad_finish(int n, const double* __restrict__ q, const double* __restrict__ t,
                                                     const double* __restrict__ lam, const double* __restrict__ c,
                                                     const double* __restrict__ energy, double* __restrict__ loss,
                                                     double* __restrict__ dldv) {
  __shared__ double red[4];
  double a = 0.0, b = 0.0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    double d = q[i] - t[i];
    a += d * d;
    b += lam[i] * c[i];
  }
  double A = block_sum(a, red);
  double B = block_sum(b, red);
  if (threadIdx.x == 0) {
    loss[0] = A + energy[0];
    dldv[0] = B;
  }
}

// ------------------------------------------------------------ launchers

void launch_adjoint_rhs(hipStream_t s, int n, const double* q, const double* t, const double* c, double dv, double* g) {
  hipLaunchKernelGGL(k_adjoint_rhs, dim3((n + 255) / 256), dim3(256), 0, s, n, q, t, c, dv, g);
}
void launch_sub(hipStream_t s, int n, const double* a, const double* b, double* out, const int* epos, double* out_s) {
  hipLaunchKernelGGL(k_sub, dim3((n + 255) / 256), dim3(256), 0, s, n, a, b, out, epos, out_s);
}
void launch_grad_finish(hipStream_t s, int n, const double* q, const double* t, const double* lam, const double* c,
                        const double* energy, double* loss, double* dldv) {
  hipLaunchKernelGGL(k_grad_finish, dim3(1), dim3(256), 0, s, n, q, t, lam, c, energy, loss, dldv);
}

void launch_elastance_real(hipStream_t s, int n, const double* ex, const double* ey, const double* ez,
                           const Cell& cell, double alpha, double eta, double rcut, double self_term, double* A) {
  dim3 grid((n + 15) / 16, (n + 15) / 16);
  hipLaunchKernelGGL(k_elastance_real, grid, dim3(256), 0, s, n, ex, ey, ez, cell, alpha, eta, rcut * rcut,
                     self_term, A);
}
void launch_phase_matrix(hipStream_t s, int n, int nkc, int k0, int nk, const double* kv, const double* sk,
                         const double* ex, const double* ey, const double* ez, double* C) {
  hipLaunchKernelGGL(k_phase_matrix, dim3((nkc + 255) / 256, n), dim3(256), 0, s, n, nkc, k0, nk, kv, sk, ex, ey,
                     ez, C);
}
void launch_symmetrize(hipStream_t s, int n, double* A) {
  hipLaunchKernelGGL(k_symmetrize, dim3((n + 15) / 16, (n + 15) / 16), dim3(256), 0, s, n, A);
}
void launch_gj_invert(hipStream_t s, int n, double* A, double* dinv, double* pc, double* rx, int* flag) {
  for (int k0 = 0; k0 < n; k0 += GJ_NB) {
    int nb = n - k0 < GJ_NB ? n - k0 : GJ_NB;
    hipLaunchKernelGGL(k_gj_pivot, dim3(1), dim3(256), 0, s, n, k0, nb, A, dinv, flag);
    hipLaunchKernelGGL(k_gj_panels, dim3((n + 255) / 256), dim3(256), 0, s, n, k0, nb, A, dinv, pc, rx);
    hipLaunchKernelGGL(k_gj_update, dim3((n + 63) / 64, (n + 63) / 64), dim3(256), 0, s, n, k0, nb, A, pc, rx);
  }
}
void launch_matvec(hipStream_t s, int n, const double* Mx, const double* x, double* y) {
  hipLaunchKernelGGL(k_matvec, dim3((n + 3) / 4), dim3(256), 0, s, n, Mx, x, y);
}
void launch_dot(hipStream_t s, int n, const double* a, const double* b, double* out) {
  hipLaunchKernelGGL(k_dot, dim3(1), dim3(256), 0, s, n, a, b, out);
}
void launch_rank1(hipStream_t s, int n, double* S, const double* u, const double* sc) {
  hipLaunchKernelGGL(k_rank1, dim3((n + 15) / 16, (n + 15) / 16), dim3(256), 0, s, n, S, u, sc);
}
void launch_charges(hipStream_t s, int n_frames, int n, const double* S, const double* b, const double* Sc, double dv,
                    double* Q0, double* q, const int* epos, double* qs) {
  hipLaunchKernelGGL(k_charges, dim3((n + 3) / 4, n_frames), dim3(256), 0, s, n, S, b, Sc, dv, Q0, q, epos, qs);
}
void launch_permute(hipStream_t s, int n_frames, int n, const int* epos, const double* src, double* dst) {
  if (n == 0 || n_frames == 0) return;
  hipLaunchKernelGGL(k_permute, dim3((n + 255) / 256, n_frames), dim3(256), 0, s, n, epos, src, dst);
}
void launch_expand_forces(hipStream_t s, int n_frames, int n_site, int n_dv, const double* dv, const double* comp,
                          double* out) {
  const int n3 = 3 * n_site;
  if (n3 == 0 || n_frames == 0) return;
  hipLaunchKernelGGL(k_expand_forces, dim3((n3 + 255) / 256, n_frames), dim3(256), 0, s, n3, n_dv, dv, comp, out);
}
void launch_expand_charges(hipStream_t s, int n_frames, int n_elec, int n_dv, const double* dv, const double* Q0,
                           const double* Sc, double* q) {
  hipLaunchKernelGGL(k_expand_charges, dim3((n_elec + 255) / 256, n_frames), dim3(256), 0, s, n_elec, n_dv, dv, Q0, Sc,
                     q);
}

}  // namespace cpm
