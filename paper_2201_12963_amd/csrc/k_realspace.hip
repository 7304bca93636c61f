// Real-space (short-range) sums of the Ewald splitting with Gaussian electrode
// charges (paper Eq. 1-3):
//   electrolyte potential at electrode i:  k_e sum_j Q_j g1(r),
//       g1(r) = [erfc(alpha r) - erfc(eta r)]/r,
//   force on site j: pairs with other sites through g0(r) = erfc(alpha r)/r
//   and with the electrode Gaussians through g1, plus the k-space field
//   interpolated from the mesh and, for the finite field, -Q_j dV/Lz along z.
//
// Layout: one 64-wide wavefront per target (an electrode, or a site), lanes
// test the candidate partners of the neighbouring cells and queue those
// inside the cutoff (see pair compaction below).  Partners
// are read from the cell-sorted SoA copies, so a wavefront's loads of one
// cell are contiguous; the 27 (or fewer, for cells that wrap onto
// themselves) neighbour cells cover every partner within rcut because cells
// are at least rcut wide.  Extra periodic images are looped over when the
// cell is shorter than 2 rcut.  Results are reduced across the wavefront
// with butterfly shuffles; no atomics, so every run sums in the same order.
#include "common.h"
#include "erfcx_cheb.h"

namespace cpm {

// erfcx(x) = exp(x^2) erfc(x) for 0 <= x <= ERFCX_XMAX: Clenshaw sum of the
// Chebyshev series in u(t), t = 2/(2 + x) (coefficients in erfcx_cheb.h)
__device__ __forceinline__ double erfcx_cheb(double x) {
  const double t = 2.0 / (2.0 + x);
  const double u = (t - ERFCX_TMIN) * (2.0 / (1.0 - ERFCX_TMIN)) - 1.0;
  double b1 = 0.0, b2 = 0.0;
#pragma unroll
  for (int k = ERFCX_DEG; k > 0; --k) {
    double b0 = fma(2.0 * u, b1, ERFCX_CHEB[k] - b2);
    b2 = b1;
    b1 = b0;
  }
  return fma(u, b1, ERFCX_CHEB[0] - b2);
}

// erfc(x) given e = exp(-x^2), 0 <= x <= ERFCX_XMAX (alpha rcut is checked
// against this bound when a context is created); float: the library erfcf
__device__ __forceinline__ double erfc_from_exp(double x, double e) { return e * erfcx_cheb(x); }
__device__ __forceinline__ float erfc_from_exp(float x, float) { return erfcf(x); }

__device__ __forceinline__ double t_exp(double x) { return exp(x); }
__device__ __forceinline__ float t_exp(float x) { return expf(x); }
__device__ __forceinline__ double t_sqrt(double x) { return sqrt(x); }
__device__ __forceinline__ float t_sqrt(float x) { return sqrtf(x); }

// ------------------------------------------------------- pair compaction
//
// Lanes first test candidates for r < rcut (cheap); the pairs inside the
// cutoff are appended to a per-wavefront LDS queue (ballot + popcount gives
// each lane its slot), and the transcendental pair terms are evaluated 64
// queued pairs at a time, so every lane of that pass does useful work.

template <typename T>
struct WaveQueue {
  static constexpr int CAP = 2 * WAVE;
  T* x; T* y; T* z; T* a; T* b;
  __device__ __forceinline__ void bind(T* base) {
    x = base; y = base + CAP; z = base + 2 * CAP; a = base + 3 * CAP; b = base + 4 * CAP;
  }
};

// append this lane's pair if `in`; returns the new queue length (< 2 * WAVE
// when called with fewer than WAVE entries queued)
template <typename T>
__device__ __forceinline__ int queue_push(WaveQueue<T>& q, int n, bool in, T dx, T dy, T dz, T a, T b) {
  const int lane = threadIdx.x & (WAVE - 1);
  const unsigned long long m = __ballot(in);
  if (in) {
    const int pos = n + __popcll(m & ((1ull << lane) - 1ull));
    q.x[pos] = dx; q.y[pos] = dy; q.z[pos] = dz; q.a[pos] = a; q.b[pos] = b;
  }
  __builtin_amdgcn_wave_barrier();
  return n + __popcll(m);
}

// drop the first WAVE entries (already consumed), moving the rest down
template <typename T>
__device__ __forceinline__ int queue_pop(WaveQueue<T>& q, int n) {
  const int lane = threadIdx.x & (WAVE - 1);
  const int rest = n - WAVE;
  T x = 0, y = 0, z = 0, a = 0, b = 0;
  if (lane < rest) { x = q.x[WAVE + lane]; y = q.y[WAVE + lane]; z = q.z[WAVE + lane]; a = q.a[WAVE + lane]; b = q.b[WAVE + lane]; }
  __builtin_amdgcn_wave_barrier();
  if (lane < rest) { q.x[lane] = x; q.y[lane] = y; q.z[lane] = z; q.a[lane] = a; q.b[lane] = b; }
  __builtin_amdgcn_wave_barrier();
  return rest;
}

// ------------------------------------------------------------------ b real

// erfc(eta r) and exp(-eta^2 r^2) are below 1e-18 for eta r > 6.5, far under
// FP64 resolution of the alpha terms they are added to, so they are skipped
// there (always the case for sites at least 0.33 nm from an electrode atom)
constexpr double ETA_R_SKIP = 6.5;

template <typename T>
__device__ __forceinline__ T g1_potential(T dx, T dy, T dz, T q, T alpha, T eta) {
  T r2 = dx * dx + dy * dy + dz * dz;
  T r = t_sqrt(r2);
  T e = erfc_from_exp(alpha * r, t_exp(-alpha * alpha * r2));
  if (eta * r < (T)ETA_R_SKIP) e -= erfc_from_exp(eta * r, t_exp(-eta * eta * r2));
  return q * e / r;
}

// Stencil cell number s of cell (cx, cy, cz): s enumerates the deduplicated
// neighbour offsets (z slowest).
__device__ __forceinline__ int stencil_linear(const Cell& cell, int cx, int cy, int cz, int s) {
  const int nsx = stencil_count(cell.nc[0]), nsy = stencil_count(cell.nc[1]);
  const int d = s % nsx, b = (s / nsx) % nsy, a = s / (nsx * nsy);
  const int xc = stencil_cell(cx, d, cell.nc[0]);
  const int yc = stencil_cell(cy, b, cell.nc[1]);
  const int zc = stencil_cell(cz, a, cell.nc[2]);
  return (zc * cell.nc[1] + yc) * cell.nc[0] + xc;
}

// B-spline weights of site `site` along `axis` for the orders in use
template <typename T>
__device__ __forceinline__ void site_spline(const MeshInfo& mi, T u, int axis, size_t n, size_t frame,
                                            size_t site, int* wfirst, T* w) {
  T wt[MAX_ORDER];
  int first;
  switch (mi.order) {
    case 4: first = spline_weights_p<4>(u, wt); break;
    case 5: first = spline_weights_p<5>(u, wt); break;
    case 6: first = spline_weights_p<6>(u, wt); break;
    default: first = spline_weights<T>(u, mi.order, wt); break;
  }
  const int K = mi.K[axis];
  first = ((first % K) + K) % K;
  wfirst[(frame * 3 + axis) * n + site] = first;
  for (int t = 0; t < mi.order; ++t) w[((frame * 3 + axis) * mi.order + t) * n + site] = wt[t];
}

// One wavefront per electrode atom.  The workgroups also compute the
// B-spline assignment of the sites for the mesh steps that follow, each
// workgroup taking a slice.
template <typename T>
__global__ __launch_bounds__(256) void k_real_b(Cell cell, T alpha, T eta, T rc2, ElecSet<T> el,
                                                SiteSet<T> st, T* __restrict__ phi_out, MeshInfo mi,
                                                int* __restrict__ wfirst_out, T* __restrict__ w_out) {
  __shared__ T qbuf[4][5 * WaveQueue<T>::CAP];
  const int lane = threadIdx.x & (WAVE - 1);
  const int g = blockIdx.x * (blockDim.x / WAVE) + (threadIdx.x >> 6);
  const int frame = blockIdx.y;
  const size_t fo = (size_t)frame * st.n;
  const T* sx = st.x + fo; const T* sy = st.y + fo; const T* sz = st.z + fo; const T* sq = st.q + fo;
  if (w_out) {
    const int per = (st.n + gridDim.x - 1) / gridDim.x;
    const int lo = blockIdx.x * per, hi = min(st.n, lo + per);
    for (int t = threadIdx.x; t < 3 * (hi - lo); t += blockDim.x) {
      const int site = lo + t / 3, axis = t % 3;
      const T x = axis == 0 ? sx[site] : (axis == 1 ? sy[site] : sz[site]);
      site_spline<T>(mi, x * (T)mi.invh[axis], axis, st.n, frame, site, wfirst_out, w_out);
    }
  }
  if (g >= el.n) return;
  WaveQueue<T> Q;
  Q.bind(qbuf[threadIdx.x >> 6]);
  const int* cs = st.cell_start + (size_t)frame * (cell.n_cells + 1);
  const T ex = el.x[g], ey = el.y[g], ez = el.z[g];
  const int c = el.cell[g];
  const int cx = c % cell.nc[0], cy = (c / cell.nc[0]) % cell.nc[1], cz = c / (cell.nc[0] * cell.nc[1]);
  const T L0 = (T)cell.L[0], L1 = (T)cell.L[1], L2 = (T)cell.L[2];
  const T i0 = (T)cell.invL[0], i1 = (T)cell.invL[1], i2 = (T)cell.invL[2];
  const int nst = stencil_count(cell.nc[0]) * stencil_count(cell.nc[1]) * stencil_count(cell.nc[2]);
  // site ranges of all stencil cells, loaded in parallel (lane t: cell t)
  int my_lo = 0, my_hi = 0;
  if (lane < nst) {
    int nc = stencil_linear(cell, cx, cy, cz, lane);
    my_lo = cs[nc];
    my_hi = cs[nc + 1];
  }
  T acc = 0;
  int n = 0;
  for (int t = 0; t < nst; ++t) {
    const int j0 = __shfl(my_lo, t, WAVE), j1 = __shfl(my_hi, t, WAVE);
    for (int base = j0; base < j1; base += WAVE) {
      const int j = base + lane;
      const bool valid = j < j1;
      T dx0 = 0, dy0 = 0, dz0 = 0, qj = 0;
      if (valid) {
        dx0 = min_image(ex - sx[j], L0, i0);
        dy0 = min_image(ey - sy[j], L1, i1);
        dz0 = min_image(ez - sz[j], L2, i2);
        qj = sq[j];
      }
      for (int ix = -cell.img[0]; ix <= cell.img[0]; ++ix)
        for (int iy = -cell.img[1]; iy <= cell.img[1]; ++iy)
          for (int iz = -cell.img[2]; iz <= cell.img[2]; ++iz) {
            T dx = dx0 + (T)ix * L0, dy = dy0 + (T)iy * L1, dz = dz0 + (T)iz * L2;
            bool in = valid && (dx * dx + dy * dy + dz * dz < rc2);
            n = queue_push(Q, n, in, dx, dy, dz, qj, (T)0);
            if (n >= WAVE) {
              acc += g1_potential(Q.x[lane], Q.y[lane], Q.z[lane], Q.a[lane], alpha, eta);
              n = queue_pop(Q, n);
            }
          }
    }
  }
  if (lane < n) acc += g1_potential(Q.x[lane], Q.y[lane], Q.z[lane], Q.a[lane], alpha, eta);
  acc = wave_sum(acc);
  if (lane == 0) phi_out[(size_t)frame * el.n + el.orig[g]] = (T)KE * acc;
}

template <typename T>
void launch_real_b_t(hipStream_t s, int n_frames, const Cell& cell, double alpha, double eta,
                     double rcut, const ElecSet<T>& el, const SiteSet<T>& st, T* phi_out,
                     const MeshInfo& mi, int* wfirst_out, T* w_out) {
  dim3 grid((el.n + 3) / 4, n_frames);
  hipLaunchKernelGGL(k_real_b<T>, grid, dim3(256), 0, s, cell, (T)alpha, (T)eta, (T)(rcut * rcut),
                     el, st, phi_out, mi, wfirst_out, w_out);
}

// ------------------------------------------------------------ site forces

// radial force factor g(r) = -(d kernel/dr)/r of a site pair (g0) and of a
// site-Gaussian pair (g1), and the site-pair potential erfc(alpha r)/r
template <typename T>
__device__ __forceinline__ void g0_terms(T r2, T alpha, T& g, T& pot) {
  const T two_over_sqrtpi = (T)1.1283791670955126;
  T r = t_sqrt(r2);
  T ir = (T)1 / r;
  T ex = t_exp(-alpha * alpha * r2);
  T ec = erfc_from_exp(alpha * r, ex);
  g = (ec * ir + two_over_sqrtpi * alpha * ex) * ir * ir;
  pot = ec * ir;
}
template <typename T>
__device__ __forceinline__ T g1_force(T r2, T alpha, T eta) {
  const T two_over_sqrtpi = (T)1.1283791670955126;
  T r = t_sqrt(r2);
  T ir = (T)1 / r;
  T ex = t_exp(-alpha * alpha * r2);
  T e = erfc_from_exp(alpha * r, ex);
  T x = alpha * ex;
  if (eta * r < (T)ETA_R_SKIP) {
    T exn = t_exp(-eta * eta * r2);
    e -= erfc_from_exp(eta * r, exn);
    x -= eta * exn;
  }
  return (e * ir + two_over_sqrtpi * x) * ir * ir;
}

// One wavefront per site: the k-space field is gathered with the stored
// B-spline weights (lanes over the P^3 mesh points), then the pair sums run
// over the cell ranges of the stencil, loaded in parallel up front.
template <typename T, bool TWO>
__global__ __launch_bounds__(256) void k_site_forces(Cell cell, ElecSet<T> el, SiteSet<T> st,
                                                     ForceArgs<T> fa) {
  __shared__ T qbuf[4][5 * WaveQueue<T>::CAP];
  const int lane = threadIdx.x & (WAVE - 1);
  const int j = blockIdx.x * (blockDim.x / WAVE) + (threadIdx.x >> 6);
  const int frame = blockIdx.y;
  if (j >= st.n) return;
  WaveQueue<T> Q;
  Q.bind(qbuf[threadIdx.x >> 6]);
  const size_t fo = (size_t)frame * st.n;
  const int* cs = st.cell_start + (size_t)frame * (cell.n_cells + 1);
  const T* sx = st.x + fo; const T* sy = st.y + fo; const T* sz = st.z + fo; const T* sq = st.q + fo;
  const T xj = sx[j], yj = sy[j], zj = sz[j], qj = sq[j];
  const T L0 = (T)cell.L[0], L1 = (T)cell.L[1], L2 = (T)cell.L[2];
  const T i0 = (T)cell.invL[0], i1 = (T)cell.invL[1], i2 = (T)cell.invL[2];
  const int c = cell_coord((double)xj, cell.L[0], cell.nc[0]) +
                cell.nc[0] * (cell_coord((double)yj, cell.L[1], cell.nc[1]) +
                              cell.nc[1] * cell_coord((double)zj, cell.L[2], cell.nc[2]));
  const int cx = c % cell.nc[0], cy = (c / cell.nc[0]) % cell.nc[1], cz = c / (cell.nc[0] * cell.nc[1]);
  const int nst = stencil_count(cell.nc[0]) * stencil_count(cell.nc[1]) * stencil_count(cell.nc[2]);
  // cell ranges of both lists for every stencil cell (lane t: cell t)
  int s_lo = 0, s_hi = 0, e_lo = 0, e_hi = 0;
  if (lane < nst) {
    int nc = stencil_linear(cell, cx, cy, cz, lane);
    s_lo = cs[nc]; s_hi = cs[nc + 1];
    e_lo = el.cell_start[nc]; e_hi = el.cell_start[nc + 1];
  }

  // ---- k-space field at the site: stored B-spline weights, lanes over points
  T ea[3] = {0, 0, 0}, eb[3] = {0, 0, 0};
  if (fa.Ea) {
    const int P = fa.mi.order;
    const int Kx = fa.mi.K[0], Ky = fa.mi.K[1], Kz = fa.mi.K[2], M = fa.mi.M;
    const size_t n = st.n;
    const int fx = st.wfirst[(frame * 3 + 0) * n + j];
    const int fy = st.wfirst[(frame * 3 + 1) * n + j];
    const int fz = st.wfirst[(frame * 3 + 2) * n + j];
    const T* Ef = fa.Ea + (size_t)frame * fa.Ea_frame_stride;
    for (int t = lane; t < P * P * P; t += WAVE) {
      int tx = t % P, ty = (t / P) % P, tz = t / (P * P);
      int ix = fx + tx; ix -= (ix >= Kx) ? Kx : 0;
      int iy = fy + ty; iy -= (iy >= Ky) ? Ky : 0;
      int iz = fz + tz; iz -= (iz >= Kz) ? Kz : 0;
      int m = (iz * Ky + iy) * Kx + ix;
      T w = st.w[((frame * 3 + 0) * P + tx) * n + j] * st.w[((frame * 3 + 1) * P + ty) * n + j] *
            st.w[((frame * 3 + 2) * P + tz) * n + j];
      ea[0] += w * Ef[m]; ea[1] += w * Ef[M + m]; ea[2] += w * Ef[2 * M + m];
      if (TWO) { eb[0] += w * fa.Eb[m]; eb[1] += w * fa.Eb[M + m]; eb[2] += w * fa.Eb[2 * M + m]; }
    }
  }
  if (fa.Esite && lane == 0) {
    const double* E = fa.Esite + (size_t)frame * 3 * st.n;
    ea[0] = (T)E[j]; ea[1] = (T)E[st.n + j]; ea[2] = (T)E[2 * st.n + j];
  }

  // ---- real space
  T fr[3] = {0, 0, 0};     // sum of pair force vectors / Q_j (without k_e)
  T frb[3] = {0, 0, 0};
  T u = 0;
  const double* qa = fa.qa + (size_t)frame * fa.qa_frame_stride;
  // pass 0: other sites (g0); pass 1: electrode Gaussians (g1)
  for (int pass = 0; pass < 2; ++pass) {
    int n = 0;
    const T* px = pass == 0 ? sx : el.x;
    const T* py = pass == 0 ? sy : el.y;
    const T* pz = pass == 0 ? sz : el.z;
    for (int t = 0; t < nst; ++t) {
      const int k0 = __shfl(pass == 0 ? s_lo : e_lo, t, WAVE);
      const int k1 = __shfl(pass == 0 ? s_hi : e_hi, t, WAVE);
      for (int base = k0; base < k1; base += WAVE) {
        const int k = base + lane;
        const bool valid = k < k1;
        T dx0 = 0, dy0 = 0, dz0 = 0, ca = 0, cb = 0;
        if (valid) {
          dx0 = min_image(xj - px[k], L0, i0);
          dy0 = min_image(yj - py[k], L1, i1);
          dz0 = min_image(zj - pz[k], L2, i2);
          if (pass == 0) {
            ca = sq[k];
          } else {
            int o = el.orig[k];
            ca = (T)qa[o];
            if (TWO) cb = (T)fa.qb[o];
          }
        }
        for (int ix = -cell.img[0]; ix <= cell.img[0]; ++ix)
          for (int iy = -cell.img[1]; iy <= cell.img[1]; ++iy)
            for (int iz = -cell.img[2]; iz <= cell.img[2]; ++iz) {
              T dx = dx0 + (T)ix * L0, dy = dy0 + (T)iy * L1, dz = dz0 + (T)iz * L2;
              bool self = pass == 0 && k == j && ix == 0 && iy == 0 && iz == 0;
              bool in = valid && !self && (dx * dx + dy * dy + dz * dz < fa.rc2);
              n = queue_push(Q, n, in, dx, dy, dz, ca, cb);
              if (n >= WAVE) {
                T qx = Q.x[lane], qy = Q.y[lane], qz = Q.z[lane], r2 = qx * qx + qy * qy + qz * qz;
                if (pass == 0) {
                  T g, pot;
                  g0_terms(r2, fa.alpha, g, pot);
                  T w = Q.a[lane] * g;
                  fr[0] += w * qx; fr[1] += w * qy; fr[2] += w * qz;
                  u += Q.a[lane] * pot;
                } else {
                  T g = g1_force(r2, fa.alpha, fa.eta);
                  T w = Q.a[lane] * g;
                  fr[0] += w * qx; fr[1] += w * qy; fr[2] += w * qz;
                  if (TWO) { T wb = Q.b[lane] * g; frb[0] += wb * qx; frb[1] += wb * qy; frb[2] += wb * qz; }
                }
                n = queue_pop(Q, n);
              }
            }
      }
    }
    if (lane < n) {
      T qx = Q.x[lane], qy = Q.y[lane], qz = Q.z[lane], r2 = qx * qx + qy * qy + qz * qz;
      if (pass == 0) {
        T g, pot;
        g0_terms(r2, fa.alpha, g, pot);
        T w = Q.a[lane] * g;
        fr[0] += w * qx; fr[1] += w * qy; fr[2] += w * qz;
        u += Q.a[lane] * pot;
      } else {
        T g = g1_force(r2, fa.alpha, fa.eta);
        T w = Q.a[lane] * g;
        fr[0] += w * qx; fr[1] += w * qy; fr[2] += w * qz;
        if (TWO) { T wb = Q.b[lane] * g; frb[0] += wb * qx; frb[1] += wb * qy; frb[2] += wb * qz; }
      }
    }
    __builtin_amdgcn_wave_barrier();
  }
  // ---- reduce and write
  double F[3], FB[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    double e_k = (double)wave_sum(ea[d]);
    double e_r = (double)wave_sum(fr[d]);
    F[d] = fa.out_scale * (double)qj * (e_k + KE * e_r);
    if (TWO) {
      double eb_k = (double)wave_sum(eb[d]);
      double eb_r = (double)wave_sum(frb[d]);
      FB[d] = fa.out_scale * (double)qj * (eb_k + KE * eb_r);
    } else {
      FB[d] = 0.0;
    }
  }
  F[2] += (double)qj * fa.field;
  FB[2] += (double)qj * fa.fieldb;
  double us = (double)wave_sum(u);
  const int orig = st.order[fo + j];
  double* fout = fa.f_out + (size_t)frame * fa.f_frame_stride;
  for (int v = lane; v < fa.n_dv; v += WAVE) {
    double dv = fa.dv ? fa.dv[v] : 0.0;
    double* o = fout + (size_t)v * 3 * st.n;
    o[orig] = F[0] + dv * FB[0];
    o[st.n + orig] = F[1] + dv * FB[1];
    o[2 * st.n + orig] = F[2] + dv * FB[2];
  }
  if (fa.u_site && lane == 0) fa.u_site[fo + j] = 0.5 * KE * (double)qj * us;
}

template <typename T>
void launch_site_forces_t(hipStream_t s, int n_frames, const Cell& cell, const ElecSet<T>& el,
                          const SiteSet<T>& st, const ForceArgs<T>& fa) {
  dim3 grid((st.n + 3) / 4, n_frames);
  if (fa.Eb || fa.qb)
    hipLaunchKernelGGL((k_site_forces<T, true>), grid, dim3(256), 0, s, cell, el, st, fa);
  else
    hipLaunchKernelGGL((k_site_forces<T, false>), grid, dim3(256), 0, s, cell, el, st, fa);
}

// explicit instantiations used by api.cpp
template void launch_real_b_t<double>(hipStream_t, int, const Cell&, double, double, double,
                                      const ElecSet<double>&, const SiteSet<double>&, double*,
                                      const MeshInfo&, int*, double*);
template void launch_real_b_t<float>(hipStream_t, int, const Cell&, double, double, double,
                                     const ElecSet<float>&, const SiteSet<float>&, float*,
                                     const MeshInfo&, int*, float*);
template void launch_site_forces_t<double>(hipStream_t, int, const Cell&, const ElecSet<double>&,
                                           const SiteSet<double>&, const ForceArgs<double>&);
template void launch_site_forces_t<float>(hipStream_t, int, const Cell&, const ElecSet<float>&,
                                          const SiteSet<float>&, const ForceArgs<float>&);

}  // namespace cpm
