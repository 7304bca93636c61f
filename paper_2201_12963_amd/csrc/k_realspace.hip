// Real-space (short-range) sums of the Ewald splitting with Gaussian electrode
// charges (paper Eq. 1-3):
//   electrolyte potential at electrode i:  k_e sum_j Q_j g1(r),
//       g1(r) = [erfc(alpha r) - erfc(eta r)]/r,
//   force on site j: pairs with other sites through g0(r) = erfc(alpha r)/r
//   and with the electrode Gaussians through g1, plus the k-space field
//   interpolated from the mesh and, for the finite field, -Q_j dV/Lz along z.
//
// Layout: one 64-wide wavefront per target (an electrode, or a site), lanes
// stride over the candidate partners of the neighbouring cells.  Partners
// are read from the cell-sorted SoA copies, so a wavefront's loads of one
// cell are contiguous; the 27 (or fewer, for cells that wrap onto
// themselves) neighbour cells cover every partner within rcut because cells
// are at least rcut wide.  Extra periodic images are looped over when the
// cell is shorter than 2 rcut.  Results are reduced across the wavefront
// with butterfly shuffles; no atomics, so every run sums in the same order.
#include "common.h"

namespace cpm {

__device__ __forceinline__ double t_erfc(double x) { return erfc(x); }
__device__ __forceinline__ float t_erfc(float x) { return erfcf(x); }
__device__ __forceinline__ double t_exp(double x) { return exp(x); }
__device__ __forceinline__ float t_exp(float x) { return expf(x); }
__device__ __forceinline__ double t_sqrt(double x) { return sqrt(x); }
__device__ __forceinline__ float t_sqrt(float x) { return sqrtf(x); }

// ------------------------------------------------------------------ b real

template <typename T>
__global__ __launch_bounds__(256) void k_real_b(Cell cell, T alpha, T eta, T rc2, ElecSet<T> el,
                                                SiteSet<T> st, T* __restrict__ phi_out) {
  const int lane = threadIdx.x & (WAVE - 1);
  const int g = blockIdx.x * (blockDim.x / WAVE) + (threadIdx.x >> 6);
  const int frame = blockIdx.y;
  if (g >= el.n) return;
  const size_t fo = (size_t)frame * st.n;
  const int* cs = st.cell_start + (size_t)frame * (cell.n_cells + 1);
  const T* sx = st.x + fo; const T* sy = st.y + fo; const T* sz = st.z + fo; const T* sq = st.q + fo;
  const T ex = el.x[g], ey = el.y[g], ez = el.z[g];
  const int c = el.cell[g];
  const int cx = c % cell.nc[0], cy = (c / cell.nc[0]) % cell.nc[1], cz = c / (cell.nc[0] * cell.nc[1]);
  const T L0 = (T)cell.L[0], L1 = (T)cell.L[1], L2 = (T)cell.L[2];
  const T i0 = (T)cell.invL[0], i1 = (T)cell.invL[1], i2 = (T)cell.invL[2];
  T acc = 0;
  const int nsx = stencil_count(cell.nc[0]), nsy = stencil_count(cell.nc[1]), nsz = stencil_count(cell.nc[2]);
  for (int a = 0; a < nsz; ++a) {
    int zc = stencil_cell(cz, a, cell.nc[2]);
    for (int b = 0; b < nsy; ++b) {
      int yc = stencil_cell(cy, b, cell.nc[1]);
      for (int d = 0; d < nsx; ++d) {
        int xc = stencil_cell(cx, d, cell.nc[0]);
        int nc = (zc * cell.nc[1] + yc) * cell.nc[0] + xc;
        for (int j = cs[nc] + lane; j < cs[nc + 1]; j += WAVE) {
          T dx0 = min_image(ex - sx[j], L0, i0);
          T dy0 = min_image(ey - sy[j], L1, i1);
          T dz0 = min_image(ez - sz[j], L2, i2);
          T qj = sq[j];
          for (int ix = -cell.img[0]; ix <= cell.img[0]; ++ix)
            for (int iy = -cell.img[1]; iy <= cell.img[1]; ++iy)
              for (int iz = -cell.img[2]; iz <= cell.img[2]; ++iz) {
                T dx = dx0 + (T)ix * L0, dy = dy0 + (T)iy * L1, dz = dz0 + (T)iz * L2;
                T r2 = dx * dx + dy * dy + dz * dz;
                if (r2 < rc2) {
                  T r = t_sqrt(r2);
                  acc += qj * (t_erfc(alpha * r) - t_erfc(eta * r)) / r;
                }
              }
        }
      }
    }
  }
  acc = wave_sum(acc);
  if (lane == 0) phi_out[(size_t)frame * el.n + el.orig[g]] = (T)KE * acc;
}

template <typename T>
void launch_real_b_t(hipStream_t s, int n_frames, const Cell& cell, double alpha, double eta,
                     double rcut, const ElecSet<T>& el, const SiteSet<T>& st, T* phi_out) {
  dim3 grid((el.n + 3) / 4, n_frames);
  hipLaunchKernelGGL(k_real_b<T>, grid, dim3(256), 0, s, cell, (T)alpha, (T)eta, (T)(rcut * rcut),
                     el, st, phi_out);
}

// ------------------------------------------------------------ site forces

template <typename T, bool TWO>
__global__ __launch_bounds__(256) void k_site_forces(Cell cell, ElecSet<T> el, SiteSet<T> st,
                                                     ForceArgs<T> fa) {
  const int lane = threadIdx.x & (WAVE - 1);
  const int j = blockIdx.x * (blockDim.x / WAVE) + (threadIdx.x >> 6);
  const int frame = blockIdx.y;
  if (j >= st.n) return;
  const size_t fo = (size_t)frame * st.n;
  const int* cs = st.cell_start + (size_t)frame * (cell.n_cells + 1);
  const T* sx = st.x + fo; const T* sy = st.y + fo; const T* sz = st.z + fo; const T* sq = st.q + fo;
  const T xj = sx[j], yj = sy[j], zj = sz[j], qj = sq[j];
  const T L0 = (T)cell.L[0], L1 = (T)cell.L[1], L2 = (T)cell.L[2];
  const T i0 = (T)cell.invL[0], i1 = (T)cell.invL[1], i2 = (T)cell.invL[2];
  const T two_over_sqrtpi = (T)1.1283791670955126;

  // ---- k-space field at the site: B-spline interpolation of the mesh
  T ea[3] = {0, 0, 0}, eb[3] = {0, 0, 0};
  if (fa.Ea) {
    const int P = fa.mi.order;
    T wx[MAX_ORDER], wy[MAX_ORDER], wz[MAX_ORDER];
    int fxi = spline_weights<T>(xj * (T)fa.mi.invh[0], P, wx);
    int fyi = spline_weights<T>(yj * (T)fa.mi.invh[1], P, wy);
    int fzi = spline_weights<T>(zj * (T)fa.mi.invh[2], P, wz);
    const int Kx = fa.mi.K[0], Ky = fa.mi.K[1], Kz = fa.mi.K[2], M = fa.mi.M;
    const T* Ef = fa.Ea + (size_t)frame * fa.Ea_frame_stride;
    for (int t = lane; t < P * P * P; t += WAVE) {
      int tx = t % P, ty = (t / P) % P, tz = t / (P * P);
      int ix = fxi + tx; ix = (ix % Kx + Kx) % Kx;
      int iy = fyi + ty; iy = (iy % Ky + Ky) % Ky;
      int iz = fzi + tz; iz = (iz % Kz + Kz) % Kz;
      int m = (iz * Ky + iy) * Kx + ix;
      T w = wx[tx] * wy[ty] * wz[tz];
      ea[0] += w * Ef[m]; ea[1] += w * Ef[M + m]; ea[2] += w * Ef[2 * M + m];
      if (TWO) { eb[0] += w * fa.Eb[m]; eb[1] += w * fa.Eb[M + m]; eb[2] += w * fa.Eb[2 * M + m]; }
    }
  }

  if (fa.Esite && lane == 0) {
    const double* E = fa.Esite + (size_t)frame * 3 * st.n;
    ea[0] = (T)E[j]; ea[1] = (T)E[st.n + j]; ea[2] = (T)E[2 * st.n + j];
  }

  // ---- real space
  T fr[3] = {0, 0, 0};     // sum of radial-force vectors / Q_j (without k_e)
  T frb[3] = {0, 0, 0};
  T u = 0;
  const int c = cell_coord((double)xj, cell.L[0], cell.nc[0]) +
                cell.nc[0] * (cell_coord((double)yj, cell.L[1], cell.nc[1]) +
                              cell.nc[1] * cell_coord((double)zj, cell.L[2], cell.nc[2]));
  const int cx = c % cell.nc[0], cy = (c / cell.nc[0]) % cell.nc[1], cz = c / (cell.nc[0] * cell.nc[1]);
  const int nsx = stencil_count(cell.nc[0]), nsy = stencil_count(cell.nc[1]), nsz = stencil_count(cell.nc[2]);
  const double* qa = fa.qa + (size_t)frame * fa.qa_frame_stride;
  for (int a = 0; a < nsz; ++a) {
    int zc = stencil_cell(cz, a, cell.nc[2]);
    for (int b = 0; b < nsy; ++b) {
      int yc = stencil_cell(cy, b, cell.nc[1]);
      for (int d = 0; d < nsx; ++d) {
        int xc = stencil_cell(cx, d, cell.nc[0]);
        int nc = (zc * cell.nc[1] + yc) * cell.nc[0] + xc;
        // electrolyte partners: g0
        for (int k = cs[nc] + lane; k < cs[nc + 1]; k += WAVE) {
          T dx0 = min_image(xj - sx[k], L0, i0);
          T dy0 = min_image(yj - sy[k], L1, i1);
          T dz0 = min_image(zj - sz[k], L2, i2);
          T qk = sq[k];
          for (int ix = -cell.img[0]; ix <= cell.img[0]; ++ix)
            for (int iy = -cell.img[1]; iy <= cell.img[1]; ++iy)
              for (int iz = -cell.img[2]; iz <= cell.img[2]; ++iz) {
                if (k == j && ix == 0 && iy == 0 && iz == 0) continue;
                T dx = dx0 + (T)ix * L0, dy = dy0 + (T)iy * L1, dz = dz0 + (T)iz * L2;
                T r2 = dx * dx + dy * dy + dz * dz;
                if (r2 < fa.rc2) {
                  T r = t_sqrt(r2);
                  T ir = (T)1 / r;
                  T ec = t_erfc(fa.alpha * r);
                  T g = (ec * ir + two_over_sqrtpi * fa.alpha * t_exp(-fa.alpha * fa.alpha * r2)) * ir * ir;
                  fr[0] += qk * g * dx; fr[1] += qk * g * dy; fr[2] += qk * g * dz;
                  u += qk * ec * ir;
                }
              }
        }
        // electrode partners: g1 with the Gaussian charges
        for (int k = el.cell_start[nc] + lane; k < el.cell_start[nc + 1]; k += WAVE) {
          T dx0 = min_image(xj - el.x[k], L0, i0);
          T dy0 = min_image(yj - el.y[k], L1, i1);
          T dz0 = min_image(zj - el.z[k], L2, i2);
          int o = el.orig[k];
          T qk = (T)qa[o];
          T qkb = TWO ? (T)fa.qb[o] : (T)0;
          for (int ix = -cell.img[0]; ix <= cell.img[0]; ++ix)
            for (int iy = -cell.img[1]; iy <= cell.img[1]; ++iy)
              for (int iz = -cell.img[2]; iz <= cell.img[2]; ++iz) {
                T dx = dx0 + (T)ix * L0, dy = dy0 + (T)iy * L1, dz = dz0 + (T)iz * L2;
                T r2 = dx * dx + dy * dy + dz * dz;
                if (r2 < fa.rc2) {
                  T r = t_sqrt(r2);
                  T ir = (T)1 / r;
                  T g = ((t_erfc(fa.alpha * r) - t_erfc(fa.eta * r)) * ir +
                         two_over_sqrtpi * (fa.alpha * t_exp(-fa.alpha * fa.alpha * r2) -
                                            fa.eta * t_exp(-fa.eta * fa.eta * r2))) * ir * ir;
                  fr[0] += qk * g * dx; fr[1] += qk * g * dy; fr[2] += qk * g * dz;
                  if (TWO) { frb[0] += qkb * g * dx; frb[1] += qkb * g * dy; frb[2] += qkb * g * dz; }
                }
              }
        }
      }
    }
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
                                      const ElecSet<double>&, const SiteSet<double>&, double*);
template void launch_real_b_t<float>(hipStream_t, int, const Cell&, double, double, double,
                                     const ElecSet<float>&, const SiteSet<float>&, float*);
template void launch_site_forces_t<double>(hipStream_t, int, const Cell&, const ElecSet<double>&,
                                           const SiteSet<double>&, const ForceArgs<double>&);
template void launch_site_forces_t<float>(hipStream_t, int, const Cell&, const ElecSet<float>&,
                                          const SiteSet<float>&, const ForceArgs<float>&);

}  // namespace cpm
