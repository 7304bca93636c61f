// Pair machinery of the real-space (short-range) Ewald sums with Gaussian
// electrode charges (Eq. 1-3), shared by the stand-alone real-space kernels
// and the kernels that host them as extra workgroups:
//   electrolyte potential at electrode i:  k_e sum_j Q_j g1(r),
//       g1(r) = [erfc(alpha r) - erfc(eta r)]/r;
//   site-site forces through g0(r) = erfc(alpha r)/r.
//
// Layout: one 64-wide wavefront per target (an electrode, or a site), lanes
// test the candidate partners of the neighbouring cells and queue those
// inside the cutoff (pair compaction below).  Partners are read from the
// cell-sorted SoA copies, so a wavefront's loads of one cell are contiguous;
// the neighbour cells (offsets -1 .. 1, or -2 .. 2 along a z axis of cells
// at least rcut/2 thick; fewer for cells that wrap onto themselves) cover
// every partner within rcut.
// Extra periodic images are looped over when the cell is shorter than
// 2 rcut.  Results are reduced across the wavefront with butterfly shuffles;
// no atomics, so every run sums in the same order.
#pragma once
#include "common.h"
#include "erfcx_cheb.h"

namespace cpm {

// 1/d for d >= 1: the hardware reciprocal estimate refined by two Newton
// steps y <- y + y (1 - d y) (each squares the relative error, so the
// estimate's ~1e-7 falls below FP64 rounding)
__device__ __forceinline__ double recip_nr(double d) {
  double y = __builtin_amdgcn_rcp(d);
  y = fma(y, fma(-d, y, 1.0), y);
  y = fma(y, fma(-d, y, 1.0), y);
  return y;
}

// erfcx(x) = exp(x^2) erfc(x) for 0 <= x <= ERFCX_XMAX: the degree-20
// polynomial in u(t), t = 2/(2 + x) (coefficients in erfcx_cheb.h), by
// Estrin's scheme: coefficient pairs, then pairs of pairs with u^2, u^4,
// u^8, u^16, a dependency chain of ~7 operations where Horner's would be 20
__device__ __forceinline__ double erfcx_cheb(double x) {
  static_assert(ERFCX_DEG == 20, "Estrin tree below is written for degree 20");
  const double t = 2.0 * recip_nr(2.0 + x);
  const double u = (t - ERFCX_TMIN) * (2.0 / (1.0 - ERFCX_TMIN)) - 1.0;
  const double u2 = u * u, u4 = u2 * u2, u8 = u4 * u4, u16 = u8 * u8;
  const double* a = ERFCX_POLY;
  double p[11];
#pragma unroll
  for (int i = 0; i < 10; ++i) p[i] = fma(a[2 * i + 1], u, a[2 * i]);
  p[10] = a[20];
  double q[6];
#pragma unroll
  for (int i = 0; i < 5; ++i) q[i] = fma(p[2 * i + 1], u2, p[2 * i]);
  q[5] = p[10];
  const double r0 = fma(q[1], u4, q[0]), r1 = fma(q[3], u4, q[2]), r2 = fma(q[5], u4, q[4]);
  const double s0 = fma(r1, u8, r0);
  return fma(r2, u16, s0);
}

// erfc(x) given e = exp(-x^2), 0 <= x <= ERFCX_XMAX (alpha rcut is checked
// against this bound when a context is created); float: the library erfcf
__device__ __forceinline__ double erfc_from_exp(double x, double e) { return e * erfcx_cheb(x); }
__device__ __forceinline__ float erfc_from_exp(float x, float) { return erfcf(x); }

__device__ __forceinline__ double t_exp(double x) { return exp(x); }
__device__ __forceinline__ float t_exp(float x) { return expf(x); }
// 1/sqrt(x), x > 0: the hardware estimate refined by two Newton steps
// y <- y (3 - x y^2) / 2 (each squares the relative error, so the estimate's
// ~1e-7 falls below FP64 rounding); float: 1/sqrtf
__device__ __forceinline__ double t_rsqrt(double x) {
  double y = __builtin_amdgcn_rsq(x);
  const double h = 0.5 * x;
  y = y * fma(-h * y, y, 1.5);
  y = y * fma(-h * y, y, 1.5);
  return y;
}
__device__ __forceinline__ float t_rsqrt(float x) { return 1.0f / sqrtf(x); }

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

// ------------------------------------------------- candidate walking
//
// Each wavefront keeps, next to its queue, a list of at most 32 runs of
// partner indices: the stencil's cells grouped into runs of consecutive cell
// indices (a table fixed by the grid), so that the partners are walked in
// full chunks of 64; the partner data of the next chunk is loaded while the
// current one is tested and queued.

// LDS of one wavefront: its queue (5 CAP values of T) and the runs (2 x 32 ints)
template <typename T>
constexpr size_t wave_scratch_bytes() { return 5 * WaveQueue<T>::CAP * sizeof(T) + 64 * sizeof(int); }
static_assert(pair_queue_lds<double>() == 4 * wave_scratch_bytes<double>(),
              "LDS reserved for hosted pair workgroups must hold four wavefront scratch areas");
static_assert(pair_queue_lds<float>() == 4 * wave_scratch_bytes<float>(),
              "LDS reserved for hosted pair workgroups must hold four wavefront scratch areas");

// Runs of the stencil of cell c in a cell-sorted array with cell_start cs
// (one per stencil group, in increasing index order): lanes below the
// returned count write [rlo, rhi).
__device__ __forceinline__ int stencil_runs(const Cell& cell, int c, const int* cs, int* rlo, int* rhi) {
  const int lane = threadIdx.x & (WAVE - 1);
  const int ng = cell.grp_n[c];
  int glo = 0, ghi = 0;
  if (lane < STENCIL_MAX) { glo = cell.grp_lo[c * STENCIL_MAX + lane]; ghi = cell.grp_hi[c * STENCIL_MAX + lane]; }
  if (lane < ng) {
    rlo[lane] = cs[glo];
    rhi[lane] = cs[ghi];
  }
  __builtin_amdgcn_wave_barrier();
  return ng;
}

// Cell of a wrapped position (the binning's arithmetic on the wrapped
// coordinate; where the two could differ in the last bit the position lies
// on a cell face, and the stencils of both cells hold every partner within
// the cutoff: a stencil reaches at least rcut past its cell on every side)
__device__ __forceinline__ int site_cell(const Cell& cell, double x, double y, double z) {
  return (cell_coord(z, cell.L[2], cell.nc[2]) * cell.nc[1] + cell_coord(y, cell.L[1], cell.nc[1])) * cell.nc[0] +
         cell_coord(x, cell.L[0], cell.nc[0]);
}

// Runs of the electrode atoms in reach of cell c (a fixed table)
template <typename T>
__device__ __forceinline__ int elec_runs(const ElecSet<T>& el, int c, int* rlo, int* rhi) {
  const int lane = threadIdx.x & (WAVE - 1);
  const int nr = el.run_n[c];
  int lo = 0, hi = 0;
  if (lane < STENCIL_MAX) { lo = el.run_lo[c * STENCIL_MAX + lane]; hi = el.run_hi[c * STENCIL_MAX + lane]; }
  if (lane < nr) {
    rlo[lane] = lo;
    rhi[lane] = hi;
  }
  __builtin_amdgcn_wave_barrier();
  return nr;
}

// Keeps part `part` of `parts` of the candidates listed by the wavefront's
// runs (the candidates counted in run order and cut into equal shares),
// rewriting the run table in place; runs may come out empty.
__device__ __forceinline__ void split_runs(int* rlo, int* rhi, int nruns, int part, int parts) {
  const int lane = threadIdx.x & (WAVE - 1);
  int lo = 0, hi = 0;
  if (lane < nruns) { lo = rlo[lane]; hi = rhi[lane]; }
  const int len = hi - lo;
  int incl = len;                               // inclusive prefix over the (at most 32) runs
#pragma unroll
  for (int off = 1; off < 32; off <<= 1) {
    const int t = __shfl_up(incl, off, WAVE);
    if (lane >= off) incl += t;
  }
  const int total = __shfl(incl, 31, WAVE);
  const int a = (int)((long long)total * part / parts);
  const int b = (int)((long long)total * (part + 1) / parts);
  const int start = incl - len;
  const int nlo = lo + max(0, min(len, a - start));
  const int nhi = max(nlo, lo + max(0, min(len, b - start)));
  __builtin_amdgcn_wave_barrier();
  if (lane < nruns) { rlo[lane] = nlo; rhi[lane] = nhi; }
  __builtin_amdgcn_wave_barrier();
}

// Walks the partners listed by the runs 64 at a time: load(k, valid)
// returns the data of partner k (lane's index in the chunk), body(data, k,
// valid) consumes it.  The loads of the next chunk are issued before the
// body of the current one runs.
template <typename Load, typename Body>
__device__ __forceinline__ void walk_runs(const int* rlo, const int* rhi, int nruns, Load load, Body body) {
  const int lane = threadIdx.x & (WAVE - 1);
  int r = 0, base = 0, end = 0;
  if (nruns > 0) { base = rlo[0]; end = rhi[0]; }
  while (r < nruns && base >= end) {
    ++r;
    if (r < nruns) { base = rlo[r]; end = rhi[r]; }
  }
  if (r >= nruns) return;
  int ck = base + lane;
  bool cv = ck < end;
  auto cur = load(ck, cv);
  for (;;) {
    base += WAVE;
    while (r < nruns && base >= end) {
      ++r;
      if (r < nruns) { base = rlo[r]; end = rhi[r]; }
    }
    const bool more = r < nruns;
    const int nk = base + lane;
    const bool nv = more && nk < end;
    auto nxt = load(nk, nv);
    body(cur, ck, cv);
    if (!more) break;
    cur = nxt;
    ck = nk;
    cv = nv;
  }
}

// a partner site: FP64 position (displacements are formed in FP64) and charge
template <typename T>
struct Partner {
  double x, y, z;
  T a;
};

// an electrode atom: FP64 position and its charge(s) of this step
template <typename T>
struct ElecPartner {
  double x, y, z;
  T a, b;
};

// Minimum-image displacement from a partner to the target, in FP64; the
// periodic images add (ix, iy, iz) cell lengths, still in FP64, and only the
// result is rounded to the pair arithmetic's type (two ~10 nm coordinates
// differenced in FP32 would lose ~1e-6 nm).
struct Disp {
  double d0, d1, d2;
};
__device__ __forceinline__ Disp min_disp(const Cell& cell, double tx, double ty, double tz, double px, double py,
                                         double pz) {
  return Disp{min_image(tx - px, cell.L[0], cell.invL[0]), min_image(ty - py, cell.L[1], cell.invL[1]),
              min_image(tz - pz, cell.L[2], cell.invL[2])};
}
// The displacement to periodic image (ix, iy, iz), rounded to T, and whether
// the pair lies inside the cutoff: that decision is taken in FP64 in every
// precision, so that all paths keep the same pairs.
template <typename T>
__device__ __forceinline__ bool image_pair(const Cell& cell, const Disp& d, int ix, int iy, int iz, double rc2, T& dx,
                                           T& dy, T& dz) {
  const double x = d.d0 + ix * cell.L[0];
  const double y = d.d1 + iy * cell.L[1];
  const double z = d.d2 + iz * cell.L[2];
  dx = (T)x; dy = (T)y; dz = (T)z;
  return x * x + y * y + z * z < rc2;
}

// ------------------------------------------------------------------ b real

// erfc(eta r) and exp(-eta^2 r^2) are below 1e-18 for eta r > 6.5, far under
// FP64 resolution of the alpha terms they are added to, so they are skipped
// there (always the case for sites at least 0.33 nm from an electrode atom)
constexpr double ETA_R_SKIP = 6.5;

template <typename T>
__device__ __forceinline__ T g1_potential(T dx, T dy, T dz, T q, T alpha, T eta) {
  T r2 = dx * dx + dy * dy + dz * dz;
  const T ir = t_rsqrt(r2);
  const T r = r2 * ir;
  T e = erfc_from_exp(alpha * r, t_exp(-alpha * alpha * r2));
  if (eta * r < (T)ETA_R_SKIP) e -= erfc_from_exp(eta * r, t_exp(-eta * eta * r2));
  return q * e * ir;
}

// Real-space electrolyte potential at electrode atom g of a frame, one
// wavefront: k_e sum_j Q_j g1(r) over the sites of the stencil cells.
// scratch: this wavefront's LDS (wave_scratch_bytes<T>()).
template <typename T>
__device__ __forceinline__ void real_b_wave(const Cell& cell, T alpha, T eta, double rc2, const ElecSet<T>& el,
                                            const SiteSet<T>& st, T* __restrict__ phi_out, int g, int frame,
                                            T* scratch) {
  const int lane = threadIdx.x & (WAVE - 1);
  const size_t fo = (size_t)frame * st.n;
  const double* sx = st.x + fo; const double* sy = st.y + fo; const double* sz = st.z + fo;
  const double* sq = st.q + fo;
  WaveQueue<T> Q;
  Q.bind(scratch);
  int* rlo = reinterpret_cast<int*>(scratch + 5 * WaveQueue<T>::CAP);
  int* rhi = rlo + 32;
  const int* cs = st.cell_start + (size_t)frame * (cell.n_cells + 1);
  const double ex = el.x[g], ey = el.y[g], ez = el.z[g];
  const int c = el.cell[g];
  const int og = el.orig[g];                   // read now, used at the end
  const int nruns = stencil_runs(cell, c, cs, rlo, rhi);
  T acc = 0;
  int n = 0;
  walk_runs(rlo, rhi, nruns,
            [&](int k, bool v) {
              Partner<T> p{0, 0, 0, (T)0};
              if (v) { p.x = sx[k]; p.y = sy[k]; p.z = sz[k]; p.a = (T)sq[k]; }
              return p;
            },
            [&](const Partner<T>& p, int k, bool valid) {
              const Disp d = min_disp(cell, ex, ey, ez, p.x, p.y, p.z);
              for (int ix = -cell.img[0]; ix <= cell.img[0]; ++ix)
                for (int iy = -cell.img[1]; iy <= cell.img[1]; ++iy)
                  for (int iz = -cell.img[2]; iz <= cell.img[2]; ++iz) {
                    T dx, dy, dz;
                    const bool in = image_pair(cell, d, ix, iy, iz, rc2, dx, dy, dz) && valid;
                    n = queue_push(Q, n, in, dx, dy, dz, p.a, (T)0);
                    if (n >= WAVE) {
                      acc += g1_potential(Q.x[lane], Q.y[lane], Q.z[lane], Q.a[lane], alpha, eta);
                      n = queue_pop(Q, n);
                    }
                  }
            });
  if (lane < n) acc += g1_potential(Q.x[lane], Q.y[lane], Q.z[lane], Q.a[lane], alpha, eta);
  acc = wave_sum(acc);
  if (lane == 0) phi_out[(size_t)frame * el.n + og] = (T)KE * acc;
}

// ------------------------------------------------------------ site forces

// radial force factor g(r) = -(d kernel/dr)/r of a site pair (g0) and of a
// site-Gaussian pair (g1), and the site-pair potential erfc(alpha r)/r
template <typename T>
__device__ __forceinline__ void g0_terms(T r2, T alpha, T& g, T& pot) {
  const T two_over_sqrtpi = (T)1.1283791670955126;
  const T ir = t_rsqrt(r2);
  const T r = r2 * ir;
  T ex = t_exp(-alpha * alpha * r2);
  T ec = erfc_from_exp(alpha * r, ex);
  g = (ec * ir + two_over_sqrtpi * alpha * ex) * ir * ir;
  pot = ec * ir;
}
template <typename T>
__device__ __forceinline__ T g1_force(T r2, T alpha, T eta) {
  const T two_over_sqrtpi = (T)1.1283791670955126;
  const T ir = t_rsqrt(r2);
  const T r = r2 * ir;
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

// queued site pairs: force factor and pair potential (g0)
template <typename T>
__device__ __forceinline__ void eval_g0(const WaveQueue<T>& Q, int lane, T alpha, T* fr, T& u) {
  const T qx = Q.x[lane], qy = Q.y[lane], qz = Q.z[lane];
  T g, pot;
  g0_terms(qx * qx + qy * qy + qz * qz, alpha, g, pot);
  const T w = Q.a[lane] * g;
  fr[0] += w * qx; fr[1] += w * qy; fr[2] += w * qz;
  u += Q.a[lane] * pot;
}

// queued site-Gaussian pairs: force factor (g1) for the charges a (and b)
template <typename T, bool TWO>
__device__ __forceinline__ void eval_g1(const WaveQueue<T>& Q, int lane, T alpha, T eta, T* fr, T* frb) {
  const T qx = Q.x[lane], qy = Q.y[lane], qz = Q.z[lane];
  const T g = g1_force(qx * qx + qy * qy + qz * qz, alpha, eta);
  const T w = Q.a[lane] * g;
  fr[0] += w * qx; fr[1] += w * qy; fr[2] += w * qz;
  if (TWO) { const T wb = Q.b[lane] * g; frb[0] += wb * qx; frb[1] += wb * qy; frb[2] += wb * qz; }
}

// Site-site part of the force on site j of a frame, one wavefront (it does
// not depend on the electrode charges): f_pair gets sum_j' Q_j' g0(r) r_vec
// (without k_e and Q_j), u_site the pair energy
// 1/2 k_e Q_j sum_j' Q_j' erfc(alpha r)/r.  scratch: as for real_b_wave.
template <typename T>
__device__ __forceinline__ void site_pairs_wave(const Cell& cell, const SiteSet<T>& st, T alpha, double rc2,
                                                double* __restrict__ f_pair, double* __restrict__ u_site,
                                                int j, int frame, T* scratch) {
  const int lane = threadIdx.x & (WAVE - 1);
  WaveQueue<T> Q;
  Q.bind(scratch);
  int* rlo = reinterpret_cast<int*>(scratch + 5 * WaveQueue<T>::CAP);
  int* rhi = rlo + 32;
  const size_t fo = (size_t)frame * st.n;
  const int* cs = st.cell_start + (size_t)frame * (cell.n_cells + 1);
  const double* sx = st.x + fo; const double* sy = st.y + fo; const double* sz = st.z + fo;
  const double* sq = st.q + fo;
  const double xj = sx[j], yj = sy[j], zj = sz[j], qj = sq[j];
  const int nruns = stencil_runs(cell, site_cell(cell, xj, yj, zj), cs, rlo, rhi);
  T fr[3] = {0, 0, 0};
  T u = 0;
  int n = 0;
  walk_runs(rlo, rhi, nruns,
            [&](int k, bool v) {
              Partner<T> p{0, 0, 0, (T)0};
              if (v) { p.x = sx[k]; p.y = sy[k]; p.z = sz[k]; p.a = (T)sq[k]; }
              return p;
            },
            [&](const Partner<T>& p, int k, bool valid) {
              const Disp d = min_disp(cell, xj, yj, zj, p.x, p.y, p.z);
              for (int ix = -cell.img[0]; ix <= cell.img[0]; ++ix)
                for (int iy = -cell.img[1]; iy <= cell.img[1]; ++iy)
                  for (int iz = -cell.img[2]; iz <= cell.img[2]; ++iz) {
                    T dx, dy, dz;
                    const bool self = k == j && ix == 0 && iy == 0 && iz == 0;
                    const bool in = image_pair(cell, d, ix, iy, iz, rc2, dx, dy, dz) && valid && !self;
                    n = queue_push(Q, n, in, dx, dy, dz, p.a, (T)0);
                    if (n >= WAVE) {
                      eval_g0(Q, lane, alpha, fr, u);
                      n = queue_pop(Q, n);
                    }
                  }
            });
  if (lane < n) eval_g0(Q, lane, alpha, fr, u);
  const T v8[8] = {fr[0], fr[1], fr[2], u, (T)0, (T)0, (T)0, (T)0};
  const T s8 = wave_sum8(v8);                 // lane 8k: total of v8[k]
  double e[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) e[d] = (double)read_lane(s8, 8 * d);
  const double us = (double)read_lane(s8, 24);
  if (lane == 0) {
    double* o = f_pair + (size_t)frame * 3 * st.n;
    o[j] = e[0]; o[st.n + j] = e[1]; o[2 * st.n + j] = e[2];
    if (u_site) u_site[fo + j] = 0.5 * KE * qj * us;
  }
}

}  // namespace cpm
