// Cell-tile form of the real-space pair sums (Eq. 1-3): one workgroup of
// 256 threads takes the targets of one cell (a chunk of at most TILE_TGT of
// them) against every candidate of the cell's stencil.
//
//   * the stencil's candidates are index runs of a cell-sorted array (one per
//     stencil group, as in the wavefront walker), staged in LDS, TILE_CAND at
//     a time;
//   * thread (ti, sl) keeps target ti of the chunk in registers and tests
//     candidates sl, sl + nsl, ... (nsl = 256 / chunk size): the lanes of a
//     wavefront read few distinct candidates, which LDS broadcasts;
//   * pairs inside the cutoff go to a per-wavefront queue (ballot compaction)
//     and are evaluated 64 at a time; each result is added to its target's
//     LDS accumulator with an LDS atomic;
//   * one thread per target writes the sums, contiguous in the sorted order.
// Compared with one wavefront per target, no per-target cross-lane
// reductions or stencil set-up remain, and a target with few candidates
// costs only its share of the tests.  The summation order of a target's
// pairs follows the atomics' arrival, so results can differ between runs
// by rounding.
#pragma once
#include "pairs.h"

namespace cpm {

constexpr int TILE_THREADS = 256;
constexpr int TILE_CAND = 512;   // candidates staged in LDS per pass
constexpr int TILE_TGT = 64;     // targets per chunk

// merged candidate runs of a stencil: [lo, hi) of the source array, with
// exclusive offsets into the flattened candidate list
struct TileRuns {
  int lo[32], hi[32], off[32];
  int n, total;
};

// Wavefront 0 of the workgroup: runs of the stencil of cell c in the
// cell_start array cs, with offsets and total.
__device__ __forceinline__ void tile_runs(const Cell& cell, int c, const int* cs, TileRuns* R) {
  const int lane = threadIdx.x & (WAVE - 1);
  const int nr = stencil_runs(cell, c, cs, R->lo, R->hi);
  const int len = lane < nr ? R->hi[lane] - R->lo[lane] : 0;
  int incl = len;
  for (int o = 1; o < 32; o <<= 1) {
    const int t = __shfl_up(incl, o, WAVE);
    if (lane >= o) incl += t;
  }
  if (lane < nr) R->off[lane] = incl - len;
  const int total = __shfl(incl, 31, WAVE);
  if (lane == 0) { R->n = nr; R->total = total; }
}

// source index of flattened candidate k
__device__ __forceinline__ int tile_src(const TileRuns* R, int k) {
  int r = 0;
  while (r + 1 < R->n && R->off[r + 1] <= k) ++r;
  return R->lo[r] + (k - R->off[r]);
}

// per-wavefront queue of NV values of T and a target index per pair
template <typename T, int NV>
struct TileQ {
  static constexpr int CAP = 2 * WAVE;
  T* v;        // [NV][CAP]
  int* t;      // [CAP]
  static constexpr size_t bytes() { return (size_t)CAP * (NV * sizeof(T) + sizeof(int)); }
  __device__ __forceinline__ void bind(unsigned char* base) {
    v = reinterpret_cast<T*>(base);
    t = reinterpret_cast<int*>(base + (size_t)NV * CAP * sizeof(T));
  }
};

template <typename T, int NV>
__device__ __forceinline__ int tq_push(const TileQ<T, NV>& q, int n, bool in, const T (&val)[NV], int ti) {
  const int lane = threadIdx.x & (WAVE - 1);
  const unsigned long long m = __ballot(in);
  if (in) {
    const int pos = n + __popcll(m & ((1ull << lane) - 1ull));
#pragma unroll
    for (int u = 0; u < NV; ++u) q.v[u * TileQ<T, NV>::CAP + pos] = val[u];
    q.t[pos] = ti;
  }
  __builtin_amdgcn_wave_barrier();
  return n + __popcll(m);
}

template <typename T, int NV>
__device__ __forceinline__ int tq_pop(const TileQ<T, NV>& q, int n) {
  const int lane = threadIdx.x & (WAVE - 1);
  const int rest = n - WAVE;
  constexpr int CAP = TileQ<T, NV>::CAP;
  T v[NV];
  int t = 0;
  if (lane < rest) {
#pragma unroll
    for (int u = 0; u < NV; ++u) v[u] = q.v[u * CAP + WAVE + lane];
    t = q.t[WAVE + lane];
  }
  __builtin_amdgcn_wave_barrier();
  if (lane < rest) {
#pragma unroll
    for (int u = 0; u < NV; ++u) q.v[u * CAP + lane] = v[u];
    q.t[lane] = t;
  }
  __builtin_amdgcn_wave_barrier();
  return rest;
}

// LDS of a tile workgroup: runs, staged candidates (FP64 position, NQ
// charges of T, one int), four queues of NV values, NACC FP64 accumulators
// per target (FP64 LDS atomics in every precision: FP32 ones measured
// several times slower here)
template <typename T, int NQ, int NV, int NACC>
struct TileLds {
  static constexpr size_t runs = 0;
  static constexpr size_t cand = (sizeof(TileRuns) + 15) / 16 * 16;
  static constexpr size_t cand_bytes = (size_t)TILE_CAND * (3 * sizeof(double) + NQ * sizeof(T) + sizeof(int));
  static constexpr size_t queue = cand + (cand_bytes + 15) / 16 * 16;
  static constexpr size_t queue_bytes = (TileQ<T, NV>::bytes() + 15) / 16 * 16;
  static constexpr size_t acc = queue + 4 * queue_bytes;
  static constexpr size_t total = acc + (size_t)NACC * TILE_TGT * sizeof(double);
};

// staged candidates
template <typename T, int NQ>
struct TileCand {
  double *x, *y, *z;
  T* q[NQ > 0 ? NQ : 1];
  int* k;
  __device__ __forceinline__ void bind(unsigned char* base) {
    x = reinterpret_cast<double*>(base);
    y = x + TILE_CAND;
    z = y + TILE_CAND;
    T* qb = reinterpret_cast<T*>(z + TILE_CAND);
#pragma unroll
    for (int u = 0; u < (NQ > 0 ? NQ : 1); ++u) q[u] = qb + u * TILE_CAND;
    k = reinterpret_cast<int*>(qb + NQ * TILE_CAND);
  }
};

// Targets [t_lo, t_hi) of one chunk and the thread's place in it.
struct TileMap {
  int ntc, nsl, ti, sl;
  bool act;
  __device__ __forceinline__ TileMap(int ntc_) : ntc(ntc_) {
    nsl = TILE_THREADS / ntc;
    ti = (int)threadIdx.x % ntc;
    sl = (int)threadIdx.x / ntc;
    act = sl < nsl;
  }
};

// ------------------------------------------------------------ site pairs

// queued site pair of this lane: g0 force factor and pair potential added
// to its target's accumulators
template <typename T>
__device__ __forceinline__ void tile_eval_g0(const TileQ<T, 4>& Q, int lane, T alpha, double* acc) {
  constexpr int CAP = TileQ<T, 4>::CAP;
  const T qx = Q.v[lane], qy = Q.v[CAP + lane], qz = Q.v[2 * CAP + lane], qa = Q.v[3 * CAP + lane];
  const int tt = Q.t[lane];
  T g, pot;
  g0_terms(qx * qx + qy * qy + qz * qz, alpha, g, pot);
  const T w = qa * g;
  atomicAdd(acc + tt, (double)(w * qx));
  atomicAdd(acc + TILE_TGT + tt, (double)(w * qy));
  atomicAdd(acc + 2 * TILE_TGT + tt, (double)(w * qz));
  atomicAdd(acc + 3 * TILE_TGT + tt, (double)(qa * pot));
}

// Site-site sums of the targets [t_lo, t_hi) of cell c (a frame's sorted
// sites): f_pair gets sum_j' Q_j' g0(r) r_vec (without k_e and Q_j), u_site
// 1/2 k_e Q_j sum_j' Q_j' erfc(alpha r)/r.  lds: TileLds<T, 1, 4, 4>::total bytes.
template <typename T>
__device__ __forceinline__ void site_pairs_tile(const Cell& cell, const SiteSet<T>& st, T alpha, double rc2,
                                                double* __restrict__ f_pair, double* __restrict__ u_site, int c,
                                                int t_lo, int t_hi, int frame, unsigned char* lds) {
  using L = TileLds<T, 1, 4, 4>;
  TileRuns* R = reinterpret_cast<TileRuns*>(lds + L::runs);
  TileCand<T, 1> C;
  C.bind(lds + L::cand);
  TileQ<T, 4> Q;
  Q.bind(lds + L::queue + (threadIdx.x >> 6) * L::queue_bytes);
  double* acc = reinterpret_cast<double*>(lds + L::acc);     // [4][TILE_TGT]
  const int lane = threadIdx.x & (WAVE - 1);
  const size_t fo = (size_t)frame * st.n;
  const int* cs = st.cell_start + (size_t)frame * (cell.n_cells + 1);
  const double* sx = st.x + fo; const double* sy = st.y + fo; const double* sz = st.z + fo;
  const double* sq = st.q + fo;
  if (threadIdx.x < WAVE) tile_runs(cell, c, cs, R);
  const bool no_img = (cell.img[0] | cell.img[1] | cell.img[2]) == 0;
  for (int t0 = t_lo; t0 < t_hi; t0 += TILE_TGT) {
    const TileMap m(min(TILE_TGT, t_hi - t0));
    const int j = t0 + m.ti;
    const double xt = sx[j], yt = sy[j], zt = sz[j];
    for (int i = threadIdx.x; i < 4 * TILE_TGT; i += TILE_THREADS) acc[i] = 0.0;
    for (int c0 = 0;; c0 += TILE_CAND) {
      __syncthreads();
      const int total = R->total;
      if (c0 >= total && c0 > 0) break;
      const int nck = min(TILE_CAND, total - c0);
      for (int k = threadIdx.x; k < nck; k += TILE_THREADS) {
        const int s = tile_src(R, c0 + k);
        C.x[k] = sx[s]; C.y[k] = sy[s]; C.z[k] = sz[s]; C.q[0][k] = (T)sq[s]; C.k[k] = s;
      }
      __syncthreads();
      const int n_iter = (nck + m.nsl - 1) / m.nsl;
      int n = 0;
      for (int it = 0; it < n_iter; ++it) {
        const int k = m.sl + it * m.nsl;
        const bool valid = m.act && k < nck;
        double px = xt, py = yt, pz = zt;
        T pq = 0;
        int pk = j;
        if (valid) { px = C.x[k]; py = C.y[k]; pz = C.z[k]; pq = C.q[0][k]; pk = C.k[k]; }
        const Disp d = min_disp(cell, xt, yt, zt, px, py, pz);
        if (no_img) {
          T dx, dy, dz;
          const bool in = image_pair(cell, d, 0, 0, 0, rc2, dx, dy, dz) && valid && pk != j;
          const T val[4] = {dx, dy, dz, pq};
          n = tq_push(Q, n, in, val, m.ti);
          if (n >= WAVE) {
            tile_eval_g0(Q, lane, alpha, acc);
            n = tq_pop(Q, n);
          }
          continue;
        }
        for (int ix = -cell.img[0]; ix <= cell.img[0]; ++ix)
          for (int iy = -cell.img[1]; iy <= cell.img[1]; ++iy)
            for (int iz = -cell.img[2]; iz <= cell.img[2]; ++iz) {
              T dx, dy, dz;
              const bool self = pk == j && ix == 0 && iy == 0 && iz == 0;
              const bool in = image_pair(cell, d, ix, iy, iz, rc2, dx, dy, dz) && valid && !self;
              const T val[4] = {dx, dy, dz, pq};
              n = tq_push(Q, n, in, val, m.ti);
              if (n >= WAVE) {
                tile_eval_g0(Q, lane, alpha, acc);
                n = tq_pop(Q, n);
              }
            }
      }
      if (lane < n) tile_eval_g0(Q, lane, alpha, acc);
      if (c0 + TILE_CAND >= total) break;
    }
    __syncthreads();
    if ((int)threadIdx.x < m.ntc) {
      const int jj = t0 + threadIdx.x;
      double* o = f_pair + (size_t)frame * 3 * st.n;
      o[jj] = acc[threadIdx.x];
      o[st.n + jj] = acc[TILE_TGT + threadIdx.x];
      o[2 * (size_t)st.n + jj] = acc[2 * TILE_TGT + threadIdx.x];
      if (u_site) u_site[fo + jj] = 0.5 * KE * sq[jj] * acc[3 * TILE_TGT + threadIdx.x];
    }
    __syncthreads();
  }
}

// workgroup b of a frame's site-pair work: with tsplit > 0, share b mod
// tsplit of the sites of cell b / tsplit (tiles); with tsplit == 0, sites
// 4b .. 4b+3 (one wavefront each)
template <typename T>
__device__ __forceinline__ void site_pairs_block(const PairArgs<T>& pa, int b, int frame, unsigned char* lds) {
  if (pa.tsplit == 0) {
    // one wavefront per site, four per workgroup
    const int j = b * (TILE_THREADS / WAVE) + (threadIdx.x >> 6);
    if (j < pa.st.n)
      site_pairs_wave(pa.cell, pa.st, pa.alpha, pa.rc2, pa.f_pair, pa.u_site, j, frame,
                      reinterpret_cast<T*>(lds + (threadIdx.x >> 6) * wave_scratch_bytes<T>()));
    return;
  }
  const int c = b / pa.tsplit, s = b - c * pa.tsplit;
  const int* cs = pa.st.cell_start + (size_t)frame * (pa.cell.n_cells + 1);
  const int lo = cs[c], n = cs[c + 1] - lo;
  const int t_lo = lo + (int)(((long long)n * s) / pa.tsplit);
  const int t_hi = lo + (int)(((long long)n * (s + 1)) / pa.tsplit);
  site_pairs_tile(pa.cell, pa.st, pa.alpha, pa.rc2, pa.f_pair, pa.u_site, c, t_lo, t_hi, frame, lds);
}

}  // namespace cpm
