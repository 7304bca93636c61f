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


// merged candidate runs of a stencil: [lo, hi) of the source array, with
// exclusive offsets into the flattened candidate list
struct TileRuns {
  int lo[32], hi[32], off[32];
  int n, total;
};

// One wavefront: lanes below nr hold run [lo, hi); R gets the runs, their
// exclusive offsets and the total.
__device__ __forceinline__ void tile_scan_runs(int nr, int lo, int hi, TileRuns* R) {
  const int lane = threadIdx.x & (WAVE - 1);
  const int len = lane < nr ? hi - lo : 0;
  if (lane < nr) { R->lo[lane] = lo; R->hi[lane] = hi; }
  int incl = len;
  for (int o = 1; o < 32; o <<= 1) {
    const int t = __shfl_up(incl, o, WAVE);
    if (lane >= o) incl += t;
  }
  if (lane < nr) R->off[lane] = incl - len;
  const int total = __shfl(incl, 31, WAVE);
  if (lane == 0) { R->n = nr; R->total = total; }
}

// runs of the stencil of cell c in the cell_start array cs
__device__ __forceinline__ void tile_runs(const Cell& cell, int c, const int* cs, TileRuns* R) {
  const int lane = threadIdx.x & (WAVE - 1);
  const int ng = cell.grp_n[c];
  int lo = 0, hi = 0;
  if (lane < ng) { lo = cs[cell.grp_lo[c * STENCIL_MAX + lane]]; hi = cs[cell.grp_hi[c * STENCIL_MAX + lane]]; }
  tile_scan_runs(ng, lo, hi, R);
}

// runs of the electrode atoms in reach of cell c (a fixed table)
template <typename T>
__device__ __forceinline__ void tile_elec_runs(const ElecSet<T>& el, int c, TileRuns* R) {
  const int lane = threadIdx.x & (WAVE - 1);
  const int nr = el.run_n[c];
  int lo = 0, hi = 0;
  if (lane < nr) { lo = el.run_lo[c * STENCIL_MAX + lane]; hi = el.run_hi[c * STENCIL_MAX + lane]; }
  tile_scan_runs(nr, lo, hi, R);
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
  static constexpr size_t runs = 0;           // two run lists (sites, electrodes)
  static constexpr size_t cand = (2 * sizeof(TileRuns) + 15) / 16 * 16;
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

// queue entries: the displacement (3 values of T) and one int holding the
// target (low 8 bits) and the candidate's slot in the staged list (above):
// the charges are read from the staged candidates when the pair is
// evaluated, which keeps the queues (and the workgroup's LDS) small
template <typename T> using TileQP = TileQ<T, 3>;
template <typename T> using PairLds = TileLds<T, 2, 3, 10>;
__device__ __forceinline__ int tq_pack(int target, int slot) { return target | (slot << 8); }
static_assert(TILE_TGT <= 256 && TILE_CAND <= (1 << 22), "queue entry packing");
// accumulators per target: 0-2 site-site force sum, 3 site-site potential,
// 4-6 site-electrode force sum with charges a, 7-9 with charges b

// One candidate phase of a target chunk: the candidates listed by R, staged
// into C by stage(slot, source index), tested against the chunk's targets
// (self pairs excluded when self_excl), pairs inside the cutoff evaluated by
// eval(lane) 64 at a time.
template <typename T, typename Stage, typename Eval>
__device__ __forceinline__ void tile_phase(const Cell& cell, double rc2, const TileRuns* R, const TileMap& m, int j,
                                           double xt, double yt, double zt, bool self_excl, const TileCand<T, 2>& C,
                                           const TileQP<T>& Q, Stage stage, Eval eval) {
  const int lane = threadIdx.x & (WAVE - 1);
  const bool no_img = (cell.img[0] | cell.img[1] | cell.img[2]) == 0;
  for (int c0 = 0;; c0 += TILE_CAND) {
    __syncthreads();
    const int total = R->total;
    const int nck = min(TILE_CAND, total - c0);
    for (int k = threadIdx.x; k < nck; k += TILE_THREADS) stage(k, tile_src(R, c0 + k));
    __syncthreads();
    const int n_iter = nck > 0 ? (nck + m.nsl - 1) / m.nsl : 0;
    int n = 0;
    if (no_img) {
      // two candidates per step: their tests are independent chains that
      // the compiler interleaves (three wavefronts per SIMD hide little)
      for (int it = 0; it < n_iter; it += 2) {
        double px[2], py[2], pz[2];
        int kk[2];
        bool in[2];
        T dx[2], dy[2], dz[2];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const int k = m.sl + (it + h) * m.nsl;
          const bool valid = m.act && it + h < n_iter && k < nck;
          kk[h] = k;
          px[h] = xt; py[h] = yt; pz[h] = zt;
          int pk = -1;
          if (valid) {
            px[h] = C.x[k]; py[h] = C.y[k]; pz[h] = C.z[k];
            pk = C.k[k];
          }
          const Disp d = min_disp(cell, xt, yt, zt, px[h], py[h], pz[h]);
          dx[h] = (T)d.d0; dy[h] = (T)d.d1; dz[h] = (T)d.d2;
          in[h] = d.d0 * d.d0 + d.d1 * d.d1 + d.d2 * d.d2 < rc2 && valid && !(self_excl && pk == j);
        }
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const T val[3] = {dx[h], dy[h], dz[h]};
          n = tq_push(Q, n, in[h], val, tq_pack(m.ti, kk[h]));
          if (n >= WAVE) {
            eval(lane);
            n = tq_pop(Q, n);
          }
        }
      }
      if (lane < n) eval(lane);
      if (c0 + TILE_CAND >= total) break;
      continue;
    }
    for (int it = 0; it < n_iter; ++it) {
      const int k = m.sl + it * m.nsl;
      const bool valid = m.act && k < nck;
      double px = xt, py = yt, pz = zt;
      int pk = -1;
      if (valid) { px = C.x[k]; py = C.y[k]; pz = C.z[k]; pk = C.k[k]; }
      const bool self_pk = self_excl && pk == j;
      const Disp d = min_disp(cell, xt, yt, zt, px, py, pz);
      for (int ix = -cell.img[0]; ix <= cell.img[0]; ++ix)
        for (int iy = -cell.img[1]; iy <= cell.img[1]; ++iy)
          for (int iz = -cell.img[2]; iz <= cell.img[2]; ++iz) {
            T dx, dy, dz;
            const bool self = self_pk && ix == 0 && iy == 0 && iz == 0;
            const bool in = image_pair(cell, d, ix, iy, iz, rc2, dx, dy, dz) && valid && !self;
            const T val[3] = {dx, dy, dz};
            n = tq_push(Q, n, in, val, tq_pack(m.ti, k));
            if (n >= WAVE) {
              eval(lane);
              n = tq_pop(Q, n);
            }
          }
    }
    if (lane < n) eval(lane);
    if (c0 + TILE_CAND >= total) break;
  }
}

// Real-space sums of the targets [t_lo, t_hi) of cell c (a frame's sorted
// sites): f_pair gets sum_j' Q_j' g0(r) r_vec (without k_e and Q_j), u_site
// 1/2 k_e Q_j sum_j' Q_j' erfc(alpha r)/r; with pa.f_elec also the
// site-electrode sums sum_i q_i g1(r) r_vec for the charges qa and qb
// (without k_e and Q_j).  lds: PairLds<T>::total bytes.
template <typename T>
__device__ __forceinline__ void site_pairs_tile(const PairArgs<T>& pa, int c, int t_lo, int t_hi, int frame,
                                                unsigned char* lds) {
  using L = PairLds<T>;
  constexpr int CAP = TileQP<T>::CAP;
  const Cell& cell = pa.cell;
  const SiteSet<T>& st = pa.st;
  TileRuns* R = reinterpret_cast<TileRuns*>(lds + L::runs);
  TileRuns* RE = R + 1;
  TileCand<T, 2> C;
  C.bind(lds + L::cand);
  TileQP<T> Q;
  Q.bind(lds + L::queue + (threadIdx.x >> 6) * L::queue_bytes);
  double* acc = reinterpret_cast<double*>(lds + L::acc);     // [10][TILE_TGT]
  const size_t fo = (size_t)frame * st.n;
  const int* cs = st.cell_start + (size_t)frame * (cell.n_cells + 1);
  const double* sx = st.x + fo; const double* sy = st.y + fo; const double* sz = st.z + fo;
  const double* sq = st.q + fo;
  const bool elec = pa.f_elec != nullptr;
  if (threadIdx.x < WAVE) tile_runs(cell, c, cs, R);
  else if (elec && threadIdx.x < 2 * WAVE) tile_elec_runs(pa.el, c, RE);
  const double* qa_e = elec ? pa.qa_s + (size_t)frame * pa.qa_stride : nullptr;
  for (int t0 = t_lo; t0 < t_hi; t0 += TILE_TGT) {
    const TileMap m(min(TILE_TGT, t_hi - t0));
    const int j = t0 + m.ti;
    const double xt = sx[j], yt = sy[j], zt = sz[j];
    for (int i = threadIdx.x; i < 10 * TILE_TGT; i += TILE_THREADS) acc[i] = 0.0;
    // sites: g0 force factor and pair potential
    tile_phase<T>(cell, pa.rc2, R, m, j, xt, yt, zt, true, C, Q,
                  [&](int k, int s) {
                    C.x[k] = sx[s]; C.y[k] = sy[s]; C.z[k] = sz[s];
                    C.q[0][k] = (T)sq[s]; C.q[1][k] = (T)0; C.k[k] = s;
                  },
                  [&](int l) {
                    const T qx = Q.v[l], qy = Q.v[CAP + l], qz = Q.v[2 * CAP + l];
                    const int e = Q.t[l];
                    const int tt = e & 255;
                    const T qa = C.q[0][e >> 8];
                    T g, pot;
                    g0_terms(qx * qx + qy * qy + qz * qz, pa.alpha, g, pot);
                    const T w = qa * g;
                    atomicAdd(acc + tt, (double)(w * qx));
                    atomicAdd(acc + TILE_TGT + tt, (double)(w * qy));
                    atomicAdd(acc + 2 * TILE_TGT + tt, (double)(w * qz));
                    atomicAdd(acc + 3 * TILE_TGT + tt, (double)(qa * pot));
                  });
    // electrode atoms: g1 force factor for both charge sets
    if (elec)
      tile_phase<T>(cell, pa.rc2, RE, m, j, xt, yt, zt, false, C, Q,
                    [&](int k, int s) {
                      C.x[k] = pa.el.x[s]; C.y[k] = pa.el.y[s]; C.z[k] = pa.el.z[s];
                      C.q[0][k] = (T)qa_e[s]; C.q[1][k] = pa.qb_s ? (T)pa.qb_s[s] : (T)0; C.k[k] = -1;
                    },
                    [&](int l) {
                      const T qx = Q.v[l], qy = Q.v[CAP + l], qz = Q.v[2 * CAP + l];
                      const int e = Q.t[l];
                      const int tt = e & 255;
                      const T qa = C.q[0][e >> 8], qb = C.q[1][e >> 8];
                      const T g = g1_force(qx * qx + qy * qy + qz * qz, pa.alpha, pa.eta);
                      const T wa = qa * g, wb = qb * g;
                      atomicAdd(acc + 4 * TILE_TGT + tt, (double)(wa * qx));
                      atomicAdd(acc + 5 * TILE_TGT + tt, (double)(wa * qy));
                      atomicAdd(acc + 6 * TILE_TGT + tt, (double)(wa * qz));
                      atomicAdd(acc + 7 * TILE_TGT + tt, (double)(wb * qx));
                      atomicAdd(acc + 8 * TILE_TGT + tt, (double)(wb * qy));
                      atomicAdd(acc + 9 * TILE_TGT + tt, (double)(wb * qz));
                    });
    __syncthreads();
    if ((int)threadIdx.x < m.ntc) {
      const int jj = t0 + threadIdx.x;
      double* o = pa.f_pair + (size_t)frame * 3 * st.n;
      o[jj] = acc[threadIdx.x];
      o[st.n + jj] = acc[TILE_TGT + threadIdx.x];
      o[2 * (size_t)st.n + jj] = acc[2 * TILE_TGT + threadIdx.x];
      if (pa.u_site) pa.u_site[fo + jj] = 0.5 * KE * sq[jj] * acc[3 * TILE_TGT + threadIdx.x];
      if (elec) {
        double* e = pa.f_elec + (size_t)frame * 6 * st.n;
#pragma unroll
        for (int u = 0; u < 6; ++u) e[(size_t)u * st.n + jj] = acc[(4 + u) * TILE_TGT + threadIdx.x];
      }
    }
    __syncthreads();
  }
}

// Real-space electrolyte potential at the electrode atoms of one work item
// (atoms [t_lo, t_hi) of cell c, t_hi - t_lo <= TILE_TGT):
// k_e sum_j Q_j g1(r) over the sites of the stencil.  lds: PairLds<T>::total.
template <typename T>
__device__ __forceinline__ void real_b_tile(const RealBArgs<T>& rb, int c, int t_lo, int t_hi, int frame,
                                            unsigned char* lds) {
  using L = PairLds<T>;
  constexpr int CAP = TileQP<T>::CAP;
  const SiteSet<T>& st = rb.st;
  TileRuns* R = reinterpret_cast<TileRuns*>(lds + L::runs);
  TileCand<T, 2> C;
  C.bind(lds + L::cand);
  TileQP<T> Q;
  Q.bind(lds + L::queue + (threadIdx.x >> 6) * L::queue_bytes);
  double* acc = reinterpret_cast<double*>(lds + L::acc);
  const size_t fo = (size_t)frame * st.n;
  const int* cs = st.cell_start + (size_t)frame * (rb.cell.n_cells + 1);
  const double* sx = st.x + fo; const double* sy = st.y + fo; const double* sz = st.z + fo;
  const double* sq = st.q + fo;
  if (threadIdx.x < WAVE) tile_runs(rb.cell, c, cs, R);
  const TileMap m(t_hi - t_lo);
  const int g = t_lo + m.ti;
  const double xt = rb.el.x[g], yt = rb.el.y[g], zt = rb.el.z[g];
  for (int i = threadIdx.x; i < TILE_TGT; i += TILE_THREADS) acc[i] = 0.0;
  tile_phase<T>(rb.cell, rb.rc2, R, m, -1, xt, yt, zt, false, C, Q,
                [&](int k, int s) {
                  C.x[k] = sx[s]; C.y[k] = sy[s]; C.z[k] = sz[s];
                  C.q[0][k] = (T)sq[s]; C.q[1][k] = (T)0; C.k[k] = s;
                },
                [&](int l) {
                  const int e = Q.t[l];
                  atomicAdd(acc + (e & 255), (double)g1_potential(Q.v[l], Q.v[CAP + l], Q.v[2 * CAP + l],
                                                                  C.q[0][e >> 8], rb.alpha, rb.eta));
                });
  __syncthreads();
  if ((int)threadIdx.x < m.ntc) {
    const int gg = t_lo + threadIdx.x;
    rb.phi_out[(size_t)frame * rb.el.n + rb.el.orig[gg]] = (T)(KE * acc[threadIdx.x]);
  }
}

// workgroup b of a frame's real-space b work
template <typename T>
__device__ __forceinline__ void real_b_block(const RealBArgs<T>& rb, int b, int frame, unsigned char* lds) {
  if (!rb.tiles) {
    const int g = b * (TILE_THREADS / WAVE) + (threadIdx.x >> 6);
    if (g < rb.el.n)
      real_b_wave(rb.cell, rb.alpha, rb.eta, rb.rc2, rb.el, rb.st, rb.phi_out, g, frame,
                  reinterpret_cast<T*>(lds + (threadIdx.x >> 6) * wave_scratch_bytes<T>()));
    return;
  }
  real_b_tile(rb, rb.item_c[b], rb.item_lo[b], rb.item_hi[b], frame, lds);
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
  site_pairs_tile(pa, c, t_lo, t_hi, frame, lds);
}

}  // namespace cpm
