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
//
// Without periodic images the site-site pairs take a form of their own
// (site_pairs_n3_tile below) that evaluates every pair once, and the
// site-electrode pairs a launch of their own (site_elec_tile).
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

// runs of the forward half of the stencil of cell c (tables as Cell::grp_*)
__device__ __forceinline__ void tile_runs_fwd(const int* fn, const int* flo, const int* fhi, int c, const int* cs,
                                              TileRuns* R) {
  const int lane = threadIdx.x & (WAVE - 1);
  const int ng = fn[c];
  int lo = 0, hi = 0;
  if (lane < ng) { lo = cs[flo[c * STENCIL_MAX + lane]]; hi = cs[fhi[c * STENCIL_MAX + lane]]; }
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

// per-wavefront queue of packed pair indices alone (the displacement is
// recomputed when the pair is evaluated)
struct TileQI {
  static constexpr int CAP = 2 * WAVE;
  int* t;      // [CAP]
  static constexpr size_t bytes() { return (size_t)CAP * sizeof(int); }
  __device__ __forceinline__ void bind(unsigned char* base) { t = reinterpret_cast<int*>(base); }
};

__device__ __forceinline__ int tqi_push(const TileQI& q, int n, bool in, int e) {
  const unsigned long long m = __ballot(in);
  if (in) q.t[n + (int)__builtin_amdgcn_mbcnt_hi((unsigned)(m >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)m, 0u))] = e;
  __builtin_amdgcn_wave_barrier();
  return n + __popcll(m);
}

__device__ __forceinline__ int tqi_pop(const TileQI& q, int n) {
  const int lane = threadIdx.x & (WAVE - 1);
  const int rest = n - WAVE;
  const int e = lane < rest ? q.t[WAVE + lane] : 0;
  __builtin_amdgcn_wave_barrier();
  if (lane < rest) q.t[lane] = e;
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

// ------------------------------------------------- site pairs, each once

// LDS of the each-pair-once tile: the stencil runs, the staged candidates
// (two 16-byte arrays: x and y; z and the sorted index; then the charges),
// four FP64 sums per candidate and per target (force, potential), the
// targets' positions and charges, one queue of packed pair indices per
// wavefront
template <typename T>
struct PairN3Lds {
  static constexpr size_t runs = 0;
  static constexpr size_t rec = (sizeof(TileRuns) + 31) / 32 * 32;     // xy [TILE_CAND], then zs [TILE_CAND]
  static constexpr size_t cq = rec + (size_t)TILE_CAND * 32;
  static constexpr size_t cacc = cq + ((size_t)TILE_CAND * sizeof(T) + 15) / 16 * 16;
  static constexpr size_t tacc = cacc + 4 * (size_t)TILE_CAND * sizeof(double);
  static constexpr size_t tpos = tacc + 4 * (size_t)TILE_TGT * sizeof(double);     // x, y, z [TILE_TGT]
  static constexpr size_t tq = tpos + 3 * (size_t)TILE_TGT * sizeof(double);
  static constexpr size_t queue = tq + ((size_t)TILE_TGT * sizeof(T) + 15) / 16 * 16;
  static constexpr size_t queue_bytes = (TileQI::bytes() + 15) / 16 * 16;
  static constexpr size_t total = queue + (TILE_THREADS / WAVE) * queue_bytes;
};

// Site-site sums of the targets [t_lo, t_hi) of cell c with every pair once
// (no periodic images): the candidates are the sites of the forward half of
// the stencil (pa.fwd_*) of larger sorted index than the target, so each
// pair inside the cutoff is met by exactly one work item, which adds
// Q_k g0(r) r_vec to the target's and -Q_j g0(r) r_vec to the candidate's
// force sum, and Q_k erfc(alpha r)/r, Q_j erfc(alpha r)/r to their
// potential sums.  Thread (ti, sl) tests the candidates of block sl of the
// nsl contiguous blocks of a staged set, starting at offset ti within it,
// so that the lanes of a wavefront read, and later add into, distinct
// candidates.  The candidates' sums go to f_pair and u_site with FP64
// atomic adds after every staged set, the targets' after the last one: both
// arrays are cleared before the launch.  lds: PairN3Lds<T>::total bytes.
template <typename T, bool ZS>
__device__ __forceinline__ void site_pairs_n3_tile(const PairArgs<T>& pa, int c, int t_lo, int t_hi, int frame,
                                                   unsigned char* lds) {
  using L = PairN3Lds<T>;
  TileRuns* R = reinterpret_cast<TileRuns*>(lds + L::runs);
  double2* rxy = reinterpret_cast<double2*>(lds + L::rec);      // [TILE_CAND] x, y
  double2* rzs = rxy + TILE_CAND;                                 // [TILE_CAND] z, sorted index
  T* cq = reinterpret_cast<T*>(lds + L::cq);                      // [TILE_CAND]
  double* cacc = reinterpret_cast<double*>(lds + L::cacc);       // [4][TILE_CAND]
  double* tacc = reinterpret_cast<double*>(lds + L::tacc);       // [4][TILE_TGT]
  double* tpx = reinterpret_cast<double*>(lds + L::tpos);        // [3][TILE_TGT]
  T* tq = reinterpret_cast<T*>(lds + L::tq);                      // [TILE_TGT]
  TileQI Q;
  Q.bind(lds + L::queue + (threadIdx.x >> 6) * L::queue_bytes);
  const int lane = threadIdx.x & (WAVE - 1);
  const int n = pa.st.n;
  const size_t fo = (size_t)frame * n;
  const int* cs = pa.st.cell_start + (size_t)frame * (pa.cell.n_cells + 1);
  const double* sx = pa.st.x + fo; const double* sy = pa.st.y + fo; const double* sz = pa.st.z + fo;
  const double* sq = pa.st.q + fo;
  double* fp = pa.f_pair + (size_t)frame * 3 * n;
  double* us = pa.u_site ? pa.u_site + fo : nullptr;
  const double L0 = pa.cell.L[0], L1 = pa.cell.L[1], L2 = pa.cell.L[2];
  const double iL0 = pa.cell.invL[0], iL1 = pa.cell.invL[1], iL2 = pa.cell.invL[2];
  const double rc2 = pa.rc2;
  const T alpha = pa.alpha;
  // ZS: the z image nearest the target cell's centre zc, fixed at staging
  const int ncz = pa.cell.nc[2];
  const double zc = ((double)(c / (pa.cell.nc[0] * pa.cell.nc[1])) + 0.5) * (L2 / ncz);
  if (threadIdx.x < WAVE) tile_runs_fwd(pa.fwd_n, pa.fwd_lo, pa.fwd_hi, c, cs, R);

  // queued pair e = target | candidate << 8: the displacement again (the
  // same operations as the test, so the same bits), then both ends' sums
  auto eval = [&](int l) {
    const int e = Q.t[l];
    const int tt = e & 255, kc = e >> 8;
    const double2 cxy = rxy[kc];
    const double cz = rzs[kc].x;
    double ex = tpx[tt] - cxy.x, ey = tpx[TILE_TGT + tt] - cxy.y, ez = tpx[2 * TILE_TGT + tt] - cz;
    ex = fma(-L0, rint(ex * iL0), ex);
    ey = fma(-L1, rint(ey * iL1), ey);
    if (!ZS) ez = fma(-L2, rint(ez * iL2), ez);
    const T qx = (T)ex, qy = (T)ey, qz = (T)ez;
    const T qc = cq[kc], qt = tq[tt];
    T g, pot;
    g0_terms(qx * qx + qy * qy + qz * qz, alpha, g, pot);
    const T wc = qc * g, wt = qt * g;
    atomicAdd(tacc + tt, (double)(wc * qx));
    atomicAdd(tacc + TILE_TGT + tt, (double)(wc * qy));
    atomicAdd(tacc + 2 * TILE_TGT + tt, (double)(wc * qz));
    atomicAdd(tacc + 3 * TILE_TGT + tt, (double)(qc * pot));
    atomicAdd(cacc + kc, (double)(-wt * qx));
    atomicAdd(cacc + TILE_CAND + kc, (double)(-wt * qy));
    atomicAdd(cacc + 2 * TILE_CAND + kc, (double)(-wt * qz));
    atomicAdd(cacc + 3 * TILE_CAND + kc, (double)(qt * pot));
  };

  for (int t0 = t_lo; t0 < t_hi; t0 += TILE_TGT) {
    const TileMap m(min(TILE_TGT, t_hi - t0));
    const int j = t0 + m.ti;
    const double xt = sx[j], yt = sy[j], zt = sz[j];
    for (int i = threadIdx.x; i < 4 * TILE_TGT; i += TILE_THREADS) tacc[i] = 0.0;
    if ((int)threadIdx.x < m.ntc) {
      tq[threadIdx.x] = (T)sq[t0 + threadIdx.x];
      tpx[threadIdx.x] = xt; tpx[TILE_TGT + threadIdx.x] = yt; tpx[2 * TILE_TGT + threadIdx.x] = zt;
    }
    for (int c0 = 0;; c0 += TILE_CAND) {
      __syncthreads();
      const int total = R->total;
      const int nck = min(TILE_CAND, total - c0);
      for (int k = threadIdx.x; k < nck; k += TILE_THREADS) {
        const int s = tile_src(R, c0 + k);
        double z = sz[s];
        if (ZS) z -= L2 * rint((z - zc) * iL2);
        rxy[k] = make_double2(sx[s], sy[s]);
        rzs[k] = make_double2(z, __longlong_as_double((long long)s));
        cq[k] = (T)sq[s];
#pragma unroll
        for (int u = 0; u < 4; ++u) cacc[u * TILE_CAND + k] = 0.0;
      }
      __syncthreads();
      const int bs = nck > 0 ? (nck + m.nsl - 1) / m.nsl : 0;     // block length
      const int b0 = m.sl * bs, bend = b0 + bs;
      int k = b0 + (bs > 0 ? m.ti % bs : 0);
      int nq = 0;
      // two candidates per step: both records are read before either is
      // tested (independent chains the compiler interleaves)
      for (int it = 0; it < bs; it += 2) {
        int kk[2], kr[2];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          kk[h] = k;
          kr[h] = k < nck ? k : 0;
          if (++k == bend) k = b0;
        }
        double2 pxy[2], pzs[2];
#pragma unroll
        for (int h = 0; h < 2; ++h) { pxy[h] = rxy[kr[h]]; pzs[h] = rzs[kr[h]]; }
        bool in[2];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const bool valid = m.act && it + h < bs && kk[h] < nck;
          double ex = xt - pxy[h].x, ey = yt - pxy[h].y, ez = zt - pzs[h].x;
          ex = fma(-L0, rint(ex * iL0), ex);
          ey = fma(-L1, rint(ey * iL1), ey);
          if (!ZS) ez = fma(-L2, rint(ez * iL2), ez);
          in[h] = valid && (int)__double_as_longlong(pzs[h].y) > j && fma(ez, ez, fma(ey, ey, ex * ex)) < rc2;
        }
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          nq = tqi_push(Q, nq, in[h], tq_pack(m.ti, kk[h]));
          if (nq >= WAVE) {
            eval(lane);
            nq = tqi_pop(Q, nq);
          }
        }
      }
      if (lane < nq) eval(lane);
      __syncthreads();
      // the candidates' sums (each site appears in one staged set of a work item)
      for (int k2 = threadIdx.x; k2 < nck; k2 += TILE_THREADS) {
        const double fx = cacc[k2], fy = cacc[TILE_CAND + k2], fz = cacc[2 * TILE_CAND + k2];
        const double u = cacc[3 * TILE_CAND + k2];
        if (fx != 0.0 || fy != 0.0 || fz != 0.0 || u != 0.0) {
          const int s = (int)__double_as_longlong(rzs[k2].y);
          atomicAdd(fp + s, fx);
          atomicAdd(fp + n + s, fy);
          atomicAdd(fp + 2 * (size_t)n + s, fz);
          if (us) atomicAdd(us + s, 0.5 * KE * sq[s] * u);
        }
      }
      if (c0 + TILE_CAND >= total) break;
    }
    // the targets' sums (their staged sets are done: the last barrier above
    // follows every evaluation)
    if ((int)threadIdx.x < m.ntc) {
      const int jj = t0 + threadIdx.x;
      atomicAdd(fp + jj, tacc[threadIdx.x]);
      atomicAdd(fp + n + jj, tacc[TILE_TGT + threadIdx.x]);
      atomicAdd(fp + 2 * (size_t)n + jj, tacc[2 * TILE_TGT + threadIdx.x]);
      if (us) atomicAdd(us + jj, 0.5 * KE * sq[jj] * tacc[3 * TILE_TGT + threadIdx.x]);
    }
    __syncthreads();
  }
}

// ------------------------------------------------ site-electrode pairs

// LDS of the site-electrode tile: the runs, the staged atoms (x, y, z and
// the two charge sets), six FP64 sums and the position of every target, one
// queue of packed pair indices per wavefront
template <typename T>
struct ElecTileLds {
  static constexpr size_t runs = 0;
  static constexpr size_t pos = (sizeof(TileRuns) + 15) / 16 * 16;                  // x, y, z [TILE_CAND]
  static constexpr size_t qab = pos + 3 * (size_t)TILE_CAND * sizeof(double);       // qa, qb [TILE_CAND]
  static constexpr size_t tacc = qab + (2 * (size_t)TILE_CAND * sizeof(T) + 15) / 16 * 16;
  static constexpr size_t tpos = tacc + 6 * (size_t)TILE_TGT * sizeof(double);      // x, y, z [TILE_TGT]
  static constexpr size_t queue = tpos + 3 * (size_t)TILE_TGT * sizeof(double);
  static constexpr size_t queue_bytes = (TileQI::bytes() + 15) / 16 * 16;
  static constexpr size_t total = queue + (TILE_THREADS / WAVE) * queue_bytes;
};

// Site-electrode sums of the targets [t_lo, t_hi) of cell c (a launch of
// their own beside site_pairs_n3_tile): f_elec gets sum_i q_i g1(r) r_vec
// for the charges qa_s and qb_s (without k_e and Q_j).  A cell with no
// electrode atom in reach writes zeros.  Thread (ti, sl) tests candidates
// sl, sl + nsl, ... (the lanes of a wavefront read few distinct atoms,
// which LDS broadcasts); pairs inside the cutoff are evaluated 64 at a time
// from the wavefront's queue.  lds: ElecTileLds<T>::total bytes.
template <typename T, bool ZS>
__device__ __forceinline__ void site_elec_tile(const PairArgs<T>& pa, int c, int t_lo, int t_hi, int frame,
                                               unsigned char* lds) {
  using L = ElecTileLds<T>;
  const int n = pa.st.n;
  double* fe = pa.f_elec + (size_t)frame * 6 * n;
  if (pa.el.run_n[c] == 0) {
    for (int i = t_lo + threadIdx.x; i < t_hi; i += TILE_THREADS)
#pragma unroll
      for (int u = 0; u < 6; ++u) fe[(size_t)u * n + i] = 0.0;
    return;
  }
  TileRuns* R = reinterpret_cast<TileRuns*>(lds + L::runs);
  double* px = reinterpret_cast<double*>(lds + L::pos);
  double* py = px + TILE_CAND;
  double* pz = py + TILE_CAND;
  T* qa = reinterpret_cast<T*>(lds + L::qab);
  T* qb = qa + TILE_CAND;
  double* tacc = reinterpret_cast<double*>(lds + L::tacc);       // [6][TILE_TGT]
  double* tpx = reinterpret_cast<double*>(lds + L::tpos);        // [3][TILE_TGT]
  TileQI Q;
  Q.bind(lds + L::queue + (threadIdx.x >> 6) * L::queue_bytes);
  const int lane = threadIdx.x & (WAVE - 1);
  const size_t fo = (size_t)frame * n;
  const double* sx = pa.st.x + fo; const double* sy = pa.st.y + fo; const double* sz = pa.st.z + fo;
  const double* qa_e = pa.qa_s + (size_t)frame * pa.qa_stride;
  const double* qb_e = pa.qb_s;
  const double L0 = pa.cell.L[0], L1 = pa.cell.L[1], L2 = pa.cell.L[2];
  const double iL0 = pa.cell.invL[0], iL1 = pa.cell.invL[1], iL2 = pa.cell.invL[2];
  const double rc2 = pa.rc2;
  const T alpha = pa.alpha, eta = pa.eta;
  // ZS: the z image nearest the target cell's centre zc, fixed at staging
  const int ncz = pa.cell.nc[2];
  const double zc = ((double)(c / (pa.cell.nc[0] * pa.cell.nc[1])) + 0.5) * (L2 / ncz);
  if (threadIdx.x < WAVE) tile_elec_runs(pa.el, c, R);

  // queued pair e = target | atom << 8: the displacement again (the same
  // operations as the test), then the target's sums for both charge sets
  auto eval = [&](int l) {
    const int e = Q.t[l];
    const int tt = e & 255, kc = e >> 8;
    double ex = tpx[tt] - px[kc], ey = tpx[TILE_TGT + tt] - py[kc], ez = tpx[2 * TILE_TGT + tt] - pz[kc];
    ex = fma(-L0, rint(ex * iL0), ex);
    ey = fma(-L1, rint(ey * iL1), ey);
    if (!ZS) ez = fma(-L2, rint(ez * iL2), ez);
    const T qx = (T)ex, qy = (T)ey, qz = (T)ez;
    const T g = g1_force(qx * qx + qy * qy + qz * qz, alpha, eta);
    const T wa = qa[kc] * g, wb = qb[kc] * g;
    atomicAdd(tacc + tt, (double)(wa * qx));
    atomicAdd(tacc + TILE_TGT + tt, (double)(wa * qy));
    atomicAdd(tacc + 2 * TILE_TGT + tt, (double)(wa * qz));
    atomicAdd(tacc + 3 * TILE_TGT + tt, (double)(wb * qx));
    atomicAdd(tacc + 4 * TILE_TGT + tt, (double)(wb * qy));
    atomicAdd(tacc + 5 * TILE_TGT + tt, (double)(wb * qz));
  };

  for (int t0 = t_lo; t0 < t_hi; t0 += TILE_TGT) {
    const TileMap m(min(TILE_TGT, t_hi - t0));
    const double xt = sx[t0 + m.ti], yt = sy[t0 + m.ti], zt = sz[t0 + m.ti];
    for (int i = threadIdx.x; i < 6 * TILE_TGT; i += TILE_THREADS) tacc[i] = 0.0;
    if ((int)threadIdx.x < m.ntc) {
      tpx[threadIdx.x] = xt; tpx[TILE_TGT + threadIdx.x] = yt; tpx[2 * TILE_TGT + threadIdx.x] = zt;
    }
    for (int c0 = 0;; c0 += TILE_CAND) {
      __syncthreads();
      const int total = R->total;
      const int nck = min(TILE_CAND, total - c0);
      for (int k = threadIdx.x; k < nck; k += TILE_THREADS) {
        const int s = tile_src(R, c0 + k);
        double z = pa.el.z[s];
        if (ZS) z -= L2 * rint((z - zc) * iL2);
        px[k] = pa.el.x[s]; py[k] = pa.el.y[s]; pz[k] = z;
        qa[k] = (T)qa_e[s];
        qb[k] = qb_e ? (T)qb_e[s] : (T)0;
      }
      __syncthreads();
      const int n_iter = nck > 0 ? (nck + m.nsl - 1) / m.nsl : 0;
      int nq = 0;
      for (int it = 0; it < n_iter; it += 2) {
        int kk[2], kr[2];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          kk[h] = m.sl + (it + h) * m.nsl;
          kr[h] = kk[h] < nck ? kk[h] : 0;
        }
        double ax[2], ay[2], az[2];
#pragma unroll
        for (int h = 0; h < 2; ++h) { ax[h] = px[kr[h]]; ay[h] = py[kr[h]]; az[h] = pz[kr[h]]; }
        bool in[2];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          double ex = xt - ax[h], ey = yt - ay[h], ez = zt - az[h];
          ex = fma(-L0, rint(ex * iL0), ex);
          ey = fma(-L1, rint(ey * iL1), ey);
          if (!ZS) ez = fma(-L2, rint(ez * iL2), ez);
          in[h] = m.act && kk[h] < nck && fma(ez, ez, fma(ey, ey, ex * ex)) < rc2;
        }
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          nq = tqi_push(Q, nq, in[h], tq_pack(m.ti, kk[h]));
          if (nq >= WAVE) {
            eval(lane);
            nq = tqi_pop(Q, nq);
          }
        }
      }
      if (lane < nq) eval(lane);
      if (c0 + TILE_CAND >= total) break;
    }
    __syncthreads();
    if ((int)threadIdx.x < m.ntc) {
      const int jj = t0 + threadIdx.x;
#pragma unroll
      for (int u = 0; u < 6; ++u) fe[(size_t)u * n + jj] = tacc[u * TILE_TGT + threadIdx.x];
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

// work item b of a frame's tiles (tsplit > 0): share b mod tsplit of the
// sorted sites [t_lo, t_hi) of cell b / tsplit
__device__ __forceinline__ void tile_item(int b, int tsplit, const int* cs, int& c, int& t_lo, int& t_hi) {
  c = b / tsplit;
  const int s = b - c * tsplit;
  const int lo = cs[c], n = cs[c + 1] - lo;
  t_lo = lo + (int)(((long long)n * s) / tsplit);
  t_hi = lo + (int)(((long long)n * (s + 1)) / tsplit);
}

// workgroup b of a frame's site-pair work: with tsplit > 0, share b mod
// tsplit of the sites of cell b / tsplit (tiles; MODE 1: the site-electrode
// sums alone, MODE 2: the site-site sums with every pair once; ZS: z images
// fixed at staging, PairArgs::zshift); with tsplit == 0, sites 4b .. 4b+3
// (one wavefront each)
template <typename T, int MODE = 0, bool ZS = false>
__device__ __forceinline__ void site_pairs_block(const PairArgs<T>& pa, int b, int frame, unsigned char* lds) {
  if (pa.tsplit == 0) {
    // one wavefront per site, four per workgroup
    const int j = b * (TILE_THREADS / WAVE) + (threadIdx.x >> 6);
    if (j < pa.st.n)
      site_pairs_wave(pa.cell, pa.st, pa.alpha, pa.rc2, pa.f_pair, pa.u_site, j, frame,
                      reinterpret_cast<T*>(lds + (threadIdx.x >> 6) * wave_scratch_bytes<T>()));
    return;
  }
  int c, t_lo, t_hi;
  tile_item(b, pa.tsplit, pa.st.cell_start + (size_t)frame * (pa.cell.n_cells + 1), c, t_lo, t_hi);
  if (MODE == 2) site_pairs_n3_tile<T, ZS>(pa, c, t_lo, t_hi, frame, lds);
  else if (MODE == 1) site_elec_tile<T, ZS>(pa, c, t_lo, t_hi, frame, lds);
  else site_pairs_tile(pa, c, t_lo, t_hi, frame, lds);
}

}  // namespace cpm
