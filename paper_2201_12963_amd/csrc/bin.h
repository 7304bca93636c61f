// Cell binning of the electrolyte sites (the neighbour-list stage of an MD
// step, one of the itemised costs of the paper's timing breakdown), as the
// body of one workgroup of NT threads per frame:
//   1. cell id of every site (double precision, bit-identical to the integer
//      reference), kept in LDS; non-finite coordinates raise a status flag
//      and count as 0;
//   2. each wave owns a contiguous range of sites and walks it 64 at a time;
//      lanes with equal keys are grouped by AND-ing one ballot per key bit
//      (no atomics), every site records its rank among the earlier sites of
//      its wave and cell, and the lowest lane of each group advances the
//      wave's count of that cell;
//   3. a scan over (cell, wave) gives every wave its write offset per cell and
//      the cell_start array;
//   4. every site goes to offset + rank, all sites in parallel, so the sites
//      of a cell appear in increasing original index (a stable counting sort).
// The wrapped coordinates come from the same quotient x/L as the cell index,
// computed once in step 1 and carried to step 4 in one of two ways:
//   KEEP: every thread holds those of its first BATCH sites (and their
//     charges) in registers; sites beyond BATCH x NT are read and wrapped
//     again in step 4 (the same operations, so the same bits).  No scratch
//     round trip, for the one-frame launch, where the workgroup's latency
//     is the step's;
//   otherwise: a scratch array in global memory, which keeps the register
//     count (and the occupancy of the many-frame launches) down.
// The sorted FP64 SoA copies (wrapped x, y, z and the charge) are what the
// later kernels stream; the body also sums Q_j Z_j for the finite-field energy.
#pragma once
#include "common.h"

namespace cpm {


// sites per thread whose loads are issued together (KEEP: held in
// registers, 3 x 1024 sites for the one-frame workgroup)
constexpr int BIN_BATCH = 6;
constexpr int BIN_BATCH_KEEP = 3;

// LDS of the body (ints): cell ids, ranks, per-wave histograms, cell totals
template <int NT>
size_t bin_body_lds(int n_site, int n_cells) {
  return sizeof(int) * (2 * (size_t)n_site + (size_t)(NT / WAVE + 1) * n_cells);
}

// wrapped coordinate x - L floor(x/L) and cell index min(floor(f n), n - 1),
// f = x/L - floor(x/L), from one quotient (the same operations as
// cell_coord)
__device__ __forceinline__ double wrap_and_cell(double x, double L, int n, int& c) {
  const double t = x / L;
  const double fl = floor(t);
  const int ci = (int)floor((t - fl) * (double)n);
  c = ci < n - 1 ? ci : n - 1;
  return x - L * fl;
}

template <int NT, bool KEEP, int BATCH>
__device__ __forceinline__ void bin_block(const BinArgs& a, int frame, int* lds) {
  constexpr int NW = NT / WAVE;
  const int n_site = a.n_site;
  const Cell& cell = a.cell;
  const int n_cells = cell.n_cells;
  int* cid = lds;                              // [n_site]
  int* rnk = cid + n_site;                     // [n_site]
  int* hist = rnk + n_site;                    // [NW][n_cells]
  int* tot = hist + NW * n_cells;              // [n_cells]
  __shared__ double red[NW];

  const int tid = threadIdx.x;
  const int lane = tid & (WAVE - 1);
  const int wave = tid >> 6;
  const double* x = a.xyz_all + frame * a.frame_stride;
  const double* y = x + n_site;
  const double* z = y + n_site;
  int* cell_start = a.cell_start_all + (size_t)frame * (n_cells + 1);
  int* order = a.order_all + (size_t)frame * n_site;

  // KEEP: the first batch of every thread (wrapped coordinates and charges)
  double kx[BATCH], ky[BATCH], kz[BATCH], kq[BATCH];
  // otherwise: the scratch array
  double* wx = a.wrap_all + (size_t)frame * 3 * n_site;
  double* wy = wx + n_site;
  double* wz = wy + n_site;

  // 1. cell ids and wrapped coordinates; the loads of BATCH sites per
  // thread are issued together
  double zd = 0.0;
  int bad = 0;
  for (int i0 = tid; i0 < n_site; i0 += BATCH * NT) {
    double xv[BATCH], yv[BATCH], zv[BATCH], qv[BATCH];
#pragma unroll
    for (int u = 0; u < BATCH; ++u) {
      const int i = i0 + u * NT;
      xv[u] = yv[u] = zv[u] = qv[u] = 0.0;
      if (i < n_site) { xv[u] = x[i]; yv[u] = y[i]; zv[u] = z[i]; qv[u] = a.site_q[i]; }
    }
#pragma unroll
    for (int u = 0; u < BATCH; ++u) {
      const int i = i0 + u * NT;
      double ax = 0.0, ay = 0.0, az = 0.0;
      if (i < n_site) {
        double xi = xv[u], yi = yv[u], zi = zv[u];
        if (!isfinite(xi) || !isfinite(yi) || !isfinite(zi)) { bad = 1; xi = yi = zi = 0.0; }
        int cx, cy, cz;
        ax = wrap_and_cell(xi, cell.L[0], cell.nc[0], cx);
        ay = wrap_and_cell(yi, cell.L[1], cell.nc[1], cy);
        az = wrap_and_cell(zi, cell.L[2], cell.nc[2], cz);
        cid[i] = (cz * cell.nc[1] + cy) * cell.nc[0] + cx;
        if (!KEEP) { wx[i] = ax; wy[i] = ay; wz[i] = az; }
        zd += qv[u] * az;
      }
      if (KEEP && i0 == tid) { kx[u] = ax; ky[u] = ay; kz[u] = az; kq[u] = qv[u]; }
    }
  }
  if (bad) atomicOr(a.status, 1);
  for (int i = tid; i < NW * n_cells; i += NT) hist[i] = 0;
  zd = wave_sum(zd);
  if (lane == 0) red[wave] = zd;
  __syncthreads();
  if (tid == 0 && a.zdip_all) {
    double s = 0.0;
    for (int w = 0; w < NW; ++w) s += red[w];
    a.zdip_all[frame] = s;
  }

  // 2. ranks within (wave, cell) and per-wave counts; keys 0..n_cells
  // (n_cells pads the last batch)
  const int nbits = 32 - __clz(n_cells);
  const unsigned long long lt = (1ull << lane) - 1ull;
  const int per_wave = ((n_site + NW - 1) / NW + WAVE - 1) / WAVE * WAVE;
  const int lo = wave * per_wave;
  const int hi = min(n_site, lo + per_wave);
  // (the next batch's keys are read before this batch's ballots, so that
  // their LDS latency overlaps them)
  int key_next = (lo + lane < hi) ? cid[lo + lane] : n_cells;
  for (int base = lo; base < hi; base += WAVE) {
    const int i = base + lane;
    const int key = key_next;
    key_next = (i + WAVE < hi) ? cid[i + WAVE] : n_cells;
    unsigned long long eq = ~0ull;
    for (int b = 0; b < nbits; ++b) {
      const unsigned long long bb = __ballot((key >> b) & 1);
      eq &= ((key >> b) & 1) ? bb : ~bb;
    }
    const int r = __popcll(eq & lt);
    // rank in the low 24 bits, owning wave above (no division by per_wave later)
    if (key < n_cells) rnk[i] = (wave << 24) | (hist[wave * n_cells + key] + r);
    // every lane has read the count; the group leader advances it
    __builtin_amdgcn_wave_barrier();
    if (key < n_cells && r == 0) hist[wave * n_cells + key] += __popcll(eq);
    __builtin_amdgcn_wave_barrier();
  }
  __syncthreads();

  // 3. offsets: per cell, exclusive over waves (hist); then exclusive scan
  // over cells (tot); a site goes to tot + hist + rank
  for (int c = tid; c < n_cells; c += NT) {
    int run = 0;
    for (int w = 0; w < NW; ++w) {
      const int h = hist[w * n_cells + c];
      hist[w * n_cells + c] = run;
      run += h;
    }
    tot[c] = run;
  }
  __syncthreads();
  if (wave == 0) {
    int carry = 0;
    for (int c0 = 0; c0 < n_cells; c0 += WAVE) {
      const int c = c0 + lane;
      const int v = (c < n_cells) ? tot[c] : 0;
      int incl = v;
      for (int off = 1; off < WAVE; off <<= 1) {
        const int t = __shfl_up(incl, off, WAVE);
        if (lane >= off) incl += t;
      }
      if (c < n_cells) {
        tot[c] = carry + incl - v;     // exclusive start
        cell_start[c] = carry + incl - v;
      }
      carry += __shfl(incl, WAVE - 1, WAVE);
    }
    if (lane == 0) cell_start[n_cells] = carry;
  }
  __syncthreads();
  if (!KEEP) {
    // (many frames: the cell starts folded into the offsets here, one
    // register fewer in step 4, which keeps the spread's occupancy)
    for (int i = tid; i < NW * n_cells; i += NT) hist[i] += tot[i % n_cells];
    __syncthreads();
  }

  // 4. placement, every site independently
  double* sx = a.sx_all + (size_t)frame * n_site;
  double* sy = a.sy_all + (size_t)frame * n_site;
  double* sz = a.sz_all + (size_t)frame * n_site;
  double* sq = a.sq_all + (size_t)frame * n_site;
  // (all loads of a batch before any store: the output may not be assumed
  // apart from the input)
  for (int i0 = tid; i0 < n_site; i0 += BATCH * NT) {
    double xv[BATCH], yv[BATCH], zv[BATCH], qv[BATCH];
    int pv[BATCH];
    const bool first = KEEP && i0 == tid;
#pragma unroll
    for (int u = 0; u < BATCH; ++u) {
      const int i = i0 + u * NT;
      if (KEEP) { xv[u] = kx[u]; yv[u] = ky[u]; zv[u] = kz[u]; qv[u] = kq[u]; }
      else { xv[u] = yv[u] = zv[u] = qv[u] = 0.0; }
      pv[u] = 0;
      if (i < n_site) {
        if (!KEEP) { xv[u] = wx[i]; yv[u] = wy[i]; zv[u] = wz[i]; qv[u] = a.site_q[i]; }
        else if (!first) { xv[u] = x[i]; yv[u] = y[i]; zv[u] = z[i]; qv[u] = a.site_q[i]; }
        const int rw = rnk[i];
        const int c = cid[i];
        pv[u] = (KEEP ? tot[c] : 0) + hist[(rw >> 24) * n_cells + c] + (rw & 0xffffff);
      }
    }
#pragma unroll
    for (int u = 0; u < BATCH; ++u) {
      const int i = i0 + u * NT;
      if (i < n_site) {
        double xi = xv[u], yi = yv[u], zi = zv[u];
        if (KEEP && !first) {
          if (!isfinite(xi) || !isfinite(yi) || !isfinite(zi)) xi = yi = zi = 0.0;
          int c;
          xi = wrap_and_cell(xi, cell.L[0], cell.nc[0], c);
          yi = wrap_and_cell(yi, cell.L[1], cell.nc[1], c);
          zi = wrap_and_cell(zi, cell.L[2], cell.nc[2], c);
        }
        const int pos = pv[u];
        order[pos] = i;
        sx[pos] = xi; sy[pos] = yi; sz[pos] = zi; sq[pos] = qv[u];
      }
    }
  }
}

}  // namespace cpm
