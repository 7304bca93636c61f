// Cell binning of the electrolyte sites (the neighbour-list stage of an MD
// step, one of the four itemised costs in the paper's timing breakdown).
//
// One workgroup of 1024 threads bins one frame:
//   1. cell id of every site (double precision, bit-identical to the integer
//      reference), kept in LDS; non-finite coordinates raise a status flag;
//   2. per-wave histograms: each of the 16 waves owns a contiguous range of
//      sites and counts it 64 at a time; lanes with equal keys are grouped by
//      AND-ing one ballot per key bit (no atomics), and the lowest lane of each
//      group adds the group size;
//   3. a scan over (cell, wave) gives every wave its write offset per cell and
//      the cell_start array;
//   4. the same grouping places each site at offset + rank, so the sites of a
//      cell appear in increasing original index (a stable counting sort).
// The sorted SoA copies (wrapped x, y, z and the charge) are what the later
// kernels stream; the kernel also clears the frame's charge mesh and sums
// Q_j Z_j for the finite-field energy.
#include "common.h"

namespace cpm {

constexpr int BIN_THREADS = 1024;
constexpr int BIN_WAVES = BIN_THREADS / WAVE;

__global__ __launch_bounds__(BIN_THREADS) void k_bin_sites(
    int n_site, const double* __restrict__ xyz_all, size_t frame_stride,
    const double* __restrict__ site_q, Cell cell, int* __restrict__ cell_start_all,
    int* __restrict__ order_all, double* __restrict__ sx_all, double* __restrict__ sy_all,
    double* __restrict__ sz_all, double* __restrict__ sq_all, float* __restrict__ fx_all,
    float* __restrict__ fy_all, float* __restrict__ fz_all, float* __restrict__ fq_all,
    double* __restrict__ zdip_all, int* __restrict__ status) {
  extern __shared__ __align__(16) int lds[];
  const int n_cells = cell.n_cells;
  int* cid = lds;                              // [n_site]
  int* hist = lds + n_site;                    // [BIN_WAVES][n_cells]
  int* tot = hist + BIN_WAVES * n_cells;       // [n_cells]
  __shared__ double red[BIN_WAVES];
  __shared__ int carry_s;

  const int frame = blockIdx.x;
  const int tid = threadIdx.x;
  const int lane = tid & (WAVE - 1);
  const int wave = tid >> 6;
  const double* x = xyz_all + frame * frame_stride;
  const double* y = x + n_site;
  const double* z = y + n_site;
  int* cell_start = cell_start_all + (size_t)frame * (n_cells + 1);
  int* order = order_all + (size_t)frame * n_site;


  // 1. cell ids
  double zd = 0.0;
  int bad = 0;
  for (int i = tid; i < n_site; i += BIN_THREADS) {
    double xi = x[i], yi = y[i], zi = z[i];
    if (!isfinite(xi) || !isfinite(yi) || !isfinite(zi)) { bad = 1; xi = yi = zi = 0.0; }
    int cx = cell_coord(xi, cell.L[0], cell.nc[0]);
    int cy = cell_coord(yi, cell.L[1], cell.nc[1]);
    int cz = cell_coord(zi, cell.L[2], cell.nc[2]);
    cid[i] = (cz * cell.nc[1] + cy) * cell.nc[0] + cx;
    zd += site_q[i] * (zi - cell.L[2] * floor(zi / cell.L[2]));
  }
  if (bad) atomicOr(status, 1);
  for (int i = tid; i < BIN_WAVES * n_cells; i += BIN_THREADS) hist[i] = 0;
  zd = wave_sum(zd);
  if (lane == 0) red[wave] = zd;
  __syncthreads();
  if (tid == 0 && zdip_all) {
    double s = 0.0;
    for (int w = 0; w < BIN_WAVES; ++w) s += red[w];
    zdip_all[frame] = s;
  }

  // bits needed to hold keys 0..n_cells (n_cells is the padding key)
  int nbits = 32 - __clz(n_cells);
  const int per_wave = ((n_site + BIN_WAVES - 1) / BIN_WAVES + WAVE - 1) / WAVE * WAVE;
  const int lo = wave * per_wave;
  const int hi = min(n_site, lo + per_wave);
  const unsigned long long lt = (1ull << lane) - 1ull;

  // 2. per-wave histograms
  for (int base = lo; base < hi; base += WAVE) {
    int i = base + lane;
    int key = (i < hi) ? cid[i] : n_cells;
    unsigned long long eq = ~0ull;
    for (int b = 0; b < nbits; ++b) {
      unsigned long long bb = __ballot((key >> b) & 1);
      eq &= ((key >> b) & 1) ? bb : ~bb;
    }
    if (key < n_cells && (eq & lt) == 0ull) hist[wave * n_cells + key] += __popcll(eq);
  }
  __syncthreads();

  // 3. offsets: per cell, exclusive over waves; then exclusive scan over cells
  for (int c = tid; c < n_cells; c += BIN_THREADS) {
    int run = 0;
    for (int w = 0; w < BIN_WAVES; ++w) {
      int h = hist[w * n_cells + c];
      hist[w * n_cells + c] = run;
      run += h;
    }
    tot[c] = run;
  }
  __syncthreads();
  if (wave == 0) {
    int carry = 0;
    for (int c0 = 0; c0 < n_cells; c0 += WAVE) {
      int c = c0 + lane;
      int v = (c < n_cells) ? tot[c] : 0;
      int incl = v;
      for (int off = 1; off < WAVE; off <<= 1) {
        int t = __shfl_up(incl, off, WAVE);
        if (lane >= off) incl += t;
      }
      if (c < n_cells) {
        tot[c] = carry + incl - v;     // exclusive start
        cell_start[c] = carry + incl - v;
      }
      carry += __shfl(incl, WAVE - 1, WAVE);
    }
    if (lane == 0) { cell_start[n_cells] = carry; carry_s = carry; }
  }
  __syncthreads();
  for (int i = tid; i < BIN_WAVES * n_cells; i += BIN_THREADS) hist[i] += tot[i % n_cells];
  __syncthreads();

  // 4. stable placement
  double* sx = sx_all ? sx_all + (size_t)frame * n_site : nullptr;
  double* sy = sy_all ? sy_all + (size_t)frame * n_site : nullptr;
  double* sz = sz_all ? sz_all + (size_t)frame * n_site : nullptr;
  double* sq = sq_all ? sq_all + (size_t)frame * n_site : nullptr;
  float* fx = fx_all ? fx_all + (size_t)frame * n_site : nullptr;
  float* fy = fy_all ? fy_all + (size_t)frame * n_site : nullptr;
  float* fz = fz_all ? fz_all + (size_t)frame * n_site : nullptr;
  float* fq = fq_all ? fq_all + (size_t)frame * n_site : nullptr;
  for (int base = lo; base < hi; base += WAVE) {
    int i = base + lane;
    int key = (i < hi) ? cid[i] : n_cells;
    unsigned long long eq = ~0ull;
    for (int b = 0; b < nbits; ++b) {
      unsigned long long bb = __ballot((key >> b) & 1);
      eq &= ((key >> b) & 1) ? bb : ~bb;
    }
    int rank = __popcll(eq & lt);
    int pos = 0;
    if (key < n_cells) pos = hist[wave * n_cells + key] + rank;
    if (key < n_cells) {
      double xi = x[i], yi = y[i], zi = z[i];
      if (!isfinite(xi) || !isfinite(yi) || !isfinite(zi)) xi = yi = zi = 0.0;
      xi -= cell.L[0] * floor(xi / cell.L[0]);
      yi -= cell.L[1] * floor(yi / cell.L[1]);
      zi -= cell.L[2] * floor(zi / cell.L[2]);
      order[pos] = i;
      if (sx) { sx[pos] = xi; sy[pos] = yi; sz[pos] = zi; sq[pos] = site_q[i]; }
      if (fx) { fx[pos] = (float)xi; fy[pos] = (float)yi; fz[pos] = (float)zi; fq[pos] = (float)site_q[i]; }
    }
    // every lane has read its offset; the group leader advances it
    __builtin_amdgcn_wave_barrier();
    if (key < n_cells && rank == 0) hist[wave * n_cells + key] += __popcll(eq);
    __builtin_amdgcn_wave_barrier();
  }
}

size_t bin_lds_bytes(int n_site, int n_cells) {
  return sizeof(int) * ((size_t)n_site + (size_t)(BIN_WAVES + 1) * n_cells);
}

void launch_bin_sites(hipStream_t s, int n_frames, int n_site, const double* xyz, size_t frame_stride,
                      const double* site_q, Cell cell, int* cell_start, int* site_order,
                      double* sx, double* sy, double* sz, double* sq, float* fx, float* fy, float* fz,
                      float* fq, double* zdip, int* status) {
  size_t lds = bin_lds_bytes(n_site, cell.n_cells);
  hipLaunchKernelGGL(k_bin_sites, dim3(n_frames), dim3(BIN_THREADS), lds, s, n_site, xyz,
                     frame_stride, site_q, cell, cell_start, site_order, sx, sy, sz, sq, fx, fy, fz, fq,
                     zdip, status);
}

}  // namespace cpm
