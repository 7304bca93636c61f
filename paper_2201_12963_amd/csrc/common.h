// Internal declarations shared by the HIP translation units of libcpm.
// Device helpers, parameter blocks passed by value to kernels, and the host
// launchers each .hip file exports to the C-ABI layer (api.cpp).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace cpm {

constexpr double KE = 1.43996454784;   // eV nm / e^2
constexpr double EPS0 = 1.0 / (4.0 * M_PI * KE);   // e / (V nm)
constexpr int WAVE = 64;
constexpr int MAX_FFT_FACTORS = 12;
constexpr int MAX_ORDER = 7;
constexpr int STENCIL_MAX = 32;   // index runs of the neighbour cells of a cell (one wavefront half)
// dynamic LDS a launch may ask for (of the 160 KiB of a gfx950 CU)
constexpr size_t LDS_LIMIT = 150 * 1024;
// cell tiles of the real-space sums: workgroup size, candidates staged in
// LDS per pass (256: ~32 KB of LDS per workgroup, five per CU; 512 left
// three and measured 8% slower), targets per chunk
constexpr int TILE_THREADS = 256;
constexpr int TILE_CAND = 256;
constexpr int TILE_TGT = 64;

// ---------------------------------------------------------------- geometry

struct Cell {          // periodic orthorhombic cell and its cell-list grid
  double L[3];
  double invL[3];
  int nc[3];           // cells per axis, n_d = max(1, floor(L_d / rcut))
  int img[3];          // extra images per axis: floor(rcut/L + 1/2)
  int n_cells;
  // stencil of every cell (device tables, fixed by the grid): the distinct
  // neighbour cells sorted and joined into groups of consecutive cell
  // indices [lo, hi); cell c has grp_n[c] <= STENCIL_MAX groups, at
  // grp_lo/grp_hi[c * STENCIL_MAX + k] (a fixed stride, so the groups are read
  // in the same step as their count).  A group's members are one contiguous
  // index range [cs[lo], cs[hi]) of any cell-sorted array with cell_start cs.
  const int* grp_n;
  const int* grp_lo;
  const int* grp_hi;
};

struct FFTPlan1D {     // mixed-radix Stockham plan for one axis
  int n;
  int nfac;
  int fac[MAX_FFT_FACTORS];
  const double2* tw;   // e^{-2 pi i t / n}, t = 0..n-1
  const float2* twf;
  int planes;          // x plan only: most planes per many-frame x-y workgroup (0: as many as fit)
};

struct MeshInfo {
  int K[3];
  int M;               // Kx*Ky*Kz
  int order;
  double h[3];
  double invh[3];
};

// ------------------------------------------------------------ device utils

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, WAVE);
  return v;
}

// Sums of eight values over the wavefront in 10 exchanges instead of 8 x 6:
// each exchange step halves the values a lane keeps (it sends the half its
// partner keeps), down to one, then the last three steps sum that one.
// Afterwards lane l holds the total of value l >> 3.
template <typename T>
__device__ __forceinline__ T wave_sum8(const T (&v)[8]) {
  const int lane = threadIdx.x & (WAVE - 1);
  T a[4], b[2];
  const bool h32 = lane & 32, h16 = lane & 16, h8 = lane & 8;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const T keep = h32 ? v[i + 4] : v[i], send = h32 ? v[i] : v[i + 4];
    a[i] = keep + __shfl_xor(send, 32, WAVE);
  }
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    const T keep = h16 ? a[i + 2] : a[i], send = h16 ? a[i] : a[i + 2];
    b[i] = keep + __shfl_xor(send, 16, WAVE);
  }
  T c = (h8 ? b[1] : b[0]) + __shfl_xor(h8 ? b[0] : b[1], 8, WAVE);
  c += __shfl_xor(c, 4, WAVE);
  c += __shfl_xor(c, 2, WAVE);
  c += __shfl_xor(c, 1, WAVE);
  return c;
}

// value of v in lane l (l uniform), for every lane
__device__ __forceinline__ float read_lane(float v, int l) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}
__device__ __forceinline__ double read_lane(double v, int l) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), l);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// sum over a 256-thread workgroup (red: 4 doubles of LDS); every thread gets the total
__device__ __forceinline__ double block_sum_d(double v, double* red) {
  v = wave_sum(v);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  return red[0] + red[1] + red[2] + red[3];
}

__device__ __forceinline__ double wrap01(double t) { return t - floor(t); }

// cell index of a coordinate along one axis, bit-identical to the integer
// reference: f = x/L - floor(x/L); c = min(floor(f * n), n - 1)
__device__ __forceinline__ int cell_coord(double x, double L, int n) {
  double t = x / L;
  double f = t - floor(t);
  int c = (int)floor(f * (double)n);
  return c < n - 1 ? c : n - 1;
}

// minimum-image displacement component
__device__ __forceinline__ double min_image(double d, double L, double invL) {
  return d - L * rint(d * invL);
}
__device__ __forceinline__ float min_image(float d, float L, float invL) {
  return d - L * rintf(d * invL);
}

// neighbouring cells along one axis without repeats: offsets -1,0,1 when
// n >= 3, {0,1} when n == 2, {0} when n == 1
__device__ __forceinline__ int stencil_count(int n) { return n >= 3 ? 3 : n; }
__device__ __forceinline__ int stencil_cell(int c, int s, int n) {
  if (n >= 3) { int v = c + s - 1; return v < 0 ? v + n : (v >= n ? v - n : v); }
  return (c + s) % n;
}

// Workgroups of a launch are dispatched to the 8 XCDs in turn (block b to
// XCD b mod 8).  Mapping dispatch index b of nb blocks to the logical index
// returned here gives each XCD one contiguous range of logical blocks, so a
// kernel whose neighbouring logical blocks share data (cell-sorted targets)
// keeps that data in one XCD's L2.  A bijection on [0, nb) whatever the
// actual placement.  Worth it only where every target costs about the same:
// contiguous ranges put unequal targets on unequal XCDs.
__device__ __forceinline__ int xcd_block(int b, int nb) {
  const int x = b & 7, i = b >> 3, q = nb >> 3, r = nb & 7;
  return x * q + (x < r ? x : r) + i;
}

template <typename T> struct Real2;
template <> struct Real2<double> { using type = double2; };
template <> struct Real2<float> { using type = float2; };


// ------------------------------------------------------ kernel arguments

template <typename T>
struct SiteSet {       // cell-sorted sites of frame 0 (add frame * n to index)
  // positions and charges stay FP64 in every precision: displacements are
  // formed in FP64 and only the pair arithmetic runs in T
  const double* x; const double* y; const double* z; const double* q;
  const int* order; const int* cell_start;
  int n;
};

template <typename T>
struct ElecSet {       // cell-sorted electrode atoms (static), FP64 positions
  const double* x; const double* y; const double* z;
  const int* orig; const int* cell; const int* cell_start;
  int n;
  // electrode atoms in reach of every cell: run_n[c] <= STENCIL_MAX index
  // runs [run_lo, run_hi) of the sorted atoms at [c * STENCIL_MAX + k]
  // (non-empty only)
  const int* run_n; const int* run_lo; const int* run_hi;
};

// Many frames: the site-force interpolation done by the field's inverse x-y
// pass, plane by plane, while each plane's field is in LDS.  A site's
// stencil covers P consecutive planes (slot = plane - first plane, mod K_z);
// the workgroup of a plane writes, for every site its stencil reaches, the
// plane's share of the interpolated field, sum over the in-plane points of
// w_x w_y E times w_z of the slot, for the frame's field (components 0-2)
// and the static second field Eb (3-5).  The site-force kernel sums the P
// slots.  Candidates come from the binning's z layers around the planes.
template <typename T>
struct InterpArgs {
  const double* sx; const double* sy; const double* sz;   // [frame][n] cell-sorted wrapped positions
  const int* cell_start;        // [frame][n_cells + 1]
  int n, n_cells, nxy, ncz;     // sites; cells; cells per z layer; z layers
  double inv_wz;                // z layers per nm
  const T* Eb;                  // [3][M] static second field, or nullptr
  T* part;                      // [frame][6 P][n]: share (slot, component) at row slot * 6 + component, sites in sorted order
  MeshInfo mi;
};

template <typename T>
struct ForceArgs {
  T alpha, eta;
  double rc2;                  // squared cutoff (the cutoff test is FP64 in every precision)
  // k-space field meshes (V/nm, k_e included), [frame][3][M] and a shared
  // second set (or nullptr); mesh geometry for the spline gather
  const T* Ea; size_t Ea_frame_stride;
  const T* Eb;
  MeshInfo mi;
  // explicit-Ewald path instead of a mesh: k-space field at the sites,
  // [frame][3][n_site] in cell-sorted order (V/nm), or nullptr
  const double* Esite;
  // electrode charges, original order: qa per frame (stride n_elec), qb shared;
  // the same in the electrodes' cell-sorted order (what the pair walk reads)
  const double* qa; size_t qa_frame_stride;
  const double* qb;
  const double* qa_s;
  const double* qb_s;
  double out_scale;          // multiplies the Coulomb force (e.g. -1 for a gradient)
  double field;              // -dV/Lz for the finite field (0 otherwise), added along z
  double fieldb;             // same for the second set (per unit dV)
  // slab geometry: the uniform Coulomb field of the dipole correction,
  // -k_e 4 pi / V (sum_j Q_j Z_j + z.qa) per frame (V/nm), added along z and
  // scaled by out_scale like the rest of the Coulomb force; nullptr otherwise
  const double* field_frame;
  // outputs
  double* f_out; size_t f_frame_stride;   // [frame][n_dv][3][n_site] original order
  // instead of f_out (if non-null): [frame][2][3][n_site] original order,
  // the force at dV = 0 and its derivative by dV, expanded over the sweep
  // by launch_expand_forces
  double* f_comp;
  int n_dv; const double* dv;             // dV values of the sweep (n_dv == 1: dv may be nullptr)
  double* u_site;                          // [frame][n_site] 1/2 Q_j sum Q_j' g0 (sorted order), or nullptr
  // site-electrode sums already made by the pair tiles, [frame][6][n_site]
  // sorted order (charges a, then b), or nullptr: the site-force kernel
  // then walks the electrode atoms itself
  const double* f_elec;
  // site-site real-space sum of every site, sum_j' Q_j' g0(r) r_vec without
  // k_e and Q_j, [frame][3][n_site] sorted order: written by the site-pair
  // kernel, read by the site-force kernel
  double* f_pair;
};

// LDS of the pair scratch of one 256-thread workgroup: four wavefronts,
// each with a queue of 5 x 128 values and 64 ints of partner runs
template <typename T>
constexpr size_t pair_queue_lds() { return 4 * (5 * 128 * sizeof(T) + 64 * sizeof(int)); }

// real-space part of b: one wavefront per electrode atom, four per
// workgroup (tiles == 0; hosted as extra workgroups of another launch for
// one frame), or cell tiles over fixed work items of at most TILE_TGT atoms
// of one cell (tiles != 0; many frames)
template <typename T>
struct RealBArgs {
  int n_blocks;                // workgroups per frame (ceil(n_elec / 4), or the item count), 0: none
  Cell cell;
  SiteSet<T> st;               // cell-sorted sites
  T alpha, eta;
  double rc2;
  ElecSet<T> el;
  T* phi_out;                  // [frame][n_elec] original order
  int tiles;
  const int* item_c;           // cell of item b
  const int* item_lo;          // its atoms [item_lo, item_hi) of the sorted electrode arrays
  const int* item_hi;
};

// site-site forces hosted as extra workgroups of another launch: cell tiles
// (tsplit > 0 workgroups per cell, each a contiguous share of its sites;
// for many frames) or one wavefront per site (tsplit == 0; for one frame,
// where the shorter per-wavefront chains win)
template <typename T>
struct PairArgs {
  int n_blocks;                // workgroups per frame (n_cells * tsplit, or ceil(n_site / 4)), 0: none
  int tsplit;
  Cell cell;
  SiteSet<T> st;
  T alpha;
  double rc2;
  double* f_pair;              // [frame][3][n_site] sorted order
  double* u_site;              // [frame][n_site] sorted order, or nullptr
  // tiles only, once the electrode charges are known (batched form): the
  // site-electrode sums as well, for the charges qa_s (per frame, stride
  // qa_stride) and qb_s (shared, or nullptr), in the atoms' sorted order;
  // f_elec [frame][6][n_site] sorted order, or nullptr for none
  ElecSet<T> el;
  T eta;
  const double* qa_s; size_t qa_stride;
  const double* qb_s;
  double* f_elec;
  // tiles without periodic images: the forward half of every cell's stencil
  // (the cell itself and its neighbours of larger index, as runs like
  // Cell::grp_*), or nullptr; with it every site pair is evaluated once and
  // both ends are accumulated (f_pair and u_site then take atomic adds and
  // are cleared before the launch)
  const int* fwd_n;
  const int* fwd_lo;
  const int* fwd_hi;
  // z images fixed per work item (no periodic images, the z axis cut into at
  // least five cells and longer than 2 rcut plus a cell): candidates are
  // staged at the z image nearest the centre of the target cell, which for
  // every pair inside the cutoff is the minimum image, so the tests skip the
  // z minimum image
  int zshift;
};

// z pass: a lane prefetches the multiplier (and saved spectrum) of the
// first ZPASS_PREFETCH of its column's points into registers, the rest is
// read when used; columns of at most ZPASS_MAX_POINTS points
constexpr int ZPASS_PREFETCH = 8;
constexpr int ZPASS_MAX_POINTS = 2048;

struct ZPassArgs {
  int Kx, Ky, Kz;
  int cpw;                 // (x, y) columns per workgroup, one wavefront each (<= 4)
  int n_blocks;            // workgroups per frame: ceil(Kx Ky / cpw)
  int mode;                // 0: potential, 1: field (ik)
  double twopi_L[3];       // 2 pi / L_d
};

// Many-frame z passes and the planes the electrode stencils reach (bit z of
// w; K_z <= 256): the field pass reads the electrode spectrum only there
// (the other planes are taken as zero), the potential pass writes its
// result only there (nothing else reads it)
struct ZMask {
  unsigned long long w[4];
};

struct EnergyArgs {
  int n_elec, n_site, n_ek;
  const double* Q0; const double* b;            // [frame][n_elec]
  const double* Sc; const double* c; const double* d; const double* ze;   // [n_elec]
  const double* u_site;                          // [frame][n_site]
  const double* ek;                              // [frame][n_ek] k-space energy parts
  const double* zdip;                            // [frame]
  double self_energy;
  int ff; double Lz;
  double slab_kappa;                             // slab: k_e 4 pi / V (U_elyt += kappa/2 zdip^2), else 0
  int n_dv; const double* dv; double dv_single;
  double* out;                                   // [frame][n_dv][2]
};

// Centred cardinal B-spline weights along one axis.  A particle at scaled
// coordinate u (mesh units) touches the P mesh points m = first + t,
// t = 0..P-1, first = floor(u - P/2) + 1, with weight M_P(u - m + P/2).
// Writing s = u - P/2 and f = s - floor(s), the argument for point t is
// f + (P - 1 - t).  The values B[j] = M_n(f + j), j = 0..P-1, follow from
// the Cox-de Boor recursion M_n(x) = [x M_{n-1}(x) + (n - x) M_{n-1}(x-1)]/(n-1)
// starting at M_1(f + j) = [j == 0].
// The recursion is evaluated as a triangle for an order P (<= MAX_ORDER)
// known only at run time, fully unrolled so that it stays in registers:
// B[j] (j < P) is the weight of mesh point first + P - 1 - j; returns first
// (not wrapped).  The scaled coordinate u (up to K) is given in FP64: the
// stencil start and the fractional offset are taken in FP64, the weights in T.
// ORD = 5: the order is known to be 5; ORD = -1: it is known not to be
// (either keeps only one of the two evaluations below in the kernel, which
// saves registers); ORD = 0: decided at run time.
template <typename T, int ORD = 0>
__device__ __forceinline__ int spline_triangle_d(double u, int P, T (&B)[MAX_ORDER]) {
  if (ORD == 5) P = 5;
  const double s = u - (double)P * 0.5;
  const double fl = floor(s);
  const T f = (T)(s - fl);
  if (ORD == 5 || (ORD == 0 && P == 5)) {
    // order 5 (the quartic B-spline): the triangle below written out as
    // polynomials in f, 24 B_j = f^4, 1 + 4f + 6f^2 + 4f^3 - 4f^4,
    // 11 + 12f - 6f^2 - 12f^3 + 6f^4, 11 - 12f - 6f^2 + 12f^3 - 4f^4,
    // (1 - f)^4 (Horner: a short dependent chain instead of ten steps)
    const T c = (T)(1.0 / 24.0);
    const T f2 = f * f, g = (T)1 - f, g2 = g * g;
    B[0] = c * (f2 * f2);
    B[1] = c * ((T)1 + f * ((T)4 + f * ((T)6 + f * ((T)4 - (T)4 * f))));
    B[2] = c * ((T)11 + f * ((T)12 + f * ((T)-6 + f * ((T)-12 + (T)6 * f))));
    B[3] = c * ((T)11 + f * ((T)-12 + f * ((T)-6 + f * ((T)12 - (T)4 * f))));
    B[4] = c * (g2 * g2);
#pragma unroll
    for (int j = 5; j < MAX_ORDER; ++j) B[j] = (T)0;
    return (int)fl + 1;
  }
  B[0] = (T)1;
#pragma unroll
  for (int j = 1; j < MAX_ORDER; ++j) B[j] = (T)0;
#pragma unroll
  for (int n = 2; n <= MAX_ORDER; ++n) {
    if (n <= P) {
      const T inv = (T)1 / (T)(n - 1);
#pragma unroll
      for (int j = n - 1; j >= 0; --j) {
        T x = f + (T)j;
        T prev = (j > 0) ? B[j - 1] : (T)0;
        B[j] = (x * B[j] + ((T)n - x) * prev) * inv;
      }
    }
  }
  return (int)fl + 1;
}

// first mesh point of the stencil of scaled coordinate u, as spline_triangle_d
template <typename T>
__device__ __forceinline__ int spline_first(T u, int P) {
  return (int)floor(u - (T)P * (T)0.5) + 1;
}


// --------------------------------------------------------------- launchers

// cell binning (bin.h, k_bin.hip)
struct BinArgs {
  int n_site;
  const double* xyz_all;       // [frame][3][n_site], frame_stride apart
  size_t frame_stride;
  const double* site_q;        // [n_site]
  Cell cell;
  int* cell_start_all;         // [frame][n_cells + 1]
  int* order_all;              // [frame][n_site]
  double *sx_all, *sy_all, *sz_all, *sq_all;   // [frame][n_site]
  double* zdip_all;            // [frame]
  int* status;
  double* wrap_all;            // scratch [frame][3][n_site]: wrapped coordinates, original order
};
void launch_bin_sites(hipStream_t s, int n_frames, const BinArgs& a);

// real-space sums (k_realspace.hip)
template <typename T>
void launch_real_b_t(hipStream_t s, int n_frames, const RealBArgs<T>& rb);
template <typename T>
void launch_site_pairs_t(hipStream_t s, int n_frames, const PairArgs<T>& pa);
// LDS of a site-pair workgroup (tsplit > 0: tile form)
template <typename T>
size_t site_pairs_lds(int tsplit, bool n3);
// forces: the site-force workgroups; ea (or nullptr): one more workgroup per
// frame that reduces the energies
template <typename T>
// epart (many frames): the interpolated fields as per-plane shares written
// by the field's inverse x-y pass ([frame][6 P][n_site], see InterpArgs), in
// place of the gathers from fa.Ea and fa.Eb, or nullptr
void launch_site_forces_t(hipStream_t s, int n_frames, const Cell& cell, const ElecSet<T>& el,
                          const SiteSet<T>& st, const ForceArgs<T>& fa, bool forces, const EnergyArgs* ea,
                          const T* epart = nullptr);
size_t bin_lds_bytes(int n_site, int n_cells);

// particle-mesh steps (k_pppm.hip)
// Slab geometry's dipole correction (charged-sheet correction of the
// z-periodic box): kappa = k_e 4 pi / V, electrode heights ze (wrapped),
// the electrolyte dipole zdip[frame] = sum_j Q_j Z_j; kappa == 0 means none
struct SlabTerms {
  double kappa;
  const double* ze;
  const double* zdip;
  int n_elec;
};

// b_i -= kappa z_i zdip (the electrolyte-electrode block of the correction)
__device__ __forceinline__ double slab_b_term(const SlabTerms& sl, int i, int frame) {
  return sl.kappa != 0.0 ? sl.kappa * sl.ze[i] * sl.zdip[frame] : 0.0;
}

// One workgroup: field[frame] = -kappa (zdip[frame] + z.q), q of that frame
__device__ __forceinline__ void slab_field_block(const SlabTerms& sl, const double* q, double* field, int frame) {
  __shared__ double red[16];
  double acc = 0.0;
  for (int i = threadIdx.x; i < sl.n_elec; i += blockDim.x) acc += sl.ze[i] * q[i];
  acc = wave_sum(acc);
  if ((threadIdx.x & (WAVE - 1)) == 0) red[threadIdx.x / WAVE] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < (int)(blockDim.x / WAVE); ++w) t += red[w];
    field[frame] = -sl.kappa * (sl.zdip[frame] + t);
  }
}

template <typename T>
void launch_spread_elec_t(hipStream_t s, int n_frames, int n_touch, const int* touch, const int* rowptr,
                          const int* col, const T* val, const double* q, size_t q_stride, T* rho, int M,
                          const SlabTerms& sl = SlabTerms{}, double* slab_field = nullptr, int n_elec = 0);
// the slab field alone (one workgroup per frame), where no spread launch hosts it
void launch_slab_field(hipStream_t s, int n_frames, const SlabTerms& sl, const double* q, size_t q_stride,
                       double* field);
template <typename T>
void launch_gather_b_t(hipStream_t s, int n_frames, int n_elec, int P3, const int* gidx, const T* gw,
                       const T* phi, int M, const T* phi_real, double* b, const SlabTerms& sl = SlabTerms{});

struct MDArgs;   // the MD loop's arguments (below)

// FFT passes (k_fft.hip)
template <typename T, typename T2>
void launch_fft_xy_t(hipStream_t s, int n_frames, const FFTPlan1D& px, const FFTPlan1D& py, int Kz,
                     int mode, const T* in_re, const T2* in_c, T2* out_c, T* out_re, T* out_im,
                     size_t out_re_stride = 0, const int* zl = nullptr, int n_zl = 0);
// (zl: many frames only, the n_zl planes to transform, ascending; nullptr: all)
// inverse x-y pass of the field: c1 -> E[0] (re), E[1] (im); c2 -> E[2];
// both in one launch; E frames frame_stride apart, components M apart
template <typename T, typename T2>
void launch_fft_xy_field_inv_t(hipStream_t s, int n_frames, const FFTPlan1D& px, const FFTPlan1D& py, int Kz,
                               const T2* c1, const T2* c2, T* E, size_t frame_stride,
                               const InterpArgs<T>* ia = nullptr);
// z pass; z_pass false launches only the workgroups of pa (if any)
template <typename T, typename T2>
void launch_fft_z_t(hipStream_t s, int n_frames, const FFTPlan1D& pz, const ZPassArgs& za, const T* G,
                    T2* data1, T2* data2, T2* save, int add_saved, double* energy_part, bool z_pass = true,
                    const RealBArgs<T>* rb = nullptr, const PairArgs<T>* pa = nullptr, const ZMask* zm = nullptr,
                    const T2* in1 = nullptr, const MDArgs* lj = nullptr);
// (in1: the input spectrum if not data1, which then only takes the result;
// the masked many-frame launches work in place)
template <typename T, typename T2>
size_t fft_xy_spread_lds(int Kx, int Ky, int pl = 1);
// dynamic LDS of an x-y launch holding `planes` planes of elt_bytes complex values
size_t fft_xy_lds_bytes(int Kx, int Ky, int elt_bytes, int planes);
// threads of the spread + x-y transform workgroups (which also run the
// binning): many-frame launches SPREAD_THREADS (256 measured faster than
// 512 there: 3.7 -> 2.5 ms per 4096 frames), one-frame launches
// SPREAD_THREADS_ONE (four wavefronts per SIMD for the binning workgroup,
// which is then on the step's critical path); the planes' staging is done
// by the first SPREAD_THREADS threads in either case
constexpr int SPREAD_THREADS = 256;
constexpr int SPREAD_THREADS_ONE = 1024;
// sites per thread whose z is read together by the spread's staging (the
// per-wavefront lists hold SPREAD_LIST / 64 entries per wavefront, SPREAD_LIST
// entries per workgroup in either configuration)
constexpr int SPREAD_LIST = 4096;
// LDS of such a workgroup running the binning body
size_t bin_lds_spread(int n_site, int n_cells);
template <typename T, typename T2>
void launch_fft_xy_spread_t(hipStream_t s, int n_frames, const FFTPlan1D& px, const FFTPlan1D& py, int Kz,
                            const MeshInfo& mi, const BinArgs& ba, T* rho_out, T2* out_c, bool planes = true,
                            bool bin = false);

// explicit Ewald (k_ewald.hip)
void launch_ewald_sf(hipStream_t s, int n_frames, int nk, const double* kv, const double* ew,
                     const SiteSet<double>& st, double2* rho, double* ek);
void launch_ewald_phi(hipStream_t s, int n_frames, int nk, int n_elec, const double* ew, const double2* eph,
                      const double2* rho, const double* phi_real, double* b, const SlabTerms& sl = SlabTerms{});
void launch_ewald_rho_all(hipStream_t s, int n_frames, int nk, int n_elec, const double2* eph, const double* q,
                          size_t q_stride, const double2* rho, double2* out);
void launch_ewald_field(hipStream_t s, int n_frames, int nk, const double* kv, const double* ew,
                        const SiteSet<double>& st, const double2* rho, double* E);

// dense linear algebra (k_linalg.hip)
constexpr int GJ_BLOCK = 32;
void launch_elastance_real(hipStream_t s, int n, const double* ex, const double* ey, const double* ez,
                           const Cell& cell, double alpha, double eta, double rcut, double self_term, double* A);
void launch_phase_matrix(hipStream_t s, int n, int nkc, int k0, int nk, const double* kv, const double* sk,
                         const double* ex, const double* ey, const double* ez, double* C);
void launch_gemm_nt(hipStream_t s, int M, int N, int K, double alpha, const double* A, int lda, const double* B,
                    int ldb, double beta, double* D, int ldd);
void launch_symmetrize(hipStream_t s, int n, double* A);
void launch_gj_invert(hipStream_t s, int n, double* A, double* dinv, double* pc, double* rx, int* flag);
void launch_matvec(hipStream_t s, int n, const double* Mx, const double* x, double* y);
void launch_dot(hipStream_t s, int n, const double* a, const double* b, double* out);
void launch_rank1(hipStream_t s, int n, double* S, const double* u, const double* sc);
void launch_charges(hipStream_t s, int n_frames, int n, const double* S, const double* b, const double* Sc, double dv,
                    double* Q0, double* q, const int* epos = nullptr, double* qs = nullptr);
// dst[f][epos[i]] = src[f][i] for n values of n_frames frames
void launch_permute(hipStream_t s, int n_frames, int n, const int* epos, const double* src, double* dst);
void launch_expand_charges(hipStream_t s, int n_frames, int n_elec, int n_dv, const double* dv, const double* Q0,
                           const double* Sc, double* q);
// out[f][v][k] = comp[f][0][k] + dv[v] comp[f][1][k] over the 3 n_site
// values k of every frame f and dV v
void launch_expand_forces(hipStream_t s, int n_frames, int n_site, int n_dv, const double* dv, const double* comp,
                          double* out);

void launch_adjoint_rhs(hipStream_t s, int n, const double* q, const double* t, const double* c, double dv, double* g);
void launch_sub(hipStream_t s, int n, const double* a, const double* b, double* out, const int* epos = nullptr,
                double* out_s = nullptr);
void launch_grad_finish(hipStream_t s, int n, const double* q, const double* t, const double* lam, const double* c,
                        const double* energy, double* loss, double* dldv);

// mixed precision (k_mixed.hip)
void launch_split_matrix(hipStream_t s, int n, int n_pad, const double* S, float* Sf, unsigned short* split);
void launch_split_b(hipStream_t s, int n_frames, int n, int n_pad, const double* b, unsigned short* split);
// column sums of Sf over the neutrality groups, colsum [2][n] (FP64)
void launch_colsum(hipStream_t s, int n, const float* Sf, const unsigned char* sub1, double* colsum);
// one-frame mixed charges: q = Sf b - (colsum_g . b)/n_g + dV S c, FP64 products
void launch_charges_mixed(hipStream_t s, int n_frames, int n, const float* Sf, const double* colsum,
                          const unsigned char* sub1, double inv_n0, double inv_n1, const double* b, const double* Sc,
                          double dv, double* Q0, double* q, const int* epos, double* qs);
void launch_reproject(hipStream_t s, int n_frames, int n, const unsigned char* sub1, double* Q0);
void launch_gemm_bf16x6(hipStream_t s, int M, int N, int K, const unsigned short* A, size_t a_plane,
                        const unsigned short* B, size_t b_plane, double* D, int ldd);


// ------------------------------------------- potential profile (k_profile.hip)

constexpr int PROFILE_THREADS = 256;          // histogram workgroups
constexpr int PROFILE_SOLVE_THREADS = 1024;   // the one solving workgroup (n_bins <= 2048)
constexpr int PROFILE_MAX_BINS = 2048;
constexpr int PROFILE_MAX_HEIGHTS = 2048;
constexpr int PROFILE_MAX_PARTS = 128;

struct ProfileArgs {
  int n_frames, n_site, n_elec, n_bins, n_heights, n_part;
  int slab;                 // 1: zero field at z = 0 (slab); 0: the rise over a period is `jump`
  const double* xyz;        // [frame][3][n_site]
  const double* site_q;     // [n_site]
  const double* q;          // electrode charges, frame f at q + f * q_stride
  size_t q_stride;
  const int* height_of;     // [n_elec] index of the atom's height
  const double* heights;    // [n_heights] distinct wrapped electrode heights
  double Lz, inv_Lz, inv_h, area, eta, jump, bulk_lo, bulk_hi;
  double* part;             // scratch [n_part][n_bins + n_heights]
  double* rho_out;          // [n_bins] e / nm^3
  double* psi_out;          // [n_bins] V
};
// file-scope scratch of cpm_profile_noalloc (k_profile.hip): 4 MiB per GPU
constexpr size_t PROFILE_STATIC_DOUBLES = (size_t)PROFILE_MAX_PARTS * (PROFILE_MAX_BINS + PROFILE_MAX_HEIGHTS);
constexpr int PROFILE_MAX_DEVICES = 64;
// device address of that scratch on `device` (current in the caller), looked
// up once per device; 0 on success
int profile_static_scratch(int device, double** out);
size_t profile_partial_lds(int n_bins, int n_heights);
size_t profile_solve_lds(int n_bins, int n_heights);
void launch_profile(hipStream_t s, const ProfileArgs& p);

// ----------------------------------------------------- MD loop (k_md.hip)

constexpr int MD_MAX_GROUPS = 2;      // thermostat groups (doubled cell: one per sub-cell)
constexpr int MD_MAX_ITER = 500;      // SHAKE / RATTLE sweeps
constexpr double MD_TOL = 1e-13;      // relative constraint tolerance
constexpr int MD_THERMO = 4;          // per-step record: KE, U_LJ, E_cp (last update), thermostat energy (kJ/mol)
constexpr int MD_PART = MD_MAX_GROUPS + 1;   // per-workgroup partials: sum m v^2 per group, sum U_LJ
inline int md_workgroups(int n_mol) { return (n_mol + WAVE - 1) / WAVE; }   // integrator: a wavefront per 64 molecules

struct MDArgs {
  int n_site, n_mol, n_groups, n_lj_elec, thermostat;
  double* x; double* v;                 // [3][n_site] positions (nm), velocities (nm/ps)
  double* f_lj;                         // [3][n_site] kJ/mol/nm (written by k_lj)
  const double* f_c;                    // [3][n_site] Coulomb force, eV/nm
  double* u_lj;                         // [n_site] Lennard-Jones energy share per site (written by k_lj)
  const double* mass; const double* sigma; const double* sqeps;   // [n_site] (sqeps: sqrt(epsilon))
  const int* mol_start; const int* mol_size; const int* mol_group; const int* mol_of;
  const double* cx;                     // [3][n_lj_elec] graphene atoms, sorted by wrapped z
  double carbon_sigma, carbon_sqeps, lj_cut, bond, dt, kt;
  // partners by z window (the electrostatic binning of the same positions):
  // a site of z layer cz (of nc_z layers of the cell grid, nxy cells each)
  // meets the sites of layers cz - lj_reach .. cz + lj_reach (all of them when
  // that spans the axis) and the graphene atoms of carbon_run[4 cz ..] (two
  // index ranges [lo, hi) of the sorted atoms within lj_cut of the layer);
  // cell_start / order: the binning's per-cell starts and sorted-to-original
  // site indices
  const int* cell_start; const int* order; const int* carbon_run;
  int nc_z, nxy, lj_reach;
  double Lz;
  double box[3], inv_box[3];
  double nf[MD_MAX_GROUPS], Q[MD_MAX_GROUPS];
  double* xi; double* eta;              // [n_groups] thermostat state (device)
  double* nh_in;                        // [2][MD_MAX_GROUPS] xi, eta as the update found them
  double* md_part;                      // [md_workgroups(n_mol)][MD_PART] the integrator's partial sums
  const double* energy;                 // [2] the last charge update's {U_coul, E_cp} (eV)
  double* thermo_out;                   // [step][MD_THERMO] or nullptr
};
void launch_lj(hipStream_t s, const MDArgs& a);
void launch_md_integrate(hipStream_t s, const MDArgs& a, int mode, int rec_step);

}  // namespace cpm
