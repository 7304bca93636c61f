// C-ABI of libcpm: context set-up, host-side tables, and the orchestration
// of the per-step kernels (see include/cpm.h for the contract).
#include "../../include/cpm.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <limits>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <string>
#include <type_traits>
#include <vector>

#include "common.h"

using namespace cpm;

namespace {

thread_local std::string g_create_error;

struct GraphEntry {
  const void* p[6];
  double dv;
  int kind;
  hipGraphExec_t exec;
  unsigned long long last_use;
};

}  // namespace

struct cpm_ctx {
  // ---- descriptor
  int geometry = 0, kspace = 0, precision = 0;
  double box[3] = {0, 0, 0};
  double eta = 0, alpha = 0, rcut = 0, kcut = 0;
  double alpha_b = 0, rcut_b = 0, kcut_b = 0;
  int mesh[3] = {0, 0, 0}, order = 0;
  int n_elec = 0, n_site = 0;
  hipStream_t stream = nullptr;
  std::string err;
  bool built = false;
  bool graph_flag = false;   // CPM_FLAG_GRAPH
  bool use_graph = false;    // graph_flag and a non-null stream

  std::vector<double> hx, hy, hz;          // electrodes (host)
  std::vector<signed char> side;
  std::vector<unsigned char> sub;
  std::vector<double> hq;                  // site charges (host)
  std::vector<void*> allocs;

  Cell cell{};
  Cell cell_b{};                           // image counts for the elastance build
  double self_energy = 0.0;

  // ---- device: electrodes
  double *d_ex = nullptr, *d_ey = nullptr, *d_ez = nullptr;
  double *d_c = nullptr, *d_d = nullptr, *d_ze = nullptr, *d_e1 = nullptr;
  double *d_A = nullptr, *d_S = nullptr, *d_Sc = nullptr;
  double* d_Sc_s = nullptr;                // S c in the electrodes' cell-sorted order
  int* d_epos = nullptr;                   // cell-sorted position of every electrode atom
  double* d_qs = nullptr;                  // [frame][n_elec] charges of the force pass, cell-sorted
  // work items of the real-space b tiles: at most TILE_TGT atoms of one cell
  int n_items = 0;
  int *d_item_c = nullptr, *d_item_lo = nullptr, *d_item_hi = nullptr;
  float* d_Sf = nullptr;
  double* d_colsum = nullptr;              // [2][n_elec] column sums of d_Sf per neutrality group (mixed)
  double inv_n0 = 0.0, inv_n1 = 0.0;       // 1 / atoms per group
  unsigned short *d_Ssplit = nullptr, *d_bsplit = nullptr;   // three bf16 terms each
  unsigned char* d_sub1 = nullptr;
  int n_pad = 0;
  ElecSet<double> el{};
  ElecSet<float> elf{};
  double* d_site_q = nullptr;

  // ---- per-step buffers (capacity cap_frames)
  int cap_frames = 0;
  int *d_cell_start = nullptr, *d_order = nullptr, *d_status = nullptr;
  double* d_fpair = nullptr;      // site-site force sums [frame][3][n_site]
  double* d_wrap = nullptr;       // binning scratch: wrapped coordinates [frame][3][n_site]
  double *d_sx = nullptr, *d_sy = nullptr, *d_sz = nullptr, *d_sq = nullptr;
  double *d_zdip = nullptr, *d_b = nullptr, *d_Q0 = nullptr, *d_qint = nullptr, *d_usite = nullptr;
  double *d_ek = nullptr, *d_ftmp = nullptr, *d_fcomp = nullptr, *d_felec = nullptr, *d_energy_tmp = nullptr, *d_lam = nullptr, *d_scalar = nullptr;
  double *d_g = nullptr, *d_qa = nullptr, *d_dv = nullptr;
  int cap_dv = 0;
  int batch_chunk = 0;                     // frames per batched launch chosen by the tuner (0: not yet)
  int pair_tsplit = 1;                     // batched site-pair tiles: workgroups per cell (tuned)
  int *d_fwd_n = nullptr, *d_fwd_lo = nullptr, *d_fwd_hi = nullptr;   // forward stencils (no images only)
  // k-space field mesh of the electrode charges S c alone (batched dV sweep)
  double* d_ESc = nullptr;
  float* d_EScf = nullptr;
  bool esc_ready = false;
  double* d_phir = nullptr;
  float* d_phirf = nullptr;
  int n_ek = 0;
  // slab geometry: k_e 4 pi / V, z.(S c) and the per-frame field of the dipole correction
  double slab_kappa = 0.0, slab_zSc = 0.0;
  double* d_slabfield = nullptr;

  // ---- potential profile: distinct electrode heights and the histogram scratch
  int n_heights = 0;
  int* d_height_of = nullptr;
  double* d_heights = nullptr;
  double* d_prof = nullptr;
  size_t cap_prof = 0;
  double* d_prof_static = nullptr;         // this device's file-scope profile scratch (cpm_profile_noalloc)

  // ---- PPPM
  MeshInfo mi{};
  FFTPlan1D px{}, py{}, pz{};
  ZPassArgs za_pot{}, za_field{};
  ZMask zmask_e{};             // the electrode charge's planes (many-frame field pass)
  // The MD loop's charges stay fixed between updates, and with them the
  // electrode charge's x-y spectrum: elec_mode 1 makes the one-frame FP64
  // force pass keep that spectrum in d_c1e (the field's z pass then reads
  // it there), 2 reuses it (no electrode spread, x-y pass or charge
  // permutation); elec_owner names the MD loop whose charges d_c1e and the
  // sorted charges d_qs hold, and every other enqueue clears it
  double2* d_c1e = nullptr;
  int elec_mode = 0;
  // set by enqueue_b when it leaves out the potential's z pass (forces at
  // given charges with the kept spectrum: the field pass then transforms the
  // electrolyte and electrode spectra summed, and no b is needed)
  bool fold_pot = false;
  // the MD loop's Lennard-Jones sums to ride in its field pass (set by the
  // loop around its force enqueue), and whether they did
  const MDArgs* host_lj = nullptr;
  bool lj_hosted = false;
  const void* elec_owner = nullptr;
  bool zmask_ok = false;       // K_z <= 256: the field pass can take the mask
  int* d_zl = nullptr;         // the planes the electrode stencils reach, ascending
  int n_zl = 0;
  double *d_G = nullptr, *d_rho = nullptr, *d_phi = nullptr, *d_E = nullptr, *d_rho_e = nullptr;
  double* d_fpart = nullptr;   // [frame][6 P][n_site] per-plane field shares at the sites (FP64, or FP32 in the mixed form)
  double2 *d_c1 = nullptr, *d_c2 = nullptr, *d_save = nullptr;
  float *d_Gf = nullptr, *d_rhof = nullptr, *d_phif = nullptr, *d_Ef = nullptr, *d_rho_ef = nullptr;
  float2 *d_c1f = nullptr, *d_c2f = nullptr, *d_savef = nullptr;
  int *d_gidx = nullptr, *d_touch = nullptr, *d_rowptr = nullptr, *d_col = nullptr;
  double *d_gw = nullptr, *d_val = nullptr;
  float *d_gwf = nullptr, *d_valf = nullptr;
  int n_touch = 0, P3 = 0;

  // ---- explicit Ewald
  int nk = 0;
  double *d_kv = nullptr, *d_ew = nullptr, *d_Esite = nullptr;
  double2 *d_eph = nullptr, *d_rhok = nullptr, *d_rhok_all = nullptr;

  // ---- most recent launch of each step kernel, for timing (cpm_replay_kernel)
  std::function<void()> last_launch[CPM_KERNEL_COUNT];

  // ---- graphs
  std::vector<GraphEntry> graphs;
  unsigned long long tick = 0;
};

struct cpm_md {
  cpm_ctx* c = nullptr;
  MDArgs a{};
  int charge_every = 5;
  long long step = 0;
  bool started = false;
  double* d_q = nullptr;       // electrode charges of the last update
  double* d_fc = nullptr;      // Coulomb forces (eV/nm)
  double* d_energy = nullptr;  // {U_coul, E_cp} of the last update
  std::vector<void*> allocs;
};

namespace {

int fail(cpm_ctx* c, int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  if (c) c->err = buf; else g_create_error = buf;
  return code;
}

#define HIP_TRY(ctx, expr)                                                                  \
  do {                                                                                      \
    hipError_t e_ = (expr);                                                                 \
    if (e_ != hipSuccess) return fail(ctx, CPM_EDEVICE, "%s: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

template <typename T>
int dalloc(cpm_ctx* c, T** p, size_t n) {
  *p = nullptr;
  if (n == 0) n = 1;
  hipError_t e = hipMalloc((void**)p, n * sizeof(T));
  if (e != hipSuccess) return fail(c, CPM_ENOMEM, "hipMalloc of %zu bytes failed: %s", n * sizeof(T), hipGetErrorString(e));
  c->allocs.push_back(*p);
  return CPM_OK;
}

template <typename T>
int upload(cpm_ctx* c, T** p, const std::vector<T>& h) {
  int r = dalloc(c, p, h.size());
  if (r) return r;
  if (!h.empty()) HIP_TRY(c, hipMemcpy(*p, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice));
  return CPM_OK;
}

#define TRY(expr) do { int r_ = (expr); if (r_ != CPM_OK) return r_; } while (0)

bool factorize(int n, FFTPlan1D& p) {
  p.n = n;
  p.nfac = 0;
  int m = n;
  while (m % 4 == 0) { p.fac[p.nfac++] = 4; m /= 4; if (p.nfac >= MAX_FFT_FACTORS) return false; }
  while (m % 2 == 0) { p.fac[p.nfac++] = 2; m /= 2; if (p.nfac >= MAX_FFT_FACTORS) return false; }
  while (m % 3 == 0) { p.fac[p.nfac++] = 3; m /= 3; if (p.nfac >= MAX_FFT_FACTORS) return false; }
  while (m % 5 == 0) { p.fac[p.nfac++] = 5; m /= 5; if (p.nfac >= MAX_FFT_FACTORS) return false; }
  return m == 1;
}

// cardinal B-spline M_P(x) on [0, P] (Cox-de Boor recursion)
double bspline_host(int P, double x) {
  if (P == 1) return (x >= 0.0 && x < 1.0) ? 1.0 : 0.0;
  return (x * bspline_host(P - 1, x) + (P - x) * bspline_host(P - 1, x - 1.0)) / (P - 1);
}

int cell_coord_host(double x, double L, int n) {
  double t = x / L;
  double f = t - std::floor(t);
  int c = (int)std::floor(f * (double)n);
  return c < n - 1 ? c : n - 1;
}

double wrap_host(double x, double L) { return x - L * std::floor(x / L); }

// Stencil groups of every cell of the grid: the distinct neighbour cells
// (offsets -r .. r along an axis of reach r: 1, or 2 along a z axis cut into
// cells half the cutoff thick; fewer where the axis has under 2r + 1 cells),
// sorted and joined into runs of consecutive cell indices [lo, hi); n[c]
// groups per cell at [c * STENCIL_MAX + k] (unused entries 0).  forward:
// only the cells of index >= c (the stencil is symmetric, so every pair of
// neighbouring cells appears once, in the lower cell's list).  Returns the
// largest group count.
int stencil_groups(const Cell& cl, const int* reach, std::vector<int>& n, std::vector<int>& lo, std::vector<int>& hi,
                   bool forward = false) {
  n.assign(cl.n_cells, 0);
  lo.assign((size_t)cl.n_cells * STENCIL_MAX, 0);
  hi.assign((size_t)cl.n_cells * STENCIL_MAX, 0);
  int most = 0;
  for (int c = 0; c < cl.n_cells; ++c) {
    const int cc[3] = {c % cl.nc[0], (c / cl.nc[0]) % cl.nc[1], c / (cl.nc[0] * cl.nc[1])};
    std::vector<int> nbr[3];
    for (int a = 0; a < 3; ++a) {
      const int m = cl.nc[a], r = reach[a];
      if (m >= 2 * r + 1)
        for (int s = -r; s <= r; ++s) nbr[a].push_back(((cc[a] + s) % m + m) % m);
      else
        for (int s = 0; s < m; ++s) nbr[a].push_back(s);
    }
    std::vector<int> cells;
    for (int z : nbr[2])
      for (int y : nbr[1])
        for (int x : nbr[0]) cells.push_back((z * cl.nc[1] + y) * cl.nc[0] + x);
    std::sort(cells.begin(), cells.end());
    cells.erase(std::unique(cells.begin(), cells.end()), cells.end());
    if (forward) cells.erase(std::remove_if(cells.begin(), cells.end(), [c](int v) { return v < c; }), cells.end());
    int k = -1;
    for (size_t t = 0; t < cells.size(); ++t) {
      if (t == 0 || cells[t] != cells[t - 1] + 1) {
        if (++k >= STENCIL_MAX) return STENCIL_MAX + 1;
        lo[(size_t)c * STENCIL_MAX + k] = cells[t];
      }
      hi[(size_t)c * STENCIL_MAX + k] = cells[t] + 1;
    }
    n[c] = k + 1;
    most = std::max(most, k + 1);
  }
  return most;
}

// half-space k-vectors with 0 < |k| <= kcut: (n1 > 0) or (n1 == 0, n2 > 0) or (n1 == n2 == 0, n3 > 0)
void half_kvectors(const double* box, double kcut, std::vector<double>& kx, std::vector<double>& ky,
                   std::vector<double>& kz) {
  int nmax[3];
  for (int d = 0; d < 3; ++d) nmax[d] = (int)std::floor(kcut * box[d] / (2 * M_PI));
  for (int a = 0; a <= nmax[0]; ++a)
    for (int b = -nmax[1]; b <= nmax[1]; ++b)
      for (int c = -nmax[2]; c <= nmax[2]; ++c) {
        if (a == 0 && (b < 0 || (b == 0 && c <= 0))) continue;
        double k0 = 2 * M_PI * a / box[0], k1 = 2 * M_PI * b / box[1], k2 = 2 * M_PI * c / box[2];
        double kk = k0 * k0 + k1 * k1 + k2 * k2;
        if (kk > kcut * kcut) continue;
        kx.push_back(k0); ky.push_back(k1); kz.push_back(k2);
      }
}

double kweight_host(double k2, double alpha, double vol) {
  return 4 * M_PI / vol * std::exp(-k2 / (4 * alpha * alpha)) / k2;
}

// Hockney-Eastwood optimal influence function for ik differentiation, times
// k_e / V so that the unnormalised inverse transform gives volts.  Layout
// [kz][ky][kx].  Aliases per axis: every m with |n + m K| <= 2.5 K.
void influence_host(const double* box, const int* K, int P, double alpha, std::vector<double>& G) {
  const double vol = box[0] * box[1] * box[2];
  const int M = K[0] * K[1] * K[2];
  G.assign(M, 0.0);
  // per axis and index: alias wavevectors and U^2 factors
  std::vector<std::vector<double>> ka[3], u2[3];
  std::vector<double> kb[3];
  for (int d = 0; d < 3; ++d) {
    double h = box[d] / K[d];
    ka[d].resize(K[d]);
    u2[d].resize(K[d]);
    kb[d].resize(K[d]);
    for (int i = 0; i < K[d]; ++i) {
      int n = (i < (K[d] + 1) / 2) ? i : i - K[d];
      kb[d][i] = 2 * M_PI * n / box[d];
      for (int m = -3; m <= 3; ++m) {
        int nm = n + m * K[d];
        if (std::abs((double)nm) > 2.5 * K[d]) continue;
        double k = 2 * M_PI * nm / box[d];
        double x = k * h / 2;
        double sinc = (x == 0.0) ? 1.0 : std::sin(x) / x;
        ka[d][i].push_back(k);
        u2[d][i].push_back(std::pow(sinc, 2 * P));
      }
    }
  }
  for (int iz = 0; iz < K[2]; ++iz)
    for (int iy = 0; iy < K[1]; ++iy)
      for (int ix = 0; ix < K[0]; ++ix) {
        double k0 = kb[0][ix], k1 = kb[1][iy], k2 = kb[2][iz];
        double kk = k0 * k0 + k1 * k1 + k2 * k2;
        if (kk == 0.0) continue;
        double num = 0.0, den = 0.0;
        for (size_t a = 0; a < ka[0][ix].size(); ++a)
          for (size_t b = 0; b < ka[1][iy].size(); ++b)
            for (size_t c = 0; c < ka[2][iz].size(); ++c) {
              double qx = ka[0][ix][a], qy = ka[1][iy][b], qz = ka[2][iz][c];
              double U2 = u2[0][ix][a] * u2[1][iy][b] * u2[2][iz][c];
              double q2 = qx * qx + qy * qy + qz * qz;
              den += U2;
              if (q2 == 0.0) continue;
              double R = 4 * M_PI * std::exp(-q2 / (4 * alpha * alpha)) / q2;
              num += U2 * (k0 * qx + k1 * qy + k2 * qz) * R;
            }
        G[((size_t)iz * K[1] + iy) * K[0] + ix] = KE / vol * num / (kk * den * den);
      }
}

void free_graphs(cpm_ctx* c) {
  for (auto& g : c->graphs) (void)hipGraphExecDestroy(g.exec);
  c->graphs.clear();
}

// slab geometry's dipole-correction terms (kappa == 0: none)
SlabTerms slab_terms(const cpm_ctx* c) {
  SlabTerms sl{};
  if (c->geometry == CPM_SLAB) {
    sl.kappa = c->slab_kappa;
    sl.ze = c->d_ze;
    sl.zdip = c->d_zdip;
    sl.n_elec = c->n_elec;
  }
  return sl;
}

// --------------------------------------------------------------- buffers

int alloc_frames(cpm_ctx* c, int nf) {
  if (nf <= c->cap_frames) return CPM_OK;
  // release the previous per-frame buffers by reallocating fresh ones; old
  // pointers stay in allocs and are freed at destroy (graphs referring to them
  // are dropped)
  free_graphs(c);
  const int ns = c->n_site, ne = c->n_elec, ncl = c->cell.n_cells;
  const bool mixed = c->precision == CPM_MIXED;
  TRY(dalloc(c, &c->d_cell_start, (size_t)nf * (ncl + 1)));
  TRY(dalloc(c, &c->d_order, (size_t)nf * ns));
  TRY(dalloc(c, &c->d_sx, (size_t)nf * ns));
  TRY(dalloc(c, &c->d_sy, (size_t)nf * ns));
  TRY(dalloc(c, &c->d_sz, (size_t)nf * ns));
  TRY(dalloc(c, &c->d_sq, (size_t)nf * ns));
  if (mixed) {
    TRY(dalloc(c, &c->d_phirf, (size_t)nf * ne));
  }
  TRY(dalloc(c, &c->d_phir, (size_t)nf * ne));
  TRY(dalloc(c, &c->d_zdip, (size_t)nf));
  TRY(dalloc(c, &c->d_fpair, (size_t)nf * 3 * ns));
  TRY(dalloc(c, &c->d_wrap, (size_t)nf * 3 * ns));
  TRY(dalloc(c, &c->d_b, (size_t)nf * ne));
  TRY(dalloc(c, &c->d_Q0, (size_t)nf * ne));
  TRY(dalloc(c, &c->d_qint, (size_t)nf * ne));
  TRY(dalloc(c, &c->d_lam, (size_t)nf * ne));
  TRY(dalloc(c, &c->d_g, (size_t)nf * ne));
  TRY(dalloc(c, &c->d_qa, (size_t)nf * ne));
  TRY(dalloc(c, &c->d_qs, (size_t)nf * ne));
  if (mixed) TRY(dalloc(c, &c->d_bsplit, (size_t)3 * nf * c->n_pad));
  TRY(dalloc(c, &c->d_usite, (size_t)nf * ns));
  TRY(dalloc(c, &c->d_ftmp, (size_t)nf * 3 * ns));
  TRY(dalloc(c, &c->d_fcomp, (size_t)nf * 6 * ns));
  TRY(dalloc(c, &c->d_felec, (size_t)nf * 6 * ns));
  TRY(dalloc(c, &c->d_energy_tmp, (size_t)nf * 2));
  TRY(dalloc(c, &c->d_slabfield, (size_t)nf));
  if (c->kspace == CPM_KSPACE_PPPM) {
    const size_t M = c->mi.M;
    c->n_ek = c->za_pot.n_blocks;
    TRY(dalloc(c, &c->d_ek, (size_t)nf * c->n_ek));
    if (nf > 1) TRY(dalloc(c, &c->d_fpart, (size_t)nf * ns * 6 * c->mi.order));
    // the real charge mesh is stored by one-frame solves only, and the
    // field mesh by many-frame ones only at orders other than 5 (at 5 the
    // inverse pass interpolates at the sites)
    const size_t nf_E = c->mi.order == 5 ? 1 : nf;
    if (!mixed) {
      TRY(dalloc(c, &c->d_rho, M));
      TRY(dalloc(c, &c->d_phi, nf * M));
      TRY(dalloc(c, &c->d_E, nf_E * 3 * M));
      TRY(dalloc(c, &c->d_rho_e, nf * M));
      TRY(dalloc(c, &c->d_c1, nf * M));
      TRY(dalloc(c, &c->d_c2, nf * M));
      TRY(dalloc(c, &c->d_save, nf * M));
      HIP_TRY(c, hipMemset(c->d_rho_e, 0, nf * M * sizeof(double)));
    } else {
      TRY(dalloc(c, &c->d_rhof, M));
      TRY(dalloc(c, &c->d_phif, nf * M));
      TRY(dalloc(c, &c->d_Ef, nf_E * 3 * M));
      TRY(dalloc(c, &c->d_rho_ef, nf * M));
      TRY(dalloc(c, &c->d_c1f, nf * M));
      TRY(dalloc(c, &c->d_c2f, nf * M));
      TRY(dalloc(c, &c->d_savef, nf * M));
      HIP_TRY(c, hipMemset(c->d_rho_ef, 0, nf * M * sizeof(float)));
    }
  } else {
    c->n_ek = c->nk;
    TRY(dalloc(c, &c->d_ek, (size_t)nf * c->nk));
    TRY(dalloc(c, &c->d_rhok, (size_t)nf * c->nk));
    TRY(dalloc(c, &c->d_rhok_all, (size_t)nf * c->nk));
    TRY(dalloc(c, &c->d_Esite, (size_t)nf * 3 * ns));
  }
  HIP_TRY(c, hipDeviceSynchronize());
  c->cap_frames = nf;
  return CPM_OK;
}

// ------------------------------------------------------------ the step

// launch on stream s now and remember the launch (arguments by value) for
// cpm_replay_kernel, which re-runs it on the context's stream
template <typename F>
void rec(cpm_ctx* c, int id, hipStream_t s, F f) {
  c->last_launch[id] = [c, f]() { f(c->stream); };
  f(s);
}

// remember a launch for cpm_replay_kernel without running it now (a part of
// a launch that hosts several kernels' workgroups, timed on its own)
template <typename F>
void keep(cpm_ctx* c, int id, F f) {
  c->last_launch[id] = [c, f]() { f(c->stream); };
}

template <typename T> struct Bufs;
template <> struct Bufs<double> {
  using T2 = double2;
  static SiteSet<double> sites(cpm_ctx* c) {
    return SiteSet<double>{c->d_sx, c->d_sy, c->d_sz, c->d_sq, c->d_order, c->d_cell_start, c->n_site};
  }
  static const ElecSet<double>& elec(cpm_ctx* c) { return c->el; }
  static double* phir(cpm_ctx* c) { return c->d_phir; }
  static double* rho(cpm_ctx* c) { return c->d_rho; }
  static double* phi(cpm_ctx* c) { return c->d_phi; }
  static double* E(cpm_ctx* c) { return c->d_E; }
  static double* rho_e(cpm_ctx* c) { return c->d_rho_e; }
  static double2* c1(cpm_ctx* c) { return c->d_c1; }
  static double2* c2(cpm_ctx* c) { return c->d_c2; }
  static double2* save(cpm_ctx* c) { return c->d_save; }
  static const double* G(cpm_ctx* c) { return c->d_G; }
  static const double* gw(cpm_ctx* c) { return c->d_gw; }
  static const double* val(cpm_ctx* c) { return c->d_val; }
};
template <> struct Bufs<float> {
  using T2 = float2;
  static SiteSet<float> sites(cpm_ctx* c) {
    return SiteSet<float>{c->d_sx, c->d_sy, c->d_sz, c->d_sq, c->d_order, c->d_cell_start, c->n_site};
  }
  static const ElecSet<float>& elec(cpm_ctx* c) { return c->elf; }
  static float* phir(cpm_ctx* c) { return c->d_phirf; }
  static float* rho(cpm_ctx* c) { return c->d_rhof; }
  static float* phi(cpm_ctx* c) { return c->d_phif; }
  static float* E(cpm_ctx* c) { return c->d_Ef; }
  static float* rho_e(cpm_ctx* c) { return c->d_rho_ef; }
  static float2* c1(cpm_ctx* c) { return c->d_c1f; }
  static float2* c2(cpm_ctx* c) { return c->d_c2f; }
  static float2* save(cpm_ctx* c) { return c->d_savef; }
  static const float* G(cpm_ctx* c) { return c->d_Gf; }
  static const float* gw(cpm_ctx* c) { return c->d_gwf; }
  static const float* val(cpm_ctx* c) { return c->d_valf; }
};

// Stage 1: positions -> binned sites -> b (frames 0..nf-1).  With PPPM the
// binning runs as one more workgroup per frame of the first mesh launch (the
// spread scans the raw positions and needs no cell list), and the real-space
// part of b as extra workgroups of the z pass that follows.
template <typename T>
int enqueue_b(cpm_ctx* c, int nf, const double* xyz, bool forces, bool need_b = true) {
  using B = Bufs<T>;
  using T2 = typename B::T2;
  hipStream_t s = c->stream;
  c->elec_owner = nullptr;
  const bool mixed = std::is_same<T, float>::value;
  BinArgs ba{};
  ba.n_site = c->n_site;
  ba.xyz_all = xyz;
  ba.frame_stride = (size_t)3 * c->n_site;
  ba.site_q = c->d_site_q;
  ba.cell = c->cell;
  ba.cell_start_all = c->d_cell_start;
  ba.order_all = c->d_order;
  ba.sx_all = c->d_sx; ba.sy_all = c->d_sy; ba.sz_all = c->d_sz; ba.sq_all = c->d_sq;
  ba.zdip_all = c->d_zdip;
  ba.status = c->d_status;
  ba.wrap_all = c->d_wrap;
  SiteSet<T> st = B::sites(c);
  // real-space b: one frame, a wavefront per electrode atom (hosted in the
  // potential's z pass); many frames, cell tiles in a launch of their own
  RealBArgs<T> rb{};
  rb.tiles = nf > 1;
  rb.n_blocks = rb.tiles ? c->n_items : (c->n_elec + 3) / 4;
  rb.cell = c->cell;
  rb.st = st;
  rb.alpha = (T)c->alpha;
  rb.eta = (T)c->eta;
  rb.rc2 = c->rcut * c->rcut;
  rb.el = B::elec(c);
  rb.phi_out = B::phir(c);
  rb.item_c = c->d_item_c;
  rb.item_lo = c->d_item_lo;
  rb.item_hi = c->d_item_hi;
  if (c->kspace == CPM_KSPACE_PPPM) {
    // (the real charge mesh is kept for inspection after one frame only)
    rec(c, CPM_KERNEL_FFT_XY_FWD, s, [=](hipStream_t s) {
      launch_fft_xy_spread_t<T, T2>(s, nf, c->px, c->py, c->mi.K[2], c->mi, ba, nf == 1 ? B::rho(c) : nullptr,
                                    B::c1(c), true, true);
    });
    keep(c, CPM_KERNEL_BIN, [=](hipStream_t s) {
      launch_fft_xy_spread_t<T, T2>(s, nf, c->px, c->py, c->mi.K[2], c->mi, ba, B::rho(c), B::c1(c), false, true);
    });
    if (rb.tiles) rec(c, CPM_KERNEL_REAL_B, s, [=](hipStream_t s) { launch_real_b_t<T>(s, nf, rb); });
    // forces at given charges in the MD loop (its electrode spectrum kept):
    // no potential pass, the field pass folds the two spectra
    c->fold_pot = !need_b && nf == 1 && c->elec_mode != 0 && c->d_c1e && std::is_same<T, double>::value;
    if (!c->fold_pot) {
      rec(c, CPM_KERNEL_FFT_Z_POT, s, [=](hipStream_t s) {
        // (many frames: the result only on the planes the electrode stencils read)
        launch_fft_z_t<T, T2>(s, nf, c->pz, c->za_pot, B::G(c), B::c1(c), nullptr,
                              forces ? B::save(c) : nullptr, 0, c->d_ek, true,
                              (rb.tiles || !need_b) ? nullptr : &rb, nullptr,
                              nf > 1 && c->zmask_ok ? &c->zmask_e : nullptr);
      });
    }
    // forces at given charges (MD steps between charge updates): only the
    // saved site spectrum is needed, not b
    if (!need_b) return CPM_OK;
    // timed alone through the stand-alone kernel with the same body
    if (!rb.tiles) keep(c, CPM_KERNEL_REAL_B, [=](hipStream_t s) { launch_real_b_t<T>(s, nf, rb); });
    // (many frames: only the planes the electrode stencils read)
    rec(c, CPM_KERNEL_FFT_XY_INV, s, [=](hipStream_t s) {
      launch_fft_xy_t<T, T2>(s, nf, c->px, c->py, c->mi.K[2], 1, nullptr, B::c1(c), nullptr, B::phi(c), nullptr, 0,
                             c->d_zl, c->n_zl);
    });
    rec(c, CPM_KERNEL_GATHER_B, s, [=](hipStream_t s) {
      launch_gather_b_t<T>(s, nf, c->n_elec, c->P3, c->d_gidx, B::gw(c), B::phi(c), c->mi.M, B::phir(c), c->d_b,
                           slab_terms(c));
    });
  } else {
    rec(c, CPM_KERNEL_BIN, s, [=](hipStream_t s) { launch_bin_sites(s, nf, ba); });
    SiteSet<double> sd = Bufs<double>::sites(c);
    if (!need_b) {
      launch_ewald_sf(s, nf, c->nk, c->d_kv, c->d_ew, sd, c->d_rhok, c->d_ek);
      return CPM_OK;
    }
    rec(c, CPM_KERNEL_REAL_B, s, [=](hipStream_t s) { launch_real_b_t<T>(s, nf, rb); });
    launch_ewald_sf(s, nf, c->nk, c->d_kv, c->d_ew, sd, c->d_rhok, c->d_ek);
    launch_ewald_phi(s, nf, c->nk, c->n_elec, c->d_ew, c->d_eph, c->d_rhok, c->d_phir, c->d_b, slab_terms(c));
  }
  return CPM_OK;
}

// Stage 3: Coulomb forces on the sites for electrode charges qa (+ optional
// second set qb on a shared field mesh Eb; qa_s: qa in the electrodes'
// cell-sorted order, same frame stride) and, if ea is given, the energies.  The site-site forces (independent of the charges) run as extra
// workgroups of the z pass of the field, the energies as extra workgroups
// of the site-force launch.
template <typename T>
int enqueue_forces(cpm_ctx* c, int nf, const double* qa, size_t qa_stride, const double* qa_s, ForceArgs<T> fa,
                   const EnergyArgs* ea) {
  using B = Bufs<T>;
  using T2 = typename B::T2;
  hipStream_t s = c->stream;
  SiteSet<T> st = B::sites(c);
  fa.alpha = (T)c->alpha;
  fa.eta = (T)c->eta;
  fa.rc2 = c->rcut * c->rcut;
  fa.qa = qa;
  fa.qa_frame_stride = qa_stride;
  fa.qa_s = qa_s;
  fa.qb_s = fa.qb ? c->d_Sc_s : nullptr;     // the only second set is S c
  fa.mi = c->mi;
  fa.f_pair = c->d_fpair;
  // slab: the uniform field of the dipole correction for the charges qa,
  // made by one more workgroup per frame of the electrode spread (PPPM) or
  // by a launch of its own (explicit Ewald)
  const SlabTerms sl = slab_terms(c);
  fa.field_frame = c->geometry == CPM_SLAB ? c->d_slabfield : nullptr;
  PairArgs<T> pa{};
  // one frame: a wavefront per site (short chains, all in flight at once);
  // many frames: cell tiles
  pa.tsplit = nf == 1 ? 0 : c->pair_tsplit;
  pa.n_blocks = c->n_site == 0 ? 0 : pa.tsplit > 0 ? c->cell.n_cells * pa.tsplit : (c->n_site + 3) / 4;
  pa.cell = c->cell;
  pa.st = st;
  pa.alpha = fa.alpha;
  pa.rc2 = fa.rc2;
  pa.f_pair = c->d_fpair;
  pa.u_site = c->d_usite;
  if (pa.tsplit > 0) {
    // tiles run after the charge solve: they take the site-electrode pairs
    // too, and the site-force kernel then skips its own electrode walk
    pa.el = B::elec(c);
    pa.eta = fa.eta;
    pa.qa_s = qa_s;
    pa.qa_stride = qa_stride;
    pa.qb_s = fa.qb_s;
    pa.f_elec = c->d_felec;
    fa.f_elec = c->d_felec;
    pa.fwd_n = c->d_fwd_n; pa.fwd_lo = c->d_fwd_lo; pa.fwd_hi = c->d_fwd_hi;
    // |z_target - z_centre| <= w/2, so a pair within rcut has the staged
    // image's |dz| < rcut + w/2 < Lz/2 when Lz > 2 rcut + w: the same image
    // as the minimum image of the pair
    const Cell& cl = c->cell;
    pa.zshift = (cl.img[0] | cl.img[1] | cl.img[2]) == 0 && cl.nc[2] >= 5 &&
                cl.L[2] > 2.0 * c->rcut + cl.L[2] / cl.nc[2];
  }
  const T* epart = nullptr;   // the interpolation's per-plane shares (many frames, order 5)
  if (c->kspace == CPM_KSPACE_PPPM) {
    // (the MD loop's kept electrode spectrum: FP64 one-frame passes only)
    const int em = (nf == 1 && std::is_same<T, double>::value && c->d_c1e) ? c->elec_mode : 0;
    T2* espec = em ? reinterpret_cast<T2*>(c->d_c1e) : B::c1(c);
    if (em != 2) {
      // the electrode spread stays a kernel of its own: only the few planes
      // near the electrodes hold charge, and a per-plane fusion would leave
      // that work to a handful of workgroups
      rec(c, CPM_KERNEL_SPREAD_ELEC, s, [=](hipStream_t s) {
        launch_spread_elec_t<T>(s, nf, c->n_touch, c->d_touch, c->d_rowptr, c->d_col, B::val(c), qa, qa_stride,
                                B::rho_e(c), c->mi.M, sl, fa.field_frame ? c->d_slabfield : nullptr, c->n_elec);
      });
    } else if (fa.field_frame) {
      launch_slab_field(s, nf, sl, qa, qa_stride, c->d_slabfield);
    }
    // many frames: only the planes holding electrode charge, which the
    // field pass then reads alone (the others are zero)
    const bool planes = nf > 1 && c->zmask_ok;
    if (em != 2)
      rec(c, CPM_KERNEL_FFT_XY_FWD_E, s, [=](hipStream_t s) {
        launch_fft_xy_t<T, T2>(s, nf, c->px, c->py, c->mi.K[2], 0, B::rho_e(c), nullptr, espec, nullptr, nullptr, 0,
                               planes ? c->d_zl : nullptr, planes ? c->n_zl : 0);
      });
    // one frame: the site-pair workgroups ride in the z pass (latency);
    // many frames: a launch of their own, so that the z pass keeps its small
    // LDS footprint and occupancy (throughput)
    const bool host_pairs = nf == 1;
    const bool fold = em != 0 && c->fold_pot;
    const bool with_lj = em != 0 && c->host_lj;
    const MDArgs ljv = with_lj ? *c->host_lj : MDArgs{};
    c->lj_hosted = with_lj;
    rec(c, CPM_KERNEL_FFT_Z_FIELD, s, [=](hipStream_t s) {
      launch_fft_z_t<T, T2>(s, nf, c->pz, c->za_field, B::G(c), B::c1(c), B::c2(c), fold ? nullptr : B::save(c),
                            fold ? 2 : 1, nullptr, true, nullptr, host_pairs ? &pa : nullptr,
                            planes ? &c->zmask_e : nullptr, espec, with_lj ? &ljv : nullptr);
    });
    if (host_pairs)   // timed alone through the stand-alone kernel with the same body
      keep(c, CPM_KERNEL_SITE_PAIRS, [=](hipStream_t s) { launch_site_pairs_t<T>(s, nf, pa); });
    else
      rec(c, CPM_KERNEL_SITE_PAIRS, s, [=](hipStream_t s) { launch_site_pairs_t<T>(s, nf, pa); });
    // c1 -> Ex (re), Ey (im); c2 -> Ez; field meshes are [frame][3][M]
    T* E = B::E(c);
    const size_t M = c->mi.M;
    fa.Ea = E;
    fa.Ea_frame_stride = 3 * M;
    fa.Esite = nullptr;
    if (nf > 1 && fa.f_elec && c->mi.order == 5) {
      // many frames, with the site-electrode sums in the tiles (order 5):
      // the inverse pass interpolates the field at the sites plane by plane
      // (no field mesh is written), and the site-force kernel sums those
      // shares
      InterpArgs<T> ia{};
      const Cell& cl = c->cell;
      ia.sx = c->d_sx; ia.sy = c->d_sy; ia.sz = c->d_sz;
      ia.cell_start = c->d_cell_start;
      ia.n = c->n_site; ia.n_cells = cl.n_cells; ia.nxy = cl.nc[0] * cl.nc[1]; ia.ncz = cl.nc[2];
      ia.inv_wz = cl.nc[2] / cl.L[2];
      ia.Eb = fa.Eb;
      ia.part = reinterpret_cast<T*>(c->d_fpart);
      ia.mi = c->mi;
      epart = ia.part;
      rec(c, CPM_KERNEL_FFT_XY_INV_E, s, [=](hipStream_t s) {
        launch_fft_xy_field_inv_t<T, T2>(s, nf, c->px, c->py, c->mi.K[2], B::c1(c), B::c2(c), nullptr, 3 * M, &ia);
      });
    } else {
      rec(c, CPM_KERNEL_FFT_XY_INV_E, s, [=](hipStream_t s) {
        launch_fft_xy_field_inv_t<T, T2>(s, nf, c->px, c->py, c->mi.K[2], B::c1(c), B::c2(c), E, 3 * M);
      });
    }
  } else {
    rec(c, CPM_KERNEL_SITE_PAIRS, s, [=](hipStream_t s) { launch_site_pairs_t<T>(s, nf, pa); });
    if (fa.field_frame) launch_slab_field(s, nf, sl, qa, qa_stride, c->d_slabfield);
    SiteSet<double> sd = Bufs<double>::sites(c);
    launch_ewald_rho_all(s, nf, c->nk, c->n_elec, c->d_eph, qa, qa_stride, c->d_rhok, c->d_rhok_all);
    launch_ewald_field(s, nf, c->nk, c->d_kv, c->d_ew, sd, c->d_rhok_all, c->d_Esite);
    fa.Ea = nullptr;
    fa.Esite = c->d_Esite;
  }
  const bool with_e = ea != nullptr;
  const EnergyArgs e = with_e ? *ea : EnergyArgs{};
  rec(c, CPM_KERNEL_SITE_FORCES, s, [=](hipStream_t s) {
    launch_site_forces_t<T>(s, nf, c->cell, B::elec(c), st, fa, true, with_e ? &e : nullptr, epart);
  });
  if (with_e)
    keep(c, CPM_KERNEL_ENERGY, [=](hipStream_t s) {
      launch_site_forces_t<T>(s, nf, c->cell, B::elec(c), st, fa, false, &e, epart);
    });
  return CPM_OK;
}

// energy reduction of the step: dV sweep of n_dv values (dv) or one (dv_single)
EnergyArgs energy_args(cpm_ctx* c, int n_dv, const double* dv, double dv_single, double* out) {
  EnergyArgs ea{};
  ea.n_elec = c->n_elec; ea.n_site = c->n_site; ea.n_ek = c->n_ek;
  ea.Q0 = c->d_Q0; ea.b = c->d_b; ea.Sc = c->d_Sc; ea.c = c->d_c; ea.d = c->d_d; ea.ze = c->d_ze;
  ea.u_site = c->d_usite; ea.ek = c->d_ek; ea.zdip = c->d_zdip; ea.self_energy = c->self_energy;
  ea.ff = c->geometry == CPM_FINITE_FIELD; ea.Lz = c->box[2];
  ea.slab_kappa = c->geometry == CPM_SLAB ? c->slab_kappa : 0.0;
  ea.n_dv = n_dv; ea.dv = dv; ea.dv_single = dv_single; ea.out = out;
  return ea;
}

template <typename T>
int enqueue_solve(cpm_ctx* c, const double* xyz, double dv, double* q_out, double* f_out, double* e_out) {
  hipStream_t s = c->stream;
  const bool need_forces = f_out || e_out;
  TRY(enqueue_b<T>(c, 1, xyz, need_forces));
  if (std::is_same<T, float>::value) {
    // FP32-stored S, FP64 products, neutrality by the precomputed column
    // sums: one launch, half the bytes of the FP64 GEMV
    rec(c, CPM_KERNEL_CHARGES, s, [=](hipStream_t s) {
      launch_charges_mixed(s, 1, c->n_elec, c->d_Sf, c->d_colsum, c->d_sub1, c->inv_n0, c->inv_n1, c->d_b, c->d_Sc,
                           dv, c->d_Q0, q_out, c->d_epos, c->d_qs);
    });
  } else {
    rec(c, CPM_KERNEL_CHARGES, s, [=](hipStream_t s) {
      launch_charges(s, 1, c->n_elec, c->d_S, c->d_b, c->d_Sc, dv, c->d_Q0, q_out, c->d_epos, c->d_qs);
    });
  }
  if (need_forces) {
    ForceArgs<T> fa{};
    fa.out_scale = 1.0;
    fa.field = (c->geometry == CPM_FINITE_FIELD) ? -dv / c->box[2] : 0.0;
    fa.f_out = f_out ? f_out : c->d_ftmp;
    fa.f_frame_stride = 3 * (size_t)c->n_site;
    fa.n_dv = 1;
    fa.dv = nullptr;
    fa.u_site = c->d_usite;
    const EnergyArgs ea = energy_args(c, 1, nullptr, dv, e_out);
    TRY(enqueue_forces<T>(c, 1, q_out, c->n_elec, c->d_qs, fa, e_out ? &ea : nullptr));
  }
  return CPM_OK;
}

// Coulomb forces on the sites at given electrode charges q (device, original
// order), without b or a charge solve: the MD steps between charge updates
template <typename T>
int enqueue_forces_at(cpm_ctx* c, const double* xyz, double dv, const double* q, double* f_out) {
  hipStream_t s = c->stream;
  TRY(enqueue_b<T>(c, 1, xyz, true, false));
  if (c->elec_mode != 2) launch_permute(s, 1, c->n_elec, c->d_epos, q, c->d_qs);
  ForceArgs<T> fa{};
  fa.out_scale = 1.0;
  fa.field = (c->geometry == CPM_FINITE_FIELD) ? -dv / c->box[2] : 0.0;
  fa.f_out = f_out;
  fa.f_frame_stride = 3 * (size_t)c->n_site;
  fa.n_dv = 1;
  fa.dv = nullptr;
  fa.u_site = c->d_usite;
  return enqueue_forces<T>(c, 1, q, c->n_elec, c->d_qs, fa, nullptr);
}

// Adjoint of L = sum (q - t)^2 + U_coul through q* = S v(R)
template <typename T>
int enqueue_grad(cpm_ctx* c, const double* xyz, double dv, const double* t, double* loss, double* dldx,
                 double* dldv, double* q_out) {
  hipStream_t s = c->stream;
  const int n = c->n_elec;
  double* q = q_out ? q_out : c->d_qint;
  TRY(enqueue_b<T>(c, 1, xyz, true));
  launch_charges(s, 1, n, c->d_S, c->d_b, c->d_Sc, dv, c->d_Q0, q);
  launch_adjoint_rhs(s, n, q, t, c->d_c, dv, c->d_g);
  launch_charges(s, 1, n, c->d_S, c->d_g, c->d_Sc, 0.0, c->d_lam, nullptr);    // lambda = S g
  launch_sub(s, n, q, c->d_lam, c->d_qa, c->d_epos, c->d_qs);
  ForceArgs<T> fa{};
  fa.out_scale = -1.0;
  fa.field = 0.0;
  fa.f_out = dldx;
  fa.f_frame_stride = 3 * (size_t)c->n_site;
  fa.n_dv = 1;
  fa.u_site = c->d_usite;
  const EnergyArgs ea = energy_args(c, 1, nullptr, dv, c->d_energy_tmp);
  TRY(enqueue_forces<T>(c, 1, c->d_qa, n, c->d_qs, fa, &ea));
  launch_grad_finish(s, n, q, t, c->d_lam, c->d_c, c->d_energy_tmp, loss, dldv);
  return CPM_OK;
}

// The field mesh of the electrode charges S c alone: frame-independent, made once.
template <typename T>
void enqueue_esc_mesh(cpm_ctx* c, T* out) {
  using B = Bufs<T>;
  using T2 = typename B::T2;
  hipStream_t s = c->stream;
  const size_t M = c->mi.M;
  launch_spread_elec_t<T>(s, 1, c->n_touch, c->d_touch, c->d_rowptr, c->d_col, B::val(c), c->d_Sc, c->n_elec,
                          B::rho_e(c), c->mi.M);
  launch_fft_xy_t<T, T2>(s, 1, c->px, c->py, c->mi.K[2], 0, B::rho_e(c), nullptr, B::c1(c), nullptr, nullptr);
  launch_fft_z_t<T, T2>(s, 1, c->pz, c->za_field, B::G(c), B::c1(c), B::c2(c), nullptr, 0, nullptr);
  launch_fft_xy_field_inv_t<T, T2>(s, 1, c->px, c->py, c->mi.K[2], B::c1(c), B::c2(c), out, 3 * M);
}

// Frames [0, nf) of a batch: b for every frame, Q0 = S B in one GEMM, the
// forces F_A(Q0) + dV (F_B(S c) + field) and energies for every dV, and the
// charges Q0 + dV S c.
template <typename T>
int enqueue_batch(cpm_ctx* c, int nf, const double* xyz, int n_dv, double* q_out, double* f_out, double* e_out) {
  hipStream_t s = c->stream;
  const int n = c->n_elec;
  const bool need_forces = f_out || e_out;
  TRY(enqueue_b<T>(c, nf, xyz, need_forces));
  // Q0[f][i] = sum_j B[f][j] S[i][j]
  if (std::is_same<T, float>::value) {
    launch_split_b(s, nf, n, c->n_pad, c->d_b, c->d_bsplit);
    rec(c, CPM_KERNEL_GEMM, s, [=](hipStream_t s) {
      launch_gemm_bf16x6(s, nf, n, c->n_pad, c->d_bsplit, (size_t)nf * c->n_pad, c->d_Ssplit, (size_t)n * c->n_pad,
                         c->d_Q0, n);
    });
    launch_reproject(s, nf, n, c->d_sub1, c->d_Q0);
  } else {
    rec(c, CPM_KERNEL_GEMM, s, [=](hipStream_t s) {
      launch_gemm_nt(s, nf, n, n, 1.0, c->d_b, n, c->d_S, n, 0.0, c->d_Q0, n);
    });
  }
  rec(c, CPM_KERNEL_EXPAND_Q, s, [=](hipStream_t s) {
    launch_expand_charges(s, nf, n, n_dv, c->d_dv, c->d_Q0, c->d_Sc, q_out);
  });
  if (f_out || e_out) launch_permute(s, nf, n, c->d_epos, c->d_Q0, c->d_qs);
  if (need_forces) {
    ForceArgs<T> fa{};
    fa.out_scale = 1.0;
    fa.field = 0.0;
    // the applied field per unit dV (finite field), or the dipole
    // correction's field from the charges dV S c (slab)
    fa.fieldb = c->geometry == CPM_FINITE_FIELD ? -1.0 / c->box[2]
              : c->geometry == CPM_SLAB ? -c->slab_kappa * c->slab_zSc : 0.0;
    fa.qb = c->d_Sc;
    if (c->kspace == CPM_KSPACE_PPPM) fa.Eb = std::is_same<T, float>::value ? (const T*)c->d_EScf : (const T*)c->d_ESc;
    // forces at dV = 0 and per unit dV, then the sweep in a streaming pass
    fa.f_out = c->d_ftmp;
    fa.f_comp = f_out ? c->d_fcomp : nullptr;
    fa.n_dv = 0;
    fa.dv = c->d_dv;
    fa.u_site = c->d_usite;
    const EnergyArgs ea = energy_args(c, n_dv, c->d_dv, 0.0, e_out);
    TRY(enqueue_forces<T>(c, nf, c->d_Q0, n, c->d_qs, fa, e_out ? &ea : nullptr));
    if (f_out)
      rec(c, CPM_KERNEL_EXPAND_F, s, [=](hipStream_t s) {
        launch_expand_forces(s, nf, c->n_site, n_dv, c->d_dv, c->d_fcomp, f_out);
      });
  }
  return CPM_OK;
}

// Frames per batched launch.  Many frames per launch amortise launch costs;
// fewer keep a launch's intermediate meshes (~2 MB per frame of the paper
// cell) within the last-level cache for the next kernel.  The tuner times
// each candidate size on the caller's first frames (second of two runs,
// HIP events on the context's stream, so it synchronises once) and keeps
// the fastest per frame.  Its runs write outputs that the real run
// overwrites.
constexpr int BATCH_CHUNK_MAX = 4096;
constexpr int BATCH_TUNE_MIN = 64;

template <typename Run>
int tune_batch_chunk(cpm_ctx* c, int n_frames, Run run) {
  std::vector<int> cand;
  for (int k = BATCH_TUNE_MIN; k <= std::min(n_frames, BATCH_CHUNK_MAX); k *= 2) cand.push_back(k);
  if (cand.empty()) return CPM_OK;
  if (c->cap_frames < cand.back()) {
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    int r = alloc_frames(c, cand.back());
    if (r) return r;
  }
  hipEvent_t e0, e1;
  HIP_TRY(c, hipEventCreate(&e0));
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return fail(c, CPM_EDEVICE, "hipEventCreate failed");
  }
  int best = cand.back();
  float best_t = 0.0f;
  int rc = CPM_OK;
  for (int k : cand) {
    float ms = 0.0f;
    for (int rep = 0; rep < 2 && rc == CPM_OK; ++rep) {
      if (hipEventRecord(e0, c->stream) != hipSuccess) { rc = fail(c, CPM_EDEVICE, "hipEventRecord failed"); break; }
      rc = run(k, 0);
      if (rc) break;
      if (hipEventRecord(e1, c->stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
          hipEventElapsedTime(&ms, e0, e1) != hipSuccess)
        rc = fail(c, CPM_EDEVICE, "timing a batch size failed");
    }
    if (rc) break;
    const float per_frame = ms / (float)k;
    if (k == cand.front() || per_frame < best_t) { best_t = per_frame; best = k; }
  }
  // then the launch shapes at that size: site-pair tiles per cell and x-y
  // planes per workgroup, each the fastest of its candidates with the other
  // at its current setting
  auto time_run = [&](int k, float& ms) -> int {
    ms = 0.0f;
    for (int rep = 0; rep < 2; ++rep) {
      if (hipEventRecord(e0, c->stream) != hipSuccess) return fail(c, CPM_EDEVICE, "hipEventRecord failed");
      int r = run(k, 0);
      if (r) return r;
      if (hipEventRecord(e1, c->stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
          hipEventElapsedTime(&ms, e0, e1) != hipSuccess)
        return fail(c, CPM_EDEVICE, "timing a launch shape failed");
    }
    return CPM_OK;
  };
  if (rc == CPM_OK) {
    float t_best = 0.0f;
    int ts_best = c->pair_tsplit;
    for (int ts : {1, 2, 4}) {
      c->pair_tsplit = ts;
      float ms;
      if ((rc = time_run(best, ms))) break;
      if (ts == 1 || ms < t_best) { t_best = ms; ts_best = ts; }
    }
    c->pair_tsplit = ts_best;
  }
  if (rc == CPM_OK) {
    float t_best = 0.0f;
    int pl_best = 0;
    for (int pl : {0, 1}) {
      c->px.planes = pl;
      float ms;
      if ((rc = time_run(best, ms))) break;
      if (pl == 0 || ms < t_best) { t_best = ms; pl_best = pl; }
    }
    c->px.planes = pl_best;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc == CPM_OK) c->batch_chunk = best;
  return rc;
}

// z.(S c) for the slab's batched dV sweep (host copy of S c; the stream is idle)
int slab_zsc(cpm_ctx* c) {
  if (c->geometry != CPM_SLAB) return CPM_OK;
  std::vector<double> sc(c->n_elec);
  HIP_TRY(c, hipMemcpy(sc.data(), c->d_Sc, sc.size() * sizeof(double), hipMemcpyDeviceToHost));
  double t = 0.0;
  for (int i = 0; i < c->n_elec; ++i) t += wrap_host(c->hz[i], c->box[2]) * sc[i];
  c->slab_zSc = t;
  return CPM_OK;
}

int check_launch(cpm_ctx* c) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(c, CPM_EDEVICE, "kernel launch failed: %s", hipGetErrorString(e));
  return CPM_OK;
}

}  // namespace

// =================================================================== C-ABI

extern "C" {

int cpm_create(const cpm_desc* d, void* hip_stream, cpm_ctx** out) {
  if (out) *out = nullptr;
  if (!d || !out) return fail(nullptr, CPM_EINVAL, "null descriptor or output pointer");
  for (int k = 0; k < 3; ++k)
    if (!(d->box[k] > 0.0) || !std::isfinite(d->box[k])) return fail(nullptr, CPM_EINVAL, "box lengths must be positive");
  if (d->geometry != CPM_FINITE_FIELD && d->geometry != CPM_DOUBLED_CELL && d->geometry != CPM_SLAB)
    return fail(nullptr, CPM_EINVAL, "unknown geometry %d", d->geometry);
  if (d->kspace != CPM_KSPACE_EWALD && d->kspace != CPM_KSPACE_PPPM)
    return fail(nullptr, CPM_EINVAL, "unknown kspace %d", d->kspace);
  if (d->precision != CPM_FP64 && d->precision != CPM_MIXED)
    return fail(nullptr, CPM_EINVAL, "unknown precision %d", d->precision);
  if (d->precision == CPM_MIXED && d->kspace != CPM_KSPACE_PPPM)
    return fail(nullptr, CPM_EINVAL, "mixed precision needs the PPPM k-space");
  if (!(d->eta > 0) || !(d->alpha > 0) || !(d->rcut > 0))
    return fail(nullptr, CPM_EINVAL, "eta, alpha and rcut must be positive");
  if (!(d->alpha < d->eta / std::sqrt(2.0)) || !(d->alpha_build < d->eta / std::sqrt(2.0)))
    return fail(nullptr, CPM_EINVAL, "alpha must be below eta/sqrt(2) (A would not be positive definite)");
  if (!(d->alpha_build > 0) || !(d->rcut_build > 0) || !(d->kcut_build > 0))
    return fail(nullptr, CPM_EINVAL, "elastance build parameters must be positive");
  if (d->alpha * d->rcut > 8.0)
    return fail(nullptr, CPM_EINVAL, "alpha * rcut must not exceed 8 (the real-space sums are converged long before)");
  if (d->n_elec < 2 || !d->elec_xyz || !d->elec_side) return fail(nullptr, CPM_EINVAL, "need >= 2 electrode atoms");
  if (d->n_site < 0 || (d->n_site > 0 && !d->site_q)) return fail(nullptr, CPM_EINVAL, "bad site charges");
  if (d->kspace == CPM_KSPACE_EWALD && !(d->kcut > 0)) return fail(nullptr, CPM_EINVAL, "EWALD needs kcut > 0");
  if (d->kspace == CPM_KSPACE_PPPM && (d->order < 2 || d->order > MAX_ORDER))
    return fail(nullptr, CPM_EINVAL, "PPPM order must be 2..%d", MAX_ORDER);
  if (d->kspace == CPM_KSPACE_PPPM)
    for (int k = 0; k < 3; ++k)
      if (d->mesh[k] < d->order)
        return fail(nullptr, CPM_EINVAL, "PPPM mesh needs at least `order` points per axis (axis %d has %d)", k,
                    d->mesh[k]);
  if (d->kspace == CPM_KSPACE_PPPM) {
    // everything about the mesh that needs no device: factorable axes, the
    // z-column limit and the LDS of the x-y planes (one-frame launches hold
    // one plane; many-frame launches fall back to one plane per workgroup
    // when several do not fit)
    const int elt = d->precision == CPM_MIXED ? (int)sizeof(float2) : (int)sizeof(double2);
    for (int k = 0; k < 3; ++k) {
      FFTPlan1D p{};
      if (!factorize(d->mesh[k], p))
        return fail(nullptr, CPM_EINVAL, "mesh size %d is not a product of 2, 3 and 5", d->mesh[k]);
    }
    if (d->mesh[2] > ZPASS_MAX_POINTS)
      return fail(nullptr, CPM_EINVAL, "mesh has more than %d points along z", ZPASS_MAX_POINTS);
    if (fft_xy_lds_bytes(d->mesh[0], d->mesh[1], elt, 1) > LDS_LIMIT)
      return fail(nullptr, CPM_EINVAL, "x-y mesh plane too large for LDS");
    const size_t spread = d->precision == CPM_MIXED ? fft_xy_spread_lds<float, float2>(d->mesh[0], d->mesh[1])
                                                    : fft_xy_spread_lds<double, double2>(d->mesh[0], d->mesh[1]);
    if (spread > LDS_LIMIT)
      return fail(nullptr, CPM_EINVAL, "mesh plane and site staging area (%zu bytes) exceed LDS", spread);
  }
  if (d->geometry == CPM_DOUBLED_CELL && !d->elec_sub) return fail(nullptr, CPM_EINVAL, "doubled cell needs elec_sub");
  if (d->flags & ~CPM_FLAG_GRAPH) return fail(nullptr, CPM_EINVAL, "unknown descriptor flags 0x%x", d->flags);
  double qsum = 0.0, qabs = 0.0;
  for (int j = 0; j < d->n_site; ++j) {
    if (!std::isfinite(d->site_q[j])) return fail(nullptr, CPM_ENONFINITE, "non-finite site charge");
    qsum += d->site_q[j];
    qabs += std::fabs(d->site_q[j]);
  }
  if (std::fabs(qsum) > 1e-9 * std::max(1.0, qabs)) return fail(nullptr, CPM_EINVAL, "electrolyte is not neutral (sum %g)", qsum);
  int n1 = 0, npos = 0;
  for (int i = 0; i < d->n_elec; ++i) {
    for (int k = 0; k < 3; ++k)
      if (!std::isfinite(d->elec_xyz[k * d->n_elec + i])) return fail(nullptr, CPM_ENONFINITE, "non-finite electrode position");
    if (d->elec_side[i] != 1 && d->elec_side[i] != -1) return fail(nullptr, CPM_EINVAL, "elec_side must be +1 or -1");
    npos += d->elec_side[i] > 0;
    if (d->geometry == CPM_DOUBLED_CELL) n1 += d->elec_sub[i] != 0;
  }
  if (npos == 0 || npos == d->n_elec) return fail(nullptr, CPM_EINVAL, "need atoms on both electrodes");
  if (d->geometry == CPM_FINITE_FIELD) {
    // the drive d - z/Lz uses z wrapped into [0, Lz): the applied ramp must
    // not jump inside an electrode, so neither may cross z = 0
    for (int side = -1; side <= 1; side += 2) {
      double lo = 1e300, hi = -1e300;
      for (int i = 0; i < d->n_elec; ++i) {
        if (d->elec_side[i] != side) continue;
        const double z = d->elec_xyz[2 * d->n_elec + i];
        const double zw = z - d->box[2] * std::floor(z / d->box[2]);
        lo = std::min(lo, zw);
        hi = std::max(hi, zw);
      }
      if (hi - lo > 0.5 * d->box[2])
        return fail(nullptr, CPM_EINVAL, "finite field: an electrode crosses the cell boundary z = 0 "
                                         "(place the boundary behind the electrodes)");
    }
  }
  if (d->geometry == CPM_SLAB) {
    // the dipole correction needs the electrodes (and the electrolyte between
    // them) inside one period with empty space across z = 0: the electrodes'
    // wrapped heights may span at most half the period
    double lo = 1e300, hi = -1e300;
    for (int i = 0; i < d->n_elec; ++i) {
      const double z = d->elec_xyz[2 * d->n_elec + i];
      const double zw = z - d->box[2] * std::floor(z / d->box[2]);
      lo = std::min(lo, zw);
      hi = std::max(hi, zw);
    }
    if (hi - lo > 0.5 * d->box[2])
      return fail(nullptr, CPM_EINVAL, "slab: the electrodes must lie within half of the z period, with the empty "
                                       "space across z = 0");
  }
  if (d->geometry == CPM_DOUBLED_CELL && (n1 == 0 || n1 == d->n_elec))
    return fail(nullptr, CPM_EINVAL, "doubled cell needs atoms in both sub-cells");

  cpm_ctx* c = new cpm_ctx();
  c->geometry = d->geometry; c->kspace = d->kspace; c->precision = d->precision;
  for (int k = 0; k < 3; ++k) { c->box[k] = d->box[k]; c->mesh[k] = d->mesh[k]; }
  c->eta = d->eta; c->alpha = d->alpha; c->rcut = d->rcut; c->kcut = d->kcut;
  c->alpha_b = d->alpha_build; c->rcut_b = d->rcut_build; c->kcut_b = d->kcut_build;
  c->order = d->order;
  c->n_elec = d->n_elec; c->n_site = d->n_site;
  c->stream = (hipStream_t)hip_stream;
  c->graph_flag = (d->flags & CPM_FLAG_GRAPH) != 0;
  c->use_graph = hip_stream != nullptr && c->graph_flag;
  const int ne = c->n_elec, ns = c->n_site;
  c->hx.assign(d->elec_xyz, d->elec_xyz + ne);
  c->hy.assign(d->elec_xyz + ne, d->elec_xyz + 2 * ne);
  c->hz.assign(d->elec_xyz + 2 * ne, d->elec_xyz + 3 * ne);
  c->side.assign(d->elec_side, d->elec_side + ne);
  if (d->geometry == CPM_DOUBLED_CELL) c->sub.assign(d->elec_sub, d->elec_sub + ne);
  c->hq.assign(d->site_q, d->site_q + ns);

  auto bad = [&](int code) { std::string e = c->err; cpm_destroy(c); g_create_error = e; return code; };
  int r;

  // cells
  Cell& cl = c->cell;
  cl.n_cells = 1;
  // cells at least rcut wide (offsets -1, 0, 1 cover the cutoff), except
  // that a z axis of three or more rcut is cut into cells at least rcut/2
  // thick with offsets -2 .. 2: the candidates of a cell then span 2.5 rcut
  // of z instead of 3 (the electrolyte fills whole x-y planes of the cells
  // this method simulates, so the z window sets the count)
  int reach[3] = {1, 1, 1};
  for (int k = 0; k < 3; ++k) {
    cl.L[k] = c->box[k];
    cl.invL[k] = 1.0 / c->box[k];
    cl.nc[k] = std::max(1, (int)std::floor(c->box[k] / c->rcut));
    cl.img[k] = (int)std::floor(c->rcut / c->box[k] + 0.5);
  }
  if (cl.nc[2] >= 3) {
    cl.nc[2] = (int)std::floor(2.0 * c->box[2] / c->rcut);
    reach[2] = 2;
  }
  for (int k = 0; k < 3; ++k) cl.n_cells *= cl.nc[k];
  std::vector<int> gn, glo, ghi;
  if (stencil_groups(cl, reach, gn, glo, ghi) > STENCIL_MAX) {
    fail(c, CPM_EINVAL, "cell stencil needs more than %d index runs", STENCIL_MAX);
    return bad(CPM_EINVAL);
  }
  {
    int *dn, *dl, *dh;
    if ((r = upload(c, &dn, gn)) || (r = upload(c, &dl, glo)) || (r = upload(c, &dh, ghi))) return bad(r);
    cl.grp_n = dn; cl.grp_lo = dl; cl.grp_hi = dh;
  }
  if (cl.img[0] == 0 && cl.img[1] == 0 && cl.img[2] == 0) {
    // forward stencils for the many-frame pair tiles (each pair once)
    std::vector<int> fn, flo, fhi;
    stencil_groups(cl, reach, fn, flo, fhi, true);
    if ((r = upload(c, &c->d_fwd_n, fn)) || (r = upload(c, &c->d_fwd_lo, flo)) || (r = upload(c, &c->d_fwd_hi, fhi)))
      return bad(r);
  }
  c->cell_b = cl;
  for (int k = 0; k < 3; ++k) c->cell_b.img[k] = (int)std::floor(c->rcut_b / c->box[k] + 0.5);
  if (bin_lds_bytes(ns, cl.n_cells) > LDS_LIMIT) {
    fail(c, CPM_EINVAL, "%d sites in %d cells exceed the single-workgroup binning limit", ns, cl.n_cells);
    return bad(CPM_EINVAL);
  }
  c->slab_kappa = KE * 4.0 * M_PI / (c->box[0] * c->box[1] * c->box[2]);
  double q2 = 0.0;
  for (double q : c->hq) q2 += q * q;
  c->self_energy = KE * c->alpha / std::sqrt(M_PI) * q2;

  // electrodes in original order and cell-sorted
  std::vector<double> dd(ne), ze(ne), cc(ne), e1(ne, 0.0);
  for (int i = 0; i < ne; ++i) {
    dd[i] = 0.5 * c->side[i];
    ze[i] = wrap_host(c->hz[i], c->box[2]);
    cc[i] = (c->geometry == CPM_FINITE_FIELD) ? dd[i] - ze[i] / c->box[2] : dd[i];
    if (c->geometry == CPM_DOUBLED_CELL) e1[i] = c->sub[i] ? 1.0 : 0.0;
  }
  std::vector<int> ecell(ne), eorder(ne);
  for (int i = 0; i < ne; ++i)
    ecell[i] = (cell_coord_host(c->hz[i], cl.L[2], cl.nc[2]) * cl.nc[1] + cell_coord_host(c->hy[i], cl.L[1], cl.nc[1])) *
                   cl.nc[0] + cell_coord_host(c->hx[i], cl.L[0], cl.nc[0]);
  for (int i = 0; i < ne; ++i) eorder[i] = i;
  std::stable_sort(eorder.begin(), eorder.end(), [&](int a, int b) { return ecell[a] < ecell[b]; });
  std::vector<int> ecs(cl.n_cells + 1, 0), ecell_sorted(ne);
  std::vector<double> sxe(ne), sye(ne), sze(ne);
  for (int k = 0; k < ne; ++k) {
    int i = eorder[k];
    ecs[ecell[i] + 1]++;
    ecell_sorted[k] = ecell[i];
    sxe[k] = wrap_host(c->hx[i], c->box[0]);
    sye[k] = wrap_host(c->hy[i], c->box[1]);
    sze[k] = wrap_host(c->hz[i], c->box[2]);
  }
  for (int k = 0; k < cl.n_cells; ++k) ecs[k + 1] += ecs[k];
  std::vector<int> epos(ne);
  for (int k = 0; k < ne; ++k) epos[eorder[k]] = k;
  if ((r = upload(c, &c->d_epos, epos))) return bad(r);
  {
    // each cell's atoms in equal chunks of at most TILE_TGT
    std::vector<int> ic, il, ih;
    for (int cc2 = 0; cc2 < cl.n_cells; ++cc2) {
      const int lo = ecs[cc2], n = ecs[cc2 + 1] - lo;
      const int nch = (n + TILE_TGT - 1) / TILE_TGT;
      for (int k = 0; k < nch; ++k) {
        ic.push_back(cc2);
        il.push_back(lo + (int)((long long)n * k / nch));
        ih.push_back(lo + (int)((long long)n * (k + 1) / nch));
      }
    }
    c->n_items = (int)ic.size();
    if ((r = upload(c, &c->d_item_c, ic)) || (r = upload(c, &c->d_item_lo, il)) || (r = upload(c, &c->d_item_hi, ih)))
      return bad(r);
  }
  if ((r = upload(c, &c->d_ex, c->hx)) || (r = upload(c, &c->d_ey, c->hy)) || (r = upload(c, &c->d_ez, c->hz)) ||
      (r = upload(c, &c->d_c, cc)) || (r = upload(c, &c->d_d, dd)) || (r = upload(c, &c->d_ze, ze)) ||
      (r = upload(c, &c->d_e1, e1)) || (r = upload(c, &c->d_site_q, c->hq)))
    return bad(r);
  {
    // distinct wrapped electrode heights (the potential profile adds each
    // height's Gaussian once with the summed charge of its atoms)
    std::vector<double> hs;
    std::vector<int> hof(ne);
    for (int i = 0; i < ne; ++i) hs.push_back(ze[i]);
    std::sort(hs.begin(), hs.end());
    hs.erase(std::unique(hs.begin(), hs.end()), hs.end());
    for (int i = 0; i < ne; ++i) hof[i] = (int)(std::lower_bound(hs.begin(), hs.end(), ze[i]) - hs.begin());
    c->n_heights = (int)hs.size();
    if ((r = upload(c, &c->d_height_of, hof)) || (r = upload(c, &c->d_heights, hs))) return bad(r);
  }
  // electrode atoms in reach of every cell: the stencil cells' ranges of the
  // sorted atoms, empty ones dropped and adjacent ones joined.  Without
  // periodic images a stencil cell is also dropped when the bounding box of
  // its atoms lies at least rcut from the cell (minimum-image distance per
  // axis, with a margin for the rounding of the cell bounds): the electrodes
  // are fixed, so the sites next to an electrode's cell but beyond the cutoff
  // from its atoms test none of them.
  const bool no_img = cl.img[0] == 0 && cl.img[1] == 0 && cl.img[2] == 0;
  std::vector<double> bb((size_t)cl.n_cells * 6, 0.0);      // per cell: lo[3], hi[3] of its atoms
  for (int e = 0; e < cl.n_cells; ++e)
    for (int k = ecs[e]; k < ecs[e + 1]; ++k) {
      const double p[3] = {sxe[k], sye[k], sze[k]};
      for (int a = 0; a < 3; ++a) {
        if (k == ecs[e] || p[a] < bb[(size_t)e * 6 + a]) bb[(size_t)e * 6 + a] = p[a];
        if (k == ecs[e] || p[a] > bb[(size_t)e * 6 + 3 + a]) bb[(size_t)e * 6 + 3 + a] = p[a];
      }
    }
  auto in_reach = [&](int cc2, int e) {
    if (!no_img) return true;
    const int ci[3] = {cc2 % cl.nc[0], (cc2 / cl.nc[0]) % cl.nc[1], cc2 / (cl.nc[0] * cl.nc[1])};
    double d2 = 0.0;
    for (int a = 0; a < 3; ++a) {
      const double L = cl.L[a], w = L / cl.nc[a], margin = 1e-9 * L;
      const double c0 = ci[a] * w - margin, c1 = (ci[a] + 1) * w + margin;
      const double b0 = bb[(size_t)e * 6 + a], b1 = bb[(size_t)e * 6 + 3 + a];
      double gap = std::numeric_limits<double>::infinity();
      for (int sh = -1; sh <= 1; ++sh)
        gap = std::min(gap, std::max(0.0, std::max(b0 + sh * L - c1, c0 - (b1 + sh * L))));
      d2 += gap * gap;
    }
    return d2 < c->rcut * c->rcut;
  };
  std::vector<int> rn(cl.n_cells, 0), rlo((size_t)cl.n_cells * STENCIL_MAX, 0), rhi((size_t)cl.n_cells * STENCIL_MAX, 0);
  for (int cc2 = 0; cc2 < cl.n_cells; ++cc2) {
    int k = 0;
    const size_t base = (size_t)cc2 * STENCIL_MAX;
    for (int g = 0; g < gn[cc2]; ++g)
      for (int e = glo[base + g]; e < ghi[base + g]; ++e) {
        const int lo = ecs[e], hi = ecs[e + 1];
        if (hi <= lo || !in_reach(cc2, e)) continue;
        if (k > 0 && rhi[base + k - 1] == lo) rhi[base + k - 1] = hi;
        else { rlo[base + k] = lo; rhi[base + k] = hi; ++k; }
      }
    rn[cc2] = k;
  }
  {
    double *x, *y, *z; int *o, *ce, *cs, *rp, *rl, *rh;
    if ((r = upload(c, &x, sxe)) || (r = upload(c, &y, sye)) || (r = upload(c, &z, sze)) ||
        (r = upload(c, &o, eorder)) || (r = upload(c, &ce, ecell_sorted)) || (r = upload(c, &cs, ecs)) ||
        (r = upload(c, &rp, rn)) || (r = upload(c, &rl, rlo)) || (r = upload(c, &rh, rhi)))
      return bad(r);
    c->el = ElecSet<double>{x, y, z, o, ce, cs, ne, rp, rl, rh};
    c->elf = ElecSet<float>{x, y, z, o, ce, cs, ne, rp, rl, rh};
  }
  if ((r = dalloc(c, &c->d_A, (size_t)ne * ne)) || (r = dalloc(c, &c->d_S, (size_t)ne * ne)) ||
      (r = dalloc(c, &c->d_Sc, ne)) || (r = dalloc(c, &c->d_Sc_s, ne)) || (r = dalloc(c, &c->d_status, 4)) ||
      (r = dalloc(c, &c->d_scalar, 8)))
    return bad(r);
  c->n_pad = (ne + 31) / 32 * 32;          // rows of the bf16 split operands: whole 32-deep MFMA slabs
  if (c->precision == CPM_MIXED) {
    if ((r = dalloc(c, &c->d_Sf, (size_t)ne * ne)) || (r = dalloc(c, &c->d_Ssplit, (size_t)3 * ne * c->n_pad)) ||
        (r = dalloc(c, &c->d_colsum, (size_t)2 * ne)))
      return bad(r);
    int n1 = 0;
    if (c->geometry == CPM_DOUBLED_CELL)
      for (int i = 0; i < ne; ++i) n1 += c->sub[i] != 0;
    c->inv_n0 = 1.0 / (ne - n1);
    c->inv_n1 = n1 > 0 ? 1.0 / n1 : 0.0;
  }
  if (c->geometry == CPM_DOUBLED_CELL && (r = upload(c, &c->d_sub1, c->sub))) return bad(r);
  if (hipMemset(c->d_status, 0, 4 * sizeof(int)) != hipSuccess) { fail(c, CPM_EDEVICE, "memset"); return bad(CPM_EDEVICE); }

  if (c->kspace == CPM_KSPACE_PPPM) {
    MeshInfo& mi = c->mi;
    for (int k = 0; k < 3; ++k) {
      if (c->mesh[k] < 2) { fail(c, CPM_EINVAL, "mesh must have >= 2 points per axis"); return bad(CPM_EINVAL); }
      mi.K[k] = c->mesh[k];
      mi.h[k] = c->box[k] / mi.K[k];
      mi.invh[k] = mi.K[k] / c->box[k];
    }
    mi.M = mi.K[0] * mi.K[1] * mi.K[2];
    mi.order = c->order;
    c->P3 = c->order * c->order * c->order;
    FFTPlan1D* plans[3] = {&c->px, &c->py, &c->pz};
    for (int k = 0; k < 3; ++k) {
      if (!factorize(mi.K[k], *plans[k])) {
        fail(c, CPM_EINVAL, "mesh size %d is not a product of 2, 3 and 5", mi.K[k]);
        return bad(CPM_EINVAL);
      }
      std::vector<double2> tw(mi.K[k]);
      std::vector<float2> twf(mi.K[k]);
      for (int t = 0; t < mi.K[k]; ++t) {
        double a = -2 * M_PI * t / mi.K[k];
        tw[t] = double2{std::cos(a), std::sin(a)};
        twf[t] = float2{(float)tw[t].x, (float)tw[t].y};
      }
      double2* dt; float2* dtf;
      if ((r = upload(c, &dt, tw)) || (r = upload(c, &dtf, twf))) return bad(r);
      plans[k]->tw = dt;
      plans[k]->twf = dtf;
    }
    const size_t elt = c->precision == CPM_MIXED ? sizeof(float2) : sizeof(double2);
    // z pass: one wavefront per (x, y) column, up to 4 per workgroup, each
    // with three lines of Kz points in LDS (plus the shared twiddles)
    const int cpw = (int)std::max<size_t>(1, std::min<size_t>(4, (LDS_LIMIT / elt - mi.K[2]) / (3 * (size_t)mi.K[2])));
    ZPassArgs za{};
    za.Kx = mi.K[0]; za.Ky = mi.K[1]; za.Kz = mi.K[2];
    za.cpw = cpw;
    za.n_blocks = (mi.K[0] * mi.K[1] + cpw - 1) / cpw;
    for (int k = 0; k < 3; ++k) za.twopi_L[k] = 2 * M_PI / c->box[k];
    za.mode = 0;
    c->za_pot = za;
    za.mode = 1;
    c->za_field = za;
    std::vector<double> G;
    influence_host(c->box, mi.K, c->order, c->alpha, G);
    std::vector<float> Gf(G.begin(), G.end());
    if ((r = upload(c, &c->d_G, G)) || (r = upload(c, &c->d_Gf, Gf))) return bad(r);
    // electrode stencils (original order) and their transpose by mesh point
    const int P = c->order, P3 = c->P3;
    std::vector<int> gidx((size_t)ne * P3);
    std::vector<double> gw((size_t)ne * P3);
    const double* pos[3] = {c->hx.data(), c->hy.data(), c->hz.data()};
    for (int i = 0; i < ne; ++i) {
      int first[3];
      double w[3][MAX_ORDER];
      for (int k = 0; k < 3; ++k) {
        double u = wrap_host(pos[k][i], c->box[k]) * mi.invh[k];
        first[k] = (int)std::floor(u - P / 2.0) + 1;
        for (int t = 0; t < P; ++t) w[k][t] = bspline_host(P, u - (first[k] + t) + P / 2.0);
      }
      for (int tz = 0; tz < P; ++tz)
        for (int ty = 0; ty < P; ++ty)
          for (int tx = 0; tx < P; ++tx) {
            int ix = ((first[0] + tx) % mi.K[0] + mi.K[0]) % mi.K[0];
            int iy = ((first[1] + ty) % mi.K[1] + mi.K[1]) % mi.K[1];
            int iz = ((first[2] + tz) % mi.K[2] + mi.K[2]) % mi.K[2];
            size_t t = (size_t)i * P3 + (tz * P + ty) * P + tx;
            gidx[t] = (iz * mi.K[1] + iy) * mi.K[0] + ix;
            gw[t] = w[0][tx] * w[1][ty] * w[2][tz];
          }
    }
    std::vector<int> cnt(mi.M, 0);
    for (size_t t = 0; t < gidx.size(); ++t) cnt[gidx[t]]++;
    std::vector<int> touch, rowptr(1, 0), col;
    std::vector<int> slot(mi.M, -1);
    for (int m = 0; m < mi.M; ++m)
      if (cnt[m]) { slot[m] = (int)touch.size(); touch.push_back(m); rowptr.push_back(rowptr.back() + cnt[m]); }
    col.resize(gidx.size());
    std::vector<double> val(gidx.size());
    std::vector<int> fillp(rowptr.begin(), rowptr.end() - 1);
    for (int i = 0; i < ne; ++i)
      for (int t = 0; t < P3; ++t) {
        size_t k = (size_t)i * P3 + t;
        int sl = slot[gidx[k]];
        col[fillp[sl]] = i;
        val[fillp[sl]] = gw[k];
        fillp[sl]++;
      }
    c->n_touch = (int)touch.size();
    // the planes the electrode stencils reach: many-frame launches transform
    // only these for the electrode charge (the other planes hold none) and
    // for the potential (read only at the electrode atoms)
    std::vector<int> zl;
    {
      std::vector<char> used(mi.K[2], 0);
      for (int g : gidx) used[g / (mi.K[0] * mi.K[1])] = 1;
      for (int z = 0; z < mi.K[2]; ++z)
        if (used[z]) zl.push_back(z);
    }
    c->n_zl = (int)zl.size();
    c->zmask_ok = mi.K[2] <= 256;
    if (c->zmask_ok)
      for (int z : zl) c->zmask_e.w[z >> 6] |= 1ull << (z & 63);
    if (bin_lds_spread(ns, cl.n_cells) > LDS_LIMIT) {
      fail(c, CPM_EINVAL, "%d sites in %d cells exceed the binning workgroup's LDS", ns, cl.n_cells);
      return bad(CPM_EINVAL);
    }
    std::vector<float> gwf(gw.begin(), gw.end()), valf(val.begin(), val.end());
    if ((r = upload(c, &c->d_gidx, gidx)) || (r = upload(c, &c->d_gw, gw)) || (r = upload(c, &c->d_gwf, gwf)) ||
        (r = upload(c, &c->d_touch, touch)) || (r = upload(c, &c->d_zl, zl)) || (r = upload(c, &c->d_rowptr, rowptr)) || (r = upload(c, &c->d_col, col)) ||
        (r = upload(c, &c->d_val, val)) || (r = upload(c, &c->d_valf, valf)))
      return bad(r);
  } else {
    std::vector<double> kx, ky, kz;
    half_kvectors(c->box, c->kcut, kx, ky, kz);
    c->nk = (int)kx.size();
    if (c->nk == 0) { fail(c, CPM_EINVAL, "kcut admits no k-vectors"); return bad(CPM_EINVAL); }
    const double vol = c->box[0] * c->box[1] * c->box[2];
    std::vector<double> kv(3 * (size_t)c->nk), ew(c->nk);
    std::vector<double2> eph((size_t)c->nk * ne);
    for (int k = 0; k < c->nk; ++k) {
      kv[k] = kx[k]; kv[c->nk + k] = ky[k]; kv[2 * c->nk + k] = kz[k];
      double k2 = kx[k] * kx[k] + ky[k] * ky[k] + kz[k] * kz[k];
      ew[k] = 2 * KE * kweight_host(k2, c->alpha, vol);
      for (int i = 0; i < ne; ++i) {
        double ph = kx[k] * c->hx[i] + ky[k] * c->hy[i] + kz[k] * c->hz[i];
        eph[(size_t)k * ne + i] = double2{std::cos(ph), std::sin(ph)};
      }
    }
    if ((r = upload(c, &c->d_kv, kv)) || (r = upload(c, &c->d_ew, ew)) || (r = upload(c, &c->d_eph, eph)))
      return bad(r);
  }
  if ((r = alloc_frames(c, 1))) return bad(r);
  {
    // set-up of cpm_profile_noalloc: this device's address of its scratch
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || profile_static_scratch(dev, &c->d_prof_static) != 0) {
      fail(c, CPM_EDEVICE, "cannot resolve the profile scratch on device %d", dev);
      return bad(CPM_EDEVICE);
    }
  }
  *out = c;
  return CPM_OK;
}

int cpm_set_stream(cpm_ctx* c, void* hip_stream) {
  if (!c) return CPM_EINVAL;
  if ((hipStream_t)hip_stream != c->stream) free_graphs(c);
  c->stream = (hipStream_t)hip_stream;
  c->use_graph = hip_stream != nullptr && c->graph_flag;
  return CPM_OK;
}

int cpm_build_elastance(cpm_ctx* c) {
  if (!c) return CPM_EINVAL;
  const int n = c->n_elec;
  hipStream_t s = c->stream;
  // real space and self term
  const double self_term = (std::sqrt(2.0) * c->eta - 2.0 * c->alpha_b) / std::sqrt(M_PI);
  launch_elastance_real(s, n, c->d_ex, c->d_ey, c->d_ez, c->cell_b, c->alpha_b, c->eta, c->rcut_b, self_term, c->d_A);
  // k space: A += C C^T over chunks of k-vectors
  std::vector<double> kx, ky, kz;
  half_kvectors(c->box, c->kcut_b, kx, ky, kz);
  const int nk = (int)kx.size();
  const double vol = c->box[0] * c->box[1] * c->box[2];
  std::vector<double> kv(3 * (size_t)nk), sk(nk);
  for (int k = 0; k < nk; ++k) {
    kv[k] = kx[k]; kv[nk + k] = ky[k]; kv[2 * nk + k] = kz[k];
    double k2 = kx[k] * kx[k] + ky[k] * ky[k] + kz[k] * kz[k];
    sk[k] = std::sqrt(2 * KE * kweight_host(k2, c->alpha_b, vol));
  }
  double *d_kv = nullptr, *d_sk = nullptr, *d_C = nullptr, *d_work = nullptr;
  int r;
  const int chunk = std::max(64, std::min(nk, (int)((size_t)(256u << 20) / (16 * (size_t)n))));
  if ((r = upload(c, &d_kv, kv)) || (r = upload(c, &d_sk, sk)) || (r = dalloc(c, &d_C, (size_t)n * 2 * chunk)))
    return r;
  for (int k0 = 0; k0 < nk; k0 += chunk) {
    int nkc = std::min(chunk, nk - k0);
    launch_phase_matrix(s, n, nkc, k0, nk, d_kv, d_sk, c->d_ex, c->d_ey, c->d_ez, d_C);
    launch_gemm_nt(s, n, n, 2 * nkc, 1.0, d_C, 2 * nkc, d_C, 2 * nkc, 1.0, c->d_A, n);
  }
  launch_symmetrize(s, n, c->d_A);
  if (c->geometry == CPM_SLAB) {
    // the dipole correction's electrode block: A += kappa z z^T (a rank-one
    // update S -= u u^T / s with u = z and s = -1/kappa)
    const double inv = -1.0 / c->slab_kappa;
    HIP_TRY(c, hipStreamSynchronize(s));
    HIP_TRY(c, hipMemcpy(c->d_scalar, &inv, sizeof(double), hipMemcpyHostToDevice));
    launch_rank1(s, n, c->d_A, c->d_ze, c->d_scalar);
  }
  // inverse (in d_S), projections
  HIP_TRY(c, hipMemcpyAsync(c->d_S, c->d_A, (size_t)n * n * sizeof(double), hipMemcpyDeviceToDevice, s));
  double *dinv, *pc, *rx, *u;
  if ((r = dalloc(c, &dinv, GJ_BLOCK * GJ_BLOCK)) || (r = dalloc(c, &pc, (size_t)n * GJ_BLOCK)) ||
      (r = dalloc(c, &rx, (size_t)n * GJ_BLOCK)) || (r = dalloc(c, &u, n)))
    return r;
  HIP_TRY(c, hipMemsetAsync(c->d_status + 1, 0, sizeof(int), s));
  launch_gj_invert(s, n, c->d_S, dinv, pc, rx, c->d_status + 1);
  TRY(check_launch(c));
  int flag = 0;
  HIP_TRY(c, hipMemcpyAsync(&flag, c->d_status + 1, sizeof(int), hipMemcpyDeviceToHost, s));
  HIP_TRY(c, hipStreamSynchronize(s));
  if (flag) return fail(c, CPM_ENOTSPD, "elastance matrix is not positive definite (coincident electrode atoms?)");
  launch_matvec(s, n, c->d_S, nullptr, u);                 // u = A^-1 e
  launch_dot(s, n, u, nullptr, c->d_scalar);                // e.u
  launch_rank1(s, n, c->d_S, u, c->d_scalar);               // S = A^-1 - u u^T / e.u
  if (c->geometry == CPM_DOUBLED_CELL) {
    launch_matvec(s, n, c->d_S, c->d_e1, u);                // w = S e1
    launch_dot(s, n, u, c->d_e1, c->d_scalar);              // e1.w
    launch_rank1(s, n, c->d_S, u, c->d_scalar);             // S -= w w^T / e1.w
  }
  launch_matvec(s, n, c->d_S, c->d_c, c->d_Sc);            // S c
  launch_permute(s, 1, n, c->d_epos, c->d_Sc, c->d_Sc_s);
  if (c->precision == CPM_MIXED) {
    launch_split_matrix(s, n, c->n_pad, c->d_S, c->d_Sf, c->d_Ssplit);
    launch_colsum(s, n, c->d_Sf, c->d_sub1, c->d_colsum);
  }
  TRY(check_launch(c));
  HIP_TRY(c, hipStreamSynchronize(s));
  TRY(slab_zsc(c));
  // the chunk buffers are released now (they are large)
  for (void* p : {(void*)d_kv, (void*)d_sk, (void*)d_C, (void*)dinv, (void*)pc, (void*)rx, (void*)u}) {
    (void)hipFree(p);
    c->allocs.erase(std::remove(c->allocs.begin(), c->allocs.end(), p), c->allocs.end());
  }
  c->built = true;
  c->esc_ready = false;
  free_graphs(c);
  return CPM_OK;
}

int cpm_set_matrix(cpm_ctx* c, const double* host_S) {
  if (!c || !host_S) return CPM_EINVAL;
  const int n = c->n_elec;
  HIP_TRY(c, hipMemcpy(c->d_S, host_S, (size_t)n * n * sizeof(double), hipMemcpyHostToDevice));
  launch_matvec(c->stream, n, c->d_S, c->d_c, c->d_Sc);
  launch_permute(c->stream, 1, n, c->d_epos, c->d_Sc, c->d_Sc_s);
  if (c->precision == CPM_MIXED) {
    launch_split_matrix(c->stream, n, c->n_pad, c->d_S, c->d_Sf, c->d_Ssplit);
    launch_colsum(c->stream, n, c->d_Sf, c->d_sub1, c->d_colsum);
  }
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  TRY(slab_zsc(c));
  c->built = true;
  c->esc_ready = false;
  free_graphs(c);
  return CPM_OK;
}

int cpm_solve(cpm_ctx* c, const double* xyz, double dv, double* q_out, double* f_out, double* e_out) {
  if (!c) return CPM_EINVAL;
  if (!c->built) return fail(c, CPM_ESTATE, "cpm_solve before cpm_build_elastance");
  if (!xyz || !q_out) return fail(c, CPM_EINVAL, "site_xyz and q_out are required");
  if (!std::isfinite(dv)) return fail(c, CPM_ENONFINITE, "non-finite dV");
  // (a replayed graph does not pass through the enqueue, which clears the MD
  // loop's claim on the sorted charges that this solve overwrites)
  c->elec_owner = nullptr;
  auto enqueue = [&]() {
    return c->precision == CPM_MIXED ? enqueue_solve<float>(c, xyz, dv, q_out, f_out, e_out)
                                     : enqueue_solve<double>(c, xyz, dv, q_out, f_out, e_out);
  };
  if (!c->use_graph) {
    TRY(enqueue());
    return check_launch(c);
  }
  const void* key[6] = {xyz, q_out, f_out, e_out, nullptr, nullptr};
  for (auto& g : c->graphs) {
    if (g.kind == 0 && g.dv == dv && std::memcmp(g.p, key, sizeof(key)) == 0) {
      g.last_use = ++c->tick;
      HIP_TRY(c, hipGraphLaunch(g.exec, c->stream));
      return CPM_OK;
    }
  }
  hipGraph_t graph;
  HIP_TRY(c, hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
  int r = enqueue();
  hipError_t e = hipStreamEndCapture(c->stream, &graph);
  if (r != CPM_OK) return r;
  if (e != hipSuccess) return fail(c, CPM_EDEVICE, "graph capture failed: %s", hipGetErrorString(e));
  GraphEntry ge{};
  std::memcpy(ge.p, key, sizeof(key));
  ge.dv = dv;
  ge.kind = 0;
  e = hipGraphInstantiate(&ge.exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (e != hipSuccess) return fail(c, CPM_EDEVICE, "graph instantiate failed: %s", hipGetErrorString(e));
  ge.last_use = ++c->tick;
  if (c->graphs.size() >= 16) {
    auto it = std::min_element(c->graphs.begin(), c->graphs.end(),
                               [](const GraphEntry& a, const GraphEntry& b) { return a.last_use < b.last_use; });
    (void)hipGraphExecDestroy(it->exec);
    c->graphs.erase(it);
  }
  c->graphs.push_back(ge);
  HIP_TRY(c, hipGraphLaunch(ge.exec, c->stream));
  return CPM_OK;
}

int cpm_solve_batch(cpm_ctx* c, int n_frames, const double* xyz, int n_dv, const double* dv_host, double* q_out,
                    double* f_out, double* e_out) {
  if (!c) return CPM_EINVAL;
  if (!c->built) return fail(c, CPM_ESTATE, "cpm_solve_batch before cpm_build_elastance");
  if (n_frames < 0 || n_dv < 1 || !dv_host || (n_frames > 0 && (!xyz || !q_out)))
    return fail(c, CPM_EINVAL, "bad batch arguments");
  if (c->kspace != CPM_KSPACE_PPPM) return fail(c, CPM_EINVAL, "the batched form runs on the PPPM k-space");
  if (n_frames == 0) return CPM_OK;
  for (int v = 0; v < n_dv; ++v)
    if (!std::isfinite(dv_host[v])) return fail(c, CPM_ENONFINITE, "non-finite dV");
  if (c->cap_dv < n_dv) {
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    int r = dalloc(c, &c->d_dv, n_dv);
    if (r) return r;
    c->cap_dv = n_dv;
  }
  HIP_TRY(c, hipMemcpyAsync(c->d_dv, dv_host, n_dv * sizeof(double), hipMemcpyHostToDevice, c->stream));
  const bool mixed = c->precision == CPM_MIXED;
  if ((f_out || e_out) && c->kspace == CPM_KSPACE_PPPM && !c->esc_ready) {
    int r = mixed ? dalloc(c, &c->d_EScf, 3 * (size_t)c->mi.M) : dalloc(c, &c->d_ESc, 3 * (size_t)c->mi.M);
    if (r) return r;
    if (mixed) enqueue_esc_mesh<float>(c, c->d_EScf);
    else enqueue_esc_mesh<double>(c, c->d_ESc);
    c->esc_ready = true;
  }
  auto run = [&](int nf, int f0) {
    const size_t xs3 = (size_t)3 * c->n_site;
    double* q = q_out + (size_t)f0 * n_dv * c->n_elec;
    double* f = f_out ? f_out + (size_t)f0 * n_dv * xs3 : nullptr;
    double* e = e_out ? e_out + (size_t)f0 * n_dv * 2 : nullptr;
    return mixed ? enqueue_batch<float>(c, nf, xyz + f0 * xs3, n_dv, q, f, e)
                 : enqueue_batch<double>(c, nf, xyz + f0 * xs3, n_dv, q, f, e);
  };
  // frames per launch: set by CPM_BATCH_CHUNK, else tuned on the first call
  // with enough frames, else all of them (at most BATCH_CHUNK_MAX)
  int chunk_max;
  if (const char* env = std::getenv("CPM_BATCH_CHUNK")) {
    chunk_max = (int)std::max<long>(1, std::atol(env));
  } else {
    if (c->batch_chunk == 0 && n_frames >= 2 * BATCH_TUNE_MIN) {
      int r = tune_batch_chunk(c, n_frames, run);
      if (r) return r;
    }
    chunk_max = c->batch_chunk > 0 ? c->batch_chunk : BATCH_CHUNK_MAX;
  }
  chunk_max = std::max(1, std::min(chunk_max, n_frames));
  if (c->cap_frames < chunk_max) {
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    int r = alloc_frames(c, chunk_max);
    if (r) return r;
  }
  for (int f0 = 0; f0 < n_frames; f0 += chunk_max) {
    int r = run(std::min(chunk_max, n_frames - f0), f0);
    if (r) return r;
  }
  return check_launch(c);
}

int cpm_set_batch_shape(cpm_ctx* c, int frames_per_launch, int tiles_per_cell, int xy_planes) {
  if (!c) return CPM_EINVAL;
  if (frames_per_launch < 1 || frames_per_launch > BATCH_CHUNK_MAX)
    return fail(c, CPM_EINVAL, "frames per launch must be 1..%d", BATCH_CHUNK_MAX);
  if (tiles_per_cell < 1 || tiles_per_cell > TILE_TGT) return fail(c, CPM_EINVAL, "tiles per cell must be 1..%d", TILE_TGT);
  if (xy_planes != 0 && xy_planes != 1) return fail(c, CPM_EINVAL, "x-y planes per workgroup must be 0 or 1");
  c->batch_chunk = frames_per_launch;
  c->pair_tsplit = tiles_per_cell;
  c->px.planes = xy_planes;
  return CPM_OK;
}

int cpm_grad(cpm_ctx* c, const double* xyz, double dv, const double* q_target, double* loss_out, double* dl_dxyz,
             double* dl_ddv, double* q_out) {
  if (!c) return CPM_EINVAL;
  if (!c->built) return fail(c, CPM_ESTATE, "cpm_grad before cpm_build_elastance");
  if (!xyz || !q_target || !loss_out || !dl_dxyz || !dl_ddv) return fail(c, CPM_EINVAL, "null argument");
  if (!std::isfinite(dv)) return fail(c, CPM_ENONFINITE, "non-finite dV");
  int r = c->precision == CPM_MIXED ? enqueue_grad<float>(c, xyz, dv, q_target, loss_out, dl_dxyz, dl_ddv, q_out)
                                    : enqueue_grad<double>(c, xyz, dv, q_target, loss_out, dl_dxyz, dl_ddv, q_out);
  if (r) return r;
  return check_launch(c);
}

namespace {

// arguments of a profile call, checked; part is left for the caller to set
int profile_args(cpm_ctx* c, int n_frames, const double* xyz, const double* q, long long q_stride, double dv,
                 int n_bins, double bulk_lo, double bulk_hi, double* rho_out, double* psi_out, ProfileArgs& p) {
  if (n_frames < 1 || !xyz || !q || !rho_out || !psi_out) return fail(c, CPM_EINVAL, "bad profile arguments");
  if (n_bins < 2 || n_bins > PROFILE_MAX_BINS) return fail(c, CPM_EINVAL, "n_bins must be 2..%d", PROFILE_MAX_BINS);
  if (q_stride < c->n_elec) return fail(c, CPM_EINVAL, "q_stride must be at least n_elec");
  if (!std::isfinite(dv) || !std::isfinite(bulk_lo) || !std::isfinite(bulk_hi))
    return fail(c, CPM_ENONFINITE, "non-finite profile argument");
  if (c->n_heights > PROFILE_MAX_HEIGHTS)
    return fail(c, CPM_EINVAL, "more than %d distinct electrode heights", PROFILE_MAX_HEIGHTS);
  const double h = c->box[2] / n_bins;
  int in_bulk = 0;
  for (int k = 0; k < n_bins; ++k) in_bulk += ((k + 0.5) * h >= bulk_lo && (k + 0.5) * h < bulk_hi);
  if (in_bulk == 0) return fail(c, CPM_EINVAL, "the bulk window holds no bin centre");
  p = ProfileArgs{};
  p.n_frames = n_frames; p.n_site = c->n_site; p.n_elec = c->n_elec; p.n_bins = n_bins;
  p.n_heights = c->n_heights;
  const long long work = (long long)n_frames * std::max(c->n_site, c->n_elec);
  p.n_part = (int)std::max<long long>(1, std::min<long long>(PROFILE_MAX_PARTS, (work + 8191) / 8192));
  p.slab = c->geometry == CPM_SLAB;
  p.xyz = xyz; p.site_q = c->d_site_q; p.q = q; p.q_stride = (size_t)q_stride;
  p.height_of = c->d_height_of; p.heights = c->d_heights;
  p.Lz = c->box[2]; p.inv_Lz = 1.0 / c->box[2]; p.inv_h = n_bins / c->box[2];
  p.area = c->box[0] * c->box[1]; p.eta = c->eta;
  p.jump = c->geometry == CPM_FINITE_FIELD ? dv : 0.0;
  p.bulk_lo = bulk_lo; p.bulk_hi = bulk_hi;
  p.rho_out = rho_out; p.psi_out = psi_out;
  return CPM_OK;
}

}  // namespace

int cpm_profile(cpm_ctx* c, int n_frames, const double* site_xyz, const double* q, long long q_stride, double dv,
                int n_bins, double bulk_lo, double bulk_hi, double* rho_out, double* psi_out) {
  if (!c) return CPM_EINVAL;
  ProfileArgs p;
  TRY(profile_args(c, n_frames, site_xyz, q, q_stride, dv, n_bins, bulk_lo, bulk_hi, rho_out, psi_out, p));
  const size_t need = (size_t)p.n_part * (p.n_bins + p.n_heights);
  if (need > c->cap_prof) {
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    TRY(dalloc(c, &c->d_prof, need));
    c->cap_prof = need;
  }
  p.part = c->d_prof;
  launch_profile(c->stream, p);
  return check_launch(c);
}

int cpm_profile_noalloc(cpm_ctx* c, int n_frames, const double* site_xyz, const double* q, long long q_stride,
                        double dv, int n_bins, double bulk_lo, double bulk_hi, double* rho_out, double* psi_out) {
  if (!c) return CPM_EINVAL;
  ProfileArgs p;
  TRY(profile_args(c, n_frames, site_xyz, q, q_stride, dv, n_bins, bulk_lo, bulk_hi, rho_out, psi_out, p));
  const size_t need = (size_t)p.n_part * (p.n_bins + p.n_heights);
  if (need > PROFILE_STATIC_DOUBLES)
    return fail(c, CPM_EINVAL, "profile scratch of %zu doubles exceeds the static %zu", need, PROFILE_STATIC_DOUBLES);
  if (!c->d_prof_static) return fail(c, CPM_ESTATE, "profile scratch not set up");
  p.part = c->d_prof_static;
  launch_profile(c->stream, p);
  return check_launch(c);
}

int cpm_md_create(cpm_ctx* c, const cpm_md_desc* d, cpm_md** out) {
  if (out) *out = nullptr;
  if (!c || !d || !out) return CPM_EINVAL;
  if (!c->built) return fail(c, CPM_ESTATE, "cpm_md_create before cpm_build_elastance");
  if (c->precision != CPM_FP64) return fail(c, CPM_EINVAL, "the MD loop runs the FP64 path");
  if (d->n_mol < 1 || !d->mol_size || !d->mol_group || !d->site_mass || !d->site_sigma || !d->site_eps)
    return fail(c, CPM_EINVAL, "bad molecule or site tables");
  if (d->n_groups < 1 || d->n_groups > MD_MAX_GROUPS) return fail(c, CPM_EINVAL, "n_groups must be 1..%d", MD_MAX_GROUPS);
  if (d->n_lj_elec < 0 || (d->n_lj_elec > 0 && !d->lj_elec_xyz)) return fail(c, CPM_EINVAL, "bad graphene atoms");
  if (!(d->dt > 0) || !(d->temperature > 0) || !(d->tau > 0) || !(d->lj_cut > 0) || !(d->bond > 0) ||
      d->charge_every < 1)
    return fail(c, CPM_EINVAL, "dt, temperature, tau, lj_cut, bond and charge_every must be positive");
  if (2.0 * d->lj_cut > std::min(c->box[0], std::min(c->box[1], c->box[2])))
    return fail(c, CPM_EINVAL, "the Lennard-Jones cutoff must be below half the smallest box length");
  const int ns = c->n_site;
  std::vector<int> start(d->n_mol), mol_of(ns);
  std::vector<double> nsite_g(d->n_groups, 0.0), ncon_g(d->n_groups, 0.0);
  int at = 0;
  for (int m = 0; m < d->n_mol; ++m) {
    const int k = d->mol_size[m], g = d->mol_group[m];
    if (k != 1 && k != 3) return fail(c, CPM_EINVAL, "molecules have 1 or 3 sites");
    if (g < 0 || g >= d->n_groups) return fail(c, CPM_EINVAL, "molecule %d: group out of range", m);
    if (at + k > ns) return fail(c, CPM_EINVAL, "molecules hold more sites than the context");
    start[m] = at;
    for (int t = 0; t < k; ++t) {
      if (!(d->site_mass[at + t] > 0)) return fail(c, CPM_EINVAL, "site masses must be positive");
      mol_of[at + t] = m;
    }
    nsite_g[g] += k;
    ncon_g[g] += k == 3 ? 3 : 0;
    at += k;
  }
  if (at != ns) return fail(c, CPM_EINVAL, "molecules hold %d sites, the context %d", at, ns);
  cpm_md* md = new cpm_md();
  md->c = c;
  md->charge_every = d->charge_every;
  auto bad = [&](int code) {
    for (void* p : md->allocs) (void)hipFree(p);
    delete md;
    return code;
  };
  auto up = [&](auto** p, const auto* h, size_t n) -> int {
    using T = std::remove_const_t<std::remove_pointer_t<decltype(h)>>;
    T* q = nullptr;
    if (hipMalloc((void**)&q, std::max<size_t>(1, n) * sizeof(T)) != hipSuccess)
      return fail(c, CPM_ENOMEM, "hipMalloc failed");
    md->allocs.push_back(q);
    if (n && h && hipMemcpy(q, h, n * sizeof(T), hipMemcpyHostToDevice) != hipSuccess)
      return fail(c, CPM_EDEVICE, "upload failed");
    *p = q;
    return CPM_OK;
  };
  MDArgs& a = md->a;
  a.n_site = ns; a.n_mol = d->n_mol; a.n_groups = d->n_groups; a.n_lj_elec = d->n_lj_elec; a.thermostat = 1;
  a.carbon_sigma = d->carbon_sigma; a.carbon_sqeps = std::sqrt(d->carbon_eps); a.lj_cut = d->lj_cut; a.bond = d->bond;
  a.dt = d->dt; a.kt = 0.0083144626 * d->temperature;
  for (int k = 0; k < 3; ++k) { a.box[k] = c->box[k]; a.inv_box[k] = 1.0 / c->box[k]; }
  for (int g = 0; g < d->n_groups; ++g) {
    a.nf[g] = 3.0 * nsite_g[g] - ncon_g[g];
    a.Q[g] = a.nf[g] * a.kt * d->tau * d->tau;
  }
  const double* mass_c; const double* sig_c; const double* eps_c; const int *ms, *mz, *mg, *mo; const double* cx;
  double *f_lj, *u_lj, *xi, *eta, *nh_in, *part, *q, *fc, *en;
  int r;
  std::vector<double> zeros(2 * MD_MAX_GROUPS, 0.0);
  std::vector<int> sizes(d->mol_size, d->mol_size + d->n_mol), groups(d->mol_group, d->mol_group + d->n_mol);
  std::vector<double> sqeps(ns);
  for (int j = 0; j < ns; ++j) {
    if (!(d->site_eps[j] >= 0.0)) { for (void* p : md->allocs) (void)hipFree(p); delete md; return fail(c, CPM_EINVAL, "epsilon must be >= 0"); }
    sqeps[j] = std::sqrt(d->site_eps[j]);
  }
  // z windows of the Lennard-Jones partners over the electrostatic cell grid:
  // the graphene atoms sorted by wrapped z, and per z layer the (at most
  // two, across the periodic boundary) index ranges of those within lj_cut
  const Cell& cl = c->cell;
  const int ncz = cl.nc[2], nlj = d->n_lj_elec;
  const double Lz = cl.L[2], wz = Lz / ncz;
  std::vector<int> cord(nlj);
  std::vector<double> cz(nlj);
  for (int i = 0; i < nlj; ++i) { cord[i] = i; cz[i] = wrap_host(d->lj_elec_xyz[2 * nlj + i], Lz); }
  std::stable_sort(cord.begin(), cord.end(), [&](int p1, int p2) { return cz[p1] < cz[p2]; });
  std::vector<double> cxs(3 * (size_t)nlj), czs(nlj);
  for (int i = 0; i < nlj; ++i) {
    for (int k = 0; k < 3; ++k) cxs[(size_t)k * nlj + i] = d->lj_elec_xyz[(size_t)k * nlj + cord[i]];
    czs[i] = cz[cord[i]];
  }
  std::vector<int> crun(4 * (size_t)ncz, 0);
  auto lower = [&](double z) { return (int)(std::lower_bound(czs.begin(), czs.end(), z) - czs.begin()); };
  const double pad = d->lj_cut + 1e-9 * Lz;                  // margin for the rounding of the layer bounds
  for (int L = 0; L < ncz; ++L) {
    const double lo = L * wz - pad, hi = (L + 1) * wz + pad;
    int* q2 = &crun[4 * (size_t)L];
    if (hi - lo >= Lz) { q2[0] = 0; q2[1] = nlj; continue; }
    if (lo < 0.0) {                 // [lo + Lz, Lz) and [0, hi)
      q2[0] = lower(lo + Lz); q2[1] = nlj; q2[2] = 0; q2[3] = lower(hi);
    } else if (hi > Lz) {           // [lo, Lz) and [0, hi - Lz)
      q2[0] = lower(lo); q2[1] = nlj; q2[2] = 0; q2[3] = lower(hi - Lz);
    } else {
      q2[0] = lower(lo); q2[1] = lower(hi);
    }
  }
  const int reach = (int)std::ceil(pad / wz);                 // layers of sites within lj_cut, the same margin
  const int* crun_d;
  if ((r = up(&mass_c, d->site_mass, ns)) || (r = up(&sig_c, d->site_sigma, ns)) || (r = up(&eps_c, sqeps.data(), ns)) ||
      (r = up(&ms, start.data(), d->n_mol)) || (r = up(&mz, sizes.data(), d->n_mol)) ||
      (r = up(&mg, groups.data(), d->n_mol)) || (r = up(&mo, mol_of.data(), ns)) ||
      (r = up(&cx, cxs.data(), 3 * (size_t)nlj)) || (r = up(&crun_d, crun.data(), 4 * (size_t)ncz)) ||
      (r = up(&f_lj, (const double*)nullptr, 3 * (size_t)ns)) ||
      (r = up(&u_lj, (const double*)nullptr, ns)) || (r = up(&xi, zeros.data(), MD_MAX_GROUPS)) ||
      (r = up(&eta, zeros.data(), MD_MAX_GROUPS)) ||
      (r = up(&nh_in, zeros.data(), 2 * MD_MAX_GROUPS)) || (r = up(&part, (const double*)nullptr, (size_t)md_workgroups(d->n_mol) * MD_PART)) || (r = up(&q, (const double*)nullptr, c->n_elec)) ||
      (r = up(&fc, (const double*)nullptr, 3 * (size_t)ns)) || (r = up(&en, zeros.data(), 2)))
    return bad(r);
  a.mass = mass_c; a.sigma = sig_c; a.sqeps = eps_c; a.mol_start = ms; a.mol_size = mz; a.mol_group = mg; a.mol_of = mo;
  a.cx = cx; a.f_lj = f_lj; a.u_lj = u_lj; a.xi = xi; a.eta = eta; a.nh_in = nh_in; a.md_part = part; a.f_c = fc; a.energy = en;
  a.cell_start = c->d_cell_start; a.order = c->d_order; a.carbon_run = crun_d;
  a.nc_z = ncz; a.nxy = cl.nc[0] * cl.nc[1]; a.lj_reach = reach; a.Lz = Lz;
  md->d_q = q; md->d_fc = fc; md->d_energy = en;
  if (c->kspace == CPM_KSPACE_PPPM && !c->d_c1e && dalloc(c, &c->d_c1e, (size_t)c->mi.M) != CPM_OK)
    return bad(CPM_ENOMEM);
  *out = md;
  return CPM_OK;
}

namespace {

// forces at the current positions: Lennard-Jones, and the Coulomb forces
// with a charge solve (update) or at the charges of the last update
int md_forces(cpm_md* md, double* x, double dv, bool update) {
  cpm_ctx* c = md->c;
  // the Coulomb part first: its binning of x gives the Lennard-Jones sums
  // their z windows, and its field pass hosts them (PPPM; else a launch of
  // their own follows).  Between charge updates the electrode spectrum and
  // the sorted charges of the last update are reused, if nothing else has
  // run on the context since
  c->elec_mode = (!update && c->elec_owner == md) ? 2 : 1;
  md->a.cell_start = c->d_cell_start;
  md->a.order = c->d_order;
  c->host_lj = &md->a;                 // the Lennard-Jones sums ride in the field pass (PPPM)
  c->lj_hosted = false;
  const int r = update ? enqueue_solve<double>(c, x, dv, md->d_q, md->d_fc, md->d_energy)
                       : enqueue_forces_at<double>(c, x, dv, md->d_q, md->d_fc);
  c->elec_mode = 0;
  c->host_lj = nullptr;
  TRY(r);
  if (c->d_c1e) c->elec_owner = md;
  if (!c->lj_hosted) launch_lj(c->stream, md->a);
  c->lj_hosted = false;
  return CPM_OK;
}

}  // namespace

int cpm_md_run(cpm_md* md, double* x, double* v, double dv, int n_steps, double* q_out, double* thermo_out) {
  if (!md) return CPM_EINVAL;
  cpm_ctx* c = md->c;
  if (!x || !v || n_steps < 0) return fail(c, CPM_EINVAL, "bad MD run arguments");
  if (!std::isfinite(dv)) return fail(c, CPM_ENONFINITE, "non-finite dV");
  MDArgs& a = md->a;
  a.x = x; a.v = v; a.thermo_out = nullptr;
  hipStream_t s = c->stream;
  if (!md->started) {
    // velocities normal to the constraints, forces with fresh charges
    launch_md_integrate(s, a, 4, 0);
    TRY(md_forces(md, x, dv, true));
    md->started = true;
  }
  a.thermo_out = thermo_out;
  for (int i = 0; i < n_steps; ++i) {
    // end of the previous step (from the second step of this call on), start of this one
    launch_md_integrate(s, a, i == 0 ? 2 : 3, i - 1);
    ++md->step;
    TRY(md_forces(md, x, dv, md->step % md->charge_every == 0));
  }
  if (n_steps > 0) launch_md_integrate(s, a, 1, n_steps - 1);
  if (q_out) HIP_TRY(c, hipMemcpyAsync(q_out, md->d_q, c->n_elec * sizeof(double), hipMemcpyDeviceToDevice, s));
  return check_launch(c);
}

int cpm_md_state(cpm_md* md, double* xi_host, double* eta_host, long long* step_host) {
  if (!md) return CPM_EINVAL;
  cpm_ctx* c = md->c;
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  if (xi_host) HIP_TRY(c, hipMemcpy(xi_host, md->a.xi, md->a.n_groups * sizeof(double), hipMemcpyDeviceToHost));
  if (eta_host) HIP_TRY(c, hipMemcpy(eta_host, md->a.eta, md->a.n_groups * sizeof(double), hipMemcpyDeviceToHost));
  if (step_host) *step_host = md->step;
  return CPM_OK;
}

int cpm_md_set_thermostat(cpm_md* md, int on) {
  if (!md) return CPM_EINVAL;
  md->a.thermostat = on ? 1 : 0;
  return CPM_OK;
}

void cpm_md_destroy(cpm_md* md) {
  if (!md) return;
  if (md->c && md->c->elec_owner == md) md->c->elec_owner = nullptr;
  if (md->c && md->c->stream) (void)hipStreamSynchronize(md->c->stream);
  for (void* p : md->allocs) (void)hipFree(p);
  delete md;
}

int cpm_get_matrix(cpm_ctx* c, int which, double* host_out) {
  if (!c || !host_out) return CPM_EINVAL;
  if (!c->built) return fail(c, CPM_ESTATE, "matrices not built");
  const size_t n = c->n_elec;
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  if (which == 0) HIP_TRY(c, hipMemcpy(host_out, c->d_A, n * n * sizeof(double), hipMemcpyDeviceToHost));
  else if (which == 1) HIP_TRY(c, hipMemcpy(host_out, c->d_S, n * n * sizeof(double), hipMemcpyDeviceToHost));
  else if (which == 2) HIP_TRY(c, hipMemcpy(host_out, c->d_Sc, n * sizeof(double), hipMemcpyDeviceToHost));
  else return fail(c, CPM_EINVAL, "unknown matrix %d", which);
  return CPM_OK;
}

long long cpm_get_buffer(cpm_ctx* c, int which, void* host_out) {
  if (!c) return CPM_EINVAL;
  const bool pppm = c->kspace == CPM_KSPACE_PPPM;
  const bool mixed = c->precision == CPM_MIXED;
  const size_t M = c->mi.M;
  const void* src = nullptr;
  size_t count = 0, elt = sizeof(double);
  std::vector<double> conv;
  switch (which) {
    case CPM_BUF_CELL_START: src = c->d_cell_start; count = c->cell.n_cells + 1; elt = sizeof(int); break;
    case CPM_BUF_SITE_ORDER: src = c->d_order; count = c->n_site; elt = sizeof(int); break;
    case CPM_BUF_PHI_REAL: src = mixed ? (const void*)c->d_phirf : c->d_phir; count = c->n_elec; if (mixed) elt = 4; break;
    case CPM_BUF_B: src = c->d_b; count = c->n_elec; break;
    case CPM_BUF_RHO_MESH: if (!pppm) return 0; src = mixed ? (const void*)c->d_rhof : c->d_rho; count = M; if (mixed) elt = 4; break;
    case CPM_BUF_PHI_MESH: if (!pppm) return 0; src = mixed ? (const void*)c->d_phif : c->d_phi; count = M; if (mixed) elt = 4; break;
    case CPM_BUF_FIELD_MESH: if (!pppm) return 0; src = mixed ? (const void*)c->d_Ef : c->d_E; count = 3 * M; if (mixed) elt = 4; break;
    case CPM_BUF_NCELL:
      if (host_out) std::memcpy(host_out, c->cell.nc, 3 * sizeof(int));
      return 3;
    case CPM_BUF_BATCH_CHUNK:
      if (host_out) {
        const int v[3] = {c->batch_chunk, c->pair_tsplit, c->px.planes};
        std::memcpy(host_out, v, sizeof(v));
      }
      return 3;
    default: return fail(c, CPM_EINVAL, "unknown buffer %d", which);
  }
  if (!host_out) return (long long)count;
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  if (elt == 4 && which != CPM_BUF_CELL_START && which != CPM_BUF_SITE_ORDER) {
    std::vector<float> tmp(count);
    HIP_TRY(c, hipMemcpy(tmp.data(), src, count * 4, hipMemcpyDeviceToHost));
    double* o = (double*)host_out;
    for (size_t i = 0; i < count; ++i) o[i] = tmp[i];
  } else {
    HIP_TRY(c, hipMemcpy(host_out, src, count * elt, hipMemcpyDeviceToHost));
  }
  return (long long)count;
}

int cpm_replay_kernel(cpm_ctx* c, int kernel, int reps) {
  if (!c) return CPM_EINVAL;
  if (kernel < 0 || kernel >= CPM_KERNEL_COUNT || reps < 0) return fail(c, CPM_EINVAL, "bad kernel id or count");
  if (!c->last_launch[kernel]) return fail(c, CPM_ESTATE, "kernel %d has not run yet", kernel);
  for (int i = 0; i < reps; ++i) c->last_launch[kernel]();
  return check_launch(c);
}

int cpm_sync_status(cpm_ctx* c) {
  if (!c) return CPM_EINVAL;
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  int st = 0;
  HIP_TRY(c, hipMemcpy(&st, c->d_status, sizeof(int), hipMemcpyDeviceToHost));
  HIP_TRY(c, hipMemset(c->d_status, 0, sizeof(int)));
  if (st & 1) return fail(c, CPM_ENONFINITE, "non-finite site position");
  return CPM_OK;
}

const char* cpm_last_error(const cpm_ctx* c) {
  if (!c) return g_create_error.c_str();
  return c->err.c_str();
}

void cpm_destroy(cpm_ctx* c) {
  if (!c) return;
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  else (void)hipDeviceSynchronize();
  free_graphs(c);
  for (void* p : c->allocs) (void)hipFree(p);
  delete c;
}

}  // extern "C"
