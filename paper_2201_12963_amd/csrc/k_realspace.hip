// Real-space kernels of the step (Eq. 1-3): the electrolyte potential at the
// electrodes (one wavefront per electrode atom), the site-site forces (one
// wavefront per site) and the rest of the force on every site once the
// electrode charges are known; the pair machinery is in pairs.h.
#include "pairs.h"
#include "tiles.h"
#include "energy.h"

namespace cpm {

template <typename T>
__global__ __launch_bounds__(TILE_THREADS) void k_real_b(RealBArgs<T> rb) {
  extern __shared__ __align__(16) unsigned char lds[];
  real_b_block(rb, xcd_block(blockIdx.x, gridDim.x), blockIdx.y, lds);
}

template <typename T>
void launch_real_b_t(hipStream_t s, int n_frames, const RealBArgs<T>& rb) {
  if (rb.n_blocks == 0 || n_frames == 0) return;
  const size_t lds = rb.tiles ? PairLds<T>::total : 4 * wave_scratch_bytes<T>();
  hipLaunchKernelGGL(k_real_b<T>, dim3(rb.n_blocks, n_frames), dim3(TILE_THREADS), lds, s, rb);
}

template <typename T>
__global__ __launch_bounds__(TILE_THREADS) void k_site_pairs(PairArgs<T> pa) {
  extern __shared__ __align__(16) unsigned char lds[];
  site_pairs_block(pa, xcd_block(blockIdx.x, gridDim.x), blockIdx.y, lds);
}

// The cell-tile form (many frames) as a kernel of its own, held to five
// wavefronts per SIMD (its ~32 KB of LDS allow five workgroups per CU; the
// few registers it then spills cost less than the fifth workgroup gains).
template <typename T>
__global__ __launch_bounds__(TILE_THREADS, 5) void k_site_pairs_tiles(PairArgs<T> pa) {
  extern __shared__ __align__(16) unsigned char lds[];
  site_pairs_block<T, 0>(pa, xcd_block(blockIdx.x, gridDim.x), blockIdx.y, lds);
}

// The site-electrode sums of many frames beside k_site_pairs_n3 (~20 KB of
// LDS in FP64): four workgroups per CU leave the FP64 form its registers,
// the FP32 form fits six.
template <typename T, bool ZS>
__global__ __launch_bounds__(TILE_THREADS, sizeof(T) == 8 ? 4 : 6) void k_site_elec_tiles(PairArgs<T> pa) {
  extern __shared__ __align__(16) unsigned char lds[];
  site_pairs_block<T, 1, ZS>(pa, xcd_block(blockIdx.x, gridDim.x), blockIdx.y, lds);
}

// The site-site sums of many frames with every pair once (no periodic
// images): ~25 KB of LDS in FP64; four workgroups per CU in FP64 (a fifth
// would spill registers in the pair loop), six in FP32.
template <typename T, bool ZS>
__global__ __launch_bounds__(TILE_THREADS, sizeof(T) == 8 ? 4 : 6) void k_site_pairs_n3(PairArgs<T> pa) {
  extern __shared__ __align__(16) unsigned char lds[];
  site_pairs_block<T, 2, ZS>(pa, xcd_block(blockIdx.x, gridDim.x), blockIdx.y, lds);
}

// clears n doubles (the atomic targets of the each-pair-once tiles)
__global__ __launch_bounds__(256) void k_zero(double* __restrict__ p, size_t n) {
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) p[i] = 0.0;
}

void launch_zero(hipStream_t s, double* p, size_t n) {
  if (n == 0) return;
  const size_t blocks = std::min<size_t>((n + 255) / 256, 8192);
  hipLaunchKernelGGL(k_zero, dim3((unsigned)blocks), dim3(256), 0, s, p, n);
}

template <typename T>
size_t site_pairs_lds(int tsplit, bool n3) {
  return tsplit > 0 ? (n3 ? PairN3Lds<T>::total : PairLds<T>::total) : 4 * wave_scratch_bytes<T>();
}


// The rest of the force on every site, once the electrode charges are known
// (one-frame launches; many-frame ones take k_site_forces_g16 below): pairs
// with the electrode Gaussians (g1), walked here; the k-space field,
// interpolated from the mesh with the site's B-spline weights (three lanes
// build the weights of one axis each in LDS, then the lanes run over the P^3
// points) or taken from the explicit Ewald sum; the site-site sum of
// k_site_pairs; the applied field.  One wavefront per site (or two, see
// below).  Workgroups from n_force_blocks on reduce the energies of their
// frame instead (they read nothing this kernel writes, so they run beside
// the force workgroups).
template <typename T, bool TWO>
__global__ __launch_bounds__(256) void k_site_forces(Cell cell, ElecSet<T> el, SiteSet<T> st,
                                                     ForceArgs<T> fa, int n_force_blocks, EnergyArgs en,
                                                     int walk_parts) {
  int bx = blockIdx.x, frame = blockIdx.y;
  if (gridDim.y > 1) {
    // many frames: each XCD takes a contiguous range of whole frames, so a
    // frame's field meshes are fetched into one L2 and its output lines are
    // filled there (one frame keeps the plain order: its targets differ in
    // cost, and contiguous ranges would load the XCDs unevenly)
    const int L = xcd_block(blockIdx.y * gridDim.x + blockIdx.x, gridDim.x * gridDim.y);
    frame = L / gridDim.x;
    bx = L - frame * gridDim.x;
  }
  if (bx >= n_force_blocks) {
    energy_block(en, frame);
    return;
  }
  __shared__ __align__(16) unsigned char scratch[4 * wave_scratch_bytes<T>()];
  __shared__ T wsp[4][3][MAX_ORDER];
  __shared__ int fsp[4][3];
  const int lane = threadIdx.x & (WAVE - 1);
  const int wv = threadIdx.x >> 6;
  // parts == 2: two wavefronts per site, each walking half of the site's
  // electrode candidates (the walk is the kernel's longest chain); the
  // second hands its sums to the first through LDS.  A wavefront past the
  // last site mirrors it, writes nothing and still meets the barrier.
  const int parts = walk_parts;
  const int part = parts == 2 ? (wv & 1) : 0;
  const int jw = parts == 2 ? bx * 2 + (wv >> 1) : bx * 4 + wv;
  if (parts == 1 && jw >= st.n) return;
  const bool live = jw < st.n;
  const int j = live ? jw : st.n - 1;
  T* ws = reinterpret_cast<T*>(scratch + wv * wave_scratch_bytes<T>());
  WaveQueue<T> Q;
  Q.bind(ws);
  int* rlo = reinterpret_cast<int*>(ws + 5 * WaveQueue<T>::CAP);
  int* rhi = rlo + 32;
  const size_t fo = (size_t)frame * st.n;
  const double xj = st.x[fo + j], yj = st.y[fo + j], zj = st.z[fo + j];
  const double qj = st.q[fo + j];
  // read now, used at the end: their latency overlaps the work in between
  const int orig = st.order[fo + j];
  const double* fp = fa.f_pair + (size_t)frame * 3 * st.n;
  const double fp0 = fp[j], fp1 = fp[st.n + j], fp2 = fp[2 * (size_t)st.n + j];
  const int cj = site_cell(cell, xj, yj, zj);
  // the electrode runs of the site's cell, read before the k-space part so
  // that their latency overlaps it
  const int nruns = elec_runs(el, cj, rlo, rhi);
  if (parts == 2) split_runs(rlo, rhi, nruns, part, 2);

  // ---- k-space field at the site
  T ea[3] = {0, 0, 0}, eb[3] = {0, 0, 0};
  if (fa.Ea && part == 0) {
    const int P = fa.mi.order;
    const int Kx = fa.mi.K[0], Ky = fa.mi.K[1], Kz = fa.mi.K[2], M = fa.mi.M;
    if (lane < 3) {
      const double xa = lane == 0 ? xj : (lane == 1 ? yj : zj);
      const double ih = lane == 0 ? fa.mi.invh[0] : (lane == 1 ? fa.mi.invh[1] : fa.mi.invh[2]);
      const int K = lane == 0 ? Kx : (lane == 1 ? Ky : Kz);
      T B[MAX_ORDER];
      int first = spline_triangle_d<T>(xa * ih, P, B);
      fsp[wv][lane] = ((first % K) + K) % K;
#pragma unroll
      for (int b = 0; b < MAX_ORDER; ++b)
        if (b < P) wsp[wv][lane][P - 1 - b] = B[b];
    }
    __builtin_amdgcn_wave_barrier();
    const int fx = fsp[wv][0], fy = fsp[wv][1], fz = fsp[wv][2];
    const T* Ef = fa.Ea + (size_t)frame * fa.Ea_frame_stride;
    // point t = (tz P + ty) P + tx: quotients through a float reciprocal,
    // exact for t < 7^3 (the fractions stay >= 1/98 away from integers)
    const float invP = 1.0f / (float)P, invP2 = 1.0f / (float)(P * P);
    for (int t = lane; t < P * P * P; t += WAVE) {
      const int tz = (int)(((float)t + 0.5f) * invP2);
      const int rz = t - tz * P * P;
      const int ty = (int)(((float)rz + 0.5f) * invP);
      const int tx = rz - ty * P;
      int ix = fx + tx; ix -= (ix >= Kx) ? Kx : 0;
      int iy = fy + ty; iy -= (iy >= Ky) ? Ky : 0;
      int iz = fz + tz; iz -= (iz >= Kz) ? Kz : 0;
      const int m = (iz * Ky + iy) * Kx + ix;
      const T w = wsp[wv][0][tx] * wsp[wv][1][ty] * wsp[wv][2][tz];
      ea[0] += w * Ef[m]; ea[1] += w * Ef[M + m]; ea[2] += w * Ef[2 * M + m];
      if (TWO) { eb[0] += w * fa.Eb[m]; eb[1] += w * fa.Eb[M + m]; eb[2] += w * fa.Eb[2 * M + m]; }
    }
  }
  if (fa.Esite && lane == 0 && part == 0) {
    const double* E = fa.Esite + (size_t)frame * 3 * st.n;
    ea[0] = (T)E[j]; ea[1] = (T)E[st.n + j]; ea[2] = (T)E[2 * st.n + j];
  }

  // ---- real space: electrode Gaussians (g1)
  T fr[3] = {0, 0, 0};
  T frb[3] = {0, 0, 0};
  {
  // the charges in the atoms' sorted order, loaded with their positions
  const double* qa = fa.qa_s + (size_t)frame * fa.qa_frame_stride;
  int n = 0;
  walk_runs(rlo, rhi, nruns,
            [&](int k, bool v) {
              ElecPartner<T> p{0, 0, 0, (T)0, (T)0};
              if (v) {
                p.x = el.x[k]; p.y = el.y[k]; p.z = el.z[k];
                p.a = (T)qa[k];
                if (TWO) p.b = (T)fa.qb_s[k];
              }
              return p;
            },
            [&](const ElecPartner<T>& p, int k, bool valid) {
              const T ca = p.a, cb = p.b;
              const Disp d = min_disp(cell, xj, yj, zj, p.x, p.y, p.z);
              for (int ix = -cell.img[0]; ix <= cell.img[0]; ++ix)
                for (int iy = -cell.img[1]; iy <= cell.img[1]; ++iy)
                  for (int iz = -cell.img[2]; iz <= cell.img[2]; ++iz) {
                    T dx, dy, dz;
                    const bool in = image_pair(cell, d, ix, iy, iz, fa.rc2, dx, dy, dz) && valid;
                    n = queue_push(Q, n, in, dx, dy, dz, ca, cb);
                    if (n >= WAVE) {
                      eval_g1<T, TWO>(Q, lane, fa.alpha, fa.eta, fr, frb);
                      n = queue_pop(Q, n);
                    }
                  }
            });
  if (lane < n) eval_g1<T, TWO>(Q, lane, fa.alpha, fa.eta, fr, frb);
  }

  // ---- reduce and write
  const double fpd[3] = {fp0, fp1, fp2};
  double F[3], FB[3];
  const T va[8] = {ea[0], ea[1], ea[2], fr[0], fr[1], fr[2], (T)0, (T)0};
  const T sa = wave_sum8(va);                 // lane 8k: total of va[k]
  T sb = (T)0;
  if (TWO) {
    const T vb[8] = {eb[0], eb[1], eb[2], frb[0], frb[1], frb[2], (T)0, (T)0};
    sb = wave_sum8(vb);
  }
  // walk sums of the site (both halves when split)
  double wa[3], wb[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    wa[d] = (double)read_lane(sa, 24 + 8 * d);
    wb[d] = TWO ? (double)read_lane(sb, 24 + 8 * d) : 0.0;
  }
  if (parts == 2) {
    __shared__ double half[2][6];
    const int sl = wv >> 1;
    if (part == 1 && lane == 0) {
#pragma unroll
      for (int d = 0; d < 3; ++d) { half[sl][d] = wa[d]; half[sl][3 + d] = wb[d]; }
    }
    __syncthreads();
    if (part == 1 || !live) return;
#pragma unroll
    for (int d = 0; d < 3; ++d) { wa[d] += half[sl][d]; wb[d] += half[sl][3 + d]; }
  }
#pragma unroll
  for (int d = 0; d < 3; ++d)
    F[d] = fa.out_scale * qj * ((double)read_lane(sa, 8 * d) + KE * (wa[d] + fpd[d]));
  if (TWO) {
#pragma unroll
    for (int d = 0; d < 3; ++d)
      FB[d] = fa.out_scale * qj * ((double)read_lane(sb, 8 * d) + KE * wb[d]);
  } else {
    FB[0] = FB[1] = FB[2] = 0.0;
  }
  F[2] += qj * fa.field;
  FB[2] += qj * fa.fieldb;
  if (fa.field_frame) F[2] += fa.out_scale * qj * fa.field_frame[frame];
  if (fa.f_comp) {
    if (lane < 6) {
      const double val = lane == 0 ? F[0] : lane == 1 ? F[1] : lane == 2 ? F[2]
                       : lane == 3 ? FB[0] : lane == 4 ? FB[1] : FB[2];
      fa.f_comp[((size_t)frame * 6 + lane) * st.n + orig] = val;
    }
    return;
  }
  double* fout = fa.f_out + (size_t)frame * fa.f_frame_stride;
  for (int v = lane; v < fa.n_dv; v += WAVE) {
    const double dv = fa.dv ? fa.dv[v] : 0.0;
    double* o = fout + (size_t)v * 3 * st.n;
    o[orig] = F[0] + dv * FB[0];
    o[st.n + orig] = F[1] + dv * FB[1];
    o[2 * st.n + orig] = F[2] + dv * FB[2];
  }
}

// The same when the pair tiles have already made the site-electrode sums
// (many frames): no walk is left, only the interpolation, so 16 lanes take a
// site, a wavefront four and a workgroup of G16_THREADS lanes 64 (larger
// workgroups measured faster than 256 or 512 lanes here).  Every lane evaluates the
// site's three weight sets itself and gathers the points t = sub, sub + 16,
// ... of the P^3 stencil; the 16 lanes then sum by butterfly shuffles.  A
// group past the last site mirrors it and writes nothing.
constexpr int G16_THREADS = 1024;
template <typename T, bool TWO>
__global__ __launch_bounds__(G16_THREADS) void k_site_forces_g16(SiteSet<T> st, ForceArgs<T> fa, int n_force_blocks,
                                                         EnergyArgs en) {
  int bx = blockIdx.x, frame = blockIdx.y;
  if (gridDim.y > 1) {
    // each XCD takes a contiguous range of whole frames (as k_site_forces)
    const int L = xcd_block(blockIdx.y * gridDim.x + blockIdx.x, gridDim.x * gridDim.y);
    frame = L / gridDim.x;
    bx = L - frame * gridDim.x;
  }
  if (bx >= n_force_blocks) {
    energy_block(en, frame);
    return;
  }
  const int sub = threadIdx.x & 15;
  const int jw = bx * (blockDim.x / 16) + (threadIdx.x >> 4);
  const bool live = jw < st.n;
  const int j = live ? jw : st.n - 1;
  const size_t fo = (size_t)frame * st.n;
  const double xj = st.x[fo + j], yj = st.y[fo + j], zj = st.z[fo + j];
  const double qj = st.q[fo + j];
  const int orig = st.order[fo + j];
  const double* fp = fa.f_pair + (size_t)frame * 3 * st.n;
  const double* fep = fa.f_elec + (size_t)frame * 6 * st.n;
  double fpd[3], fe[6];
#pragma unroll
  for (int d = 0; d < 3; ++d) fpd[d] = fp[(size_t)d * st.n + j];
#pragma unroll
  for (int u = 0; u < 6; ++u) fe[u] = fep[(size_t)u * st.n + j];

  T ea[3] = {0, 0, 0}, eb[3] = {0, 0, 0};
  if (fa.Ea) {
    const int P = fa.mi.order;
    const int Kx = fa.mi.K[0], Ky = fa.mi.K[1], Kz = fa.mi.K[2], M = fa.mi.M;
    T Bx[MAX_ORDER], By[MAX_ORDER], Bz[MAX_ORDER];
    int fx = spline_triangle_d<T>(xj * fa.mi.invh[0], P, Bx);
    int fy = spline_triangle_d<T>(yj * fa.mi.invh[1], P, By);
    int fz = spline_triangle_d<T>(zj * fa.mi.invh[2], P, Bz);
    fx = ((fx % Kx) + Kx) % Kx;
    fy = ((fy % Ky) + Ky) % Ky;
    fz = ((fz % Kz) + Kz) % Kz;
    const T* Ef = fa.Ea + (size_t)frame * fa.Ea_frame_stride;
    // point t = (tz P + ty) P + tx: quotients through a float reciprocal,
    // exact for t < 7^3 (the fractions stay >= 1/98 away from integers)
    const float invP = 1.0f / (float)P, invP2 = 1.0f / (float)(P * P);
    for (int t = sub; t < P * P * P; t += 16) {
      const int tz = (int)(((float)t + 0.5f) * invP2);
      const int rz = t - tz * P * P;
      const int ty = (int)(((float)rz + 0.5f) * invP);
      const int tx = rz - ty * P;
      // weight of stencil offset o along an axis: B[P - 1 - o] (selected,
      // not indexed, so that the weights stay in registers)
      T wx = 0, wy = 0, wz = 0;
#pragma unroll
      for (int b = 0; b < MAX_ORDER; ++b) {
        wx = (b == P - 1 - tx) ? Bx[b] : wx;
        wy = (b == P - 1 - ty) ? By[b] : wy;
        wz = (b == P - 1 - tz) ? Bz[b] : wz;
      }
      int ix = fx + tx; ix -= (ix >= Kx) ? Kx : 0;
      int iy = fy + ty; iy -= (iy >= Ky) ? Ky : 0;
      int iz = fz + tz; iz -= (iz >= Kz) ? Kz : 0;
      const int m = (iz * Ky + iy) * Kx + ix;
      const T w = wx * wy * wz;
      ea[0] += w * Ef[m]; ea[1] += w * Ef[M + m]; ea[2] += w * Ef[2 * M + m];
      if (TWO) { eb[0] += w * fa.Eb[m]; eb[1] += w * fa.Eb[M + m]; eb[2] += w * fa.Eb[2 * M + m]; }
    }
  } else if (fa.Esite && sub == 0) {
    const double* E = fa.Esite + (size_t)frame * 3 * st.n;
    ea[0] = (T)E[j]; ea[1] = (T)E[st.n + j]; ea[2] = (T)E[2 * st.n + j];
  }
#pragma unroll
  for (int off = 8; off > 0; off >>= 1) {
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      ea[d] += __shfl_xor(ea[d], off, 16);
      if (TWO) eb[d] += __shfl_xor(eb[d], off, 16);
    }
  }
  double F[3], FB[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    F[d] = fa.out_scale * qj * ((double)ea[d] + KE * (fpd[d] + fe[d]));
    FB[d] = TWO ? fa.out_scale * qj * ((double)eb[d] + KE * fe[3 + d]) : 0.0;
  }
  F[2] += qj * fa.field;
  FB[2] += qj * fa.fieldb;
  if (fa.field_frame) F[2] += fa.out_scale * qj * fa.field_frame[frame];
  if (!live) return;
  if (fa.f_comp) {
    if (sub < 6) {
      const double val = sub == 0 ? F[0] : sub == 1 ? F[1] : sub == 2 ? F[2]
                       : sub == 3 ? FB[0] : sub == 4 ? FB[1] : FB[2];
      fa.f_comp[((size_t)frame * 6 + sub) * st.n + orig] = val;
    }
    return;
  }
  double* fout = fa.f_out + (size_t)frame * fa.f_frame_stride;
  for (int v = sub; v < fa.n_dv; v += 16) {
    const double dv = fa.dv ? fa.dv[v] : 0.0;
    double* o = fout + (size_t)v * 3 * st.n;
    o[orig] = F[0] + dv * FB[0];
    o[st.n + orig] = F[1] + dv * FB[1];
    o[2 * st.n + orig] = F[2] + dv * FB[2];
  }
}

// The same when the field's inverse pass has interpolated plane by plane
// (epart, many frames, order 5): a thread per site sums its P slots of the
// six components (the frame's field and the static second field) and
// combines them with the pair sums as above.
template <typename T, bool TWO>
__global__ __launch_bounds__(256) void k_site_forces_sum(SiteSet<T> st, ForceArgs<T> fa, const T* __restrict__ epart,
                                                         int n_force_blocks, EnergyArgs en) {
  int bx = blockIdx.x, frame = blockIdx.y;
  if (gridDim.y > 1) {
    const int L = xcd_block(blockIdx.y * gridDim.x + blockIdx.x, gridDim.x * gridDim.y);
    frame = L / gridDim.x;
    bx = L - frame * gridDim.x;
  }
  if (bx >= n_force_blocks) {
    energy_block(en, frame);
    return;
  }
  const int j = bx * blockDim.x + threadIdx.x;
  if (j >= st.n) return;
  const size_t fo = (size_t)frame * st.n;
  const double qj = st.q[fo + j];
  const int orig = st.order[fo + j];
  const double* fp = fa.f_pair + (size_t)frame * 3 * st.n;
  const double* fep = fa.f_elec + (size_t)frame * 6 * st.n;
  const int P = fa.mi.order;
  const T* pp = epart + (size_t)frame * 6 * P * st.n + j;   // share (slot, component) at [(slot 6 + component) n]
  T e[6] = {0, 0, 0, 0, 0, 0};
  for (int sl = 0; sl < P; ++sl)
#pragma unroll
    for (int u = 0; u < 6; ++u) e[u] += pp[(size_t)(sl * 6 + u) * st.n];
  double F[3], FB[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    F[d] = fa.out_scale * qj * ((double)e[d] + KE * (fp[(size_t)d * st.n + j] + fep[(size_t)d * st.n + j]));
    FB[d] = TWO ? fa.out_scale * qj * ((double)e[3 + d] + KE * fep[(size_t)(3 + d) * st.n + j]) : 0.0;
  }
  F[2] += qj * fa.field;
  FB[2] += qj * fa.fieldb;
  if (fa.field_frame) F[2] += fa.out_scale * qj * fa.field_frame[frame];
  if (fa.f_comp) {
    double* o = fa.f_comp + (size_t)frame * 6 * st.n + orig;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      o[(size_t)d * st.n] = F[d];
      o[(size_t)(3 + d) * st.n] = FB[d];
    }
    return;
  }
  double* fout = fa.f_out + (size_t)frame * fa.f_frame_stride;
  for (int v = 0; v < fa.n_dv; ++v) {
    const double dv = fa.dv ? fa.dv[v] : 0.0;
    double* o = fout + (size_t)v * 3 * st.n;
    o[orig] = F[0] + dv * FB[0];
    o[st.n + orig] = F[1] + dv * FB[1];
    o[2 * st.n + orig] = F[2] + dv * FB[2];
  }
}

template <typename T>
void launch_site_pairs_t(hipStream_t s, int n_frames, const PairArgs<T>& pa) {
  if (pa.n_blocks == 0 || n_frames == 0) return;
  const dim3 grid(pa.n_blocks, n_frames);
  if (pa.tsplit > 0 && pa.fwd_n) {
    // site-site pairs once each (both ends take atomic adds), then the
    // site-electrode pairs
    launch_zero(s, pa.f_pair, (size_t)n_frames * 3 * pa.st.n);
    if (pa.u_site) launch_zero(s, pa.u_site, (size_t)n_frames * pa.st.n);
    const size_t lds = site_pairs_lds<T>(pa.tsplit, true);
    if (pa.zshift)
      hipLaunchKernelGGL(HIP_KERNEL_NAME(k_site_pairs_n3<T, true>), grid, dim3(TILE_THREADS), lds, s, pa);
    else
      hipLaunchKernelGGL(HIP_KERNEL_NAME(k_site_pairs_n3<T, false>), grid, dim3(TILE_THREADS), lds, s, pa);
    if (pa.f_elec && pa.zshift)
      hipLaunchKernelGGL(HIP_KERNEL_NAME(k_site_elec_tiles<T, true>), grid, dim3(TILE_THREADS), ElecTileLds<T>::total,
                         s, pa);
    else if (pa.f_elec)
      hipLaunchKernelGGL(HIP_KERNEL_NAME(k_site_elec_tiles<T, false>), grid, dim3(TILE_THREADS), ElecTileLds<T>::total,
                         s, pa);
  } else if (pa.tsplit > 0) {
    hipLaunchKernelGGL(k_site_pairs_tiles<T>, grid, dim3(TILE_THREADS), site_pairs_lds<T>(pa.tsplit, false), s, pa);
  } else {
    hipLaunchKernelGGL(k_site_pairs<T>, grid, dim3(TILE_THREADS), site_pairs_lds<T>(pa.tsplit, false), s, pa);
  }
}

template <typename T>
void launch_site_forces_t(hipStream_t s, int n_frames, const Cell& cell, const ElecSet<T>& el,
                          const SiteSet<T>& st, const ForceArgs<T>& fa, bool forces, const EnergyArgs* ea,
                          const T* epart) {
  // TWO: a second charge set; walk: the kernel walks the electrode atoms
  // itself (no site-electrode sums from the pair tiles; else k_site_forces_g16)
  const bool two = fa.Eb || fa.qb, walk = fa.f_elec == nullptr;
  // walking sites take two wavefronts each when all of them can be resident
  // at once (otherwise the second half of the sites would wait for slots
  // held by the first, whose halves wait for each other at a barrier)
  int parts = 1;
  if (walk && forces) {
    // wavefronts of the walking kernel a device holds (kept for devices 0-15,
    // queried on every call for others); a failed query leaves one
    // wavefront per site
    static int resident[16][2] = {};
    int dev = 0, r = 0;
    if (hipGetDevice(&dev) == hipSuccess) {
      int* kept = dev >= 0 && dev < 16 ? &resident[dev][two ? 1 : 0] : nullptr;
      r = kept ? *kept : 0;
      if (r <= 0) {
        int cus = 0, blocks = 0;
        const hipError_t e1 = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        const hipError_t e2 =
            two ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, k_site_forces<T, true>, 256, 0)
                : hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, k_site_forces<T, false>, 256, 0);
        r = (e1 == hipSuccess && e2 == hipSuccess) ? cus * blocks * 4 : 0;
        if (kept) *kept = r;
      }
    }
    parts = 2 * st.n * n_frames <= r ? 2 : 1;
  }
  const EnergyArgs e = ea ? *ea : EnergyArgs{};
  if (!walk && epart) {
    // a thread per site sums the interpolation's per-plane shares
    const int nfb = forces ? (st.n + 255) / 256 : 0;
    dim3 grid(nfb + (ea ? 1 : 0), n_frames);
    if (grid.x == 0) return;
    if (two)
      hipLaunchKernelGGL((k_site_forces_sum<T, true>), grid, dim3(256), 0, s, st, fa, epart, nfb, e);
    else
      hipLaunchKernelGGL((k_site_forces_sum<T, false>), grid, dim3(256), 0, s, st, fa, epart, nfb, e);
    return;
  }
  if (!walk) {
    // sixteen lanes per site
    const int nfb = forces ? (st.n + G16_THREADS / 16 - 1) / (G16_THREADS / 16) : 0;
    dim3 grid(nfb + (ea ? 1 : 0), n_frames);
    if (grid.x == 0) return;
    // energies alone: one frame's sums are short, 256 lanes reduce them sooner
    const dim3 block(nfb ? G16_THREADS : 256);
    if (two)
      hipLaunchKernelGGL((k_site_forces_g16<T, true>), grid, block, 0, s, st, fa, nfb, e);
    else
      hipLaunchKernelGGL((k_site_forces_g16<T, false>), grid, block, 0, s, st, fa, nfb, e);
    return;
  }
  const int nfb = forces ? (parts == 2 ? (st.n + 1) / 2 : (st.n + 3) / 4) : 0;
  dim3 grid(nfb + (ea ? 1 : 0), n_frames);
  if (grid.x == 0) return;
  if (two)
    hipLaunchKernelGGL((k_site_forces<T, true>), grid, dim3(256), 0, s, cell, el, st, fa, nfb, e, parts);
  else
    hipLaunchKernelGGL((k_site_forces<T, false>), grid, dim3(256), 0, s, cell, el, st, fa, nfb, e, parts);
}

// explicit instantiations used by api.cpp
template void launch_real_b_t<double>(hipStream_t, int, const RealBArgs<double>&);
template void launch_real_b_t<float>(hipStream_t, int, const RealBArgs<float>&);
template void launch_site_pairs_t<double>(hipStream_t, int, const PairArgs<double>&);
template void launch_site_pairs_t<float>(hipStream_t, int, const PairArgs<float>&);
template size_t site_pairs_lds<double>(int, bool);
template size_t site_pairs_lds<float>(int, bool);
template void launch_site_forces_t<double>(hipStream_t, int, const Cell&, const ElecSet<double>&,
                                           const SiteSet<double>&, const ForceArgs<double>&, bool,
                                           const EnergyArgs*, const double*);
template void launch_site_forces_t<float>(hipStream_t, int, const Cell&, const ElecSet<float>&,
                                          const SiteSet<float>&, const ForceArgs<float>&, bool,
                                          const EnergyArgs*, const float*);

}  // namespace cpm
