// 3D FFT of the PPPM mesh and the Green's-function step, hand-written for
// the small meshes of this path (a few 10^4 points per frame).
//
// Mixed-radix (2, 3, 4, 5) Stockham autosort transform, staged entirely in
// LDS: a stage of radix R reads R points N/R apart, applies the twiddles
// e^{-+2 pi i r (j mod Ns)/(Ns R)}, does a length-R DFT and writes R points
// Ns apart into the other buffer (Ns = product of the radices done so far);
// after the last stage the data are in natural order.  Twiddles come from a
// per-length table of e^{-2 pi i t / N}.
//
// The 3D transform of one frame is two kernels:
//   * k_fft_xy: one workgroup per z-plane (Kx x Ky points) transforms x and
//     y (forward from a real mesh, or inverse to real output meshes);
//   * k_fft_z:  one workgroup per (y, block of x columns) transforms along
//     z, multiplies by the influence function (and by -i k for the field,
//     ik differentiation), transforms back along z, and writes in place.
// A round trip real mesh -> potential (or field) mesh is therefore
// fft_xy(forward) -> fft_z -> fft_xy(inverse).  Mesh layout [z][y][x].
#include <cstdio>
#include <cstdlib>

#include "common.h"
#include "lj.h"
#include "bin.h"
#include "pairs.h"

namespace cpm {

template <typename T2> struct CT;
template <> struct CT<double2> { using R = double; };
template <> struct CT<float2> { using R = float; };

template <typename T2> __device__ __forceinline__ T2 cadd(T2 a, T2 b) { return T2{a.x + b.x, a.y + b.y}; }
template <typename T2> __device__ __forceinline__ T2 csub(T2 a, T2 b) { return T2{a.x - b.x, a.y - b.y}; }
template <typename T2> __device__ __forceinline__ T2 cmul(T2 a, T2 b) {
  return T2{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
template <typename T2, typename R> __device__ __forceinline__ T2 cscale(T2 a, R s) { return T2{a.x * s, a.y * s}; }
// multiply by sigma * i
template <typename T2> __device__ __forceinline__ T2 cmul_si(T2 a, int sigma) {
  return sigma > 0 ? T2{-a.y, a.x} : T2{a.y, -a.x};
}

// X[m] = sum_r v[r] exp(sigma 2 pi i r m / R), R in {2,3,4,5}; R is a
// compile-time constant so v stays in registers
template <int R, typename T2>
__device__ __forceinline__ void small_dft(T2* v, int sigma) {
  using Rl = typename CT<T2>::R;
  if constexpr (R == 2) {
    T2 a = cadd(v[0], v[1]), b = csub(v[0], v[1]);
    v[0] = a; v[1] = b;
  } else if constexpr (R == 4) {
    T2 s02 = cadd(v[0], v[2]), d02 = csub(v[0], v[2]);
    T2 s13 = cadd(v[1], v[3]), d13 = cmul_si(csub(v[1], v[3]), sigma);
    v[0] = cadd(s02, s13); v[2] = csub(s02, s13);
    v[1] = cadd(d02, d13); v[3] = csub(d02, d13);
  } else if constexpr (R == 3) {
    const Rl h = (Rl)0.86602540378443865;    // sqrt(3)/2
    T2 s = cadd(v[1], v[2]);
    T2 d = cmul_si(cscale(csub(v[1], v[2]), h), sigma);
    T2 m = csub(v[0], cscale(s, (Rl)0.5));
    v[0] = cadd(v[0], s);
    v[1] = cadd(m, d);
    v[2] = csub(m, d);
  } else {  // R == 5
    const Rl c1 = (Rl)0.30901699437494742, c2 = (Rl)-0.80901699437494742;
    const Rl s1 = (Rl)0.95105651629515357, s2 = (Rl)0.58778525229247313;
    T2 s14 = cadd(v[1], v[4]), d14 = csub(v[1], v[4]);
    T2 s23 = cadd(v[2], v[3]), d23 = csub(v[2], v[3]);
    T2 a1 = cadd(v[0], cadd(cscale(s14, c1), cscale(s23, c2)));
    T2 a2 = cadd(v[0], cadd(cscale(s14, c2), cscale(s23, c1)));
    T2 b1 = cmul_si(cadd(cscale(d14, s1), cscale(d23, s2)), sigma);
    T2 b2 = cmul_si(csub(cscale(d14, s2), cscale(d23, s1)), sigma);
    v[0] = cadd(v[0], cadd(s14, s23));
    v[1] = cadd(a1, b1); v[4] = csub(a1, b1);
    v[2] = cadd(a2, b2); v[3] = csub(a2, b2);
  }
}

template <typename T2> __device__ __forceinline__ const T2* twiddles(const FFTPlan1D& p);
template <> __device__ __forceinline__ const double2* twiddles<double2>(const FFTPlan1D& p) { return p.tw; }
template <> __device__ __forceinline__ const float2* twiddles<float2>(const FFTPlan1D& p) { return p.twf; }

// Transform nlines lines of length p.n held in LDS buffer a (element stride
// es, line stride ls), ping-ponging with b; tw is the plan's twiddle table
// staged in LDS.  Returns the buffer holding the result.  sigma = -1
// forward, +1 inverse (unnormalised).
// Copy the twiddle table of plan p into LDS (the caller synchronises).
template <typename T2>
__device__ __forceinline__ void load_twiddles(const FFTPlan1D& p, T2* dst) {
  const T2* src = twiddles<T2>(p);
  for (int i = threadIdx.x; i < p.n; i += blockDim.x) dst[i] = src[i];
}

// floor(u / d) for small non-negative u and d (u + d below 2^21) from a
// single-precision reciprocal rd = 1/d: (u + 1/2) / d lies at least 1/(2d)
// from an integer, farther than the product's rounding error can move it.
// Three operations instead of an integer division's twenty on the
// dependent chain of a stage.
__device__ __forceinline__ int div_small(int u, float rd) { return (int)(((float)u + 0.5f) * rd); }

// One Stockham stage of radix R over nlines lines (see the file comment) of
// each of nplanes planes pstride apart.
template <int R, typename T2>
__device__ __forceinline__ void fft_stage(const T2* src, T2* dst, int N, int Ns, int nlines, int es, int ls,
                                          const T2* tw, int sigma, int nplanes, int pstride) {
  const int nb = N / R;
  const int tstep = N / (Ns * R);
  const int lnb = nlines * nb;
  const float rnb = 1.0f / (float)nb, rns = 1.0f / (float)Ns, rlnb = 1.0f / (float)lnb;
  for (int u = threadIdx.x; u < nplanes * lnb; u += blockDim.x) {
    const int pl = nplanes > 1 ? div_small(u, rlnb) : 0;
    const int ul = u - pl * lnb;
    const int line = div_small(ul, rnb);
    const int j = ul - line * nb;
    const T2* in = src + pl * pstride + line * ls;
    T2* out = dst + pl * pstride + line * ls;
    T2 v[R];
#pragma unroll
    for (int r = 0; r < R; ++r) v[r] = in[(j + r * nb) * es];
    const int jq = div_small(j, rns);
    const int k = j - jq * Ns;
    if (Ns > 1) {
#pragma unroll
      for (int r = 1; r < R; ++r) {
        T2 w = tw[r * k * tstep];
        if (sigma > 0) w.y = -w.y;
        v[r] = cmul(v[r], w);
      }
    }
    small_dft<R>(v, sigma);
    const int base = jq * Ns * R + k;
#pragma unroll
    for (int r = 0; r < R; ++r) out[(base + r * Ns) * es] = v[r];
  }
}

template <typename T2>
__device__ T2* fft_lines(T2* a, T2* b, const FFTPlan1D& p, const T2* tw, int nlines, int es, int ls, int sigma,
                         int nplanes = 1, int pstride = 0) {
  const int N = p.n;
  T2* src = a;
  T2* dst = b;
  int Ns = 1;
  for (int f = 0; f < p.nfac; ++f) {
    const int R = p.fac[f];
    switch (R) {
      case 2: fft_stage<2>(src, dst, N, Ns, nlines, es, ls, tw, sigma, nplanes, pstride); break;
      case 3: fft_stage<3>(src, dst, N, Ns, nlines, es, ls, tw, sigma, nplanes, pstride); break;
      case 4: fft_stage<4>(src, dst, N, Ns, nlines, es, ls, tw, sigma, nplanes, pstride); break;
      default: fft_stage<5>(src, dst, N, Ns, nlines, es, ls, tw, sigma, nplanes, pstride); break;
    }
    __syncthreads();
    T2* t = src; src = dst; dst = t;
    Ns *= R;
  }
  return src;
}

// Lines of at most DFT_DIRECT_MAX points: the plane transforms are bound
// by the latency of their dependent stages (a thread's butterfly of one
// stage is a chain of index arithmetic, two LDS reads, the twiddle products
// and the writes, then a barrier), so short lines are summed directly
// instead: thread (line, k) forms X_k = sum_n x_n e^{-+2 pi i n k / N} from
// the same twiddle table, its index advanced by k modulo N.  One pass and
// one barrier per direction; the result lands in b in natural order.  Taken
// only while every thread of the plane has a single task (a second round of
// N-term sums costs more than the stages it saves, as at 36 x 36).
constexpr int DFT_DIRECT_MAX = 32;
// points per LDS round trip of the direct sum (even)
constexpr int DFT_CHUNK = 6;

// threads of a plane workgroup: one-frame launches use XY_THREADS (an
// 18 x 18 plane is then one direct-sum task per thread), many-frame
// launches XY_THREADS_MANY (more workgroups per CU for the Stockham stages)
constexpr int XY_THREADS = 512;
constexpr int XY_THREADS_MANY = 256;
// planes per workgroup of many-frame x-y launches (measured over 2, 3 and 4
// at 18 x 18: FP64 best at 3, FP32 at 4)
template <typename T2> constexpr int xy_planes_many() { return sizeof(T2) == 16 ? 3 : 4; }

template <typename T2>
__device__ T2* dft_lines(const T2* a, T2* b, int N, const T2* tw, int nlines, int es, int ls, int sigma) {
  using T = typename CT<T2>::R;
  const T sg = sigma > 0 ? (T)-1 : (T)1;             // conjugate the table for the inverse
  // even N: a thread gives X_k and X_{k+N/2} (k < N/2) from the sums E and O
  // over even and odd n, as e^{-+2 pi i n (k + N/2) / N} = (-1)^n e^{-+2 pi i n k / N}:
  // X_k = E + O, X_{k+N/2} = E - O, every point and twiddle read serving two
  // outputs; odd N: one output per thread
  const int half = (N & 1) ? N : N / 2;
  const float rh = 1.0f / (float)half;
  for (int u = threadIdx.x; u < nlines * half; u += blockDim.x) {
    const int line = div_small(u, rh);
    const int k = u - line * half;
    const T2* in = a + line * ls;
    // DFT_CHUNK points and their twiddles are read together (one LDS round
    // trip per chunk); the chunk starts at an even n, so its even entries
    // go to E and its odd ones to O
    T er = 0, ei = 0, orr = 0, oi = 0;
    int t = 0;
    for (int n0 = 0; n0 < N; n0 += DFT_CHUNK) {
      T2 xv[DFT_CHUNK], wv[DFT_CHUNK];
#pragma unroll
      for (int c = 0; c < DFT_CHUNK; ++c) {
        xv[c] = T2{0, 0};
        wv[c] = T2{0, 0};
        if (n0 + c < N) {
          xv[c] = in[(n0 + c) * es];
          wv[c] = tw[t];
          t += k; t -= (t >= N) ? N : 0;
        }
      }
#pragma unroll
      for (int c = 0; c < DFT_CHUNK; c += 2) {
        const T wy0 = sg * wv[c].y, wy1 = sg * wv[c + 1].y;
        er += xv[c].x * wv[c].x - xv[c].y * wy0;
        ei += xv[c].x * wy0 + xv[c].y * wv[c].x;
        orr += xv[c + 1].x * wv[c + 1].x - xv[c + 1].y * wy1;
        oi += xv[c + 1].x * wy1 + xv[c + 1].y * wv[c + 1].x;
      }
    }
    T2* out = b + line * ls;
    out[k * es] = T2{er + orr, ei + oi};
    if (half != N) out[(k + half) * es] = T2{er - orr, ei - oi};
  }
  __syncthreads();
  return b;
}

// One direction of a plane: the direct sum for short lines in the one-frame
// launches (direct), else the Stockham stages, which do fewer operations and
// serve the many-frame launches better, where throughput counts
template <typename T2>
__device__ T2* plane_lines(T2* a, T2* b, const FFTPlan1D& p, const T2* tw, int nlines, int es, int ls, int sigma,
                           bool direct, int nplanes = 1, int pstride = 0) {
  if (direct && nplanes == 1 && p.n <= DFT_DIRECT_MAX && nlines * ((p.n & 1) ? p.n : p.n / 2) <= (int)blockDim.x)
    return dft_lines(a, b, p.n, tw, nlines, es, ls, sigma);
  return fft_lines(a, b, p, tw, nlines, es, ls, sigma, nplanes, pstride);
}

// One Stockham stage of radix R over one contiguous line, by the lanes of
// one wavefront (no workgroup barrier; the caller orders the stages)
template <int R, typename T2>
__device__ __forceinline__ void fft_stage_w(const T2* src0, T2* dst0, int N, int Ns, const T2* tw, int sigma, int nl,
                                            int lstride) {
  const int lane = threadIdx.x & (WAVE - 1);
  const int nb = N / R;
  const int tstep = N / (Ns * R);
  const float rns = 1.0f / (float)Ns, rnb = 1.0f / (float)nb;
  for (int u = lane; u < nl * nb; u += WAVE) {
    const int l = nl > 1 ? div_small(u, rnb) : 0;
    const int j = u - l * nb;
    const T2* src = src0 + l * lstride;
    T2* dst = dst0 + l * lstride;
    T2 v[R];
#pragma unroll
    for (int r = 0; r < R; ++r) v[r] = src[j + r * nb];
    const int jq = div_small(j, rns);
    const int k = j - jq * Ns;
    if (Ns > 1) {
#pragma unroll
      for (int r = 1; r < R; ++r) {
        T2 w = tw[r * k * tstep];
        if (sigma > 0) w.y = -w.y;
        v[r] = cmul(v[r], w);
      }
    }
    small_dft<R>(v, sigma);
    const int base = jq * Ns * R + k;
#pragma unroll
    for (int r = 0; r < R; ++r) dst[base + r * Ns] = v[r];
  }
}

// Transform nl lines of p.n points (lstride apart) held in a wavefront's own
// LDS buffer a, ping-ponging with b; the stages are ordered by wavefront
// barriers only (a wavefront's LDS operations complete in order).  Returns
// the buffer holding the result.
template <typename T2>
__device__ T2* fft_line_w(T2* a, T2* b, const FFTPlan1D& p, const T2* tw, int sigma, int nl = 1, int lstride = 0) {
  const int N = p.n;
  T2* src = a;
  T2* dst = b;
  int Ns = 1;
  __builtin_amdgcn_wave_barrier();
  for (int f = 0; f < p.nfac; ++f) {
    const int R = p.fac[f];
    switch (R) {
      case 2: fft_stage_w<2>(src, dst, N, Ns, tw, sigma, nl, lstride); break;
      case 3: fft_stage_w<3>(src, dst, N, Ns, tw, sigma, nl, lstride); break;
      case 4: fft_stage_w<4>(src, dst, N, Ns, tw, sigma, nl, lstride); break;
      default: fft_stage_w<5>(src, dst, N, Ns, tw, sigma, nl, lstride); break;
    }
    __builtin_amdgcn_wave_barrier();
    T2* t = src; src = dst; dst = t;
    Ns *= R;
  }
  return src;
}

// ------------------------------------------- site interpolation by plane

// The field planes z .. z + np - 1 of one frame are in E (part 0: Ex in .x,
// Ey in .y; part 1: Ez in .x); `free` holds as many planes.  Every site whose
// stencil reaches one of them gets, per reached plane, its partial sums of
// the frame's field and of the static field Eb (InterpArgs).  B-splines of
// order 5 (the launch takes this path only then), with the stencil start and
// the weights of the site-force gather (the same spline_triangle_d calls on
// the same coordinates); a site's stencil covers planes first .. first + 4
// (mod K_z), i.e. scaled z within 5/2 of the plane, so the candidates are the
// sites of the binning's z layers that meet that distance (plus 1e-6 nm for
// rounding, far above it and far below a layer).  A thread takes a site, its
// planes one after the other and their rows one after the other (few
// registers: the x-y pass it rides in keeps its occupancy).
// What plane_interp needs from global memory, loaded before the transform so
// that its latency passes under the transform's stages (which wait on LDS
// only): the candidate ranges, this thread's first candidate and its
// position, and this thread's first four points of the static field.
template <typename T, typename T2>
struct InterpPre {
  int lo0, n0, lo1, n_cand;     // candidates: n0 sites from lo0, then from lo1
  int j;                        // this thread's first candidate (cell-sorted index), or -1
  double x, y, z;               // its wrapped position
  T2 eb[4];                     // static field at plane points threadIdx.x + k blockDim.x
};

template <typename T, typename T2>
__device__ __forceinline__ void interp_pre(const InterpArgs<T>& ia, int frame, int part, int z0, int np, int NP,
                                           InterpPre<T, T2>& pre) {
  constexpr int P = 5;
  const size_t M = ia.mi.M;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int i = threadIdx.x + k * blockDim.x;
    const size_t m = (size_t)z0 * NP + i;
    pre.eb[k] = T2{(T)0, (T)0};
    if (ia.Eb && i < np * NP) pre.eb[k] = part ? T2{ia.Eb[2 * M + m], (T)0} : T2{ia.Eb[m], ia.Eb[M + m]};
  }
  // candidate sites: the z layers that meet scaled z within P/2 of the
  // group's planes (a margin of 1e-6 nm for rounding), as one or two ranges
  // of the cell-sorted sites
  const double h = ia.mi.h[2];
  const int la = (int)floor(((z0 - 0.5 * P) * h - 1e-6) * ia.inv_wz);
  const int lb = (int)floor(((z0 + np - 1 + 0.5 * P) * h + 1e-6) * ia.inv_wz);
  const int* cs = ia.cell_start + (size_t)frame * (ia.n_cells + 1);
  int lo0 = 0, hi0 = ia.n, lo1 = 0, hi1 = 0;
  if (lb - la + 1 < ia.ncz) {
    const int a = ((la % ia.ncz) + ia.ncz) % ia.ncz, b = ((lb % ia.ncz) + ia.ncz) % ia.ncz;
    if (a <= b) { lo0 = cs[a * ia.nxy]; hi0 = cs[(b + 1) * ia.nxy]; }
    else { lo0 = cs[a * ia.nxy]; hi0 = ia.n; lo1 = 0; hi1 = cs[(b + 1) * ia.nxy]; }
  }
  pre.lo0 = lo0; pre.n0 = hi0 - lo0; pre.lo1 = lo1; pre.n_cand = pre.n0 + (hi1 - lo1);
  pre.j = -1;
  const int c = threadIdx.x;
  if (c < pre.n_cand) {
    const int j = c < pre.n0 ? lo0 + c : lo1 + (c - pre.n0);
    const size_t o = (size_t)frame * ia.n + j;
    pre.j = j;
    pre.x = ia.sx[o]; pre.y = ia.sy[o]; pre.z = ia.sz[o];
  }
}

template <typename T, typename T2>
__device__ void plane_interp(const InterpArgs<T>& ia, const InterpPre<T, T2>& pre, const T2* E, T2* free, int frame,
                             int part, int z0, int np, int Kx, int Ky, int Kz) {
  constexpr int P = 5;
  const int NP = Kx * Ky;
  const size_t M = ia.mi.M;
  // the static field's planes beside the frame's
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int i = threadIdx.x + k * blockDim.x;
    if (i < np * NP) free[i] = pre.eb[k];
  }
  for (int i = threadIdx.x + 4 * blockDim.x; i < np * NP; i += blockDim.x) {
    const size_t m = (size_t)z0 * NP + i;
    T2 v = T2{(T)0, (T)0};
    if (ia.Eb) v = part ? T2{ia.Eb[2 * M + m], (T)0} : T2{ia.Eb[m], ia.Eb[M + m]};
    free[i] = v;
  }
  __syncthreads();
  const size_t fo = (size_t)frame * ia.n;
  for (int c = threadIdx.x; c < pre.n_cand; c += blockDim.x) {
    const bool first = c == (int)threadIdx.x;
    const int j = first ? pre.j : (c < pre.n0 ? pre.lo0 + c : pre.lo1 + (c - pre.n0));
    const double zj = first ? pre.z : ia.sz[fo + j];
    const double uz = zj * ia.mi.invh[2];
    // the stencil start as spline_triangle_d takes it (the weights only for
    // the sites kept)
    int fz = (int)floor(uz - 0.5 * P) + 1;
    fz = ((fz % Kz) + Kz) % Kz;
    int d0 = z0 - fz;
    d0 += d0 < 0 ? Kz : 0;               // slot of plane z0; plane z0 + p has slot d0 + p (mod Kz)
    int d1 = d0 + np - 1;
    d1 -= d1 >= Kz ? Kz : 0;
    if (d0 >= P && d1 >= P && d1 >= d0) continue;     // no plane of the group within the stencil
    T Bx[MAX_ORDER], By[MAX_ORDER], Bz[MAX_ORDER];
    spline_triangle_d<T, 5>(uz, P, Bz);
    int fx = spline_triangle_d<T, 5>((first ? pre.x : ia.sx[fo + j]) * ia.mi.invh[0], P, Bx);
    int fy = spline_triangle_d<T, 5>((first ? pre.y : ia.sy[fo + j]) * ia.mi.invh[1], P, By);
    fx = ((fx % Kx) + Kx) % Kx;
    fy = ((fy % Ky) + Ky) % Ky;
    T* out = ia.part + (size_t)frame * 6 * P * ia.n + j;      // share (slot, component) at [(slot 6 + component) n]
#pragma unroll 1
    for (int p = 0; p < np; ++p) {
      int sl = d0 + p;
      sl -= sl >= Kz ? Kz : 0;
      if (sl >= P) continue;
      T ax = 0, ay = 0, bx = 0, by = 0;
#pragma unroll 1
      for (int ty = 0; ty < P; ++ty) {
        // offset o takes weight B[P - 1 - o] (selected: the weights stay in registers)
        const T wy = ty == 0 ? By[4] : ty == 1 ? By[3] : ty == 2 ? By[2] : ty == 3 ? By[1] : By[0];
        int iy = fy + ty;
        iy -= iy >= Ky ? Ky : 0;
        const T2* er = E + p * NP + iy * Kx;
        const T2* fr = free + p * NP + iy * Kx;
#pragma unroll
        for (int tx = 0; tx < P; ++tx) {
          int ix = fx + tx;
          ix -= ix >= Kx ? Kx : 0;
          const T w = Bx[P - 1 - tx] * wy;
          const T2 e = er[ix];
          ax += w * e.x; ay += w * e.y;
        }
#pragma unroll
        for (int tx = 0; tx < P; ++tx) {
          int ix = fx + tx;
          ix -= ix >= Kx ? Kx : 0;
          const T w = Bx[P - 1 - tx] * wy;
          const T2 f = fr[ix];
          bx += w * f.x; by += w * f.y;
        }
      }
      const T wz = sl == 0 ? Bz[4] : sl == 1 ? Bz[3] : sl == 2 ? Bz[2] : sl == 3 ? Bz[1] : Bz[0];
      T* o6 = out + (size_t)sl * 6 * ia.n;
      if (part == 0) {
        o6[0] = wz * ax; o6[(size_t)ia.n] = wz * ay;
        o6[3 * (size_t)ia.n] = wz * bx; o6[4 * (size_t)ia.n] = wz * by;
      } else {
        o6[2 * (size_t)ia.n] = wz * ax;
        o6[5 * (size_t)ia.n] = wz * bx;
      }
    }
  }
}

// ------------------------------------------------------------------ x-y pass

// mode 0: forward, real input -> complex output
// mode 1: inverse, complex input -> real part to out_re (and imaginary part to out_im if given)
// split (mode 1 only): blockIdx.y = 2 frame + part; part 1 transforms in_c2
// into out_re2 (real part only), part 0 in_c as above
// DIRECT: a one-frame launch (short lines are summed directly, see dft_lines)
// INTERP (many frames, the field's split inverse): instead of writing the
// field planes, interpolate them at the sites (plane_interp)
// zl (many frames): transform only the n_zl planes listed (ascending), PL
// list entries per workgroup, or every plane if nullptr
// (the body; k_fft_xy and k_fft_xy_many below are its launches)
template <typename T, typename T2, bool DIRECT, int PL, bool INTERP>
__device__ __forceinline__ void fft_xy_body(const FFTPlan1D& px, const FFTPlan1D& py, int Kz, int mode,
                                            const T* __restrict__ in_re, const T2* __restrict__ in_c,
                                            T2* __restrict__ out_c, T* __restrict__ out_re,
                                            T* __restrict__ out_im, size_t out_re_stride, int split,
                                            const T2* __restrict__ in_c2, T* __restrict__ out_re2,
                                            const int* __restrict__ zl, int n_zl, const InterpArgs<T>& ia) {
  extern __shared__ __align__(16) unsigned char smem[];
  // PL consecutive planes per workgroup (many frames: the stages of several
  // 18-point planes fill a 256-thread workgroup better than one; one plane
  // where that many do not fit in LDS), held one after the other in A and in B
  static_assert(!DIRECT || PL == 1, "a one-frame launch takes one plane per workgroup");
  const int Kx = px.n, Ky = py.n, NP = Kx * Ky;
  T2* A = reinterpret_cast<T2*>(smem);
  T2* B = A + PL * NP;
  T2* twx = B + PL * NP;
  T2* twy = twx + Kx;
  load_twiddles(px, twx);
  load_twiddles(py, twy);
  if (DIRECT || INTERP) zl = nullptr;                       // (a plane list only in plain many-frame launches)
  const int z = blockIdx.x * PL;                            // first plane (or list entry)
  const int np = min(PL, (zl ? n_zl : Kz) - z);
  const int part = split ? (int)(blockIdx.y & 1) : 0;
  const int frame = split ? (int)(blockIdx.y >> 1) : (int)blockIdx.y;
  if (part) { in_c = in_c2; out_re = out_re2; out_im = nullptr; }
  const size_t off = ((size_t)frame * Kz + z) * NP;         // the workgroup's planes are contiguous
  // mesh offset (within the frame) of the workgroup's point i: listed planes
  // need not be contiguous
  auto listed = [&](int i) -> size_t {
    const int p = i / NP;
    return (size_t)zl[z + p] * NP + (i - p * NP);
  };
  if (zl) {
    const size_t fo = (size_t)frame * Kz * NP;
    if (mode == 0) {
      for (int i = threadIdx.x; i < np * NP; i += blockDim.x) A[i] = T2{in_re[fo + listed(i)], (T)0};
    } else {
      for (int i = threadIdx.x; i < np * NP; i += blockDim.x) A[i] = in_c[fo + listed(i)];
    }
  } else if (mode == 0) {
    for (int i = threadIdx.x; i < np * NP; i += blockDim.x) A[i] = T2{in_re[off + i], (T)0};
  } else {
    for (int i = threadIdx.x; i < np * NP; i += blockDim.x) A[i] = in_c[off + i];
  }
  InterpPre<T, T2> pre;
  if (INTERP) interp_pre<T, T2>(ia, frame, part, z, np, NP, pre);
  __syncthreads();
  const int sigma = mode == 0 ? -1 : 1;
  T2* r1 = plane_lines(A, B, px, twx, Ky, 1, Kx, sigma, DIRECT, np, NP);        // along x
  T2* o1 = (r1 == A) ? B : A;
  T2* r2 = plane_lines(r1, o1, py, twy, Kx, Kx, 1, sigma, DIRECT, np, NP);      // along y
  if (INTERP) {
    plane_interp<T, T2>(ia, pre, r2, (r2 == A) ? B : A, frame, part, z, np, Kx, Ky, Kz);
  } else if (zl) {
    const size_t fo = (size_t)frame * Kz * NP, ro = (size_t)frame * out_re_stride;
    for (int i = threadIdx.x; i < np * NP; i += blockDim.x) {
      const size_t m = listed(i);
      if (mode == 0) {
        out_c[fo + m] = r2[i];
      } else {
        out_re[ro + m] = r2[i].x;
        if (out_im) out_im[ro + m] = r2[i].y;
      }
    }
  } else if (mode == 0) {
    for (int i = threadIdx.x; i < np * NP; i += blockDim.x) out_c[off + i] = r2[i];
  } else {
    const size_t ro = (size_t)frame * out_re_stride + (size_t)z * NP;
    for (int i = threadIdx.x; i < np * NP; i += blockDim.x) {
      out_re[ro + i] = r2[i].x;
      if (out_im) out_im[ro + i] = r2[i].y;
    }
  }
}

// one frame (DIRECT) or many frames with every plane
template <typename T, typename T2, bool DIRECT, int PL>
__global__ __launch_bounds__(XY_THREADS) void k_fft_xy(FFTPlan1D px, FFTPlan1D py, int Kz, int mode,
                                                const T* __restrict__ in_re, const T2* __restrict__ in_c,
                                                T2* __restrict__ out_c, T* __restrict__ out_re,
                                                T* __restrict__ out_im, size_t out_re_stride, int split,
                                                const T2* __restrict__ in_c2, T* __restrict__ out_re2) {
  fft_xy_body<T, T2, DIRECT, PL, false>(px, py, Kz, mode, in_re, in_c, out_c, out_re, out_im, out_re_stride, split,
                                        in_c2, out_re2, nullptr, 0, InterpArgs<T>{});
}

// many frames: a plane list (zl) or the interpolation at the sites (INTERP)
template <typename T, typename T2, int PL, bool INTERP>
__global__ __launch_bounds__(INTERP ? XY_THREADS_MANY : XY_THREADS, INTERP ? 5 : 1) void k_fft_xy_many(
    FFTPlan1D px, FFTPlan1D py, int Kz, int mode, const T* __restrict__ in_re, const T2* __restrict__ in_c,
    T2* __restrict__ out_c, T* __restrict__ out_re, T* __restrict__ out_im, size_t out_re_stride, int split,
    const T2* __restrict__ in_c2, T* __restrict__ out_re2, const int* __restrict__ zl, int n_zl, InterpArgs<T> ia) {
  fft_xy_body<T, T2, false, PL, INTERP>(px, py, Kz, mode, in_re, in_c, out_c, out_re, out_im, out_re_stride, split,
                                        in_c2, out_re2, zl, n_zl, ia);
}

// ------------------------------------------------- spread fused with x-y

// Forward x-y transform of one z-plane of the electrolyte charge mesh, whose
// real values are first assembled in LDS.  The plane's workgroup scans every
// site (wrapped into the box as the binning does), stages those whose
// B-spline stencil reaches the plane in per-wavefront lists, and each staged
// site adds its P x P in-plane contributions with LDS atomics, its weights
// computed on the spot.  The scan needs no cell list, so the binning of the
// same frame runs as one more workgroup of this launch (index n_planes).
// The assembled plane is also written to rho_out (the charge mesh, for
// inspection), then transformed as in k_fft_xy.  ONE: a one-frame launch
// (1024 threads; the binning keeps its sites in registers, the planes use
// the direct sum).  P5: B-splines of order 5 (else any other order).  SPL:
// consecutive planes per workgroup (many frames), which share the scan of
// the sites and every staged site's weights; n_planes counts the workgroups
// of planes.
template <typename T, typename T2, bool ONE, bool P5, int SPL>
__global__ __launch_bounds__(ONE ? SPREAD_THREADS_ONE : SPREAD_THREADS) void k_fft_xy_spread(FFTPlan1D px, FFTPlan1D py, int Kz, MeshInfo mi,
                                                       BinArgs ba, T* __restrict__ rho_out,
                                                       T2* __restrict__ out_c, int n_planes) {
  static_assert(!ONE || SPL == 1, "a one-frame launch takes one plane per workgroup");
  // 16-byte alignment for the complex values and the FP64 LDS atomics
  extern __shared__ __align__(16) unsigned char smem[];
  if ((int)blockIdx.x >= n_planes) {
    if constexpr (ONE)
      bin_block<SPREAD_THREADS_ONE, true, BIN_BATCH_KEEP>(ba, blockIdx.y, reinterpret_cast<int*>(smem));
    else
      bin_block<SPREAD_THREADS, false, BIN_BATCH>(ba, blockIdx.y, reinterpret_cast<int*>(smem));
    return;
  }
  const int Kx = px.n, Ky = py.n, NP = Kx * Ky;
  T2* A = reinterpret_cast<T2*>(smem);
  T2* B = A + SPL * NP;
  T2* twx = B + SPL * NP;
  T2* twy = twx + Kx;
  // the real planes accumulate in FP64 in every precision (FP32 LDS atomics
  // measured slower than FP64 ones: 6.6 against 3.5 ms for a 4096-frame spread)
  double* acc = reinterpret_cast<double*>(twy + Ky);       // SPL * NP values
  int* list = reinterpret_cast<int*>(acc + SPL * NP);      // staged (site, z slot) entries, or sites (SPL > 1)
  load_twiddles(px, twx);
  load_twiddles(py, twy);
  const int iz = blockIdx.x * SPL;                         // first plane of the workgroup
  const int npl = min(SPL, Kz - iz);
  const int frame = blockIdx.y;
  for (int i = threadIdx.x; i < npl * NP; i += blockDim.x) acc[i] = 0.0;
  __syncthreads();
  const int P = mi.order;
  const int n = ba.n_site;
  const double* sx = ba.xyz_all + frame * ba.frame_stride;
  const double* sy = sx + n;
  const double* sz = sy + n;
  const double* q = ba.site_q;
  const double Lx = ba.cell.L[0], Ly = ba.cell.L[1], Lz = ba.cell.L[2];
  const double ihx = mi.invh[0], ihy = mi.invh[1], ihz = mi.invh[2];
  // wrapped into the box through the reciprocal box lengths (the spread's
  // weights vanish continuously at the stencil ends, so a last-bit
  // difference from the binning's quotient is immaterial; the staging and
  // the weights below use the same function, so they agree on the stencil)
  const double rLx = 1.0 / Lx, rLy = 1.0 / Ly, rLz = 1.0 / Lz;
  auto wrap = [](double x, double L, double rL) { return x - L * floor(x * rL); };
  // one staged entry: the site's B-spline weights, then its P x P in-plane
  // contributions to each plane of the workgroup its stencil reaches, added
  // with LDS atomics (SPL == 1: the entry carries the plane's z slot)
  auto add_site = [&](int e) {
    const int j = SPL == 1 ? e >> 3 : e;
    double xj = sx[j], yj = sy[j];
    if (!isfinite(xj)) xj = 0.0;
    if (!isfinite(yj)) yj = 0.0;
    double zj = sz[j];
    if (!isfinite(zj)) zj = 0.0;
    T Bx[MAX_ORDER], By[MAX_ORDER], Bz[MAX_ORDER];
    constexpr int ORD = P5 ? 5 : -1;
    int fx = spline_triangle_d<T, ORD>(wrap(xj, Lx, rLx) * ihx, P, Bx);
    int fy = spline_triangle_d<T, ORD>(wrap(yj, Ly, rLy) * ihy, P, By);
    int fz = spline_triangle_d<T, ORD>(wrap(zj, Lz, rLz) * ihz, P, Bz);
    fx = ((fx % Kx) + Kx) % Kx;
    fy = ((fy % Ky) + Ky) % Ky;
    fz = ((fz % Kz) + Kz) % Kz;
#pragma unroll
    for (int p = 0; p < SPL; ++p) {
      int tz;
      if (SPL == 1) {
        tz = e & 7;
      } else {
        tz = iz + p - fz;
        tz += (tz < 0) ? Kz : 0;
        if (p >= npl || tz >= P) continue;
      }
      T wz = 0;
#pragma unroll
      for (int b = 0; b < MAX_ORDER; ++b) wz = (b == P - 1 - tz) ? Bz[b] : wz;
      const T qz = (T)q[j] * wz;
      double* plane = acc + p * NP;
#pragma unroll
      for (int by = 0; by < MAX_ORDER; ++by) {
        if (by < P) {
          int iy = fy + (P - 1 - by); iy -= (iy >= Ky) ? Ky : 0;
          const T qyz = qz * By[by];
          double* row = plane + iy * Kx;
#pragma unroll
          for (int bx = 0; bx < MAX_ORDER; ++bx) {
            if (bx < P) {
              int ix = fx + (P - 1 - bx); ix -= (ix >= Kx) ? Kx : 0;
              atomicAdd(row + ix, (double)(qyz * Bx[bx]));
            }
          }
        }
      }
    }
  };
  // Staging, wavefront by wavefront, by the first SPREAD_THREADS threads
  // (in a one-frame workgroup the others wait at the barrier: more
  // wavefronts only thin out the lists): a thread reads the z of SB sites
  // (the loads issued together); those whose stencil reaches the plane go to
  // the wavefront's own list (ballot and prefix count: no atomics and no
  // workgroup barrier), which the wavefront then works through with all its
  // lanes, so that every wavefront shares the weights and the atomics.
  const int lane = threadIdx.x & (WAVE - 1);
  constexpr int NT = SPREAD_THREADS;
  constexpr int SB = SPREAD_LIST / NT;
  int* wl = list + (threadIdx.x / WAVE) * (SB * WAVE);
  const unsigned long long lt = (1ull << lane) - 1ull;
  if (threadIdx.x < NT)
  for (int base = 0; base < n; base += SPREAD_LIST) {
    double zv[SB];
#pragma unroll
    for (int u = 0; u < SB; ++u) {
      const int j = base + u * NT + (int)threadIdx.x;
      zv[u] = j < n ? sz[j] : 0.0;
    }
    int cnt = 0;
#pragma unroll
    for (int u = 0; u < SB; ++u) {
      const int j = base + u * NT + (int)threadIdx.x;
      int tz = P;
      if (j < n) {
        double zj = zv[u];
        if (!isfinite(zj)) zj = 0.0;
        int fz = spline_first(wrap(zj, Lz, rLz) * ihz, P);
        fz = ((fz % Kz) + Kz) % Kz;
        tz = iz - fz;
        tz += (tz < 0) ? Kz : 0;
      }
      // (several planes: the stencil reaches the first one, or wraps past
      // Kz into one of the others)
      const bool hit = j < n && (tz < P || (SPL > 1 && tz > Kz - npl));
      const unsigned long long m = __ballot(hit);
      if (hit) wl[cnt + __popcll(m & lt)] = SPL == 1 ? j * 8 + tz : j;   // site (and its z weight slot)
      cnt += __popcll(m);
    }
    // a wavefront's LDS operations complete in order: its lanes see the list
    __builtin_amdgcn_wave_barrier();
    for (int e = lane; e < cnt; e += WAVE) add_site(wl[e]);
    __builtin_amdgcn_wave_barrier();                      // list read before the next batch writes it
  }
  __syncthreads();
  const size_t off = ((size_t)frame * Kz + iz) * NP;        // the workgroup's planes are contiguous
  for (int i = threadIdx.x; i < npl * NP; i += blockDim.x) {
    if (rho_out) rho_out[off + i] = (T)acc[i];
    A[i] = T2{(T)acc[i], (T)0};
  }
  __syncthreads();
  T2* r1p = plane_lines(A, B, px, twx, Ky, 1, Kx, -1, ONE, npl, NP);
  T2* o1 = (r1p == A) ? B : A;
  T2* r2p = plane_lines(r1p, o1, py, twy, Kx, Kx, 1, -1, ONE, npl, NP);
  for (int i = threadIdx.x; i < npl * NP; i += blockDim.x) out_c[off + i] = r2p[i];
}

// ------------------------------------------------------------------- z pass

template <typename T> __device__ __forceinline__ T mode_k(int i, int K, T twopi_L) {
  int n = (i < (K + 1) / 2) ? i : i - K;
  if ((K & 1) == 0 && n == -(K / 2)) return (T)0;   // no derivative at the Nyquist index
  return (T)n * twopi_L;
}

// mode 0 (potential): X = FFT_z(data1); if save: save = X; energy partial
//          1/2 sum G |X|^2; data1 = IFFT_z(G X)
// mode 1 (field):     X = FFT_z(data1) (+ save if add_saved == 1; with a
//          separate input, SEP, X = FFT_z(in1), or FFT_z(in1 + data1) if
//          add_saved == 2: the electrode and the electrolyte spectra summed
//          before the transform, which is linear);
//          data1 = IFFT_z((-i kx + ky) G X)  [Ex + i Ey after the x-y inverse]
//          data2 = IFFT_z(-i kz G X)         [Ez]
// MULTI: many frames, lpw columns per wavefront (else one, and hosted work)
// plane z of a masked field pass holds data (the mask words are selected,
// not indexed, so that they stay in scalar registers)
__device__ __forceinline__ bool zplane_on(const ZMask& zm, int z) {
  const unsigned long long w = z < 64 ? zm.w[0] : z < 128 ? zm.w[1] : z < 192 ? zm.w[2] : zm.w[3];
  return (w >> (z & 63)) & 1ull;
}

// (the body; k_fft_z and k_fft_z_masked below are its launches)
// SEP: the input spectrum is in1 (a copy kept elsewhere), else data1 itself
// LJ: n_lj more hosted workgroups take the Lennard-Jones sums of the MD
// loop's sites (lj_site), after those of rb and pa
template <typename T, typename T2, bool MULTI, bool MASK, bool SEP, bool LJ = false>
__device__ __forceinline__ void fft_z_body(const FFTPlan1D& pz, const ZPassArgs& za, const T* __restrict__ G,
                                           const T2* __restrict__ in1, T2* __restrict__ data1,
                                           T2* __restrict__ data2,
                                           T2* __restrict__ save, int add_saved,
                                           double* __restrict__ energy_part, int n_z_blocks,
                                           const RealBArgs<T>& rb, const PairArgs<T>& pa, int lpw, int ek_stride,
                                           const ZMask& zm, const MDArgs* lj = nullptr) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ double red[8];
  if (!MULTI && (int)blockIdx.x >= n_z_blocks) {
    // hosted work, one wavefront per target: the real-space part of b
    // (electrode atoms), then the site-site forces (sites)
    // (hosted work is always the one-wavefront-per-target form; the launcher
    // checks that)
    const int hb = (int)blockIdx.x - n_z_blocks;
    T* qbuf = reinterpret_cast<T*>(smem + (threadIdx.x >> 6) * wave_scratch_bytes<T>());
    if (hb < rb.n_blocks) {
      const int g = xcd_block(hb, rb.n_blocks) * (blockDim.x / WAVE) + (threadIdx.x >> 6);
      if (g < rb.el.n) real_b_wave(rb.cell, rb.alpha, rb.eta, rb.rc2, rb.el, rb.st, rb.phi_out, g, blockIdx.y, qbuf);
    } else if (LJ && hb >= rb.n_blocks + pa.n_blocks) {
      lj_site<4>(*lj, hb - rb.n_blocks - pa.n_blocks);
    } else {
      const int j = xcd_block(hb - rb.n_blocks, pa.n_blocks) * (blockDim.x / WAVE) + (threadIdx.x >> 6);
      if (j < pa.st.n) site_pairs_wave(pa.cell, pa.st, pa.alpha, pa.rc2, pa.f_pair, pa.u_site, j, blockIdx.y, qbuf);
    }
    return;
  }
  // one wavefront per lpw (x, y) columns of Kz points (lpw = 1 for one
  // frame; many frames put up to four short columns in a wavefront, so that
  // the stages fill its lanes), za.cpw wavefronts per workgroup; each
  // wavefront has its own three LDS buffers of lpw lines and synchronises
  // only with itself.  Lane l always takes column l mod lpw, points
  // l / lpw + u 64 / lpw of it.
  const int Kx = za.Kx, Ky = za.Ky, Kz = za.Kz;
  const int lane = threadIdx.x & (WAVE - 1), wv = threadIdx.x >> 6;
  const int L = MULTI ? lpw : 1, zs = WAVE / L;            // lpw divides 64
  T2* twz = reinterpret_cast<T2*>(smem);
  T2* A = twz + Kz + (size_t)wv * 3 * L * Kz;
  T2* B = A + L * Kz;
  T2* C = B + L * Kz;
  load_twiddles(pz, twz);
  const int c = lane & (L - 1);                            // this lane's column of the wavefront
  const int z0 = lane / L;
  const int col = (blockIdx.x * za.cpw + wv) * L + c;
  const bool wave_on = wv < za.cpw && (blockIdx.x * za.cpw + wv) * L < Kx * Ky;
  const bool active = wave_on && col < Kx * Ky;            // this lane's column exists
  const int y = active ? col / Kx : 0, x = active ? col - y * Kx : 0;
  const size_t fo = (size_t)blockIdx.y * Kx * Ky * Kz;
  const size_t plane = (size_t)Kx * Ky;
  const size_t cxy = (size_t)y * Kx + x;                   // point z of the column: z * plane + cxy
  T2* Al = A + c * Kz;
  // the columns, and the multiplier (and saved spectrum) of this lane's
  // points, loaded together so that their latencies overlap
  // the input spectrum at point z of this lane's column
  auto load_in = [&](int z) -> T2 {
    const size_t o = fo + z * plane + cxy;
    if (!SEP) return data1[o];
    T2 a = in1[o];
    if (add_saved == 2) { const T2 b = data1[o]; a.x += b.x; a.y += b.y; }
    return a;
  };
  T gk[ZPASS_PREFETCH];
  T2 sv[ZPASS_PREFETCH];
#pragma unroll
  for (int u = 0; u < ZPASS_PREFETCH; ++u) {
    const int z = z0 + u * zs;
    gk[u] = (T)0;
    sv[u] = T2{(T)0, (T)0};
    if (active && z < Kz) {
      Al[z] = (!MASK || za.mode == 0 || zplane_on(zm, z)) ? load_in(z) : T2{(T)0, (T)0};
      gk[u] = G[z * plane + cxy];
      if (za.mode == 1 && add_saved == 1) sv[u] = save[fo + z * plane + cxy];
    }
  }
  if (active)
    for (int z = z0 + ZPASS_PREFETCH * zs; z < Kz; z += zs)
      Al[z] = (!MASK || za.mode == 0 || zplane_on(zm, z)) ? load_in(z) : T2{(T)0, (T)0};
  __syncthreads();                                         // twiddles
  double e = 0.0;
  if (wave_on) {
    T2* X = fft_line_w(A, B, pz, twz, -1, L, Kz);
    T2* F1 = (X == A) ? B : A;
    T2* Xl = X + c * Kz;
    T2* F1l = F1 + c * Kz;
    if (za.mode == 0) {
      // X <- G X (energy partial 1/2 sum G |X|^2; X saved for the field pass)
      auto mul = [&](int z, T g) {
        const T2 v = Xl[z];
        if (save) save[fo + z * plane + cxy] = v;
        e += (double)g * ((double)v.x * v.x + (double)v.y * v.y);
        Xl[z] = T2{v.x * g, v.y * g};
      };
      if (active) {
#pragma unroll
        for (int u = 0; u < ZPASS_PREFETCH; ++u)
          if (z0 + u * zs < Kz) mul(z0 + u * zs, gk[u]);
        for (int z = z0 + ZPASS_PREFETCH * zs; z < Kz; z += zs) mul(z, G[z * plane + cxy]);
      }
      T2* Y = fft_line_w(X, F1, pz, twz, +1, L, Kz);
      if (active)
        for (int z = z0; z < Kz; z += zs)
          if (!MASK || zplane_on(zm, z)) data1[fo + z * plane + cxy] = Y[c * Kz + z];
    } else {
      // C keeps G X; the first inverse transforms (-i kx + ky) G X (Ex + i Ey
      // after the x-y inverse), the second -i kz G X (Ez)
      const T kx = mode_k<T>(x, Kx, (T)za.twopi_L[0]);
      const T ky = mode_k<T>(y, Ky, (T)za.twopi_L[1]);
      T2* Cl = C + c * Kz;
      auto mul = [&](int z, T g, T2 w) {
        T2 v = Xl[z];
        if (add_saved == 1) { v.x += w.x; v.y += w.y; }
        v = T2{v.x * g, v.y * g};
        Cl[z] = v;
        F1l[z] = T2{kx * v.y + ky * v.x, -kx * v.x + ky * v.y};
      };
      if (active) {
#pragma unroll
        for (int u = 0; u < ZPASS_PREFETCH; ++u)
          if (z0 + u * zs < Kz) mul(z0 + u * zs, gk[u], sv[u]);
        for (int z = z0 + ZPASS_PREFETCH * zs; z < Kz; z += zs)
          mul(z, G[z * plane + cxy], add_saved == 1 ? save[fo + z * plane + cxy] : T2{(T)0, (T)0});
      }
      T2* Y = fft_line_w(F1, X, pz, twz, +1, L, Kz);
      if (active)
        for (int z = z0; z < Kz; z += zs) data1[fo + z * plane + cxy] = Y[c * Kz + z];
      T2* W = (Y == F1) ? X : F1;                           // free after the store above
      __builtin_amdgcn_wave_barrier();
      for (int z = z0; z < Kz; z += zs) {
        const T kz = mode_k<T>(z, Kz, (T)za.twopi_L[2]);
        const T2 v = Cl[z];
        Cl[z] = T2{kz * v.y, -kz * v.x};
      }
      T2* Z = fft_line_w(C, W, pz, twz, +1, L, Kz);
      if (active)
        for (int z = z0; z < Kz; z += zs) data2[fo + z * plane + cxy] = Z[c * Kz + z];
    }
  }
  if (za.mode == 0 && energy_part) {
    e = wave_sum(e);
    if (lane == 0) red[wv] = e;
    __syncthreads();
    double* ep = energy_part + (size_t)blockIdx.y * ek_stride;
    if (threadIdx.x == 0) {
      double s = 0.0;
      for (int w = 0; w < (int)(blockDim.x >> 6); ++w) s += red[w];
      ep[blockIdx.x] = 0.5 * s;
    }
    // a frame's partials are ek_stride apart; with fewer workgroups than
    // that (several columns per wavefront) the first clears the rest
    if (blockIdx.x == 0)
      for (int b = n_z_blocks + (int)threadIdx.x; b < ek_stride; b += blockDim.x) ep[b] = 0.0;
  }
}

template <typename T, typename T2, bool MULTI>
__global__ __launch_bounds__(256) void k_fft_z(FFTPlan1D pz, ZPassArgs za, const T* __restrict__ G,
                                               T2* __restrict__ data1, T2* __restrict__ data2,
                                               T2* __restrict__ save, int add_saved,
                                               double* __restrict__ energy_part, int n_z_blocks,
                                               RealBArgs<T> rb, PairArgs<T> pa, int lpw, int ek_stride) {
  fft_z_body<T, T2, MULTI, false, false>(pz, za, G, nullptr, data1, data2, save, add_saved, energy_part, n_z_blocks,
                                         rb, pa, lpw, ek_stride, ZMask{});
}

// the same reading its input spectrum from in1 (kept apart from data1,
// which takes the result): the MD loop's field pass, with the loop's
// Lennard-Jones sums as more hosted workgroups (one per site)
template <typename T, typename T2, bool MULTI>
__global__ __launch_bounds__(256) void k_fft_z_sep(FFTPlan1D pz, ZPassArgs za, const T* __restrict__ G,
                                                   const T2* __restrict__ in1, T2* __restrict__ data1,
                                                   T2* __restrict__ data2, T2* __restrict__ save, int add_saved,
                                                   double* __restrict__ energy_part, int n_z_blocks,
                                                   RealBArgs<T> rb, PairArgs<T> pa, int lpw, int ek_stride,
                                                   MDArgs lj) {
  fft_z_body<T, T2, MULTI, false, true, true>(pz, za, G, in1, data1, data2, save, add_saved, energy_part,
                                              n_z_blocks, rb, pa, lpw, ek_stride, ZMask{}, &lj);
}

// many frames: the potential pass writing, the field pass reading, only the
// masked planes (ZMask)
template <typename T, typename T2, bool MULTI>
__global__ __launch_bounds__(256) void k_fft_z_masked(FFTPlan1D pz, ZPassArgs za, const T* __restrict__ G,
                                                      T2* __restrict__ data1, T2* __restrict__ data2,
                                                      T2* __restrict__ save, int add_saved,
                                                      double* __restrict__ energy_part, int n_z_blocks,
                                                      RealBArgs<T> rb, PairArgs<T> pa, int lpw, int ek_stride,
                                                      ZMask zm) {
  fft_z_body<T, T2, MULTI, true, false>(pz, za, G, nullptr, data1, data2, save, add_saved, energy_part, n_z_blocks,
                                        rb, pa, lpw, ek_stride, zm);
}


// ------------------------------------------------------------------ launchers

// dynamic LDS of k_fft_xy_spread over pl planes: two complex planes each,
// twiddles, the real planes and the site staging list
template <typename T, typename T2>
size_t fft_xy_spread_lds(int Kx, int Ky, int pl) {
  return (2 * (size_t)pl * Kx * Ky + Kx + Ky) * sizeof(T2) + (size_t)pl * Kx * Ky * sizeof(double) +
         (size_t)SPREAD_LIST * sizeof(int);
}

// planes per workgroup of a many-frame spread launch (where they fit)
constexpr int SPREAD_PLANES_MANY = 2;


template <typename T, typename T2>
void launch_fft_xy_spread_t(hipStream_t s, int n_frames, const FFTPlan1D& px, const FFTPlan1D& py, int Kz,
                            const MeshInfo& mi, const BinArgs& ba, T* rho_out, T2* out_c, bool planes, bool bin) {
  constexpr int S = SPREAD_PLANES_MANY;
  const bool multi = n_frames > 1 && fft_xy_spread_lds<T, T2>(px.n, py.n, S) <= LDS_LIMIT;
  const int spl = multi ? S : 1;
  const int np = planes ? (Kz + spl - 1) / spl : 0;         // workgroups of planes
  size_t lds = fft_xy_spread_lds<T, T2>(px.n, py.n, spl);
  if (bin) lds = std::max(lds, bin_lds_spread(ba.n_site, ba.cell.n_cells));
  dim3 grid(np + (bin ? 1 : 0), n_frames);
  if (grid.x == 0) return;
  auto* k = n_frames == 1 ? (mi.order == 5 ? k_fft_xy_spread<T, T2, true, true, 1> : k_fft_xy_spread<T, T2, true, false, 1>)
            : multi       ? (mi.order == 5 ? k_fft_xy_spread<T, T2, false, true, S> : k_fft_xy_spread<T, T2, false, false, S>)
                          : (mi.order == 5 ? k_fft_xy_spread<T, T2, false, true, 1> : k_fft_xy_spread<T, T2, false, false, 1>);
  hipLaunchKernelGGL(k, grid, dim3(n_frames == 1 ? SPREAD_THREADS_ONE : SPREAD_THREADS), lds, s, px, py, Kz, mi, ba, rho_out,
                     out_c, np);
}

size_t bin_lds_spread(int n_site, int n_cells) {
  return std::max(bin_body_lds<SPREAD_THREADS>(n_site, n_cells), bin_body_lds<SPREAD_THREADS_ONE>(n_site, n_cells));
}

template size_t fft_xy_spread_lds<double, double2>(int, int, int);
template size_t fft_xy_spread_lds<float, float2>(int, int, int);
template void launch_fft_xy_spread_t<double, double2>(hipStream_t, int, const FFTPlan1D&, const FFTPlan1D&, int,
                                                      const MeshInfo&, const BinArgs&, double*, double2*, bool, bool);
template void launch_fft_xy_spread_t<float, float2>(hipStream_t, int, const FFTPlan1D&, const FFTPlan1D&, int,
                                                    const MeshInfo&, const BinArgs&, float*, float2*, bool, bool);

// dynamic LDS of k_fft_xy: pl planes twice (ping-pong) and the twiddles
template <typename T2>
size_t fft_xy_lds(const FFTPlan1D& px, const FFTPlan1D& py, int pl) {
  return (2 * (size_t)pl * px.n * py.n + px.n + py.n) * sizeof(T2);
}

// planes per workgroup of a many-frame x-y launch: xy_planes_many() where
// they fit in LDS, else one
template <typename T2>
int xy_planes_fit(const FFTPlan1D& px, const FFTPlan1D& py) {
  return fft_xy_lds<T2>(px, py, xy_planes_many<T2>()) <= LDS_LIMIT ? xy_planes_many<T2>() : 1;
}

size_t fft_xy_lds_bytes(int Kx, int Ky, int elt_bytes, int planes) {
  return (2 * (size_t)planes * Kx * Ky + Kx + Ky) * (size_t)elt_bytes;
}

// many-frame x-y launch with pl planes per workgroup; grid.y = ny (frames,
// or frames x 2 parts for the split field transform)
template <typename T, typename T2>
void launch_xy_many(hipStream_t s, const FFTPlan1D& px, const FFTPlan1D& py, int Kz, int ny, int mode,
                    const T* in_re, const T2* in_c, T2* out_c, T* out_re, T* out_im, size_t out_re_stride, int split,
                    const T2* in_c2, T* out_re2, const InterpArgs<T>* ia = nullptr, const int* zl = nullptr,
                    int n_zl = 0) {
  int pl = xy_planes_fit<T2>(px, py);
  if (px.planes > 0 && px.planes < pl) pl = 1;          // the tuner's choice (one plane, or as many as fit)
  const int nz = zl ? n_zl : Kz;
  if (nz == 0) return;
  const dim3 grid((nz + pl - 1) / pl, ny);
  const size_t lds = fft_xy_lds<T2>(px, py, pl);
  if (ia || zl) {
    auto* k = pl == 1 ? k_fft_xy_many<T, T2, 1, false> : k_fft_xy_many<T, T2, xy_planes_many<T2>(), false>;
    if (ia) k = pl == 1 ? k_fft_xy_many<T, T2, 1, true> : k_fft_xy_many<T, T2, xy_planes_many<T2>(), true>;
    hipLaunchKernelGGL(k, grid, dim3(XY_THREADS_MANY), lds, s, px, py, Kz, mode, in_re, in_c, out_c, out_re, out_im,
                       out_re_stride, split, in_c2, out_re2, zl, n_zl, ia ? *ia : InterpArgs<T>{});
    return;
  }
  auto* k = pl == 1 ? k_fft_xy<T, T2, false, 1> : k_fft_xy<T, T2, false, xy_planes_many<T2>()>;
  hipLaunchKernelGGL(k, grid, dim3(XY_THREADS_MANY), lds, s, px, py, Kz, mode, in_re, in_c, out_c, out_re, out_im,
                     out_re_stride, split, in_c2, out_re2);
}

template <typename T, typename T2>
void launch_fft_xy_t(hipStream_t s, int n_frames, const FFTPlan1D& px, const FFTPlan1D& py, int Kz,
                     int mode, const T* in_re, const T2* in_c, T2* out_c, T* out_re, T* out_im,
                     size_t out_re_stride, const int* zl, int n_zl) {
  if (out_re_stride == 0) out_re_stride = (size_t)px.n * py.n * Kz;
  if (n_frames == 1)
    hipLaunchKernelGGL((k_fft_xy<T, T2, true, 1>), dim3(Kz, 1), dim3(XY_THREADS), fft_xy_lds<T2>(px, py, 1), s, px, py,
                       Kz, mode, in_re, in_c, out_c, out_re, out_im, out_re_stride, 0, (const T2*)nullptr, (T*)nullptr);
  else
    launch_xy_many<T, T2>(s, px, py, Kz, n_frames, mode, in_re, in_c, out_c, out_re, out_im, out_re_stride, 0,
                          (const T2*)nullptr, (T*)nullptr, nullptr, zl, n_zl);
}

template <typename T, typename T2>
void launch_fft_xy_field_inv_t(hipStream_t s, int n_frames, const FFTPlan1D& px, const FFTPlan1D& py, int Kz,
                               const T2* c1, const T2* c2, T* E, size_t frame_stride, const InterpArgs<T>* ia) {
  const size_t M = (size_t)px.n * py.n * Kz;
  if (n_frames == 1)
    hipLaunchKernelGGL((k_fft_xy<T, T2, true, 1>), dim3(Kz, 2), dim3(XY_THREADS), fft_xy_lds<T2>(px, py, 1), s, px, py,
                       Kz, 1, (const T*)nullptr, c1, (T2*)nullptr, E, E + M, frame_stride, 1, c2, E + 2 * M);
  else
    launch_xy_many<T, T2>(s, px, py, Kz, 2 * n_frames, 1, (const T*)nullptr, c1, (T2*)nullptr, E, E + M, frame_stride,
                          1, c2, E + 2 * M, ia);
}

template <typename T, typename T2>
void launch_fft_z_t(hipStream_t s, int n_frames, const FFTPlan1D& pz, const ZPassArgs& za, const T* G,
                    T2* data1, T2* data2, T2* save, int add_saved, double* energy_part, bool z_pass,
                    const RealBArgs<T>* rb, const PairArgs<T>* pa, const ZMask* zm, const T2* in1,
                    const MDArgs* lj) {
  if (!in1) in1 = data1;
  if (lj && (in1 == data1 || n_frames != 1)) {
    std::fprintf(stderr, "cpm: the Lennard-Jones sums ride only in a one-frame field pass with a kept input\n");
    std::abort();
  }
  const int n_lj = lj ? lj->n_site : 0;
  const RealBArgs<T> r = rb ? *rb : RealBArgs<T>{};
  const PairArgs<T> p = pa ? *pa : PairArgs<T>{};
  // columns per wavefront: one for one frame (the chain of a column is the
  // latency); many frames put up to four short columns in a wavefront
  // (Kz = 64: a radix-4 stage has 16 butterflies per column), while the
  // workgroup's LDS stays within 64 KiB
  int lpw = 1;
  if (n_frames > 1)
    while (lpw < 4 && 2 * lpw * za.Kz <= 4 * WAVE &&
           (3 * (size_t)za.cpw * 2 * lpw * za.Kz + za.Kz) * sizeof(T2) <= 64 * 1024)
      lpw *= 2;
  const int per_block = za.cpw * lpw;
  const int nzb = z_pass ? (za.Kx * za.Ky + per_block - 1) / per_block : 0;
  size_t lds = (3 * (size_t)za.cpw * lpw * za.Kz + za.Kz) * sizeof(T2);
  if (r.n_blocks + p.n_blocks > 0) lds = std::max(lds, pair_queue_lds<T>());
  if ((r.n_blocks > 0 && r.tiles) || (p.n_blocks > 0 && p.tsplit > 0)) {
    std::fprintf(stderr, "cpm: only the one-wavefront-per-target pair forms ride in the z pass\n");
    std::abort();
  }
  dim3 grid(nzb + r.n_blocks + p.n_blocks + n_lj, n_frames);
  if (grid.x == 0) return;
  // energy partials: za.n_blocks per frame (the one-column-per-wavefront
  // count the buffers are sized for)
  if (lpw > 1 && r.n_blocks + p.n_blocks > 0) {
    std::fprintf(stderr, "cpm: no hosted work in a z pass of several columns per wavefront\n");
    std::abort();
  }
  if (zm && in1 != data1) {
    std::fprintf(stderr, "cpm: a masked z pass works in place\n");
    std::abort();
  }
  if (zm && lpw > 1)
    hipLaunchKernelGGL((k_fft_z_masked<T, T2, true>), grid, dim3(256), lds, s, pz, za, G, data1, data2, save,
                       add_saved, energy_part, nzb, r, p, lpw, za.n_blocks, *zm);
  else if (zm)
    hipLaunchKernelGGL((k_fft_z_masked<T, T2, false>), grid, dim3(256), lds, s, pz, za, G, data1, data2, save,
                       add_saved, energy_part, nzb, r, p, 1, za.n_blocks, *zm);
  else if (in1 != data1 && lpw > 1)
    hipLaunchKernelGGL((k_fft_z_sep<T, T2, true>), grid, dim3(256), lds, s, pz, za, G, in1, data1, data2, save,
                       add_saved, energy_part, nzb, r, p, lpw, za.n_blocks, lj ? *lj : MDArgs{});
  else if (in1 != data1)
    hipLaunchKernelGGL((k_fft_z_sep<T, T2, false>), grid, dim3(256), lds, s, pz, za, G, in1, data1, data2, save,
                       add_saved, energy_part, nzb, r, p, 1, za.n_blocks, lj ? *lj : MDArgs{});
  else if (lpw > 1)
    hipLaunchKernelGGL((k_fft_z<T, T2, true>), grid, dim3(256), lds, s, pz, za, G, data1, data2, save, add_saved,
                       energy_part, nzb, r, p, lpw, za.n_blocks);
  else
    hipLaunchKernelGGL((k_fft_z<T, T2, false>), grid, dim3(256), lds, s, pz, za, G, data1, data2, save, add_saved,
                       energy_part, nzb, r, p, 1, za.n_blocks);
}

template void launch_fft_xy_t<double, double2>(hipStream_t, int, const FFTPlan1D&, const FFTPlan1D&, int,
                                               int, const double*, const double2*, double2*, double*,
                                               double*, size_t, const int*, int);
template void launch_fft_xy_t<float, float2>(hipStream_t, int, const FFTPlan1D&, const FFTPlan1D&, int, int,
                                             const float*, const float2*, float2*, float*, float*, size_t,
                                             const int*, int);
template void launch_fft_z_t<double, double2>(hipStream_t, int, const FFTPlan1D&, const ZPassArgs&,
                                              const double*, double2*, double2*, double2*, int, double*, bool,
                                              const RealBArgs<double>*, const PairArgs<double>*, const ZMask*,
                                              const double2*, const MDArgs*);
template void launch_fft_z_t<float, float2>(hipStream_t, int, const FFTPlan1D&, const ZPassArgs&,
                                            const float*, float2*, float2*, float2*, int, double*, bool,
                                            const RealBArgs<float>*, const PairArgs<float>*, const ZMask*,
                                            const float2*, const MDArgs*);
template void launch_fft_xy_field_inv_t<double, double2>(hipStream_t, int, const FFTPlan1D&, const FFTPlan1D&,
                                                         int, const double2*, const double2*, double*, size_t,
                                                         const InterpArgs<double>*);
template void launch_fft_xy_field_inv_t<float, float2>(hipStream_t, int, const FFTPlan1D&, const FFTPlan1D&, int,
                                                       const float2*, const float2*, float*, size_t,
                                                       const InterpArgs<float>*);

}  // namespace cpm
