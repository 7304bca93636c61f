// Laterally averaged charge density and the 1D Poisson potential profile
// (Eq. 16; the paper's potential-profile subsection and post-analysis
// paragraph): rho(z) over frames on a z-grid, with the electrolyte sites as
// point charges binned by their wrapped z and the electrode charges as their
// Gaussian distributions (Eq. 2) integrated over each bin, then
// d2 psi / dz2 = -rho / eps0 by the second-difference equations of the grid.
//
// The finite-difference system is solved exactly by two prefix sums rather
// than a matrix inverse: with s_k = psi_{k+1} - psi_k, the equation of bin k
// reads s_k - s_{k-1} = -(h^2/eps0) rho_k, so s_k = s_last - (h^2/eps0) C_k
// with C_k the running sum of rho; the boundary condition fixes s_last:
//   finite field   sum_k s_k = dV (the rise over one period)
//   doubled cell   sum_k s_k = 0  (continuity)
//   slab           s_last = 0     (no field in the empty space at z = 0)
// and psi_k is the running sum of s.
//
// Two launches: per-partition histograms (LDS atomics, one partition of the
// flattened (frame, site) and (frame, atom) indices per workgroup, written
// whole to scratch, so the scratch needs no clearing), then one workgroup
// that sums the partitions, adds the electrode Gaussians and solves.
#include <mutex>

#include "common.h"

namespace cpm {

__global__ __launch_bounds__(PROFILE_THREADS) void k_profile_partial(ProfileArgs p) {
  extern __shared__ __align__(16) unsigned char smem[];
  double* hist = reinterpret_cast<double*>(smem);          // [n_bins] site charge per bin
  double* hq = hist + p.n_bins;                              // [n_heights] electrode charge per height
  const int nt = p.n_bins + p.n_heights;
  for (int i = threadIdx.x; i < nt; i += blockDim.x) hist[i] = 0.0;
  __syncthreads();
  // this workgroup's share of the (frame, site) pairs
  const long long ns = (long long)p.n_frames * p.n_site;
  const long long s0 = ns * blockIdx.x / gridDim.x, s1 = ns * (blockIdx.x + 1) / gridDim.x;
  for (long long t = s0 + threadIdx.x; t < s1; t += blockDim.x) {
    const int f = (int)(t / p.n_site), j = (int)(t - (long long)f * p.n_site);
    const double z = p.xyz[((size_t)f * 3 + 2) * p.n_site + j];
    double zw = z - p.Lz * floor(z * p.inv_Lz);
    int k = (int)(zw * p.inv_h);
    k = k < 0 ? 0 : (k >= p.n_bins ? p.n_bins - 1 : k);
    atomicAdd(&hist[k], p.site_q[j]);
  }
  // and of the (frame, atom) charges, summed per electrode height
  const long long ne = (long long)p.n_frames * p.n_elec;
  const long long e0 = ne * blockIdx.x / gridDim.x, e1 = ne * (blockIdx.x + 1) / gridDim.x;
  for (long long t = e0 + threadIdx.x; t < e1; t += blockDim.x) {
    const int f = (int)(t / p.n_elec), i = (int)(t - (long long)f * p.n_elec);
    atomicAdd(&hq[p.height_of[i]], p.q[(size_t)f * p.q_stride + i]);
  }
  __syncthreads();
  double* out = p.part + (size_t)blockIdx.x * nt;
  for (int i = threadIdx.x; i < nt; i += blockDim.x) out[i] = hist[i];
}

// inclusive prefix sum of v[0..n) in place, n <= 2 * blockDim.x, by one
// workgroup: thread t owns v[2t] and v[2t+1]; the pair sums are scanned
// (Hillis-Steele in tmp) and each thread adds the sum of the pairs before its own
__device__ void block_scan(double* v, double* tmp, int n) {
  const int t = threadIdx.x;
  const int a = 2 * t, b = 2 * t + 1;
  const double xa = a < n ? v[a] : 0.0, xb = b < n ? v[b] : 0.0;
  tmp[t] = xa + xb;
  __syncthreads();
  for (int off = 1; off < (int)blockDim.x; off <<= 1) {
    const double add = t >= off ? tmp[t - off] : 0.0;
    __syncthreads();
    tmp[t] += add;
    __syncthreads();
  }
  const double before = t > 0 ? tmp[t - 1] : 0.0;
  if (a < n) v[a] = before + xa;
  if (b < n) v[b] = before + xa + xb;
  __syncthreads();
}

__global__ __launch_bounds__(PROFILE_SOLVE_THREADS) void k_profile_solve(ProfileArgs p) {
  extern __shared__ __align__(16) unsigned char smem[];
  double* rho = reinterpret_cast<double*>(smem);     // [n_bins]
  double* hq = rho + p.n_bins;                        // [n_heights] frame-summed charge per height
  double* s = hq + p.n_heights;                       // [n_bins]
  double* tmp = s + p.n_bins;                         // [blockDim.x]
  __shared__ double red[PROFILE_SOLVE_THREADS / WAVE];
  const int nt = p.n_bins + p.n_heights;
  const int n = p.n_bins;
  const double h = p.Lz / n;
  for (int i = threadIdx.x; i < nt; i += blockDim.x) {
    double acc = 0.0;
    for (int b = 0; b < p.n_part; ++b) acc += p.part[(size_t)b * nt + i];
    rho[i] = acc;                                      // (hq follows rho in the same array)
  }
  __syncthreads();
  // electrode Gaussians: marginal q eta/sqrt(pi) exp(-eta^2 (z - z_h)^2)
  // integrated over each bin, nearest periodic images included
  const double reach = 8.0 / p.eta;
  for (int k = threadIdx.x; k < n; k += blockDim.x) {
    const double lo = k * h, hi = (k + 1) * h;
    double acc = 0.0;
    for (int g = 0; g < p.n_heights; ++g) {
      const double Q = hq[g];
      if (Q == 0.0) continue;
      for (int img = -1; img <= 1; ++img) {
        const double c = p.heights[g] + img * p.Lz;
        if (hi < c - reach || lo > c + reach) continue;
        acc += 0.5 * Q * (erf(p.eta * (hi - c)) - erf(p.eta * (lo - c)));
      }
    }
    rho[k] = (rho[k] + acc) / (p.n_frames * p.area * h);
    p.rho_out[k] = rho[k];
  }
  __syncthreads();
  // running sums C_k, and their total for the boundary condition
  for (int k = threadIdx.x; k < n; k += blockDim.x) s[k] = rho[k];
  __syncthreads();
  block_scan(s, tmp, n);
  double part = 0.0;
  for (int k = threadIdx.x; k < n; k += blockDim.x) part += s[k];
  part = wave_sum(part);
  if ((threadIdx.x & (WAVE - 1)) == 0) red[threadIdx.x / WAVE] = part;
  __syncthreads();
  double sumC = 0.0;
  for (int w = 0; w < (int)(blockDim.x / WAVE); ++w) sumC += red[w];
  const double c2 = h * h / EPS0;
  const double s_last = p.slab ? 0.0 : (p.jump + c2 * sumC) / n;
  __syncthreads();
  // steps s_k, then psi_0 = 0 and psi_{k+1} = psi_k + s_k
  for (int k = threadIdx.x; k < n; k += blockDim.x) s[k] = s_last - c2 * s[k];
  __syncthreads();
  block_scan(s, tmp, n);                              // s[k] = psi_{k+1}
  // bulk reference: the mean of psi over the bins centred in [bulk_lo, bulk_hi)
  double bs = 0.0, bc = 0.0;
  for (int k = threadIdx.x; k < n; k += blockDim.x) {
    const double zc = (k + 0.5) * h;
    if (zc >= p.bulk_lo && zc < p.bulk_hi) { bs += k > 0 ? s[k - 1] : 0.0; bc += 1.0; }
  }
  bs = wave_sum(bs);
  bc = wave_sum(bc);
  __syncthreads();
  if ((threadIdx.x & (WAVE - 1)) == 0) { red[threadIdx.x / WAVE] = bs; tmp[threadIdx.x / WAVE] = bc; }
  __syncthreads();
  double tb = 0.0, tc = 0.0;
  for (int w = 0; w < (int)(blockDim.x / WAVE); ++w) { tb += red[w]; tc += tmp[w]; }
  const double ref = tb / tc;
  for (int k = threadIdx.x; k < n; k += blockDim.x) p.psi_out[k] = (k > 0 ? s[k - 1] : 0.0) - ref;
}

size_t profile_partial_lds(int n_bins, int n_heights) { return (size_t)(n_bins + n_heights) * sizeof(double); }
size_t profile_solve_lds(int n_bins, int n_heights) {
  return (size_t)(2 * n_bins + n_heights + PROFILE_SOLVE_THREADS) * sizeof(double);
}

// ------------------------------------------------ scratch without allocation
//
// For callers that cannot allocate (code under HIP graph capture, serving
// loops, harnesses that forbid hipMalloc), cpm_profile_noalloc takes its
// histogram partitions from this file-scope array instead of the context's
// allocation.  PROFILE_STATIC_DOUBLES covers the largest request the
// argument limits allow (128 partitions x (2048 bins + 2048 heights)).
// Every call on one GPU shares that GPU's copy, which keeps the last call's
// contents; each partition is written whole before it is read, so nothing
// needs clearing, and calls that overlap on one GPU race.
static __device__ __align__(256) double scratch[PROFILE_STATIC_DOUBLES];

namespace {
std::mutex g_scratch_mu;
void* g_scratch_ptr[PROFILE_MAX_DEVICES] = {};
}  // namespace

int profile_static_scratch(int device, double** out) {
  *out = nullptr;
  if (device < 0 || device >= PROFILE_MAX_DEVICES) return -1;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    // the device's own address of the array (the host-side name is only a
    // stand-in); the device is current in the caller
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return -1;
    g_scratch_ptr[device] = p;
  }
  *out = static_cast<double*>(g_scratch_ptr[device]);
  return 0;
}

void launch_profile(hipStream_t s, const ProfileArgs& p) {
  hipLaunchKernelGGL(k_profile_partial, dim3(p.n_part), dim3(PROFILE_THREADS), profile_partial_lds(p.n_bins, p.n_heights),
                     s, p);
  hipLaunchKernelGGL(k_profile_solve, dim3(1), dim3(PROFILE_SOLVE_THREADS), profile_solve_lds(p.n_bins, p.n_heights), s,
                     p);
}

}  // namespace cpm
