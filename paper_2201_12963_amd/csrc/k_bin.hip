// Stand-alone cell binning: one workgroup of 1024 threads per frame running
// the binning body of bin.h (the PPPM step runs the same body as extra
// workgroups of its first mesh launch instead).
#include "bin.h"

namespace cpm {

constexpr int BIN_THREADS = 1024;

__global__ __launch_bounds__(BIN_THREADS) void k_bin_sites(BinArgs a) {
  extern __shared__ __align__(16) int lds[];
  bin_block<BIN_THREADS, false, BIN_BATCH>(a, blockIdx.x, lds);
}

size_t bin_lds_bytes(int n_site, int n_cells) { return bin_body_lds<BIN_THREADS>(n_site, n_cells); }

void launch_bin_sites(hipStream_t s, int n_frames, const BinArgs& a) {
  size_t lds = bin_lds_bytes(a.n_site, a.cell.n_cells);
  hipLaunchKernelGGL(k_bin_sites, dim3(n_frames), dim3(BIN_THREADS), lds, s, a);
}

}  // namespace cpm
