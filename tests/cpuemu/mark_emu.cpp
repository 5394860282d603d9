// The marking kernels for the CPU emulation (the device radix sort of the
// library is not available to a host compiler): the same contract, a stable
// descending sort of (estimate, leaf index) pairs in host memory, which is
// device memory in the emulation.
#include <algorithm>
#include <cstdint>
#include <numeric>
#include <vector>

#include "hip/hip_runtime.h"

namespace gmg {

size_t mark_temp_bytes(int64_t) { return 256; }

void mark_top(const double* eta, int64_t n, int64_t m, double* keys_out, int32_t* idx_in, int32_t* idx_out,
              void*, size_t, uint8_t* flags, hipStream_t) {
  if (n <= 0) return;
  std::iota(idx_in, idx_in + n, 0);
  std::copy(idx_in, idx_in + n, idx_out);
  std::stable_sort(idx_out, idx_out + n, [&](int32_t a, int32_t b) { return eta[a] > eta[b]; });
  for (int64_t r = 0; r < n; ++r) {
    keys_out[r] = eta[idx_out[r]];
    flags[idx_out[r]] = r < m ? 1 : 0;
  }
}

}  // namespace gmg
