// Marking of the adaptive loop (Sec. 4.3): the leaves with the m largest
// estimates, equal values in leaf order, by a stable descending radix sort of
// (estimate, leaf index) pairs.
#include <hip/hip_runtime.h>
#include <hipcub/hipcub.hpp>

#include <string>

#include "host/common.hpp"
#include "problem.hpp"

namespace gmg {

namespace {

__global__ void iota32(int64_t n, int32_t* __restrict__ idx) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) idx[i] = (int32_t)i;
}

__global__ void flag_rank(int64_t n, int64_t m, const int32_t* __restrict__ idx, uint8_t* __restrict__ flags) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r < n) flags[idx[r]] = r < m ? 1 : 0;
}

void check(hipError_t e, const char* what) {
  if (e != hipSuccess) fail(GMG_E_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

}  // namespace

size_t mark_temp_bytes(int64_t n) {
  size_t bytes = 0;
  check(hipcub::DeviceRadixSort::SortPairsDescending(nullptr, bytes, (const double*)nullptr, (double*)nullptr,
                                                     (const int32_t*)nullptr, (int32_t*)nullptr, (int)n),
        "radix sort size");
  return std::max<size_t>(bytes, 256);
}

void mark_top(const double* eta, int64_t n, int64_t m, double* keys_out, int32_t* idx_in, int32_t* idx_out,
              void* temp, size_t temp_bytes, uint8_t* flags, hipStream_t s) {
  if (n <= 0) return;
  if (n > INT32_MAX) fail(GMG_E_INVAL, "too many leaves to mark");
  const unsigned g = (unsigned)((n + 255) / 256);
  hipLaunchKernelGGL(iota32, dim3(g), dim3(256), 0, s, n, idx_in);
  size_t tb = temp_bytes;
  check(hipcub::DeviceRadixSort::SortPairsDescending(temp, tb, eta, keys_out, idx_in, idx_out, (int)n, 0,
                                                     (int)(sizeof(double) * 8), s),
        "radix sort");
  hipLaunchKernelGGL(flag_rank, dim3(g), dim3(256), 0, s, n, m, idx_out, flags);
  check(hipGetLastError(), "marking");
}

}  // namespace gmg
