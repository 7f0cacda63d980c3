// Reflection-major order of the (tile, reflection) pairs of the culling lists, for the
// fixed-order reduction of the adjoint sums (fdtbx_pair_reduce): a stable radix sort of the
// pairs' reflection indices (rocPRIM), whose values are the pairs' positions in the lists, so
// every reflection's pairs come out in ascending list position whatever the schedule.
#include <hip/hip_runtime.h>

#include <cstring>
#include <rocprim/device/device_radix_sort.hpp>

#include "internal.h"

namespace fdtbx {

// keys[i] = idx[i] for the first n_pairs entries (n_pairs read on the device when given), the
// sentinel n_hkl after them; vals[i] = i.
__global__ void k_pair_keys(const int32_t* __restrict__ idx, int64_t cap, const int64_t* __restrict__ n_pairs_dev,
                            int32_t n_hkl, int32_t* __restrict__ keys, int32_t* __restrict__ vals) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= cap) return;
  const int64_t n = n_pairs_dev ? *n_pairs_dev : cap;
  keys[i] = i < n ? idx[i] : n_hkl;
  vals[i] = (int32_t)i;
}

// refl_ptr[r] = first position of key r in the sorted keys, for r = 0 .. n_hkl (the sentinel
// n_hkl, and the end of the array, close the last reflection's range).
__global__ void k_pair_ptr(const int32_t* __restrict__ sorted, int64_t cap, int32_t n_hkl, int64_t* __restrict__ refl_ptr) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i > cap) return;
  const int64_t prev = i > 0 ? (int64_t)sorted[i - 1] : -1;
  const int64_t cur = i < cap ? (int64_t)sorted[i] : (int64_t)n_hkl;
  for (int64_t k = prev + 1; k <= cur && k <= n_hkl; ++k) refl_ptr[k] = i;
}

// Bits of the sort keys 0 .. n_hkl (the sentinel included).
static int end_bit_of(int64_t n_hkl) {
  int b = 1;
  while (b < 31 && (int64_t{1} << b) <= n_hkl) ++b;
  return b;
}

static size_t sort_bytes(int64_t cap, int64_t n_hkl) {
  size_t bytes = 0;
  const hipError_t e = rocprim::radix_sort_pairs(nullptr, bytes, (const int32_t*)nullptr, (int32_t*)nullptr,
                                                 (const int32_t*)nullptr, (int32_t*)nullptr, (size_t)cap, 0,
                                                 end_bit_of(n_hkl), (hipStream_t)0);
  return e == hipSuccess ? bytes : 0;
}

}  // namespace fdtbx

using namespace fdtbx;

extern "C" size_t fdtbx_pair_transpose_workspace(int64_t n_hkl, int64_t pair_cap) {
  if (n_hkl <= 0 || pair_cap <= 0) return 256;  // nothing is used; a non-zero size keeps allocations valid
  if (pair_cap >= (int64_t{1} << 31) || n_hkl >= (int64_t{1} << 30)) return 0;
  const size_t sb = sort_bytes(pair_cap, n_hkl);
  if (sb == 0) return 0;
  return 3 * align_up((size_t)pair_cap * sizeof(int32_t), 256) + align_up(sb, 256);
}

extern "C" int fdtbx_pair_transpose(int64_t n_hkl, const int32_t* idx, int64_t pair_cap, const int64_t* n_pairs,
                                    int64_t* refl_ptr, int32_t* refl_pairs, void* ws, size_t ws_bytes, void* stream) {
  if (n_hkl < 0 || pair_cap < 0) return fail(FDTBX_ERR_INVALID_ARGUMENT, "n_hkl and pair_cap must be non-negative");
  if (pair_cap >= (int64_t{1} << 31) || n_hkl >= (int64_t{1} << 30))
    return fail(FDTBX_ERR_UNSUPPORTED, "pair transpose: pair_cap must be below 2^31 and n_hkl below 2^30");
  hipStream_t s = (hipStream_t)stream;
  if (n_hkl == 0) return FDTBX_OK;
  if (!refl_ptr) return fail(FDTBX_ERR_INVALID_ARGUMENT, "null pointer");
  if (pair_cap == 0) return fill(refl_ptr, n_hkl + 1, (int64_t)0, s);
  if (!idx || !refl_pairs || !ws) return fail(FDTBX_ERR_INVALID_ARGUMENT, "null pointer");
  const size_t need = fdtbx_pair_transpose_workspace(n_hkl, pair_cap);
  if (need == 0) return fail(FDTBX_ERR_HIP, "pair transpose: the sort library gave no workspace size");
  if (ws_bytes < need) return fail(FDTBX_ERR_BUFFER_TOO_SMALL, "pair transpose workspace too small");
  const size_t arr = align_up((size_t)pair_cap * sizeof(int32_t), 256);
  char* w = (char*)ws;
  int32_t* keys = (int32_t*)w;
  int32_t* sorted = (int32_t*)(w + arr);
  int32_t* vals = (int32_t*)(w + 2 * arr);
  void* tmp = w + 3 * arr;
  size_t tmp_bytes = sort_bytes(pair_cap, n_hkl);
  hipLaunchKernelGGL(k_pair_keys, dim3((unsigned)ceil_div(pair_cap, 256)), dim3(256), 0, s, idx, pair_cap, n_pairs,
                     (int32_t)n_hkl, keys, vals);
  FDTBX_LAUNCH_CHECK("pair keys");
  const hipError_t e = rocprim::radix_sort_pairs(tmp, tmp_bytes, (const int32_t*)keys, sorted, (const int32_t*)vals,
                                                 refl_pairs, (size_t)pair_cap, 0, end_bit_of(n_hkl), s);
  if (e != hipSuccess) return hip_fail(e, "pair transpose: radix sort");
  hipLaunchKernelGGL(k_pair_ptr, dim3((unsigned)ceil_div(pair_cap + 1, 256)), dim3(256), 0, s, sorted, pair_cap,
                     (int32_t)n_hkl, refl_ptr);
  FDTBX_LAUNCH_CHECK("pair row pointers");
  return FDTBX_OK;
}
