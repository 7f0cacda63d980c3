// Launch order of the per-tile kernels (fdtbx_tile_order).  Workgroups are dealt to the 8
// XCDs round-robin and run as slots free up; when the launch holds only a few rounds of
// workgroups per slot, the order in which heavy tiles start sets the makespan.  Tiles are
// grouped into superblocks (order_super) that run on one XCD in consecutive dispatch slots,
// consecutive superblocks on different XCDs.  Work order: superblocks by decreasing length
// of their longest tile list, the tiles of a superblock by decreasing list length (ties in
// index order).  Spatial order: superblocks and their tiles in index order, for launches of
// many rounds, where the L2 reuse between neighbouring superblocks matters more.
#include <hip/hip_runtime.h>

#include "internal.h"
#include "profile_common.h"

namespace fdtbx {

// tiles_x, tiles_y: the launched tile columns and rows (all, or the left or top half under the
// mirror folds); stride: tile columns of the detector (tile t = ty * stride + tx).
struct OrderParams {
  int32_t tiles_x, tiles_y, S, sbw, sbh, stride;
  int64_t nsb;
};

__device__ static inline int64_t tile_len(const OrderParams& p, const int64_t* offsets, int64_t sb, int i) {
  const int64_t tx = (sb % p.sbw) * p.S + i % p.S, ty = (sb / p.sbw) * p.S + i / p.S;
  if (tx >= p.tiles_x || ty >= p.tiles_y) return -1;
  const int64_t t = ty * p.stride + tx;
  return offsets[t + 1] - offsets[t];
}

// Per superblock (one wave; lane i holds tile i of the S^2 <= 64): its key (longest list) and
// the rank order of its tiles, each lane counting the tiles that go before its own.
__global__ void __launch_bounds__(64) k_order_keys(OrderParams p, const int64_t* __restrict__ offsets,
                                                   int64_t* __restrict__ key, uint8_t* __restrict__ inner) {
  const int64_t sb = blockIdx.x;
  const int i = threadIdx.x;
  const int n = p.S * p.S;
  const int64_t ci = i < n ? tile_len(p, offsets, sb, i) : -1;
  int rank = 0;
  for (int k = 0; k < n; ++k) {
    const int64_t ck = __shfl(ci, k, 64);
    rank += (ck > ci || (ck == ci && k < i)) ? 1 : 0;
  }
  if (i < n) inner[sb * n + rank] = (uint8_t)i;
  int64_t best = ci;
  for (int o = 32; o >= 1; o >>= 1) {
    const int64_t other = __shfl_xor(best, o, 64);
    best = other > best ? other : best;
  }
  if (i == 0) key[sb] = best;
}

// Superblocks by decreasing key (ties in index order).
__global__ void __launch_bounds__(256) k_order_rank(OrderParams p, const int64_t* __restrict__ key,
                                                    int32_t* __restrict__ sorted) {
  const int64_t sb = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (sb >= p.nsb) return;
  const int64_t kj = key[sb];
  int64_t rank = 0;
  for (int64_t i = 0; i < p.nsb; ++i) {
    const int64_t ki = key[i];
    rank += (ki > kj || (ki == kj && i < sb)) ? 1 : 0;
  }
  sorted[rank] = (int32_t)sb;
}

// order[b]: workgroup b runs on XCD b % 8 as the k = b / 8-th of that XCD; its superblock
// is the (k / S^2) * 8 + (b % 8)-th of the sequence, its tile the (k % S^2)-th within it.
__global__ void __launch_bounds__(256) k_order_fill(OrderParams p, int64_t n_blocks, const int32_t* __restrict__ sorted,
                                                    const uint8_t* __restrict__ inner, int32_t* __restrict__ order) {
  const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= n_blocks) return;
  const int64_t n = (int64_t)p.S * p.S;
  const int64_t x = b % kXcds, k = b / kXcds;
  const int64_t slot = (k / n) * kXcds + x;
  int32_t t = -1;
  if (slot < p.nsb) {
    const int64_t sb = sorted ? sorted[slot] : slot;
    const int i = sorted ? inner[sb * n + k % n] : (int)(k % n);
    const int64_t tx = (sb % p.sbw) * p.S + i % p.S, ty = (sb / p.sbw) * p.S + i / p.S;
    if (tx < p.tiles_x && ty < p.tiles_y) t = (int32_t)(ty * p.stride + tx);
  }
  order[b] = t;
}

static void order_params(const fdtbx_geometry* g, OrderParams* p) {
  p->tiles_x = lcols_of(g);
  p->tiles_y = lrows_of(g);
  p->stride = tiles_x_of(g);
  p->S = order_super(p->tiles_x, p->tiles_y);
  p->sbw = (int32_t)ceil_div(p->tiles_x, p->S);
  p->sbh = (int32_t)ceil_div(p->tiles_y, p->S);
  p->nsb = (int64_t)p->sbw * p->sbh;
}

}  // namespace fdtbx

using namespace fdtbx;

extern "C" int64_t fdtbx_tile_order_size(const fdtbx_geometry* geom) {
  if (!geom || check_geometry(geom)) return 0;
  return order_grid(lcols_of(geom), lrows_of(geom));
}

extern "C" size_t fdtbx_tile_order_workspace(const fdtbx_geometry* geom) {
  if (!geom || check_geometry(geom)) return 0;
  OrderParams p;
  order_params(geom, &p);
  return align_up((size_t)p.nsb * sizeof(int64_t), 256) + align_up((size_t)p.nsb * sizeof(int32_t), 256) +
         align_up((size_t)p.nsb * p.S * p.S, 256);
}

extern "C" int fdtbx_tile_order(const fdtbx_geometry* geom, const int64_t* offsets, int32_t* order, void* ws,
                                size_t ws_bytes, void* stream) {
  if (!geom || !offsets || !order || !ws) return fail(FDTBX_ERR_INVALID_ARGUMENT, "null pointer");
  int rc = check_geometry(geom);
  if (rc) return rc;
  if (ws_bytes < fdtbx_tile_order_workspace(geom)) return fail(FDTBX_ERR_BUFFER_TOO_SMALL, "tile order workspace too small");
  OrderParams p;
  order_params(geom, &p);
  const int64_t n_blocks = fdtbx_tile_order_size(geom);
  // few rounds of workgroups per slot: work order; else spatial
  int dev = 0, cus = 256;
  FDTBX_HIP(hipGetDevice(&dev));
  FDTBX_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  const int64_t slots = (int64_t)cus * 16;
  const bool work = (int64_t)p.tiles_x * p.tiles_y <= 8 * slots;
  char* w = (char*)ws;
  int64_t* key = (int64_t*)w;
  w += align_up((size_t)p.nsb * sizeof(int64_t), 256);
  int32_t* sorted = (int32_t*)w;
  w += align_up((size_t)p.nsb * sizeof(int32_t), 256);
  uint8_t* inner = (uint8_t*)w;
  hipStream_t s = (hipStream_t)stream;
  const unsigned nb = (unsigned)ceil_div(p.nsb, 256);
  if (work) {
    hipLaunchKernelGGL(k_order_keys, dim3((unsigned)p.nsb), dim3(64), 0, s, p, offsets, key, inner);
    FDTBX_LAUNCH_CHECK("tile order keys");
    hipLaunchKernelGGL(k_order_rank, dim3(nb), dim3(256), 0, s, p, (const int64_t*)key, sorted);
    FDTBX_LAUNCH_CHECK("tile order ranks");
  }
  hipLaunchKernelGGL(k_order_fill, dim3((unsigned)ceil_div(n_blocks, 256)), dim3(256), 0, s, p, n_blocks,
                     work ? (const int32_t*)sorted : nullptr, (const uint8_t*)inner, order);
  FDTBX_LAUNCH_CHECK("tile order");
  return FDTBX_OK;
}
