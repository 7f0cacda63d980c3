// Profile pattern: per pixel, the sum over the reflections of its tile list of
// W_hkl r0^2 sum_k omega_k Z(p* - s_k) (Eq. direct_sum with the lineshape's per-axis
// profile: Eq. I_shape with N -> N_eff, or its Gaussian or Hosemann (Eq. Z) form of the
// same integral breadth), times the Lorentz factor delta/(R + delta) (Eq. lorentz).
//
// Mapping: one to four 64-lane waves per pixel tile (tile_w x 64/tile_w pixels, 8x8 by
// default; the waves split the tile's list), one lane per pixel, pixel sums in
// registers.  Reflections of the tile list are uniform across the wave (their
// records come through scalar loads).  For each (tile, reflection) the wave
// bounds the node window that the tile's query points can reach, builds the
// per-node offsets for 64 window nodes at a time (one node per lane) into LDS, and
// then every lane walks those 64 nodes with broadcast LDS reads.
//
// Per (pixel, reflection) the lattice coordinates are written relative to D so
// that nothing of size h_i is cancelled in float32:
//   y_i = (N_i/2) a_i.(p* - s_k) = alpha_i - kappa_ik,
//   alpha_i = (N_i/2) [(R - R_D)(a_i.e_perp) + (Z - Z_D) a_i,z]           (per pixel)
//   kappa_ik = (N_i r0/2) [(c_k - 1) a_i.S + c_k d1 a_i.e1 + c_k d2 a_i.e2] (per node),
// so that N_i sinc^2(N_i u_i) = N_i sin^2(2 pi y_i)/(2 pi y_i)^2 with the hardware
// sine taking its argument in turns.  Support: max_i |y_i| <= m/2.  The Gaussian
// lineshape uses the same y (N exp(-pi N^2 u^2) = N exp(-4 pi y^2)); the Hosemann one
// writes the record with scale 1 instead of N_i/2 (y_i = u_i, support |y_i| <= 1/2).
#include <hip/hip_runtime.h>

#include <math.h>

#include "internal.h"
#include "profile_common.h"
#include "profile_tile.h"

namespace fdtbx {

// COUNT: counting pass (support test only, the same for every lineshape); LS: lineshape;
// WAVES: waves per tile (each its share of the tile's list).
template <bool COUNT, int LS, int WAVES>
__global__ void __launch_bounds__(64 * WAVES) __attribute__((amdgpu_waves_per_eu(7))) k_profile(ProfParams q, const float* __restrict__ refl,
                                                        const float* __restrict__ nodes, const double* __restrict__ pix,
                                                        const double* __restrict__ tile, const int64_t* __restrict__ offsets,
                                                        const int32_t* __restrict__ idx, float* __restrict__ image,
                                                        unsigned long long* __restrict__ counts,
                                                        const int32_t* __restrict__ order) {
  // per wave, the queues of window nodes that can be inside the support of some pixel of the
  // tile (candidates, then those inside the support of every pixel)
  __shared__ float4 qn[256 * WAVES];
  __shared__ int bq[64 * WAVES];
  __shared__ float xacc[WAVES > 1 ? 64 * (WAVES - 1) : 1];
  __shared__ int qk[LS == FDTBX_LINESHAPE_HOSEMANN ? 128 * WAVES : 1];  // node indices (support edge)
  const int t = order ? order[blockIdx.x] : tile_of_block(q, blockIdx.x);
  if (t < 0) return;  // uniform across the workgroup
  profile_tile<COUNT, LS, WAVES>(q, refl, nodes, pix, tile, offsets, idx, image, counts, t, qn, bq, xacc,
                                 LS == FDTBX_LINESHAPE_HOSEMANN ? qk : nullptr);
}

template <int WAVES>
static void launch_profile(const ProfParams& q, dim3 grid, hipStream_t s, const float* refl, const float* nodes,
                           const double* pix, const double* tile, const int64_t* offsets, const int32_t* idx,
                           const int32_t* order, float* image, int64_t* counts) {
  const dim3 block(64 * WAVES);
  unsigned long long* const nc = nullptr;
  if (counts)
    hipLaunchKernelGGL((k_profile<true, FDTBX_LINESHAPE_LAUE, WAVES>), grid, block, 0, s, q, refl, nodes, pix, tile, offsets,
                       idx, image, (unsigned long long*)counts, order);
  else if (q.lineshape == FDTBX_LINESHAPE_GAUSSIAN)
    hipLaunchKernelGGL((k_profile<false, FDTBX_LINESHAPE_GAUSSIAN, WAVES>), grid, block, 0, s, q, refl, nodes, pix, tile,
                       offsets, idx, image, nc, order);
  else if (q.lineshape == FDTBX_LINESHAPE_HOSEMANN)
    hipLaunchKernelGGL((k_profile<false, FDTBX_LINESHAPE_HOSEMANN, WAVES>), grid, block, 0, s, q, refl, nodes, pix, tile,
                       offsets, idx, image, nc, order);
  else
    hipLaunchKernelGGL((k_profile<false, FDTBX_LINESHAPE_LAUE, WAVES>), grid, block, 0, s, q, refl, nodes, pix, tile, offsets,
                       idx, image, nc, order);
}

// Batched models, persistent: every wave takes (model, tile) items from a shared counter
// until the list is exhausted (the exit every wave reaches).
__global__ void __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(6))) k_b_profile(const fdtbx_batch_entry* __restrict__ ent, const int64_t* __restrict__ items,
                                                  int64_t n_items, const float* __restrict__ refl,
                                                  const float* __restrict__ nodes, const double* __restrict__ pix,
                                                  const double* __restrict__ tile, const int64_t* __restrict__ rowptr,
                                                  const int32_t* __restrict__ idx, float* __restrict__ image,
                                                  unsigned long long* __restrict__ counter) {
  __shared__ float4 qn[128];
  __shared__ int bq[64];
  __shared__ int qk[128];  // node indices of the queue (the Hosemann support edge)
  for (;;) {
    const int64_t it = next_item(counter);
    if (it >= n_items) break;
    const int64_t packed = items[it];
    const int m = (int)(packed >> 40);
    const int t = (int)(packed & ((1ll << 40) - 1));
    const fdtbx_batch_entry& e = ent[m];
    ProfParams q;
    prof_params(&e.model, &q);
    const float* rf = refl + (int64_t)FDTBX_REFL_FLOATS * e.hkl_off;
    const float* nd = nodes + (int64_t)FDTBX_NODE_FLOATS * e.node_off;
    const double* px = pix + 2 * e.pix_off;
    const double* tb = tile + 8 * e.tile_off;
    const int64_t* rp = rowptr + e.rowptr_off;
    const int32_t* ix = idx + e.pair_off;
    float* im = image + e.pix_off;
    switch (q.lineshape) {  // uniform across the wave
      case FDTBX_LINESHAPE_GAUSSIAN:
        profile_tile<false, FDTBX_LINESHAPE_GAUSSIAN, 1, true, false>(q, rf, nd, px, tb, rp, ix, im, nullptr, t, qn, bq);
        break;
      case FDTBX_LINESHAPE_HOSEMANN:
        profile_tile<false, FDTBX_LINESHAPE_HOSEMANN, 1, true, false>(q, rf, nd, px, tb, rp, ix, im, nullptr, t, qn, bq,
                                                                      nullptr, qk);
        break;
      default:
        profile_tile<false, FDTBX_LINESHAPE_LAUE, 1, true, false>(q, rf, nd, px, tb, rp, ix, im, nullptr, t, qn, bq);
    }
  }
}

// ---------------------------------------------------------------- balanced launch
// The per-tile launch ends with a tail: a tile with a long list runs as one workgroup while
// the compute units around it have drained.  The balanced launch cuts every launched tile's
// list into units of at most U pairs, which persistent waves take from eight queues, one per
// XCD: slot b of the per-tile launch order (the tile order of fdtbx_tile_order, whose slot b
// runs on XCD b % 8) puts its tile's units in queue b % 8, in slot order (heavy tiles first
// under the work order), so the units of neighbouring tiles still share an XCD's L2.  A wave
// whose queue is empty takes units from the next queues.  Each unit writes its 64 pixel sums
// to its own slot of the partial sums, and a second kernel adds a tile's units in unit order:
// the image does not depend on which wave ran which unit.
//
// Units per position (and the pairs per unit, from the pair count, by the first thread).
__global__ void __launch_bounds__(256) k_unit_count(ProfParams q, UnitTable T, const int64_t* __restrict__ offsets,
                                                    int64_t n_tiles) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t U = T.fixed_U > 0 ? T.fixed_U : default_unit_pairs(offsets[n_tiles]);
  if (p == 0) T.meta[1] = U;
  if (p < kXcds) T.ctr[p] = 0;
  if (p >= kXcds * T.nj) return;
  const int64_t b = (p % T.nj) * kXcds + p / T.nj;
  const int t = slot_tile(q, T, b);
  T.qscan[p] = t >= 0 ? ceil_div_dev(offsets[t + 1] - offsets[t], U) : 0;
}

// unit_slot over each slot's units (within the capacity).
__global__ void __launch_bounds__(256) k_unit_fill(ProfParams q, UnitTable T, const int64_t* __restrict__ offsets) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= kXcds * T.nj) return;
  const int64_t b = (p % T.nj) * kXcds + p / T.nj;
  const int t = slot_tile(q, T, b);
  if (t < 0) return;
  const int64_t U = T.meta[1];
  const int64_t n = ceil_div_dev(offsets[t + 1] - offsets[t], U), s = T.qscan[p];
  for (int64_t k = 0; k < n && s + k < T.max_units; ++k) T.unit_slot[s + k] = (int32_t)b;
}

// Persistent: every wave takes units from its XCD's queue, then from the following queues,
// until all are empty (the exit every wave reaches: each queue's counter only grows).
template <int LS>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(7))) k_profile_units(ProfParams q, const float* __restrict__ refl,
                                                       const float* __restrict__ nodes, const double* __restrict__ pix,
                                                       const double* __restrict__ tile, const int64_t* __restrict__ offsets,
                                                       const int32_t* __restrict__ idx, UnitTable T,
                                                       float* __restrict__ partials) {
  __shared__ float4 qn[256 * 4];
  __shared__ int bq[64 * 4];
  __shared__ int qk[LS == FDTBX_LINESHAPE_HOSEMANN ? 128 * 4 : 1];  // node indices (support edge)
  const int wv = (int)(threadIdx.x >> 6), lane = (int)(threadIdx.x & 63);
  const int64_t U = T.meta[1];
  const int64_t total = U > 0 ? min(T.meta[0], T.max_units) : 0;
  const int home = (int)(blockIdx.x % kXcds);
  for (int k = 0; k < kXcds; ++k) {
    const int x = (home + k) % kXcds;
    int64_t qb, qe;
    queue_span(T, x, total, &qb, &qe);
    for (;;) {
      int got = 0;
      if (lane == 0) got = atomicAdd(&T.ctr[x], 1);
      const int64_t u = qb + (int64_t)__builtin_amdgcn_readfirstlane(got);
      if (u >= qe) break;  // uniform
      int64_t p0, p1;
      const int t = unit_range(q, T, offsets, u, U, &p0, &p1);
      if (t < 0) continue;
      const TilePixel px = tile_pixel(q, pix, tile, t, lane);
      unsigned long long cnt = 0;
      partials[u * 64 + lane] = pairs_sum<false, LS>(q, refl, nodes, idx, px.box, px.R, px.Z, p0, p1, 64,
                                                     qn + 256 * wv, bq + 64 * wv, cnt,
                                                     LS == FDTBX_LINESHAPE_HOSEMANN ? qk + 128 * wv : nullptr);
    }
  }
}

// Per launched tile: its units' pixel sums added in unit order, times the Lorentz factor,
// written with the mirror folds.
__global__ void __launch_bounds__(64) k_unit_reduce(ProfParams q, UnitTable T, const double* __restrict__ pix,
                                                    const double* __restrict__ tile, const int64_t* __restrict__ offsets,
                                                    const float* __restrict__ partials, float* __restrict__ image) {
  const int64_t b = blockIdx.x;
  const int t = slot_tile(q, T, b);
  if (t < 0) return;  // uniform
  const int lane = (int)threadIdx.x;
  const TilePixel px = tile_pixel(q, pix, tile, t, lane);
  const int64_t U = T.meta[1];
  const int64_t n = U > 0 ? ceil_div_dev(offsets[t + 1] - offsets[t], U) : 0, s = T.qscan[queue_pos(b, T.nj)];
  float acc = 0.0f;
  for (int64_t k = 0; k < n && s + k < T.max_units; ++k)
    if (s + k >= 0) acc += partials[(s + k) * 64 + lane];
  if (!px.in) return;
  write_folded(q, image, px.i, px.j, px.tx, px.ty, (float)(q.delta / (px.R + q.delta)) * acc);
}

__global__ void k_zero_u64(unsigned long long* v, int n) {
  if ((int)threadIdx.x < n) v[threadIdx.x] = 0ull;
}

static constexpr unsigned kPersistentBlocks = 8192;

int launch_batch_profile(const fdtbx_batch_entry* ent, const int64_t* items, int64_t n_items, const float* refl,
                         const float* nodes, const double* pix, const double* tile, const int64_t* rowptr, const int32_t* idx,
                         float* image, int64_t* counter, hipStream_t s) {
  hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(64), 0, s, (unsigned long long*)counter, 1);
  FDTBX_LAUNCH_CHECK("batch profile counter");
  if (n_items <= 0) return FDTBX_OK;
  unsigned nb = n_items < (int64_t)kPersistentBlocks ? (unsigned)n_items : kPersistentBlocks;
  hipLaunchKernelGGL(k_b_profile, dim3(nb), dim3(64), 0, s, ent, items, n_items, refl, nodes, pix, tile, rowptr, idx, image,
                     (unsigned long long*)counter);
  FDTBX_LAUNCH_CHECK("batch profile");
  return FDTBX_OK;
}

// Batched models on stacked tiles: every wave takes (model, stacked tile) items as k_b_profile
// takes tiles.  Stacked tile s = sy tiles_x + sx holds tile rows 2 sy and 2 sy + 1 (the second
// when it is launched) of tile column sx; its box, row pointers and list start at the model's
// offsets in soff ([m][3]: first box, first row pointer, first list entry; the row pointers are
// relative to the model's first list entry).
__global__ void __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(5))) k_b_profile_stacked(const fdtbx_batch_entry* __restrict__ ent,
                                                          const int64_t* __restrict__ soff,
                                                          const int64_t* __restrict__ items, int64_t n_items,
                                                          const float* __restrict__ refl,
                                                          const float* __restrict__ nodes,
                                                          const double* __restrict__ pix,
                                                          const double* __restrict__ tile,
                                                          const double* __restrict__ stile,
                                                          const int64_t* __restrict__ srowptr,
                                                          const int32_t* __restrict__ sidx, float* __restrict__ image,
                                                          unsigned long long* __restrict__ counter) {
  __shared__ float4 qn[128];
  __shared__ int bq[64];
  __shared__ int qk[128];  // node indices of the queue (the Hosemann support edge)
  const int lane = threadIdx.x & 63;
  for (;;) {
    const int64_t it = next_item(counter);
    if (it >= n_items) break;
    const int64_t packed = items[it];
    const int m = (int)(packed >> 40);
    const int st = (int)(packed & ((1ll << 40) - 1));
    const fdtbx_batch_entry& e = ent[m];
    ProfParams q;
    prof_params(&e.model, &q);
    const double* px = pix + 2 * e.pix_off;
    const double* tb = tile + 8 * e.tile_off;
    const double* sbox = stile + 8 * (soff[3 * m] + st);
    const int64_t* rp = srowptr + soff[3 * m + 1];
    const int32_t* ix = sidx + soff[3 * m + 2];
    float* im = image + e.pix_off;
    const int sx = st % q.tiles_x, sy = st / q.tiles_x;
    const int ta = 2 * sy * q.tiles_x + sx;
    const bool two = 2 * sy + 1 < q.lrows;  // uniform
    const TilePixel pa = tile_pixel(q, px, tb, ta, lane);
    TilePixel pb = tile_pixel(q, px, tb, two ? ta + q.tiles_x : ta, lane);
    if (!two) {
      pb.in = false;
      pb.R = 1.0e30;
      pb.Z = 0.0;
    }
    const TileBox box = {sbox[0], sbox[1], sbox[2], sbox[3]};
    const float* rf = refl + (int64_t)FDTBX_REFL_FLOATS * e.hkl_off;
    const float* nd = nodes + (int64_t)FDTBX_NODE_FLOATS * e.node_off;
    const int64_t p0 = rp[st], p1 = rp[st + 1];
    float sa = 0.0f, sb = 0.0f;
    switch (q.lineshape) {  // uniform across the wave
      case FDTBX_LINESHAPE_GAUSSIAN:
        pairs_sum_stacked<FDTBX_LINESHAPE_GAUSSIAN>(q, rf, nd, ix, box, pa.R, pa.Z, pb.R, pb.Z, p0, p1, qn, bq, &sa,
                                                    &sb);
        break;
      case FDTBX_LINESHAPE_HOSEMANN:
        pairs_sum_stacked<FDTBX_LINESHAPE_HOSEMANN>(q, rf, nd, ix, box, pa.R, pa.Z, pb.R, pb.Z, p0, p1, qn, bq, &sa,
                                                    &sb, qk);
        break;
      default:
        pairs_sum_stacked<FDTBX_LINESHAPE_LAUE>(q, rf, nd, ix, box, pa.R, pa.Z, pb.R, pb.Z, p0, p1, qn, bq, &sa,
                                                &sb);
    }
    if (pa.in) write_folded(q, im, pa.i, pa.j, pa.tx, pa.ty, (float)(q.delta / (pa.R + q.delta)) * sa);
    if (pb.in) write_folded(q, im, pb.i, pb.j, pb.tx, pb.ty, (float)(q.delta / (pb.R + q.delta)) * sb);
  }
}

int launch_batch_profile_stacked(const fdtbx_batch_entry* ent, const int64_t* soff, const int64_t* items,
                                 int64_t n_items, const float* refl, const float* nodes, const double* pix,
                                 const double* tile, const double* stile, const int64_t* srowptr, const int32_t* sidx,
                                 float* image, int64_t* counter, hipStream_t s) {
  hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(64), 0, s, (unsigned long long*)counter, 1);
  FDTBX_LAUNCH_CHECK("stacked batch profile counter");
  if (n_items <= 0) return FDTBX_OK;
  unsigned nb = n_items < (int64_t)kPersistentBlocks ? (unsigned)n_items : kPersistentBlocks;
  hipLaunchKernelGGL(k_b_profile_stacked, dim3(nb), dim3(64), 0, s, ent, soff, items, n_items, refl, nodes, pix, tile,
                     stile, srowptr, sidx, image, (unsigned long long*)counter);
  FDTBX_LAUNCH_CHECK("stacked batch profile");
  return FDTBX_OK;
}

// The persistent grid: as many 4-wave workgroups as the compute units hold at once.
template <int LS>
static int launch_units(const ProfParams& q, const float* refl, const float* nodes, const double* pix,
                        const double* tile, const int64_t* offsets, const int32_t* idx, const UnitTable& T,
                        float* partials, hipStream_t s) {
  int dev = 0, cus = 0, per_cu = 0;
  FDTBX_HIP(hipGetDevice(&dev));
  FDTBX_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  FDTBX_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void*>(&k_profile_units<LS>),
                                                         256, 0));
  const unsigned n_wg = (unsigned)(cus > 0 ? cus : 1) * (unsigned)(per_cu > 0 ? per_cu : 1);
  hipLaunchKernelGGL(k_profile_units<LS>, dim3(n_wg), dim3(256), 0, s, q, refl, nodes, pix, tile, offsets, idx, T,
                     partials);
  FDTBX_LAUNCH_CHECK("balanced profile");
  return FDTBX_OK;
}

size_t balanced_workspace(const fdtbx_model* model, int64_t pair_cap) {
  ProfParams q;
  prof_params(model, &q);
  const int64_t U = model->geom.unit_pairs;
  const UnitLayout a = unit_layout(q, true, pair_cap, U), b = unit_layout(q, false, pair_cap, U);
  return a.total > b.total ? a.total : b.total;
}

int launch_balanced(const fdtbx_model* model, const float* refl, const float* nodes, const double* pix,
                    const double* tile, const int64_t* offsets, const int32_t* idx, const int32_t* order,
                    int64_t pair_cap, float* image, void* ws, size_t ws_bytes, hipStream_t s) {
  ProfParams q;
  prof_params(model, &q);
  const UnitLayout L = unit_layout(q, order != nullptr, pair_cap, model->geom.unit_pairs);
  if (ws_bytes < L.total) return fail(FDTBX_ERR_BUFFER_TOO_SMALL, "balanced profile workspace too small");
  if (L.max_units >= (int64_t{1} << 31) || L.n_slots >= (int64_t{1} << 31))
    return fail(FDTBX_ERR_UNSUPPORTED, "balanced profile: too many units or tiles");
  const UnitTable T = unit_view(L, order, model->geom.unit_pairs, ws);
  float* partials = (float*)((char*)ws + L.partials);
  const int64_t n_tiles = (int64_t)q.tiles_x * q.tiles_y;
  const unsigned gp = (unsigned)ceil_div(kXcds * L.nj, 256);
  hipLaunchKernelGGL(k_unit_count, dim3(gp), dim3(256), 0, s, q, T, offsets, n_tiles);
  FDTBX_LAUNCH_CHECK("balanced profile: unit count");
  hipLaunchKernelGGL(k_scan_inplace, dim3(1), dim3(1024), 0, s, T.qscan, kXcds * L.nj, T.meta);
  FDTBX_LAUNCH_CHECK("balanced profile: unit scan");
  hipLaunchKernelGGL(k_unit_fill, dim3(gp), dim3(256), 0, s, q, T, offsets);
  FDTBX_LAUNCH_CHECK("balanced profile: unit fill");
  int rc;
  if (q.lineshape == FDTBX_LINESHAPE_GAUSSIAN)
    rc = launch_units<FDTBX_LINESHAPE_GAUSSIAN>(q, refl, nodes, pix, tile, offsets, idx, T, partials, s);
  else if (q.lineshape == FDTBX_LINESHAPE_HOSEMANN)
    rc = launch_units<FDTBX_LINESHAPE_HOSEMANN>(q, refl, nodes, pix, tile, offsets, idx, T, partials, s);
  else
    rc = launch_units<FDTBX_LINESHAPE_LAUE>(q, refl, nodes, pix, tile, offsets, idx, T, partials, s);
  if (rc) return rc;
  hipLaunchKernelGGL(k_unit_reduce, dim3((unsigned)L.n_slots), dim3(64), 0, s, q, T, pix, tile, offsets,
                     (const float*)partials, image);
  FDTBX_LAUNCH_CHECK("balanced profile: reduce");
  return FDTBX_OK;
}

}  // namespace fdtbx

using namespace fdtbx;

extern "C" int fdtbx_profile(const fdtbx_model* model, const float* refl, const float* nodes, const double* pix,
                             const double* tile, const int64_t* offsets, const int32_t* idx, const int32_t* order,
                             float* image, int64_t* counts, void* stream) {
  if (!model || !refl || !nodes || !pix || !tile || !offsets || !idx) return fail(FDTBX_ERR_INVALID_ARGUMENT, "null pointer");
  if (!counts && !image) return fail(FDTBX_ERR_INVALID_ARGUMENT, "image is NULL");
  int rc = check_model(model);
  if (rc) return rc;
  ProfParams q;
  prof_params(model, &q);
  hipStream_t s = (hipStream_t)stream;
  const dim3 grid((unsigned)(order ? order_grid(q.lcols, q.lrows) : tile_grid(q)));
  int waves = 1;
  rc = tile_waves(&model->geom, (int64_t)q.lcols * q.lrows, &waves);
  if (rc) return rc;
  if (waves == 4)
    launch_profile<4>(q, grid, s, refl, nodes, pix, tile, offsets, idx, order, image, counts);
  else if (waves == 2)
    launch_profile<2>(q, grid, s, refl, nodes, pix, tile, offsets, idx, order, image, counts);
  else
    launch_profile<1>(q, grid, s, refl, nodes, pix, tile, offsets, idx, order, image, counts);
  FDTBX_LAUNCH_CHECK("profile");
  return FDTBX_OK;
}

extern "C" int64_t fdtbx_unit_pairs(int64_t n_pairs) { return n_pairs < 0 ? 0 : default_unit_pairs(n_pairs); }

extern "C" size_t fdtbx_profile_balanced_workspace(const fdtbx_model* model, int64_t pair_cap) {
  if (!model || pair_cap < 0 || check_model(model)) return 0;
  if (model->geom.unit_pairs < 0) return 0;
  return balanced_workspace(model, pair_cap);
}

extern "C" int fdtbx_profile_balanced(const fdtbx_model* model, const float* refl, const float* nodes,
                                      const double* pix, const double* tile, const int64_t* offsets,
                                      const int32_t* idx, const int32_t* order, int64_t pair_cap, float* image,
                                      void* ws, size_t ws_bytes, void* stream) {
  if (!model || !refl || !nodes || !pix || !tile || !offsets || !idx || !image || !ws)
    return fail(FDTBX_ERR_INVALID_ARGUMENT, "null pointer");
  if (pair_cap < 0) return fail(FDTBX_ERR_INVALID_ARGUMENT, "pair_cap must be non-negative");
  int rc = check_model(model);
  if (rc) return rc;
  if (model->geom.unit_pairs < 0) return fail(FDTBX_ERR_INVALID_ARGUMENT, "unit_pairs must be non-negative");
  return launch_balanced(model, refl, nodes, pix, tile, offsets, idx, order, pair_cap, image, ws, ws_bytes,
                         (hipStream_t)stream);
}
