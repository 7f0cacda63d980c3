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
__global__ void __launch_bounds__(64 * WAVES) k_profile(ProfParams q, const float* __restrict__ refl,
                                                        const float* __restrict__ nodes, const double* __restrict__ pix,
                                                        const double* __restrict__ tile, const int64_t* __restrict__ offsets,
                                                        const int32_t* __restrict__ idx, float* __restrict__ image,
                                                        unsigned long long* __restrict__ counts,
                                                        const int32_t* __restrict__ order) {
  // per wave, the queue of window nodes that can be inside the support of some pixel of the tile
  __shared__ float4 qn[128 * WAVES];
  __shared__ int bq[64 * WAVES];
  __shared__ float xacc[WAVES > 1 ? 64 * (WAVES - 1) : 1];
  const int t = order ? order[blockIdx.x] : tile_of_block(q, blockIdx.x);
  if (t < 0) return;  // uniform across the workgroup
  profile_tile<COUNT, LS, WAVES>(q, refl, nodes, pix, tile, offsets, idx, image, counts, t, qn, bq, xacc);
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
__global__ void __launch_bounds__(64) k_b_profile(const fdtbx_batch_entry* __restrict__ ent, const int64_t* __restrict__ items,
                                                  int64_t n_items, const float* __restrict__ refl,
                                                  const float* __restrict__ nodes, const double* __restrict__ pix,
                                                  const double* __restrict__ tile, const int64_t* __restrict__ rowptr,
                                                  const int32_t* __restrict__ idx, float* __restrict__ image,
                                                  unsigned long long* __restrict__ counter) {
  __shared__ float4 qn[128];
  __shared__ int bq[64];
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
        profile_tile<false, FDTBX_LINESHAPE_GAUSSIAN, 1>(q, rf, nd, px, tb, rp, ix, im, nullptr, t, qn, bq);
        break;
      case FDTBX_LINESHAPE_HOSEMANN:
        profile_tile<false, FDTBX_LINESHAPE_HOSEMANN, 1>(q, rf, nd, px, tb, rp, ix, im, nullptr, t, qn, bq);
        break;
      default:
        profile_tile<false, FDTBX_LINESHAPE_LAUE, 1>(q, rf, nd, px, tb, rp, ix, im, nullptr, t, qn, bq);
    }
  }
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
