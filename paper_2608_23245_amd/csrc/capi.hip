// Host side of the C ABI: argument checks, error reporting, and the one-call
// pattern entry point that chains the building blocks on one stream.
#include <hip/hip_runtime.h>

#include <math.h>

#include <mutex>

#include "internal.h"

namespace fdtbx {

static thread_local const char* g_msg = "no error";
static thread_local int g_hip = 0;

int fail(int code, const char* msg) {
  g_msg = msg;
  return code;
}

int hip_fail(hipError_t e, const char* where) {
  g_hip = (int)e;
  g_msg = where;
  return FDTBX_ERR_HIP;
}

bool finite_pos(double v) { return isfinite(v) && v > 0.0; }

int check_cell(const fdtbx_cell* c) {
  if (!c) return fail(FDTBX_ERR_INVALID_ARGUMENT, "null cell");
  if (!finite_pos(c->a) || !finite_pos(c->b) || !finite_pos(c->c))
    return fail(FDTBX_ERR_GEOMETRY, "cell edges must be positive and finite");
  const double angs[3] = {c->alpha, c->beta, c->gamma};
  for (double a : angs)
    if (!(isfinite(a) && a > 0.0 && a < M_PI)) return fail(FDTBX_ERR_GEOMETRY, "cell angles must be in (0, pi) radians");
  double ca = cos(c->alpha), cb = cos(c->beta), cg = cos(c->gamma);
  if (!(1.0 - ca * ca - cb * cb - cg * cg + 2.0 * ca * cb * cg > 1e-12))
    return fail(FDTBX_ERR_GEOMETRY, "cell angles do not span a parallelepiped");
  return FDTBX_OK;
}

int check_geometry(const fdtbx_geometry* g) {
  if (!g) return fail(FDTBX_ERR_INVALID_ARGUMENT, "null geometry");
  if (!finite_pos(g->wavelength) || !finite_pos(g->distance) || !finite_pos(g->pixel))
    return fail(FDTBX_ERR_GEOMETRY, "wavelength, distance and pixel must be positive and finite");
  if (g->width < 1 || g->height < 1 || g->width > 65536 || g->height > 65536)
    return fail(FDTBX_ERR_INVALID_ARGUMENT, "detector size must be in 1..65536 pixels");
  if (!isfinite(g->center_x) || !isfinite(g->center_y)) return fail(FDTBX_ERR_INVALID_ARGUMENT, "beam centre not finite");
  if (!(fabs(g->tilt) < 0.5 * M_PI)) return fail(FDTBX_ERR_GEOMETRY, "fibre tilt must be finite with |tilt| < pi/2");
  if (!(fabs(g->det_tilt) < 0.5 * M_PI))
    return fail(FDTBX_ERR_GEOMETRY, "detector tilt must be finite with |det_tilt| < pi/2");
  if (g->det_tilt != 0.0) {  // the outermost rows must face the sample
    const double sd = sin(g->det_tilt);
    const double z0 = (0.5 - g->center_y) * g->pixel, z1 = (((double)g->height - 0.5) - g->center_y) * g->pixel;
    if (!(g->distance - z0 * sd > 0.0) || !(g->distance - z1 * sd > 0.0))
      return fail(FDTBX_ERR_GEOMETRY, "detector tilt puts pixel rows behind the sample");
  }
  const int32_t tw = g->tile_w;
  if (!(tw == 0 || tw == 2 || tw == 4 || tw == 8 || tw == 16 || tw == 32))
    return fail(FDTBX_ERR_INVALID_ARGUMENT, "tile_w must be 0, 2, 4, 8, 16 or 32");
  if (g->mirror < 0 || g->mirror > 3) return fail(FDTBX_ERR_INVALID_ARGUMENT, "mirror must be 0, 1, 2 or 3");
  if (!(g->tile_waves == 0 || g->tile_waves == 1 || g->tile_waves == 2 || g->tile_waves == 4))
    return fail(FDTBX_ERR_INVALID_ARGUMENT, "tile_waves must be 0, 1, 2 or 4");
  const int32_t tww = tw ? tw : FDTBX_TILE;
  if ((g->mirror & 1) && !(g->center_x == 0.5 * g->width && g->width % tww == 0))
    return fail(FDTBX_ERR_INVALID_ARGUMENT, "the left-right fold needs center_x = width/2 and width a multiple of tile_w");
  if ((g->mirror & 2) &&
      !(g->center_y == 0.5 * g->height && g->tilt == 0.0 && g->det_tilt == 0.0 && g->height % (64 / tww) == 0))
    return fail(FDTBX_ERR_INVALID_ARGUMENT,
                "the up-down fold needs center_y = height/2, no fibre or detector tilt and height a multiple of 64/tile_w");
  return FDTBX_OK;
}

int check_model(const fdtbx_model* m) {
  if (!m) return fail(FDTBX_ERR_INVALID_ARGUMENT, "null model");
  int rc = check_cell(&m->cell);
  if (rc) return rc;
  rc = check_geometry(&m->geom);
  if (rc) return rc;
  const fdtbx_disorder& d = m->dis;
  if (!(isfinite(d.sigma_theta) && d.sigma_theta >= 0) || !(isfinite(d.gamma_theta) && d.gamma_theta >= 0))
    return fail(FDTBX_ERR_INVALID_ARGUMENT, "angular widths must be finite and non-negative");
  if (d.sigma_theta == 0.0 && d.gamma_theta == 0.0)
    return fail(FDTBX_ERR_INVALID_ARGUMENT, "sigma_theta and gamma_theta are both zero");
  for (int i = 0; i < 3; ++i) {
    if (!finite_pos(d.N_base[i])) return fail(FDTBX_ERR_INVALID_ARGUMENT, "N_base must be positive and finite");
    if (!(isfinite(d.g[i]) && d.g[i] >= 0.0 && d.g[i] < 1.0)) return fail(FDTBX_ERR_INVALID_ARGUMENT, "g must be in [0, 1)");
  }
  if (d.intensity_model != 0 && d.intensity_model != 1) return fail(FDTBX_ERR_INVALID_ARGUMENT, "intensity_model must be 0 or 1");
  if (d.lineshape < FDTBX_LINESHAPE_LAUE || d.lineshape > FDTBX_LINESHAPE_HOSEMANN)
    return fail(FDTBX_ERR_INVALID_ARGUMENT, "lineshape must be FDTBX_LINESHAPE_LAUE, _GAUSSIAN or _HOSEMANN");
  for (int i = 0; i < 3; ++i)
    if (!isfinite(d.B_axis[i])) return fail(FDTBX_ERR_INVALID_ARGUMENT, "B_axis must be finite");
  const fdtbx_quadrature& q = m->quad;
  if (q.n_nodes < 1 || q.n_nodes > 256) return fail(FDTBX_ERR_INVALID_ARGUMENT, "n_nodes must be in 1..256");
  if (!(q.T > 0.0 && q.T < 10.0)) return fail(FDTBX_ERR_INVALID_ARGUMENT, "T must be in (0, 10)");
  if (!finite_pos(q.sigma_r)) return fail(FDTBX_ERR_INVALID_ARGUMENT, "sigma_r must be positive");
  if (q.m < 1 || q.m > 8) return fail(FDTBX_ERR_INVALID_ARGUMENT, "m must be in 1..8");
  if (!finite_pos(q.delta)) return fail(FDTBX_ERR_INVALID_ARGUMENT, "delta must be positive");
  if (!finite_pos(q.d_min)) return fail(FDTBX_ERR_INVALID_ARGUMENT, "d_min must be positive");
  if (isnan(q.d_max) || (q.d_max > 0 && !(q.d_max > q.d_min))) return fail(FDTBX_ERR_INVALID_ARGUMENT, "d_max must exceed d_min");
  if (!isfinite(q.extinction)) return fail(FDTBX_ERR_INVALID_ARGUMENT, "extinction limit must be finite");
  return FDTBX_OK;
}

struct PatternLayout {
  size_t refl, cull, nodes, pix, tile, offsets, cullws, order, orderws, idx, total;
};

static PatternLayout layout(const fdtbx_model* m, int64_t n_hkl, int64_t pair_cap) {
  PatternLayout L;
  int64_t tiles = (int64_t)tiles_x_of(&m->geom) * tiles_y_of(&m->geom);
  size_t o = 0;
  L.refl = o;
  o += align_up((size_t)n_hkl * FDTBX_REFL_FLOATS * sizeof(float), 256);
  L.cull = o;
  o += align_up((size_t)n_hkl * FDTBX_CULL_DOUBLES * sizeof(double), 256);
  L.nodes = o;
  o += align_up((size_t)node_rows(m->quad.n_nodes) * FDTBX_NODE_FLOATS * sizeof(float), 256);
  L.pix = o;
  o += align_up((size_t)m->geom.width * m->geom.height * 2 * sizeof(double), 256);
  L.tile = o;
  o += align_up((size_t)tiles * 8 * sizeof(double), 256);
  L.offsets = o;
  o += align_up((size_t)(tiles + 1) * sizeof(int64_t), 256);
  // the culling workspace, and after the culling the balanced launch's unit tables and sums
  L.cullws = o;
  const size_t cw = fdtbx_cull_workspace(&m->geom, n_hkl), bw = balanced_workspace(m, pair_cap);
  o += align_up(cw > bw ? cw : bw, 256);
  L.order = o;
  o += align_up((size_t)fdtbx_tile_order_size(&m->geom) * sizeof(int32_t), 256);
  L.orderws = o;
  o += align_up(fdtbx_tile_order_workspace(&m->geom), 256);
  L.idx = o;
  o += align_up((size_t)(pair_cap > 0 ? pair_cap : 1) * sizeof(int32_t), 256);
  L.total = o;
  return L;
}

}  // namespace fdtbx

using namespace fdtbx;

extern "C" const char* fdtbx_error_string(int code) {
  if (code == FDTBX_OK) return "ok";
  return g_msg;
}

extern "C" int fdtbx_last_hip_error(void) { return g_hip; }

// Waves per tile of a profile launch over n_tiles tiles: the geometry's tile_waves, or the
// library's choice.
// The library's choice: a launch of a few rounds of one-wave workgroups (32 per compute unit)
// ends with its longest tiles, so 4 waves share each tile up to eight rounds (measured best or
// equal from half a round, the medium workload under both mirror folds, to eight, the unfolded
// large one); beyond that, 2.
int fdtbx::tile_waves(const fdtbx_geometry* g, int64_t n_tiles, int* waves) {
  if (g->tile_waves) {
    *waves = g->tile_waves;
    return FDTBX_OK;
  }
  int dev = 0, cus = 256;
  FDTBX_HIP(hipGetDevice(&dev));
  FDTBX_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  const int64_t round = (int64_t)cus * 32;
  *waves = n_tiles <= 8 * round ? 4 : 2;
  return FDTBX_OK;
}

extern "C" int fdtbx_launch_waves(const fdtbx_geometry* geom, int32_t* waves) {
  if (!geom || !waves) return fail(FDTBX_ERR_INVALID_ARGUMENT, "null pointer");
  int rc = check_geometry(geom);
  if (rc) return rc;
  int w = 1;
  rc = tile_waves(geom, (int64_t)lcols_of(geom) * lrows_of(geom), &w);
  *waves = w;
  return rc;
}

extern "C" int fdtbx_tile_grid(const fdtbx_geometry* geom, int32_t* tiles_x, int32_t* tiles_y) {
  if (!geom || !tiles_x || !tiles_y) return fail(FDTBX_ERR_INVALID_ARGUMENT, "null pointer");
  int rc = check_geometry(geom);
  if (rc) return rc;
  *tiles_x = tiles_x_of(geom);
  *tiles_y = tiles_y_of(geom);
  return FDTBX_OK;
}

extern "C" size_t fdtbx_pattern_workspace(const fdtbx_model* model, int64_t n_hkl, int64_t pair_cap) {
  if (!model || check_model(model) || n_hkl < 0 || pair_cap < 0) return 0;
  return layout(model, n_hkl, pair_cap).total;
}

extern "C" int fdtbx_profile_pattern(const fdtbx_model* model, const int32_t* hkl, int64_t n_hkl, const float* F2,
                                     float* image, int64_t pair_cap, int64_t* pairs_needed, void* ws, size_t ws_bytes,
                                     void* stream) {
  if (!model || !image || !ws) return fail(FDTBX_ERR_INVALID_ARGUMENT, "null pointer");
  if (n_hkl < 0) return fail(FDTBX_ERR_INVALID_ARGUMENT, "n_hkl must be non-negative");
  if (pair_cap < 0) return fail(FDTBX_ERR_INVALID_ARGUMENT, "pair_cap must be non-negative");
  int rc = check_model(model);
  if (rc) return rc;
  if (n_hkl > 0 && (!hkl || !F2)) return fail(FDTBX_ERR_INVALID_ARGUMENT, "null pointer");
  PatternLayout L = layout(model, n_hkl, pair_cap);
  if (ws_bytes < L.total) return fail(FDTBX_ERR_BUFFER_TOO_SMALL, "pattern workspace too small");
  char* w = (char*)ws;
  float* refl = (float*)(w + L.refl);
  double* cull = (double*)(w + L.cull);
  float* nodes = (float*)(w + L.nodes);
  double* pix = (double*)(w + L.pix);
  double* tile = (double*)(w + L.tile);
  int64_t* offsets = (int64_t*)(w + L.offsets);
  int32_t* idx = (int32_t*)(w + L.idx);
  int32_t* order = (int32_t*)(w + L.order);
  rc = fdtbx_reflection_prep(model, hkl, n_hkl, F2, refl, cull, stream);
  if (rc) return rc;
  rc = fdtbx_node_table(&model->dis, &model->quad, nodes, stream);
  if (rc) return rc;
  rc = fdtbx_pixel_map(&model->geom, pix, tile, stream);
  if (rc) return rc;
  int64_t n_pairs = 0;
  rc = fdtbx_cull(&model->geom, tile, n_hkl, cull, offsets, idx, pair_cap, &n_pairs, w + L.cullws,
                  fdtbx_cull_workspace(&model->geom, n_hkl), stream);
  if (pairs_needed) *pairs_needed = n_pairs;
  if (rc) return rc;
  rc = fdtbx_tile_order(&model->geom, offsets, order, w + L.orderws, fdtbx_tile_order_workspace(&model->geom), stream);
  if (rc) return rc;
  return launch_balanced(model, refl, nodes, pix, tile, offsets, idx, order, pair_cap, image, w + L.cullws,
                         balanced_workspace(model, pair_cap), (hipStream_t)stream);
}

namespace fdtbx {
// The statistics' fixed fields and the first stamp.
__global__ void k_stats_begin(fdtbx_stats* st, int64_t n_hkl, int64_t pair_cap, int64_t khz, int32_t counted) {
  if (threadIdx.x != 0) return;
  st->n_hkl = n_hkl;
  st->n_pairs = 0;
  st->pair_cap = pair_cap;
  st->useful_evals = counted ? 0 : -1;
  st->overflow = 0;
  st->n_stamps = FDTBX_STATS_STAMPS;
  st->clock_khz = khz;
  for (int k = 0; k < FDTBX_STATS_STAMPS; ++k) st->stamp[k] = 0;
  st->stamp[0] = wall_clock64();
}

// Stamp k: the kernels of the steps before it have finished (same stream).
__global__ void k_stamp(fdtbx_stats* st, int k) {
  if (threadIdx.x == 0) st->stamp[k] = wall_clock64();
}
}  // namespace fdtbx

extern "C" int fdtbx_profile_pattern_async(const fdtbx_model* model, const int32_t* hkl, int64_t n_hkl, const float* F2,
                                           float* image, int64_t pair_cap, int32_t count_evals, fdtbx_stats* stats,
                                           void* ws, size_t ws_bytes, void* stream) {
  if (!model || !image || !ws) return fail(FDTBX_ERR_INVALID_ARGUMENT, "null pointer");
  if (n_hkl < 0) return fail(FDTBX_ERR_INVALID_ARGUMENT, "n_hkl must be non-negative");
  if (pair_cap < 0) return fail(FDTBX_ERR_INVALID_ARGUMENT, "pair_cap must be non-negative");
  int rc = check_model(model);
  if (rc) return rc;
  if (n_hkl > 0 && (!hkl || !F2)) return fail(FDTBX_ERR_INVALID_ARGUMENT, "null pointer");
  PatternLayout L = layout(model, n_hkl, pair_cap);
  if (ws_bytes < L.total) return fail(FDTBX_ERR_BUFFER_TOO_SMALL, "pattern workspace too small");
  hipStream_t s = (hipStream_t)stream;
  int khz = 0;
  if (stats) {
    int dev = 0;
    FDTBX_HIP(hipGetDevice(&dev));
    FDTBX_HIP(hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev));
    hipLaunchKernelGGL(k_stats_begin, dim3(1), dim3(64), 0, s, stats, n_hkl, pair_cap, (int64_t)khz, count_evals ? 1 : 0);
    FDTBX_LAUNCH_CHECK("stats");
  }
  auto stamp = [&](int k) -> int {
    if (!stats) return FDTBX_OK;
    hipLaunchKernelGGL(k_stamp, dim3(1), dim3(64), 0, s, stats, k);
    FDTBX_LAUNCH_CHECK("stats stamp");
    return FDTBX_OK;
  };
  char* w = (char*)ws;
  float* refl = (float*)(w + L.refl);
  double* cull = (double*)(w + L.cull);
  float* nodes = (float*)(w + L.nodes);
  double* pix = (double*)(w + L.pix);
  double* tile = (double*)(w + L.tile);
  int64_t* offsets = (int64_t*)(w + L.offsets);
  int32_t* idx = (int32_t*)(w + L.idx);
  int32_t* order = (int32_t*)(w + L.order);
  rc = fdtbx_reflection_prep(model, hkl, n_hkl, F2, refl, cull, stream);
  if (rc || (rc = stamp(1))) return rc;
  rc = fdtbx_node_table(&model->dis, &model->quad, nodes, stream);
  if (rc || (rc = stamp(2))) return rc;
  rc = fdtbx_pixel_map(&model->geom, pix, tile, stream);
  if (rc || (rc = stamp(3))) return rc;
  rc = cull_on_device(&model->geom, tile, n_hkl, cull, offsets, idx, pair_cap, stats, w + L.cullws,
                      fdtbx_cull_workspace(&model->geom, n_hkl), s);
  if (rc || (rc = stamp(4))) return rc;
  rc = fdtbx_tile_order(&model->geom, offsets, order, w + L.orderws, fdtbx_tile_order_workspace(&model->geom), stream);
  if (rc || (rc = stamp(5))) return rc;
  rc = launch_balanced(model, refl, nodes, pix, tile, offsets, idx, order, pair_cap, image, w + L.cullws,
                       balanced_workspace(model, pair_cap), s);
  if (rc || (rc = stamp(6))) return rc;
  if (count_evals && stats) {
    rc = fdtbx_profile(model, refl, nodes, pix, tile, offsets, idx, order, nullptr, &stats->useful_evals, stream);
    if (rc) return rc;
  }
  return stamp(7);
}

extern "C" size_t fdtbx_backward_workspace(int64_t n_hkl, int64_t n_atoms) {
  if (n_hkl < 0) return 0;
  if (n_hkl == 0) return 256;  // nothing is used; a non-zero size keeps callers' allocations valid
  size_t b = align_up((size_t)n_hkl * 6 * sizeof(double), 256);
  b += align_up(fdtbx_adjoint_finish_workspace(n_hkl), 256);
  b += align_up((size_t)n_hkl * sizeof(float), 256);
  b += 256;  // queue counters of the balanced adjoint launch
  if (n_atoms > 0) b += align_up(fdtbx_sf_adjoint_workspace(n_hkl, n_atoms), 256);
  return b;
}

extern "C" int fdtbx_pattern_backward(const fdtbx_model* model, const int32_t* hkl, int64_t n_hkl, const float* F,
                                      const float* grad_image, const void* fwd_ws, size_t fwd_ws_bytes, int64_t pair_cap,
                                      int64_t n_atoms, const float* x, const float* y, const float* z, const float* B,
                                      const float* occ, const int32_t* type, const float* ff, int32_t n_types, float* d_x,
                                      float* d_y, float* d_z, float* d_B, float* d_occ, double* d_globals, float* dF2,
                                      void* ws, size_t ws_bytes, void* stream) {
  if (!model || !grad_image || !fwd_ws || !d_globals || !ws) return fail(FDTBX_ERR_INVALID_ARGUMENT, "null pointer");
  if (n_hkl < 0 || pair_cap < 0) return fail(FDTBX_ERR_INVALID_ARGUMENT, "bad sizes");
  int rc = check_model(model);
  if (rc) return rc;
  const bool atoms = d_x || d_y || d_z || d_B || d_occ;
  if (n_hkl == 0) {  // no reflections: every gradient is zero
    hipStream_t s0 = (hipStream_t)stream;
    rc = fill(d_globals, (int64_t)FDTBX_N_GLOBALS, 0.0, s0);
    if (rc || !atoms) return rc;
    float* const outs[5] = {d_x, d_y, d_z, d_B, d_occ};
    for (float* o : outs) {
      rc = fill(o, n_atoms, 0.0f, s0);
      if (rc) return rc;
    }
    return FDTBX_OK;
  }
  if (!hkl || !F) return fail(FDTBX_ERR_INVALID_ARGUMENT, "null pointer");
  if (atoms && (n_atoms <= 0 || !x || !y || !z || !B || !occ || !type || !ff))
    return fail(FDTBX_ERR_INVALID_ARGUMENT, "atom arrays required for atom gradients");
  PatternLayout L = layout(model, n_hkl, pair_cap);
  if (fwd_ws_bytes < L.total) return fail(FDTBX_ERR_BUFFER_TOO_SMALL, "forward workspace smaller than the layout for pair_cap");
  if (ws_bytes < fdtbx_backward_workspace(n_hkl, atoms ? n_atoms : 0)) return fail(FDTBX_ERR_BUFFER_TOO_SMALL, "backward workspace too small");
  const char* fw = (const char*)fwd_ws;
  const float* refl = (const float*)(fw + L.refl);
  const float* nodes = (const float*)(fw + L.nodes);
  const double* pix = (const double*)(fw + L.pix);
  const double* tile = (const double*)(fw + L.tile);
  const int64_t* offsets = (const int64_t*)(fw + L.offsets);
  const int32_t* idx = (const int32_t*)(fw + L.idx);
  const int32_t* order = (const int32_t*)(fw + L.order);
  char* w = (char*)ws;
  double* sums = (double*)w;
  w += align_up((size_t)n_hkl * 6 * sizeof(double), 256);
  void* fin = w;
  size_t fin_bytes = fdtbx_adjoint_finish_workspace(n_hkl);
  w += align_up(fin_bytes, 256);
  float* g2 = dF2 ? dF2 : (float*)w;
  w += align_up((size_t)n_hkl * sizeof(float), 256);
  int32_t* ctr = (int32_t*)w;
  w += 256;
  hipStream_t s = (hipStream_t)stream;
  rc = fill(sums, 6 * n_hkl, 0.0, s);
  if (rc) return rc;
  // the work units of the balanced forward launch, still in the forward workspace
  rc = launch_adjoint_units(model, refl, nodes, pix, tile, offsets, idx, order, pair_cap, fw + L.cullws, ctr, n_hkl,
                            grad_image, sums, nullptr, s);
  if (rc) return rc;
  rc = fdtbx_adjoint_finish(model, hkl, n_hkl, refl, sums, F, g2, d_globals, fin, fin_bytes, stream);
  if (rc) return rc;
  if (!atoms) return FDTBX_OK;
  return fdtbx_sf_adjoint(&model->cell, n_atoms, x, y, z, B, occ, type, ff, n_types, hkl, n_hkl, F, g2, d_x, d_y, d_z, d_B,
                          d_occ, w, fdtbx_sf_adjoint_workspace(n_hkl, n_atoms), stream);
}

extern "C" size_t fdtbx_backward_deterministic_workspace(int64_t n_hkl, int64_t n_atoms, int64_t pair_cap) {
  if (n_hkl < 0 || pair_cap < 0) return 0;
  size_t b = fdtbx_backward_workspace(n_hkl, n_atoms);
  if (n_hkl == 0) return b;
  const size_t t = fdtbx_pair_transpose_workspace(n_hkl, pair_cap);
  if (t == 0) return 0;
  b += align_up((size_t)pair_cap * 12 * sizeof(float), 256);       // per-pair partials
  b += align_up((size_t)(n_hkl + 1) * sizeof(int64_t), 256);      // reflection row pointers
  b += align_up((size_t)pair_cap * sizeof(int32_t), 256);         // pairs in reflection order
  b += align_up(t, 256);
  return b;
}

extern "C" int fdtbx_pattern_backward_deterministic(
    const fdtbx_model* model, const int32_t* hkl, int64_t n_hkl, const float* F, const float* grad_image,
    const void* fwd_ws, size_t fwd_ws_bytes, int64_t pair_cap, int64_t n_atoms, const float* x, const float* y,
    const float* z, const float* B, const float* occ, const int32_t* type, const float* ff, int32_t n_types, float* d_x,
    float* d_y, float* d_z, float* d_B, float* d_occ, double* d_globals, float* dF2, void* ws, size_t ws_bytes,
    void* stream) {
  if (!model || !grad_image || !fwd_ws || !d_globals || !ws) return fail(FDTBX_ERR_INVALID_ARGUMENT, "null pointer");
  if (n_hkl < 0 || pair_cap < 0) return fail(FDTBX_ERR_INVALID_ARGUMENT, "bad sizes");
  int rc = check_model(model);
  if (rc) return rc;
  const bool atoms = d_x || d_y || d_z || d_B || d_occ;
  if (n_hkl == 0)  // no reflections: every gradient is zero, as in fdtbx_pattern_backward
    return fdtbx_pattern_backward(model, hkl, n_hkl, F, grad_image, fwd_ws, fwd_ws_bytes, pair_cap, n_atoms, x, y, z, B,
                                  occ, type, ff, n_types, d_x, d_y, d_z, d_B, d_occ, d_globals, dF2, ws, ws_bytes, stream);
  if (!hkl || !F) return fail(FDTBX_ERR_INVALID_ARGUMENT, "null pointer");
  if (atoms && (n_atoms <= 0 || !x || !y || !z || !B || !occ || !type || !ff))
    return fail(FDTBX_ERR_INVALID_ARGUMENT, "atom arrays required for atom gradients");
  PatternLayout L = layout(model, n_hkl, pair_cap);
  if (fwd_ws_bytes < L.total) return fail(FDTBX_ERR_BUFFER_TOO_SMALL, "forward workspace smaller than the layout for pair_cap");
  const size_t need = fdtbx_backward_deterministic_workspace(n_hkl, atoms ? n_atoms : 0, pair_cap);
  if (need == 0) return fail(FDTBX_ERR_UNSUPPORTED, "deterministic backward: pair_cap or n_hkl too large");
  if (ws_bytes < need) return fail(FDTBX_ERR_BUFFER_TOO_SMALL, "backward workspace too small");
  const char* fw = (const char*)fwd_ws;
  const float* refl = (const float*)(fw + L.refl);
  const float* nodes = (const float*)(fw + L.nodes);
  const double* pix = (const double*)(fw + L.pix);
  const double* tile = (const double*)(fw + L.tile);
  const int64_t* offsets = (const int64_t*)(fw + L.offsets);
  const int32_t* idx = (const int32_t*)(fw + L.idx);
  const int32_t* order = (const int32_t*)(fw + L.order);
  int32_t tiles_x = 0, tiles_y = 0;
  rc = fdtbx_tile_grid(&model->geom, &tiles_x, &tiles_y);
  if (rc) return rc;
  const int64_t* n_pairs_dev = offsets + (int64_t)tiles_x * tiles_y;  // the total, written by fdtbx_cull
  char* w = (char*)ws;
  double* sums = (double*)w;
  w += align_up((size_t)n_hkl * 6 * sizeof(double), 256);
  void* fin = w;
  const size_t fin_bytes = fdtbx_adjoint_finish_workspace(n_hkl);
  w += align_up(fin_bytes, 256);
  float* g2 = dF2 ? dF2 : (float*)w;
  w += align_up((size_t)n_hkl * sizeof(float), 256);
  int32_t* ctr = (int32_t*)w;
  w += 256;
  void* sfw = w;
  if (atoms) w += align_up(fdtbx_sf_adjoint_workspace(n_hkl, n_atoms), 256);
  float* partials = (float*)w;
  w += align_up((size_t)pair_cap * 12 * sizeof(float), 256);
  int64_t* refl_ptr = (int64_t*)w;
  w += align_up((size_t)(n_hkl + 1) * sizeof(int64_t), 256);
  int32_t* refl_pairs = (int32_t*)w;
  w += align_up((size_t)pair_cap * sizeof(int32_t), 256);
  hipStream_t s = (hipStream_t)stream;
  rc = fill(partials, 12 * pair_cap, 0.0f, s);
  if (rc) return rc;
  // the work units of the balanced forward launch, still in the forward workspace
  rc = launch_adjoint_units(model, refl, nodes, pix, tile, offsets, idx, order, pair_cap, fw + L.cullws, ctr, n_hkl,
                            grad_image, nullptr, partials, s);
  if (rc) return rc;
  rc = fdtbx_pair_transpose(n_hkl, idx, pair_cap, n_pairs_dev, refl_ptr, refl_pairs, w,
                            fdtbx_pair_transpose_workspace(n_hkl, pair_cap), stream);
  if (rc) return rc;
  rc = fdtbx_pair_reduce(n_hkl, refl_ptr, refl_pairs, partials, nullptr, (model->geom.mirror & 2) ? 1 : 0, sums, stream);
  if (rc) return rc;
  rc = fdtbx_adjoint_finish(model, hkl, n_hkl, refl, sums, F, g2, d_globals, fin, fin_bytes, stream);
  if (rc) return rc;
  if (!atoms) return FDTBX_OK;
  return fdtbx_sf_adjoint(&model->cell, n_atoms, x, y, z, B, occ, type, ff, n_types, hkl, n_hkl, F, g2, d_x, d_y, d_z, d_B,
                          d_occ, sfw, fdtbx_sf_adjoint_workspace(n_hkl, n_atoms), stream);
}

// ------------------------------------------------------------------ backward without allocation
// The workspace of fdtbx_pattern_backward_noalloc: a file-scope device array, one copy per
// device, held until the process ends.  In host code the name `scratch` is a host-side stand-in,
// not a device address: host code uses only the address hipGetSymbolAddress gives for the
// current device.
static __device__ __align__(256) unsigned char scratch[FDTBX_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int kScratchDevices = 64;
std::mutex g_scratch_mutex;
void* g_scratch[kScratchDevices];  // device address of `scratch`, per device, once looked up
}  // namespace

// The current device's copy of the scratch array, looked up on the first call on that device.
static int scratch_on_current_device(void** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  if (dev < 0 || dev >= kScratchDevices) return fail(FDTBX_ERR_UNSUPPORTED, "no-alloc scratch: device index above 63");
  std::lock_guard<std::mutex> lock(g_scratch_mutex);
  if (!g_scratch[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
    if (!p) return fail(FDTBX_ERR_HIP, "hipGetSymbolAddress(scratch) gave no address");
    g_scratch[dev] = p;
  }
  *out = g_scratch[dev];
  return FDTBX_OK;
}

extern "C" int fdtbx_pattern_backward_noalloc(const fdtbx_model* model, const int32_t* hkl, int64_t n_hkl, const float* F,
                                              const float* grad_image, const void* fwd_ws, size_t fwd_ws_bytes,
                                              int64_t pair_cap, int64_t n_atoms, const float* x, const float* y,
                                              const float* z, const float* B, const float* occ, const int32_t* type,
                                              const float* ff, int32_t n_types, float* d_x, float* d_y, float* d_z,
                                              float* d_B, float* d_occ, double* d_globals, float* dF2, void* stream) {
  if (n_hkl < 0 || pair_cap < 0 || n_atoms < 0) return fail(FDTBX_ERR_INVALID_ARGUMENT, "bad sizes");
  const bool atoms = d_x || d_y || d_z || d_B || d_occ;
  const size_t need = fdtbx_backward_workspace(n_hkl, atoms ? n_atoms : 0);
  if (need > (size_t)FDTBX_NOALLOC_SCRATCH_BYTES)
    return fail(FDTBX_ERR_BUFFER_TOO_SMALL,
                "fdtbx_pattern_backward_noalloc: the backward workspace for n_hkl and n_atoms exceeds the "
                "library's scratch array (FDTBX_NOALLOC_SCRATCH_BYTES); use fdtbx_pattern_backward");
  void* ws = nullptr;
  const int rc = scratch_on_current_device(&ws);
  if (rc) return rc;
  // the same steps as fdtbx_pattern_backward; every kernel there writes its workspace before
  // reading it (the per-reflection sums are cleared by a kernel), so what an earlier call
  // left in the array does not matter
  return fdtbx_pattern_backward(model, hkl, n_hkl, F, grad_image, fwd_ws, fwd_ws_bytes, pair_cap, n_atoms, x, y, z, B, occ,
                                type, ff, n_types, d_x, d_y, d_z, d_B, d_occ, d_globals, dF2, ws,
                                (size_t)FDTBX_NOALLOC_SCRATCH_BYTES, stream);
}

extern "C" int fdtbx_batch_forward(const fdtbx_batch_entry* entries, int32_t n_models, const int64_t* refl_blocks, int64_t n_rb,
                                   const int64_t* node_blocks, int64_t n_nb, const int64_t* tile_items, int64_t n_items,
                                   const int32_t* hkl, const float* x, const float* y, const float* z, const float* B,
                                   const float* occ, const int32_t* type, const float* ff, const double* pix,
                                   const double* tile, const int64_t* rowptr, const int32_t* idx, float* F, float* F2,
                                   float* refl, float* nodes, float* image, int64_t* counter, void* stream) {
  if (!entries || n_models <= 0 || n_rb < 0 || n_nb < 0 || n_items < 0) return fail(FDTBX_ERR_INVALID_ARGUMENT, "bad sizes");
  if (!refl_blocks || !node_blocks || !tile_items || !hkl || !x || !y || !z || !B || !occ || !type || !ff || !pix || !tile ||
      !rowptr || !idx || !F || !F2 || !refl || !nodes || !image || !counter)
    return fail(FDTBX_ERR_INVALID_ARGUMENT, "null pointer");
  hipStream_t s = (hipStream_t)stream;
  int rc = launch_batch_sf(entries, refl_blocks, n_rb, x, y, z, B, occ, type, ff, hkl, F, F2, s);
  if (rc) return rc;
  rc = launch_batch_prep(entries, refl_blocks, n_rb, hkl, F2, refl, s);
  if (rc) return rc;
  rc = launch_batch_nodes(entries, node_blocks, n_nb, nodes, s);
  if (rc) return rc;
  return launch_batch_profile(entries, tile_items, n_items, refl, nodes, pix, tile, rowptr, idx, image, counter, s);
}

extern "C" int fdtbx_batch_profile_stacked(const fdtbx_batch_entry* entries, int32_t n_models, const int64_t* stack_off,
                                           const int64_t* stack_items, int64_t n_items, const float* refl,
                                           const float* nodes, const double* pix, const double* tile,
                                           const double* stile, const int64_t* srowptr, const int32_t* sidx,
                                           float* image, int64_t* counter, void* stream) {
  if (!entries || n_models <= 0 || n_items < 0) return fail(FDTBX_ERR_INVALID_ARGUMENT, "bad sizes");
  if (!stack_off || !stack_items || !refl || !nodes || !pix || !tile || !stile || !srowptr || !sidx || !image || !counter)
    return fail(FDTBX_ERR_INVALID_ARGUMENT, "null pointer");
  return launch_batch_profile_stacked(entries, stack_off, stack_items, n_items, refl, nodes, pix, tile, stile, srowptr,
                                      sidx, image, counter, (hipStream_t)stream);
}

extern "C" int fdtbx_batch_backward(const fdtbx_batch_entry* entries, int32_t n_models, const int64_t* refl_blocks, int64_t n_rb,
                                    const int64_t* model_rb, const int64_t* atom_blocks, int64_t n_ab, const int64_t* tile_items,
                                    int64_t n_items, int64_t n_hkl_total, const int32_t* hkl, const float* x, const float* y,
                                    const float* z, const float* B, const float* occ, const int32_t* type, const float* ff,
                                    const double* pix, const double* tile, const int64_t* rowptr, const int32_t* idx,
                                    const float* F, const float* refl, const float* nodes, const float* grad_image,
                                    double* sums, double* part, float* dF2, float* d_x, float* d_y, float* d_z, float* d_B,
                                    float* d_occ, double* d_globals, int64_t* counter, void* stream) {
  if (!entries || n_models <= 0 || n_rb < 0 || n_ab < 0 || n_items < 0 || n_hkl_total < 0)
    return fail(FDTBX_ERR_INVALID_ARGUMENT, "bad sizes");
  if (!refl_blocks || !model_rb || !atom_blocks || !tile_items || !hkl || !x || !y || !z || !B || !occ || !type || !ff ||
      !pix || !tile || !rowptr || !idx || !F || !refl || !nodes || !grad_image || !sums || !part || !dF2 || !d_globals ||
      !counter)
    return fail(FDTBX_ERR_INVALID_ARGUMENT, "null pointer");
  return launch_batch_backward(entries, n_models, refl_blocks, n_rb, model_rb, atom_blocks, n_ab, tile_items, n_items,
                               n_hkl_total, hkl, x, y, z, B, occ, type, ff, pix, tile, rowptr, idx, F, refl, nodes, grad_image,
                               sums, part, dF2, d_x, d_y, d_z, d_B, d_occ, d_globals, counter, nullptr, (hipStream_t)stream);
}

extern "C" int fdtbx_batch_backward_deterministic(
    const fdtbx_batch_entry* entries, int32_t n_models, const int64_t* refl_blocks, int64_t n_rb, const int64_t* model_rb,
    const int64_t* atom_blocks, int64_t n_ab, const int64_t* tile_items, int64_t n_items, int64_t n_hkl_total,
    const int32_t* hkl, const float* x, const float* y, const float* z, const float* B, const float* occ,
    const int32_t* type, const float* ff, const double* pix, const double* tile, const int64_t* rowptr, const int32_t* idx,
    const float* F, const float* refl, const float* nodes, const float* grad_image, int64_t n_pairs_total,
    const int64_t* refl_ptr, const int32_t* refl_pairs, const int64_t* mate, float* partials, double* sums, double* part,
    float* dF2, float* d_x, float* d_y, float* d_z, float* d_B, float* d_occ, double* d_globals, int64_t* counter,
    void* stream) {
  if (!entries || n_models <= 0 || n_rb < 0 || n_ab < 0 || n_items < 0 || n_hkl_total < 0 || n_pairs_total < 0)
    return fail(FDTBX_ERR_INVALID_ARGUMENT, "bad sizes");
  if (!refl_blocks || !model_rb || !atom_blocks || !tile_items || !hkl || !x || !y || !z || !B || !occ || !type || !ff ||
      !pix || !tile || !rowptr || !idx || !F || !refl || !nodes || !grad_image || !sums || !part || !dF2 || !d_globals ||
      !counter || !refl_ptr || !mate || (n_pairs_total > 0 && (!refl_pairs || !partials)))
    return fail(FDTBX_ERR_INVALID_ARGUMENT, "null pointer");
  const PairOrder fixed = {partials, n_pairs_total, refl_ptr, refl_pairs, mate};
  return launch_batch_backward(entries, n_models, refl_blocks, n_rb, model_rb, atom_blocks, n_ab, tile_items, n_items,
                               n_hkl_total, hkl, x, y, z, B, occ, type, ff, pix, tile, rowptr, idx, F, refl, nodes, grad_image,
                               sums, part, dF2, d_x, d_y, d_z, d_B, d_occ, d_globals, counter, &fixed, (hipStream_t)stream);
}

extern "C" size_t fdtbx_batch_entry_size(void) { return sizeof(fdtbx_batch_entry); }
