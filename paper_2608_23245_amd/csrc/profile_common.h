// Shared by the forward and adjoint profile kernels: launch parameters and the
// node window of a (tile, reflection) pair.
#pragma once

#include <hip/hip_runtime.h>

#include <math.h>

#include "internal.h"

namespace fdtbx {

struct ProfParams {
  int32_t W, H, tiles_x, tiles_y;
  int32_t n;        // nodes per side
  float T, inv_h;   // grid half extent, 1/spacing
  float half_m;     // m/2
  float cmin;       // (1 + 2T^2)^(-1/2)
  float tiny;       // added to |y|: keeps sin(2 pi y)/y finite at y = 0, exact in float32 for |y| > 1e-5
  float margin;     // slack of the tile-level node test, in y units
  double delta;     // Lorentz regulariser
};

struct Window {
  int i1lo, i1hi, i2lo, i2hi;
};

// Node index range that the query points of a tile box can reach.  A node in the
// support of p satisfies |s.v - p.v| <= rho_v for v in {S, e1, e2}; s.S = r0 c is in
// [r0 cmin, r0]; d_j = (s.e_j)/(s.S).  One extra node of margin on each side absorbs the
// float32 rounding of these bounds (hardware reciprocals included).
__device__ static inline bool node_window(const ProfParams& q, const float* rec, float Rlo, float Rhi, float Zlo, float Zhi,
                                          Window* w) {
  auto range = [&](float cR, float cZ, float* lo, float* hi) {
    float a = Rlo * cR, b = Rhi * cR, c = Zlo * cZ, d = Zhi * cZ;
    *lo = fminf(a, b) + fminf(c, d);
    *hi = fmaxf(a, b) + fmaxf(c, d);
  };
  const float r0 = rec[RS_R0];
  float sl, sh, l1, h1, l2, h2;
  range(rec[RS_CS], rec[RS_CS + 1], &sl, &sh);
  range(rec[RS_C1], rec[RS_C1 + 1], &l1, &h1);
  range(rec[RS_C2], rec[RS_C2 + 1], &l2, &h2);
  const float rS = rec[RS_RHO] * 1.0001f, r1 = rec[RS_RHO + 1] * 1.0001f, r2 = rec[RS_RHO + 2] * 1.0001f;
  float dlo_s = fmaxf(sl - rS, r0 * q.cmin * 0.9999f);
  float dhi_s = fminf(sh + rS, r0 * 1.0001f);
  if (!(dlo_s <= dhi_s)) return false;
  const float inv_lo = __builtin_amdgcn_rcpf(dlo_s), inv_hi = __builtin_amdgcn_rcpf(dhi_s);
  auto bounds = [&](float nl, float nh, float* dlo, float* dhi) {
    *dlo = nl * (nl >= 0.0f ? inv_hi : inv_lo);
    *dhi = nh * (nh >= 0.0f ? inv_lo : inv_hi);
  };
  float d1l, d1h, d2l, d2h;
  bounds(l1 - r1, h1 + r1, &d1l, &d1h);
  bounds(l2 - r2, h2 + r2, &d2l, &d2h);
  // node i sits at d = -T + (i + 1/2) h
  auto lo_idx = [&](float d) { return (int)ceilf((d + q.T) * q.inv_h - 0.5f) - 1; };
  auto hi_idx = [&](float d) { return (int)floorf((d + q.T) * q.inv_h - 0.5f) + 1; };
  float big = 2.0f * q.T;
  d1l = fmaxf(d1l, -big);
  d2l = fmaxf(d2l, -big);
  d1h = fminf(d1h, big);
  d2h = fminf(d2h, big);
  w->i1lo = max(lo_idx(d1l), 0);
  w->i1hi = min(hi_idx(d1h), q.n - 1);
  w->i2lo = max(lo_idx(d2l), 0);
  w->i2hi = min(hi_idx(d2h), q.n - 1);
  return w->i1lo <= w->i1hi && w->i2lo <= w->i2hi;
}

// Window node wi -> (i1, i2) for a window nw1 nodes wide, through a float reciprocal
// (exact integers below 2^24) with a one-step correction instead of an integer division.
__device__ static inline void window_node(int wi, int nw1, float inv_nw1, int* i1, int* i2) {
  int q2 = (int)((float)wi * inv_nw1);
  int q1 = wi - q2 * nw1;
  if (q1 < 0) {
    q2 -= 1;
    q1 += nw1;
  } else if (q1 >= nw1) {
    q2 += 1;
    q1 -= nw1;
  }
  *i1 = q1;
  *i2 = q2;
}

__host__ __device__ inline void prof_params(const fdtbx_model* model, ProfParams* q) {
  q->W = model->geom.width;
  q->H = model->geom.height;
  q->tiles_x = (q->W + FDTBX_TILE - 1) / FDTBX_TILE;
  q->tiles_y = (q->H + FDTBX_TILE - 1) / FDTBX_TILE;
  q->n = model->quad.n_nodes;
  q->T = (float)model->quad.T;
  q->inv_h = (float)(model->quad.n_nodes / (2.0 * model->quad.T));
  q->half_m = 0.5f * (float)model->quad.m;
  q->cmin = (float)(1.0 / sqrt(1.0 + 2.0 * model->quad.T * model->quad.T));
  q->tiny = 1.0e-12f;
  q->margin = 1.0e-3f;
  q->delta = model->quad.delta;
}

}  // namespace fdtbx
