// Shared by the forward and adjoint profile kernels: launch parameters and the
// node window of a (tile, reflection) pair.
#pragma once

#include <hip/hip_runtime.h>

#include <math.h>

#include "internal.h"

namespace fdtbx {

struct ProfParams {
  int32_t W, H, tiles_x, tiles_y;
  int32_t tlg;      // tiles are 2^tlg pixels wide and 64 >> tlg high
  int32_t lcols;    // tile columns launched: tiles_x, or the left half under the left-right fold
  int32_t lrows;    // tile rows launched: tiles_y, or the top half under the up-down fold
  int32_t mirror;   // bit 0: each computed pixel is also written to (W - 1 - i, j); bit 1: to
                    // (i, H - 1 - j); both: also to (W - 1 - i, H - 1 - j)
  int32_t lineshape;
  int32_t n;        // nodes per side
  float T, inv_h;   // grid half extent, 1/spacing
  float half_m;     // support half-width in y (lineshape_half)
  float cmin;       // (1 + 2T^2)^(-1/2)
  float margin;     // slack of the tile-level node test, in y units
  double delta;     // Lorentz regulariser
  int32_t sbw;      // superblocks per tile row in the XCD-aware tile order; 0: plain order
  double T64, h64;  // grid half extent and spacing in binary64 (the Hosemann walk's edge decisions)
};

// Tile order of the per-tile launches.  Workgroups are dealt to the 8 XCDs in round-robin
// order and each XCD has its own L2.  Neighbouring tiles share most of their reflections,
// so the tiles are grouped into kSuper x kSuper superblocks whose tiles run on one XCD in
// consecutive dispatch slots, consecutive superblocks going to different XCDs (which keeps
// the XCDs' loads balanced).  Used when there are at least 8 superblocks per XCD.
constexpr int kXcds = 8, kSuper = 8;

__host__ __device__ inline int32_t superblocks_per_row(int32_t tiles_x, int32_t tiles_y) {
  const int64_t sbw = (tiles_x + kSuper - 1) / kSuper, sbh = (tiles_y + kSuper - 1) / kSuper;
  return sbw * sbh >= 8 * kXcds ? (int32_t)sbw : 0;
}

// Workgroups of a per-tile launch (the padded superblock grid of the launched tiles, or one
// per launched tile).
__host__ __device__ inline int64_t tile_grid(const ProfParams& q) {
  if (q.sbw == 0) return (int64_t)q.lcols * q.lrows;
  const int64_t nsb = (int64_t)q.sbw * ((q.lrows + kSuper - 1) / kSuper);
  return (int64_t)kXcds * kSuper * kSuper * ((nsb + kXcds - 1) / kXcds);
}

// Superblock side of the launch orders of fdtbx_tile_order: kSuper when the detector has
// at least 8 superblocks per XCD, else single tiles; and the workgroups of such a launch.
__host__ __device__ inline int32_t order_super(int32_t tiles_x, int32_t tiles_y) {
  return superblocks_per_row(tiles_x, tiles_y) ? kSuper : 1;
}
__host__ __device__ inline int64_t order_grid(int32_t tiles_x, int32_t tiles_y) {
  const int64_t S = order_super(tiles_x, tiles_y);
  const int64_t nsb = ((tiles_x + S - 1) / S) * ((tiles_y + S - 1) / S);
  return (int64_t)kXcds * S * S * ((nsb + kXcds - 1) / kXcds);
}

// Tile of workgroup b, or -1 for a padding workgroup (past the launched columns or rows).
__device__ inline int tile_of_block(const ProfParams& q, int b) {
  if (q.sbw == 0) return (b / q.lcols) * q.tiles_x + b % q.lcols;
  const int x = b % kXcds, k = b / kXcds;
  const int sb = (k / (kSuper * kSuper)) * kXcds + x, i = k % (kSuper * kSuper);
  const int tx = (sb % q.sbw) * kSuper + i % kSuper, ty = (sb / q.sbw) * kSuper + i / kSuper;
  return tx < q.lcols && ty < q.lrows ? ty * q.tiles_x + tx : -1;
}

__host__ __device__ inline int64_t ceil_div_dev(int64_t a, int64_t b) { return (a + b - 1) / b; }

// Pairs per work unit of the balanced launch (fdtbx_profile_balanced) for a launch of n_pairs
// culled pairs: at most 2^19 units in all besides one partial unit per tile (64 per wave of
// 256 compute units with 32 waves each), at least 32 pairs.  A function of the pair count
// alone, so that the image does not depend on the device.
constexpr int64_t kUnitTarget = int64_t{1} << 19;
__host__ __device__ inline int64_t default_unit_pairs(int64_t n_pairs) {
  const int64_t U = (n_pairs + kUnitTarget - 1) / kUnitTarget;
  return U < 32 ? 32 : U;
}

// Mirror folds.  Tile column tiles_x - 1 - tx holds the left-right mirror pixels of column tx
// and tile row tiles_y - 1 - ty the up-down ones of row ty; a middle column or row (odd count)
// is its own mirror, its pixels all computed.  write_folded stores a computed value at pixel
// (i, j) of tile (tx, ty) and at the mirror pixels no launched tile computes; folded_weights
// gives the adjoint's weights of the value, an image-shaped weight summed over those pixels.
__device__ inline void write_folded(const ProfParams& q, float* image, int i, int j, int tx, int ty, float v) {
  const bool mx = (q.mirror & 1) && 2 * tx + 1 != q.tiles_x;
  const bool my = (q.mirror & 2) && 2 * ty + 1 != q.tiles_y;
  const int64_t row = (int64_t)j * q.W, mrow = (int64_t)(q.H - 1 - j) * q.W;
  image[row + i] = v;
  if (mx) image[row + (q.W - 1 - i)] = v;
  if (my) image[mrow + i] = v;
  if (mx && my) image[mrow + (q.W - 1 - i)] = v;
}
// The adjoint's two weights of a computed pixel: *wa = g over the pixel and its left-right
// mirror (the same reflection gives both the same value), *wb = g over its up-down mirrors
// (whose value the Friedel mate of the reflection gives at this pixel); 0 where no such
// mirror is folded onto the pixel.
__device__ inline void folded_weights(const ProfParams& q, const float* g, int i, int j, int tx, int ty, float* wa,
                                      float* wb) {
  const bool mx = (q.mirror & 1) && 2 * tx + 1 != q.tiles_x;
  const bool my = (q.mirror & 2) && 2 * ty + 1 != q.tiles_y;
  const int64_t row = (int64_t)j * q.W, mrow = (int64_t)(q.H - 1 - j) * q.W;
  float a = g[row + i], b = 0.0f;
  if (mx) a += g[row + (q.W - 1 - i)];
  if (my) {
    b = g[mrow + i];
    if (mx) b += g[mrow + (q.W - 1 - i)];
  }
  *wa = a;
  *wb = b;
}

struct Window {
  int i1lo, i1hi, i2lo, i2hi;
};

// The per-pair line of one reflection's record (slots RS_HOT..RS_HOT + 31, everything a
// (tile, reflection) pair reads), loaded with one batch of 16-byte loads so that a pair waits
// for memory once.
struct PairRec {
  float v[32];
  __device__ float at(int slot) const { return v[slot - RS_HOT]; }
  __device__ double at_f64(int slot) const {
    return __hiloint2double(__float_as_int(v[slot - RS_HOT + 1]), __float_as_int(v[slot - RS_HOT]));
  }
};

__device__ __forceinline__ void load_pair(const float* __restrict__ rec, PairRec& f) {
  const float4* r4 = (const float4*)(rec + RS_HOT);
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    const float4 x = r4[k];
    f.v[4 * k + 0] = x.x;
    f.v[4 * k + 1] = x.y;
    f.v[4 * k + 2] = x.z;
    f.v[4 * k + 3] = x.w;
  }
  // An empty statement that reads the fields: it keeps the compiler from sinking some of
  // the loads below the window test, so that the pair waits for memory once, not three times.
  asm volatile("" ::"s"(f.v[0]), "s"(f.v[1]), "s"(f.v[2]), "s"(f.v[3]), "s"(f.v[4]), "s"(f.v[5]), "s"(f.v[6]),
               "s"(f.v[7]), "s"(f.v[8]), "s"(f.v[9]), "s"(f.v[10]), "s"(f.v[11]), "s"(f.v[12]), "s"(f.v[13]),
               "s"(f.v[14]), "s"(f.v[15]));
  asm volatile("" ::"s"(f.v[16]), "s"(f.v[17]), "s"(f.v[18]), "s"(f.v[19]), "s"(f.v[20]), "s"(f.v[21]),
               "s"(f.v[22]), "s"(f.v[23]), "s"(f.v[24]), "s"(f.v[25]), "s"(f.v[26]), "s"(f.v[27]), "s"(f.v[28]),
               "s"(f.v[29]), "s"(f.v[30]));
}

// Node index range that query points p with p.S in [sl, sh], p.e1 in [l1, h1] and
// p.e2 in [l2, h2] can reach.  A node in the support of p satisfies |s.v - p.v| <= rho_v
// for v in {S, e1, e2} (rho_v: support extents); s.S = r0 c is in [r0 cmin, r0];
// d_j = (s.e_j)/(s.S).  One extra node of margin on each side absorbs the float32 rounding
// of these bounds (hardware reciprocals included).
__device__ static inline bool node_window_ranges(const ProfParams& q, float r0, float sl, float sh, float l1, float h1,
                                                 float l2, float h2, float rhoS, float rho1, float rho2, Window* w) {
  const float rS = rhoS * 1.0001f, r1 = rho1 * 1.0001f, r2 = rho2 * 1.0001f;
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

// Per-pair set-up of the forward and adjoint tile loops, done lane-parallel (each lane one
// pair of the tile's list, so that this uniform per-pair arithmetic costs a 64th of a wave
// instruction per pair): the pair's node window, packed as two ints (low and high 16 bits:
// first and last index along d1, then along d2; the query points p = R e_perp + Z z of the
// tile's (R, Z) box have p.v = R (e_perp.v) + Z v_z, extreme at the box corners), and the
// tile's alpha box, the ranges of
// alpha_i over the tile's (R, Z) box (linear in R, Z: extremes at the corners) widened by the
// support half-width and the margin.  With PRE, a window of at most kPreBlocks node blocks is then
// narrowed to the blocks that can hold a queued node: each block record bounds the offsets
// kappa of its nodes (the block test of scan_window), and every node whose kappa lies in the
// alpha box lies in a passing block, so the nodes the scan queues are the same, in the same
// relative order, and a pair whose blocks all fail has none.  With fl, fh (the forward's
// split walk), also the full box of the pair: the offsets kappa that lie inside the support
// of every pixel of the tile, [max alpha - half_m + m, min alpha + half_m - m] per axis.  Its
// margin m = margin + 2^-19 sum_v max |coef_v d_v| exceeds the float32 rounding of alpha at
// any pixel of the box (a few units in the last place of the two products, whose magnitudes
// the sum bounds), of the tags (at most 2^-18) and of y = alpha - kappa (a unit in the last
// place of half_m), so a node in the full box passes the support test at every pixel of the
// detector that the tile holds.  Returns false if the window is empty.
struct TileBox {
  double Rlo, Rhi, Zlo, Zhi;
};

constexpr int kPreBlocks = 16;

// PRE: narrow the window by its node blocks (the batched launches, whose pairs carry few
// evaluations and often queue none: there it saves a tenth of the time; the single-model
// launches keep their registers for the walk).
template <bool PRE>
__device__ static inline bool pair_setup(const ProfParams& q, const float* __restrict__ rec,
                                         const float* __restrict__ nodes, const TileBox& b, int* w01, int* w23,
                                         float* lo, float* hi, float* fl = nullptr, float* fh = nullptr) {
  // xj: slots RS_HOT + 4j .. + 4j + 3 of the per-pair line
  const float4 x0 = *(const float4*)(rec + RS_HOT);
  const float4 x3 = *(const float4*)(rec + RS_HOT + 8);
  const float4 x4 = *(const float4*)(rec + RS_HOT + 12);
  const float4 x5 = *(const float4*)(rec + RS_HOT + 16);
  const float4 x6 = *(const float4*)(rec + RS_HOT + 20);
  const float4 x7 = *(const float4*)(rec + RS_HOT + 24);
  const float4 x8 = *(const float4*)(rec + RS_HOT + 28);
  static_assert(RS_R0 == RS_HOT && RS_B == RS_HOT + 2 && RS_G1 == RS_HOT + 5 && RS_G2 == RS_HOT + 8 &&
                    RS_TR == RS_HOT + 11 && RS_TZ == RS_HOT + 14 && RS_RD == RS_HOT + 18 && RS_ZD == RS_HOT + 20 &&
                    RS_CS == RS_HOT + 22 && RS_C1 == RS_HOT + 24 && RS_C2 == RS_HOT + 26 && RS_RHO == RS_HOT + 28,
                "the loads below read the record by these positions");
  const float tr[3] = {x3.w, x4.x, x4.y}, tz[3] = {x4.z, x4.w, x5.x};
  const double RD = __hiloint2double(__float_as_int(x5.w), __float_as_int(x5.z));
  const double ZD = __hiloint2double(__float_as_int(x6.y), __float_as_int(x6.x));
  const float dRl = (float)(b.Rlo - RD), dRh = (float)(b.Rhi - RD);
  const float dZl = (float)(b.Zlo - ZD), dZh = (float)(b.Zhi - ZD);
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const float r1 = tr[a] * dRl, r2 = tr[a] * dRh, z1 = tz[a] * dZl, z2 = tz[a] * dZh;
    const float amin = fminf(r1, r2) + fminf(z1, z2), amax = fmaxf(r1, r2) + fmaxf(z1, z2);
    lo[a] = amin - q.half_m - q.margin;
    hi[a] = amax + q.half_m + q.margin;
    if (fl) {
      const float mag = fmaxf(fabsf(r1), fabsf(r2)) + fmaxf(fabsf(z1), fabsf(z2));
      const float m = fmaf(mag, 0x1p-19f, q.margin);
      fl[a] = amax - q.half_m + m;
      fh[a] = amin + q.half_m - m;
    }
  }
  const float Rlo = (float)b.Rlo, Rhi = (float)b.Rhi, Zlo = (float)b.Zlo, Zhi = (float)b.Zhi;
  auto range = [&](float cR, float cZ, float* l, float* h) {
    const float a = Rlo * cR, bb = Rhi * cR, c = Zlo * cZ, d = Zhi * cZ;
    *l = fminf(a, bb) + fminf(c, d);
    *h = fmaxf(a, bb) + fmaxf(c, d);
  };
  float sl, sh, l1, h1, l2, h2;
  range(x6.z, x6.w, &sl, &sh);
  range(x7.x, x7.y, &l1, &h1);
  range(x7.z, x7.w, &l2, &h2);
  Window w;
  if (!node_window_ranges(q, x0.x, sl, sh, l1, h1, l2, h2, x8.x, x8.y, x8.z, &w)) return false;
  constexpr int NB = FDTBX_NODE_BLOCK;
  const int b1lo = w.i1lo / NB, b1hi = w.i1hi / NB, b2lo = w.i2lo / NB, b2hi = w.i2hi / NB;
  if (PRE && (b1hi - b1lo + 1) * (b2hi - b2lo + 1) <= kPreBlocks) {
    const float4 x1 = *(const float4*)(rec + RS_HOT + 4);
    const float Bv[3] = {x0.z, x0.w, x1.x}, G1[3] = {x1.y, x1.z, x1.w}, G2[3] = {x3.x, x3.y, x3.z};
    float sl3[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) sl3[a] = 4.0e-6f * (fabsf(Bv[a]) + fabsf(G1[a]) + fabsf(G2[a]));
    const float* blocks = nodes + (int64_t)FDTBX_NODE_FLOATS * q.n * q.n;
    const int nbs = (q.n + NB - 1) / NB;
    int k1lo = b1hi + 1, k1hi = b1lo - 1, k2lo = b2hi + 1, k2hi = b2lo - 1;
    for (int b2i = b2lo; b2i <= b2hi; ++b2i)
      for (int b1i = b1lo; b1i <= b1hi; ++b1i) {
        const float* br = blocks + (int64_t)FDTBX_NODE_FLOATS * (b2i * nbs + b1i);
        const float4 cm = *(const float4*)br, rr = *(const float4*)(br + 4);
        bool keep = true;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
          const float ec = fmaf(cm.x, Bv[a], fmaf(cm.y, G1[a], cm.z * G2[a]));
          const float er = fmaf(sl3[a], cm.w, fmaf(rr.x, fabsf(Bv[a]), fmaf(rr.y, fabsf(G1[a]), rr.z * fabsf(G2[a]))));
          keep = keep && ec - er <= hi[a] && ec + er >= lo[a];
        }
        if (keep) {
          k1lo = min(k1lo, b1i);
          k1hi = max(k1hi, b1i);
          k2lo = min(k2lo, b2i);
          k2hi = max(k2hi, b2i);
        }
      }
    if (k1hi < k1lo) return false;  // no block can hold a queued node
    w.i1lo = max(w.i1lo, k1lo * NB);
    w.i1hi = min(w.i1hi, k1hi * NB + NB - 1);
    w.i2lo = max(w.i2lo, k2lo * NB);
    w.i2hi = min(w.i2hi, k2hi * NB + NB - 1);
  }
  *w01 = w.i1lo | (w.i1hi << 16);
  *w23 = w.i2lo | (w.i2hi << 16);
  return true;
}

__device__ __forceinline__ int lane_int(int v, int src) { return __builtin_amdgcn_readlane(v, src); }
__device__ __forceinline__ float lane_float(float v, int src) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), src));
}

// Window node wi -> (i1, i2) for a window nw1 nodes wide, through an approximate float
// reciprocal (integers below 2^24; the quotient is off by at most one) with a one-step
// correction instead of an integer division.
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

// Windows of at most this many nodes are scanned node by node; larger ones first test
// the FDTBX_NODE_BLOCK^2 node blocks that overlap them.
constexpr int kPlainScanMax = 192;

// Candidate nodes of one (tile, reflection) pair: the nodes k of window w whose offsets
// e_a = B_a (c - 1) + G1_a c d1 + G2_a c d2 lie in [lo_a, hi_a] for a = 0, 1, 2.  Calls
// sink(keep, k, e) on every lane of the wave with uniform control flow, 64 candidates a
// call, where keep marks a candidate, k is its node index and e = (e_0, e_1, e_2, omega).
// The candidates are the same on both paths; the order in which they are offered differs.
// bq: LDS scratch of 64 ints.
template <class Sink>
__device__ __forceinline__ void scan_window(const ProfParams& q, const float* __restrict__ nodes, const Window& w,
                                            const float* Bv, const float* G1, const float* G2, const float* lo,
                                            const float* hi, int* bq, Sink&& sink) {
  const int lane = threadIdx.x & 63;
  auto node_e = [&](int k, float4* e) {
    const float4 nd = *(const float4*)(nodes + (int64_t)FDTBX_NODE_FLOATS * k);
    e->x = fmaf(nd.x, Bv[0], fmaf(nd.y, G1[0], nd.z * G2[0]));
    e->y = fmaf(nd.x, Bv[1], fmaf(nd.y, G1[1], nd.z * G2[1]));
    e->z = fmaf(nd.x, Bv[2], fmaf(nd.y, G1[2], nd.z * G2[2]));
    e->w = nd.w;
    return e->x >= lo[0] && e->x <= hi[0] && e->y >= lo[1] && e->y <= hi[1] && e->z >= lo[2] && e->z <= hi[2];
  };
  const int nw1 = w.i1hi - w.i1lo + 1;
  const int nwin = nw1 * (w.i2hi - w.i2lo + 1);
  if (nwin <= kPlainScanMax) {
    const float inv_nw1 = __builtin_amdgcn_rcpf((float)nw1);
    for (int w0 = 0; w0 < nwin; w0 += 64) {
      const int wi = w0 + lane;
      float4 e = make_float4(0.f, 0.f, 0.f, 0.f);
      bool keep = false;
      int k = 0;
      if (wi < nwin) {
        int d1, d2;
        window_node(wi, nw1, inv_nw1, &d1, &d2);
        k = (w.i2lo + d2) * q.n + (w.i1lo + d1);
        keep = node_e(k, &e);
      }
      sink(keep, k, e);
    }
    return;
  }
  // Block test: a block record holds the centre c_j and half-width r_j of the block's
  // node coordinates (every node value lies in c_j +- r_j exactly) and mag = max_j |c_j| + r_j.
  // The block is kept if [E(c) - E(r) - slack, E(c) + E(r) + slack] meets [lo, hi], with E
  // the map above (absolute coefficients for r); the slack covers the float32 rounding of
  // these sums and of the node test (a few units in the last place of sum |coef| mag).
  const float* blocks = nodes + (int64_t)FDTBX_NODE_FLOATS * q.n * q.n;
  const int nbs = (q.n + FDTBX_NODE_BLOCK - 1) / FDTBX_NODE_BLOCK;
  const int b1lo = w.i1lo / FDTBX_NODE_BLOCK, b1hi = w.i1hi / FDTBX_NODE_BLOCK;
  const int b2lo = w.i2lo / FDTBX_NODE_BLOCK, b2hi = w.i2hi / FDTBX_NODE_BLOCK;
  const int nb1 = b1hi - b1lo + 1;
  const int nbw = nb1 * (b2hi - b2lo + 1);
  const float inv_nb1 = __builtin_amdgcn_rcpf((float)nb1);
  float aB[3], aG1[3], aG2[3], sl[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    aB[a] = fabsf(Bv[a]);
    aG1[a] = fabsf(G1[a]);
    aG2[a] = fabsf(G2[a]);
    sl[a] = 4.0e-6f * (aB[a] + aG1[a] + aG2[a]);
  }
  constexpr int kBB = FDTBX_NODE_BLOCK * FDTBX_NODE_BLOCK;
  constexpr int kPer = 64 / kBB;  // blocks expanded per pass
  for (int c0 = 0; c0 < nbw; c0 += 64) {
    const int bi = c0 + lane;
    bool keep = false;
    int base = 0;  // first node of the block: i1 in the low 16 bits, i2 in the high 16 bits
    if (bi < nbw) {
      int d1, d2;
      window_node(bi, nb1, inv_nb1, &d1, &d2);
      const int bid = (b2lo + d2) * nbs + (b1lo + d1);
      base = ((b1lo + d1) * FDTBX_NODE_BLOCK) | (((b2lo + d2) * FDTBX_NODE_BLOCK) << 16);
      const float4 cm = *(const float4*)(blocks + (int64_t)FDTBX_NODE_FLOATS * bid);
      const float4 rr = *(const float4*)(blocks + (int64_t)FDTBX_NODE_FLOATS * bid + 4);
      keep = true;
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        const float ec = fmaf(cm.x, Bv[a], fmaf(cm.y, G1[a], cm.z * G2[a]));
        const float er = fmaf(sl[a], cm.w, fmaf(rr.x, aB[a], fmaf(rr.y, aG1[a], rr.z * aG2[a])));
        keep = keep && ec - er <= hi[a] && ec + er >= lo[a];
      }
    }
    const unsigned long long b = __ballot(keep);
    const int nk = __popcll(b);
    if (keep) bq[(int)__builtin_amdgcn_mbcnt_hi((unsigned)(b >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)b, 0u))] = base;
    wave_sync();
    for (int k0 = 0; k0 < nk; k0 += kPer) {
      const int kk = k0 + lane / kBB;
      float4 e = make_float4(0.f, 0.f, 0.f, 0.f);
      bool keepn = false;
      int k = 0;
      if (kk < nk) {
        const int bb = bq[kk];
        const int sub = lane % kBB;
        const int i1 = (bb & 0xffff) + sub % FDTBX_NODE_BLOCK;
        const int i2 = (bb >> 16) + sub / FDTBX_NODE_BLOCK;
        if (i1 >= w.i1lo && i1 <= w.i1hi && i2 >= w.i2lo && i2 <= w.i2hi) {
          k = i2 * q.n + i1;
          keepn = node_e(k, &e);
        }
      }
      sink(keepn, k, e);
    }
    wave_sync();
  }
}

// ---------------------------------------------------------------- work units of the balanced launches
// The launched tiles' lists cut into units of at most U pairs (see fdtbx_profile_balanced).
// Queue-major position of slot b: (b % 8) nj + b / 8, nj = ceil(n_slots / 8).  qscan holds the
// units per position, then (after k_scan_inplace) the first unit of each position; queue x
// spans the units qscan[x nj] .. qscan[(x + 1) nj] (the total for the last queue).
struct UnitTable {
  const int32_t* order;  // tile of each slot, or null: the plain per-tile grid (tile_of_block)
  int64_t n_slots, nj;
  int64_t max_units;     // capacity of unit_slot and of the partial sums
  int64_t fixed_U;       // pairs per unit, or 0: chosen from the pair count (default_unit_pairs)
  int64_t* qscan;        // [8 nj]
  int64_t* meta;         // [0]: total units, [1]: pairs per unit
  int32_t* ctr;          // [8] queue counters
  int32_t* unit_slot;    // [max_units] slot of each unit
};

__host__ __device__ inline int64_t queue_pos(int64_t b, int64_t nj) { return (b % kXcds) * nj + b / kXcds; }

__device__ inline int slot_tile(const ProfParams& q, const UnitTable& T, int64_t b) {
  if (b >= T.n_slots) return -1;
  return T.order ? T.order[b] : tile_of_block(q, (int)b);
}

// Workspace of the balanced launch: the unit tables and the partial sums.
struct UnitLayout {
  int64_t n_slots, nj, max_units;
  size_t qscan, meta, ctr, unit_slot, partials, total;
};

inline UnitLayout unit_layout(const ProfParams& q, bool has_order, int64_t pair_cap, int64_t fixed_U) {
  UnitLayout L;
  L.n_slots = has_order ? order_grid(q.lcols, q.lrows) : tile_grid(q);
  L.nj = ceil_div(L.n_slots, kXcds);
  // sum over tiles of ceil(len / U) <= pair_cap / U + n_slots, and U >= 32 with U >= n_pairs / 2^19
  // when it is the library's choice
  const int64_t by_cap = ceil_div(pair_cap, fixed_U > 0 ? fixed_U : 32);
  L.max_units = (fixed_U > 0 ? by_cap : (by_cap < kUnitTarget ? by_cap : kUnitTarget)) + L.n_slots;
  size_t o = 0;
  L.qscan = o;
  o += align_up((size_t)(kXcds * L.nj) * sizeof(int64_t), 256);
  L.meta = o;
  o += 256;
  L.ctr = o;
  o += 256;
  L.unit_slot = o;
  o += align_up((size_t)L.max_units * sizeof(int32_t), 256);
  L.partials = o;
  o += align_up((size_t)L.max_units * 64 * sizeof(float), 256);
  L.total = o;
  return L;
}


// Unit u's tile and pair range [*p0, *p1), or -1 when the tables do not describe such a unit
// (only tables that a launch over other lists left behind would fail these checks; they keep
// every read in bounds).
__device__ inline int unit_range(const ProfParams& q, const UnitTable& T, const int64_t* __restrict__ offsets,
                                 int64_t u, int64_t U, int64_t* p0, int64_t* p1) {
  const int64_t b = T.unit_slot[u];
  if (b < 0 || b >= T.n_slots) return -1;
  const int t = slot_tile(q, T, b);
  if (t < 0) return -1;
  const int64_t k = u - T.qscan[queue_pos(b, T.nj)];
  const int64_t a = offsets[t] + k * U, e = offsets[t + 1];
  if (k < 0 || a >= e) return -1;
  *p0 = a;
  *p1 = a + U < e ? a + U : e;
  return t;
}

// Queue x's units [*qb, *qe), clamped to the first `total` units.
__device__ inline void queue_span(const UnitTable& T, int x, int64_t total, int64_t* qb, int64_t* qe) {
  int64_t b = T.qscan[x * T.nj];
  int64_t e = x + 1 < kXcds ? T.qscan[(x + 1) * T.nj] : T.meta[0];
  b = b < 0 ? 0 : (b > total ? total : b);
  e = e < b ? b : (e > total ? total : e);
  *qb = b;
  *qe = e;
}

// The unit tables inside a workspace laid out by unit_layout (order and the fixed pairs per
// unit as for the launch that built them).
inline UnitTable unit_view(const UnitLayout& L, const int32_t* order, int64_t fixed_U, void* ws) {
  char* w = (char*)ws;
  UnitTable T;
  T.order = order;
  T.n_slots = L.n_slots;
  T.nj = L.nj;
  T.max_units = L.max_units;
  T.fixed_U = fixed_U;
  T.qscan = (int64_t*)(w + L.qscan);
  T.meta = (int64_t*)(w + L.meta);
  T.ctr = (int32_t*)(w + L.ctr);
  T.unit_slot = (int32_t*)(w + L.unit_slot);
  return T;
}

__host__ __device__ inline void prof_params(const fdtbx_model* model, ProfParams* q) {
  q->W = model->geom.width;
  q->H = model->geom.height;
  const int tw = model->geom.tile_w ? model->geom.tile_w : FDTBX_TILE, th = 64 / tw;
  q->tlg = __builtin_ctz((unsigned)tw);
  q->tiles_x = (q->W + tw - 1) / tw;
  q->tiles_y = (q->H + th - 1) / th;
  q->mirror = model->geom.mirror;
  q->lcols = (q->mirror & 1) ? (q->tiles_x + 1) / 2 : q->tiles_x;
  q->lrows = (q->mirror & 2) ? (q->tiles_y + 1) / 2 : q->tiles_y;
  q->n = model->quad.n_nodes;
  q->T = (float)model->quad.T;
  q->inv_h = (float)(model->quad.n_nodes / (2.0 * model->quad.T));
  q->lineshape = model->dis.lineshape;
  q->half_m = (float)lineshape_half(model->dis.lineshape, model->quad.m);
  q->cmin = (float)(1.0 / sqrt(1.0 + 2.0 * model->quad.T * model->quad.T));
  q->margin = 1.0e-3f;
  q->delta = model->quad.delta;
  q->sbw = superblocks_per_row(q->lcols, q->lrows);
  q->T64 = model->quad.T;
  q->h64 = 2.0 * model->quad.T / model->quad.n_nodes;
}

}  // namespace fdtbx
