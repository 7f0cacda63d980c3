// Per-tile body of the forward profile kernel, shared by the single-model and the
// batched launches.
#pragma once

#include "profile_common.h"

namespace fdtbx {

// Per-pair constants of the Hosemann lineshape: den_i = c0_i - c1_i cos(2 pi y_i) with
// c0 = 1 + A'^2, c1 = 2 A'; e0, e1: the same times 0 or 1 (0 where A' is held at 0), for the
// N-derivative of the adjoint.
struct HoseK {
  float c0[3], c1[3], e0[3], e1[3];
};

__device__ __forceinline__ void hose_constants(const float* rec, HoseK& h) {
  const float4 a = *(const float4*)(rec + RS_AH);
  const float A[3] = {a.x, a.y, a.z};
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    h.c0[i] = fmaf(A[i], A[i], 1.0f);
    h.c1[i] = 2.0f * A[i];
    const float q = A[i] > 0.0f ? 1.0f : 0.0f;
    h.e0[i] = q * h.c0[i];
    h.e1[i] = q * h.c1[i];
  }
}

// exp(-4 pi s) = exp2(kGauss s)
constexpr float kGauss = -18.129440567308775f;

// Laue lattice offsets y = alpha - kappa without a zero.  The pixel's alpha gets a last
// mantissa bit of 1 and a magnitude clamped to [2^-18, 2^30] (tag_alpha); the node's kappa
// gets a last mantissa bit of 0 (tag_kappa, a zero stays a zero).  Then alpha != kappa: if
// |kappa| >= 2^-18 the two floats differ in their last bit within one binade or in their
// binade, and if |kappa| < 2^-18 they differ in magnitude.  So y, an exactly rounded
// difference, is not 0 and sin(2 pi y)/y needs no guard; |y| >= 2^-42 (the spacing of floats
// just below 2^-18), so the product of three y stays a normal float.  Both tags are odd
// functions of their argument (a Friedel mate, whose alpha and kappa are exact negatives,
// gets exactly negated offsets), except for the sign that a zero alpha takes, which is rare.
// They move a value by at most one unit in its last place, alpha by less than 2^-18 near
// zero (where sin(2 pi y)/y is flat); the upper clamp turns the far-away alpha of lanes
// outside the detector into a finite value outside every support.
__device__ __forceinline__ float tag_alpha(float v) {
  const float a = __builtin_amdgcn_fmed3f(fabsf(v), 0x1p-18f, 0x1p30f);
  return copysignf(__int_as_float(__float_as_int(a) | 1), v);
}
__device__ __forceinline__ float tag_kappa(float v) { return __int_as_float(__float_as_int(v) & ~1); }
__device__ __forceinline__ float4 tag_kappa4(float4 e) {
  return make_float4(tag_kappa(e.x), tag_kappa(e.y), tag_kappa(e.z), e.w);
}

// Per-lane evaluation of one queued node: returns omega times the lineshape's profile
// product (without its per-reflection constant) if the node is inside this pixel's support,
// else 0 (and counts it in COUNT mode).  TEST = false: the node lies in the pair's full box
// (inside the support of every pixel of the tile), so the support test is left out.
//   Laue:     (prod_i sin(2 pi y_i)/y_i)^2      (y_i = N_i u_i/2; al from tag_alpha and
//                                                nd from tag_kappa, so no y_i is 0)
//   Gaussian: exp(-4 pi sum_i y_i^2)            (y_i = N_i u_i/2)
//   Hosemann: 1/prod_i (c0_i - c1_i cos(2 pi y_i))   (y_i = u_i)
template <bool COUNT, int LS, bool TEST = true>
__device__ __forceinline__ void eval_node(const float4 nd, float al0, float al1, float al2, float half_m,
                                          const HoseK& hk, float& accr, unsigned long long& cnt) {
  float ya = al0 - nd.x, yb = al1 - nd.y, yc = al2 - nd.z;
  if (!TEST || fmaxf(fmaxf(fabsf(ya), fabsf(yb)), fabsf(yc)) <= half_m) {
    if (COUNT) {
      ++cnt;
    } else if (LS == FDTBX_LINESHAPE_GAUSSIAN) {
      const float s2 = fmaf(ya, ya, fmaf(yb, yb, yc * yc));
      accr = fmaf(nd.w, __builtin_amdgcn_exp2f(kGauss * s2), accr);
    } else if (LS == FDTBX_LINESHAPE_HOSEMANN) {
      const float da = fmaf(-hk.c1[0], __builtin_amdgcn_cosf(ya), hk.c0[0]);
      const float db = fmaf(-hk.c1[1], __builtin_amdgcn_cosf(yb), hk.c0[1]);
      const float dc = fmaf(-hk.c1[2], __builtin_amdgcn_cosf(yc), hk.c0[2]);
      accr = fmaf(nd.w, __builtin_amdgcn_rcpf(da * db * dc), accr);
    } else {
      // |y| throughout (free input modifiers): the hardware sine of a negative argument in
      // turns is reduced from another fraction, so sin(-y) = -sin(y) need not hold to the last
      // bit; with |y| a reflection and its Friedel mate give bit-identical terms
      ya = fabsf(ya);
      yb = fabsf(yb);
      yc = fabsf(yc);
      const float num = __builtin_amdgcn_sinf(ya) * __builtin_amdgcn_sinf(yb) * __builtin_amdgcn_sinf(yc);
      const float rr = num * __builtin_amdgcn_rcpf(ya * yb * yc);
      accr = fmaf(nd.w, rr * rr, accr);
    }
  }
}

// The Hosemann support edge.  The Hosemann factor does not vanish at |y| = 1/2, the edge of
// its one-period support, so where float32 and binary64 disagree on the side of the edge a node
// lies on, the pixel gains or loses that node's whole term.  A node whose float32 max_i |y_i| lies
// within the pair's edge band of the edge is decided again in binary64: the record's
// coefficients as hi + lo (float32 slot and residual, RS_LO: 2^-48 relative), the node's
// offsets recomputed from its index as the node table defines them, and the lane's binary64
// R - R_D, Z - Z_D.  The band bounds the float32 error of
// y_i = T_R,i dR + T_Z,i dZ - (B_i (c - 1) + G1_i c d1 + G2_i c d2), |c - 1| and |c d| <= 1,
// formed from float32 values with about six roundings, each within 2^-24 of
// mag_i = |T_R,i| max|dR| + |T_Z,i| max|dZ| + |B_i| + |G1_i| + |G2_i| (max over the tile's box):
// the band is 2^-20 max_i mag_i (16 such roundings), and never below 1e-6.  A node with
// mx = max_i |y_i| <= lo = 1/2 - band (in float32) is inside; one with lo < mx < hi = 1/2 + band
// is decided in binary64; the others are outside.  The context is uniform across the wave; the
// terms stay float32.
struct EdgeCtx {
  const float* rec;  // the pair's reflection record
  float lo, hi;      // the edge band's bounds on mx
  const int* qk;     // node index of each entry of the queue being walked
};

__device__ __forceinline__ EdgeCtx edge_ctx(const float* __restrict__ rec, const TileBox& box, const int* qk) {
  EdgeCtx ec;
  ec.rec = rec;
  const double RD = *(const double*)(rec + RS_RD), ZD = *(const double*)(rec + RS_ZD);
  const float mR = (float)fmax(fabs(box.Rlo - RD), fabs(box.Rhi - RD));
  const float mZ = (float)fmax(fabs(box.Zlo - ZD), fabs(box.Zhi - ZD));
  float mag = 0.0f;
  for (int a = 0; a < 3; ++a)
    mag = fmaxf(mag, fabsf(rec[RS_TR + a]) * mR + fabsf(rec[RS_TZ + a]) * mZ + fabsf(rec[RS_B + a]) +
                         fabsf(rec[RS_G1 + a]) + fabsf(rec[RS_G2 + a]));
  const float band = __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(fmaxf(1.0e-6f, mag * 0x1p-20f))));
  ec.lo = 0.5f - band;
  ec.hi = 0.5f + band;
  ec.qk = qk;
  return ec;
}

// Whether node k is inside the support (every |u_i| <= half_m) in binary64, for the query
// point's binary64 lattice offsets al_of(i) = scale_i a_i.(p - D) (formed axis by axis, inside
// the loop, which keeps this rare path's registers few).  The node's offsets are formed as the
// node table defines them, with c = 1/sqrt(1 + rho^2) from the binary64 reciprocal square root
// (within a few units in the last place) and c - 1 formed directly: its absolute error, about
// 1e-16, is all that enters u.
template <class AlOf>
__device__ __forceinline__ bool hose_inside64_f(const ProfParams& q, const float* rec, int k, AlOf&& al_of) {
  // coefficient c of axis a (c = 0..2: B, G1, G2) as hi + lo
  auto x64 = [&](int ca) { return (double)rec[RS_B + ca] + (double)rec[RS_LO + ca]; };
  int i1, i2;
  window_node(k, q.n, __builtin_amdgcn_rcpf((float)q.n), &i1, &i2);
  const double d1 = -q.T64 + ((double)i1 + 0.5) * q.h64, d2 = -q.T64 + ((double)i2 + 0.5) * q.h64;
  const double c = rsqrt(fma(d1, d1, fma(d2, d2, 1.0)));
  const double cm1 = c - 1.0, cd1 = c * d1, cd2 = c * d2;
  bool in = true;
#pragma unroll 1
  for (int a = 0; a < 3; ++a) {
    const double kap = fma(x64(a), cm1, fma(x64(3 + a), cd1, x64(6 + a) * cd2));
    in = in && fabs(al_of(a) - kap) <= (double)q.half_m;
  }
  return in;
}

// hose_inside64_f for offsets already formed in binary64 (the splat's samples, the points).
__device__ __forceinline__ bool hose_inside64_al(const ProfParams& q, const float* rec, int k, const double* al64) {
  return hose_inside64_f(q, rec, k, [&](int a) { return al64[a]; });
}

// hose_inside64_f at the query point p = D + dR e_perp + dY e_az + dZ z (a pixel: dY = 0; a
// ring point of the cylindrical average: dY = R sin(phi)), its offsets from the record's
// T_R, T_A, T_Z as hi + lo.
__device__ __forceinline__ bool hose_inside64(const ProfParams& q, const float* rec, int k, double dR, double dY,
                                              double dZ) {
  auto x64 = [&](int slot, int lo) { return (double)rec[slot] + (double)rec[lo]; };
  return hose_inside64_f(q, rec, k, [&](int a) {
    const double ta = dY != 0.0 ? x64(RS_TA + a, RS_LO_TA + a) * dY : 0.0;
    return fma(x64(RS_TR + a, RS_LO + 9 + a), dR, fma(x64(RS_TZ + a, RS_LO + 12 + a), dZ, ta));
  });
}

// hose_inside64 at the pixel (R, Z).
__device__ __forceinline__ bool hose_inside64_px(const ProfParams& q, const float* rec, int k, double R, double Z) {
  return hose_inside64(q, rec, k, R - *(const double*)(rec + RS_RD), 0.0, Z - *(const double*)(rec + RS_ZD));
}

// The Hosemann profile product at offsets (ya, yb, yc), before the node weight, as eval_node
// forms it.
__device__ __forceinline__ float hose_prod(float ya, float yb, float yc, const HoseK& hk) {
  const float da = fmaf(-hk.c1[0], __builtin_amdgcn_cosf(ya), hk.c0[0]);
  const float db = fmaf(-hk.c1[1], __builtin_amdgcn_cosf(yb), hk.c0[1]);
  const float dc = fmaf(-hk.c1[2], __builtin_amdgcn_cosf(yc), hk.c0[2]);
  return __builtin_amdgcn_rcpf(da * db * dc);
}

// The Hosemann walks in two passes.  The walk proper (eval_node_hose_main, queue entry jj) adds
// the nodes with mx <= lo and leaves out those in the band, setting bit jj of the wave's mask
// um where some lane met one; a second pass over the entries of um (hose_edge_pass) adds those
// whose binary64 decision is inside.  The double-precision work stays out of the walk's loop.
__device__ __forceinline__ bool hose_band(float mx, float lo, float hi) { return !(mx <= lo) && mx < hi; }

__device__ __forceinline__ void eval_node_hose_main(const float4 nd, const float* al, float lo, float hi,
                                                    const HoseK& hk, float& accr, int jj, unsigned long long& um) {
  const float ya = al[0] - nd.x, yb = al[1] - nd.y, yc = al[2] - nd.z;
  const float mx = fmaxf(fmaxf(fabsf(ya), fabsf(yb)), fabsf(yc));
  const bool sure = mx <= lo;
  // the band's lanes as (mx < hi) and not sure: two compares, the rest scalar
  const unsigned long long band = __builtin_amdgcn_ballot_w64(mx < hi) & ~__builtin_amdgcn_ballot_w64(sure);
  um = band ? um | (1ull << jj) : um;
  if (sure) accr = fmaf(nd.w, hose_prod(ya, yb, yc, hk), accr);
}

// The second pass: the entries um of the queue qn (node indices ec.qk) at the pixel (R, Z)
// with offsets al; adds the terms of the band's nodes that are inside in binary64.
__device__ __forceinline__ void hose_edge_pass(const ProfParams& q, const float4* qn, unsigned long long um,
                                               const float* al, const HoseK& hk, const EdgeCtx& ec, double R,
                                               double Z, float& accr) {
  float part = 0.0f;
  while (um) {  // uniform
    const int jj = (int)__builtin_ctzll(um);
    um &= um - 1;
    const float4 nd = qn[jj];
    const float ya = al[0] - nd.x, yb = al[1] - nd.y, yc = al[2] - nd.z;
    const float mx = fmaxf(fmaxf(fabsf(ya), fabsf(yb)), fabsf(yc));
    if (hose_band(mx, ec.lo, ec.hi) && hose_inside64_px(q, ec.rec, ec.qk[jj], R, Z))
      part = fmaf(nd.w, hose_prod(ya, yb, yc, hk), part);
  }
  accr += part;
}

// The walk of one wave's node queue (128 entries of LDS; see pairs_sum below).
// Every lane walks the first cnt queue entries; the read of entry jj + 1 is issued before
// entry jj is evaluated (the buffer holds 128 entries, cnt <= 64, so it stays in bounds).
// The queue is addressed from threadIdx.y (always 0: the launches are one-dimensional), which
// keeps its address in a vector register; the unrolled reads then use instruction offsets
// instead of moving a scalar loop counter into a vector register for every entry.
// With an edge context (the Hosemann lineshape's tested walks) the support edge is decided in
// the two passes above for the pixel (R, Z); ec->qk is then the queue's node indices.
template <bool COUNT, int LS, bool TEST = true>
__device__ __forceinline__ void walk_queue(const float4* qn, int cnt, const float* al, float half_m,
                                           const HoseK& hk, float& accr, unsigned long long& cnt_eval,
                                           const ProfParams* qe = nullptr, const EdgeCtx* ec = nullptr,
                                           double R = 0.0, double Z = 0.0) {
  constexpr bool EDGE = LS == FDTBX_LINESHAPE_HOSEMANN && TEST && !COUNT;
  const float4* const q0 = qn;
  qn += threadIdx.y;
  float4 nxt = qn[0];
  float part = 0.0f;  // a block sum of at most 64 terms, added once: keeps long sums accurate
  unsigned long long um = 0;
  const float lo = EDGE && ec ? ec->lo : 0.0f, hi = EDGE && ec ? ec->hi : 0.0f;
  for (int jj = 0; jj < cnt; ++jj) {
    const float4 cur = nxt;
    nxt = qn[jj + 1];
    if (EDGE && ec)
      eval_node_hose_main(cur, al, lo, hi, hk, part, jj, um);
    else
      eval_node<COUNT, LS, TEST>(cur, al[0], al[1], al[2], half_m, hk, part, cnt_eval);
    // without the support test the unrolled entries form one block, which the scheduler would
    // interleave at the cost of registers (and occupancy); keep each entry's arithmetic together
    if (!TEST) __builtin_amdgcn_sched_barrier(0);
  }
  accr += part;
  if (EDGE && ec && um) hose_edge_pass(*qe, q0, um, al, hk, *ec, R, Z, accr);
}

// Appends the lanes' candidates (keep) to a queue of len entries at qn (len is uniform).
// With qk, node index k goes to the same position of qk.
template <int LS>
__device__ __forceinline__ void queue_append(float4* qn, int& len, bool keep, float4 e, int* qk = nullptr,
                                             int k = 0) {
  const unsigned long long b = __ballot(keep);
  if (keep) {
    const int pos = len + (int)__builtin_amdgcn_mbcnt_hi((unsigned)(b >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)b, 0u));
    qn[pos] = LS == FDTBX_LINESHAPE_LAUE ? tag_kappa4(e) : e;
    if (qk) qk[pos] = k;
  }
  len += __popcll(b);
}

// Walks the first 64 entries of a queue by all lanes once it holds that many (the rest move
// to the front).
template <bool COUNT, int LS, bool TEST>
__device__ __forceinline__ void queue_flush(float4* qn, int& len, const float* al, float half_m, const HoseK& hk,
                                            float& accr, unsigned long long& cnt, const ProfParams* qe = nullptr,
                                            const EdgeCtx* ec = nullptr, int* qk = nullptr, double R = 0.0,
                                            double Z = 0.0) {
  if (len >= 64) {
    const int lane = threadIdx.x & 63;
    walk_queue<COUNT, LS, TEST>(qn, 64, al, half_m, hk, accr, cnt, qe, ec, R, Z);
    len -= 64;
    wave_sync();
    if (lane < len) {
      qn[lane] = qn[64 + lane];
      if (qk) qk[lane] = qk[64 + lane];
    }
    wave_sync();
  }
}

// A lane's pixel sum over pairs of one tile's list: the chunks of 64 pairs that start at
// from, from + step, from + 2 step, ... below p1 (each lane sets up one pair of a chunk: its
// node window and alpha box; the wave then works through the pairs with a non-empty window,
// reading their set-up from that lane).  R, Z: the lane's pixel; box: the tile's (R, Z) box.
// qn, bq: this wave's LDS queues (256 float4; 128 without SPLIT) and scratch (64 ints).  The
// pair's candidate nodes go to the queue at qn; with SPLIT, those in the pair's full box
// (inside the support of every pixel of the tile) go to a second queue at qn + 128 instead,
// whose walk leaves out the support test.  Each queue is walked 64 entries at a time as it
// fills, and both at the end of the pair, the full queue first; the pixel sum adds each walk's
// block sum in that order.
template <bool COUNT, int LS, bool PRE = false, bool SPLIT = !COUNT>
__device__ __forceinline__ float pairs_sum(const ProfParams& q, const float* __restrict__ refl,
                                           const float* __restrict__ nodes, const int32_t* __restrict__ idx,
                                           const TileBox& box, double R, double Z, int64_t from, int64_t p1,
                                           int64_t step, float4* qn, int* bq, unsigned long long& cnt,
                                           int* qk = nullptr) {
  static_assert(!(SPLIT && COUNT), "the counting pass tests every node");
  constexpr bool EDGE = LS == FDTBX_LINESHAPE_HOSEMANN && !COUNT;
  const int lane = threadIdx.x & 63;
  float acc = 0.0f;
  for (int64_t base = from; base < p1; base += step) {
    int32_t rl = 0;
    int w01 = 0, w23 = 0;
    float lol[3] = {0.f, 0.f, 0.f}, hil[3] = {0.f, 0.f, 0.f}, fll[3] = {0.f, 0.f, 0.f}, fhl[3] = {0.f, 0.f, 0.f};
    bool ok = false;
    if (base + lane < p1) {
      rl = idx[base + lane];
      ok = pair_setup<PRE>(q, refl + (int64_t)FDTBX_REFL_FLOATS * rl, nodes, box, &w01, &w23, lol, hil,
                           SPLIT ? fll : nullptr, SPLIT ? fhl : nullptr);
    }
    unsigned long long todo = __ballot(ok);
    while (todo) {
      const int src = (int)__builtin_ctzll(todo);
      todo &= todo - 1;
      const int32_t r = lane_int(rl, src);
      const int a01 = lane_int(w01, src), a23 = lane_int(w23, src);
      const Window w = {a01 & 0xffff, a01 >> 16, a23 & 0xffff, a23 >> 16};
      float al[3], lo[3], hi[3], fl[3], fh[3], Bv[3], G1[3], G2[3];
      PairRec f;
      load_pair(refl + (int64_t)FDTBX_REFL_FLOATS * r, f);
      const float dR = (float)(R - f.at_f64(RS_RD)), dZ = (float)(Z - f.at_f64(RS_ZD));
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        al[a] = fmaf(f.at(RS_TR + a), dR, f.at(RS_TZ + a) * dZ);
        if (LS == FDTBX_LINESHAPE_LAUE) al[a] = tag_alpha(al[a]);
        lo[a] = lane_float(lol[a], src);
        hi[a] = lane_float(hil[a], src);
        fl[a] = SPLIT ? lane_float(fll[a], src) : 0.0f;
        fh[a] = SPLIT ? lane_float(fhl[a], src) : 0.0f;
        Bv[a] = f.at(RS_B + a);
        G1[a] = f.at(RS_G1 + a);
        G2[a] = f.at(RS_G2 + a);
      }
      HoseK hk = {};
      if (LS == FDTBX_LINESHAPE_HOSEMANN && !COUNT) hose_constants(refl + (int64_t)FDTBX_REFL_FLOATS * r, hk);
      // the Hosemann support edge is decided in binary64 (hose_edge_pass): the tested queue
      // then carries its node indices in qk
      EdgeCtx ec = {};
      if (EDGE) ec = edge_ctx(refl + (int64_t)FDTBX_REFL_FLOATS * r, box, qk);
      const EdgeCtx* ecp = EDGE ? &ec : nullptr;
      int* qkp = EDGE ? qk : nullptr;
      float accr = 0.0f;
      int qlen = 0, flen = 0;  // uniform
      // candidates go to the LDS queues; every 64 queued nodes are walked by all lanes
      scan_window(q, nodes, w, Bv, G1, G2, lo, hi, bq, [&](bool keep, int k, float4 e) {
        if (SPLIT) {
          const bool full = keep && e.x >= fl[0] && e.x <= fh[0] && e.y >= fl[1] && e.y <= fh[1] && e.z >= fl[2] &&
                            e.z <= fh[2];
          queue_append<LS>(qn + 128, flen, full, e);
          queue_append<LS>(qn, qlen, keep && !full, e, qkp, k);
          wave_sync();
          queue_flush<COUNT, LS, false>(qn + 128, flen, al, q.half_m, hk, accr, cnt);
        } else {
          queue_append<LS>(qn, qlen, keep, e, qkp, k);
          wave_sync();
        }
        queue_flush<COUNT, LS, true>(qn, qlen, al, q.half_m, hk, accr, cnt, &q, ecp, qkp, R, Z);
      });
      if (SPLIT) walk_queue<COUNT, LS, false>(qn + 128, flen, al, q.half_m, hk, accr, cnt);
      walk_queue<COUNT, LS>(qn, qlen, al, q.half_m, hk, accr, cnt, &q, ecp, R, Z);
      wave_sync();
      if (!COUNT) acc = fmaf(f.at(RS_WK), accr, acc);
    }
  }
  return acc;
}

// The walk of walk_queue for a lane holding two pixels (al, bl: their tagged alpha): each
// entry is tested and evaluated for both, with a block sum each.
// For the Hosemann lineshape the support edge is decided in the two passes of walk_queue (ec,
// the pair's edge context, and the pixels (RA, ZA) and (RB, ZB)).
template <int LS>
__device__ __forceinline__ void walk_queue2(const ProfParams& q, const float4* qn, int cnt, const float* al,
                                            const float* bl, const HoseK& hk, const EdgeCtx& ec, double RA,
                                            double ZA, double RB, double ZB, float& acca, float& accb) {
  constexpr bool EDGE = LS == FDTBX_LINESHAPE_HOSEMANN;
  const float4* const q0 = qn;
  qn += threadIdx.y;
  float4 nxt = qn[0];
  float pa = 0.0f, pb = 0.0f;
  unsigned long long none = 0, ua = 0, ub = 0;  // ua, ub: the edge masks of the two pixels
  for (int jj = 0; jj < cnt; ++jj) {
    const float4 cur = nxt;
    nxt = qn[jj + 1];
    if (EDGE) {
      eval_node_hose_main(cur, al, ec.lo, ec.hi, hk, pa, jj, ua);
      eval_node_hose_main(cur, bl, ec.lo, ec.hi, hk, pb, jj, ub);
    } else {
      eval_node<false, LS>(cur, al[0], al[1], al[2], q.half_m, hk, pa, none);
      eval_node<false, LS>(cur, bl[0], bl[1], bl[2], q.half_m, hk, pb, none);
    }
  }
  acca += pa;
  accb += pb;
  if (EDGE && ua) hose_edge_pass(q, q0, ua, al, hk, ec, RA, ZA, acca);
  if (EDGE && ub) hose_edge_pass(q, q0, ub, bl, hk, ec, RB, ZB, accb);
}

// pairs_sum for a stacked tile: two vertically adjacent tiles walked by one wave, lane l
// holding pixel l of the upper tile (RA, ZA) and of the lower one (RB, ZB; far from every
// reflection when the stacked tile has one row of tiles).  The pairs are those of the stacked
// tile's list, set up against its box (the union of the two tiles' boxes) with the block
// narrowing of the batched launches; one queue serves both pixels, so each pair's set-up,
// window scan and queue reads are shared by the two tiles.  *sa, *sb: the two pixel sums.
template <int LS>
__device__ __forceinline__ void pairs_sum_stacked(const ProfParams& q, const float* __restrict__ refl,
                                                  const float* __restrict__ nodes, const int32_t* __restrict__ idx,
                                                  const TileBox& box, double RA, double ZA, double RB, double ZB,
                                                  int64_t from, int64_t p1, float4* qn, int* bq, float* sa,
                                                  float* sb, int* qk = nullptr) {
  const int lane = threadIdx.x & 63;
  constexpr bool EDGE = LS == FDTBX_LINESHAPE_HOSEMANN;
  float acca = 0.0f, accb = 0.0f;
  for (int64_t base = from; base < p1; base += 64) {
    int32_t rl = 0;
    int w01 = 0, w23 = 0;
    float lol[3] = {0.f, 0.f, 0.f}, hil[3] = {0.f, 0.f, 0.f};
    bool ok = false;
    if (base + lane < p1) {
      rl = idx[base + lane];
      ok = pair_setup<true>(q, refl + (int64_t)FDTBX_REFL_FLOATS * rl, nodes, box, &w01, &w23, lol, hil);
    }
    unsigned long long todo = __ballot(ok);
    while (todo) {
      const int src = (int)__builtin_ctzll(todo);
      todo &= todo - 1;
      const int32_t r = lane_int(rl, src);
      const int a01 = lane_int(w01, src), a23 = lane_int(w23, src);
      const Window w = {a01 & 0xffff, a01 >> 16, a23 & 0xffff, a23 >> 16};
      float al[3], bl[3], lo[3], hi[3], Bv[3], G1[3], G2[3];
      PairRec f;
      load_pair(refl + (int64_t)FDTBX_REFL_FLOATS * r, f);
      const double RD = f.at_f64(RS_RD), ZD = f.at_f64(RS_ZD);
      const float dRa = (float)(RA - RD), dZa = (float)(ZA - ZD);
      const float dRb = (float)(RB - RD), dZb = (float)(ZB - ZD);
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        al[a] = fmaf(f.at(RS_TR + a), dRa, f.at(RS_TZ + a) * dZa);
        bl[a] = fmaf(f.at(RS_TR + a), dRb, f.at(RS_TZ + a) * dZb);
        if (LS == FDTBX_LINESHAPE_LAUE) {
          al[a] = tag_alpha(al[a]);
          bl[a] = tag_alpha(bl[a]);
        }
        lo[a] = lane_float(lol[a], src);
        hi[a] = lane_float(hil[a], src);
        Bv[a] = f.at(RS_B + a);
        G1[a] = f.at(RS_G1 + a);
        G2[a] = f.at(RS_G2 + a);
      }
      HoseK hk = {};
      if (LS == FDTBX_LINESHAPE_HOSEMANN) hose_constants(refl + (int64_t)FDTBX_REFL_FLOATS * r, hk);
      EdgeCtx ec = {};
      if (EDGE) ec = edge_ctx(refl + (int64_t)FDTBX_REFL_FLOATS * r, box, qk);
      int* qkp = EDGE ? qk : nullptr;
      float ra = 0.0f, rb = 0.0f;
      int qlen = 0;  // uniform
      scan_window(q, nodes, w, Bv, G1, G2, lo, hi, bq, [&](bool keep, int k, float4 e) {
        queue_append<LS>(qn, qlen, keep, e, qkp, k);
        wave_sync();
        if (qlen >= 64) {
          walk_queue2<LS>(q, qn, 64, al, bl, hk, ec, RA, ZA, RB, ZB, ra, rb);
          qlen -= 64;
          wave_sync();
          if (lane < qlen) {
            qn[lane] = qn[64 + lane];
            if (EDGE) qk[lane] = qk[64 + lane];
          }
          wave_sync();
        }
      });
      walk_queue2<LS>(q, qn, qlen, al, bl, hk, ec, RA, ZA, RB, ZB, ra, rb);
      wave_sync();
      acca = fmaf(f.at(RS_WK), ra, acca);
      accb = fmaf(f.at(RS_WK), rb, accb);
    }
  }
  *sa = acca;
  *sb = accb;
}

// The pixel of lane `lane` in tile t: its column i, row j, whether it lies on the detector,
// and its ring coordinates (lanes outside the detector sit far from every reflection, so all
// supports fail); and the tile's (R, Z) box.
struct TilePixel {
  int tx, ty, i, j;
  bool in;
  double R, Z;
  TileBox box;
};

__device__ __forceinline__ TilePixel tile_pixel(const ProfParams& q, const double* __restrict__ pix,
                                                const double* __restrict__ tile, int t, int lane) {
  TilePixel p;
  p.tx = t % q.tiles_x;
  p.ty = t / q.tiles_x;
  p.i = (p.tx << q.tlg) + (lane & ((1 << q.tlg) - 1));
  p.j = p.ty * (64 >> q.tlg) + (lane >> q.tlg);
  p.in = p.i < q.W && p.j < q.H;
  p.R = p.in ? pix[2 * ((int64_t)p.j * q.W + p.i) + 0] : 1.0e30;
  p.Z = p.in ? pix[2 * ((int64_t)p.j * q.W + p.i) + 1] : 0.0;
  p.box = {tile[8 * (int64_t)t + 0], tile[8 * (int64_t)t + 1], tile[8 * (int64_t)t + 2], tile[8 * (int64_t)t + 3]};
  return p;
}

// WAVES waves share a tile: wave w takes the chunks w, w + WAVES, ... of 64 pairs of the
// tile's list (its own LDS queues: qn + 256 w, bq + 64 w; 128 float4 per wave suffice
// without SPLIT; for the Hosemann lineshape also qk + 128 w, the node indices of the tested
// queue), and wave 0 adds the others' pixel sums (xacc, 64 floats per extra wave) in wave
// order before it writes the tile.
template <bool COUNT, int LS, int WAVES = 1, bool PRE = false, bool SPLIT = !COUNT>
__device__ __forceinline__ void profile_tile(const ProfParams& q, const float* __restrict__ refl,
                                             const float* __restrict__ nodes, const double* __restrict__ pix,
                                             const double* __restrict__ tile, const int64_t* __restrict__ offsets,
                                             const int32_t* __restrict__ idx, float* __restrict__ image,
                                             unsigned long long* __restrict__ counts, const int t, float4* qn, int* bq,
                                             float* xacc = nullptr, int* qk = nullptr) {
  const int lane = threadIdx.x & 63;
  const int wv = WAVES > 1 ? (int)(threadIdx.x >> 6) : 0;
  qn += 256 * wv;
  bq += 64 * wv;
  if (qk) qk += 128 * wv;
  const TilePixel px = tile_pixel(q, pix, tile, t, lane);
  unsigned long long cnt = 0;
  float acc = pairs_sum<COUNT, LS, PRE, SPLIT>(q, refl, nodes, idx, px.box, px.R, px.Z, offsets[t] + 64 * wv,
                                              offsets[t + 1], 64 * WAVES, qn, bq, cnt, qk);
  if (COUNT) {
    for (int o = 32; o >= 1; o >>= 1) cnt += __shfl_xor(cnt, o, 64);
    if (lane == 0 && cnt) atomicAdd(counts, cnt);
  } else {
    if (WAVES > 1) {
      if (wv > 0) xacc[64 * (wv - 1) + lane] = acc;
      __syncthreads();
      if (wv > 0) return;
      for (int k = 1; k < WAVES; ++k) acc += xacc[64 * (k - 1) + lane];
    }
    if (!px.in) return;
    write_folded(q, image, px.i, px.j, px.tx, px.ty, (float)(q.delta / (px.R + q.delta)) * acc);
  }
}

}  // namespace fdtbx
