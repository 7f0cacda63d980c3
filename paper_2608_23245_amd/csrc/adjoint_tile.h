// Per-tile body of the adjoint profile kernel, shared by the single-model and the
// batched launches (see adjoint.hip for the quantities it accumulates).
#pragma once

#include "profile_common.h"
#include "profile_tile.h"

namespace fdtbx {

// Adjoint of eval_node for one queued node (nd = kappa, omega; dw = d omega/d sigma,
// d omega/d gamma), before the lane's pixel weight (applied once per (tile, reflection) pair).
// With Z' the lineshape's profile product as in eval_node:
//   acc[0] += omega Z',  acc[1] += dw.x Z',  acc[2] += dw.y Z',
//   acc[3+i] += omega N_i (dZ/dN_i)/C   (the profile's N-derivative at fixed u, C its
//                                        per-reflection constant; see the header).
// Laue:     S_i (4 pi cos(2 pi y_i) - S_i) prod_{j!=i} S_j^2 with S_i = sin(2 pi y_i)/y_i.
// Gaussian: Z' (1 - 8 pi y_i^2).
// Hosemann: Z' (c_i (1 + A_i^2) - 2 A_i)/den_i with c_i = cos(2 pi y_i) (0 where A_i is held at 0).
// adj_term adds the node's terms at offsets (ya, yb, yc); eval_node_adj tests the support
// first.  For the Hosemann lineshape with um, nodes in the edge band (lo, hi) are left out and
// bit jj of *um is set where some lane met one, for the second pass of walk_queue_adj (the two
// passes of the forward walk).
template <int LS>
__device__ __forceinline__ void adj_term(float ya, float yb, float yc, const float4 nd, const float2 dw,
                                         const HoseK& hk, float* acc) {
  {
    if (LS == FDTBX_LINESHAPE_GAUSSIAN) {
      const float P = __builtin_amdgcn_exp2f(kGauss * fmaf(ya, ya, fmaf(yb, yb, yc * yc)));
      acc[0] = fmaf(nd.w, P, acc[0]);
      acc[1] = fmaf(dw.x, P, acc[1]);
      acc[2] = fmaf(dw.y, P, acc[2]);
      const float t2 = nd.w * P;
      const float m8pi = -25.132741228718345f;
      acc[3] = fmaf(t2, fmaf(m8pi, ya * ya, 1.0f), acc[3]);
      acc[4] = fmaf(t2, fmaf(m8pi, yb * yb, 1.0f), acc[4]);
      acc[5] = fmaf(t2, fmaf(m8pi, yc * yc, 1.0f), acc[5]);
    } else if (LS == FDTBX_LINESHAPE_HOSEMANN) {
      const float ca = __builtin_amdgcn_cosf(ya), cb = __builtin_amdgcn_cosf(yb), cc = __builtin_amdgcn_cosf(yc);
      const float da = fmaf(-hk.c1[0], ca, hk.c0[0]);
      const float db = fmaf(-hk.c1[1], cb, hk.c0[1]);
      const float dc = fmaf(-hk.c1[2], cc, hk.c0[2]);
      const float dab = da * db;
      const float P = __builtin_amdgcn_rcpf(dab * dc);
      acc[0] = fmaf(nd.w, P, acc[0]);
      acc[1] = fmaf(dw.x, P, acc[1]);
      acc[2] = fmaf(dw.y, P, acc[2]);
      // 1/den_a = P db dc, ...
      const float t2 = nd.w * P * P;
      acc[3] = fmaf(t2 * (db * dc), fmaf(ca, hk.e0[0], -hk.e1[0]), acc[3]);
      acc[4] = fmaf(t2 * (da * dc), fmaf(cb, hk.e0[1], -hk.e1[1]), acc[4]);
      acc[5] = fmaf(t2 * dab, fmaf(cc, hk.e0[2], -hk.e1[2]), acc[5]);
    } else {
      // no y is 0 (tag_alpha, tag_kappa); every factor below is even in its y, and |y| keeps
      // the hardware sine and cosine on positive arguments as in the forward
      ya = fabsf(ya);
      yb = fabsf(yb);
      yc = fabsf(yc);
      const float sa = __builtin_amdgcn_sinf(ya), sb = __builtin_amdgcn_sinf(yb), sc = __builtin_amdgcn_sinf(yc);
      const float ca = __builtin_amdgcn_cosf(ya), cb = __builtin_amdgcn_cosf(yb), cc = __builtin_amdgcn_cosf(yc);
      const float yab = ya * yb;
      const float inv = __builtin_amdgcn_rcpf(yab * yc);
      const float Sa = sa * (inv * (yb * yc));
      const float Sb = sb * (inv * (ya * yc));
      const float Sc = sc * (inv * yab);
      const float Pa = Sa * Sa, Pb = Sb * Sb, Pc = Sc * Sc;
      const float Pab = Pa * Pb;
      const float P = Pab * Pc;
      acc[0] = fmaf(nd.w, P, acc[0]);
      acc[1] = fmaf(dw.x, P, acc[1]);
      acc[2] = fmaf(dw.y, P, acc[2]);
      const float four_pi = 12.566370614359172f;
      acc[3] = fmaf(nd.w, Sa * fmaf(four_pi, ca, -Sa) * (Pb * Pc), acc[3]);
      acc[4] = fmaf(nd.w, Sb * fmaf(four_pi, cb, -Sb) * (Pa * Pc), acc[4]);
      acc[5] = fmaf(nd.w, Sc * fmaf(four_pi, cc, -Sc) * Pab, acc[5]);
    }
  }
}

template <int LS>
__device__ __forceinline__ void eval_node_adj(const float4 nd, const float2 dw, float al0, float al1, float al2,
                                              float half_m, const HoseK& hk, float* acc, float lo = 0.0f,
                                              float hi = 0.0f, int jj = 0, unsigned long long* um = nullptr) {
  const float ya = al0 - nd.x, yb = al1 - nd.y, yc = al2 - nd.z;
  const float mx = fmaxf(fmaxf(fabsf(ya), fabsf(yb)), fabsf(yc));
  bool in = mx <= half_m;
  if (LS == FDTBX_LINESHAPE_HOSEMANN && um) {
    in = mx <= lo;
    const unsigned long long band = __builtin_amdgcn_ballot_w64(mx < hi) & ~__builtin_amdgcn_ballot_w64(in);
    *um = band ? *um | (1ull << jj) : *um;
  }
  if (in) adj_term<LS>(ya, yb, yc, nd, dw, hk, acc);
}

// Every lane walks the first cnt queue entries, reading entry jj + 1 before evaluating jj.
// The queue addresses go through threadIdx.y (always 0) so that they stay in vector
// registers and the unrolled reads use instruction offsets.
template <int LS>
__device__ __forceinline__ void walk_queue_adj(const float4* qn, const float2* qd, int cnt, const float* al, float half_m,
                                               const HoseK& hk, float* acc, const ProfParams* qe = nullptr,
                                               const EdgeCtx* ec = nullptr, double R = 0.0, double Z = 0.0) {
  constexpr bool EDGE = LS == FDTBX_LINESHAPE_HOSEMANN;
  const float4* const q0 = qn;
  const float2* const d0 = qd;
  qn += threadIdx.y;
  qd += threadIdx.y;
  float4 nxt = qn[0];
  float2 nxt2 = qd[0];
  unsigned long long um = 0;
  const float lo = EDGE && ec ? ec->lo : 0.0f, hi = EDGE && ec ? ec->hi : 0.0f;
  for (int jj = 0; jj < cnt; ++jj) {
    const float4 cur = nxt;
    const float2 cur2 = nxt2;
    nxt = qn[jj + 1];
    nxt2 = qd[jj + 1];
    eval_node_adj<LS>(cur, cur2, al[0], al[1], al[2], half_m, hk, acc, lo, hi, jj, EDGE && ec ? &um : nullptr);
  }
  // the second pass: the band's nodes that are inside in binary64 (hose_edge_pass)
  while (EDGE && ec && um) {  // uniform
    const int jj = (int)__builtin_ctzll(um);
    um &= um - 1;
    const float4 nd = q0[jj];
    const float ya = al[0] - nd.x, yb = al[1] - nd.y, yc = al[2] - nd.z;
    const float mx = fmaxf(fmaxf(fabsf(ya), fabsf(yb)), fabsf(yc));
    if (hose_band(mx, lo, hi) && hose_inside64_px(*qe, ec->rec, ec->qk[jj], R, Z))
      adj_term<LS>(ya, yb, yc, nd, d0[jj], hk, acc);
  }
}

// One tile t of one model, walked by WAVES 64-lane waves: wave w takes the chunks w,
// w + WAVES, ... of 64 pairs of the tile's list (each pair's sums go out on their own, so the
// waves need no combining).  qn, qd: LDS queues of 128 entries per wave; bq: LDS scratch of
// 64 ints per wave for the block test; qk (the Hosemann lineshape): the queue's node indices,
// 128 per wave, for the binary64 support-edge decisions.
//
// Each lane holds two pixel weights: gA = L(R) (G of the pixel + G of its left-right mirror,
// which has the same profile value from the same reflection) and gB = L(R) (G of its up-down
// mirrors, under bit 1 of the fold), whose profile value comes from the Friedel mate -r at this
// pixel (I_r(R, -Z) = I_{-r}(R, Z)).  Per pair the six unweighted lane sums are weighted by gA
// into reflection r's sums and by gB into its mate's, n_hkl - 1 - r (the reflection list is
// closed under negation in that order).  With partials == nullptr they are added into sums
// (binary64 [n_hkl][6]) with hardware atomics; otherwise pair p of the culling lists stores its
// twelve float32 sums (r's six, then the mate's six; zero without the up-down fold) at
// partials[12 p], for a reduction in a fixed order (fdtbx_pair_reduce).
//
// adjoint_range walks the chunks of 64 pairs of tile t's list that start at from, from + step,
// ... below p1, with this wave's queues qn, qd, bq; adjoint_tile gives each of its WAVES waves
// its share of the list, and the balanced launch gives a wave one unit of the list at a time.
template <int LS, bool PRE = false>
__device__ __forceinline__ void adjoint_range(const ProfParams& q, const float* __restrict__ refl,
                                              const float* __restrict__ nodes, const double* __restrict__ pix,
                                              const double* __restrict__ tile, const int32_t* __restrict__ idx,
                                              const float* __restrict__ grad_image, int64_t n_hkl,
                                              double* __restrict__ sums, float* __restrict__ partials, const int t,
                                              int64_t from, int64_t p1, int64_t step, float4* qn, float2* qd, int* bq,
                                              int* qk = nullptr) {
  const int lane = threadIdx.x & 63;
  constexpr bool EDGE = LS == FDTBX_LINESHAPE_HOSEMANN;
  const int tx = t % q.tiles_x, ty = t / q.tiles_x;
  const int i = (tx << q.tlg) + (lane & ((1 << q.tlg) - 1));
  const int j = ty * (64 >> q.tlg) + (lane >> q.tlg);
  const bool in = i < q.W && j < q.H;
  const double R = in ? pix[2 * ((int64_t)j * q.W + i) + 0] : 1.0e30;
  const double Z = in ? pix[2 * ((int64_t)j * q.W + i) + 1] : 0.0;
  // under the mirror folds this pixel also stands for its mirror images
  float wa = 0.0f, wb = 0.0f;
  if (in) folded_weights(q, grad_image, i, j, tx, ty, &wa, &wb);
  const bool mate = (q.mirror & 2) && 2 * ty + 1 != q.tiles_y;  // uniform: the tile has mirror rows
  const float lor = (float)(q.delta / (R + q.delta));
  const float gA = wa * lor, gB = wb * lor;
  const TileBox box = {tile[8 * (int64_t)t + 0], tile[8 * (int64_t)t + 1], tile[8 * (int64_t)t + 2],
                       tile[8 * (int64_t)t + 3]};
  // a tile whose pixels all carry zero weight adds nothing
  if (__ballot(gA != 0.0f || gB != 0.0f) == 0ull) return;
  // 64 pairs at a time, set up lane-parallel as in the forward tile loop
  for (int64_t base = from; base < p1; base += step) {
    int32_t rl = 0;
    int w01 = 0, w23 = 0;
    float lol[3] = {0.f, 0.f, 0.f}, hil[3] = {0.f, 0.f, 0.f};
    bool ok = false;
    if (base + lane < p1) {
      rl = idx[base + lane];
      ok = pair_setup<PRE>(q, refl + (int64_t)FDTBX_REFL_FLOATS * rl, nodes, box, &w01, &w23, lol, hil);
    }
    unsigned long long todo = __ballot(ok);
    while (todo) {
      const int src = (int)__builtin_ctzll(todo);
      todo &= todo - 1;
      const int32_t r = lane_int(rl, src);
      const int a01 = lane_int(w01, src), a23 = lane_int(w23, src);
      const Window w = {a01 & 0xffff, a01 >> 16, a23 & 0xffff, a23 >> 16};
      float al[3], lo[3], hi[3], Bv[3], G1[3], G2[3];
      PairRec f;
      load_pair(refl + (int64_t)FDTBX_REFL_FLOATS * r, f);
      const float dR = (float)(R - f.at_f64(RS_RD)), dZ = (float)(Z - f.at_f64(RS_ZD));
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        al[a] = fmaf(f.at(RS_TR + a), dR, f.at(RS_TZ + a) * dZ);
        if (LS == FDTBX_LINESHAPE_LAUE) al[a] = tag_alpha(al[a]);
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
      const EdgeCtx* ecp = EDGE ? &ec : nullptr;
      float acc[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
      int qlen = 0, queued = 0;  // uniform
      scan_window(q, nodes, w, Bv, G1, G2, lo, hi, bq, [&](bool keep, int k, float4 e) {
        const unsigned long long b = __ballot(keep);
        if (keep) {
          const int pos = qlen + (int)__builtin_amdgcn_mbcnt_hi((unsigned)(b >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)b, 0u));
          qn[pos] = LS == FDTBX_LINESHAPE_LAUE ? tag_kappa4(e) : e;
          qd[pos] = *(const float2*)(nodes + (int64_t)FDTBX_NODE_FLOATS * k + 4);
          if (EDGE) qk[pos] = k;
        }
        qlen += __popcll(b);
        queued += __popcll(b);
        wave_sync();
        if (qlen >= 64) {
          walk_queue_adj<LS>(qn, qd, 64, al, q.half_m, hk, acc, &q, ecp, R, Z);
          qlen -= 64;
          wave_sync();
          if (lane < qlen) {
            qn[lane] = qn[64 + lane];
            qd[lane] = qd[64 + lane];
            if (EDGE) qk[lane] = qk[64 + lane];
          }
          wave_sync();
        }
      });
      walk_queue_adj<LS>(qn, qd, qlen, al, q.half_m, hk, acc, &q, ecp, R, Z);
      wave_sync();
      if (queued == 0) continue;  // no node within reach of the tile: nothing to add
      // the weighted lane sums are summed over the wave in binary64 (a float times a float is
      // exact there): the pixel weights G carry both signs, and the sums cancel
      double sA[6], sB[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
      bool anyA = false, anyB = false;
#pragma unroll
      for (int c = 0; c < 6; ++c) {
        sA[c] = wave_sum_f64((double)gA * (double)acc[c]);
        anyA |= sA[c] != 0.0;
      }
      if (mate) {
#pragma unroll
        for (int c = 0; c < 6; ++c) {
          sB[c] = wave_sum_f64((double)gB * (double)acc[c]);
          anyB |= sB[c] != 0.0;
        }
      }
      if (lane == 0 && (anyA || anyB)) {
        if (partials) {
          float* o = partials + 12 * (base + src);
#pragma unroll
          for (int c = 0; c < 6; ++c) {
            o[c] = (float)sA[c];
            o[6 + c] = (float)sB[c];
          }
        } else {
          if (anyA) {
#pragma unroll
            for (int c = 0; c < 6; ++c) unsafeAtomicAdd(&sums[6 * (int64_t)r + c], sA[c]);
          }
          if (anyB) {
            const int64_t rm = n_hkl - 1 - r;
#pragma unroll
            for (int c = 0; c < 6; ++c) unsafeAtomicAdd(&sums[6 * rm + c], sB[c]);
          }
        }
      }
    }
  }
}

template <int LS, int WAVES = 1, bool PRE = false>
__device__ __forceinline__ void adjoint_tile(const ProfParams& q, const float* __restrict__ refl, const float* __restrict__ nodes,
                                             const double* __restrict__ pix, const double* __restrict__ tile,
                                             const int64_t* __restrict__ offsets, const int32_t* __restrict__ idx,
                                             const float* __restrict__ grad_image, int64_t n_hkl, double* __restrict__ sums,
                                             float* __restrict__ partials, const int t, float4* qn, float2* qd, int* bq,
                                             int* qk = nullptr) {
  const int wv = WAVES > 1 ? (int)(threadIdx.x >> 6) : 0;
  adjoint_range<LS, PRE>(q, refl, nodes, pix, tile, idx, grad_image, n_hkl, sums, partials, t, offsets[t] + 64 * wv,
                    offsets[t + 1], 64 * WAVES, qn + 128 * wv, qd + 128 * wv, bq + 64 * wv,
                    qk ? qk + 128 * wv : nullptr);
}

}  // namespace fdtbx
