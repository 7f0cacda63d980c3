// Exact cylindrical average of the pattern (Eq. cyl-average): per pixel with ring
// coordinates (R, Z),
//   image = sum_h W_h (1/2 pi) sum_j dphi I_h(p_h(phi_j)),
//   p_h(phi) = R cos(phi) e_perp + R sin(phi) e_az + Z z,   e_az = z x e_perp,
// by the periodic trapezoid rule phi_j = j dphi, dphi = 2 pi/n, n = max(8, ceil(2 pi R/arc)),
// j = -floor(n/2) .. ceil(n/2) - 1, with I_h the shell quadrature of Eq. direct_sum.  Unlike the
// profile kernel (one query point per pixel at each reflection's own azimuth, weighted by the
// Lorentz factor of Eq. lorentz), every point of the ring is visited; no Lorentz factor enters.
//
// Mapping: one to four 64-lane waves per pixel tile (8x8 by default) over the tile's list under the cylindrical
// culling description (fdtbx_cyl_records).  Per (tile, reflection) each lane bounds the part
// of its ring that can reach the reflection's support (the ball of radius rho_B about D) and
// the wave steps a shared index j over the union of those ranges, kJB indices at a time; the
// 64 x kJB ring points of a step are treated like the splat's samples: node window from their
// coordinates, the node queue of the profile kernel, and kJB evaluations per lane and queued
// node.  cos and sin of j dphi come from a binary64 rotation recurrence per lane.
#include <hip/hip_runtime.h>

#include <math.h>

#include "internal.h"
#include "profile_common.h"
#include "profile_tile.h"

namespace fdtbx {

struct CylParams {
  ProfParams q;
  double arc;
};

// Ring indices evaluated together: they share the node window, queue and walk.
constexpr int kJB = 8;

// The queue walk of walk_queue, each entry evaluated at the lane's kJB ring points.
template <bool COUNT, int LS>
__device__ __forceinline__ void walk_ring(const float4* qn, int cnt, const float (*al)[3], float half_m,
                                          const HoseK& hk, float& accr, unsigned long long& cnt_eval) {
  qn += threadIdx.y;
  float4 nxt = qn[0];
  float part = 0.0f;
  for (int jj = 0; jj < cnt; ++jj) {
    const float4 cur = nxt;
    nxt = qn[jj + 1];
#pragma unroll
    for (int u = 0; u < kJB; ++u) eval_node<COUNT, LS>(cur, al[u][0], al[u][1], al[u][2], half_m, hk, part, cnt_eval);
  }
  accr += part;
}

// walk_ring for the Hosemann lineshape with its support edge decided in binary64, in the two
// passes of the pattern walks (profile_tile.h): the walk adds the (node, ring point) terms with
// max|y_i| <= lo and marks the queue entries where some lane's ring point falls in the band
// (lo, hi); the second pass decides those in binary64 at ring point jb + u of the lane's ring
// (angle (jb + u) dphi from the reflection's azimuth), node index qk[jj].
__device__ __forceinline__ void walk_ring_edge(const ProfParams& q, const float4* qn, const int* qk, int cnt,
                                               const float (*al)[3], float lo, float hi, const HoseK& hk,
                                               const float* rec, double R, double Z, int jb, double dphi,
                                               float& accr) {
  const float4* const q0 = qn;
  qn += threadIdx.y;
  float4 nxt = qn[0];
  float part = 0.0f;
  unsigned long long um = 0;
  for (int jj = 0; jj < cnt; ++jj) {
    const float4 cur = nxt;
    nxt = qn[jj + 1];
    unsigned long long band = 0;
#pragma unroll
    for (int u = 0; u < kJB; ++u) {
      const float ya = al[u][0] - cur.x, yb = al[u][1] - cur.y, yc = al[u][2] - cur.z;
      const float mx = fmaxf(fmaxf(fabsf(ya), fabsf(yb)), fabsf(yc));
      const bool sure = mx <= lo;
      band |= __builtin_amdgcn_ballot_w64(mx < hi) & ~__builtin_amdgcn_ballot_w64(sure);
      if (sure) part = fmaf(cur.w, hose_prod(ya, yb, yc, hk), part);
    }
    um = band ? um | (1ull << jj) : um;
  }
  accr += part;
  float fix = 0.0f;
  const double RD = *(const double*)(rec + RS_RD), dZ = Z - *(const double*)(rec + RS_ZD);
  while (um) {  // uniform
    const int jj = (int)__builtin_ctzll(um);
    um &= um - 1;
    const float4 nd = q0[jj];
    const int k = qk[jj];
#pragma unroll 1
    for (int u = 0; u < kJB; ++u) {
      const float ya = al[u][0] - nd.x, yb = al[u][1] - nd.y, yc = al[u][2] - nd.z;
      const float mx = fmaxf(fmaxf(fabsf(ya), fabsf(yb)), fabsf(yc));
      if (hose_band(mx, lo, hi)) {
        const double ph = (double)(jb + u) * dphi;
        if (hose_inside64(q, rec, k, R * cos(ph) - RD, R * sin(ph), dZ)) fix = fmaf(nd.w, hose_prod(ya, yb, yc, hk), fix);
      }
    }
  }
  accr += fix;
}

// WAVES waves share a tile: per (tile, reflection), wave w takes the blocks w, w + WAVES, ...
// of kJB ring indices (its own LDS queue), and wave 0 adds the others' pixel sums in wave
// order at the end.
template <bool COUNT, int LS, int WAVES>
__global__ void __launch_bounds__(64 * WAVES) k_cyl(CylParams p, const float* __restrict__ refl,
                                                    const float* __restrict__ nodes, const double* __restrict__ pix,
                                                    const int64_t* __restrict__ offsets, const int32_t* __restrict__ idx,
                                                    float* __restrict__ image, unsigned long long* __restrict__ counts,
                                                    const int32_t* __restrict__ order) {
  // the Hosemann support edge is decided in binary64 (walk_ring_edge): the queue then carries
  // its node indices in qk
  constexpr bool EDGE = LS == FDTBX_LINESHAPE_HOSEMANN && !COUNT;
  __shared__ float4 qn_all[128 * WAVES];
  __shared__ int bq_all[64 * WAVES];
  __shared__ float xacc[WAVES > 1 ? 64 * (WAVES - 1) : 1];
  __shared__ int qk_all[EDGE ? 128 * WAVES : 1];
  const ProfParams& q = p.q;
  const int lane = threadIdx.x & 63;
  const int wv = WAVES > 1 ? (int)(threadIdx.x >> 6) : 0;
  float4* const qn = qn_all + 128 * wv;
  int* const bq = bq_all + 64 * wv;
  int* const qk = qk_all + (EDGE ? 128 * wv : 0);
  const int t = order ? order[blockIdx.x] : tile_of_block(q, blockIdx.x);
  if (t < 0) return;  // uniform across the workgroup
  const int tx = t % q.tiles_x, ty = t / q.tiles_x;
  const int pi_ = (tx << q.tlg) + (lane & ((1 << q.tlg) - 1));
  const int pj = ty * (64 >> q.tlg) + (lane >> q.tlg);
  const bool in = pi_ < q.W && pj < q.H;
  const double R = in ? pix[2 * ((int64_t)pj * q.W + pi_) + 0] : 0.0;
  const double Z = in ? pix[2 * ((int64_t)pj * q.W + pi_) + 1] : 0.0;
  // periodic trapezoid rule over this pixel's ring
  const double nf = ceil(2.0 * M_PI * R / p.arc);
  const int n = nf < 8.0 ? 8 : (int)nf;
  const double dphi = 2.0 * M_PI / (double)n;
  const int ring_lo = -(n / 2), ring_hi = n - n / 2 - 1;
  const double cd = cos(dphi), sd = sin(dphi);
  // rotation over the blocks of the other waves
  const double cw = WAVES > 1 ? cos((double)(kJB * (WAVES - 1)) * dphi) : 1.0;
  const double sw = WAVES > 1 ? sin((double)(kJB * (WAVES - 1)) * dphi) : 0.0;
  const int64_t p0 = offsets[t], p1 = offsets[t + 1];
  float acc = 0.0f;
  unsigned long long cnt = 0;
  int32_t r_next = p0 < p1 ? idx[p0] : 0;
  for (int64_t pp = p0; pp < p1; ++pp) {
    const int32_t r = r_next;
    r_next = idx[pp + 1 < p1 ? pp + 1 : pp];
    const float* rec = refl + (int64_t)FDTBX_REFL_FLOATS * r;
    PairRec f;
    load_pair(rec, f);
    static_assert(RS_AZ == 31 && RS_TA == 34, "the load below reads slots 32..35 as e_az.e1, e_az.e2, TA_0, TA_1");
    const float4 x1 = *(const float4*)(rec + 32);
    const float az[3] = {f.at(RS_AZ), x1.x, x1.y};
    const float ta[3] = {x1.z, x1.w, rec[RS_TA + 2]};
    const double RD = f.at_f64(RS_RD), ZD = f.at_f64(RS_ZD);
    float Bv[3], G1[3], G2[3], tr[3], tz[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      Bv[a] = f.at(RS_B + a);
      G1[a] = f.at(RS_G1 + a);
      G2[a] = f.at(RS_G2 + a);
      tr[a] = f.at(RS_TR + a);
      tz[a] = f.at(RS_TZ + a);
    }
    // ring points within rho_B of D: |p(phi) - D|^2 = R^2 + R_D^2 + (Z - Z_D)^2 - 2 R R_D cos(phi)
    const float rS = f.at(RS_RHO), r1 = f.at(RS_RHO + 1), r2 = f.at(RS_RHO + 2);
    const float r0 = f.at(RS_R0);
    const double rhoB = ((double)(2.0f * r0 * sqrtf(0.5f * (1.0f - q.cmin))) + (double)sqrtf(rS * rS + r1 * r1 + r2 * r2)) *
                            1.001 + 1.0e-7;
    int jl = 1, jh = 0;  // empty
    if (in) {
      const double dz = Z - ZD;
      const double num = ((R * R + RD * RD) + dz * dz) - rhoB * rhoB;
      const double den = 2.0 * R * RD;
      if (!(den > 0.0)) {
        if (num <= 0.0) {
          jl = ring_lo;
          jh = ring_hi;
        }
      } else {
        const double cmin = num / den;
        if (cmin <= -1.0) {
          jl = ring_lo;
          jh = ring_hi;
        } else if (cmin < 1.0) {
          const int jm = (int)floor(acos(cmin) / dphi) + 1;
          jl = max(ring_lo, -jm);
          jh = min(ring_hi, jm);
        }
      }
    }
    const bool has = jl <= jh;
    const int J0 = wave_min_i32(has ? jl : 0x7fffffff), J1 = wave_max_i32(has ? jh : -0x7fffffff);
    if (J0 > J1) continue;
    HoseK hk = {};
    if (LS == FDTBX_LINESHAPE_HOSEMANN && !COUNT) hose_constants(rec, hk);
    // the edge band (profile_tile.h) for y_i = T_R,i (R cos phi - R_D) + T_A,i R sin phi +
    // T_Z,i (Z - Z_D) - kappa_i, with |R cos phi - R_D| <= R + |R_D| and |R sin phi| <= R
    float elo = 0.0f, ehi = 0.0f;
    if (EDGE) {
      const float mX = wave_max(in ? (float)(R + fabs(RD)) : 0.0f), mY = wave_max(in ? (float)R : 0.0f);
      const float mZ = wave_max(in ? (float)fabs(Z - ZD) : 0.0f);
      float mag = 0.0f;
#pragma unroll
      for (int a = 0; a < 3; ++a)
        mag = fmaxf(mag, fabsf(tr[a]) * mX + fabsf(ta[a]) * mY + fabsf(tz[a]) * mZ + fabsf(Bv[a]) + fabsf(G1[a]) +
                             fabsf(G2[a]));
      const float band = fmaxf(1.0e-6f, mag * 0x1p-20f);
      elo = q.half_m - band;
      ehi = q.half_m + band;
    }
    double cj = cos((double)(J0 + kJB * wv) * dphi), sj = sin((double)(J0 + kJB * wv) * dphi);
    const float fZ = (float)(Z - ZD), fz = (float)Z;
    float accp = 0.0f;
    // kJB consecutive ring indices share one node window, queue and walk
    for (int jb = J0 + kJB * wv; jb <= J1; jb += kJB * WAVES) {
      float al[kJB][3];
      float amin[3] = {INFINITY, INFINITY, INFINITY}, amax[3] = {-INFINITY, -INFINITY, -INFINITY};
      float pmin[3] = {INFINITY, INFINITY, INFINITY}, pmax[3] = {-INFINITY, -INFINITY, -INFINITY};
#pragma unroll
      for (int u = 0; u < kJB; ++u) {
        const int jj = jb + u;
        const bool act = has && jj >= jl && jj <= jh;
        const float fX = (float)(R * cj - RD), fY = (float)(R * sj);
        // the ring point's coordinates along S, e1, e2
        const float Rc = (float)(R * cj), Rs = (float)(R * sj);
        const float pv[3] = {fmaf(Rc, f.at(RS_CS), fmaf(Rs, az[0], fz * f.at(RS_CS + 1))),
                             fmaf(Rc, f.at(RS_C1), fmaf(Rs, az[1], fz * f.at(RS_C1 + 1))),
                             fmaf(Rc, f.at(RS_C2), fmaf(Rs, az[2], fz * f.at(RS_C2 + 1)))};
#pragma unroll
        for (int a = 0; a < 3; ++a) {
          const float v = fmaf(tr[a], fX, fmaf(ta[a], fY, tz[a] * fZ));
          al[u][a] = act ? (LS == FDTBX_LINESHAPE_LAUE ? tag_alpha(v) : v) : 1.0e30f;
          amin[a] = act ? fminf(amin[a], v) : amin[a];
          amax[a] = act ? fmaxf(amax[a], v) : amax[a];
          pmin[a] = act ? fminf(pmin[a], pv[a]) : pmin[a];
          pmax[a] = act ? fmaxf(pmax[a], pv[a]) : pmax[a];
        }
        const double cn = cj * cd - sj * sd;
        sj = sj * cd + cj * sd;
        cj = cn;
      }
      if (WAVES > 1) {
        const double cn = cj * cw - sj * sw;
        sj = sj * cw + cj * sw;
        cj = cn;
      }
      float lo[3], hi[3];
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        lo[a] = wave_min(amin[a]) - q.half_m - q.margin;
        hi[a] = wave_max(amax[a]) + q.half_m + q.margin;
      }
      const float sl = wave_min(pmin[0]), sh = wave_max(pmax[0]);
      const float l1 = wave_min(pmin[1]), h1 = wave_max(pmax[1]);
      const float l2 = wave_min(pmin[2]), h2 = wave_max(pmax[2]);
      Window w;
      if (node_window_ranges(q, r0, sl, sh, l1, h1, l2, h2, rS, r1, r2, &w)) {
        float accr = 0.0f;
        int qlen = 0;  // uniform
        scan_window(q, nodes, w, Bv, G1, G2, lo, hi, bq, [&](bool keep, int k, float4 e) {
          const unsigned long long bal = __ballot(keep);
          if (keep) {
            const int pos = qlen + (int)__builtin_amdgcn_mbcnt_hi((unsigned)(bal >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)bal, 0u));
            qn[pos] = LS == FDTBX_LINESHAPE_LAUE ? tag_kappa4(e) : e;
            if (EDGE) qk[pos] = k;
          }
          qlen += __popcll(bal);
          wave_sync();
          if (qlen >= 64) {
            if (EDGE)
              walk_ring_edge(q, qn, qk, 64, al, elo, ehi, hk, rec, R, Z, jb, dphi, accr);
            else
              walk_ring<COUNT, LS>(qn, 64, al, q.half_m, hk, accr, cnt);
            qlen -= 64;
            wave_sync();
            if (lane < qlen) {
              qn[lane] = qn[64 + lane];
              if (EDGE) qk[lane] = qk[64 + lane];
            }
            wave_sync();
          }
        });
        if (EDGE)
          walk_ring_edge(q, qn, qk, qlen, al, elo, ehi, hk, rec, R, Z, jb, dphi, accr);
        else
          walk_ring<COUNT, LS>(qn, qlen, al, q.half_m, hk, accr, cnt);
        wave_sync();
        accp += accr;
      }
    }
    acc = fmaf(f.at(RS_WK), accp, acc);
  }
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
    if (!in) return;
    write_folded(q, image, pi_, pj, tx, ty, acc * (float)(dphi / (2.0 * M_PI)));
  }
}

__global__ void k_zero_count(unsigned long long* c) {
  if (threadIdx.x == 0) *c = 0ull;
}

template <int WAVES>
static void launch_cyl(const CylParams& p, dim3 grid, hipStream_t s, const float* refl, const float* nodes,
                       const double* pix, const int64_t* offsets, const int32_t* idx, const int32_t* order, float* image,
                       unsigned long long* counts) {
  const dim3 block(64 * WAVES);
  if (counts)
    hipLaunchKernelGGL((k_cyl<true, FDTBX_LINESHAPE_LAUE, WAVES>), grid, block, 0, s, p, refl, nodes, pix, offsets, idx, image,
                       counts, order);
  else if (p.q.lineshape == FDTBX_LINESHAPE_GAUSSIAN)
    hipLaunchKernelGGL((k_cyl<false, FDTBX_LINESHAPE_GAUSSIAN, WAVES>), grid, block, 0, s, p, refl, nodes, pix, offsets, idx,
                       image, counts, order);
  else if (p.q.lineshape == FDTBX_LINESHAPE_HOSEMANN)
    hipLaunchKernelGGL((k_cyl<false, FDTBX_LINESHAPE_HOSEMANN, WAVES>), grid, block, 0, s, p, refl, nodes, pix, offsets, idx,
                       image, counts, order);
  else
    hipLaunchKernelGGL((k_cyl<false, FDTBX_LINESHAPE_LAUE, WAVES>), grid, block, 0, s, p, refl, nodes, pix, offsets, idx, image,
                       counts, order);
}

}  // namespace fdtbx

using namespace fdtbx;

extern "C" int fdtbx_profile_cyl(const fdtbx_model* model, const float* refl, const float* nodes, const double* pix,
                                 const int64_t* offsets, const int32_t* idx, const int32_t* order, double arc, float* image,
                                 int64_t* counts, void* stream) {
  if (!model || !refl || !nodes || !pix || !offsets || !idx) return fail(FDTBX_ERR_INVALID_ARGUMENT, "null pointer");
  if (!counts && !image) return fail(FDTBX_ERR_INVALID_ARGUMENT, "image is NULL");
  int rc = check_model(model);
  if (rc) return rc;
  if (!(arc >= 1.0e-5 && arc < 1.0)) return fail(FDTBX_ERR_INVALID_ARGUMENT, "arc must be in [1e-5, 1) 1/A");
  CylParams p;
  prof_params(model, &p.q);
  p.arc = arc;
  // without an order: the plain tile order (the ring work of a few reflections concentrates on
  // a few superblocks, which the spatially grouped order would pile onto few XCDs)
  p.q.sbw = 0;
  hipStream_t s = (hipStream_t)stream;
  const dim3 grid((unsigned)(order ? order_grid(p.q.lcols, p.q.lrows) : tile_grid(p.q)));
  unsigned long long* cp = (unsigned long long*)counts;
  if (counts) {
    hipLaunchKernelGGL(k_zero_count, dim3(1), dim3(64), 0, s, cp);
    FDTBX_LAUNCH_CHECK("cylindrical average counter");
  }
  int waves = 1;
  rc = tile_waves(&model->geom, (int64_t)p.q.lcols * p.q.lrows, &waves);
  if (rc) return rc;
  if (waves == 4)
    launch_cyl<4>(p, grid, s, refl, nodes, pix, offsets, idx, order, image, cp);
  else if (waves == 2)
    launch_cyl<2>(p, grid, s, refl, nodes, pix, offsets, idx, order, image, cp);
  else
    launch_cyl<1>(p, grid, s, refl, nodes, pix, offsets, idx, order, image, cp);
  FDTBX_LAUNCH_CHECK("cylindrical average");
  return FDTBX_OK;
}
