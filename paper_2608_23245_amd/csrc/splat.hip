// Deterministic forward splat: every reflection is sampled on its shell in (r, d1, d2)
// coordinates and each sample is projected onto the detector (section "Numerical
// evaluation: per-reflection shell quadrature"; section "Lorentz correction on a sampled
// reciprocal lattice"; section "Analytical Solution of the Ewald Diffraction Condition").
//
// For reflection h (radius r0, tangent frame S0, e1, e2) the samples are
//   r_a = r0 - dr + (a + 1/2)(2 dr/n_r),  d_b = -Ts + (b + 1/2)(2 Ts/n_s),
//   S   = (r c)((S0 + d1 e1) + d2 e2),  c = 1/sqrt((1 + d1^2) + d2^2)       (Eq. gnomonic)
// with dr the corner radius of the support box (culling bounds of the support half-widths)
// and Ts = min(T + 2 dr/r0, 10).  Each sample carries
//   w = W I(S) L(R_S) dV,  I(S) = r0^2 sum_k omega_k Z(S - s_k)  (Eq. direct_sum),
//   L = delta/(R_S + delta) (Eq. lorentz),  dV = r^2 (2 dr/n_r) c^3 (2 Ts/n_s)^2,
// and is deposited at both rotations about the fibre axis that satisfy the diffraction
// condition (Eqs. harmonic, solutions).  Those are written algebraically: with n the
// (tilted) fibre axis and k_in = x/lambda, the rotated S has S_x = -lambda |S|^2/2,
// S.n = Z_S, S_y = +-sqrt(|S|^2 - S_x^2 - S_z^2); k_out = k_in + S meets the detector at
// y = SF k_y/k_x, z = SF k_z/k_x (a detector tilted by d: y = SF k_y cos d/D, z = SF k_z/D with
// D = k_x cos d + k_z sin d).
//
// Mapping: one 64-lane wave per (reflection, radial sample) walks the n_s x n_s tangent
// samples in 8x8 patches, one sample per lane.  Per patch the wave bounds the node window
// from the samples' own coordinates, queues the nodes whose offsets can reach some
// sample (the same block test, queue and walk as the profile kernel), evaluates I(S) per
// lane and deposits with float atomics.  Sample positions and the projection are binary64
// without fused multiply-adds (this file is compiled with -ffp-contract=off), so the pixel
// each sample lands in is reproducible bit for bit.
#include <hip/hip_runtime.h>

#include <math.h>

#include "frame.h"
#include "internal.h"
#include "profile_common.h"
#include "profile_tile.h"

namespace fdtbx {

struct SplatParams {
  ProfParams q;
  Frame f;
  double Nb[3], g[3], m, T;
  double lam, SF, pixel, cx, cy, st, ct, delta;
  double sd, cd;  // sine and cosine of the detector tilt
  int32_t W, H, n_r, n_s, tiles_s, lineshape;
};

// Both diffraction-condition pixels of fibre-frame point S (index j W + i, or -1).
__device__ static inline void splat_pixels(const SplatParams& p, const double* S, int64_t* out) {
  out[0] = out[1] = -1;
  const double q = (S[0] * S[0] + S[1] * S[1]) + S[2] * S[2];
  const double sx = -(p.lam * q) / 2.0;
  const double sz = (S[2] - sx * p.st) / p.ct;
  const double sy2 = (q - sx * sx) - sz * sz;
  if (!(sy2 >= 0.0)) return;
  const double sy = sqrt(sy2);
  const double kx = 1.0 / p.lam + sx;
  // k_out meets the detector plane (normal (cos d, 0, sin d) through (SF, 0, 0)) where
  // t k_out . n = SF cos d; its detector coordinates are y = SF k_y cos d / D, z = SF k_z / D
  const double D = kx * p.cd + sz * p.sd;
  if (!(D > 0.0)) return;
  for (int b = 0; b < 2; ++b) {
    const double ky = b == 0 ? sy : -sy;
    const double y = p.SF * ky * p.cd / D, z = p.SF * sz / D;
    const double fi = floor(y / p.pixel + p.cx), fj = floor(z / p.pixel + p.cy);
    if (fi >= 0.0 && fi < (double)p.W && fj >= 0.0 && fj < (double)p.H) out[b] = (int64_t)fj * p.W + (int64_t)fi;
  }
}


// walk_queue for the Hosemann lineshape with its support edge decided in binary64, in the two
// passes of the pattern walks (profile_tile.h): the walk adds the nodes with max|y_i| <= lo and
// marks the queue entries where some lane's sample falls in the band (lo, hi); the second pass
// decides those from the sample's binary64 lattice offsets al64, node index qk[jj].
__device__ __forceinline__ void walk_queue_edge_al(const ProfParams& q, const float4* qn, const int* qk, int cnt,
                                                   const float* al, float lo, float hi, const HoseK& hk,
                                                   const float* rec, const double* al64, float& accr) {
  const float4* const q0 = qn;
  qn += threadIdx.y;
  float4 nxt = qn[0];
  float part = 0.0f;
  unsigned long long um = 0;
  for (int jj = 0; jj < cnt; ++jj) {
    const float4 cur = nxt;
    nxt = qn[jj + 1];
    eval_node_hose_main(cur, al, lo, hi, hk, part, jj, um);
  }
  accr += part;
  float fix = 0.0f;
  while (um) {  // uniform
    const int jj = (int)__builtin_ctzll(um);
    um &= um - 1;
    const float4 nd = q0[jj];
    const float ya = al[0] - nd.x, yb = al[1] - nd.y, yc = al[2] - nd.z;
    const float mx = fmaxf(fmaxf(fabsf(ya), fabsf(yb)), fabsf(yc));
    if (hose_band(mx, lo, hi) && hose_inside64_al(q, rec, qk[jj], al64)) fix = fmaf(nd.w, hose_prod(ya, yb, yc, hk), fix);
  }
  accr += fix;
}

template <bool COUNT, int LS>
__global__ void __launch_bounds__(64) k_splat(SplatParams p, const int32_t* __restrict__ hkl, const float* __restrict__ refl,
                                              const float* __restrict__ nodes, float* __restrict__ image,
                                              unsigned long long* __restrict__ counts) {
  // the Hosemann support edge is decided in binary64 (walk_queue_edge_al): the queue then
  // carries its node indices in qk
  constexpr bool EDGE = LS == FDTBX_LINESHAPE_HOSEMANN && !COUNT;
  __shared__ float4 qn[128];
  __shared__ int bq[64];
  __shared__ int qk[EDGE ? 128 : 1];
  const int lane = threadIdx.x & 63;
  const int64_t h = (int64_t)blockIdx.x / p.n_r;
  const int a = (int)((int64_t)blockIdx.x % p.n_r);
  const ProfParams& q = p.q;
  const double hh[3] = {(double)hkl[3 * h + 0], (double)hkl[3 * h + 1], (double)hkl[3 * h + 2]};
  ReflFrame F;
  refl_frame(p.f, hh, &F);
  double wb[3];
  support_bounds(p.lineshape, p.m, p.Nb, p.g, hh, wb);
  double dr = wb[0] * sqrt(dotv(&p.f.s[0], &p.f.s[0]));
  dr = dr + wb[1] * sqrt(dotv(&p.f.s[3], &p.f.s[3]));
  dr = dr + wb[2] * sqrt(dotv(&p.f.s[6], &p.f.s[6]));
  const double Ts = fmin(p.T + 2.0 * dr / F.r0, 10.0);
  const double hr = 2.0 * dr / p.n_r, hs = 2.0 * Ts / p.n_s;
  const double r = (F.r0 - dr) + (a + 0.5) * hr;

  const float* rec = refl + (int64_t)FDTBX_REFL_FLOATS * h;
  PairRec f;
  load_pair(rec, f);
  float Bv[3], G1[3], G2[3], sc[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    Bv[i] = f.at(RS_B + i);
    G1[i] = f.at(RS_G1 + i);
    G2[i] = f.at(RS_G2 + i);
    // the record's scale of the lattice offsets (the counting pass runs one instantiation
    // for every lineshape, so this follows the model, not the template)
    sc[i] = q.lineshape == FDTBX_LINESHAPE_HOSEMANN ? 1.0f : 0.5f * rec[RS_N + i];
  }
  HoseK hk = {};
  if (LS == FDTBX_LINESHAPE_HOSEMANN && !COUNT) hose_constants(rec, hk);
  const float wk = f.at(RS_WK);
  unsigned long long cnt = 0;

  for (int t = 0; t < p.tiles_s * p.tiles_s; ++t) {
    const int b1 = (t % p.tiles_s) * 8 + (lane & 7);
    const int b2 = (t / p.tiles_s) * 8 + (lane >> 3);
    const bool in = b1 < p.n_s && b2 < p.n_s;
    const double d1 = -Ts + (b1 + 0.5) * hs, d2 = -Ts + (b2 + 0.5) * hs;
    const double c = 1.0 / sqrt((1.0 + d1 * d1) + d2 * d2);
    double S[3];
    for (int j = 0; j < 3; ++j) S[j] = (r * c) * ((F.S[j] + d1 * F.e1[j]) + d2 * F.e2[j]);
    // lattice offsets of the sample relative to D, and its coordinates along S0, e1, e2
    const double X[3] = {S[0] - F.D[0], S[1] - F.D[1], S[2] - F.D[2]};
    float al[3], lo[3], hi[3];
    // the Hosemann lattice offsets in binary64 (scale 1) and the edge band (profile_tile.h):
    // the float32 y_i rounds al64_i once and forms kappa_i as the pattern walks do
    double al64[3] = {0.0, 0.0, 0.0};
    float elo = 0.0f, ehi = 0.0f;
    if (EDGE) {
      float mag = 0.0f;
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        al64[i] = dotv(&p.f.a[3 * i], X);
        mag = fmaxf(mag, wave_max(in ? fabsf((float)al64[i]) : 0.0f) + fabsf(Bv[i]) + fabsf(G1[i]) + fabsf(G2[i]));
      }
      const float band = fmaxf(1.0e-6f, mag * 0x1p-20f);
      elo = q.half_m - band;
      ehi = q.half_m + band;
    }
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      al[i] = in ? (float)dotv(&p.f.a[3 * i], X) * sc[i] : 1.0e30f;
      lo[i] = wave_min(in ? al[i] : INFINITY) - q.half_m - q.margin;
      hi[i] = wave_max(in ? al[i] : -INFINITY) + q.half_m + q.margin;
      if (LS == FDTBX_LINESHAPE_LAUE) al[i] = tag_alpha(al[i]);
    }
    const float pS = (float)dotv(S, F.S), p1 = (float)dotv(S, F.e1), p2 = (float)dotv(S, F.e2);
    const float sl = wave_min(in ? pS : INFINITY), sh = wave_max(in ? pS : -INFINITY);
    const float l1 = wave_min(in ? p1 : INFINITY), h1 = wave_max(in ? p1 : -INFINITY);
    const float l2 = wave_min(in ? p2 : INFINITY), h2 = wave_max(in ? p2 : -INFINITY);
    Window w;
    float accr = 0.0f;
    if (node_window_ranges(q, f.at(RS_R0), sl, sh, l1, h1, l2, h2, f.at(RS_RHO), f.at(RS_RHO + 1), f.at(RS_RHO + 2),
                           &w)) {
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
            walk_queue_edge_al(q, qn, qk, 64, al, elo, ehi, hk, rec, al64, accr);
          else
            walk_queue<COUNT, LS>(qn, 64, al, q.half_m, hk, accr, cnt);
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
        walk_queue_edge_al(q, qn, qk, qlen, al, elo, ehi, hk, rec, al64, accr);
      else
        walk_queue<COUNT, LS>(qn, qlen, al, q.half_m, hk, accr, cnt);
      wave_sync();
    }
    if (!COUNT && in && accr != 0.0f) {
      int64_t px[2];
      splat_pixels(p, S, px);
      const double RS = sqrt(S[0] * S[0] + S[1] * S[1]);
      const double dV = ((r * r) * hr) * ((c * c) * c) * (hs * hs);
      const float wgt = wk * accr * (float)((p.delta / (RS + p.delta)) * dV);
      for (int k = 0; k < 2; ++k)
        if (px[k] >= 0) unsafeAtomicAdd(image + px[k], wgt);
    }
  }
  if (COUNT) {
    for (int o = 32; o >= 1; o >>= 1) cnt += __shfl_xor(cnt, o, 64);
    if (lane == 0 && cnt) atomicAdd(counts, cnt);
  }
}

__global__ void k_zero_splat(float* __restrict__ v, int64_t n, unsigned long long* __restrict__ counts) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v && k < n) v[k] = 0.0f;
  if (counts && k == 0) *counts = 0ull;
}

}  // namespace fdtbx

using namespace fdtbx;

extern "C" int fdtbx_splat(const fdtbx_model* model, const int32_t* hkl, int64_t n_hkl, const float* refl, const float* nodes,
                           int32_t n_r, int32_t n_s, float* image, int64_t* counts, void* stream) {
  if (!model || !nodes) return fail(FDTBX_ERR_INVALID_ARGUMENT, "null pointer");
  if (!counts && !image) return fail(FDTBX_ERR_INVALID_ARGUMENT, "image is NULL");
  if (n_hkl < 0) return fail(FDTBX_ERR_INVALID_ARGUMENT, "n_hkl must be non-negative");
  if (n_hkl > 0 && (!hkl || !refl)) return fail(FDTBX_ERR_INVALID_ARGUMENT, "null pointer");
  if (n_r < 1 || n_r > 1024 || n_s < 1 || n_s > 4096) return fail(FDTBX_ERR_INVALID_ARGUMENT, "n_r must be in 1..1024, n_s in 1..4096");
  if ((int64_t)n_hkl * n_r > 0x7fffffffll) return fail(FDTBX_ERR_INVALID_ARGUMENT, "n_hkl * n_r exceeds the launch grid");
  int rc = check_model(model);
  if (rc) return rc;
  SplatParams p;
  prof_params(model, &p.q);
  make_frame(model->cell, &p.f);
  for (int i = 0; i < 3; ++i) {
    p.Nb[i] = model->dis.N_base[i];
    p.g[i] = model->dis.g[i];
  }
  p.m = (double)model->quad.m;
  p.T = model->quad.T;
  p.lam = model->geom.wavelength;
  p.SF = model->geom.distance;
  p.pixel = model->geom.pixel;
  p.cx = model->geom.center_x;
  p.cy = model->geom.center_y;
  p.st = sin(model->geom.tilt);
  p.ct = cos(model->geom.tilt);
  p.sd = sin(model->geom.det_tilt);
  p.cd = cos(model->geom.det_tilt);
  p.delta = model->quad.delta;
  p.W = model->geom.width;
  p.H = model->geom.height;
  p.n_r = n_r;
  p.n_s = n_s;
  p.tiles_s = (n_s + 7) / 8;
  p.lineshape = model->dis.lineshape;
  hipStream_t s = (hipStream_t)stream;
  const int64_t npix = (int64_t)p.W * p.H;
  float* img = counts ? nullptr : image;
  hipLaunchKernelGGL(k_zero_splat, dim3((unsigned)ceil_div(npix, 256)), dim3(256), 0, s, img, npix,
                     (unsigned long long*)counts);
  FDTBX_LAUNCH_CHECK("splat zero");
  if (n_hkl == 0) return FDTBX_OK;
  const dim3 grid((unsigned)(n_hkl * n_r));
  unsigned long long* cp = (unsigned long long*)counts;
  if (counts)
    hipLaunchKernelGGL((k_splat<true, FDTBX_LINESHAPE_LAUE>), grid, dim3(64), 0, s, p, hkl, refl, nodes, image, cp);
  else if (p.lineshape == FDTBX_LINESHAPE_GAUSSIAN)
    hipLaunchKernelGGL((k_splat<false, FDTBX_LINESHAPE_GAUSSIAN>), grid, dim3(64), 0, s, p, hkl, refl, nodes, image, cp);
  else if (p.lineshape == FDTBX_LINESHAPE_HOSEMANN)
    hipLaunchKernelGGL((k_splat<false, FDTBX_LINESHAPE_HOSEMANN>), grid, dim3(64), 0, s, p, hkl, refl, nodes, image, cp);
  else
    hipLaunchKernelGGL((k_splat<false, FDTBX_LINESHAPE_LAUE>), grid, dim3(64), 0, s, p, hkl, refl, nodes, image, cp);
  FDTBX_LAUNCH_CHECK("splat");
  return FDTBX_OK;
}
