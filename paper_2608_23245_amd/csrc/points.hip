// Test-facing entry points: the per-reflection term of Eq. direct_sum at arbitrary
// reciprocal-space points, and the forward Ewald projection of reciprocal points onto the
// detector (section "Analytical Solution of the Ewald Diffraction Condition", Eqs.
// harmonic, solutions, valid).  One thread per point; the node loop of a point runs over
// the node window that the point can reach.  Compiled without floating-point contraction
// (frame.h).
#include <hip/hip_runtime.h>

#include <math.h>

#include "frame.h"
#include "internal.h"
#include "profile_common.h"
#include "profile_tile.h"

namespace fdtbx {

struct PointParams {
  ProfParams q;
  Frame f;
};

// out[k] = W_h r0^2 sum_nodes omega Z(p_k - s_node) for reflection h = ridx[k] (the term of
// reflection h in the pattern's sum at p_k, before the Lorentz factor).  The lattice
// offsets alpha_i = scale_i a_i.(p - D) are formed in binary64 from the reflection's frame.
// For the Hosemann lineshape a node within the edge band of its support (profile_tile.h) is
// decided in binary64 from those offsets (hose_inside64_al).
template <int LS>
__global__ void __launch_bounds__(256) k_profile_points(PointParams p, const int32_t* __restrict__ hkl,
                                                        const float* __restrict__ refl, const float* __restrict__ nodes,
                                                        const int32_t* __restrict__ ridx, const double* __restrict__ pts,
                                                        int64_t n, float* __restrict__ out) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const ProfParams& q = p.q;
  const int32_t r = ridx[k];
  const double hh[3] = {(double)hkl[3 * (int64_t)r + 0], (double)hkl[3 * (int64_t)r + 1], (double)hkl[3 * (int64_t)r + 2]};
  ReflFrame F;
  refl_frame(p.f, hh, &F);
  const float* rec = refl + (int64_t)FDTBX_REFL_FLOATS * r;
  const double P[3] = {pts[3 * k + 0], pts[3 * k + 1], pts[3 * k + 2]};
  const double x[3] = {P[0] - F.D[0], P[1] - F.D[1], P[2] - F.D[2]};
  float al[3], Bv[3], G1[3], G2[3];
  double al64[3];
  for (int i = 0; i < 3; ++i) {
    const double sc = LS == FDTBX_LINESHAPE_HOSEMANN ? 1.0 : 0.5 * (double)rec[RS_N + i];
    al64[i] = sc * dotv(&p.f.a[3 * i], x);
    al[i] = (float)al64[i];
    if (LS == FDTBX_LINESHAPE_LAUE) al[i] = tag_alpha(al[i]);
    Bv[i] = rec[RS_B + i];
    G1[i] = rec[RS_G1 + i];
    G2[i] = rec[RS_G2 + i];
  }
  const float pS = (float)dotv(P, F.S), p1 = (float)dotv(P, F.e1), p2 = (float)dotv(P, F.e2);
  Window w;
  if (!node_window_ranges(q, rec[RS_R0], pS, pS, p1, p1, p2, p2, rec[RS_RHO], rec[RS_RHO + 1], rec[RS_RHO + 2], &w)) {
    out[k] = 0.0f;
    return;
  }
  HoseK hk = {};
  float elo = 0.0f, ehi = 0.0f;  // the Hosemann edge band's bounds on max|y_i|
  if (LS == FDTBX_LINESHAPE_HOSEMANN) {
    hose_constants(rec, hk);
    float mag = 0.0f;
    for (int i = 0; i < 3; ++i) mag = fmaxf(mag, fabsf(al[i]) + fabsf(Bv[i]) + fabsf(G1[i]) + fabsf(G2[i]));
    const float band = fmaxf(1.0e-6f, mag * 0x1p-20f);
    elo = q.half_m - band;
    ehi = q.half_m + band;
  }
  float acc = 0.0f;
  unsigned long long cnt = 0;
  for (int i2 = w.i2lo; i2 <= w.i2hi; ++i2) {
    for (int i1 = w.i1lo; i1 <= w.i1hi; ++i1) {
      const float4 nd = *(const float4*)(nodes + (int64_t)FDTBX_NODE_FLOATS * (i2 * q.n + i1));
      float4 e;
      e.x = fmaf(nd.x, Bv[0], fmaf(nd.y, G1[0], nd.z * G2[0]));
      e.y = fmaf(nd.x, Bv[1], fmaf(nd.y, G1[1], nd.z * G2[1]));
      e.z = fmaf(nd.x, Bv[2], fmaf(nd.y, G1[2], nd.z * G2[2]));
      e.w = nd.w;
      if (LS == FDTBX_LINESHAPE_LAUE) e = tag_kappa4(e);
      if (LS == FDTBX_LINESHAPE_HOSEMANN) {
        const float ya = al[0] - e.x, yb = al[1] - e.y, yc = al[2] - e.z;
        const float mx = fmaxf(fmaxf(fabsf(ya), fabsf(yb)), fabsf(yc));
        if (mx <= elo || (hose_band(mx, elo, ehi) && hose_inside64_al(q, rec, i2 * q.n + i1, al64)))
          acc = fmaf(e.w, hose_prod(ya, yb, yc, hk), acc);
      } else {
        eval_node<false, LS>(e, al[0], al[1], al[2], q.half_m, hk, acc, cnt);
      }
    }
  }
  out[k] = rec[RS_WK] * acc;
}

struct EwaldParams {
  double lam, SF, pixel, cx, cy, st, ct;
  double sd, cd;  // sine and cosine of the detector tilt
};

// Both diffraction-condition positions of fibre-frame point S on the detector, as
// fractional pixel coordinates (column, row; pixel (i, j) spans [i, i + 1) x [j, j + 1)):
// the rotated S has S_x = -lambda |S|^2/2 (on the Ewald sphere), S.n = Z_S (n the tilted
// fibre axis) and S_y = +-sqrt(|S|^2 - S_x^2 - S_z^2); k_out = x/lambda + S meets the
// detector plane at y = SF k_y cos d/D, z = SF k_z/D with D = k_x cos d + k_z sin d (d the
// detector tilt; y = SF k_y/k_x, z = SF k_z/k_x for a detector normal to the beam).  The
// first pair is the +S_y rotation.  NaN where no rotation satisfies the condition (Eq. valid)
// or k_out runs away from the detector plane (D <= 0).
__global__ void __launch_bounds__(256) k_ewald_project(EwaldParams p, const double* __restrict__ S, int64_t n,
                                                       double* __restrict__ out) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  double* o = out + 4 * k;
  const double s0 = S[3 * k + 0], s1 = S[3 * k + 1], s2 = S[3 * k + 2];
  const double q = (s0 * s0 + s1 * s1) + s2 * s2;
  const double sx = -(p.lam * q) / 2.0;
  const double sz = (s2 - sx * p.st) / p.ct;
  const double sy2 = (q - sx * sx) - sz * sz;
  const double kx = 1.0 / p.lam + sx;
  const double D = kx * p.cd + sz * p.sd;
  if (!(sy2 >= 0.0) || !(D > 0.0)) {
    o[0] = o[1] = o[2] = o[3] = __longlong_as_double(0x7ff8000000000000ll);
    return;
  }
  const double sy = sqrt(sy2);
  for (int b = 0; b < 2; ++b) {
    const double ky = b == 0 ? sy : -sy;
    const double y = p.SF * ky * p.cd / D, z = p.SF * sz / D;
    o[2 * b + 0] = y / p.pixel + p.cx;
    o[2 * b + 1] = z / p.pixel + p.cy;
  }
}

}  // namespace fdtbx

using namespace fdtbx;

extern "C" int fdtbx_profile_points(const fdtbx_model* model, const int32_t* hkl, const float* refl, const float* nodes,
                                    const int32_t* ridx, const double* points, int64_t n, float* out, void* stream) {
  if (!model) return fail(FDTBX_ERR_INVALID_ARGUMENT, "null pointer");
  if (n < 0) return fail(FDTBX_ERR_INVALID_ARGUMENT, "n must be non-negative");
  int rc = check_model(model);
  if (rc) return rc;
  if (n == 0) return FDTBX_OK;
  if (!hkl || !refl || !nodes || !ridx || !points || !out) return fail(FDTBX_ERR_INVALID_ARGUMENT, "null pointer");
  PointParams p;
  prof_params(model, &p.q);
  make_frame(model->cell, &p.f);
  hipStream_t s = (hipStream_t)stream;
  const dim3 grid((unsigned)ceil_div(n, 256));
  if (p.q.lineshape == FDTBX_LINESHAPE_GAUSSIAN)
    hipLaunchKernelGGL(k_profile_points<FDTBX_LINESHAPE_GAUSSIAN>, grid, dim3(256), 0, s, p, hkl, refl, nodes, ridx, points, n,
                       out);
  else if (p.q.lineshape == FDTBX_LINESHAPE_HOSEMANN)
    hipLaunchKernelGGL(k_profile_points<FDTBX_LINESHAPE_HOSEMANN>, grid, dim3(256), 0, s, p, hkl, refl, nodes, ridx, points, n,
                       out);
  else
    hipLaunchKernelGGL(k_profile_points<FDTBX_LINESHAPE_LAUE>, grid, dim3(256), 0, s, p, hkl, refl, nodes, ridx, points, n,
                       out);
  FDTBX_LAUNCH_CHECK("profile at points");
  return FDTBX_OK;
}

extern "C" int fdtbx_ewald_project(const fdtbx_geometry* geom, const double* S, int64_t n, double* out, void* stream) {
  if (!geom) return fail(FDTBX_ERR_INVALID_ARGUMENT, "null pointer");
  if (n < 0) return fail(FDTBX_ERR_INVALID_ARGUMENT, "n must be non-negative");
  int rc = check_geometry(geom);
  if (rc) return rc;
  if (n == 0) return FDTBX_OK;
  if (!S || !out) return fail(FDTBX_ERR_INVALID_ARGUMENT, "null pointer");
  EwaldParams p;
  p.lam = geom->wavelength;
  p.SF = geom->distance;
  p.pixel = geom->pixel;
  p.cx = geom->center_x;
  p.cy = geom->center_y;
  p.st = sin(geom->tilt);
  p.ct = cos(geom->tilt);
  p.sd = sin(geom->det_tilt);
  p.cd = cos(geom->det_tilt);
  hipLaunchKernelGGL(k_ewald_project, dim3((unsigned)ceil_div(n, 256)), dim3(256), 0, (hipStream_t)stream, p, S, n, out);
  FDTBX_LAUNCH_CHECK("ewald projection");
  return FDTBX_OK;
}
