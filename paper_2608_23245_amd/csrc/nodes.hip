// Node table of the shell quadrature (Eqs. gnomonic, node_weight) with the unit-peak
// angular shapes of the section "Angular peak shapes".  Binary64 on the device,
// stored as float32.  The Voigt shape and its width derivatives go through the
// Faddeeva function w(z) = exp(-z^2) erfc(-i z), evaluated with Weideman's rational
// series (J. A. C. Weideman, SIAM J. Numer. Anal. 31 (1994) 1497-1518):
//   w(z) = 2 p(Z)/(L - i z)^2 + (1/sqrt(pi))/(L - i z),   Z = (L + i z)/(L - i z),
//   p(Z) = sum_{n=0}^{N-1} a_{n+1} Z^n,  L = sqrt(N/sqrt(2)),
// where a_n are the Fourier coefficients of f(theta) = exp(-t^2)(L^2 + t^2),
// t = L tan(theta/2), obtained with the trapezoid rule on 4N points.  Its derivative is
// taken from the same rational form, with D = L - i z and dZ/dz = 2 i L/D^2:
//   w'(z) = 4 i L p'(Z)/D^4 + 4 i p(Z)/D^3 + (i/sqrt(pi))/D^2.
// (The identity w' = -2 z w + 2 i/sqrt(pi) cancels two terms of size 1 down to the
// 1/z^2 of w' itself and loses about 2 log10|z| digits, a few per cent at |z| = 1e7.)
#include <hip/hip_runtime.h>

#include <math.h>

#include "internal.h"

namespace fdtbx {

static constexpr int kWN = 40;  // series length (relative error of w and w' below 1e-13 on Im z >= 0)

struct cplx {
  double re, im;
};
__device__ static inline cplx cmul(cplx a, cplx b) { return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; }
__device__ static inline cplx cdiv(cplx a, cplx b) {
  double d = b.re * b.re + b.im * b.im;
  return {(a.re * b.re + a.im * b.im) / d, (a.im * b.re - a.re * b.im) / d};
}

// a_{n}, n = 1..kWN, into coef[0..kWN-1]; called by threads 0..kWN-1 of a block.
__device__ static double weideman_coef(int n, double L) {
  const int M = 2 * kWN, M2 = 2 * M;
  double sum = 0.0;
  for (int k = -M + 1; k <= M - 1; ++k) {
    double th = k * M_PI / M;
    double t = L * tan(0.5 * th);
    double f = exp(-t * t) * (L * L + t * t);
    sum += f * cos(n * th);
  }
  return sum / M2;  // the theta = -pi sample has f = 0
}

// w(z) and w'(z) (Im z >= 0).
__device__ static void faddeeva(cplx z, const double* coef, double L, cplx* w, cplx* wp) {
  cplx iz = {-z.im, z.re};
  cplx den = {L - iz.re, -iz.im};          // D = L - i z
  cplx num = {L + iz.re, iz.im};           // L + i z
  cplx Z = cdiv(num, den);
  cplx p = {coef[kWN - 1], 0.0}, dp = {0.0, 0.0};
  for (int n = kWN - 2; n >= 0; --n) {
    dp = cmul(dp, Z);
    dp.re += p.re;
    dp.im += p.im;
    p = cmul(p, Z);
    p.re += coef[n];
  }
  const double c = 1.0 / sqrt(M_PI);
  cplx inv = cdiv({1.0, 0.0}, den);        // 1/D
  cplx inv2 = cmul(inv, inv), inv3 = cmul(inv2, inv), inv4 = cmul(inv2, inv2);
  cplx a = cmul({2.0 * p.re, 2.0 * p.im}, inv2);
  *w = {a.re + c * inv.re, a.im + c * inv.im};
  // i * (4 L p' D^-4 + 4 p D^-3 + c D^-2)
  cplx t1 = cmul({4.0 * L * dp.re, 4.0 * L * dp.im}, inv4);
  cplx t2 = cmul({4.0 * p.re, 4.0 * p.im}, inv3);
  cplx sum = {t1.re + t2.re + c * inv2.re, t1.im + t2.im + c * inv2.im};
  *wp = {-sum.im, sum.re};
}

// E(z) = d(z w(z))/dz = w(z) + z w'(z) (Im z >= 0).  For |z| < 10 from the rational form
// (the two terms cancel to the |z|^-2 of their size there, two digits at most); for |z| >= 10
// from the asymptotic series of z w(z) = (i/sqrt(pi)) sum_n a_n z^-2n, a_n = (2n-1)!!/2^n:
//   E(z) = -(i/sqrt(pi)) sum_{n>=1} 2 n a_n z^-(2n+1),
// summed until a term falls below 1e-18 of the sum (the terms shrink by about (2n+1)/(2|z|^2)).
__device__ static cplx faddeeva_E(cplx z, cplx w, cplx wp) {
  const double r2 = z.re * z.re + z.im * z.im;
  if (r2 < 100.0) {
    const cplx zw = cmul(z, wp);
    return {w.re + zw.re, w.im + zw.im};
  }
  const cplx zi = {z.re / r2, -z.im / r2};   // 1/z
  const cplx zi2 = cmul(zi, zi);
  cplx pw = cmul(zi2, zi);                   // z^-3
  cplx sum = pw;                             // n = 1: 2 * 1 * a_1 = 1
  double an = 0.5;
  for (int n = 2; n < 60; ++n) {
    an *= 0.5 * (2 * n - 1);
    pw = cmul(pw, zi2);
    const double c = 2.0 * n * an;
    const cplx t = {c * pw.re, c * pw.im};
    sum.re += t.re;
    sum.im += t.im;
    if (t.re * t.re + t.im * t.im < 1e-36 * (sum.re * sum.re + sum.im * sum.im)) break;
  }
  const double q = 1.0 / sqrt(M_PI);
  return {q * sum.im, -q * sum.re};          // -(i q) sum
}

struct NodeParams {
  int32_t n;
  double T, h, sigma_r, sig, gam;
};

// g and its derivatives with respect to sigma_theta and gamma_theta at angle D.
// gamma = 0: Gaussian value; the gamma derivative is the one-sided derivative of the
// Voigt at gamma = 0+.  sigma = 0: Lorentzian; its sigma derivative vanishes.
// Voigt, with u = Re w(z), v = Re w(z0), z = (D + i gamma) k, z0 = i gamma k, k = 1/(sigma sqrt 2):
// dz/dsigma = -z/sigma, so du/dsigma = -Re(z w'(z))/sigma = (u - Re E(z))/sigma and likewise for
// v; the quotient rule's u v terms cancel exactly, leaving
//   dg/dsigma = -(v Re E(z) - u Re E(z0))/(sigma v^2),
// which keeps its accuracy near the Lorentzian limit, where the quotient rule written with
// Re(z w') cancels two terms of size sigma to a result of size sigma^3.
__device__ static void shape(double D, double s, double g, const double* coef, double L, double* val, double* ds,
                             double* dg) {
  if (s == 0.0) {
    double den = D * D + g * g;
    *val = g * g / den;
    *ds = 0.0;
    *dg = 2.0 * g * D * D / (den * den);
    return;
  }
  const double sq2 = sqrt(2.0);
  double k = 1.0 / (s * sq2);
  cplx z = {D * k, g * k};
  cplx z0 = {0.0, g * k};
  cplx w, w0, wp, wp0;
  faddeeva(z, coef, L, &w, &wp);
  faddeeva(z0, coef, L, &w0, &wp0);
  // d z/d gamma = i k
  double u = w.re, v = w0.re;
  double du_g = -wp.im * k;
  double dv_g = -wp0.im * k;
  if (g == 0.0) {
    double t = D / s;
    *val = exp(-0.5 * t * t);
    *ds = *val * t * t / s;
  } else {
    *val = u / v;
    const cplx E = faddeeva_E(z, w, wp), E0 = faddeeva_E(z0, w0, wp0);
    *ds = -(v * E.re - u * E0.re) / (s * v * v);
  }
  *dg = (du_g * v - u * dv_g) / (v * v);
}

// Position of node (i1, i2) on the unit sphere about the origin of the tangent frame:
// (c - 1, c d1, c d2), with c - 1 written without cancellation.
__device__ static void node_xyz(const NodeParams& p, int i1, int i2, double* d1o, double* d2o, double* co, float* v) {
  const double d1 = -p.T + ((double)i1 + 0.5) * p.h;
  const double d2 = -p.T + ((double)i2 + 0.5) * p.h;
  const double rho2 = d1 * d1 + d2 * d2;
  const double sq = sqrt(1.0 + rho2);
  const double c = 1.0 / sq;
  v[0] = (float)(-rho2 / (sq * (1.0 + sq)));
  v[1] = (float)(c * d1);
  v[2] = (float)(c * d2);
  *d1o = d1;
  *d2o = d2;
  *co = c;
}

// Block record b (layout in fdtbx.h): centre and rounded-up half-width of the float32
// node coordinates of the block.
__device__ static void block_record(const NodeParams& p, int b, float* o) {
  const int nb = (p.n + FDTBX_NODE_BLOCK - 1) / FDTBX_NODE_BLOCK;
  const int b1 = b % nb, b2 = b / nb;
  double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
  for (int s2 = 0; s2 < FDTBX_NODE_BLOCK; ++s2)
    for (int s1 = 0; s1 < FDTBX_NODE_BLOCK; ++s1) {
      const int i1 = b1 * FDTBX_NODE_BLOCK + s1, i2 = b2 * FDTBX_NODE_BLOCK + s2;
      if (i1 >= p.n || i2 >= p.n) continue;
      double d1, d2, c;
      float v[3];
      node_xyz(p, i1, i2, &d1, &d2, &c, v);
      for (int j = 0; j < 3; ++j) {
        lo[j] = fmin(lo[j], (double)v[j]);
        hi[j] = fmax(hi[j], (double)v[j]);
      }
    }
  double mag = 0.0;
  for (int j = 0; j < 3; ++j) {
    const float cf = (float)(0.5 * (lo[j] + hi[j]));
    const double r = fmax(hi[j] - (double)cf, (double)cf - lo[j]);  // exact: differences of nearby floats
    float rf = (float)r;
    if ((double)rf < r) rf = nextafterf(rf, INFINITY);
    o[j] = cf;
    o[4 + j] = rf;
    mag = fmax(mag, fabs((double)cf) + (double)rf);
  }
  o[3] = (float)mag * 1.0000002f;
  o[7] = 0.0f;
}

__device__ static void node_record(const NodeParams& p, int k, const double* coef, double L, float* o) {
  int i1 = k % p.n, i2 = k / p.n;
  double d1, d2, c;
  float v[3];
  node_xyz(p, i1, i2, &d1, &d2, &c, v);
  double rho2 = d1 * d1 + d2 * d2;
  double Delta = atan(sqrt(rho2));
  double g, gs, gg;
  shape(Delta, p.sig, p.gam, coef, L, &g, &gs, &gg);
  double base = p.sigma_r * sqrt(2.0 * M_PI) * c * c * c * p.h * p.h;
  o[0] = v[0];
  o[1] = v[1];
  o[2] = v[2];
  o[3] = (float)(base * g);
  o[4] = (float)(base * gs);
  o[5] = (float)(base * gg);
  o[6] = (float)d1;
  o[7] = (float)d2;
}

__global__ void __launch_bounds__(256) k_nodes(NodeParams p, float* __restrict__ out) {
  __shared__ double coef[kWN];
  const double L = sqrt(kWN / sqrt(2.0));
  if (threadIdx.x < kWN && p.sig != 0.0) coef[threadIdx.x] = weideman_coef(threadIdx.x + 1, L);
  __syncthreads();
  int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < p.n * p.n)
    node_record(p, k, coef, L, out + (int64_t)FDTBX_NODE_FLOATS * k);
  else if (k < node_rows(p.n))
    block_record(p, k - p.n * p.n, out + (int64_t)FDTBX_NODE_FLOATS * k);
}

// Batched models: block b of node_blocks covers nodes [first, first + 256) of one model.
__global__ void __launch_bounds__(256) k_b_nodes(const fdtbx_batch_entry* __restrict__ ent, const int64_t* __restrict__ blocks,
                                                 float* __restrict__ out) {
  __shared__ double coef[kWN];
  const int64_t item = blocks[blockIdx.x];
  const int m = (int)(item >> 40);
  const int k = (int)(item & ((1ll << 40) - 1)) + threadIdx.x;
  const fdtbx_batch_entry& e = ent[m];
  NodeParams p;
  p.n = e.model.quad.n_nodes;
  p.T = e.model.quad.T;
  p.h = 2.0 * p.T / p.n;
  p.sigma_r = e.model.quad.sigma_r;
  p.sig = e.model.dis.sigma_theta;
  p.gam = e.model.dis.gamma_theta;
  const double L = sqrt(kWN / sqrt(2.0));
  if (threadIdx.x < kWN && p.sig != 0.0) coef[threadIdx.x] = weideman_coef(threadIdx.x + 1, L);
  __syncthreads();
  float* o = out + (int64_t)FDTBX_NODE_FLOATS * (e.node_off + k);
  if (k < p.n * p.n)
    node_record(p, k, coef, L, o);
  else if (k < node_rows(p.n))
    block_record(p, k - p.n * p.n, o);
}

int launch_batch_nodes(const fdtbx_batch_entry* ent, const int64_t* blocks, int64_t n_nb, float* nodes, hipStream_t s) {
  if (n_nb <= 0) return FDTBX_OK;
  hipLaunchKernelGGL(k_b_nodes, dim3((unsigned)n_nb), dim3(256), 0, s, ent, blocks, nodes);
  FDTBX_LAUNCH_CHECK("batch nodes");
  return FDTBX_OK;
}

}  // namespace fdtbx

using namespace fdtbx;

extern "C" int64_t fdtbx_node_rows(int32_t n_nodes) {
  if (n_nodes < 1 || n_nodes > 256) return 0;
  return node_rows(n_nodes);
}

extern "C" int fdtbx_node_table(const fdtbx_disorder* dis, const fdtbx_quadrature* quad, float* nodes, void* stream) {
  if (!dis || !quad || !nodes) return fail(FDTBX_ERR_INVALID_ARGUMENT, "null pointer");
  if (!(quad->n_nodes >= 1 && quad->n_nodes <= 256)) return fail(FDTBX_ERR_INVALID_ARGUMENT, "n_nodes must be in 1..256");
  if (!(quad->T > 0 && quad->T < 10)) return fail(FDTBX_ERR_INVALID_ARGUMENT, "T must be in (0, 10)");
  if (!(quad->sigma_r > 0) || !isfinite(quad->sigma_r)) return fail(FDTBX_ERR_INVALID_ARGUMENT, "sigma_r must be positive");
  if (!(dis->sigma_theta >= 0) || !(dis->gamma_theta >= 0) || !isfinite(dis->sigma_theta) || !isfinite(dis->gamma_theta))
    return fail(FDTBX_ERR_INVALID_ARGUMENT, "angular widths must be finite and non-negative");
  if (dis->sigma_theta == 0.0 && dis->gamma_theta == 0.0)
    return fail(FDTBX_ERR_INVALID_ARGUMENT, "sigma_theta and gamma_theta are both zero");
  NodeParams p;
  p.n = quad->n_nodes;
  p.T = quad->T;
  p.h = 2.0 * quad->T / quad->n_nodes;
  p.sigma_r = quad->sigma_r;
  p.sig = dis->sigma_theta;
  p.gam = dis->gamma_theta;
  const int64_t rows = node_rows(p.n);
  hipLaunchKernelGGL(k_nodes, dim3((unsigned)ceil_div(rows, 256)), dim3(256), 0, (hipStream_t)stream, p, nodes);
  FDTBX_LAUNCH_CHECK("node table");
  return FDTBX_OK;
}
