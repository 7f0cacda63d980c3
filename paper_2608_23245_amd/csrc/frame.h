// Binary64 geometry shared by the bit-reproducible kernels (exact.hip, splat.hip): the
// cell frame (Eq. recip_basis), reciprocal vectors, the extinction exponent, each
// reflection's tangent frame (Eq. gnomonic) and the culling contract's support bounds.
// Every translation unit that includes it is compiled with -ffp-contract=off, so these
// expressions round identically everywhere they are used.
#pragma once

#include <hip/hip_runtime.h>

#include <math.h>

#include "internal.h"

namespace fdtbx {

// ---------------------------------------------------------------- frame (Eq. recip_basis)
// c = (0,0,c); b = (0, b sin(alpha), b cos(alpha)); a_z = a cos(beta),
// a_y = a (cos(gamma) - cos(alpha) cos(beta))/sin(alpha), a_x = sqrt(a^2 - a_y^2 - a_z^2);
// V = a.(b x c); a* = (b x c)/V, b* = (c x a)/V, c* = (a x b)/V.
__host__ __device__ static inline void cross3(const double* u, const double* v, double* w) {
  w[0] = u[1] * v[2] - u[2] * v[1];
  w[1] = u[2] * v[0] - u[0] * v[2];
  w[2] = u[0] * v[1] - u[1] * v[0];
}


__host__ __device__ static void make_frame(const fdtbx_cell c, Frame* f) {
  double ca = cos(c.alpha), cb = cos(c.beta), cg = cos(c.gamma), sa = sin(c.alpha);
  double cv[3] = {0.0, 0.0, c.c};
  double bv[3] = {0.0, c.b * sa, c.b * ca};
  double az = c.a * cb;
  double ay = c.a * (cg - ca * cb) / sa;
  double ax = sqrt(c.a * c.a - ay * ay - az * az);
  double av[3] = {ax, ay, az};
  double bxc[3], cxa[3], axb[3];
  cross3(bv, cv, bxc);
  cross3(cv, av, cxa);
  cross3(av, bv, axb);
  double V = (av[0] * bxc[0] + av[1] * bxc[1]) + av[2] * bxc[2];
  for (int j = 0; j < 3; ++j) {
    f->a[0 * 3 + j] = av[j];
    f->a[1 * 3 + j] = bv[j];
    f->a[2 * 3 + j] = cv[j];
    f->s[0 * 3 + j] = bxc[j] / V;
    f->s[1 * 3 + j] = cxa[j] / V;
    f->s[2 * 3 + j] = axb[j] / V;
  }
  f->V = V;
}

// D = h a* + k b* + l c*, componentwise (h a*_j + k b*_j) + l c*_j.
__device__ static inline void recip(const Frame& f, double h, double k, double l, double* D) {
  for (int j = 0; j < 3; ++j) D[j] = (h * f.s[0 * 3 + j] + k * f.s[1 * 3 + j]) + l * f.s[2 * 3 + j];
}

static const double kPi2 = M_PI * M_PI;

// 2 pi^2 ((g_a^2 h^2 + g_b^2 k^2) + g_c^2 l^2): exponent of prod_i A_i (Eq. Ah).
__device__ static inline double extinction_arg(double ga, double gb, double gc, double h, double k, double l) {
  double t = (ga * ga) * (h * h) + (gb * gb) * (k * k);
  t = t + (gc * gc) * (l * l);
  return (2.0 * kPi2) * t;
}

__device__ static inline double dotv(const double* u, const double* v) { return (u[0] * v[0] + u[1] * v[1]) + u[2] * v[2]; }

struct ReflFrame {
  double D[3], r0, S[3], e1[3], e2[3], ep[3];
  bool merid;
};

// Frame of one reflection (Eq. gnomonic's tangent vectors): S = D/r0, e1 = z x S/|z x S|,
// e2 = S x e1, e_perp = radial unit vector of D about z; on the meridian e1 = x x S/|x x S|
// and e_perp = sign(D_z) y.
__device__ static void refl_frame(const Frame& f, const double* hh, ReflFrame* F) {
  double* D = F->D;
  recip(f, hh[0], hh[1], hh[2], D);
  double q = (D[0] * D[0] + D[1] * D[1]) + D[2] * D[2];
  double r0 = sqrt(q);
  F->r0 = r0;
  double* S = F->S;
  S[0] = D[0] / r0;
  S[1] = D[1] / r0;
  S[2] = D[2] / r0;
  double RD = sqrt(D[0] * D[0] + D[1] * D[1]);
  double* e1 = F->e1;
  double* ep = F->ep;
  F->merid = !(RD > 1e-12);
  if (!F->merid) {
    e1[0] = -D[1] / RD;
    e1[1] = D[0] / RD;
    e1[2] = 0.0;
    ep[0] = D[0] / RD;
    ep[1] = D[1] / RD;
    ep[2] = 0.0;
  } else {
    double nrm = sqrt(D[1] * D[1] + D[2] * D[2]);
    e1[0] = 0.0;
    e1[1] = -D[2] / nrm;
    e1[2] = D[1] / nrm;
    ep[0] = 0.0;
    ep[1] = D[2] > 0 ? 1.0 : (D[2] < 0 ? -1.0 : 0.0);
    ep[2] = 0.0;
  }
  double* e2 = F->e2;
  e2[0] = S[1] * e1[2] - S[2] * e1[1];
  e2[1] = S[2] * e1[0] - S[0] * e1[2];
  e2[2] = S[0] * e1[1] - S[1] * e1[0];
}

// Upper bound of the support half-width in u per axis, without transcendentals: m/N_eff,i
// <= m (1/N_base,i + min(pi^2 g_i^2 h_i^2, 1)) (tanh t <= min(t, 1)), or 1/2 for the Hosemann
// lineshape (one lattice period).
__device__ static inline void support_bounds(int32_t lineshape, double m, const double* Nb, const double* g,
                                             const double* hh, double* w) {
  for (int i = 0; i < 3; ++i) {
    double t = (kPi2 * (g[i] * g[i])) * (hh[i] * hh[i]);
    w[i] = lineshape == FDTBX_LINESHAPE_HOSEMANN ? 0.5 : m * (1.0 / Nb[i] + fmin(t, 1.0));
  }
}

}  // namespace fdtbx
