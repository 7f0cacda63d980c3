/*
 * FP64 CPU oracle, compiled part.  TEST INFRASTRUCTURE ONLY: nothing on the
 * product path links, loads or calls this file; only the tests, the smoke
 * check and the benchmark's CPU-baseline leg do.
 *
 * Plain loops, IEEE binary64, no fused multiply-add (built with
 * -ffp-contract=off).  The per-reflection inputs (frames, effective sizes,
 * weights) and the node table come from the Python half of the oracle; this
 * file holds the two loops that are too slow in Python:
 *
 *   oracle_pattern   -- the detector image at a list of pixels
 *   oracle_grad      -- the adjoint of that image for a weighted residual
 *   oracle_splat     -- the forward splat of sampled shell points onto the detector
 *   oracle_cyl       -- the exact cylindrical average at a list of pixels
 *
 * Both follow the section "Numerical evaluation: per-reflection shell
 * quadrature" (Eqs. I_shape, gnomonic, node_weight, direct_sum; Eqs. Z and
 * breadth for the Hosemann lineshape), the
 * section "Lorentz correction on a sampled reciprocal lattice" (Eq. lorentz)
 * and the section "Index-dependent paracrystalline disorder" (Eqs. Ah, Neff,
 * Ipara) of the paper.
 */
#include <math.h>
#include <stdint.h>
#include <stddef.h>
#include <stdlib.h>

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

typedef struct {
  /* per reflection, all [n_hkl] or [n_hkl][3] */
  int64_t n_hkl;
  const double* W;      /* |F|^2 * I_para */
  const double* N;      /* effective cells N_eff along a,b,c  [n][3] */
  const double* r0;     /* |D| */
  const double* S;      /* unit D                              [n][3] */
  const double* e1;     /* tangent vector 1                    [n][3] */
  const double* e2;     /* tangent vector 2                    [n][3] */
  const double* ep;     /* unit radial direction of D about z  [n][3] */
  const double* astar;  /* reciprocal basis rows a*, b*, c*    [3][3] */
  const double* avec;   /* real basis rows a, b, c             [3][3] */
  /* node table */
  int64_t n_nodes;
  const double* d1;
  const double* d2;
  const double* omega;  /* sigma_r sqrt(2 pi) g(Delta) c^3 h^2 */
  int32_t m;            /* kernel zeros kept per axis */
  double delta;         /* Lorentz regulariser */
  int32_t use_skip;     /* 1: skip reflections whose support provably misses the query point */
  int32_t lineshape;    /* per-axis peak form: 0 Laue, 1 Gaussian, 2 Hosemann */
} oracle_problem;

/* N sinc^2(N u), sinc(x) = sin(pi x)/(pi x), sinc(0) = 1 (Eq. I_shape, one axis). */
static double laue_axis(double N, double u) {
  double x = N * u;
  if (x == 0.0) return N;
  double s = sin(M_PI * x) / (M_PI * x);
  return N * s * s;
}

/* Coefficient of Hosemann's factor (Eq. Z) whose integral breadth (1 - A)/(1 + A)
 * (Eq. breadth) equals 1/N; 0 when N <= 1 (no narrower peak exists). */
static double hosemann_A(double N) { return N > 1.0 ? (N - 1.0) / (N + 1.0) : 0.0; }

/* Per-axis peak of integral breadth 1/N, unit integral per period, peak N:
 * Laue N sinc^2(N u) (Eq. I_shape), Gaussian N exp(-pi N^2 u^2), or Hosemann
 * (1 - A^2)/(1 - 2 A cos(2 pi u) + A^2) (Eq. Z). */
static double axis_profile(int lineshape, double N, double u) {
  if (lineshape == 0) return laue_axis(N, u);
  if (lineshape == 1) return N * exp(-M_PI * N * N * u * u);
  double A = hosemann_A(N);
  return (1.0 - A * A) / (1.0 - 2.0 * A * cos(2.0 * M_PI * u) + A * A);
}

/* Support half-width in u: m/N (Laue, Gaussian) or half a lattice period (Hosemann). */
static double support_half(const oracle_problem* P, double N) { return P->lineshape == 2 ? 0.5 : P->m / N; }

static double dot3(const double* a, const double* b) { return (a[0] * b[0] + a[1] * b[1]) + a[2] * b[2]; }

/* Largest |x| over the support box {x : |a_i . x| <= w_i} = {sum u_i a*_i : |u_i| <= w_i}:
 * the longest of its corner vectors. */
static double support_radius(const oracle_problem* P, int64_t h) {
  double best = 0.0;
  const double w0 = support_half(P, P->N[3 * h + 0]), w1 = support_half(P, P->N[3 * h + 1]);
  const double w2 = support_half(P, P->N[3 * h + 2]);
  for (int sa = -1; sa <= 1; sa += 2)
    for (int sb = -1; sb <= 1; sb += 2)
      for (int sc = -1; sc <= 1; sc += 2) {
        double v[3];
        for (int j = 0; j < 3; ++j)
          v[j] = sa * w0 * P->astar[0 * 3 + j] + sb * w1 * P->astar[1 * 3 + j] + sc * w2 * P->astar[2 * 3 + j];
        double r = sqrt(dot3(v, v));
        if (r > best) best = r;
      }
  return best;
}

/* Exact-zero skip: every node lies on the sphere |s| = r0 within angle theta_nodes of S.
 * A node can only be inside the support of p if |p - s| <= rho, which needs
 * | |p| - r0 | <= rho and angle(p, S) <= theta_nodes + asin(rho/|p|).  When either fails,
 * no node passes the support test and the reflection adds nothing; skipping it leaves
 * the sum bit-identical.  Margins keep the test conservative under rounding. */
static int provably_empty(const oracle_problem* P, int64_t h, const double* p, double theta_nodes) {
  double rho = support_radius(P, h) * (1.0 + 1e-6) + 1e-12;
  double pn = sqrt(dot3(p, p));
  if (fabs(pn - P->r0[h]) > rho) return 1;
  if (pn > rho) {
    double cosang = dot3(p, &P->S[3 * h]) / pn;
    if (cosang > 1.0) cosang = 1.0;
    if (cosang < -1.0) cosang = -1.0;
    double ang = acos(cosang);
    double lim = theta_nodes + asin(rho / pn) + 1e-6;
    if (ang > lim) return 1;
  }
  return 0;
}

static double nodes_max_angle(const oracle_problem* P) {
  double best = 0.0;
  for (int64_t k = 0; k < P->n_nodes; ++k) {
    double a = atan(sqrt(P->d1[k] * P->d1[k] + P->d2[k] * P->d2[k]));
    if (a > best) best = a;
  }
  return best;
}

/* Query point of pixel ring (R, Z) for reflection h: the point of the ring at the
 * reflection's own azimuth, p = R e_perp + Z z. */
static void query_point(const oracle_problem* P, int64_t h, double R, double Z, double* p) {
  p[0] = R * P->ep[3 * h + 0];
  p[1] = R * P->ep[3 * h + 1];
  p[2] = R * P->ep[3 * h + 2] + Z;
}

/* Shell-quadrature profile of reflection h at Cartesian point p (Eq. direct_sum):
 * sum over nodes k with |a_i.(p - s_k)| <= m/N_i of w_k Z(p - s_k),
 * s_k = r0 (S + d1 e1 + d2 e2)/sqrt(1 + d1^2 + d2^2)   (Eq. gnomonic),
 * w_k = r0^2 omega_k                                   (Eq. node_weight). */
static double profile_at(const oracle_problem* P, int64_t h, const double* p, int64_t* n_eval) {
  const double r0 = P->r0[h];
  const double* S = &P->S[3 * h];
  const double* e1 = &P->e1[3 * h];
  const double* e2 = &P->e2[3 * h];
  const double* N = &P->N[3 * h];
  double I = 0.0;
  int64_t cnt = 0;
  for (int64_t k = 0; k < P->n_nodes; ++k) {
    double d1 = P->d1[k], d2 = P->d2[k];
    double c = 1.0 / sqrt(1.0 + d1 * d1 + d2 * d2);
    double x[3];
    for (int j = 0; j < 3; ++j) {
      double s = r0 * c * (S[j] + d1 * e1[j] + d2 * e2[j]);
      x[j] = p[j] - s;
    }
    double u[3];
    int inside = 1;
    for (int i = 0; i < 3; ++i) {
      u[i] = dot3(&P->avec[3 * i], x);
      if (fabs(u[i]) > support_half(P, N[i])) inside = 0;
    }
    if (!inside) continue;
    double Zk = axis_profile(P->lineshape, N[0], u[0]) * axis_profile(P->lineshape, N[1], u[1]) *
                axis_profile(P->lineshape, N[2], u[2]);
    I += r0 * r0 * P->omega[k] * Zk;
    ++cnt;
  }
  if (n_eval) *n_eval += cnt;
  return I;
}

/* Detector image at n_pix pixels with ring coordinates (R[p], Z[p]):
 * P = L(R) sum_h W_h I_h(p*_h), L = delta/(R + delta) (Eq. lorentz), summed over
 * reflections in ascending order in FP64.  n_evals (optional) receives the number
 * of (pixel, reflection, node) triples that passed the support test. */
void oracle_pattern(const oracle_problem* P, int64_t n_pix, const double* R, const double* Z, double* out,
                    int64_t* n_evals) {
  double theta_nodes = nodes_max_angle(P);
  int64_t total = 0;
#pragma omp parallel for schedule(dynamic, 1) reduction(+ : total)
  for (int64_t q = 0; q < n_pix; ++q) {
    double acc = 0.0;
    int64_t cnt = 0;
    for (int64_t h = 0; h < P->n_hkl; ++h) {
      double p[3];
      query_point(P, h, R[q], Z[q], p);
      if (P->use_skip && provably_empty(P, h, p, theta_nodes)) continue;
      acc += P->W[h] * profile_at(P, h, p, &cnt);
    }
    out[q] = P->delta / (R[q] + P->delta) * acc;
    total += cnt;
  }
  if (n_evals) *n_evals = total;
}

/* Reflections whose support can reach the query point of at least one of n_pix pixels:
 * reach[h] = 1 unless provably_empty holds for every listed pixel.  Every other reflection
 * adds exactly nothing to oracle_pattern at those pixels, so the pattern over the reachable
 * reflections alone is bit-identical to the pattern over all of them. */
void oracle_reach(const oracle_problem* P, int64_t n_pix, const double* R, const double* Z, unsigned char* reach) {
  double theta_nodes = nodes_max_angle(P);
#pragma omp parallel for schedule(dynamic, 256)
  for (int64_t h = 0; h < P->n_hkl; ++h) {
    unsigned char any = 0;
    for (int64_t q = 0; q < n_pix && !any; ++q) {
      double p[3];
      query_point(P, h, R[q], Z[q], p);
      if (!provably_empty(P, h, p, theta_nodes)) any = 1;
    }
    reach[h] = any;
  }
}

/* Per-reflection profile values at each pixel, [n_pix][n_hkl] (no W, no Lorentz):
 * used by tests that check the culling lists and the per-reflection adjoint.  With use_skip,
 * the reflections the exact skip rules out hold 0 (which profile_at would return too). */
void oracle_profile_table(const oracle_problem* P, int64_t n_pix, const double* R, const double* Z, double* out) {
  double theta_nodes = nodes_max_angle(P);
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t q = 0; q < n_pix; ++q) {
    for (int64_t h = 0; h < P->n_hkl; ++h) {
      double p[3];
      query_point(P, h, R[q], Z[q], p);
      out[q * P->n_hkl + h] = (P->use_skip && provably_empty(P, h, p, theta_nodes)) ? 0.0 : profile_at(P, h, p, NULL);
    }
  }
}

/* W_h I_h(p) at arbitrary points: out[k] = W[h] profile_at(h, points[k]), h = ridx[k]
 * (the term of reflection h in Eq. direct_sum's pattern sum, before the Lorentz factor). */
void oracle_profile_points(const oracle_problem* P, int64_t n, const int32_t* ridx, const double* points, double* out) {
#pragma omp parallel for schedule(dynamic, 64)
  for (int64_t k = 0; k < n; ++k) out[k] = P->W[ridx[k]] * profile_at(P, ridx[k], &points[3 * k], NULL);
}

/* d/dN [N sinc^2(N u)] = sin(2 pi N u)/(pi u N) - sin^2(pi N u)/(pi^2 u^2 N^2); at u = 0 it is 1. */
static double laue_axis_dN(double N, double u) {
  if (u == 0.0) return 1.0;
  double s = sin(M_PI * N * u);
  return sin(2.0 * M_PI * N * u) / (M_PI * u * N) - s * s / (M_PI * M_PI * u * u * N * N);
}

/* d/dN of axis_profile at fixed u.  Gaussian: exp(-pi N^2 u^2)(1 - 2 pi N^2 u^2).
 * Hosemann: (dA/dN) [2 cos(2 pi u)(1 + A^2) - 4 A]/(1 - 2 A cos(2 pi u) + A^2)^2 with
 * dA/dN = 2/(N + 1)^2 for N > 1 and 0 below (where A is held at 0). */
static double axis_profile_dN(int lineshape, double N, double u) {
  if (lineshape == 0) return laue_axis_dN(N, u);
  if (lineshape == 1) return exp(-M_PI * N * N * u * u) * (1.0 - 2.0 * M_PI * N * N * u * u);
  if (!(N > 1.0)) return 0.0;
  double A = hosemann_A(N);
  double c = cos(2.0 * M_PI * u);
  double den = 1.0 - 2.0 * A * c + A * A;
  return 2.0 / ((N + 1.0) * (N + 1.0)) * (2.0 * c * (1.0 + A * A) - 4.0 * A) / (den * den);
}

/* Adjoint sums of the image for a pixel weight G (dL/dP at each listed pixel).  For every
 * reflection h, over the listed pixels q and the nodes k inside the support at p*_qh:
 *   out[h][0] = sum_q G_q L(R_q) r0^2 sum_k omega_k Z_k              (= dL/dW_h)
 *   out[h][1] = sum_q G_q L(R_q) r0^2 sum_k domega_k/dsigma Z_k
 *   out[h][2] = sum_q G_q L(R_q) r0^2 sum_k domega_k/dgamma Z_k
 *   out[h][3+i] = sum_q G_q L(R_q) r0^2 sum_k omega_k dZ_k/dN_i     (i = a, b, c)
 * with Z_k = prod_i f(N_i, u_i), f the per-axis profile of the lineshape.  For the Laue form
 * the support boundary moves with N_i but Z has a double zero there, so it adds nothing; the
 * Gaussian is below 1e-12 of its peak there; the Hosemann support (half a period) is fixed. */
void oracle_grad_sums(const oracle_problem* P, const double* domega_ds, const double* domega_dg, int64_t n_pix,
                      const double* R, const double* Z, const double* G, double* out) {
  double theta_nodes = nodes_max_angle(P);
#pragma omp parallel for schedule(dynamic, 4)
  for (int64_t h = 0; h < P->n_hkl; ++h) {
    const double r0 = P->r0[h];
    const double* S = &P->S[3 * h];
    const double* e1 = &P->e1[3 * h];
    const double* e2 = &P->e2[3 * h];
    const double* N = &P->N[3 * h];
    double acc[6] = {0, 0, 0, 0, 0, 0};
    for (int64_t q = 0; q < n_pix; ++q) {
      if (G[q] == 0.0) continue;
      double p[3];
      query_point(P, h, R[q], Z[q], p);
      if (P->use_skip && provably_empty(P, h, p, theta_nodes)) continue;
      double wq = G[q] * (P->delta / (R[q] + P->delta)) * r0 * r0;
      double a[6] = {0, 0, 0, 0, 0, 0};
      for (int64_t k = 0; k < P->n_nodes; ++k) {
        double d1 = P->d1[k], d2 = P->d2[k];
        double c = 1.0 / sqrt(1.0 + d1 * d1 + d2 * d2);
        double x[3];
        for (int j = 0; j < 3; ++j) x[j] = p[j] - r0 * c * (S[j] + d1 * e1[j] + d2 * e2[j]);
        double u[3];
        int inside = 1;
        for (int i = 0; i < 3; ++i) {
          u[i] = dot3(&P->avec[3 * i], x);
          if (fabs(u[i]) > support_half(P, N[i])) inside = 0;
        }
        if (!inside) continue;
        double f[3], df[3];
        for (int i = 0; i < 3; ++i) {
          f[i] = axis_profile(P->lineshape, N[i], u[i]);
          df[i] = axis_profile_dN(P->lineshape, N[i], u[i]);
        }
        double Zk = f[0] * f[1] * f[2];
        a[0] += P->omega[k] * Zk;
        a[1] += domega_ds[k] * Zk;
        a[2] += domega_dg[k] * Zk;
        a[3] += P->omega[k] * df[0] * f[1] * f[2];
        a[4] += P->omega[k] * f[0] * df[1] * f[2];
        a[5] += P->omega[k] * f[0] * f[1] * df[2];
      }
      for (int i = 0; i < 6; ++i) acc[i] += wq * a[i];
    }
    for (int i = 0; i < 6; ++i) out[6 * h + i] = acc[i];
  }
}

/* Structure factors (Eq. structure_factor with the isotropic Debye-Waller factor):
 * F = sum_j occ_j f_t(s) exp(-B_j s^2) (cos 2 pi phi + i sin 2 pi phi), phi = (h x + k y + l z) mod 1,
 * s^2 = |D|^2/4 given per reflection, f_t(s) = sum_g a_g exp(-b_g s^2) + c from ff[t][9]. */
void oracle_structure_factors(int64_t n_hkl, const int32_t* hkl, const double* s2, int64_t n_atoms, const double* x,
                              const double* y, const double* z, const double* B, const double* occ, const int32_t* type,
                              int32_t n_types, const double* ff, double* F_re, double* F_im) {
#pragma omp parallel for schedule(dynamic, 64)
  for (int64_t r = 0; r < n_hkl; ++r) {
    double f[64];
    for (int t = 0; t < n_types && t < 64; ++t) {
      f[t] = ff[9 * t + 8];
      for (int g = 0; g < 4; ++g) f[t] += ff[9 * t + g] * exp(-ff[9 * t + 4 + g] * s2[r]);
    }
    double h = hkl[3 * r], k = hkl[3 * r + 1], l = hkl[3 * r + 2];
    double re = 0.0, im = 0.0;
    for (int64_t j = 0; j < n_atoms; ++j) {
      double phi = (h * x[j] + k * y[j]) + l * z[j];
      phi = phi - floor(phi);
      double amp = occ[j] * f[type[j]] * exp(-B[j] * s2[r]);
      re += amp * cos(2.0 * M_PI * phi);
      im += amp * sin(2.0 * M_PI * phi);
    }
    F_re[r] = re;
    F_im[r] = im;
  }
}

/* Deterministic forward splat (section "Numerical evaluation: per-reflection shell quadrature":
 * each reflection is sampled on its shell in (r, d1, d2) and every sample is projected onto
 * the detector; section "Lorentz correction on a sampled reciprocal lattice"; section
 * "Analytical Solution of the Ewald Diffraction Condition").  For reflection h, samples
 *   r_a  = r0 - dr + (a + 1/2)(2 dr/n_r),            a = 0..n_r-1
 *   d_b  = -Ts + (b + 1/2)(2 Ts/n_s),                 b = 0..n_s-1 (both tangent axes)
 *   S    = (r c) ((S0 + d1 e1) + d2 e2),  c = 1/sqrt((1 + d1 d1) + d2 d2)   (Eq. gnomonic)
 *   dV   = r^2 (2 dr/n_r) c^3 (2 Ts/n_s)^2
 *   w    = W_h I_h(S) L(R_S) dV,  L = delta/(R_S + delta)  (Eqs. direct_sum, lorentz)
 * with dr and Ts per reflection (sp_dr, sp_Ts) and R_S = |S_xy|, Z_S = S_z about the fibre.
 * Both rotations about the fibre axis that bring S onto the Ewald sphere (Eqs. harmonic,
 * solutions) receive w: in the laboratory, with the fibre axis n = (sin t, 0, cos t) and
 * k_in = x/lambda, those are the points with cylindrical coordinates (R_S, Z_S) about n on
 * the sphere:  S_x = -lambda |S|^2/2,  S_z = (Z_S - S_x sin t)/cos t,
 * S_y = +-sqrt(|S|^2 - S_x^2 - S_z^2) (none if negative); k_out = (1/lambda + S_x, S_y, S_z)
 * meets the detector plane at y = SF k_y/k_x, z = SF k_z/k_x (k_x > 0), in pixel
 * (floor(y/p + c_x), floor(z/p + c_y)).  Binary64, no fused multiply-add. */
typedef struct {
  double lambda, SF, pixel, cx, cy, st, ct;
  double sd, cd; /* sine and cosine of the detector tilt */
  int32_t width, height;
  int32_t n_r, n_s;
  const double* dr;   /* [n_hkl] radial half-extent */
  const double* Ts;   /* [n_hkl] tangent-plane half-extent */
} oracle_splat_params;

/* One sample's two detector pixels (index j*W + i, or -1 when the projection misses). */
static void splat_pixels(const oracle_splat_params* sp, const double* S, int64_t* out) {
  out[0] = out[1] = -1;
  double q = (S[0] * S[0] + S[1] * S[1]) + S[2] * S[2];
  double RS2 = S[0] * S[0] + S[1] * S[1];
  double ZS = S[2];
  (void)RS2;
  double sx = -(sp->lambda * q) / 2.0;
  double sz = (ZS - sx * sp->st) / sp->ct;
  double sy2 = (q - sx * sx) - sz * sz;
  if (!(sy2 >= 0.0)) return;
  double sy = sqrt(sy2);
  double kx = 1.0 / sp->lambda + sx;
  /* the detector plane, normal (cos d, 0, sin d) through (SF, 0, 0), met by t k_out */
  double D = kx * sp->cd + sz * sp->sd;
  if (!(D > 0.0)) return;
  for (int b = 0; b < 2; ++b) {
    double ky = b == 0 ? sy : -sy;
    double y = sp->SF * ky * sp->cd / D, z = sp->SF * sz / D;
    double fi = floor(y / sp->pixel + sp->cx), fj = floor(z / sp->pixel + sp->cy);
    if (fi >= 0.0 && fi < (double)sp->width && fj >= 0.0 && fj < (double)sp->height)
      out[b] = (int64_t)fj * sp->width + (int64_t)fi;
  }
}

/* image[height*width] (zeroed by the caller) += the deposits of every sample of every
 * reflection; n_evals (optional) receives the (sample, node) pairs inside the support. */
void oracle_splat(const oracle_problem* P, const oracle_splat_params* sp, double* image, int64_t* n_evals) {
  int64_t npix = (int64_t)sp->width * sp->height;
  int64_t total = 0;
#pragma omp parallel reduction(+ : total)
  {
    double* local = (double*)calloc((size_t)npix, sizeof(double));
#pragma omp for schedule(dynamic, 1)
    for (int64_t h = 0; h < P->n_hkl; ++h) {
      const double r0 = P->r0[h];
      const double* S0 = &P->S[3 * h];
      const double* e1 = &P->e1[3 * h];
      const double* e2 = &P->e2[3 * h];
      const double dr = sp->dr[h], Ts = sp->Ts[h];
      const double hr = 2.0 * dr / sp->n_r, hs = 2.0 * Ts / sp->n_s;
      for (int a = 0; a < sp->n_r; ++a) {
        double r = (r0 - dr) + (a + 0.5) * hr;
        for (int b2 = 0; b2 < sp->n_s; ++b2) {
          double d2 = -Ts + (b2 + 0.5) * hs;
          for (int b1 = 0; b1 < sp->n_s; ++b1) {
            double d1 = -Ts + (b1 + 0.5) * hs;
            double c = 1.0 / sqrt((1.0 + d1 * d1) + d2 * d2);
            double S[3];
            for (int j = 0; j < 3; ++j) S[j] = (r * c) * ((S0[j] + d1 * e1[j]) + d2 * e2[j]);
            int64_t px[2];
            splat_pixels(sp, S, px);
            int64_t cnt = 0;
            double I = profile_at(P, h, S, &cnt);
            total += cnt;
            if (px[0] < 0 && px[1] < 0) continue;
            double RS = sqrt(S[0] * S[0] + S[1] * S[1]);
            double dV = ((r * r) * hr) * ((c * c) * c) * (hs * hs);
            double w = P->W[h] * I * (P->delta / (RS + P->delta)) * dV;
            for (int k = 0; k < 2; ++k)
              if (px[k] >= 0) local[px[k]] += w;
          }
        }
      }
    }
#pragma omp critical
    for (int64_t q = 0; q < npix; ++q) image[q] += local[q];
    free(local);
  }
  if (n_evals) *n_evals = total;
}

/* Exact cylindrical average (Eq. cyl-average) at n_pix pixels with ring coordinates (R, Z):
 *   out[q] = sum_h W_h (1/2 pi) sum_j dphi I_h(p_h(phi_j)),
 *   p_h(phi) = R cos(phi) e_perp + R sin(phi) e_az + Z z,  e_az = z x e_perp,
 * with the periodic trapezoid rule phi_j = j dphi, dphi = 2 pi/n, n = max(8, ceil(2 pi R/arc)),
 * j = -floor(n/2) .. ceil(n/2) - 1 (every point of the ring once, phi = 0 at the reflection's
 * own azimuth).  No Lorentz factor: the ring average is the rotation average itself. */
void oracle_cyl(const oracle_problem* P, int64_t n_pix, const double* R, const double* Z, double arc, double* out,
                int64_t* n_evals) {
  double theta_nodes = nodes_max_angle(P);
  int64_t total = 0;
#pragma omp parallel for schedule(dynamic, 1) reduction(+ : total)
  for (int64_t q = 0; q < n_pix; ++q) {
    double nf = ceil(2.0 * M_PI * R[q] / arc);
    int64_t n = nf < 8.0 ? 8 : (int64_t)nf;
    double dphi = 2.0 * M_PI / (double)n;
    double acc = 0.0;
    int64_t cnt = 0;
    for (int64_t j = -(n / 2); j < n - n / 2; ++j) {
      double phi = (double)j * dphi;
      double cp = cos(phi), sp = sin(phi);
      for (int64_t h = 0; h < P->n_hkl; ++h) {
        const double* ep = &P->ep[3 * h];
        double p[3] = {R[q] * cp * ep[0] - R[q] * sp * ep[1], R[q] * cp * ep[1] + R[q] * sp * ep[0], Z[q]};
        if (P->use_skip && provably_empty(P, h, p, theta_nodes)) continue;
        acc += P->W[h] * profile_at(P, h, p, &cnt);
      }
    }
    out[q] = acc * dphi / (2.0 * M_PI);
    total += cnt;
  }
  if (n_evals) *n_evals = total;
}

/* Threads the OpenMP loops above use, and a way to set them (the CPU baseline times the
 * oracle on one core and on all cores). */
#include <omp.h>
int oracle_threads(void) { return omp_get_max_threads(); }
void oracle_set_threads(int n) { omp_set_num_threads(n); }
