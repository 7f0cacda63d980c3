// Adjoint of the detector image for a pixel weight G = dL/dimage.
//
// k_profile_adj walks the same tile lists, node windows and tile-level node queue as
// the forward kernel and, per pixel lane inside the support, accumulates
//   z  = g omega Z',  s = g domega/dsigma Z',  y = g domega/dgamma Z',  n_i = g omega D_i
// with g = G L(R) of the pixel, Z = C Z' the lineshape's profile product (C its
// per-reflection constant) and D_i = N_i (dZ/dN_i)/C at fixed u (eval_node_adj gives D_i
// for each lineshape; for the Laue form, with y_i = N_i u_i/2 and S_j = sin(2 pi y_j)/y_j,
// D_i = S_i (4 pi cos(2 pi y_i) - S_i) prod_{j != i} S_j^2).  Per (tile, reflection) the six
// lane sums are reduced over the wave and added in binary64 to the reflection's sums.
// Profile values are recomputed, never stored.
//
// k_adj_finish applies the chain rule per reflection in binary64:
//   dL/dW = K z,  W = |F|^2 I_para D,  K = r0^2 C
//   dL/dsigma_theta += W K s,  dL/dgamma_theta += W K y
//   dL/dN_eff,i = W K n_i / N_i,  dN_eff/dN_base = N_eff^2/N_base^2            (Eq. Neff)
//   dN_eff/dA = 2 N_eff^2/(1 + A)^2,  dI_para/dA_i = I_para (1 - A^2)/(A (1 + A^2)) (Eq. Ipara)
//   dA/dg = -4 pi^2 g h^2 A                                                    (Eq. Ah)
//   D = exp(-1/4 sum_i B_i h_i^2/|a_i|^2),  dW/dB_i = -W h_i^2/(4 |a_i|^2)   (axis damping)
// and reduces the FDTBX_N_GLOBALS global gradients over reflections in a fixed order.
//
// k_sf_adj_* carry dL/d|F|^2 back to the atoms (Eq. structure_factor):
//   d|F|^2/dx_j = -4 pi h occ_j Im(F* t_j/occ_j) (likewise y with k, z with l),
//   d|F|^2/dB_j = -2 s^2 occ_j Re(F* t_j/occ_j),  d|F|^2/docc_j = 2 Re(F* t_j/occ_j).
#include <hip/hip_runtime.h>

#include <math.h>

#include "internal.h"
#include "profile_common.h"
#include "adjoint_tile.h"

namespace fdtbx {

template <int LS, int WAVES>
__global__ void __launch_bounds__(64 * WAVES) k_profile_adj(ProfParams q, const float* __restrict__ refl,
                                                            const float* __restrict__ nodes, const double* __restrict__ pix,
                                                            const double* __restrict__ tile,
                                                            const int64_t* __restrict__ offsets,
                                                            const int32_t* __restrict__ idx,
                                                            const float* __restrict__ grad_image, int64_t n_hkl,
                                                            double* __restrict__ sums, float* __restrict__ partials,
                                                            const int32_t* __restrict__ order) {
  __shared__ float4 qn[128 * WAVES];
  __shared__ float2 qd[128 * WAVES];
  __shared__ int bq[64 * WAVES];
  __shared__ int qk[LS == FDTBX_LINESHAPE_HOSEMANN ? 128 * WAVES : 1];  // node indices (support edge)
  const int t = order ? order[blockIdx.x] : tile_of_block(q, blockIdx.x);
  if (t < 0) return;
  adjoint_tile<LS, WAVES>(q, refl, nodes, pix, tile, offsets, idx, grad_image, n_hkl, sums, partials, t, qn, qd, bq,
                          LS == FDTBX_LINESHAPE_HOSEMANN ? qk : nullptr);
}

template <int WAVES>
static void launch_adj(const ProfParams& q, dim3 grid, hipStream_t s, const float* refl, const float* nodes,
                       const double* pix, const double* tile, const int64_t* offsets, const int32_t* idx,
                       const int32_t* order, const float* grad_image, int64_t n_hkl, double* sums, float* partials) {
  const dim3 block(64 * WAVES);
  if (q.lineshape == FDTBX_LINESHAPE_GAUSSIAN)
    hipLaunchKernelGGL((k_profile_adj<FDTBX_LINESHAPE_GAUSSIAN, WAVES>), grid, block, 0, s, q, refl, nodes, pix, tile,
                       offsets, idx, grad_image, n_hkl, sums, partials, order);
  else if (q.lineshape == FDTBX_LINESHAPE_HOSEMANN)
    hipLaunchKernelGGL((k_profile_adj<FDTBX_LINESHAPE_HOSEMANN, WAVES>), grid, block, 0, s, q, refl, nodes, pix, tile,
                       offsets, idx, grad_image, n_hkl, sums, partials, order);
  else
    hipLaunchKernelGGL((k_profile_adj<FDTBX_LINESHAPE_LAUE, WAVES>), grid, block, 0, s, q, refl, nodes, pix, tile, offsets,
                       idx, grad_image, n_hkl, sums, partials, order);
}

// Balanced adjoint: persistent waves over the work units of a balanced forward launch of the
// same lists (its unit tables, read only), with queue counters of their own.  A unit's pairs
// send their sums out on their own, as in the per-tile launch, so units need no combining.
template <int LS>
__global__ void __launch_bounds__(256) k_profile_adj_units(ProfParams q, const float* __restrict__ refl,
                                                           const float* __restrict__ nodes,
                                                           const double* __restrict__ pix,
                                                           const double* __restrict__ tile,
                                                           const int64_t* __restrict__ offsets,
                                                           const int32_t* __restrict__ idx,
                                                           const float* __restrict__ grad_image, int64_t n_hkl,
                                                           double* __restrict__ sums, float* __restrict__ partials,
                                                           UnitTable T) {
  __shared__ float4 qn[128 * 4];
  __shared__ float2 qd[128 * 4];
  __shared__ int bq[64 * 4];
  __shared__ int qk[LS == FDTBX_LINESHAPE_HOSEMANN ? 128 * 4 : 1];  // node indices (support edge)
  const int wv = (int)(threadIdx.x >> 6), lane = (int)(threadIdx.x & 63);
  const int64_t U = T.meta[1];
  const int64_t total = U > 0 ? min(T.meta[0], T.max_units) : 0;
  const int home = (int)(blockIdx.x % kXcds);
  for (int k = 0; k < kXcds; ++k) {
    const int x = (home + k) % kXcds;
    int64_t qb, qe;
    queue_span(T, x, total, &qb, &qe);
    for (;;) {
      int got = 0;
      if (lane == 0) got = atomicAdd(&T.ctr[x], 1);
      const int64_t u = qb + (int64_t)__builtin_amdgcn_readfirstlane(got);
      if (u >= qe) break;  // uniform
      int64_t p0, p1;
      const int t = unit_range(q, T, offsets, u, U, &p0, &p1);
      if (t < 0) continue;
      adjoint_range<LS>(q, refl, nodes, pix, tile, idx, grad_image, n_hkl, sums, partials, t, p0, p1, 64,
                        qn + 128 * wv, qd + 128 * wv, bq + 64 * wv,
                        LS == FDTBX_LINESHAPE_HOSEMANN ? qk + 128 * wv : nullptr);
    }
  }
}

__global__ void k_zero_i32(int32_t* __restrict__ v, int n) {
  if ((int)threadIdx.x < n) v[threadIdx.x] = 0;
}

template <int LS>
static int launch_adj_units(const ProfParams& q, const float* refl, const float* nodes, const double* pix,
                            const double* tile, const int64_t* offsets, const int32_t* idx, const float* grad_image,
                            int64_t n_hkl, double* sums, float* partials, const UnitTable& T, hipStream_t s) {
  int dev = 0, cus = 0, per_cu = 0;
  FDTBX_HIP(hipGetDevice(&dev));
  FDTBX_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  FDTBX_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void*>(&k_profile_adj_units<LS>),
                                                         256, 0));
  const unsigned n_wg = (unsigned)(cus > 0 ? cus : 1) * (unsigned)(per_cu > 0 ? per_cu : 1);
  hipLaunchKernelGGL(k_profile_adj_units<LS>, dim3(n_wg), dim3(256), 0, s, q, refl, nodes, pix, tile, offsets, idx,
                     grad_image, n_hkl, sums, partials, T);
  FDTBX_LAUNCH_CHECK("balanced profile adjoint");
  return FDTBX_OK;
}

// The balanced adjoint over the units that the balanced forward launch with the same model,
// lists, order and pair_cap left in units_ws; ctr: 8 int32 of device memory for its queues.
// The sums (or partials) must be cleared by the caller.
int launch_adjoint_units(const fdtbx_model* model, const float* refl, const float* nodes, const double* pix,
                         const double* tile, const int64_t* offsets, const int32_t* idx, const int32_t* order,
                         int64_t pair_cap, const void* units_ws, int32_t* ctr, int64_t n_hkl, const float* grad_image,
                         double* sums, float* partials, hipStream_t s) {
  ProfParams q;
  prof_params(model, &q);
  const UnitLayout L = unit_layout(q, order != nullptr, pair_cap, model->geom.unit_pairs);
  UnitTable T = unit_view(L, order, model->geom.unit_pairs, const_cast<void*>(units_ws));
  T.ctr = ctr;
  hipLaunchKernelGGL(k_zero_i32, dim3(1), dim3(64), 0, s, ctr, kXcds);
  FDTBX_LAUNCH_CHECK("balanced adjoint counters");
  if (q.lineshape == FDTBX_LINESHAPE_GAUSSIAN)
    return launch_adj_units<FDTBX_LINESHAPE_GAUSSIAN>(q, refl, nodes, pix, tile, offsets, idx, grad_image, n_hkl, sums,
                                                      partials, T, s);
  if (q.lineshape == FDTBX_LINESHAPE_HOSEMANN)
    return launch_adj_units<FDTBX_LINESHAPE_HOSEMANN>(q, refl, nodes, pix, tile, offsets, idx, grad_image, n_hkl, sums,
                                                      partials, T, s);
  return launch_adj_units<FDTBX_LINESHAPE_LAUE>(q, refl, nodes, pix, tile, offsets, idx, grad_image, n_hkl, sums,
                                                partials, T, s);
}

__global__ void k_zero_f64(double* __restrict__ v, int64_t n) {
  int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) v[k] = 0.0;
}

__global__ void k_zero_f32(float* __restrict__ v, int64_t n) {
  int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) v[k] = 0.0f;
}

// ---------------------------------------------------------------- fixed-order reduction
// sums[r][c] = sum over the pairs p of reflection r (refl_pairs[refl_ptr[r] .. refl_ptr[r+1]),
// ascending culling-list position) of partials[p][c], then over the pairs of its mate m
// (mate[r], or n - 1 - r when mate is NULL and updown is set; none otherwise) of
// partials[p][6 + c]; binary64, one thread per reflection, a fixed order.
__global__ void k_pair_reduce(int64_t n, const int64_t* __restrict__ refl_ptr, const int32_t* __restrict__ refl_pairs,
                              const float* __restrict__ partials, const int64_t* __restrict__ mate, int32_t updown,
                              double* __restrict__ sums) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n) return;
  double v[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  for (int64_t k = refl_ptr[r]; k < refl_ptr[r + 1]; ++k) {
    const float* o = partials + 12 * (int64_t)refl_pairs[k];
#pragma unroll
    for (int c = 0; c < 6; ++c) v[c] += (double)o[c];
  }
  const int64_t m = mate ? mate[r] : (updown ? n - 1 - r : -1);
  if (m >= 0) {
    for (int64_t k = refl_ptr[m]; k < refl_ptr[m + 1]; ++k) {
      const float* o = partials + 12 * (int64_t)refl_pairs[k] + 6;
#pragma unroll
      for (int c = 0; c < 6; ++c) v[c] += (double)o[c];
    }
  }
#pragma unroll
  for (int c = 0; c < 6; ++c) sums[6 * r + c] = v[c];
}

// ---------------------------------------------------------------- chain rule per reflection
struct FinishParams {
  double Nb[3], g[3];
  double Bax[3], ia2[3];  // axis damping B_i and 1/|a_i|^2
  int32_t intensity_model;
  int64_t n;
};

constexpr int kNG = FDTBX_N_GLOBALS;

static constexpr int kFinThreads = 256;

// Block sum of kNG doubles per thread into part[block][kNG] (fixed tree order).
__device__ static void block_sum(double v[kNG], double* part) {
  __shared__ double red[kFinThreads / 64][kNG];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  for (int c = 0; c < kNG; ++c) {
    double x = v[c];
    for (int o = 32; o >= 1; o >>= 1) x += __shfl_xor(x, o, 64);
    if (lane == 0) red[wid][c] = x;
  }
  __syncthreads();
  if (threadIdx.x < kNG) {
    double x = 0.0;
    for (int w = 0; w < kFinThreads / 64; ++w) x += red[w][threadIdx.x];
    part[kNG * (int64_t)blockIdx.x + threadIdx.x] = x;
  }
}

// Chain rule for one reflection (binary64).  Returns dL/d|F|^2 and adds the kNG global
// contributions to v.
__device__ static double finish_one(const FinishParams& p, const int32_t* hk, const float* rec, const double* sr,
                                    const float* Fr, double v[kNG]) {
  const double pi2 = M_PI * M_PI;
  double A[3], N[3], Ip = 1.0, h2[3], Dx = 0.0;
  for (int i = 0; i < 3; ++i) {
    double h = (double)hk[i];
    h2[i] = h * h;
    A[i] = exp(-2.0 * pi2 * p.g[i] * p.g[i] * h2[i]);
    N[i] = 1.0 / (1.0 / p.Nb[i] + (1.0 - A[i]) / (1.0 + A[i]));
    if (p.intensity_model) Ip *= 2.0 * A[i] / (1.0 + A[i] * A[i]);
    Dx += p.Bax[i] * h2[i] * p.ia2[i];
  }
  const double Dw = exp(-0.25 * Dx);
  const double fr = Fr[0], fi = Fr[1];
  const double f2 = fr * fr + fi * fi;
  const double W = f2 * Ip * Dw;
  const double K = (double)rec[RS_K];
  const double dW = K * sr[0];
  const double WK = W * K;
  v[0] += WK * sr[1];
  v[1] += WK * sr[2];
  const double dIp = dW * f2 * Dw;
  for (int i = 0; i < 3; ++i) {
    const double dN = WK * sr[3 + i] / N[i];
    v[2 + i] += dN * N[i] * N[i] / (p.Nb[i] * p.Nb[i]);
    double dA = dN * 2.0 * N[i] * N[i] / ((1.0 + A[i]) * (1.0 + A[i]));
    if (p.intensity_model) dA += dIp * Ip * (1.0 - A[i] * A[i]) / (A[i] * (1.0 + A[i] * A[i]));
    v[5 + i] += dA * (-4.0 * pi2 * p.g[i] * h2[i] * A[i]);
    v[8 + i] += dW * W * (-0.25 * h2[i] * p.ia2[i]);
  }
  return dW * Ip * Dw;
}

__global__ void __launch_bounds__(kFinThreads) k_adj_finish(FinishParams p, const int32_t* __restrict__ hkl,
                                                            const float* __restrict__ refl, const double* __restrict__ sums,
                                                            const float* __restrict__ F, float* __restrict__ dF2,
                                                            double* __restrict__ part) {
  const int64_t r = (int64_t)blockIdx.x * kFinThreads + threadIdx.x;
  double v[kNG] = {};
  if (r < p.n) {
    const double d = finish_one(p, hkl + 3 * r, refl + (int64_t)FDTBX_REFL_FLOATS * r, sums + 6 * r, F + 2 * r, v);
    if (dF2) dF2[r] = (float)d;
  }
  block_sum(v, part);
}

__global__ void k_sum_parts(const double* __restrict__ part, int64_t nb, double* __restrict__ out) {
  const int c = threadIdx.x;
  if (c >= kNG) return;
  double x = 0.0;
  for (int64_t b = 0; b < nb; ++b) x += part[kNG * b + c];
  out[c] = x;
}

// ---------------------------------------------------------------- atoms
static constexpr int kSAThreads = 256;
static constexpr int kSAMaxTypes = 16;
static constexpr int kReflPerChunkMax = 2048;

struct SAParams {
  double as[9];
  int64_t n_hkl, n_atoms, chunk;
  int32_t n_types, n_chunks;
};

struct ReflLds {
  int h, k, l;
  float s2, cre, cim;
};

__global__ void __launch_bounds__(kSAThreads) k_sf_adj_partial(SAParams p, const float* __restrict__ x, const float* __restrict__ y,
                                                               const float* __restrict__ z, const float* __restrict__ B,
                                                               const int32_t* __restrict__ type, const float* __restrict__ ff,
                                                               const int32_t* __restrict__ hkl, const float* __restrict__ F,
                                                               const float* __restrict__ dF2, double* __restrict__ part) {
  __shared__ ReflLds rl[kSAThreads];
  __shared__ float ft[kSAThreads][kSAMaxTypes + 1];
  const int64_t a = (int64_t)blockIdx.x * kSAThreads + threadIdx.x;
  const bool have = a < p.n_atoms;
  const double ax = have ? x[a] : 0.0, ay = have ? y[a] : 0.0, az = have ? z[a] : 0.0;
  int ta = have ? type[a] : 0;
  ta = ta < 0 ? 0 : (ta >= p.n_types ? p.n_types - 1 : ta);
  const float nBl2e = have ? -B[a] * 1.4426950408889634f : 0.0f;
  const int64_t r0 = (int64_t)blockIdx.y * p.chunk;
  const int64_t r1 = r0 + p.chunk < p.n_hkl ? r0 + p.chunk : p.n_hkl;
  double g[5] = {0.0, 0.0, 0.0, 0.0, 0.0};  // h Im, k Im, l Im, s^2 Re, Re (binary64: sums cancel strongly)
  for (int64_t g0 = r0; g0 < r1; g0 += kSAThreads) {
    __syncthreads();
    const int64_t r = g0 + threadIdx.x;
    if (r < r1) {
      const double h = hkl[3 * r], k = hkl[3 * r + 1], l = hkl[3 * r + 2];
      double D[3];
      for (int j = 0; j < 3; ++j) D[j] = (h * p.as[j] + k * p.as[3 + j]) + l * p.as[6 + j];
      const double s2 = 0.25 * ((D[0] * D[0] + D[1] * D[1]) + D[2] * D[2]);
      const float w = dF2[r];
      rl[threadIdx.x] = {(int)h, (int)k, (int)l, (float)s2, w * F[2 * r], -w * F[2 * r + 1]};
      for (int t = 0; t < p.n_types; ++t) {
        const float* c = ff + 9 * t;
        double f = c[8];
        for (int q = 0; q < 4; ++q) f += (double)c[q] * exp(-(double)c[4 + q] * s2);
        ft[threadIdx.x][t] = (float)f;
      }
    }
    __syncthreads();
    const int cnt = (int)((r1 - g0) < kSAThreads ? (r1 - g0) : kSAThreads);
    if (have) {
      for (int i = 0; i < cnt; ++i) {
        const ReflLds q = rl[i];
        const double ph = fma((double)q.h, ax, fma((double)q.k, ay, (double)q.l * az));
        const float fr = (float)(ph - floor(ph));
        const float amp = ft[i][ta] * __builtin_amdgcn_exp2f(nBl2e * q.s2);
        const float cs = __builtin_amdgcn_cosf(fr), sn = __builtin_amdgcn_sinf(fr);
        // C t/occ with C = dF2 F*: real and imaginary parts
        const float re = amp * (q.cre * cs - q.cim * sn);
        const float im = amp * (q.cre * sn + q.cim * cs);
        g[0] = fma((double)q.h, (double)im, g[0]);
        g[1] = fma((double)q.k, (double)im, g[1]);
        g[2] = fma((double)q.l, (double)im, g[2]);
        g[3] = fma((double)q.s2, (double)re, g[3]);
        g[4] += (double)re;
      }
    }
  }
  if (have)
    for (int c = 0; c < 5; ++c) part[((int64_t)blockIdx.y * 5 + c) * p.n_atoms + a] = g[c];
}

__global__ void k_sf_adj_final(int64_t n_atoms, int32_t n_chunks, const double* __restrict__ part, const float* __restrict__ occ,
                               float* dx, float* dy, float* dz, float* dB, float* docc) {
  const int64_t a = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (a >= n_atoms) return;
  double s[5] = {0, 0, 0, 0, 0};
  for (int c = 0; c < n_chunks; ++c)
    for (int k = 0; k < 5; ++k) s[k] += part[((int64_t)c * 5 + k) * n_atoms + a];
  const double o = occ[a];
  const double fpi = 4.0 * M_PI;
  if (dx) dx[a] = (float)(-fpi * o * s[0]);
  if (dy) dy[a] = (float)(-fpi * o * s[1]);
  if (dz) dz[a] = (float)(-fpi * o * s[2]);
  if (dB) dB[a] = (float)(-2.0 * o * s[3]);
  if (docc) docc[a] = (float)(2.0 * s[4]);
}

static void sa_split(int64_t n_hkl, int64_t n_atoms, int32_t* n_chunks, int64_t* chunk) {
  int64_t nb = ceil_div(n_atoms, kSAThreads);
  int64_t want = ceil_div(4096, nb);
  int64_t need = ceil_div(n_hkl, kReflPerChunkMax);
  int64_t nc = want > need ? want : need;
  int64_t maxc = ceil_div(n_hkl, 64);
  if (nc > maxc) nc = maxc;
  if (nc < 1) nc = 1;
  *chunk = ceil_div(n_hkl, nc);
  *n_chunks = (int32_t)ceil_div(n_hkl, *chunk);
}

static void recip_basis(const fdtbx_cell* cell, double* as) {
  double ca = cos(cell->alpha), cb = cos(cell->beta), cg = cos(cell->gamma), sa = sin(cell->alpha);
  double cv[3] = {0.0, 0.0, cell->c};
  double bv[3] = {0.0, cell->b * sa, cell->b * ca};
  double az = cell->a * cb, ay = cell->a * (cg - ca * cb) / sa;
  double av[3] = {sqrt(cell->a * cell->a - ay * ay - az * az), ay, az};
  auto cross = [](const double* u, const double* v, double* w) {
    w[0] = u[1] * v[2] - u[2] * v[1];
    w[1] = u[2] * v[0] - u[0] * v[2];
    w[2] = u[0] * v[1] - u[1] * v[0];
  };
  double bxc[3], cxa[3], axb[3];
  cross(bv, cv, bxc);
  cross(cv, av, cxa);
  cross(av, bv, axb);
  double V = (av[0] * bxc[0] + av[1] * bxc[1]) + av[2] * bxc[2];
  for (int j = 0; j < 3; ++j) {
    as[j] = bxc[j] / V;
    as[3 + j] = cxa[j] / V;
    as[6 + j] = axb[j] / V;
  }
}

// ---------------------------------------------------------------- batched models
__global__ void __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(5))) k_b_profile_adj(const fdtbx_batch_entry* __restrict__ ent, const int64_t* __restrict__ items,
                                                      int64_t n_items, const float* __restrict__ refl,
                                                      const float* __restrict__ nodes, const double* __restrict__ pix,
                                                      const double* __restrict__ tile, const int64_t* __restrict__ rowptr,
                                                      const int32_t* __restrict__ idx, const float* __restrict__ grad_image,
                                                      double* __restrict__ sums, float* __restrict__ partials,
                                                      unsigned long long* __restrict__ counter) {
  __shared__ float4 qn[128];
  __shared__ float2 qd[128];
  __shared__ int bq[64];
  __shared__ int qk[128];  // node indices of the queue (the Hosemann support edge)
  for (;;) {
    const int64_t it = next_item(counter);
    if (it >= n_items) break;
    const int64_t packed = items[it];
    const int m = (int)(packed >> 40);
    const int t = (int)(packed & ((1ll << 40) - 1));
    const fdtbx_batch_entry& e = ent[m];
    ProfParams q;
    prof_params(&e.model, &q);
    const float* rf = refl + (int64_t)FDTBX_REFL_FLOATS * e.hkl_off;
    const float* nd = nodes + (int64_t)FDTBX_NODE_FLOATS * e.node_off;
    const double* px = pix + 2 * e.pix_off;
    const double* tb = tile + 8 * e.tile_off;
    const int64_t* rp = rowptr + e.rowptr_off;
    const int32_t* ix = idx + e.pair_off;
    const float* gi = grad_image + e.pix_off;
    double* sm = sums + 6 * e.hkl_off;
    float* pt = partials ? partials + 12 * e.pair_off : nullptr;
    switch (q.lineshape) {  // uniform across the wave
      case FDTBX_LINESHAPE_GAUSSIAN:
        adjoint_tile<FDTBX_LINESHAPE_GAUSSIAN, 1, true>(q, rf, nd, px, tb, rp, ix, gi, e.n_hkl, sm, pt, t, qn, qd, bq);
        break;
      case FDTBX_LINESHAPE_HOSEMANN:
        adjoint_tile<FDTBX_LINESHAPE_HOSEMANN, 1, true>(q, rf, nd, px, tb, rp, ix, gi, e.n_hkl, sm, pt, t, qn, qd, bq,
                                                        qk);
        break;
      default:
        adjoint_tile<FDTBX_LINESHAPE_LAUE, 1, true>(q, rf, nd, px, tb, rp, ix, gi, e.n_hkl, sm, pt, t, qn, qd, bq);
    }
  }
}

__device__ static void finish_params_of(const fdtbx_batch_entry& e, FinishParams* p) {
  for (int i = 0; i < 3; ++i) {
    p->Nb[i] = e.model.dis.N_base[i];
    p->g[i] = e.model.dis.g[i];
    p->Bax[i] = e.model.dis.B_axis[i];
  }
  const double len[3] = {e.model.cell.a, e.model.cell.b, e.model.cell.c};
  for (int i = 0; i < 3; ++i) p->ia2[i] = 1.0 / (len[i] * len[i]);
  p->intensity_model = e.model.dis.intensity_model;
  p->n = e.n_hkl;
}

__global__ void __launch_bounds__(kFinThreads) k_b_finish(const fdtbx_batch_entry* __restrict__ ent, const int64_t* __restrict__ blocks,
                                                          const int32_t* __restrict__ hkl, const float* __restrict__ refl,
                                                          const double* __restrict__ sums, const float* __restrict__ F,
                                                          float* __restrict__ dF2, double* __restrict__ part) {
  const int64_t item = blocks[blockIdx.x];
  const int m = (int)(item >> 40);
  const fdtbx_batch_entry& e = ent[m];
  const int64_t r = (item & ((1ll << 40) - 1)) + threadIdx.x;
  double v[kNG] = {};
  if (r < e.n_hkl) {
    FinishParams p;
    finish_params_of(e, &p);
    const int64_t g = e.hkl_off + r;
    dF2[g] = (float)finish_one(p, hkl + 3 * g, refl + (int64_t)FDTBX_REFL_FLOATS * g, sums + 6 * g, F + 2 * g, v);
  }
  block_sum(v, part);
}

// d_globals[m] = sum of the model's block partials, in block order.
__global__ void k_b_globals(int32_t n_models, const int64_t* __restrict__ model_rb, const double* __restrict__ part,
                            double* __restrict__ out) {
  const int m = blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= n_models) return;
  double v[kNG] = {};
  for (int64_t b = model_rb[m]; b < model_rb[m + 1]; ++b)
    for (int c = 0; c < kNG; ++c) v[c] += part[kNG * b + c];
  for (int c = 0; c < kNG; ++c) out[kNG * (int64_t)m + c] = v[c];
}

// One thread per atom of one model; loops over all of the model's reflections.
__global__ void __launch_bounds__(kSAThreads) k_b_sf_adj(const fdtbx_batch_entry* __restrict__ ent, const int64_t* __restrict__ blocks,
                                                         const float* __restrict__ x, const float* __restrict__ y,
                                                         const float* __restrict__ z, const float* __restrict__ B,
                                                         const float* __restrict__ occ, const int32_t* __restrict__ type,
                                                         const float* __restrict__ ff, const int32_t* __restrict__ hkl,
                                                         const float* __restrict__ F, const float* __restrict__ dF2,
                                                         float* d_x, float* d_y, float* d_z, float* d_B, float* d_occ) {
  __shared__ ReflLds rl[kSAThreads];
  __shared__ float ft[kSAThreads][kSAMaxTypes + 1];
  const int64_t item = blocks[blockIdx.x];
  const int m = (int)(item >> 40);
  const fdtbx_batch_entry& e = ent[m];
  const int64_t al = (item & ((1ll << 40) - 1)) + threadIdx.x;
  const bool have = al < e.n_atoms;
  const int64_t a = e.atom_off + al;
  // kept in 1..kSAMaxTypes by fdtbx_batch_entries_check; clamped so the LDS table stays in bounds
  const int n_types = e.n_types < 1 ? 1 : (e.n_types > kSAMaxTypes ? kSAMaxTypes : e.n_types);
  const float* ffm = ff + 9 * e.ff_off;
  const double ax = have ? x[a] : 0.0, ay = have ? y[a] : 0.0, az = have ? z[a] : 0.0;
  int ta = have ? type[a] : 0;
  ta = ta < 0 ? 0 : (ta >= n_types ? n_types - 1 : ta);
  const float nBl2e = have ? -B[a] * 1.4426950408889634f : 0.0f;
  const int64_t r0 = e.hkl_off, r1 = e.hkl_off + e.n_hkl;
  double g[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  for (int64_t g0 = r0; g0 < r1; g0 += kSAThreads) {
    __syncthreads();
    const int64_t r = g0 + threadIdx.x;
    if (r < r1) {
      const double h = hkl[3 * r], k = hkl[3 * r + 1], l = hkl[3 * r + 2];
      double D[3];
      for (int j = 0; j < 3; ++j) D[j] = (h * e.frame[9 + j] + k * e.frame[12 + j]) + l * e.frame[15 + j];
      const double s2 = 0.25 * ((D[0] * D[0] + D[1] * D[1]) + D[2] * D[2]);
      const float w = dF2[r];
      rl[threadIdx.x] = {(int)h, (int)k, (int)l, (float)s2, w * F[2 * r], -w * F[2 * r + 1]};
      for (int t = 0; t < n_types; ++t) {
        const float* c = ffm + 9 * t;
        double f = c[8];
        for (int q = 0; q < 4; ++q) f += (double)c[q] * exp(-(double)c[4 + q] * s2);
        ft[threadIdx.x][t] = (float)f;
      }
    }
    __syncthreads();
    const int cnt = (int)((r1 - g0) < kSAThreads ? (r1 - g0) : kSAThreads);
    if (have) {
      for (int i = 0; i < cnt; ++i) {
        const ReflLds q = rl[i];
        const double ph = fma((double)q.h, ax, fma((double)q.k, ay, (double)q.l * az));
        const float fr = (float)(ph - floor(ph));
        const float amp = ft[i][ta] * __builtin_amdgcn_exp2f(nBl2e * q.s2);
        const float cs = __builtin_amdgcn_cosf(fr), sn = __builtin_amdgcn_sinf(fr);
        const float re = amp * (q.cre * cs - q.cim * sn);
        const float im = amp * (q.cre * sn + q.cim * cs);
        g[0] = fma((double)q.h, (double)im, g[0]);
        g[1] = fma((double)q.k, (double)im, g[1]);
        g[2] = fma((double)q.l, (double)im, g[2]);
        g[3] = fma((double)q.s2, (double)re, g[3]);
        g[4] += (double)re;
      }
    }
  }
  if (have) {
    const double o = occ[a];
    const double fpi = 4.0 * M_PI;
    if (d_x) d_x[a] = (float)(-fpi * o * g[0]);
    if (d_y) d_y[a] = (float)(-fpi * o * g[1]);
    if (d_z) d_z[a] = (float)(-fpi * o * g[2]);
    if (d_B) d_B[a] = (float)(-2.0 * o * g[3]);
    if (d_occ) d_occ[a] = (float)(2.0 * g[4]);
  }
}

__global__ void k_b_set_globals(fdtbx_batch_entry* __restrict__ ent, int32_t n_models, const double* __restrict__ glob) {
  const int m = blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= n_models) return;
  fdtbx_disorder& d = ent[m].model.dis;
  const double* gl = glob + kNG * (int64_t)m;
  d.sigma_theta = gl[0];
  d.gamma_theta = gl[1];
  int32_t stale = 0;
  for (int i = 0; i < 3; ++i) {
    d.N_base[i] = gl[2 + i];
    d.g[i] = gl[5 + i];
    d.B_axis[i] = gl[8 + i];
    // a larger g or a smaller N_base widens the support beyond the lists' (NaN counts as wider)
    if (!(gl[5 + i] <= ent[m].setup_g[i]) || !(gl[2 + i] >= ent[m].setup_N_base[i])) stale = 1;
  }
  ent[m].stale = stale;
}

static constexpr unsigned kPersistentBlocksAdj = 8192;

}  // namespace fdtbx

using namespace fdtbx;

extern "C" int fdtbx_batch_set_globals(fdtbx_batch_entry* entries, int32_t n_models, const double* globals, void* stream) {
  if (!entries || !globals || n_models <= 0) return fail(FDTBX_ERR_INVALID_ARGUMENT, "bad arguments");
  hipLaunchKernelGGL(k_b_set_globals, dim3((unsigned)ceil_div(n_models, 64)), dim3(64), 0, (hipStream_t)stream, entries,
                     n_models, globals);
  FDTBX_LAUNCH_CHECK("batch set globals");
  return FDTBX_OK;
}

namespace fdtbx {
int launch_batch_backward(const fdtbx_batch_entry* ent, int32_t n_models, const int64_t* refl_blocks, int64_t n_rb,
                          const int64_t* model_rb, const int64_t* atom_blocks, int64_t n_ab, const int64_t* items,
                          int64_t n_items, int64_t n_hkl_total, const int32_t* hkl, const float* x, const float* y,
                          const float* z, const float* B, const float* occ, const int32_t* type, const float* ff,
                          const double* pix, const double* tile, const int64_t* rowptr, const int32_t* idx, const float* F,
                          const float* refl, const float* nodes, const float* grad_image, double* sums, double* part,
                          float* dF2, float* d_x, float* d_y, float* d_z, float* d_B, float* d_occ, double* d_globals,
                          int64_t* counter, const PairOrder* fixed, hipStream_t s) {
  if (fixed) {
    hipLaunchKernelGGL(k_zero_f32, dim3((unsigned)ceil_div(12 * fixed->n_pairs, 256)), dim3(256), 0, s, fixed->partials,
                       12 * fixed->n_pairs);
    FDTBX_LAUNCH_CHECK("batch adjoint partials zero");
  } else {
    hipLaunchKernelGGL(k_zero_f64, dim3((unsigned)ceil_div(6 * n_hkl_total, 256)), dim3(256), 0, s, sums, 6 * n_hkl_total);
    FDTBX_LAUNCH_CHECK("batch adjoint zero");
  }
  hipLaunchKernelGGL(k_zero_f64, dim3(1), dim3(64), 0, s, (double*)counter, (int64_t)1);
  FDTBX_LAUNCH_CHECK("batch adjoint counter");
  if (n_items > 0) {
    unsigned nb = n_items < (int64_t)kPersistentBlocksAdj ? (unsigned)n_items : kPersistentBlocksAdj;
    hipLaunchKernelGGL(k_b_profile_adj, dim3(nb), dim3(64), 0, s, ent, items, n_items, refl, nodes, pix, tile, rowptr, idx,
                       grad_image, sums, fixed ? fixed->partials : nullptr, (unsigned long long*)counter);
    FDTBX_LAUNCH_CHECK("batch profile adjoint");
  }
  if (fixed && n_hkl_total > 0) {
    hipLaunchKernelGGL(k_pair_reduce, dim3((unsigned)ceil_div(n_hkl_total, 256)), dim3(256), 0, s, n_hkl_total,
                       fixed->refl_ptr, fixed->refl_pairs, fixed->partials, fixed->mate, 0, sums);
    FDTBX_LAUNCH_CHECK("batch adjoint pair reduction");
  }
  if (n_rb > 0) {
    hipLaunchKernelGGL(k_b_finish, dim3((unsigned)n_rb), dim3(kFinThreads), 0, s, ent, refl_blocks, hkl, refl, sums, F, dF2,
                       part);
    FDTBX_LAUNCH_CHECK("batch adjoint finish");
  }
  hipLaunchKernelGGL(k_b_globals, dim3((unsigned)ceil_div(n_models, 64)), dim3(64), 0, s, n_models, model_rb, part, d_globals);
  FDTBX_LAUNCH_CHECK("batch adjoint globals");
  if (n_ab > 0 && (d_x || d_y || d_z || d_B || d_occ)) {
    hipLaunchKernelGGL(k_b_sf_adj, dim3((unsigned)n_ab), dim3(kSAThreads), 0, s, ent, atom_blocks, x, y, z, B, occ, type, ff, hkl,
                       F, dF2, d_x, d_y, d_z, d_B, d_occ);
    FDTBX_LAUNCH_CHECK("batch sf adjoint");
  }
  return FDTBX_OK;
}
}  // namespace fdtbx

namespace fdtbx {
// The per-tile adjoint launch: atomic binary64 sums, or per-pair partials.
static int launch_profile_adjoint(const fdtbx_model* model, const float* refl, const float* nodes, const double* pix,
                                  const double* tile, const int64_t* offsets, const int32_t* idx, const int32_t* order,
                                  int64_t n_hkl, const float* grad_image, double* sums, float* partials, hipStream_t s) {
  ProfParams q;
  prof_params(model, &q);
  const dim3 grid((unsigned)(order ? order_grid(q.lcols, q.lrows) : tile_grid(q)));
  int waves = 1;
  const int rc = tile_waves(&model->geom, (int64_t)q.lcols * q.lrows, &waves);
  if (rc) return rc;
  if (waves == 4)
    launch_adj<4>(q, grid, s, refl, nodes, pix, tile, offsets, idx, order, grad_image, n_hkl, sums, partials);
  else if (waves == 2)
    launch_adj<2>(q, grid, s, refl, nodes, pix, tile, offsets, idx, order, grad_image, n_hkl, sums, partials);
  else
    launch_adj<1>(q, grid, s, refl, nodes, pix, tile, offsets, idx, order, grad_image, n_hkl, sums, partials);
  FDTBX_LAUNCH_CHECK("profile adjoint");
  return FDTBX_OK;
}
}  // namespace fdtbx

extern "C" int fdtbx_profile_adjoint(const fdtbx_model* model, const float* refl, const float* nodes, const double* pix,
                                     const double* tile, const int64_t* offsets, const int32_t* idx, const int32_t* order,
                                     int64_t n_hkl, const float* grad_image, double* sums, void* stream) {
  if (!model) return fail(FDTBX_ERR_INVALID_ARGUMENT, "null pointer");
  if (n_hkl < 0) return fail(FDTBX_ERR_INVALID_ARGUMENT, "n_hkl must be non-negative");
  int rc = check_model(model);
  if (rc) return rc;
  if (n_hkl == 0) return FDTBX_OK;  // no reflections: nothing to sum
  if (!refl || !nodes || !pix || !tile || !offsets || !idx || !grad_image || !sums)
    return fail(FDTBX_ERR_INVALID_ARGUMENT, "null pointer");
  hipStream_t s = (hipStream_t)stream;
  hipLaunchKernelGGL(k_zero_f64, dim3((unsigned)ceil_div(6 * n_hkl, 256)), dim3(256), 0, s, sums, 6 * n_hkl);
  FDTBX_LAUNCH_CHECK("adjoint zero");
  return launch_profile_adjoint(model, refl, nodes, pix, tile, offsets, idx, order, n_hkl, grad_image, sums, nullptr, s);
}

extern "C" int fdtbx_profile_adjoint_balanced(const fdtbx_model* model, const float* refl, const float* nodes,
                                              const double* pix, const double* tile, const int64_t* offsets,
                                              const int32_t* idx, const int32_t* order, int64_t pair_cap, int64_t n_hkl,
                                              const float* grad_image, double* sums, void* bal_ws, size_t bal_ws_bytes,
                                              void* stream) {
  if (!model) return fail(FDTBX_ERR_INVALID_ARGUMENT, "null pointer");
  if (n_hkl < 0 || pair_cap < 0) return fail(FDTBX_ERR_INVALID_ARGUMENT, "n_hkl and pair_cap must be non-negative");
  int rc = check_model(model);
  if (rc) return rc;
  if (model->geom.unit_pairs < 0) return fail(FDTBX_ERR_INVALID_ARGUMENT, "unit_pairs must be non-negative");
  if (n_hkl == 0) return FDTBX_OK;  // no reflections: nothing to sum
  if (!refl || !nodes || !pix || !tile || !offsets || !idx || !grad_image || !sums || !bal_ws)
    return fail(FDTBX_ERR_INVALID_ARGUMENT, "null pointer");
  ProfParams q;
  prof_params(model, &q);
  const UnitLayout L = unit_layout(q, order != nullptr, pair_cap, model->geom.unit_pairs);
  if (bal_ws_bytes < L.total) return fail(FDTBX_ERR_BUFFER_TOO_SMALL, "balanced workspace too small");
  hipStream_t s = (hipStream_t)stream;
  hipLaunchKernelGGL(k_zero_f64, dim3((unsigned)ceil_div(6 * n_hkl, 256)), dim3(256), 0, s, sums, 6 * n_hkl);
  FDTBX_LAUNCH_CHECK("adjoint zero");
  // the forward launch is done with its queue counters: the adjoint takes them over
  return launch_adjoint_units(model, refl, nodes, pix, tile, offsets, idx, order, pair_cap, bal_ws,
                              (int32_t*)((char*)bal_ws + L.ctr), n_hkl, grad_image, sums, nullptr, s);
}

extern "C" int fdtbx_profile_adjoint_pairs(const fdtbx_model* model, const float* refl, const float* nodes,
                                           const double* pix, const double* tile, const int64_t* offsets, const int32_t* idx,
                                           const int32_t* order, int64_t n_hkl, int64_t pair_cap, const float* grad_image,
                                           float* partials, void* stream) {
  if (!model) return fail(FDTBX_ERR_INVALID_ARGUMENT, "null pointer");
  if (n_hkl < 0 || pair_cap < 0) return fail(FDTBX_ERR_INVALID_ARGUMENT, "n_hkl and pair_cap must be non-negative");
  int rc = check_model(model);
  if (rc) return rc;
  if (pair_cap == 0) return FDTBX_OK;
  if (!partials) return fail(FDTBX_ERR_INVALID_ARGUMENT, "null pointer");
  hipStream_t s = (hipStream_t)stream;
  hipLaunchKernelGGL(k_zero_f32, dim3((unsigned)ceil_div(12 * pair_cap, 256)), dim3(256), 0, s, partials, 12 * pair_cap);
  FDTBX_LAUNCH_CHECK("adjoint partials zero");
  if (n_hkl == 0) return FDTBX_OK;
  if (!refl || !nodes || !pix || !tile || !offsets || !idx || !grad_image)
    return fail(FDTBX_ERR_INVALID_ARGUMENT, "null pointer");
  return launch_profile_adjoint(model, refl, nodes, pix, tile, offsets, idx, order, n_hkl, grad_image, nullptr, partials,
                                s);
}

extern "C" int fdtbx_pair_reduce(int64_t n_hkl, const int64_t* refl_ptr, const int32_t* refl_pairs, const float* partials,
                                 const int64_t* mate, int32_t updown, double* sums, void* stream) {
  if (n_hkl < 0) return fail(FDTBX_ERR_INVALID_ARGUMENT, "n_hkl must be non-negative");
  if (n_hkl == 0) return FDTBX_OK;
  if (!refl_ptr || !refl_pairs || !partials || !sums) return fail(FDTBX_ERR_INVALID_ARGUMENT, "null pointer");
  hipLaunchKernelGGL(k_pair_reduce, dim3((unsigned)ceil_div(n_hkl, 256)), dim3(256), 0, (hipStream_t)stream, n_hkl,
                     refl_ptr, refl_pairs, partials, mate, updown ? 1 : 0, sums);
  FDTBX_LAUNCH_CHECK("pair reduction");
  return FDTBX_OK;
}

extern "C" size_t fdtbx_adjoint_finish_workspace(int64_t n_hkl) {
  if (n_hkl <= 0) return 0;
  return (size_t)ceil_div(n_hkl, kFinThreads) * kNG * sizeof(double);
}

extern "C" int fdtbx_adjoint_finish(const fdtbx_model* model, const int32_t* hkl, int64_t n_hkl, const float* refl,
                                    const double* sums, const float* F, float* dF2, double* d_globals, void* ws,
                                    size_t ws_bytes, void* stream) {
  if (!model || !d_globals) return fail(FDTBX_ERR_INVALID_ARGUMENT, "null pointer");
  if (n_hkl < 0) return fail(FDTBX_ERR_INVALID_ARGUMENT, "n_hkl must be non-negative");
  int rc = check_model(model);
  if (rc) return rc;
  if (n_hkl == 0) return fill(d_globals, (int64_t)kNG, 0.0, (hipStream_t)stream);
  if (!hkl || !refl || !sums || !F || !ws) return fail(FDTBX_ERR_INVALID_ARGUMENT, "null pointer");
  if (ws_bytes < fdtbx_adjoint_finish_workspace(n_hkl)) return fail(FDTBX_ERR_BUFFER_TOO_SMALL, "finish workspace too small");
  FinishParams p;
  const double len[3] = {model->cell.a, model->cell.b, model->cell.c};
  for (int i = 0; i < 3; ++i) {
    p.Nb[i] = model->dis.N_base[i];
    p.g[i] = model->dis.g[i];
    p.Bax[i] = model->dis.B_axis[i];
    p.ia2[i] = 1.0 / (len[i] * len[i]);
  }
  p.intensity_model = model->dis.intensity_model;
  p.n = n_hkl;
  int64_t nb = ceil_div(n_hkl, kFinThreads);
  hipStream_t s = (hipStream_t)stream;
  hipLaunchKernelGGL(k_adj_finish, dim3((unsigned)nb), dim3(kFinThreads), 0, s, p, hkl, refl, sums, F, dF2, (double*)ws);
  FDTBX_LAUNCH_CHECK("adjoint finish");
  hipLaunchKernelGGL(k_sum_parts, dim3(1), dim3(64), 0, s, (const double*)ws, nb, d_globals);
  FDTBX_LAUNCH_CHECK("adjoint globals");
  return FDTBX_OK;
}

extern "C" size_t fdtbx_sf_adjoint_workspace(int64_t n_hkl, int64_t n_atoms) {
  if (n_hkl <= 0 || n_atoms <= 0) return 0;
  int32_t nc;
  int64_t chunk;
  sa_split(n_hkl, n_atoms, &nc, &chunk);
  return (size_t)nc * 5 * n_atoms * sizeof(double);
}

extern "C" int fdtbx_sf_adjoint(const fdtbx_cell* cell, int64_t n_atoms, const float* x, const float* y, const float* z,
                                const float* B, const float* occ, const int32_t* type, const float* ff, int32_t n_types,
                                const int32_t* hkl, int64_t n_hkl, const float* F, const float* dF2, float* d_x, float* d_y,
                                float* d_z, float* d_B, float* d_occ, void* ws, size_t ws_bytes, void* stream) {
  if (!cell) return fail(FDTBX_ERR_INVALID_ARGUMENT, "null pointer");
  if (n_atoms < 0 || n_hkl < 0) return fail(FDTBX_ERR_INVALID_ARGUMENT, "n_atoms and n_hkl must be non-negative");
  if (n_atoms == 0) return FDTBX_OK;
  if (n_hkl == 0) {  // no reflections: every atom gradient is zero
    hipStream_t s0 = (hipStream_t)stream;
    float* const outs[5] = {d_x, d_y, d_z, d_B, d_occ};
    for (float* o : outs) {
      const int r0 = fill(o, n_atoms, 0.0f, s0);
      if (r0) return r0;
    }
    return FDTBX_OK;
  }
  if (!x || !y || !z || !B || !occ || !type || !ff || !hkl || !F || !dF2 || !ws)
    return fail(FDTBX_ERR_INVALID_ARGUMENT, "null pointer");
  if (n_types < 1 || n_types > kSAMaxTypes) return fail(FDTBX_ERR_INVALID_ARGUMENT, "n_types must be in 1..16");
  int rc = check_cell(cell);
  if (rc) return rc;
  if (ws_bytes < fdtbx_sf_adjoint_workspace(n_hkl, n_atoms)) return fail(FDTBX_ERR_BUFFER_TOO_SMALL, "sf adjoint workspace");
  SAParams p;
  recip_basis(cell, p.as);
  p.n_hkl = n_hkl;
  p.n_atoms = n_atoms;
  p.n_types = n_types;
  sa_split(n_hkl, n_atoms, &p.n_chunks, &p.chunk);
  hipStream_t s = (hipStream_t)stream;
  double* part = (double*)ws;
  dim3 grid((unsigned)ceil_div(n_atoms, kSAThreads), (unsigned)p.n_chunks);
  hipLaunchKernelGGL(k_sf_adj_partial, grid, dim3(kSAThreads), 0, s, p, x, y, z, B, type, ff, hkl, F, dF2, part);
  FDTBX_LAUNCH_CHECK("sf adjoint");
  hipLaunchKernelGGL(k_sf_adj_final, dim3((unsigned)ceil_div(n_atoms, 256)), dim3(256), 0, s, n_atoms, p.n_chunks, part, occ, d_x,
                     d_y, d_z, d_B, d_occ);
  FDTBX_LAUNCH_CHECK("sf adjoint reduce");
  return FDTBX_OK;
}
