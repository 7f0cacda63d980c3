// Direct structure factors (Eq. structure_factor with the isotropic Debye-Waller
// factor):  F_hkl = sum_j occ_j f_t(j)(s) exp(-B_j s^2) exp(2 pi i (h x_j + k y_j + l z_j)).
//
// One thread per reflection, atoms streamed through LDS in groups of 256; the atom
// range is split over gridDim.y so that small reflection lists still fill the chip.
// The phase h x + k y + l z is formed in binary64 (exact: integer times float32),
// reduced modulo one turn there and only then rounded to float32, so the argument
// of the hardware sine/cosine (which take revolutions) carries ~3e-8 turns of error
// whatever the size of h.  Partial sums per atom chunk are reduced in a fixed order
// in binary64: deterministic, no atomics.
#include <hip/hip_runtime.h>

#include <math.h>

#include "internal.h"

namespace fdtbx {

static constexpr int kSFThreads = 256;
static constexpr int kMaxTypes = 16;
static constexpr int kAtomsPerChunkMax = 2048;

struct SFParams {
  double as[9];          // reciprocal basis rows a*, b*, c*
  int64_t n_hkl, n_atoms, chunk;
  int32_t n_types, n_chunks;
};

struct AtomLds {
  float x, y, z, nBl2e, occ;
  int type;
};

__global__ void __launch_bounds__(kSFThreads) k_sf_partial(SFParams p, const float* __restrict__ x, const float* __restrict__ y,
                                                           const float* __restrict__ z, const float* __restrict__ B,
                                                           const float* __restrict__ occ, const int32_t* __restrict__ type,
                                                           const float* __restrict__ ff, const int32_t* __restrict__ hkl,
                                                           float2* __restrict__ part) {
  __shared__ AtomLds at[kSFThreads];
  __shared__ float ftab[kMaxTypes][kSFThreads];
  const int64_t r = (int64_t)blockIdx.x * kSFThreads + threadIdx.x;
  const bool have = r < p.n_hkl;
  double h = 0, k = 0, l = 0;
  float s2 = 0.0f;
  if (have) {
    h = hkl[3 * r + 0];
    k = hkl[3 * r + 1];
    l = hkl[3 * r + 2];
    double D[3];
    for (int j = 0; j < 3; ++j) D[j] = (h * p.as[j] + k * p.as[3 + j]) + l * p.as[6 + j];
    double q = (D[0] * D[0] + D[1] * D[1]) + D[2] * D[2];
    double s2d = 0.25 * q;
    s2 = (float)s2d;
    for (int t = 0; t < p.n_types; ++t) {
      const float* c = ff + 9 * t;
      double f = c[8];
      for (int g = 0; g < 4; ++g) f += (double)c[g] * exp(-(double)c[4 + g] * s2d);
      ftab[t][threadIdx.x] = (float)f;
    }
  }
  const int64_t a0 = (int64_t)blockIdx.y * p.chunk;
  const int64_t a1 = a0 + p.chunk < p.n_atoms ? a0 + p.chunk : p.n_atoms;
  float re = 0.0f, im = 0.0f;
  const float log2e = 1.4426950408889634f;
  for (int64_t g0 = a0; g0 < a1; g0 += kSFThreads) {
    __syncthreads();
    int64_t j = g0 + threadIdx.x;
    if (j < a1) {
      int t = type[j];
      t = t < 0 ? 0 : (t >= p.n_types ? p.n_types - 1 : t);
      at[threadIdx.x] = {x[j], y[j], z[j], -B[j] * log2e, occ[j], t};
    }
    __syncthreads();
    const int cnt = (int)((a1 - g0) < kSFThreads ? (a1 - g0) : kSFThreads);
    if (have) {
      for (int i = 0; i < cnt; ++i) {
        const AtomLds a = at[i];
        double ph = fma(h, (double)a.x, fma(k, (double)a.y, l * (double)a.z));
        float frac = (float)(ph - floor(ph));
        float amp = a.occ * ftab[a.type][threadIdx.x] * __builtin_amdgcn_exp2f(a.nBl2e * s2);
        re = fmaf(amp, __builtin_amdgcn_cosf(frac), re);
        im = fmaf(amp, __builtin_amdgcn_sinf(frac), im);
      }
    }
  }
  if (have) part[(int64_t)blockIdx.y * p.n_hkl + r] = make_float2(re, im);
}

__global__ void k_sf_final(int64_t n_hkl, int32_t n_chunks, const float2* __restrict__ part, float* __restrict__ F,
                           float* __restrict__ F2) {
  int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n_hkl) return;
  double re = 0.0, im = 0.0;
  for (int c = 0; c < n_chunks; ++c) {
    float2 v = part[(int64_t)c * n_hkl + r];
    re += v.x;
    im += v.y;
  }
  if (F) {
    F[2 * r + 0] = (float)re;
    F[2 * r + 1] = (float)im;
  }
  if (F2) F2[r] = (float)(re * re + im * im);
}

// Batched models: block b of refl_blocks covers reflections [first, first + 256) of one
// model and loops over all of that model's atoms (binary64 accumulation, no partials).
__global__ void __launch_bounds__(kSFThreads) k_b_sf(const fdtbx_batch_entry* __restrict__ ent, const int64_t* __restrict__ blocks,
                                                     const float* __restrict__ x, const float* __restrict__ y,
                                                     const float* __restrict__ z, const float* __restrict__ B,
                                                     const float* __restrict__ occ, const int32_t* __restrict__ type,
                                                     const float* __restrict__ ff, const int32_t* __restrict__ hkl,
                                                     float* __restrict__ F, float* __restrict__ F2) {
  __shared__ AtomLds at[kSFThreads];
  __shared__ float ftab[kMaxTypes][kSFThreads];
  const int64_t item = blocks[blockIdx.x];
  const int m = (int)(item >> 40);
  const fdtbx_batch_entry& e = ent[m];
  const int64_t r = (item & ((1ll << 40) - 1)) + threadIdx.x;
  const bool have = r < e.n_hkl;
  const int64_t g = e.hkl_off + r;
  // fdtbx_batch_entries_check keeps n_types in 1..kMaxTypes; clamped here as well, so that the
  // LDS table is never indexed past its end
  const int n_types = e.n_types < 1 ? 1 : (e.n_types > kMaxTypes ? kMaxTypes : e.n_types);
  const float* ffm = ff + 9 * e.ff_off;
  double h = 0, k = 0, l = 0;
  float s2 = 0.0f;
  if (have) {
    h = hkl[3 * g + 0];
    k = hkl[3 * g + 1];
    l = hkl[3 * g + 2];
    double D[3];
    for (int j = 0; j < 3; ++j) D[j] = (h * e.frame[9 + j] + k * e.frame[12 + j]) + l * e.frame[15 + j];
    double q = (D[0] * D[0] + D[1] * D[1]) + D[2] * D[2];
    double s2d = 0.25 * q;
    s2 = (float)s2d;
    for (int t = 0; t < n_types; ++t) {
      const float* c = ffm + 9 * t;
      double f = c[8];
      for (int q2 = 0; q2 < 4; ++q2) f += (double)c[q2] * exp(-(double)c[4 + q2] * s2d);
      ftab[t][threadIdx.x] = (float)f;
    }
  }
  const int64_t a0 = e.atom_off, a1 = e.atom_off + e.n_atoms;
  double re = 0.0, im = 0.0;
  const float log2e = 1.4426950408889634f;
  for (int64_t g0 = a0; g0 < a1; g0 += kSFThreads) {
    __syncthreads();
    const int64_t j = g0 + threadIdx.x;
    if (j < a1) {
      int t = type[j];
      t = t < 0 ? 0 : (t >= n_types ? n_types - 1 : t);
      at[threadIdx.x] = {x[j], y[j], z[j], -B[j] * log2e, occ[j], t};
    }
    __syncthreads();
    const int cnt = (int)((a1 - g0) < kSFThreads ? (a1 - g0) : kSFThreads);
    if (have) {
      for (int i = 0; i < cnt; ++i) {
        const AtomLds a = at[i];
        double ph = fma(h, (double)a.x, fma(k, (double)a.y, l * (double)a.z));
        float frac = (float)(ph - floor(ph));
        float amp = a.occ * ftab[a.type][threadIdx.x] * __builtin_amdgcn_exp2f(a.nBl2e * s2);
        re = fma((double)amp, (double)__builtin_amdgcn_cosf(frac), re);
        im = fma((double)amp, (double)__builtin_amdgcn_sinf(frac), im);
      }
    }
  }
  if (have) {
    if (F) {
      F[2 * g + 0] = (float)re;
      F[2 * g + 1] = (float)im;
    }
    if (F2) F2[g] = (float)(re * re + im * im);
  }
}

int launch_batch_sf(const fdtbx_batch_entry* ent, const int64_t* blocks, int64_t n_rb, const float* x, const float* y,
                    const float* z, const float* B, const float* occ, const int32_t* type, const float* ff, const int32_t* hkl,
                    float* F, float* F2, hipStream_t s) {
  if (n_rb <= 0) return FDTBX_OK;
  hipLaunchKernelGGL(k_b_sf, dim3((unsigned)n_rb), dim3(kSFThreads), 0, s, ent, blocks, x, y, z, B, occ, type, ff, hkl, F, F2);
  FDTBX_LAUNCH_CHECK("batch structure factors");
  return FDTBX_OK;
}

static void sf_split(int64_t n_hkl, int64_t n_atoms, int32_t* n_chunks, int64_t* chunk) {
  int64_t nb = ceil_div(n_hkl, kSFThreads);
  int64_t want = ceil_div(4096, nb);                       // fill the chip with >= 4096 blocks
  int64_t need = ceil_div(n_atoms, kAtomsPerChunkMax);     // and keep float32 partial sums short
  int64_t nc = want > need ? want : need;
  int64_t maxc = ceil_div(n_atoms, 64);
  if (nc > maxc) nc = maxc;
  if (nc < 1) nc = 1;
  *chunk = ceil_div(n_atoms, nc);
  *n_chunks = (int32_t)ceil_div(n_atoms, *chunk);
}

}  // namespace fdtbx

using namespace fdtbx;

extern "C" size_t fdtbx_sf_workspace(int64_t n_hkl, int64_t n_atoms) {
  if (n_hkl <= 0 || n_atoms <= 0) return 0;
  int32_t nc;
  int64_t chunk;
  sf_split(n_hkl, n_atoms, &nc, &chunk);
  return (size_t)nc * n_hkl * sizeof(float2);
}

extern "C" int fdtbx_structure_factors(const fdtbx_cell* cell, int64_t n_atoms, const float* x, const float* y,
                                       const float* z, const float* B, const float* occ, const int32_t* type,
                                       const float* ff, int32_t n_types, const int32_t* hkl, int64_t n_hkl, float* F,
                                       float* F2, void* ws, size_t ws_bytes, void* stream) {
  if (!cell) return fail(FDTBX_ERR_INVALID_ARGUMENT, "null pointer");
  if (n_atoms < 0 || n_hkl < 0) return fail(FDTBX_ERR_INVALID_ARGUMENT, "n_atoms and n_hkl must be non-negative");
  if (n_hkl == 0) return FDTBX_OK;
  if (!F && !F2) return fail(FDTBX_ERR_INVALID_ARGUMENT, "F and F2 both NULL");
  if (n_atoms == 0) {  // no atoms: F = 0
    int r0 = fill(F, 2 * n_hkl, 0.0f, (hipStream_t)stream);
    if (r0) return r0;
    return fill(F2, n_hkl, 0.0f, (hipStream_t)stream);
  }
  if (!x || !y || !z || !B || !occ || !type || !ff || !hkl || !ws) return fail(FDTBX_ERR_INVALID_ARGUMENT, "null pointer");
  if (n_types < 1 || n_types > kMaxTypes) return fail(FDTBX_ERR_INVALID_ARGUMENT, "n_types must be in 1..16");
  if (n_hkl > (int64_t)0x7fffffff * kSFThreads) return fail(FDTBX_ERR_UNSUPPORTED, "too many reflections");
  int rc = check_cell(cell);
  if (rc) return rc;
  if (ws_bytes < fdtbx_sf_workspace(n_hkl, n_atoms)) return fail(FDTBX_ERR_BUFFER_TOO_SMALL, "sf workspace too small");
  SFParams p;
  {
    // reciprocal basis of the laboratory frame, the same construction as the exact unit
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
      p.as[j] = bxc[j] / V;
      p.as[3 + j] = cxa[j] / V;
      p.as[6 + j] = axb[j] / V;
    }
  }
  p.n_hkl = n_hkl;
  p.n_atoms = n_atoms;
  p.n_types = n_types;
  sf_split(n_hkl, n_atoms, &p.n_chunks, &p.chunk);
  hipStream_t s = (hipStream_t)stream;
  float2* part = (float2*)ws;
  dim3 grid((unsigned)ceil_div(n_hkl, kSFThreads), (unsigned)p.n_chunks);
  hipLaunchKernelGGL(k_sf_partial, grid, dim3(kSFThreads), 0, s, p, x, y, z, B, occ, type, ff, hkl, part);
  FDTBX_LAUNCH_CHECK("structure factors");
  hipLaunchKernelGGL(k_sf_final, dim3((unsigned)ceil_div(n_hkl, 256)), dim3(256), 0, s, n_hkl, p.n_chunks, part, F, F2);
  FDTBX_LAUNCH_CHECK("structure factor reduce");
  return FDTBX_OK;
}
