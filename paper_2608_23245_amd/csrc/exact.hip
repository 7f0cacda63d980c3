// Bit-reproducible binary64 steps: cell frame, reflection enumeration, pixel map
// and tile boxes, per-reflection records, per-tile culling lists.
//
// This translation unit is compiled with -ffp-contract=off: every expression is
// evaluated in IEEE binary64 with correctly rounded +, -, *, /, sqrt in the order
// written, so the integer results (reflection list, culling lists) do not depend
// on the compiler's choice of fused multiply-adds.  The float32 records for the
// profile kernels are derived here too (rounded once from binary64).
#include <hip/hip_runtime.h>

#include <math.h>

#include "frame.h"
#include "internal.h"

namespace fdtbx {

// ---------------------------------------------------------------- enumeration
struct EnumParams {
  Frame f;
  int32_t H, K, L;      // box half sizes
  int64_t n_cand;
  double t_hi, t_lo;    // thresholds on |D|^2; t_lo < 0 disables
  double ga, gb, gc, ext_limit;  // ext_limit <= 0 disables the extinction cull
};

static constexpr int kEnumThreads = 256;
static constexpr int kEnumPerThread = 4;
static constexpr int kEnumChunk = kEnumThreads * kEnumPerThread;

__device__ static inline bool enum_keep(const EnumParams& p, int64_t idx, int32_t* hkl) {
  int64_t nl = 2 * p.L + 1, nk = 2 * p.K + 1;
  int32_t l = (int32_t)(idx % nl) - p.L;
  int64_t r = idx / nl;
  int32_t k = (int32_t)(r % nk) - p.K;
  int32_t h = (int32_t)(r / nk) - p.H;
  hkl[0] = h;
  hkl[1] = k;
  hkl[2] = l;
  if (h == 0 && k == 0 && l == 0) return false;
  double D[3];
  recip(p.f, (double)h, (double)k, (double)l, D);
  double q = (D[0] * D[0] + D[1] * D[1]) + D[2] * D[2];
  if (!(q <= p.t_hi)) return false;
  if (p.t_lo >= 0.0 && !(q >= p.t_lo)) return false;
  if (p.ext_limit > 0.0 && extinction_arg(p.ga, p.gb, p.gc, h, k, l) > p.ext_limit) return false;
  return true;
}

// Exclusive scan over the block; *total gets the block sum.  blockDim.x is a multiple of 64.
__device__ static int64_t block_exclusive_scan(int64_t v, int64_t* lds, int64_t* total) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
  int64_t x = v;
  for (int o = 1; o < 64; o <<= 1) {
    int64_t y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  if (lane == 63) lds[wid] = x;
  __syncthreads();
  int64_t off = 0, tot = 0;
  for (int w = 0; w < nw; ++w) {
    int64_t s = lds[w];
    if (w < wid) off += s;
    tot += s;
  }
  __syncthreads();
  *total = tot;
  return off + x - v;
}

__global__ void __launch_bounds__(kEnumThreads) k_enum_count(EnumParams p, int64_t* block_counts) {
  __shared__ int64_t lds[kEnumThreads / 64];
  int64_t base = (int64_t)blockIdx.x * kEnumChunk + (int64_t)threadIdx.x * kEnumPerThread;
  int64_t c = 0;
  int32_t hkl[3];
  for (int i = 0; i < kEnumPerThread; ++i)
    if (base + i < p.n_cand && enum_keep(p, base + i, hkl)) ++c;
  int64_t tot;
  block_exclusive_scan(c, lds, &tot);
  if (threadIdx.x == 0) block_counts[blockIdx.x] = tot;
}

// Exclusive scan of n values in place with one block; writes the grand total to *total.
__global__ void __launch_bounds__(1024) k_scan_inplace(int64_t* v, int64_t n, int64_t* total) {
  __shared__ int64_t lds[16];
  __shared__ int64_t carry_s;
  if (threadIdx.x == 0) carry_s = 0;
  __syncthreads();
  for (int64_t b = 0; b < n; b += blockDim.x) {
    int64_t i = b + threadIdx.x;
    int64_t x = i < n ? v[i] : 0;
    int64_t tot;
    int64_t ex = block_exclusive_scan(x, lds, &tot);
    int64_t carry = carry_s;
    if (i < n) v[i] = carry + ex;
    __syncthreads();
    if (threadIdx.x == 0) carry_s = carry + tot;
    __syncthreads();
  }
  if (threadIdx.x == 0) *total = carry_s;
}

__global__ void __launch_bounds__(kEnumThreads) k_enum_fill(EnumParams p, const int64_t* block_offsets, int32_t* out) {
  __shared__ int64_t lds[kEnumThreads / 64];
  int64_t base = (int64_t)blockIdx.x * kEnumChunk + (int64_t)threadIdx.x * kEnumPerThread;
  int32_t hkl[kEnumPerThread][3];
  bool keep[kEnumPerThread];
  int64_t c = 0;
  for (int i = 0; i < kEnumPerThread; ++i) {
    keep[i] = base + i < p.n_cand && enum_keep(p, base + i, hkl[i]);
    c += keep[i];
  }
  int64_t tot;
  int64_t pos = block_offsets[blockIdx.x] + block_exclusive_scan(c, lds, &tot);
  for (int i = 0; i < kEnumPerThread; ++i)
    if (keep[i]) {
      out[3 * pos + 0] = hkl[i][0];
      out[3 * pos + 1] = hkl[i][1];
      out[3 * pos + 2] = hkl[i][2];
      ++pos;
    }
}

static void enum_box(const fdtbx_cell* cell, double d_min, int32_t* H, int32_t* K, int32_t* L) {
  *H = (int32_t)floor(cell->a / d_min) + 1;
  *K = (int32_t)floor(cell->b / d_min) + 1;
  *L = (int32_t)floor(cell->c / d_min) + 1;
}

}  // namespace fdtbx

using namespace fdtbx;

extern "C" int fdtbx_hkl_capacity(const fdtbx_cell* cell, double d_min, int64_t* cap) {
  if (!cell || !cap) return fail(FDTBX_ERR_INVALID_ARGUMENT, "null argument");
  int rc = check_cell(cell);
  if (rc) return rc;
  if (!finite_pos(d_min)) return fail(FDTBX_ERR_INVALID_ARGUMENT, "d_min must be positive and finite");
  if (cell->a / d_min > 4096 || cell->b / d_min > 4096 || cell->c / d_min > 4096)
    return fail(FDTBX_ERR_UNSUPPORTED, "index box larger than 4096 per axis");
  int32_t H, K, L;
  enum_box(cell, d_min, &H, &K, &L);
  *cap = (int64_t)(2 * H + 1) * (2 * K + 1) * (2 * L + 1);
  return FDTBX_OK;
}

extern "C" size_t fdtbx_enumerate_workspace(const fdtbx_cell* cell, double d_min) {
  int64_t cap = 0;
  if (fdtbx_hkl_capacity(cell, d_min, &cap)) return 0;
  return (size_t)(ceil_div(cap, kEnumChunk) + 1) * sizeof(int64_t);
}

extern "C" int fdtbx_enumerate_hkl(const fdtbx_cell* cell, double d_min, double d_max, const double* extinction,
                                   int32_t* hkl, int64_t cap, int64_t* n_out, void* ws, size_t ws_bytes,
                                   void* stream) {
  int64_t n_cand = 0;
  int rc = fdtbx_hkl_capacity(cell, d_min, &n_cand);
  if (rc) return rc;
  if (!hkl || !n_out || !ws) return fail(FDTBX_ERR_INVALID_ARGUMENT, "null pointer");
  if (isnan(d_max)) return fail(FDTBX_ERR_INVALID_ARGUMENT, "d_max is NaN");
  if (d_max > 0 && !(d_max > d_min)) return fail(FDTBX_ERR_INVALID_ARGUMENT, "d_max must exceed d_min");
  if (cap < n_cand) return fail(FDTBX_ERR_BUFFER_TOO_SMALL, "hkl capacity below fdtbx_hkl_capacity");
  if (ws_bytes < fdtbx_enumerate_workspace(cell, d_min)) return fail(FDTBX_ERR_BUFFER_TOO_SMALL, "workspace too small");
  EnumParams p;
  make_frame(*cell, &p.f);
  enum_box(cell, d_min, &p.H, &p.K, &p.L);
  p.n_cand = n_cand;
  p.t_hi = (1.0 / (d_min * d_min)) * (1.0 + 1e-9);
  p.t_lo = d_max > 0 ? (1.0 / (d_max * d_max)) * (1.0 - 1e-9) : -1.0;
  p.ga = p.gb = p.gc = 0.0;
  p.ext_limit = 0.0;
  if (extinction) {
    for (int i = 0; i < 4; ++i)
      if (!isfinite(extinction[i]) || extinction[i] < 0) return fail(FDTBX_ERR_INVALID_ARGUMENT, "bad extinction parameters");
    p.ga = extinction[0];
    p.gb = extinction[1];
    p.gc = extinction[2];
    p.ext_limit = extinction[3];
  }
  hipStream_t s = (hipStream_t)stream;
  int64_t nb = ceil_div(n_cand, kEnumChunk);
  int64_t* counts = (int64_t*)ws;
  hipLaunchKernelGGL(k_enum_count, dim3((unsigned)nb), dim3(kEnumThreads), 0, s, p, counts);
  FDTBX_LAUNCH_CHECK("enumerate count");
  hipLaunchKernelGGL(k_scan_inplace, dim3(1), dim3(1024), 0, s, counts, nb, n_out);
  FDTBX_LAUNCH_CHECK("enumerate scan");
  hipLaunchKernelGGL(k_enum_fill, dim3((unsigned)nb), dim3(kEnumThreads), 0, s, p, counts, hkl);
  FDTBX_LAUNCH_CHECK("enumerate fill");
  return FDTBX_OK;
}

namespace fdtbx {

// ---------------------------------------------------------------- pixel map (Eqs. laue, cyl-average)
struct PixParams {
  double lam, SF, p, cx, cy;
  double st, ct;  // sine and cosine of the fibre tilt
  double sd, cd;  // sine and cosine of the detector tilt
  int32_t W, H, tiles_x, tiles_y, tlg;
};

// Ewald point of pixel (i, j): y = ((i + 1/2) - c_x) p, z = ((j + 1/2) - c_y) p,
// r = |(SF, y, z)|, S = (-(y^2 + z^2)/(r (r + SF)), y/r, z/r)/lambda; cylindrical
// coordinates about the fibre axis n = (sin t, 0, cos t): Z = S.n and R = |S - Z n|,
// written with m = (cos t, 0, -sin t) as R = sqrt((S.m)^2 + S_y^2).
__device__ static inline void pixel_ewald(const PixParams& q, int i, int j, double* R, double* Z) {
  double y = (((double)i + 0.5) - q.cx) * q.p;
  double z = (((double)j + 0.5) - q.cy) * q.p;
  // the pixel's position X = (SF - z sin d, y, z cos d) on the (tilted) detector
  double Xx = q.SF - z * q.sd, Xz = z * q.cd;
  double r = sqrt((Xx * Xx + y * y) + Xz * Xz);
  double Sx = -(y * y + Xz * Xz) / ((r * (r + Xx)) * q.lam);
  double Sy = y / (r * q.lam);
  double Sz = Xz / (r * q.lam);
  double Sm = Sx * q.ct - Sz * q.st;
  *R = sqrt(Sm * Sm + Sy * Sy);
  *Z = Sx * q.st + Sz * q.ct;
}

// One 64-lane wave per tile of 2^tlg x 64 >> tlg pixels: pixel values and the tile's box.
__global__ void __launch_bounds__(64) k_pixel_map(PixParams q, double* pix, double* tile) {
  const int t = blockIdx.x;
  const int tx = t % q.tiles_x, ty = t / q.tiles_x;
  const int i = (tx << q.tlg) + (threadIdx.x & ((1 << q.tlg) - 1));
  const int j = ty * (64 >> q.tlg) + (threadIdx.x >> q.tlg);
  const bool in = i < q.W && j < q.H;
  double R = 0, Z = 0, P2 = 0;
  if (in) {
    pixel_ewald(q, i, j, &R, &Z);
    P2 = R * R + Z * Z;
    pix[2 * ((int64_t)j * q.W + i) + 0] = R;
    pix[2 * ((int64_t)j * q.W + i) + 1] = Z;
  }
  double v[6] = {in ? R : INFINITY, in ? -R : INFINITY, in ? Z : INFINITY, in ? -Z : INFINITY,
                 in ? P2 : INFINITY, in ? -P2 : INFINITY};
  for (int o = 32; o >= 1; o >>= 1)
    for (int c = 0; c < 6; ++c) v[c] = fmin(v[c], __shfl_xor(v[c], o, 64));
  if (threadIdx.x == 0) {
    double* b = tile + 8 * (int64_t)t;
    b[0] = v[0];
    b[1] = -v[1];
    b[2] = v[2];
    b[3] = -v[3];
    b[4] = v[4];
    b[5] = -v[5];
    b[6] = 0.0;
    b[7] = 0.0;
  }
}

// ---------------------------------------------------------------- per-reflection records
struct PrepParams {
  Frame f;
  double Nb[3], g[3];
  double Bax[3];     // axis damping B_i
  double T, cmin, m, ext_limit;
  int32_t intensity_model, lineshape;
  int64_t n;
};


// Culling record (see the header): conservative reach of the reflection's profile in (R, Z).
// Nodes s = r0 c (S + d1 e1 + d2 e2), |d_j| <= T, c in [cmin, 1]; query points lie in
// the support box of a node, whose extent along v is sum_i w_i |a*_i.v| with w_i = 1/2
// (Hosemann lineshape) or w_i = m/N_i, 1/N_i <= 1/N_base,i + min(pi^2 g_i^2 h_i^2, 1).
__device__ static void cull_record(const PrepParams& p, const double* hh, const ReflFrame& F, double* C) {
  const double* S = F.S;
  const double* e1 = F.e1;
  const double* e2 = F.e2;
  const double* ep = F.ep;
  const double r0 = F.r0;
  const double ez[3] = {0.0, 0.0, 1.0};
  double mN[3];
  support_bounds(p.lineshape, p.m, p.Nb, p.g, hh, mN);
  auto ext = [&](const double* v) {
    double e = (mN[0] * fabs(dotv(&p.f.s[0], v)));
    e = e + mN[1] * fabs(dotv(&p.f.s[3], v));
    e = e + mN[2] * fabs(dotv(&p.f.s[6], v));
    return e;
  };
  auto span = [&](const double* v, double* lo_out, double* hi_out) {
    double l0 = dotv(S, v), l1 = dotv(e1, v), l2 = dotv(e2, v);
    double spread = p.T * (fabs(l1) + fabs(l2));
    double lo = l0 - spread, hi = l0 + spread;
    double s_lo = r0 * fmin(p.cmin * lo, lo);
    double s_hi = r0 * fmax(p.cmin * hi, hi);
    double e = ext(v);
    *lo_out = s_lo - e;
    *hi_out = s_hi + e;
  };
  double Rlo, Rhi, Zlo, Zhi;
  span(ep, &Rlo, &Rhi);
  span(ez, &Zlo, &Zhi);
  double rho_all = (mN[0] * sqrt(dotv(&p.f.s[0], &p.f.s[0])));
  rho_all = rho_all + mN[1] * sqrt(dotv(&p.f.s[3], &p.f.s[3]));
  rho_all = rho_all + mN[2] * sqrt(dotv(&p.f.s[6], &p.f.s[6]));
  double a_lo = r0 - rho_all, a_hi = r0 + rho_all;
  C[0] = Rlo;
  C[1] = Rhi;
  C[2] = Zlo;
  C[3] = Zhi;
  C[4] = a_lo > 0.0 ? a_lo * a_lo : 0.0;
  C[5] = a_hi * a_hi;
  if (!F.merid) {
    // wedge spanned in the (R, Z) plane by the in-plane node directions S + d2 e2, |d2| <= T
    double SR = dotv(S, ep), SZ = S[2], e2R = dotv(e2, ep), e2Z = e2[2];
    double vmR = SR - p.T * e2R, vmZ = SZ - p.T * e2Z;
    double vpR = SR + p.T * e2R, vpZ = SZ + p.T * e2Z;
    double n1R = -vmZ, n1Z = vmR;
    if (n1R * vpR + n1Z * vpZ < 0.0) {
      n1R = -n1R;
      n1Z = -n1Z;
    }
    double n2R = -vpZ, n2Z = vpR;
    if (n2R * vmR + n2Z * vmZ < 0.0) {
      n2R = -n2R;
      n2Z = -n2Z;
    }
    double v1[3] = {n1R * ep[0], n1R * ep[1], n1R * ep[2] + n1Z};
    double v2[3] = {n2R * ep[0], n2R * ep[1], n2R * ep[2] + n2Z};
    C[6] = n1R;
    C[7] = n1Z;
    C[8] = ext(v1);
    C[9] = n2R;
    C[10] = n2Z;
    C[11] = ext(v2);
  } else {
    C[6] = C[7] = C[9] = C[10] = 0.0;
    C[8] = C[11] = -1.0;
  }
  bool alive = !(p.ext_limit > 0.0 && extinction_arg(p.g[0], p.g[1], p.g[2], hh[0], hh[1], hh[2]) > p.ext_limit);
  C[12] = alive ? 1.0 : 0.0;
  C[13] = C[14] = C[15] = 0.0;
}

// Profile record (float32, from binary64 values; layout of ReflSlot).
__device__ static void profile_record(const PrepParams& p, const double* hh, const ReflFrame& F, double f2, float* o) {
  const double* S = F.S;
  const double* e1 = F.e1;
  const double* e2 = F.e2;
  const double* ep = F.ep;
  const double* D = F.D;
  const double r0 = F.r0;
  double A[3], N[3], Ip = 1.0, Dx = 0.0;
  for (int i = 0; i < 3; ++i) {
    A[i] = exp(-2.0 * kPi2 * (p.g[i] * p.g[i]) * (hh[i] * hh[i]));
    N[i] = 1.0 / (1.0 / p.Nb[i] + (1.0 - A[i]) / (1.0 + A[i]));
    if (p.intensity_model) Ip *= 2.0 * A[i] / (1.0 + A[i] * A[i]);
    // axis damping: S.a_i/|a_i| = h_i/|a_i| at S = D_hkl
    const double* ai = &p.f.a[3 * i];
    Dx += p.Bax[i] * (hh[i] * hh[i]) / dotv(ai, ai);
  }
  double W = f2 * Ip * exp(-0.25 * Dx);
  // lineshape: per-reflection constant C and per-axis scale of y (see lineshape_half)
  double C = 1.0, sc[3], AH[3] = {0.0, 0.0, 0.0};
  for (int i = 0; i < 3; ++i) {
    if (p.lineshape == FDTBX_LINESHAPE_HOSEMANN) {
      AH[i] = N[i] > 1.0 ? (N[i] - 1.0) / (N[i] + 1.0) : 0.0;
      C *= 1.0 - AH[i] * AH[i];
      sc[i] = 1.0;
    } else {
      C *= p.lineshape == FDTBX_LINESHAPE_GAUSSIAN ? N[i] : N[i] / (4.0 * kPi2);
      sc[i] = 0.5 * N[i];
    }
  }
  o[RS_W] = (float)W;
  for (int i = 0; i < 3; ++i) o[RS_N + i] = (float)N[i];
  o[RS_R0] = (float)r0;
  o[RS_WK] = (float)(W * r0 * r0 * C);
  o[RS_K] = (float)(r0 * r0 * C);
  for (int i = 0; i < 3; ++i) {
    const double* ai = &p.f.a[3 * i];
    o[RS_B + i] = (float)(sc[i] * r0 * dotv(ai, S));
    o[RS_G1 + i] = (float)(sc[i] * r0 * dotv(ai, e1));
    o[RS_G2 + i] = (float)(sc[i] * r0 * dotv(ai, e2));
    o[RS_TR + i] = (float)(sc[i] * dotv(ai, ep));
    o[RS_TZ + i] = (float)(sc[i] * ai[2]);
  }
  o[RS_IP] = (float)Ip;
  double RDp = dotv(D, ep), ZD = D[2];
  *(double*)(o + RS_RD) = RDp;
  *(double*)(o + RS_ZD) = ZD;
  o[RS_CS + 0] = (float)dotv(ep, S);
  o[RS_CS + 1] = (float)S[2];
  o[RS_C1 + 0] = (float)dotv(ep, e1);
  o[RS_C1 + 1] = (float)e1[2];
  o[RS_C2 + 0] = (float)dotv(ep, e2);
  o[RS_C2 + 1] = (float)e2[2];
  const double* vs[3] = {S, e1, e2};
  for (int v = 0; v < 3; ++v) {
    double e = 0.0;
    for (int i = 0; i < 3; ++i) {
      const double w = p.lineshape == FDTBX_LINESHAPE_HOSEMANN ? 0.5 : p.m / N[i];
      e = e + w * fabs(dotv(&p.f.s[3 * i], vs[v]));
    }
    o[RS_RHO + v] = (float)e;
  }
  for (int i = 0; i < 3; ++i) {
    // ring direction at the reflection's azimuth, for query points off that azimuth
    const double az[3] = {-ep[1], ep[0], 0.0};
    const double* vv[3] = {S, e1, e2};
    o[RS_AZ + i] = (float)dotv(az, vv[i]);
    o[RS_TA + i] = (float)(sc[i] * dotv(&p.f.a[3 * i], az));
  }
  o[RS_F2] = (float)f2;
  for (int i = 0; i < 3; ++i) o[RS_AH + i] = (float)AH[i];
  for (int i = 0; i < 3; ++i) {
    const double* ai = &p.f.a[3 * i];
    const double x[5] = {sc[i] * r0 * dotv(ai, S), sc[i] * r0 * dotv(ai, e1), sc[i] * r0 * dotv(ai, e2),
                         sc[i] * dotv(ai, ep), sc[i] * ai[2]};
    for (int c = 0; c < 5; ++c) o[RS_LO + 3 * c + i] = (float)(x[c] - (double)o[RS_B + 3 * c + i]);
    const double az[3] = {-ep[1], ep[0], 0.0};
    o[RS_LO_TA + i] = (float)(sc[i] * dotv(ai, az) - (double)o[RS_TA + i]);
  }
}

__global__ void __launch_bounds__(256) k_prep(PrepParams p, const int32_t* __restrict__ hkl, const float* __restrict__ F2,
                                              float* __restrict__ refl, double* __restrict__ cull) {
  int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= p.n) return;
  const double hh[3] = {(double)hkl[3 * r + 0], (double)hkl[3 * r + 1], (double)hkl[3 * r + 2]};
  ReflFrame F;
  refl_frame(p.f, hh, &F);
  cull_record(p, hh, F, cull + FDTBX_CULL_DOUBLES * r);
  profile_record(p, hh, F, (double)F2[r], refl + (int64_t)FDTBX_REFL_FLOATS * r);
}

// Culling record for the cylindrical average (layout of the culling record): the ball of
// radius rho_B = 2 r0 sqrt((1 - cmin)/2) + rho about D holds every point a ring point at any
// azimuth can reach (nodes within arccos(cmin) of S, support corner radius rho), so
// |R - R_D| <= rho_B, |Z - Z_D| <= rho_B and | |p| - r0 | <= rho; the wedge is disabled.
__global__ void __launch_bounds__(256) k_cyl_records(PrepParams p, const int32_t* __restrict__ hkl, double* __restrict__ cull) {
  int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= p.n) return;
  const double hh[3] = {(double)hkl[3 * r + 0], (double)hkl[3 * r + 1], (double)hkl[3 * r + 2]};
  double D[3];
  recip(p.f, hh[0], hh[1], hh[2], D);
  const double r0 = sqrt((D[0] * D[0] + D[1] * D[1]) + D[2] * D[2]);
  const double RD = sqrt(D[0] * D[0] + D[1] * D[1]);
  double w[3];
  support_bounds(p.lineshape, p.m, p.Nb, p.g, hh, w);
  double rho = w[0] * sqrt(dotv(&p.f.s[0], &p.f.s[0]));
  rho = rho + w[1] * sqrt(dotv(&p.f.s[3], &p.f.s[3]));
  rho = rho + w[2] * sqrt(dotv(&p.f.s[6], &p.f.s[6]));
  const double rB = (2.0 * r0) * sqrt((1.0 - p.cmin) / 2.0) + rho;
  double* C = cull + FDTBX_CULL_DOUBLES * r;
  C[0] = RD - rB;
  C[1] = RD + rB;
  C[2] = D[2] - rB;
  C[3] = D[2] + rB;
  const double a_lo = r0 - rho, a_hi = r0 + rho;
  C[4] = a_lo > 0.0 ? a_lo * a_lo : 0.0;
  C[5] = a_hi * a_hi;
  C[6] = C[7] = C[9] = C[10] = 0.0;
  C[8] = C[11] = -1.0;
  const bool alive = !(p.ext_limit > 0.0 && extinction_arg(p.g[0], p.g[1], p.g[2], hh[0], hh[1], hh[2]) > p.ext_limit);
  C[12] = alive ? 1.0 : 0.0;
  C[13] = C[14] = C[15] = 0.0;
}

// Batched models: block b of refl_blocks covers reflections [first, first + 256) of one model.
__device__ static void prep_params_of(const fdtbx_batch_entry& e, PrepParams* p) {
  for (int k = 0; k < 9; ++k) {
    p->f.a[k] = e.frame[k];
    p->f.s[k] = e.frame[9 + k];
  }
  p->f.V = e.frame[18];
  for (int i = 0; i < 3; ++i) {
    p->Nb[i] = e.model.dis.N_base[i];
    p->g[i] = e.model.dis.g[i];
  }
  p->T = e.model.quad.T;
  p->cmin = 1.0 / sqrt(1.0 + 2.0 * p->T * p->T);
  p->m = (double)e.model.quad.m;
  p->ext_limit = e.model.quad.extinction;
  p->intensity_model = e.model.dis.intensity_model;
  p->lineshape = e.model.dis.lineshape;
  for (int i = 0; i < 3; ++i) p->Bax[i] = e.model.dis.B_axis[i];
  p->n = e.n_hkl;
}

__global__ void __launch_bounds__(256) k_b_prep(const fdtbx_batch_entry* __restrict__ ent, const int64_t* __restrict__ blocks,
                                                const int32_t* __restrict__ hkl, const float* __restrict__ F2,
                                                float* __restrict__ refl) {
  const int64_t item = blocks[blockIdx.x];
  const int m = (int)(item >> 40);
  const int64_t r = (item & ((1ll << 40) - 1)) + threadIdx.x;
  const fdtbx_batch_entry& e = ent[m];
  if (r >= e.n_hkl) return;
  PrepParams p;
  prep_params_of(e, &p);
  const int64_t g = e.hkl_off + r;
  const double hh[3] = {(double)hkl[3 * g + 0], (double)hkl[3 * g + 1], (double)hkl[3 * g + 2]};
  ReflFrame F;
  refl_frame(p.f, hh, &F);
  profile_record(p, hh, F, (double)F2[g], refl + (int64_t)FDTBX_REFL_FLOATS * g);
}

// ---------------------------------------------------------------- culling
// Superblocks of kSB x kSB tiles prefilter the reflections with the same (monotone)
// predicate on the union box; the per-tile test then runs only over the superblock's
// candidates and writes the exact per-tile lists in ascending order.
static constexpr int kSB = 4;

// lcols, lrows: tile columns and rows that get lists (all, or the left or top half under the
// mirror folds, the other tiles keeping empty lists: no launch reads them).
struct CullParams {
  int32_t tiles_x, tiles_y, sb_x, sb_y, lcols, lrows;
  int64_t n_hkl, n_words;
};

// The exact predicate of the header.  box = tile box (8 doubles), c = culling record.
__device__ static inline bool cull_test(const double* box, const double* c) {
  if (!(c[12] != 0.0)) return false;
  if (!(c[0] <= box[1] && box[0] <= c[1])) return false;
  if (!(c[2] <= box[3] && box[2] <= c[3])) return false;
  if (!(c[4] <= box[5] && box[4] <= c[5])) return false;
  if (c[8] >= 0.0) {
    double m1 = fmax(c[6] * box[0], c[6] * box[1]) + fmax(c[7] * box[2], c[7] * box[3]);
    if (!(m1 >= -c[8])) return false;
    double m2 = fmax(c[9] * box[0], c[9] * box[1]) + fmax(c[10] * box[2], c[10] * box[3]);
    if (!(m2 >= -c[11])) return false;
  }
  return true;
}

// Superblock boxes: union of the boxes of its tiles.
__global__ void k_sb_boxes(CullParams q, const double* __restrict__ tile, double* __restrict__ sb) {
  int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= q.sb_x * q.sb_y) return;
  int sx = s % q.sb_x, sy = s / q.sb_x;
  double b[6] = {INFINITY, -INFINITY, INFINITY, -INFINITY, INFINITY, -INFINITY};
  for (int dy = 0; dy < kSB; ++dy)
    for (int dx = 0; dx < kSB; ++dx) {
      int tx = sx * kSB + dx, ty = sy * kSB + dy;
      if (tx >= q.tiles_x || ty >= q.tiles_y) continue;
      const double* t = tile + 8 * ((int64_t)ty * q.tiles_x + tx);
      for (int c = 0; c < 6; c += 2) {
        b[c] = fmin(b[c], t[c]);
        b[c + 1] = fmax(b[c + 1], t[c + 1]);
      }
    }
  for (int c = 0; c < 6; ++c) sb[8 * (int64_t)s + c] = b[c];
  sb[8 * (int64_t)s + 6] = 0.0;
  sb[8 * (int64_t)s + 7] = 0.0;
}

// One wave per 64 reflections; loops over all superblocks and writes one mask word each.
__global__ void __launch_bounds__(64) k_sb_mask(CullParams q, const double* __restrict__ sb, const double* __restrict__ cull,
                                                uint64_t* __restrict__ mask) {
  int64_t w = blockIdx.x;
  int64_t r = w * 64 + threadIdx.x;
  double c[13];
  bool have = r < q.n_hkl;
  for (int k = 0; k < 13; ++k) c[k] = have ? cull[FDTBX_CULL_DOUBLES * r + k] : 0.0;
  const int nsb = q.sb_x * q.sb_y;
  for (int s = 0; s < nsb; ++s) {
    if ((s % q.sb_x) * kSB >= q.lcols || (s / q.sb_x) * kSB >= q.lrows) continue;  // no tile of it gets a list
    double box[6];
    for (int k = 0; k < 6; ++k) box[k] = sb[8 * (int64_t)s + k];
    bool hit = have && cull_test(box, c);
    uint64_t m = __ballot(hit);
    if (threadIdx.x == 0) mask[(int64_t)s * q.n_words + w] = m;
  }
}

// One block per superblock of kSB x kSB tiles, mode 0: count; mode 1: fill.  The block's
// waves split the superblock's candidate mask into kTB contiguous word ranges.  Each wave
// compacts the set bits of kWordsPer words at a time into an LDS list of reflection indices
// (ascending: words in order, bits in order within a word), reads each listed candidate's
// record once and tests it against every tile box of the superblock.  Mode 0 stores the hits
// of every (wave, tile) in part and, after a block barrier, each tile's total in counts; mode
// 1 (counts holding the exclusive offsets) writes the hits of wave w for tile t at t's offset
// plus the hits of the waves before w, so every list comes out ascending.  Tiles off the
// detector or in a column the mirror fold does not launch get no list (NaN boxes fail every
// test; their count is 0), and so do the rows the up-down fold does not launch.
static constexpr int kWordsPer = 16;
static constexpr int kTB = kSB * kSB;  // tiles and waves per block

// MODE 1 (fill) returns at once when *total exceeds cap: the lists do not fit (the launch
// that culls without a host round trip leaves the decision to the device).
template <int MODE>
__global__ void __launch_bounds__(64 * kTB) k_tile_lists(CullParams q, const double* __restrict__ tile,
                                                         const uint64_t* __restrict__ mask, const double* __restrict__ cull,
                                                         int64_t* __restrict__ counts, int32_t* __restrict__ part,
                                                         int32_t* __restrict__ idx, const int64_t* __restrict__ total,
                                                         int64_t cap) {
  __shared__ int32_t cand_all[kTB][kWordsPer * 64];
  __shared__ double boxes[kTB][6];
  __shared__ int32_t hits[kTB][kTB];  // [wave][tile]
  if (MODE && *total > cap) return;  // uniform across the grid
  const int s = blockIdx.x;
  const int sx = s % q.sb_x, sy = s / q.sb_x;
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  if (threadIdx.x < kTB * 6) {
    const int u = threadIdx.x / 6, c = threadIdx.x % 6;
    const int tx = sx * kSB + u % kSB, ty = sy * kSB + u / kSB;
    boxes[u][c] = (tx < q.lcols && ty < q.lrows) ? tile[8 * ((int64_t)ty * q.tiles_x + tx) + c] : (double)NAN;
  }
  __syncthreads();
  int cnt[kTB];
  int64_t pos[kTB];
#pragma unroll
  for (int u = 0; u < kTB; ++u) {
    cnt[u] = 0;
    pos[u] = 0;
    if (MODE) {
      const int tx = sx * kSB + u % kSB, ty = sy * kSB + u / kSB;
      if (tx < q.lcols && ty < q.lrows) {
        pos[u] = counts[(int64_t)ty * q.tiles_x + tx];
        for (int w = 0; w < wv; ++w) pos[u] += part[((int64_t)s * kTB + w) * kTB + u];
      }
    }
  }
  // superblocks wholly right of the launched columns or below the launched rows have no mask row
  if (sx * kSB < q.lcols && sy * kSB < q.lrows) {
    const int64_t per = (q.n_words + kTB - 1) / kTB;
    const int64_t wlo = per * wv, whi = wlo + per < q.n_words ? wlo + per : q.n_words;
    const uint64_t* mrow = mask + (int64_t)s * q.n_words;
    int32_t* const cand = cand_all[wv];
    for (int64_t w0 = wlo; w0 < whi; w0 += kWordsPer) {
      const uint64_t myword = (lane < kWordsPer && w0 + lane < whi) ? mrow[w0 + lane] : 0ull;
      const int c = __popcll(myword);
      int pre = c;  // inclusive prefix of the set-bit counts over the word lanes
      for (int o = 1; o < kWordsPer; o <<= 1) {
        const int v = __shfl_up(pre, o, 64);
        if (lane >= o) pre += v;
      }
      const int total = __shfl(pre, kWordsPer - 1, 64);
      if (total == 0) continue;  // uniform
      int at = pre - c;
      uint64_t m = myword;
      while (m) {
        cand[at++] = (int32_t)((w0 + lane) * 64 + __builtin_ctzll(m));
        m &= m - 1;
      }
      wave_sync();
      for (int k0 = 0; k0 < total; k0 += 64) {
        const bool have = k0 + lane < total;
        int32_t r = 0;
        double cr[13];
        for (int k = 0; k < 13; ++k) cr[k] = 0.0;
        if (have) {
          r = cand[k0 + lane];
          for (int k = 0; k < 13; ++k) cr[k] = cull[FDTBX_CULL_DOUBLES * (int64_t)r + k];
        }
#pragma unroll
        for (int u = 0; u < kTB; ++u) {
          const bool hit = have && cull_test(boxes[u], cr);
          const uint64_t hm = __ballot(hit);
          if (MODE) {
            if (hit) {
              const uint64_t below = lane ? (hm & ((~0ull) >> (64 - lane))) : 0ull;
              idx[pos[u] + __popcll(below)] = r;
            }
            pos[u] += __popcll(hm);
          } else {
            cnt[u] += __popcll(hm);
          }
        }
      }
      wave_sync();  // the list is rewritten by the next words
    }
  }
  if (!MODE) {
    if (lane == 0) {
#pragma unroll
      for (int u = 0; u < kTB; ++u) {
        hits[wv][u] = cnt[u];
        part[((int64_t)s * kTB + wv) * kTB + u] = cnt[u];
      }
    }
    __syncthreads();
    if (threadIdx.x < kTB) {
      const int u = threadIdx.x;
      const int tx = sx * kSB + u % kSB, ty = sy * kSB + u / kSB;
      if (tx < q.tiles_x && ty < q.tiles_y) {
        int64_t sum = 0;
        for (int w = 0; w < kTB; ++w) sum += hits[w][u];
        counts[(int64_t)ty * q.tiles_x + tx] = sum;  // 0 for tiles without lists
      }
    }
  }
}

}  // namespace fdtbx

using namespace fdtbx;

static void pix_params(const fdtbx_geometry* g, PixParams* q) {
  q->lam = g->wavelength;
  q->SF = g->distance;
  q->p = g->pixel;
  q->cx = g->center_x;
  q->cy = g->center_y;
  q->st = sin(g->tilt);
  q->ct = cos(g->tilt);
  q->sd = sin(g->det_tilt);
  q->cd = cos(g->det_tilt);
  q->W = g->width;
  q->H = g->height;
  q->tiles_x = tiles_x_of(g);
  q->tiles_y = tiles_y_of(g);
  q->tlg = tile_lg(g);
}

extern "C" int fdtbx_pixel_map(const fdtbx_geometry* geom, double* pix, double* tile, void* stream) {
  if (!geom || !pix || !tile) return fail(FDTBX_ERR_INVALID_ARGUMENT, "null pointer");
  int rc = check_geometry(geom);
  if (rc) return rc;
  PixParams q;
  pix_params(geom, &q);
  int64_t n_tiles = (int64_t)q.tiles_x * q.tiles_y;
  hipLaunchKernelGGL(k_pixel_map, dim3((unsigned)n_tiles), dim3(64), 0, (hipStream_t)stream, q, pix, tile);
  FDTBX_LAUNCH_CHECK("pixel map");
  return FDTBX_OK;
}

extern "C" int fdtbx_reflection_prep(const fdtbx_model* model, const int32_t* hkl, int64_t n_hkl, const float* F2,
                                     float* refl, double* cull, void* stream) {
  if (!model) return fail(FDTBX_ERR_INVALID_ARGUMENT, "null pointer");
  if (n_hkl < 0) return fail(FDTBX_ERR_INVALID_ARGUMENT, "n_hkl must be non-negative");
  int rc = check_model(model);
  if (rc) return rc;
  if (n_hkl == 0) return FDTBX_OK;
  if (!hkl || !F2 || !refl || !cull) return fail(FDTBX_ERR_INVALID_ARGUMENT, "null pointer");
  PrepParams p;
  make_frame(model->cell, &p.f);
  for (int i = 0; i < 3; ++i) {
    p.Nb[i] = model->dis.N_base[i];
    p.g[i] = model->dis.g[i];
  }
  p.T = model->quad.T;
  p.cmin = 1.0 / sqrt(1.0 + 2.0 * p.T * p.T);
  p.m = (double)model->quad.m;
  p.ext_limit = model->quad.extinction;
  p.intensity_model = model->dis.intensity_model;
  p.lineshape = model->dis.lineshape;
  for (int i = 0; i < 3; ++i) p.Bax[i] = model->dis.B_axis[i];
  p.n = n_hkl;
  hipLaunchKernelGGL(k_prep, dim3((unsigned)ceil_div(n_hkl, 256)), dim3(256), 0, (hipStream_t)stream, p, hkl, F2, refl,
                     cull);
  FDTBX_LAUNCH_CHECK("reflection prep");
  return FDTBX_OK;
}

extern "C" int fdtbx_cyl_records(const fdtbx_model* model, const int32_t* hkl, int64_t n_hkl, double* cull, void* stream) {
  if (!model) return fail(FDTBX_ERR_INVALID_ARGUMENT, "null pointer");
  if (n_hkl < 0) return fail(FDTBX_ERR_INVALID_ARGUMENT, "n_hkl must be non-negative");
  int rc = check_model(model);
  if (rc) return rc;
  if (n_hkl == 0) return FDTBX_OK;
  if (!hkl || !cull) return fail(FDTBX_ERR_INVALID_ARGUMENT, "null pointer");
  PrepParams p;
  make_frame(model->cell, &p.f);
  for (int i = 0; i < 3; ++i) {
    p.Nb[i] = model->dis.N_base[i];
    p.g[i] = model->dis.g[i];
  }
  p.T = model->quad.T;
  p.cmin = 1.0 / sqrt(1.0 + 2.0 * p.T * p.T);
  p.m = (double)model->quad.m;
  p.ext_limit = model->quad.extinction;
  p.lineshape = model->dis.lineshape;
  p.n = n_hkl;
  hipLaunchKernelGGL(k_cyl_records, dim3((unsigned)ceil_div(n_hkl, 256)), dim3(256), 0, (hipStream_t)stream, p, hkl, cull);
  FDTBX_LAUNCH_CHECK("cylindrical culling records");
  return FDTBX_OK;
}

static void cull_params(const fdtbx_geometry* g, int64_t n_hkl, CullParams* q) {
  q->tiles_x = tiles_x_of(g);
  q->tiles_y = tiles_y_of(g);
  q->lcols = lcols_of(g);
  q->lrows = lrows_of(g);
  q->sb_x = (int32_t)ceil_div(q->tiles_x, kSB);
  q->sb_y = (int32_t)ceil_div(q->tiles_y, kSB);
  q->n_hkl = n_hkl;
  q->n_words = ceil_div(n_hkl, 64);
}

// Workspace: superblock boxes | masks | tile counts scratch.
static size_t cull_workspace_of(const CullParams& q) {
  int64_t nsb = (int64_t)q.sb_x * q.sb_y;
  size_t b = align_up((size_t)nsb * 8 * sizeof(double), 256);
  b += align_up((size_t)nsb * q.n_words * sizeof(uint64_t), 256);
  b += align_up(sizeof(int64_t) * 2, 256);
  b += align_up((size_t)nsb * kTB * kTB * sizeof(int32_t), 256);
  return b;
}

extern "C" size_t fdtbx_cull_workspace(const fdtbx_geometry* geom, int64_t n_hkl) {
  if (!geom || check_geometry(geom) || n_hkl <= 0) return 0;
  CullParams q;
  cull_params(geom, n_hkl, &q);
  return cull_workspace_of(q);
}

// The lists of the tile grid q (boxes in tile, row-major), as fdtbx_cull describes them.
static int cull_lists(const CullParams& q, const double* tile, const double* cull, int64_t* offsets, int32_t* idx,
                      int64_t cap, int64_t* n_pairs, void* ws, size_t ws_bytes, hipStream_t s) {
  if (!cull || !ws) return fail(FDTBX_ERR_INVALID_ARGUMENT, "null pointer");
  if (ws_bytes < cull_workspace_of(q)) return fail(FDTBX_ERR_BUFFER_TOO_SMALL, "cull workspace too small");
  int64_t nsb = (int64_t)q.sb_x * q.sb_y;
  int64_t n_tiles = (int64_t)q.tiles_x * q.tiles_y;
  char* w = (char*)ws;
  double* sb = (double*)w;
  w += align_up((size_t)nsb * 8 * sizeof(double), 256);
  uint64_t* mask = (uint64_t*)w;
  w += align_up((size_t)nsb * q.n_words * sizeof(uint64_t), 256);
  int64_t* total = (int64_t*)w;
  w += align_up(sizeof(int64_t) * 2, 256);
  int32_t* part = (int32_t*)w;
  hipLaunchKernelGGL(k_sb_boxes, dim3((unsigned)ceil_div(nsb, 256)), dim3(256), 0, s, q, tile, sb);
  FDTBX_LAUNCH_CHECK("cull superblocks");
  hipLaunchKernelGGL(k_sb_mask, dim3((unsigned)q.n_words), dim3(64), 0, s, q, sb, cull, mask);
  FDTBX_LAUNCH_CHECK("cull masks");
  hipLaunchKernelGGL(k_tile_lists<0>, dim3((unsigned)nsb), dim3(64 * kTB), 0, s, q, tile, mask, cull, offsets, part,
                     (int32_t*)nullptr, (const int64_t*)nullptr, (int64_t)0);
  FDTBX_LAUNCH_CHECK("cull count");
  hipLaunchKernelGGL(k_scan_inplace, dim3(1), dim3(1024), 0, s, offsets, n_tiles, total);
  FDTBX_LAUNCH_CHECK("cull scan");
  int64_t h_total = 0;
  FDTBX_HIP(hipMemcpyAsync(&h_total, total, sizeof(int64_t), hipMemcpyDeviceToHost, s));
  FDTBX_HIP(hipStreamSynchronize(s));
  *n_pairs = h_total;
  FDTBX_HIP(hipMemcpyAsync(offsets + n_tiles, total, sizeof(int64_t), hipMemcpyDeviceToDevice, s));
  if (h_total > cap || (h_total > 0 && !idx)) return fail(FDTBX_ERR_BUFFER_TOO_SMALL, "culling pair capacity too small");
  if (h_total > 0) {
    hipLaunchKernelGGL(k_tile_lists<1>, dim3((unsigned)nsb), dim3(64 * kTB), 0, s, q, tile, mask, cull, offsets, part,
                       idx, (const int64_t*)total, cap);
    FDTBX_LAUNCH_CHECK("cull fill");
  }
  return FDTBX_OK;
}

extern "C" int fdtbx_cull(const fdtbx_geometry* geom, const double* tile, int64_t n_hkl, const double* cull,
                          int64_t* offsets, int32_t* idx, int64_t cap, int64_t* n_pairs, void* ws, size_t ws_bytes,
                          void* stream) {
  if (!geom || !tile || !offsets || !n_pairs) return fail(FDTBX_ERR_INVALID_ARGUMENT, "null pointer");
  if (n_hkl < 0) return fail(FDTBX_ERR_INVALID_ARGUMENT, "n_hkl must be non-negative");
  if (n_hkl > (int64_t)INT32_MAX) return fail(FDTBX_ERR_UNSUPPORTED, "more than 2^31 reflections");
  int rc = check_geometry(geom);
  if (rc) return rc;
  if (n_hkl == 0) {  // every list empty
    *n_pairs = 0;
    return fill(offsets, (int64_t)tiles_x_of(geom) * tiles_y_of(geom) + 1, (int64_t)0,
                (hipStream_t)stream);
  }
  CullParams q;
  cull_params(geom, n_hkl, &q);
  return cull_lists(q, tile, cull, offsets, idx, cap, n_pairs, ws, ws_bytes, (hipStream_t)stream);
}

// ---------------------------------------------------------------- stacked tiles
// Pairs of launched tile rows (2 sy, 2 sy + 1) form the rows sy of a grid of stacked tiles,
// tiles_x wide and ceil(lrows / 2) high (the last one a single row when lrows is odd); a
// stacked tile's box is the union of its tiles' boxes, and its list comes from the same test.
static int32_t stacked_rows_of(const fdtbx_geometry* g) { return (int32_t)ceil_div(lrows_of(g), 2); }

static void stacked_params(const fdtbx_geometry* g, int64_t n_hkl, CullParams* q) {
  q->tiles_x = tiles_x_of(g);
  q->tiles_y = stacked_rows_of(g);
  q->lcols = lcols_of(g);
  q->lrows = q->tiles_y;
  q->sb_x = (int32_t)ceil_div(q->tiles_x, kSB);
  q->sb_y = (int32_t)ceil_div(q->tiles_y, kSB);
  q->n_hkl = n_hkl;
  q->n_words = ceil_div(n_hkl, 64);
}

namespace fdtbx {
__global__ void k_stack_boxes(int32_t tiles_x, int32_t lrows, int32_t n_srows, const double* __restrict__ tile,
                              double* __restrict__ stile) {
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= (int64_t)tiles_x * n_srows) return;
  const int64_t sx = s % tiles_x, sy = s / tiles_x;
  const int64_t r0 = 2 * sy, r1 = 2 * sy + 1 < lrows ? 2 * sy + 1 : 2 * sy;
  const double* a = tile + 8 * (r0 * tiles_x + sx);
  const double* b = tile + 8 * (r1 * tiles_x + sx);
  double* o = stile + 8 * s;
  for (int c = 0; c < 6; c += 2) {
    o[c] = fmin(a[c], b[c]);
    o[c + 1] = fmax(a[c + 1], b[c + 1]);
  }
  o[6] = 0.0;
  o[7] = 0.0;
}
}  // namespace fdtbx

extern "C" int32_t fdtbx_stacked_rows(const fdtbx_geometry* geom) {
  if (!geom || check_geometry(geom)) return 0;
  return stacked_rows_of(geom);
}

extern "C" int fdtbx_stacked_boxes(const fdtbx_geometry* geom, const double* tile, double* stile, void* stream) {
  if (!geom || !tile || !stile) return fail(FDTBX_ERR_INVALID_ARGUMENT, "null pointer");
  int rc = check_geometry(geom);
  if (rc) return rc;
  const int32_t tx = tiles_x_of(geom), ns = stacked_rows_of(geom);
  const int64_t n = (int64_t)tx * ns;
  hipLaunchKernelGGL(k_stack_boxes, dim3((unsigned)ceil_div(n, 256)), dim3(256), 0, (hipStream_t)stream, tx,
                     lrows_of(geom), ns, tile, stile);
  FDTBX_LAUNCH_CHECK("stacked tile boxes");
  return FDTBX_OK;
}

extern "C" size_t fdtbx_stacked_cull_workspace(const fdtbx_geometry* geom, int64_t n_hkl) {
  if (!geom || check_geometry(geom) || n_hkl <= 0) return 0;
  CullParams q;
  stacked_params(geom, n_hkl, &q);
  return cull_workspace_of(q);
}

extern "C" int fdtbx_stacked_cull(const fdtbx_geometry* geom, const double* stile, int64_t n_hkl, const double* cull,
                                  int64_t* offsets, int32_t* idx, int64_t cap, int64_t* n_pairs, void* ws,
                                  size_t ws_bytes, void* stream) {
  if (!geom || !stile || !offsets || !n_pairs) return fail(FDTBX_ERR_INVALID_ARGUMENT, "null pointer");
  if (n_hkl < 0) return fail(FDTBX_ERR_INVALID_ARGUMENT, "n_hkl must be non-negative");
  if (n_hkl > (int64_t)INT32_MAX) return fail(FDTBX_ERR_UNSUPPORTED, "more than 2^31 reflections");
  int rc = check_geometry(geom);
  if (rc) return rc;
  CullParams q;
  stacked_params(geom, n_hkl, &q);
  if (n_hkl == 0) {
    *n_pairs = 0;
    return fill(offsets, (int64_t)q.tiles_x * q.tiles_y + 1, (int64_t)0, (hipStream_t)stream);
  }
  return cull_lists(q, stile, cull, offsets, idx, cap, n_pairs, ws, ws_bytes, (hipStream_t)stream);
}

namespace fdtbx {
// Closes the exclusive scan of the counts: offsets[n_tiles] = total and the statistics; if the
// lists need more than cap pairs every list is made empty (offsets all 0) and the overflow
// flag is set, so the kernels after it read nothing.
__global__ void k_cull_commit(int64_t* __restrict__ offsets, int64_t n_tiles, const int64_t* __restrict__ total, int64_t cap,
                              fdtbx_stats* __restrict__ stats) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t t = *total;
  const bool over = t > cap;
  if (k <= n_tiles && (over || k == n_tiles)) offsets[k] = over ? 0 : t;
  if (k == 0 && stats) {
    stats->n_pairs = t;
    stats->overflow = over ? 1 : 0;
  }
}

// fdtbx_cull without a host round trip: the capacity check happens on the device.
int cull_on_device(const fdtbx_geometry* geom, const double* tile, int64_t n_hkl, const double* cull, int64_t* offsets,
                   int32_t* idx, int64_t cap, fdtbx_stats* stats, void* ws, size_t ws_bytes, hipStream_t s) {
  if (n_hkl == 0) return fill(offsets, (int64_t)tiles_x_of(geom) * tiles_y_of(geom) + 1, (int64_t)0, s);
  if (!cull || !ws || !idx) return fail(FDTBX_ERR_INVALID_ARGUMENT, "null pointer");
  if (ws_bytes < fdtbx_cull_workspace(geom, n_hkl)) return fail(FDTBX_ERR_BUFFER_TOO_SMALL, "cull workspace too small");
  CullParams q;
  cull_params(geom, n_hkl, &q);
  const int64_t nsb = (int64_t)q.sb_x * q.sb_y;
  const int64_t n_tiles = (int64_t)q.tiles_x * q.tiles_y;
  char* w = (char*)ws;
  double* sb = (double*)w;
  w += align_up((size_t)nsb * 8 * sizeof(double), 256);
  uint64_t* mask = (uint64_t*)w;
  w += align_up((size_t)nsb * q.n_words * sizeof(uint64_t), 256);
  int64_t* total = (int64_t*)w;
  w += align_up(sizeof(int64_t) * 2, 256);
  int32_t* part = (int32_t*)w;
  hipLaunchKernelGGL(k_sb_boxes, dim3((unsigned)ceil_div(nsb, 256)), dim3(256), 0, s, q, tile, sb);
  FDTBX_LAUNCH_CHECK("cull superblocks");
  hipLaunchKernelGGL(k_sb_mask, dim3((unsigned)q.n_words), dim3(64), 0, s, q, sb, cull, mask);
  FDTBX_LAUNCH_CHECK("cull masks");
  hipLaunchKernelGGL(k_tile_lists<0>, dim3((unsigned)nsb), dim3(64 * kTB), 0, s, q, tile, mask, cull, offsets, part,
                     (int32_t*)nullptr, (const int64_t*)nullptr, (int64_t)0);
  FDTBX_LAUNCH_CHECK("cull count");
  hipLaunchKernelGGL(k_scan_inplace, dim3(1), dim3(1024), 0, s, offsets, n_tiles, total);
  FDTBX_LAUNCH_CHECK("cull scan");
  hipLaunchKernelGGL(k_tile_lists<1>, dim3((unsigned)nsb), dim3(64 * kTB), 0, s, q, tile, mask, cull, offsets, part, idx,
                     (const int64_t*)total, cap);
  FDTBX_LAUNCH_CHECK("cull fill");
  hipLaunchKernelGGL(k_cull_commit, dim3((unsigned)ceil_div(n_tiles + 1, 256)), dim3(256), 0, s, offsets, n_tiles,
                     (const int64_t*)total, cap, stats);
  FDTBX_LAUNCH_CHECK("cull commit");
  return FDTBX_OK;
}
}  // namespace fdtbx

extern "C" int fdtbx_batch_entry_init(const fdtbx_model* model, fdtbx_batch_entry* e) {
  if (!model || !e) return fail(FDTBX_ERR_INVALID_ARGUMENT, "null pointer");
  int rc = check_model(model);
  if (rc) return rc;
  e->model = *model;
  Frame f;
  make_frame(model->cell, &f);
  for (int k = 0; k < 9; ++k) {
    e->frame[k] = f.a[k];
    e->frame[9 + k] = f.s[k];
  }
  e->frame[18] = f.V;
  for (int i = 0; i < 3; ++i) {
    e->setup_g[i] = model->dis.g[i];
    e->setup_N_base[i] = model->dis.N_base[i];
  }
  e->stale = 0;
  e->reserved = 0;
  return FDTBX_OK;
}

extern "C" int fdtbx_batch_entries_check(const fdtbx_batch_entry* entries, int32_t n_models) {
  if (!entries || n_models <= 0) return fail(FDTBX_ERR_INVALID_ARGUMENT, "batch entries: null pointer or no models");
  for (int32_t m = 0; m < n_models; ++m) {
    const fdtbx_batch_entry& e = entries[m];
    if (e.n_types < 1 || e.n_types > 16) return fail(FDTBX_ERR_INVALID_ARGUMENT, "batch entry: n_types must be in 1..16");
    if (e.n_tiles < 0 || e.n_atoms < 0 || e.n_hkl < 0)
      return fail(FDTBX_ERR_INVALID_ARGUMENT, "batch entry: negative n_tiles, n_atoms or n_hkl");
    if (e.atom_off < 0 || e.hkl_off < 0 || e.pix_off < 0 || e.tile_off < 0 || e.rowptr_off < 0 || e.pair_off < 0 ||
        e.node_off < 0 || e.ff_off < 0)
      return fail(FDTBX_ERR_INVALID_ARGUMENT, "batch entry: negative offset");
    const int rc = check_model(&e.model);
    if (rc) return rc;
  }
  return FDTBX_OK;
}

namespace fdtbx {
int launch_batch_prep(const fdtbx_batch_entry* ent, const int64_t* blocks, int64_t n_rb, const int32_t* hkl, const float* F2,
                      float* refl, hipStream_t s) {
  if (n_rb <= 0) return FDTBX_OK;
  hipLaunchKernelGGL(k_b_prep, dim3((unsigned)n_rb), dim3(256), 0, s, ent, blocks, hkl, F2, refl);
  FDTBX_LAUNCH_CHECK("batch prep");
  return FDTBX_OK;
}
}  // namespace fdtbx
