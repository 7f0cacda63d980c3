// Internal declarations shared by the library's translation units (not installed).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/fdtbx.h"

namespace fdtbx {

// Error reporting: host-side checks set a thread-local message and return a code.
int fail(int code, const char* msg);
int hip_fail(hipError_t e, const char* where);
#define FDTBX_HIP(call)                                  \
  do {                                                   \
    hipError_t e_ = (call);                              \
    if (e_ != hipSuccess) return fdtbx::hip_fail(e_, #call); \
  } while (0)
#define FDTBX_LAUNCH_CHECK(where)                                 \
  do {                                                            \
    hipError_t e_ = hipGetLastError();                            \
    if (e_ != hipSuccess) return fdtbx::hip_fail(e_, where);      \
  } while (0)

bool finite_pos(double v);
int check_cell(const fdtbx_cell* c);
int check_geometry(const fdtbx_geometry* g);
int check_model(const fdtbx_model* m);
int tile_waves(const fdtbx_geometry* g, int64_t n_tiles, int* waves);
// fdtbx_cull with the capacity check on the device (no host round trip): on overflow the
// lists are left empty and stats->overflow is set (stats may be NULL).
int cull_on_device(const fdtbx_geometry* geom, const double* tile, int64_t n_hkl, const double* cull, int64_t* offsets,
                   int32_t* idx, int64_t cap, fdtbx_stats* stats, void* ws, size_t ws_bytes, hipStream_t s);

inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

// Pixel tiles of a checked geometry: 2^tile_lg columns by 64 >> tile_lg rows.
inline int tile_lg(const fdtbx_geometry* g) { return __builtin_ctz((unsigned)(g->tile_w ? g->tile_w : FDTBX_TILE)); }
inline int32_t tiles_x_of(const fdtbx_geometry* g) { return (int32_t)ceil_div(g->width, 1 << tile_lg(g)); }
inline int32_t tiles_y_of(const fdtbx_geometry* g) { return (int32_t)ceil_div(g->height, 64 >> tile_lg(g)); }
// Tile columns and rows the per-tile kernels launch: all, or the left half (with the middle
// column) under the left-right fold (mirror bit 0), the top half (with the middle row) under
// the up-down fold (mirror bit 1).
inline int32_t lcols_of(const fdtbx_geometry* g) { return (g->mirror & 1) ? (tiles_x_of(g) + 1) / 2 : tiles_x_of(g); }
inline int32_t lrows_of(const fdtbx_geometry* g) { return (g->mirror & 2) ? (tiles_y_of(g) + 1) / 2 : tiles_y_of(g); }
inline size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// v[0..n) = x, by a kernel (hipMemsetAsync nodes do not belong in captured graphs).
template <class T>
__global__ void k_fill(T* __restrict__ v, int64_t n, T x) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) v[i] = x;
}
template <class T>
inline int fill(T* v, int64_t n, T x, hipStream_t s) {
  if (n <= 0 || !v) return FDTBX_OK;
  hipLaunchKernelGGL(k_fill<T>, dim3((unsigned)ceil_div(n, 256)), dim3(256), 0, s, v, n, x);
  FDTBX_LAUNCH_CHECK("fill");
  return FDTBX_OK;
}
// Node-table rows for n nodes per side: node records, then block records.
__host__ __device__ inline int64_t node_rows(int64_t n) {
  const int64_t nb = (n + FDTBX_NODE_BLOCK - 1) / FDTBX_NODE_BLOCK;
  return n * n + nb * nb;
}

// Next item of a persistent launch: lane 0 takes it from the counter and the wave reads
// lane 0's value into scalar registers (so everything indexed by it is loaded as uniform).
__device__ inline int64_t next_item(unsigned long long* counter) {
  unsigned long long mine = 0;
  if ((threadIdx.x & 63) == 0) mine = atomicAdd(counter, 1ull);
  const unsigned lo = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)mine);
  const unsigned hi = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)(mine >> 32));
  return (int64_t)(((unsigned long long)hi << 32) | lo);
}

// Orders one wave's LDS accesses before and after this point (what __syncthreads does for a
// one-wave workgroup) without a workgroup barrier, so that several independent waves can
// share a workgroup.
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

// Wave-wide reductions (all 64 lanes active) through DPP row shifts and row broadcasts
// instead of LDS permutes: shifts by 1, 2, 4, 8 leave each row's total in its lane 15, the
// broadcasts of lanes 15 and 31 then combine the rows, and lane 63 holds the result, which is
// read into a scalar register (uniform).  Lanes whose source lies outside their row combine
// with the operation's identity.  Float minima and maxima run on an order-preserving integer
// image of the bits (x ^ 0x7fffffff for negative x), so each step is one integer min or max
// with its DPP operand.
template <int CTRL, int ROWS>
__device__ __forceinline__ int dpp_i32(int old, int v) {
  return __builtin_amdgcn_update_dpp(old, v, CTRL, ROWS, 0xf, false);
}
template <int CTRL, int ROWS>
__device__ __forceinline__ float dpp_f32(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, ROWS, 0xf, true));
}
__device__ __forceinline__ int float_order(float f) {
  const int b = __float_as_int(f);
  return b ^ ((b >> 31) & 0x7fffffff);
}
__device__ __forceinline__ float order_float(int k) { return __int_as_float(k ^ ((k >> 31) & 0x7fffffff)); }
__device__ __forceinline__ int wave_min_i32(int v) {
  v = min(v, dpp_i32<0x111, 0xf>(INT32_MAX, v));
  v = min(v, dpp_i32<0x112, 0xf>(INT32_MAX, v));
  v = min(v, dpp_i32<0x114, 0xf>(INT32_MAX, v));
  v = min(v, dpp_i32<0x118, 0xf>(INT32_MAX, v));
  v = min(v, dpp_i32<0x142, 0xa>(INT32_MAX, v));
  v = min(v, dpp_i32<0x143, 0xc>(INT32_MAX, v));
  return __builtin_amdgcn_readlane(v, 63);
}
__device__ __forceinline__ int wave_max_i32(int v) {
  v = max(v, dpp_i32<0x111, 0xf>(INT32_MIN, v));
  v = max(v, dpp_i32<0x112, 0xf>(INT32_MIN, v));
  v = max(v, dpp_i32<0x114, 0xf>(INT32_MIN, v));
  v = max(v, dpp_i32<0x118, 0xf>(INT32_MIN, v));
  v = max(v, dpp_i32<0x142, 0xa>(INT32_MIN, v));
  v = max(v, dpp_i32<0x143, 0xc>(INT32_MIN, v));
  return __builtin_amdgcn_readlane(v, 63);
}
__device__ __forceinline__ float wave_min(float v) { return order_float(wave_min_i32(float_order(v))); }
__device__ __forceinline__ float wave_max(float v) { return order_float(wave_max_i32(float_order(v))); }
// Binary64 wave sum through the same DPP steps on the two 32-bit halves.
template <int CTRL, int ROWS>
__device__ __forceinline__ double dpp_f64(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffll), CTRL, ROWS, 0xf, true);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, ROWS, 0xf, true);
  return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}
__device__ __forceinline__ double wave_sum_f64(double v) {
  v += dpp_f64<0x111, 0xf>(v);
  v += dpp_f64<0x112, 0xf>(v);
  v += dpp_f64<0x114, 0xf>(v);
  v += dpp_f64<0x118, 0xf>(v);
  v += dpp_f64<0x142, 0xa>(v);
  v += dpp_f64<0x143, 0xc>(v);
  const long long b = __double_as_longlong(v);
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(b & 0xffffffffll), 63);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(b >> 32), 63);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}
__device__ __forceinline__ float wave_sum(float v) {
  v += dpp_f32<0x111, 0xf>(v);
  v += dpp_f32<0x112, 0xf>(v);
  v += dpp_f32<0x114, 0xf>(v);
  v += dpp_f32<0x118, 0xf>(v);
  v += dpp_f32<0x142, 0xa>(v);
  v += dpp_f32<0x143, 0xc>(v);
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 63));
}

// Reflection record slots (float32, FDTBX_REFL_FLOATS = 64 per reflection: 256 bytes, two
// 128-byte cache lines).  Slots 0..31 are everything a (tile, reflection) pair of the profile
// walks reads (one aligned line, loaded whole); the second line holds what only the set-up, the
// gradient, the Hosemann lineshape and the other launches read.
enum ReflSlot {
  RS_HOT = 0,      // start of the per-pair line (slots 0..31)
  RS_R0 = 0,       // |D|
  RS_WK = 1,       // W r0^2 C: weight of the per-reflection node sum (RS_K below)
  RS_B = 2,        // scale_i r0 (a_i.S)      (2..4)
  RS_G1 = 5,       // scale_i r0 (a_i.e1)     (5..7)
  RS_G2 = 8,       // scale_i r0 (a_i.e2)     (8..10)
  RS_TR = 11,      // scale_i (a_i.e_perp)    (11..13)
  RS_TZ = 14,      // scale_i a_i,z           (14..16)
  RS_IP = 17,      // I_para
  RS_RD = 18,      // D.e_perp as float64 bits (18..19)
  RS_ZD = 20,      // D_z as float64 bits      (20..21)
  RS_CS = 22,      // (e_perp.S, S_z)
  RS_C1 = 24,      // (e_perp.e1, e1_z)
  RS_C2 = 26,      // (e_perp.e2, e2_z)
  RS_RHO = 28,     // support extent along S, e1, e2: sum_i w_i |a*_i.v|  (28..30)
  RS_AZ = 31,      // e_az.S, e_az.e1, e_az.e2 with e_az = z x e_perp (31..33)
  RS_TA = 34,      // scale_i (a_i.e_az), the lattice offset along the ring direction (34..36)
  RS_F2 = 37,      // |F|^2
  RS_K = 38,       // r0^2 C with C the lineshape's constant (Laue prod N/(2 pi)^6, Gaussian
                   // prod N, Hosemann prod (1 - A'^2)), so that RS_WK = W * RS_K
  RS_W = 39,       // |F|^2 I_para
  RS_AH = 40,      // Hosemann lineshape: A'_i = max(0, (N_i - 1)/(N_i + 1)) (40..42)
  RS_N = 43,       // N_eff a, b, c (43..45)
  RS_LO = 46,      // float32 residuals x - (float)x of the binary64 values x of B, G1, G2, TR, TZ
                   // (46..60, that order, as slots RS_B..RS_TZ) and of TA (61..63): hi + lo
                   // holds x to 2^-48 relative, for the Hosemann support-edge decisions
  RS_LO_TA = 61,
};

// Per-axis scale of the lattice offsets y_i in the record (y_i = scale_i a_i.(p - s)) and
// the support half-width in y: N_i/2 and m/2 for the Laue and Gaussian lineshapes (the
// sines and the Gaussian take y in turns of half the Laue argument), 1 and 1/2 for the
// Hosemann lineshape (y = u, one lattice period).
__host__ __device__ inline double lineshape_half(int32_t lineshape, int32_t m) {
  return lineshape == FDTBX_LINESHAPE_HOSEMANN ? 0.5 : 0.5 * (double)m;
}

// Exclusive scan of n values in place with one block of 1024 threads; writes the grand total
// to *total (exact.hip).
__global__ void k_scan_inplace(int64_t* v, int64_t n, int64_t* total);

// Balanced forward launch (profile.hip): workspace bytes for pair_cap culled pairs, and the
// launch (see fdtbx_profile_balanced).
size_t balanced_workspace(const fdtbx_model* model, int64_t pair_cap);
int launch_balanced(const fdtbx_model* model, const float* refl, const float* nodes, const double* pix,
                    const double* tile, const int64_t* offsets, const int32_t* idx, const int32_t* order,
                    int64_t pair_cap, float* image, void* ws, size_t ws_bytes, hipStream_t s);

// Balanced adjoint (adjoint.hip) over the unit tables a balanced forward launch left in
// units_ws; ctr: 8 int32 of device scratch; sums or partials cleared by the caller.
int launch_adjoint_units(const fdtbx_model* model, const float* refl, const float* nodes, const double* pix,
                         const double* tile, const int64_t* offsets, const int32_t* idx, const int32_t* order,
                         int64_t pair_cap, const void* units_ws, int32_t* ctr, int64_t n_hkl, const float* grad_image,
                         double* sums, float* partials, hipStream_t s);

// Batched launchers (one per translation unit that owns the kernels).
int launch_batch_sf(const fdtbx_batch_entry* ent, const int64_t* blocks, int64_t n_rb, const float* x, const float* y,
                    const float* z, const float* B, const float* occ, const int32_t* type, const float* ff, const int32_t* hkl,
                    float* F, float* F2, hipStream_t s);
int launch_batch_prep(const fdtbx_batch_entry* ent, const int64_t* blocks, int64_t n_rb, const int32_t* hkl, const float* F2,
                      float* refl, hipStream_t s);
int launch_batch_nodes(const fdtbx_batch_entry* ent, const int64_t* blocks, int64_t n_nb, float* nodes, hipStream_t s);
int launch_batch_profile(const fdtbx_batch_entry* ent, const int64_t* items, int64_t n_items, const float* refl,
                         const float* nodes, const double* pix, const double* tile, const int64_t* rowptr, const int32_t* idx,
                         float* image, int64_t* counter, hipStream_t s);
int launch_batch_profile_stacked(const fdtbx_batch_entry* ent, const int64_t* soff, const int64_t* items,
                                 int64_t n_items, const float* refl, const float* nodes, const double* pix,
                                 const double* tile, const double* stile, const int64_t* srowptr, const int32_t* sidx,
                                 float* image, int64_t* counter, hipStream_t s);
// Fixed-order accumulation of the adjoint sums (fdtbx_pair_reduce): per-pair partials
// float32 [n_pairs][12] and the pairs of each reflection in a fixed order.
struct PairOrder {
  float* partials;
  int64_t n_pairs;
  const int64_t* refl_ptr;    // [n_hkl + 1]
  const int32_t* refl_pairs;  // [n_pairs]
  const int64_t* mate;        // [n_hkl], -1 where the model has no up-down fold
};

int launch_batch_backward(const fdtbx_batch_entry* ent, int32_t n_models, const int64_t* refl_blocks, int64_t n_rb,
                          const int64_t* model_rb, const int64_t* atom_blocks, int64_t n_ab, const int64_t* items,
                          int64_t n_items, int64_t n_hkl_total, const int32_t* hkl, const float* x, const float* y,
                          const float* z, const float* B, const float* occ, const int32_t* type, const float* ff,
                          const double* pix, const double* tile, const int64_t* rowptr, const int32_t* idx, const float* F,
                          const float* refl, const float* nodes, const float* grad_image, double* sums, double* part,
                          float* dF2, float* d_x, float* d_y, float* d_z, float* d_B, float* d_occ, double* d_globals,
                          int64_t* counter, const PairOrder* fixed, hipStream_t s);

// Cell frame in the laboratory convention: rows of avec are a, b, c; rows of
// astar are a*, b*, c*.  Binary64, operation order fixed (compiled without
// contraction in the exact translation unit).
struct Frame {
  double a[9];
  double s[9];
  double V;
};

}  // namespace fdtbx
