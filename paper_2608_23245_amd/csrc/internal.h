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

inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }
inline size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// Reflection record slots (float32, FDTBX_REFL_FLOATS per reflection).
enum ReflSlot {
  RS_W = 0,        // |F|^2 I_para
  RS_N = 1,        // N_eff a, b, c (1..3)
  RS_R0 = 4,       // |D|
  RS_WK = 5,       // W r0^2 N_a N_b N_c / (2 pi)^6: weight of the per-reflection node sum
  RS_B = 6,        // N_i r0 (a_i.S)/2       (6..8)
  RS_G1 = 9,       // N_i r0 (a_i.e1)/2      (9..11)
  RS_G2 = 12,      // N_i r0 (a_i.e2)/2      (12..14)
  RS_TR = 15,      // N_i (a_i.e_perp)/2     (15..17)
  RS_TZ = 18,      // N_i a_i,z / 2          (18..20)
  RS_IP = 21,      // I_para
  RS_RD = 22,      // D.e_perp as float64 bits (22..23)
  RS_ZD = 24,      // D_z as float64 bits      (24..25)
  RS_CS = 26,      // (e_perp.S, S_z)
  RS_C1 = 28,      // (e_perp.e1, e1_z)
  RS_C2 = 30,      // (e_perp.e2, e2_z)
  RS_RHO = 32,     // support extent along S, e1, e2: sum_i (m/N_i)|a*_i.v|  (32..34)
  RS_A = 35,       // coherence factors A_i (35..37)
  RS_H = 38,       // h, k, l as floats (38..40)
  RS_F2 = 41,      // |F|^2
  RS_K = 42,       // r0^2 N_a N_b N_c / (2 pi)^6, so that RS_WK = W * RS_K
};

// Cell frame in the laboratory convention: rows of avec are a, b, c; rows of
// astar are a*, b*, c*.  Binary64, operation order fixed (compiled without
// contraction in the exact translation unit).
struct Frame {
  double a[9];
  double s[9];
  double V;
};

}  // namespace fdtbx
