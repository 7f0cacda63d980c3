// A detector pattern through the C ABI alone (no Python, no torch): reflection list, structure
// factors and the one-call pattern, with device buffers from hipMalloc.
//
//   fdtbx_pattern <input> <output>
//
// input (native byte order, as written by tests/test_gpu_c_caller.py): the fdtbx_model struct;
// int64 n_atoms, n_types; float32 x, y, z, B, occ [n_atoms]; int32 type [n_atoms];
// float32 ff [n_types][9].  The resolution shell and the extinction cull come from the model
// (quad.d_min, quad.d_max; dis.g with quad.extinction).
// output: float32 image [height][width], then int64 n_hkl and int32 hkl [n_hkl][3].  Prints the
// reflection and culling pair counts.  Exit status 0 on success, 1 on any library or HIP error.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>
#include <vector>

#include "fdtbx.h"

#define CHECK(call)                                                                          \
  do {                                                                                       \
    const int rc_ = (call);                                                                  \
    if (rc_ != FDTBX_OK) {                                                                   \
      std::fprintf(stderr, "%s failed: %d (%s)\n", #call, rc_, fdtbx_error_string(rc_));     \
      return 1;                                                                              \
    }                                                                                        \
  } while (0)
#define HIPCHECK(call)                                                                       \
  do {                                                                                       \
    const hipError_t e_ = (call);                                                            \
    if (e_ != hipSuccess) {                                                                  \
      std::fprintf(stderr, "%s failed: %s\n", #call, hipGetErrorString(e_));                 \
      return 1;                                                                              \
    }                                                                                        \
  } while (0)

template <class T>
static bool read_into(std::FILE* f, T* v, size_t n) {
  return std::fread(v, sizeof(T), n, f) == n;
}

template <class T>
static int to_device(const std::vector<T>& h, T** d) {
  HIPCHECK(hipMalloc((void**)d, h.size() * sizeof(T) + 16));
  HIPCHECK(hipMemcpy(*d, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice));
  return 0;
}

int main(int argc, char** argv) {
  if (argc != 3) {
    std::fprintf(stderr, "usage: %s <input> <output>\n", argv[0]);
    return 1;
  }
  std::FILE* in = std::fopen(argv[1], "rb");
  if (!in) {
    std::fprintf(stderr, "cannot open %s\n", argv[1]);
    return 1;
  }
  fdtbx_model model;
  int64_t n_atoms = 0, n_types = 0;
  bool ok = read_into(in, &model, 1) && read_into(in, &n_atoms, 1) && read_into(in, &n_types, 1) && n_atoms > 0 && n_types > 0 && n_types <= 16;
  std::vector<float> x(n_atoms > 0 ? n_atoms : 0), y(x.size()), z(x.size()), B(x.size()), occ(x.size());
  std::vector<int32_t> type(x.size());
  std::vector<float> ff(ok ? (size_t)n_types * 9 : 0);
  ok = ok && read_into(in, x.data(), x.size()) && read_into(in, y.data(), y.size()) && read_into(in, z.data(), z.size()) &&
       read_into(in, B.data(), B.size()) && read_into(in, occ.data(), occ.size()) && read_into(in, type.data(), type.size()) &&
       read_into(in, ff.data(), ff.size());
  std::fclose(in);
  if (!ok) {
    std::fprintf(stderr, "malformed input %s\n", argv[1]);
    return 1;
  }
  for (int32_t t : type)
    if (t < 0 || t >= n_types) {
      std::fprintf(stderr, "atom type out of range\n");
      return 1;
    }

  // reflection list
  const double dmin = model.quad.d_min, dmax = model.quad.d_max;
  const double ext[4] = {model.dis.g[0], model.dis.g[1], model.dis.g[2], model.quad.extinction};
  int64_t cap = 0;
  CHECK(fdtbx_hkl_capacity(&model.cell, dmin, &cap));
  int32_t* hkl = nullptr;
  int64_t* n_dev = nullptr;
  void* ews = nullptr;
  const size_t ewsb = fdtbx_enumerate_workspace(&model.cell, dmin);
  HIPCHECK(hipMalloc((void**)&hkl, (size_t)(cap > 0 ? cap : 1) * 3 * sizeof(int32_t)));
  HIPCHECK(hipMalloc((void**)&n_dev, sizeof(int64_t)));
  HIPCHECK(hipMalloc(&ews, ewsb > 0 ? ewsb : 16));
  CHECK(fdtbx_enumerate_hkl(&model.cell, dmin, dmax, ext[3] > 0 ? ext : nullptr, hkl, cap, n_dev, ews, ewsb, nullptr));
  int64_t n_hkl = 0;
  HIPCHECK(hipMemcpy(&n_hkl, n_dev, sizeof(int64_t), hipMemcpyDeviceToHost));

  // structure factors
  float *dx, *dy, *dz, *dB, *docc, *dff;
  int32_t* dtype;
  if (to_device(x, &dx) || to_device(y, &dy) || to_device(z, &dz) || to_device(B, &dB) || to_device(occ, &docc) ||
      to_device(type, &dtype) || to_device(ff, &dff))
    return 1;
  float* F2 = nullptr;
  HIPCHECK(hipMalloc((void**)&F2, (size_t)(n_hkl > 0 ? n_hkl : 1) * sizeof(float)));
  const size_t sfb = fdtbx_sf_workspace(n_hkl, n_atoms);
  void* sws = nullptr;
  HIPCHECK(hipMalloc(&sws, sfb > 0 ? sfb : 16));
  CHECK(fdtbx_structure_factors(&model.cell, n_atoms, dx, dy, dz, dB, docc, dtype, dff, (int32_t)n_types, hkl, n_hkl,
                                nullptr, F2, sws, sfb, nullptr));

  // the pattern: a first call without list capacity returns the pair count
  const size_t npix = (size_t)model.geom.width * model.geom.height;
  float* image = nullptr;
  HIPCHECK(hipMalloc((void**)&image, npix * sizeof(float)));
  int64_t pairs = 0;
  size_t wsb = fdtbx_pattern_workspace(&model, n_hkl, 0);
  void* ws = nullptr;
  HIPCHECK(hipMalloc(&ws, wsb));
  int rc = fdtbx_profile_pattern(&model, hkl, n_hkl, F2, image, 0, &pairs, ws, wsb, nullptr);
  if (rc == FDTBX_ERR_BUFFER_TOO_SMALL) {
    HIPCHECK(hipFree(ws));
    wsb = fdtbx_pattern_workspace(&model, n_hkl, pairs);
    HIPCHECK(hipMalloc(&ws, wsb));
    rc = fdtbx_profile_pattern(&model, hkl, n_hkl, F2, image, pairs, &pairs, ws, wsb, nullptr);
  }
  CHECK(rc);
  HIPCHECK(hipDeviceSynchronize());
  std::vector<float> h(npix);
  HIPCHECK(hipMemcpy(h.data(), image, npix * sizeof(float), hipMemcpyDeviceToHost));
  std::vector<int32_t> hh((size_t)n_hkl * 3);
  HIPCHECK(hipMemcpy(hh.data(), hkl, hh.size() * sizeof(int32_t), hipMemcpyDeviceToHost));
  std::FILE* out = std::fopen(argv[2], "wb");
  if (!out || std::fwrite(h.data(), sizeof(float), npix, out) != npix || std::fwrite(&n_hkl, sizeof(int64_t), 1, out) != 1 ||
      std::fwrite(hh.data(), sizeof(int32_t), hh.size(), out) != hh.size()) {
    std::fprintf(stderr, "cannot write %s\n", argv[2]);
    return 1;
  }
  std::fclose(out);
  std::printf("reflections %lld culled pairs %lld\n", (long long)n_hkl, (long long)pairs);
  return 0;
}
