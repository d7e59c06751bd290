// Shared definitions of the HIP library: complex helpers on double2/float2,
// error handling, and the sizes that every translation unit agrees on.
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>
#include <cmath>
#include <cstdint>
#include <cstddef>
#include <stdexcept>
#include <string>

#include "../../include/lsp.h"

namespace lsp {

// Error carried through the C++ layers and turned into an lsp_status at the ABI.
struct Error : std::runtime_error {
  lsp_status status;
  Error(lsp_status s, const std::string& msg) : std::runtime_error(msg), status(s) {}
};

#define LSP_HIP(call)                                                              \
  do {                                                                             \
    hipError_t e_ = (call);                                                        \
    if (e_ != hipSuccess)                                                          \
      throw ::lsp::Error(LSP_ERR_HIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

#define LSP_REQUIRE(cond, msg)                                 \
  do {                                                         \
    if (!(cond)) throw ::lsp::Error(LSP_ERR_ARG, (msg));       \
  } while (0)

// ---------------------------------------------------------------- complex math
template <typename T> struct cvec;
template <> struct cvec<double> { using type = double2; };
template <> struct cvec<float> { using type = float2; };
template <typename T> using cplx = typename cvec<T>::type;

template <typename T> __host__ __device__ inline cplx<T> mk(T re, T im) {
  cplx<T> r; r.x = re; r.y = im; return r;
}
template <typename C> __host__ __device__ inline C cadd(C a, C b) { C r; r.x = a.x + b.x; r.y = a.y + b.y; return r; }
template <typename C> __host__ __device__ inline C csub(C a, C b) { C r; r.x = a.x - b.x; r.y = a.y - b.y; return r; }
template <typename C> __host__ __device__ inline C cmul(C a, C b) {
  C r; r.x = a.x * b.x - a.y * b.y; r.y = a.x * b.y + a.y * b.x; return r;
}
// conj(a) * b
template <typename C> __host__ __device__ inline C cmulc(C a, C b) {
  C r; r.x = a.x * b.x + a.y * b.y; r.y = a.x * b.y - a.y * b.x; return r;
}
template <typename C> __host__ __device__ inline C cconj(C a) { C r; r.x = a.x; r.y = -a.y; return r; }
template <typename C, typename T> __host__ __device__ inline C cscale(C a, T s) { C r; r.x = a.x * s; r.y = a.y * s; return r; }
// a - b*c as two fused multiply-adds per component
template <typename C> __host__ __device__ inline C cfms(C a, C b, C c) {
  C r; r.x = fma(b.y, c.y, fma(-b.x, c.x, a.x)); r.y = fma(-b.y, c.x, fma(-b.x, c.y, a.y)); return r;
}
// a + b*c as two fused multiply-adds per component
template <typename C> __host__ __device__ inline C cfma(C a, C b, C c) {
  C r; r.x = fma(-b.y, c.y, fma(b.x, c.x, a.x)); r.y = fma(b.y, c.x, fma(b.x, c.y, a.y)); return r;
}
template <typename C> __host__ __device__ inline C cdiv(C a, C b) {
  // Smith's algorithm
  C r;
  if (fabs(b.x) >= fabs(b.y)) {
    auto t = b.y / b.x; auto den = b.x + b.y * t;
    r.x = (a.x + a.y * t) / den; r.y = (a.y - a.x * t) / den;
  } else {
    auto t = b.x / b.y; auto den = b.x * t + b.y;
    r.x = (a.x * t + a.y) / den; r.y = (a.y * t - a.x) / den;
  }
  return r;
}
template <typename C> __host__ __device__ inline auto cabs1(C a) -> decltype(a.x) { return fabs(a.x) + fabs(a.y); }

__host__ __device__ inline float2 to_c64(double2 a) { return make_float2((float)a.x, (float)a.y); }
__host__ __device__ inline double2 to_c128(float2 a) { return make_double2((double)a.x, (double)a.y); }
template <typename C> __host__ __device__ inline C from_c128(double2 a);
template <> __host__ __device__ inline double2 from_c128<double2>(double2 a) { return a; }
template <> __host__ __device__ inline float2 from_c128<float2>(double2 a) { return to_c64(a); }
__host__ __device__ inline double2 widen(double2 a) { return a; }
__host__ __device__ inline double2 widen(float2 a) { return to_c128(a); }

// Brackets one kernel launch with HIP events when timing is enabled
// (lsp_timing_enable); a no-op otherwise.  esize tags the element type.
// When timing is enabled, a launch takes a start and a stop event that the
// runtime records at the kernel's own start and end (hipExtLaunchKernelGGL),
// so the measured time is the kernel's execution, as a profiler sees it.
class KTimer {
 public:
  KTimer(const char* name, int esize, hipStream_t st);
  ~KTimer();
  KTimer(const KTimer&) = delete;
  KTimer& operator=(const KTimer&) = delete;
  bool active() const { return a_ != nullptr; }
  hipEvent_t start() const { return a_; }
  hipEvent_t stop() const { return b_; }
  void launched() { launched_ = true; }

 private:
  hipStream_t st_;
  hipEvent_t a_, b_;
  bool launched_ = false;
  std::string key_;
};

#define LSP_LAUNCH(name, esize, kernel, grid, block, shm, st, ...)                                      \
  do {                                                                                                  \
    ::lsp::KTimer kt_((name), (esize), (st));                                                           \
    if (kt_.active())                                                                                   \
      hipExtLaunchKernelGGL(kernel, grid, block, shm, st, kt_.start(), kt_.stop(), 0u, __VA_ARGS__);   \
    else                                                                                                \
      hipLaunchKernelGGL(kernel, grid, block, shm, st, __VA_ARGS__);                                    \
    LSP_HIP(hipGetLastError());                                                                         \
    kt_.launched();                                                                                     \
  } while (0)

inline int ipow(int b, int e) { int r = 1; while (e-- > 0) r *= b; return r; }
inline size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

constexpr int kMaxStencil = 27;   // 3^3
constexpr int kMaxClasses = 27;   // 3^3 position classes

}  // namespace lsp
