// 16x16x4 matrix-core products in FP32 and FP64 (device code only).
#pragma once

#include <hip/hip_runtime.h>

namespace lsp {

// Operand layout of the 16x16x4 MFMAs: lane l supplies A(l%16, l/16) and
// B(l/16, l%16).  Results: the FP32 form returns D(4*(l/16)+v, l%16), the
// FP64 form D(l/16+4v, l%16), v = 0..3 (checked on gfx950).
template <typename T> struct Mfma;
template <> struct Mfma<double> {
  using acc_t = __attribute__((__vector_size__(4 * sizeof(double)))) double;
  __device__ static acc_t step(double a, double b, acc_t c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }
  __device__ static int row(int lk, int v) { return lk + 4 * v; }
};
template <> struct Mfma<float> {
  using acc_t = __attribute__((__vector_size__(4 * sizeof(float)))) float;
  __device__ static acc_t step(float a, float b, acc_t c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
  __device__ static int row(int lk, int v) { return 4 * lk + v; }
};

}  // namespace lsp
