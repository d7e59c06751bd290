// Kernel table k_t = h^d G(h |t|) (Section 2.1) and its circulant embedding.
//
// G is the free-space Green's function of Section 1: (i/4) H0^(1)(w r) in 2D,
// exp(i w r) / (4 pi r) in 3D.  H0^(1) = J0 + i Y0 is evaluated here from
// published methods, not from a vendor math library:
//  * x < 20: J_k by Miller's backward recurrence J_{k-1} = (2k/x) J_k - J_{k+1},
//    normalised with J0 + 2 sum_{k>=1} J_{2k} = 1 (Abramowitz & Stegun 9.1.46),
//    and Y0 from Neumann's series
//    Y0 = (2/pi) [ (ln(x/2) + gamma) J0 - 2 sum_{k>=1} (-1)^k J_{2k} / k ]
//    (A&S 9.1.88);
//  * x >= 20: Hankel's asymptotic expansion (DLMF 10.17.5)
//    H0^(1)(x) ~ sqrt(2/(pi x)) e^{i(x - pi/4)} sum_k i^k a_k(0) / x^k,
//    a_k(0) = a_{k-1}(0) (-(2k-1)^2) / (8k), whose smallest term at x >= 20 is
//    below 1e-17, so truncation there is below double rounding.
#include "lsp_common.h"
#include "kernels.h"

namespace lsp {

namespace {

constexpr double kPi = 3.14159265358979323846;
constexpr double kEulerGamma = 0.57721566490153286061;

__device__ double2 hankel1_0(double x) {
  double J0, Y0;
  if (x < 20.0) {
    const int M = 2 * ((int)x / 2) + 42;
    double jk1 = 0.0;      // J_{k+1}
    double jk = 1e-30;     // J_k, arbitrary scale
    double norm = 0.0;     // 2 sum_{k even >= 2} J_k
    double ysum = 0.0;     // sum_{k>=1} (-1)^k J_{2k} / k
    for (int k = M; k >= 1; --k) {
      // J_k is held in jk; accumulate before stepping down.
      if ((k & 1) == 0) {
        norm += 2.0 * jk;
        int half = k / 2;
        ysum += ((half & 1) ? -jk : jk) / (double)half;
      }
      double jm1 = (2.0 * k / x) * jk - jk1;
      jk1 = jk;
      jk = jm1;
      if (fabs(jk) > 1e250) {
        jk *= 1e-250; jk1 *= 1e-250; norm *= 1e-250; ysum *= 1e-250;
      }
    }
    norm += jk;  // + J0
    J0 = jk / norm;
    Y0 = (2.0 / kPi) * ((log(0.5 * x) + kEulerGamma) * J0 - 2.0 * ysum / norm);
  } else {
    double sr = 1.0, si = 0.0;    // running sum
    double tr = 1.0, ti = 0.0;    // current term
    for (int k = 1; k < 200; ++k) {
      double f = -(double)((2 * k - 1) * (2 * k - 1)) / (8.0 * k * x);
      // t *= i * f
      double nr = -ti * f, ni = tr * f;
      tr = nr; ti = ni;
      sr += tr; si += ti;
      if (fabs(tr) + fabs(ti) < 1e-18) break;
    }
    double s, c;
    sincos(x, &s, &c);
    const double r2 = 0.70710678118654752440;  // 1/sqrt(2)
    double er = (c + s) * r2, ei = (s - c) * r2;  // e^{i(x - pi/4)}
    double amp = sqrt(2.0 / (kPi * x));
    J0 = amp * (er * sr - ei * si);
    Y0 = amp * (er * si + ei * sr);
  }
  return make_double2(J0, Y0);
}

__global__ void ktable_kernel(double2* __restrict__ k, int n, int d, double h, double omega,
                              double2 k0, long long total) {
  long long id = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= total) return;
  int n1 = n + 1;
  int t1 = (int)(id % n1);
  int t2 = (int)((id / n1) % n1);
  int t3 = d == 3 ? (int)(id / ((long long)n1 * n1)) : 0;
  if (id == 0) { k[0] = k0; return; }
  double r = h * sqrt((double)t1 * t1 + (double)t2 * t2 + (double)t3 * t3);
  double2 v;
  if (d == 2) {
    double2 H = hankel1_0(omega * r);
    // (i/4) (J0 + i Y0) h^2
    double s = 0.25 * h * h;
    v = make_double2(-H.y * s, H.x * s);
  } else {
    double sn, cs;
    sincos(omega * r, &sn, &cs);
    double s = h * h * h / (4.0 * kPi * r);
    v = make_double2(cs * s, sn * s);
  }
  k[id] = v;
}

// E[k1 + L k2 (+ L^2 k3)] = k_{|t|} at the wrapped offset t, zero on the
// index n of any axis (offsets there are never used by the convolution).
__global__ void embed_kernel(double2* __restrict__ E, const double2* __restrict__ k, int n, int d,
                             long long total) {
  long long id = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= total) return;
  int L = 2 * n, n1 = n + 1;
  int c[3] = {(int)(id % L), (int)((id / L) % L), d == 3 ? (int)(id / ((long long)L * L)) : 0};
  long long src = 0, s = 1;
  bool zero = false;
  for (int a = 0; a < d; ++a) {
    int t = c[a] < n ? c[a] : L - c[a];
    zero = zero || c[a] == n;
    src += t * s;
    s *= n1;
  }
  E[id] = zero ? make_double2(0.0, 0.0) : k[src];
}

// The spectrum in the K-matvec's order (fft.hip): for the split order
// c -> frequency 2c (c < n) or 2(c - n) + 1 (c >= n) along every axis, row
// fold(k1) [+ (n+1) fold(k2)] holds the L values along the last axis, where
// fold(k) = min(k, L - k) (the embedded kernel is even along every axis);
// scaled by 1/L^d (the inverse transform's normalisation), in FP64 and FP32.
__global__ void split_spectrum_kernel(double2* __restrict__ s64, float2* __restrict__ s32,
                                      const double2* __restrict__ E, int n, int d, double scale, long long total) {
  long long id = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= total) return;
  const int L = 2 * n, H = n + 1;
  const int c = (int)(id % L);
  const long long row = id / L;
  const int kl = c < n ? 2 * c : 2 * (c - n) + 1;
  const int fl = kl <= n ? kl : L - kl;
  long long src;
  if (d == 2) {
    src = row + (long long)L * fl;
  } else {
    const int f1 = (int)(row % H), f2 = (int)(row / H);
    src = f1 + (long long)L * f2 + (long long)L * L * fl;
  }
  double2 v = E[src];
  v.x *= scale; v.y *= scale;
  s64[id] = v;
  s32[id] = to_c64(v);
}

}  // namespace

void launch_ktable(double2* k, int n, int d, double omega, double2 k0, hipStream_t st) {
  long long total = 1;
  for (int a = 0; a < d; ++a) total *= (n + 1);
  int bs = 256;
  LSP_LAUNCH("ktable", 0, ktable_kernel, dim3((unsigned)((total + bs - 1) / bs)), dim3(bs), 0, st,
                     k, n, d, 1.0 / n, omega, k0, total);
}

void launch_embed(double2* E, const double2* k, int n, int d, hipStream_t st) {
  long long total = 1;
  for (int a = 0; a < d; ++a) total *= 2 * n;
  int bs = 256;
  LSP_LAUNCH("embed", 0, embed_kernel, dim3((unsigned)((total + bs - 1) / bs)), dim3(bs), 0, st,
                     E, k, n, d, total);
}

void launch_split_spectrum(double2* s64, float2* s32, const double2* E, int n, int d, hipStream_t st) {
  long long total = 2LL * n;
  double scale = 1.0;
  for (int a = 0; a < d; ++a) scale /= 2.0 * n;
  for (int a = 1; a < d; ++a) total *= n + 1;
  int bs = 256;
  LSP_LAUNCH("split_spectrum", 0, split_spectrum_kernel, dim3((unsigned)((total + bs - 1) / bs)), dim3(bs), 0, st,
             s64, s32, E, n, d, scale, total);
}

}  // namespace lsp
