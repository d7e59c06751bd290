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

// ---- the scattered field away from the grid (Section 1)
//
// Section 1 represents the scattered field everywhere through its values on
// Omega; with the grid quadrature of Section 2.1:
//   MODE 0 (points x):      u(x) = - sum_j h^d G(x - x_j) w2m_j (u_j + uI_j)
//                           (k_0 for a grid point j at x itself);
//   MODE 1 (directions xh): A(xh) = - c_d sum_j h^d e^{-i w xh.x_j} w2m_j (u_j + uI_j),
//                           the far-field pattern, u(x) = A e^{i w |x|} |x|^{-(d-1)/2} + ...,
//                           c_2 = e^{i pi/4} / sqrt(8 pi w), c_3 = 1 / (4 pi).
// Work split: a workgroup takes a tile of FT evaluation points (one per
// lane) and a chunk of FC grid points, its four waves every fourth grid
// point of the chunk (the same one across a wave, so grid points with
// w2m = 0 are skipped without divergence); the source density of FS grid
// points for up to FR right-hand sides is staged in LDS; the waves' sums are
// added in wave order and stored per chunk; field_reduce adds the chunks in
// order (the result does not depend on the right-hand sides' grouping).
constexpr int FT = 64, FS = 64, FR = 16, FC = 2048;

template <int MODE>
__global__ void __launch_bounds__(256) field_partial_kernel(const double2* __restrict__ u,
                                                            const double2* __restrict__ uI,
                                                            const double* __restrict__ w2m,
                                                            const double* __restrict__ pts, int npts, int nrhs,
                                                            long long N, int n, int d, double omega, double2 k0,
                                                            double2* __restrict__ partial) {
  __shared__ double2 q[FS * FR];
  __shared__ double wv[FS];
  __shared__ double yc[FS][3];
  __shared__ double2 red[FT * FR];
  const int tile = blockIdx.x, chunk = blockIdx.y;
  const int tid = threadIdx.x, wave = tid / 64, lane = tid % 64;
  const int p = tile * FT + lane;
  const bool live = p < npts;
  const double h = 1.0 / n, hd = d == 2 ? h * h : h * h * h;
  double x[3] = {0.0, 0.0, 0.0};
  if (live)
    for (int a = 0; a < d; ++a) x[a] = pts[(long long)p * d + a];
  double2 acc[FR];
#pragma unroll
  for (int k = 0; k < FR; ++k) acc[k] = make_double2(0, 0);
  const long long j0 = (long long)chunk * FC, j1 = min(N, j0 + FC);
  for (long long s0 = j0; s0 < j1; s0 += FS) {
    const int cnt = (int)min((long long)FS, j1 - s0);
    __syncthreads();  // the previous step's reads of q are done
    for (int e = tid; e < cnt * nrhs; e += 256) {
      const int c = e % cnt, k = e / cnt;
      const long long j = s0 + c;
      const double wj = w2m[j] * hd;
      const double2 a = u[(long long)k * N + j], b = uI[(long long)k * N + j];
      q[c * FR + k] = make_double2(wj * (a.x + b.x), wj * (a.y + b.y));
    }
    for (int c = tid; c < cnt; c += 256) {
      // x_j = (i + 1/2) / n per axis (the same rounding as (i + 0.5) / n on the host)
      const long long j = s0 + c;
      wv[c] = w2m[j];
      yc[c][0] = ((double)(j % n) + 0.5) / n;
      yc[c][1] = ((double)((j / n) % n) + 0.5) / n;
      yc[c][2] = d == 3 ? ((double)(j / ((long long)n * n)) + 0.5) / n : 0.0;
    }
    __syncthreads();
    for (int c = wave; c < cnt; c += 4) {
      if (wv[c] == 0.0) continue;
      const double y0 = yc[c][0], y1 = yc[c][1], y2 = yc[c][2];
      double2 g;
      if (MODE == 0) {
        const double e0 = x[0] - y0, e1 = x[1] - y1, e2 = x[2] - y2;
        const double r = sqrt(e0 * e0 + e1 * e1 + e2 * e2);
        if (r == 0.0) {
          g = make_double2(k0.x / hd, k0.y / hd);
        } else if (d == 2) {
          const double2 H = hankel1_0(omega * r);
          g = make_double2(-0.25 * H.y, 0.25 * H.x);  // (i/4) (J0 + i Y0)
        } else {
          double sn, cs;
          sincos(omega * r, &sn, &cs);
          const double s = 1.0 / (4.0 * kPi * r);
          g = make_double2(cs * s, sn * s);
        }
      } else {
        double sn, cs;
        sincos(-omega * (x[0] * y0 + x[1] * y1 + x[2] * y2), &sn, &cs);
        g = make_double2(cs, sn);
      }
#pragma unroll
      for (int k = 0; k < FR; ++k)
        if (k < nrhs) acc[k] = cadd(acc[k], cmul(g, q[c * FR + k]));
    }
  }
  for (int w = 0; w < 4; ++w) {
    __syncthreads();
    if (wave == w) {
#pragma unroll
      for (int k = 0; k < FR; ++k) red[lane * FR + k] = w == 0 ? acc[k] : cadd(red[lane * FR + k], acc[k]);
    }
  }
  __syncthreads();
  for (int e = tid; e < FT * nrhs; e += 256) {
    const int l = e % FT, k = e / FT, pp = tile * FT + l;
    if (pp < npts) partial[((long long)chunk * nrhs + k) * npts + pp] = red[l * FR + k];
  }
}

__global__ void field_reduce_kernel(const double2* __restrict__ partial, int nchunk, int nrhs, int npts, double2 scale,
                                    double2* __restrict__ out) {
  const long long id = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= (long long)nrhs * npts) return;
  const int k = (int)(id / npts), p = (int)(id % npts);
  double2 s = make_double2(0, 0);
  for (int c = 0; c < nchunk; ++c) s = cadd(s, partial[((long long)c * nrhs + k) * npts + p]);
  out[id] = cmul(scale, s);
}

}  // namespace

long long field_chunks(long long N) { return (N + FC - 1) / FC; }

void field_eval(int mode, const double2* u, const double2* uI, const double* w2m, const double* pts, int npts,
                int nrhs, int n, int d, double omega, double2 k0, double2* partial, double2* out, hipStream_t st) {
  long long N = 1;
  for (int a = 0; a < d; ++a) N *= n;
  const int nchunk = (int)field_chunks(N);
  double2 scale = make_double2(-1.0, 0.0);
  if (mode == 1) {
    if (d == 2) {
      const double a = 1.0 / sqrt(8.0 * kPi * omega), c = 0.70710678118654752440;
      scale = make_double2(-a * c, -a * c);  // -e^{i pi/4} / sqrt(8 pi w)
    } else {
      scale = make_double2(-1.0 / (4.0 * kPi), 0.0);
    }
  }
  for (int r0 = 0; r0 < nrhs; r0 += FR) {
    const int nr = nrhs - r0 < FR ? nrhs - r0 : FR;
    const dim3 grid((unsigned)((npts + FT - 1) / FT), (unsigned)nchunk);
    if (mode == 0)
      LSP_LAUNCH("field_points", 0, field_partial_kernel<0>, grid, dim3(256), 0, st, u + (long long)r0 * N,
                 uI + (long long)r0 * N, w2m, pts, npts, nr, N, n, d, omega, k0, partial);
    else
      LSP_LAUNCH("field_far", 0, field_partial_kernel<1>, grid, dim3(256), 0, st, u + (long long)r0 * N,
                 uI + (long long)r0 * N, w2m, pts, npts, nr, N, n, d, omega, k0, partial);
    const long long tot = (long long)nr * npts;
    LSP_LAUNCH("field_reduce", 0, field_reduce_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, partial,
               nchunk, nr, npts, scale, out + (long long)r0 * npts);
  }
}

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
