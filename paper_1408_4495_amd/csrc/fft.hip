// Zero-padded FFT convolution with the Green's spectrum (the K-matvec).
//
// The convolution y = K v over the n^d grid (eq:lso; Section 1 notes that its
// convolution structure allows FFT application) is computed on the (2n)^d
// circulant embedding: pad v, transform, multiply by the spectrum of the
// embedded kernel, transform back, keep the n^d block.
//
// Transforms are Stockham autosort FFTs (the formulation of Govindaraju et
// al., "High performance discrete Fourier transforms on graphics processors",
// SC 2008) of length L = 2^a 3^b held in LDS, one line per group of
// L/EPT threads, each thread staging EPT values in registers per pass.
// Passes over HBM, per right-hand side (2D):
//   FIRST  rows i2 < n: load w^2 m v (n values), pad, forward FFT along i1
//   CONV   all L columns: load n values, forward FFT along i2, multiply by the
//          spectrum, inverse FFT, store n values
//   LAST   rows i2 < n: inverse FFT along i1, keep n values, add v
// In 3D an axis-2 forward pass runs after FIRST and an axis-2 inverse pass
// before LAST; CONV then runs along i3.  Rows that are zero are never read or
// transformed (pruning).  The 1/L^d normalisation is folded into the spectrum.
#include "lsp_common.h"
#include "kernels.h"

namespace lsp {

namespace {

template <typename T>
__device__ inline cplx<T> twiddle(const cplx<T>* tw, int idx, bool inv) {
  cplx<T> w = tw[idx];
  if (inv) w.y = -w.y;
  return w;
}

template <typename T, int R> struct Dft;

template <typename T> struct Dft<T, 2> {
  __device__ static void run(cplx<T>* v, bool) {
    cplx<T> a = v[0], b = v[1];
    v[0] = cadd(a, b); v[1] = csub(a, b);
  }
};

// -i*z (forward) or +i*z (inverse)
template <typename T> __device__ inline cplx<T> rot90(cplx<T> z, bool inv) {
  return inv ? mk<T>(-z.y, z.x) : mk<T>(z.y, -z.x);
}

template <typename T> struct Dft<T, 4> {
  __device__ static void run(cplx<T>* v, bool inv) {
    cplx<T> a = cadd(v[0], v[2]), b = csub(v[0], v[2]);
    cplx<T> c = cadd(v[1], v[3]), d = csub(v[1], v[3]);
    cplx<T> rd = rot90<T>(d, inv);
    v[0] = cadd(a, c); v[2] = csub(a, c);
    v[1] = cadd(b, rd); v[3] = csub(b, rd);
  }
};

template <typename T> struct Dft<T, 8> {
  __device__ static void run(cplx<T>* v, bool inv) {
    cplx<T> e[4] = {v[0], v[2], v[4], v[6]};
    cplx<T> o[4] = {v[1], v[3], v[5], v[7]};
    Dft<T, 4>::run(e, inv);
    Dft<T, 4>::run(o, inv);
    const T r = (T)0.70710678118654752440;
    // o_k *= W8^k, W8 = exp(-+ 2 pi i / 8)
    cplx<T> o1 = o[1], o3 = o[3];
    if (!inv) {
      o[1] = mk<T>((o1.x + o1.y) * r, (o1.y - o1.x) * r);
      o[3] = mk<T>((-o3.x + o3.y) * r, (-o3.y - o3.x) * r);
    } else {
      o[1] = mk<T>((o1.x - o1.y) * r, (o1.y + o1.x) * r);
      o[3] = mk<T>((-o3.x - o3.y) * r, (-o3.y + o3.x) * r);
    }
    o[2] = rot90<T>(o[2], inv);
    for (int k = 0; k < 4; ++k) {
      v[k] = cadd(e[k], o[k]);
      v[k + 4] = csub(e[k], o[k]);
    }
  }
};

template <typename T> struct Dft<T, 3> {
  __device__ static void run(cplx<T>* v, bool inv) {
    const T s3 = (T)0.86602540378443864676;  // sqrt(3)/2
    cplx<T> t = cadd(v[1], v[2]);
    cplx<T> dd = csub(v[1], v[2]);
    cplx<T> m = mk<T>(v[0].x - (T)0.5 * t.x, v[0].y - (T)0.5 * t.y);
    // forward: y1 = m - i s3 d, y2 = m + i s3 d
    cplx<T> isd = mk<T>(-s3 * dd.y, s3 * dd.x);  // i * s3 * d
    v[0] = cadd(v[0], t);
    if (!inv) { v[1] = csub(m, isd); v[2] = cadd(m, isd); }
    else { v[1] = cadd(m, isd); v[2] = csub(m, isd); }
  }
};

// One Stockham pass of radix R over a line in LDS.
template <typename T, int R, int EPT>
__device__ inline void fft_pass(cplx<T>* s, int L, int P, int t, int Ns, const cplx<T>* tw, bool inv) {
  constexpr int NB = EPT / R;
  cplx<T> v[NB][R];
  const int stride = L / R;
  const int tstep = L / (Ns * R);
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    int j = t + b * P;
    int k = j % Ns;
#pragma unroll
    for (int r = 0; r < R; ++r) v[b][r] = s[j + r * stride];
#pragma unroll
    for (int r = 1; r < R; ++r) v[b][r] = cmul(v[b][r], twiddle<T>(tw, r * k * tstep, inv));
  }
  __syncthreads();
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    Dft<T, R>::run(v[b], inv);
    int j = t + b * P;
    int k = j % Ns;
    int base = (j - k) * R + k;
#pragma unroll
    for (int r = 0; r < R; ++r) s[base + r * Ns] = v[b][r];
  }
  __syncthreads();
}

template <typename T, int EPT>
__device__ inline void fft_line(cplx<T>* s, int L, int P, int t, const cplx<T>* tw, FftRadices rad, bool inv) {
  int Ns = 1;
  for (int ip = 0; ip < rad.npass; ++ip) {
    int R = rad.r[ip];
    if constexpr (EPT % 8 == 0) { if (R == 8) fft_pass<T, 8, EPT>(s, L, P, t, Ns, tw, inv); }
    if constexpr (EPT % 4 == 0) { if (R == 4) fft_pass<T, 4, EPT>(s, L, P, t, Ns, tw, inv); }
    if constexpr (EPT % 2 == 0) { if (R == 2) fft_pass<T, 2, EPT>(s, L, P, t, Ns, tw, inv); }
    if constexpr (EPT % 3 == 0) { if (R == 3) fft_pass<T, 3, EPT>(s, L, P, t, Ns, tw, inv); }
    Ns *= R;
  }
}

__device__ inline int fold(int k, int L) { return k <= L / 2 ? k : L - k; }

inline const char* fft_mode_name(int mode) {
  static const char* names[4] = {"fft_axis", "fft_first", "fft_conv", "fft_last"};
  return names[mode & 3];
}

// Generic line kernel.  Lines are indexed by (c, o): c in [0, ncols) runs over
// LPW consecutive lines per workgroup, o over blockIdx.y; rhs over blockIdx.z.
// Element e of line (c, o) of the work array sits at c*cs + o*os + e*es.
//   MODE_PLAIN: read rl values of W (rest zero), FFT, write wl values of W.
//   MODE_FIRST: line c is grid row c of the field x (n contiguous values):
//               read w2m .* x (or x when w2m is null), forward FFT, write L values.
//   MODE_CONV:  read rl, forward FFT, multiply by the spectrum, inverse FFT, write wl.
//   MODE_LAST:  read L values of row c, inverse FFT, write n values to y
//               (y = x + v when x is given, else y = v).
enum { MODE_PLAIN = 0, MODE_FIRST = 1, MODE_CONV = 2, MODE_LAST = 3 };

struct LineArgs {
  int n, d, L, P, LPW, Lp;
  int ncols;
  long long cs, os, es;
  int rl, wl;
  int inv;
  long long wstride;          // per-rhs stride of the work array
  long long fstride;          // per-rhs stride of fields (N)
};

template <typename T, int EPT, int MODE>
__global__ void __launch_bounds__(1024) fft_lines_kernel(cplx<T>* __restrict__ W, const double2* __restrict__ x,
                                                         double2* __restrict__ y, const double* __restrict__ w2m,
                                                         const cplx<T>* __restrict__ khat, const cplx<T>* __restrict__ tw,
                                                         FftRadices rad, LineArgs a) {
  extern __shared__ unsigned char smem_raw[];
  cplx<T>* smem = reinterpret_cast<cplx<T>*>(smem_raw);
  const int tid = threadIdx.x;
  const int nthr = blockDim.x;
  // Workgroups go to the 8 XCDs round-robin (workgroup b to XCD b mod 8),
  // each XCD with its own L2: give each XCD a contiguous range of line
  // blocks, so that the lines sharing cache lines in a strided pass (16
  // complex64 or 8 complex128 per 128 bytes) are read through one L2.
  const int bx = gridDim.x % 8 == 0 ? (blockIdx.x % 8) * (gridDim.x / 8) + blockIdx.x / 8 : blockIdx.x;
  const int c0 = bx * a.LPW;
  const int o = blockIdx.y;
  const int rhs = blockIdx.z;
  const int nl = min(a.LPW, a.ncols - c0);
  cplx<T>* Wr = W + rhs * a.wstride;
  const int L = a.L, Lp = a.Lp;

  // ---- load
  if (MODE == MODE_FIRST) {
    const double2* xr = x + rhs * a.fstride;
    for (int idx = tid; idx < a.LPW * L; idx += nthr) {
      int line = idx / L, e = idx % L;
      cplx<T> v = mk<T>(0, 0);
      if (line < nl && e < a.n) {
        long long g = (long long)(c0 + line) * a.n + e;
        double2 xv = xr[g];
        double s = w2m ? w2m[g] : 1.0;
        v = mk<T>((T)(xv.x * s), (T)(xv.y * s));
      }
      smem[line * Lp + e] = v;
    }
  } else if (MODE == MODE_LAST) {
    for (int idx = tid; idx < a.LPW * L; idx += nthr) {
      int line = idx / L, e = idx % L;
      cplx<T> v = mk<T>(0, 0);
      if (line < nl) {
        int c = c0 + line;
        long long base = (long long)(c % a.n) * L + (long long)(c / a.n) * L * L;
        v = Wr[base + e];
      }
      smem[line * Lp + e] = v;
    }
  } else {
    const long long obase = (long long)o * a.os;
    if (a.es == 1) {
      for (int idx = tid; idx < a.LPW * L; idx += nthr) {
        int line = idx / L, e = idx % L;
        cplx<T> v = mk<T>(0, 0);
        if (line < nl && e < a.rl) v = Wr[(long long)(c0 + line) * a.cs + obase + e];
        smem[line * Lp + e] = v;
      }
    } else {
      for (int idx = tid; idx < a.LPW * L; idx += nthr) {
        int line = idx % a.LPW, e = idx / a.LPW;
        cplx<T> v = mk<T>(0, 0);
        if (line < nl && e < a.rl) v = Wr[(long long)(c0 + line) * a.cs + obase + (long long)e * a.es];
        smem[line * Lp + e] = v;
      }
    }
  }
  __syncthreads();

  // ---- transform(s)
  const int line = tid / a.P, t = tid % a.P;
  cplx<T>* s = smem + line * Lp;
  bool inv = a.inv != 0;
  if (MODE == MODE_FIRST) inv = false;
  if (MODE == MODE_LAST) inv = true;
  if (MODE == MODE_CONV) inv = false;
  fft_line<T, EPT>(s, L, a.P, t, tw, rad, inv);
  if (MODE == MODE_CONV) {
    // multiply by the folded spectrum
    const int H = a.n + 1;
    if (line < nl) {
      int c = c0 + line;
      long long kb;
      int k1 = c % L;
      if (a.d == 2) kb = fold(k1, L);
      else kb = fold(k1, L) + (long long)H * fold(c / L, L);
      long long lstride = (a.d == 2) ? H : (long long)H * H;
      for (int e = t; e < L; e += a.P) s[e] = cmul(s[e], khat[kb + fold(e, L) * lstride]);
    }
    __syncthreads();
    fft_line<T, EPT>(s, L, a.P, t, tw, rad, true);
  }

  // ---- store
  if (MODE == MODE_FIRST) {
    for (int idx = tid; idx < a.LPW * L; idx += nthr) {
      int ln = idx / L, e = idx % L;
      if (ln < nl) {
        int c = c0 + ln;
        long long base = (long long)(c % a.n) * L + (long long)(c / a.n) * L * L;
        Wr[base + e] = smem[ln * Lp + e];
      }
    }
  } else if (MODE == MODE_LAST) {
    const double2* xr = x ? x + rhs * a.fstride : nullptr;
    double2* yr = y + rhs * a.fstride;
    for (int idx = tid; idx < a.LPW * a.n; idx += nthr) {
      int ln = idx / a.n, e = idx % a.n;
      if (ln < nl) {
        long long g = (long long)(c0 + ln) * a.n + e;
        double2 v = widen(smem[ln * Lp + e]);
        if (xr) { double2 xv = xr[g]; v.x += xv.x; v.y += xv.y; }
        yr[g] = v;
      }
    }
  } else {
    const long long obase = (long long)o * a.os;
    if (a.es == 1) {
      for (int idx = tid; idx < a.LPW * L; idx += nthr) {
        int ln = idx / L, e = idx % L;
        if (ln < nl && e < a.wl) Wr[(long long)(c0 + ln) * a.cs + obase + e] = smem[ln * Lp + e];
      }
    } else {
      for (int idx = tid; idx < a.LPW * L; idx += nthr) {
        int ln = idx % a.LPW, e = idx / a.LPW;
        if (ln < nl && e < a.wl) Wr[(long long)(c0 + ln) * a.cs + obase + (long long)e * a.es] = smem[ln * Lp + e];
      }
    }
  }
}

template <typename T>
int lines_per_wg(int L, int P, long long total_lines) {
  // up to 132 KB of the 160 KB LDS a gfx950 workgroup may use; a power of two
  // so that strided passes read aligned runs of consecutive lines; and no more
  // lines per workgroup than keeps about 512 workgroups in flight
  size_t per_line = (size_t)(L + 1) * sizeof(cplx<T>);
  int cap = (int)((132 * 1024) / per_line);
  long long want = std::max<long long>(1, total_lines / 512);
  int lpw = 1;
  while (lpw * 2 <= std::min<long long>(std::min(cap, 16), want) && lpw * 2 * P <= 1024) lpw *= 2;
  return lpw;
}

template <typename T, int EPT, int MODE>
void launch_lines(const FftPlanDev<T>& fp, cplx<T>* W, const double2* x, double2* y, const double* w2m,
                  int ncols, int nouter, long long cs, long long os, long long es, int rl, int wl, int inv,
                  int nrhs, hipStream_t st) {
  LineArgs a;
  a.n = fp.n; a.d = fp.d; a.L = fp.L; a.P = fp.L / EPT;
  a.LPW = lines_per_wg<T>(fp.L, a.P, (long long)ncols * nouter * nrhs);
  a.Lp = fp.L + 1;
  a.ncols = ncols; a.cs = cs; a.os = os; a.es = es; a.rl = rl; a.wl = wl; a.inv = inv;
  a.wstride = fp.wstride; a.fstride = fp.N;
  dim3 grid((ncols + a.LPW - 1) / a.LPW, nouter, nrhs);
  dim3 block(a.LPW * a.P);
  size_t lds = (size_t)a.LPW * a.Lp * sizeof(cplx<T>);
  LSP_LAUNCH(fft_mode_name(MODE), (int)sizeof(cplx<T>), (fft_lines_kernel<T, EPT, MODE>), grid, block, lds, st, W, x, y, w2m, fp.khat, fp.tw,
                     fp.rad, a);
}

template <typename T, int EPT>
void kmatvec_impl(const FftPlanDev<T>& fp, int nrhs, const double2* x, double2* y, const double* w2m,
                  bool add_x, cplx<T>* W, hipStream_t st) {
  const int n = fp.n, L = fp.L;
  const long long LL = (long long)L * L;
  if (fp.d == 2) {
    launch_lines<T, EPT, MODE_FIRST>(fp, W, x, y, w2m, n, 1, 0, 0, 1, n, L, 0, nrhs, st);
    launch_lines<T, EPT, MODE_CONV>(fp, W, x, y, w2m, L, 1, 1, 0, L, n, n, 0, nrhs, st);
    launch_lines<T, EPT, MODE_LAST>(fp, W, add_x ? x : nullptr, y, w2m, n, 1, 0, 0, 1, L, n, 1, nrhs, st);
  } else {
    launch_lines<T, EPT, MODE_FIRST>(fp, W, x, y, w2m, n * n, 1, 0, 0, 1, n, L, 0, nrhs, st);
    // axis 2 forward: lines (k1, i3 < n), elements along i2 (stride L)
    launch_lines<T, EPT, MODE_PLAIN>(fp, W, x, y, w2m, L, n, 1, LL, L, n, L, 0, nrhs, st);
    // axis 3 convolution: lines (k1 + L k2), elements along i3 (stride L^2)
    launch_lines<T, EPT, MODE_CONV>(fp, W, x, y, w2m, L * L, 1, 1, 0, LL, n, n, 0, nrhs, st);
    // axis 2 inverse
    launch_lines<T, EPT, MODE_PLAIN>(fp, W, x, y, w2m, L, n, 1, LL, L, L, n, 1, nrhs, st);
    launch_lines<T, EPT, MODE_LAST>(fp, W, add_x ? x : nullptr, y, w2m, n * n, 1, 0, 0, 1, L, n, 1, nrhs, st);
  }
}

template <typename T, int EPT>
void full_fft_impl(const FftPlanDev<T>& fp, cplx<T>* W, hipStream_t st) {
  const int L = fp.L;
  const long long LL = (long long)L * L;
  if (fp.d == 2) {
    launch_lines<T, EPT, MODE_PLAIN>(fp, W, nullptr, nullptr, nullptr, L, 1, L, 0, 1, L, L, 0, 1, st);
    launch_lines<T, EPT, MODE_PLAIN>(fp, W, nullptr, nullptr, nullptr, L, 1, 1, 0, L, L, L, 0, 1, st);
  } else {
    launch_lines<T, EPT, MODE_PLAIN>(fp, W, nullptr, nullptr, nullptr, L * L, 1, L, 0, 1, L, L, 0, 1, st);
    launch_lines<T, EPT, MODE_PLAIN>(fp, W, nullptr, nullptr, nullptr, L, L, 1, LL, L, L, L, 0, 1, st);
    launch_lines<T, EPT, MODE_PLAIN>(fp, W, nullptr, nullptr, nullptr, (int)LL, 1, 1, 0, LL, L, L, 0, 1, st);
  }
}

}  // namespace

template <typename T>
void kmatvec(const FftPlanDev<T>& fp, int nrhs, const double2* x, double2* y, const double* w2m, bool add_x,
             cplx<T>* W, hipStream_t st) {
  if (fp.ept == 8) kmatvec_impl<T, 8>(fp, nrhs, x, y, w2m, add_x, W, st);
  else if (fp.ept == 12) kmatvec_impl<T, 12>(fp, nrhs, x, y, w2m, add_x, W, st);
  else if (fp.ept == 6) kmatvec_impl<T, 6>(fp, nrhs, x, y, w2m, add_x, W, st);
  else throw Error(LSP_ERR_ARG, "unsupported FFT length");
}

template <typename T>
void full_fft_forward(const FftPlanDev<T>& fp, cplx<T>* W, hipStream_t st) {
  if (fp.ept == 8) full_fft_impl<T, 8>(fp, W, st);
  else if (fp.ept == 12) full_fft_impl<T, 12>(fp, W, st);
  else if (fp.ept == 6) full_fft_impl<T, 6>(fp, W, st);
  else throw Error(LSP_ERR_ARG, "unsupported FFT length");
}

template void kmatvec<double>(const FftPlanDev<double>&, int, const double2*, double2*, const double*, bool,
                              double2*, hipStream_t);
template void kmatvec<float>(const FftPlanDev<float>&, int, const double2*, double2*, const double*, bool,
                             float2*, hipStream_t);
template void full_fft_forward<double>(const FftPlanDev<double>&, double2*, hipStream_t);

}  // namespace lsp
