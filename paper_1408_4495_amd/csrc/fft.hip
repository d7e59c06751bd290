// Zero-padded FFT convolution with the Green's spectrum (the K-matvec).
//
// y = K v over the n^d grid (eq:lso; Section 1 notes that its convolution
// structure allows FFT application) is the n^d block of the circular
// convolution on the (2n)^d embedding: pad v, transform, multiply by the
// spectrum of the embedded kernel, transform back.
//
// Half-length transforms.  With L = 2n and v zero beyond n along an axis, a
// length-L transform of v splits into two length-n ones,
//   X[2k] = DFT_n(v)[k],   X[2k+1] = DFT_n(v_j w^j)[k],   w = exp(-2 pi i / L),
// and the first n outputs of a length-L inverse are
//   y_j = IDFT_n(Y[2k])_j + w^-j IDFT_n(Y[2k+1])_j.
// The work array keeps every transformed axis in this split order (the n
// even frequencies, then the n odd ones), so each transform of the K-matvec
// is an n-point one over data that is nonzero, and the spectrum is stored in
// the same order (one row of L values per frequency of the other axes, see
// the set-up in greens.hip).  Passes over HBM per right-hand side:
//   2D  FIRST  rows i2 < n: w^2 m v (n values), two forward transforms along
//              i1, L values out (split order)
//       CONV   all L columns: n values, two forward transforms along i2, times
//              the spectrum, two inverse transforms, n values back in place
//       LAST   rows i2 < n: L values, two inverse transforms along i1, n
//              values out (plus v for the operator)
//   3D  FIRST, then the forward pass along i2 for i3 < n (n values in, L out),
//       CONV along i3 over all L^2 lines, the inverse pass along i2, LAST.
//
// n-point transforms are Stockham autosort FFTs (the formulation of
// Govindaraju et al., "High performance discrete Fourier transforms on
// graphics processors", SC 2008), n = 2^a 3^b, P = n / EPT threads per line.
// Thread t owns elements t + m P (m < EPT) before and after a transform: the
// first radix pass takes them from registers and the last leaves them there,
// so only the passes in between exchange through LDS (one pad element per 16
// against bank conflicts).  The two n-point transforms of a line (even and
// odd half) are independent and run in lockstep: each pass loads its
// twiddles once for both and the pair shares the pass's barriers, each
// half in its own bank of LDS lines.  Lines along a strided axis are handed to
// consecutive lanes (lane = line + LPW t), so a load or store of element e
// covers LPW adjacent lines' contiguous entries.
//
// The set-up's transform of the full embedded kernel (all L values nonzero)
// uses the plain full-length line kernel at the end of this file.
#include "lsp_common.h"
#include "kernels.h"

namespace lsp {

namespace {

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

__device__ inline int fold(int k, int L) { return k <= L / 2 ? k : L - k; }

// ---------------------------------------------------------------- half-length transforms

constexpr int kHalfThreads = 256;          // largest workgroup of the half-length kernels
constexpr size_t kHalfLds = 72 * 1024;     // LDS per workgroup (two banks of lines)

__host__ __device__ __forceinline__ int padi(int e) { return e + (e >> 4); }

// Twiddles of a pass (radix R, span Ns): for butterfly b (k = (t + b P) mod
// Ns, idx = k L / (Ns R), tw[i] = w^i) the powers w^idx, w^(2 idx) and, for
// R = 8, w^(4 idx) are loaded; the other powers are products of at most two
// loaded ones (a bounded rounding depth).
template <int R> struct TwLoads { static constexpr int value = R == 2 ? 1 : (R == 8 ? 3 : 2); };

// P2: Ns and L are powers of two (modulo and division by masks and shifts).
template <typename T, int R, int NB, bool P2>
__device__ __forceinline__ void load_tw(cplx<T> (&wt)[NB * TwLoads<R>::value], const int t, const int P,
                                        const int Ns, const int L, const cplx<T>* __restrict__ tw) {
  constexpr int NL = TwLoads<R>::value;
  const int tstep = P2 ? L >> (31 - __builtin_clz(Ns * R)) : L / (Ns * R);
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    const int idx = (P2 ? (t + b * P) & (Ns - 1) : (t + b * P) % Ns) * tstep;
    wt[NL * b] = tw[idx];
    if constexpr (NL >= 2) wt[NL * b + 1] = tw[2 * idx];
    if constexpr (NL >= 3) wt[NL * b + 2] = tw[4 * idx];
  }
}

template <typename T, bool INV>
__device__ __forceinline__ cplx<T> twc(cplx<T> w) { return INV ? cconj(w) : w; }

template <typename T, int R, bool INV>
__device__ __forceinline__ void apply_tw(cplx<T> (&v)[R], const cplx<T>* w) {
  const cplx<T> w1 = twc<T, INV>(w[0]);
  v[1] = cmul(v[1], w1);
  if constexpr (R >= 3) {
    const cplx<T> w2 = twc<T, INV>(w[1]);
    v[2] = cmul(v[2], w2);
    if constexpr (R >= 4) {
      const cplx<T> w3 = cmul(w1, w2);
      v[3] = cmul(v[3], w3);
      if constexpr (R == 8) {
        const cplx<T> w4 = twc<T, INV>(w[2]);
        v[4] = cmul(v[4], w4);
        v[5] = cmul(v[5], cmul(w1, w4));
        v[6] = cmul(v[6], cmul(w2, w4));
        v[7] = cmul(v[7], cmul(w3, w4));
      }
    }
  }
}

// One radix-R pass of K n-point transforms in lockstep (the even and odd
// halves of a line: same length, same twiddles), line k in LDS at
// s + k sstep (padded index).  a[k][m] holds element t + m P of transform k:
// read by the first pass, written by the last; the other passes read and
// write LDS.  The K transforms share the twiddle loads and the barriers.
// CARRY: the twiddles of this pass are in wt8 (loaded by the previous pass)
// and those of the next pass, a radix-8 one, are loaded here, a pass ahead
// of their use; otherwise the pass loads its own.
template <typename T, int R, int EPT, int K, bool INV, bool CARRY>
__device__ __forceinline__ void half_pass(cplx<T> (&a)[K][EPT], cplx<T> (&wt8)[3], cplx<T>* __restrict__ s,
                                          const int sstep, const int t, const int P, const int n, const int L,
                                          const int Ns, const bool first, const bool last,
                                          const cplx<T>* __restrict__ tw) {
  constexpr int NB = EPT / R;
  constexpr int NL = TwLoads<R>::value;
  const int q = n / R;
  cplx<T> v[K][NB][R];
  if (first) {
#pragma unroll
    for (int k = 0; k < K; ++k)
#pragma unroll
      for (int b = 0; b < NB; ++b)
#pragma unroll
        for (int r = 0; r < R; ++r) v[k][b][r] = a[k][b + r * NB];
  } else {
#pragma unroll
    for (int k = 0; k < K; ++k)
#pragma unroll
      for (int b = 0; b < NB; ++b)
#pragma unroll
        for (int r = 0; r < R; ++r) v[k][b][r] = s[k * sstep + padi(t + b * P + r * q)];
  }
  if (!first) {
    if constexpr (CARRY) {
      // carried twiddles are radix-8 ones (the radix-2 and radix-4 passes
      // of a carried schedule are first passes)
      if constexpr (R == 8) {
#pragma unroll
        for (int k = 0; k < K; ++k) apply_tw<T, 8, INV>(v[k][0], wt8);
      }
    } else {
      cplx<T> wt[NB * NL];
      load_tw<T, R, NB, false>(wt, t, P, Ns, L, tw);
#pragma unroll
      for (int k = 0; k < K; ++k)
#pragma unroll
        for (int b = 0; b < NB; ++b) apply_tw<T, R, INV>(v[k][b], wt + NL * b);
    }
  }
  if constexpr (CARRY) {
    if (!last) load_tw<T, 8, 1, true>(wt8, t, P, Ns * R, L, tw);
  }
#pragma unroll
  for (int k = 0; k < K; ++k)
#pragma unroll
    for (int b = 0; b < NB; ++b) Dft<T, R>::run(v[k][b], INV);
  if (last) {
#pragma unroll
    for (int k = 0; k < K; ++k)
#pragma unroll
      for (int b = 0; b < NB; ++b)
#pragma unroll
        for (int r = 0; r < R; ++r) a[k][b + r * NB] = v[k][b][r];
  } else {
    __syncthreads();  // every earlier read of the lines is complete
#pragma unroll
    for (int k = 0; k < K; ++k)
#pragma unroll
      for (int b = 0; b < NB; ++b) {
        // (a carried schedule is the n = 2^a one: Ns is a power of two)
        const int j = t + b * P, kk = CARRY ? j & (Ns - 1) : j % Ns, base = (j - kk) * R + kk;
#pragma unroll
        for (int r = 0; r < R; ++r) s[k * sstep + padi(base + r * Ns)] = v[k][b][r];
      }
    __syncthreads();
  }
}

// n = 2^a (EPT = 8): a radix 2, 4 or 8 pass, then radix-8 passes, the
// twiddles of each radix-8 pass loaded a pass ahead.  n = 2^a 3^b: passes
// of radix 4, 2, 3 in the plan's order, each loading its own twiddles.
template <typename T, int EPT, int K, bool INV>
__device__ __forceinline__ void fft_half(cplx<T> (&a)[K][EPT], cplx<T>* __restrict__ s, const int sstep,
                                         const int t, const int P, const int n, const int L, const FftRadices& hr,
                                         const cplx<T>* __restrict__ tw) {
  cplx<T> wt8[3];
  if constexpr (EPT == 8) {
    const int R0 = hr.r[0], np = hr.npass;
    if (R0 == 8) half_pass<T, 8, 8, K, INV, true>(a, wt8, s, sstep, t, P, n, L, 1, true, np == 1, tw);
    else if (R0 == 4) half_pass<T, 4, 8, K, INV, true>(a, wt8, s, sstep, t, P, n, L, 1, true, np == 1, tw);
    else half_pass<T, 2, 8, K, INV, true>(a, wt8, s, sstep, t, P, n, L, 1, true, np == 1, tw);
    int Ns = R0;
    for (int ip = 1; ip < np; ++ip) {
      half_pass<T, 8, 8, K, INV, true>(a, wt8, s, sstep, t, P, n, L, Ns, false, ip + 1 == np, tw);
      Ns *= 8;
    }
  } else {
    int Ns = 1;
    for (int ip = 0; ip < hr.npass; ++ip) {
      const int R = hr.r[ip];
      const bool first = ip == 0, last = ip + 1 == hr.npass;
      if constexpr (EPT % 4 == 0) { if (R == 4) half_pass<T, 4, EPT, K, INV, false>(a, wt8, s, sstep, t, P, n, L, Ns, first, last, tw); }
      if constexpr (EPT % 2 == 0) { if (R == 2) half_pass<T, 2, EPT, K, INV, false>(a, wt8, s, sstep, t, P, n, L, Ns, first, last, tw); }
      if constexpr (EPT % 3 == 0) { if (R == 3) half_pass<T, 3, EPT, K, INV, false>(a, wt8, s, sstep, t, P, n, L, Ns, first, last, tw); }
      Ns *= R;
    }
  }
}

enum { HK_FWD_FIELD = 0, HK_FWD_WORK = 1, HK_CONV = 2, HK_INV_WORK = 3, HK_INV_FIELD = 4 };

const char* half_name(int kind) {
  static const char* names[5] = {"fft_first", "fft_axis_fwd", "fft_conv", "fft_axis_inv", "fft_last"};
  return names[kind];
}

struct HalfArgs {
  int n, L, d, P, LPW, Lp;
  int ncols, nout, nrhs;
  int ncb, GS;                 // line blocks of LPW lines; blocks per cache-line group
  long long cs, os, es;        // work-array line (c, o): element e at c cs + o os + e es
  long long wstride, fstride;  // per right-hand side: work array (L^d), fields (N)
  long long lr;                // row stride of the work array (L, padded in 2D)
  FftRadices hr;               // radices of n
};

// Line (c, o) of right-hand side rhs, by kind:
//   FWD_FIELD  field row c (n contiguous values, scaled by w2m when given) ->
//              work row c: L values at (c mod n) lr + (c div n) lr L (lr:
//              the work rows' stride, L + 16 in 2D so that a column's
//              entries are not a power of two apart and spread over the
//              L2's sets)
//   FWD_WORK   n values of the work line -> L values of the same line
//   CONV       n values -> n values in place, spectrum row of line c
//   INV_WORK   L values of the work line -> its first n values
//   INV_FIELD  work row c (L values) -> field row c (plus x when given;
//              zero where the output mask, passed in place of w2m, is 0)
// Workgroups: LPW lines of one (o, rhs), line = tid / P, t = tid % P, with
// two banks of LPW lines in LDS (the even and odd halves' transforms).  The
// GS blocks whose lines share cache lines, then the right-hand sides of a
// line block (sharing spectrum rows), are consecutive in dispatch order
// within one XCD (workgroup b goes to XCD b mod 8).  TIO: a strided line's
// loads and stores go through LDS, lane tid handling element tid / LPW +
// m P of line tid % LPW, so that one load or store covers LPW adjacent
// lines' entries (used when P lanes of one line would otherwise read single
// entries of separate cache lines).
template <typename T, int EPT, int KIND, bool TIO>
__global__ void __launch_bounds__(kHalfThreads) half_lines_kernel(cplx<T>* __restrict__ W,
                                                                  const double2* __restrict__ x,
                                                                  double2* __restrict__ y,
                                                                  const double* __restrict__ w2m,
                                                                  const cplx<T>* __restrict__ spec,
                                                                  const cplx<T>* __restrict__ tw, HalfArgs a) {
  extern __shared__ unsigned char smem_raw[];
  const int G = gridDim.x;
  const int g = G % 8 == 0 ? (int)(blockIdx.x % 8) * (G / 8) + (int)(blockIdx.x / 8) : (int)blockIdx.x;
  const int j = g % a.GS;
  const int rest = g / a.GS;
  const int rhs = rest % a.nrhs;
  const int rest2 = rest / a.nrhs;
  const int o = rest2 % a.nout;
  const int cb = (rest2 / a.nout) * a.GS + j;
  if (cb >= a.ncb) return;  // the last group's spare blocks (whole workgroups)
  const int tid = threadIdx.x;
  const int n = a.n, L = a.L, P = a.P;
  const int line = tid / P, t = tid % P;
  const int c = cb * a.LPW + line;
  const bool live = c < a.ncols;
  const int cc = live ? c : a.ncols - 1;  // lines past the end load in range and store nothing
  cplx<T>* smem = reinterpret_cast<cplx<T>*>(smem_raw);
  cplx<T>* s = smem + line * a.Lp;
  cplx<T>* Wr = W + rhs * a.wstride;
  // IO lanes of TIO kinds
  const int lio = tid % a.LPW, tio = tid / a.LPW;
  const int cio = cb * a.LPW + lio;
  const bool live_io = cio < a.ncols;
  const int ccio = live_io ? cio : a.ncols - 1;
  cplx<T>* sio = smem + lio * a.Lp;

  // n values of this thread's work line from offset off (element e at
  // base + off + e es) into d[m] = element t + m P
  // (first: nothing has used the LDS lines yet, so the loads go straight
  // to them)
  auto load_work = [&](const long long off, cplx<T> (&d)[EPT], const bool first) {
    if constexpr (TIO) {
      const long long base = ccio * a.cs + o * a.os + off;
      if (!first) __syncthreads();  // earlier reads of the lines are complete
#pragma unroll
      for (int m = 0; m < EPT; ++m) sio[padi(tio + m * P)] = Wr[base + (long long)(tio + m * P) * a.es];
      __syncthreads();
#pragma unroll
      for (int m = 0; m < EPT; ++m) d[m] = s[padi(t + m * P)];
    } else {
      const long long base = cc * a.cs + o * a.os + off;
#pragma unroll
      for (int m = 0; m < EPT; ++m) d[m] = Wr[base + (long long)(t + m * P) * a.es];
    }
  };
  auto store_work = [&](const long long off, const cplx<T> (&d)[EPT]) {
    if constexpr (TIO) {
      __syncthreads();  // earlier reads of the lines are complete
#pragma unroll
      for (int m = 0; m < EPT; ++m) s[padi(t + m * P)] = d[m];
      __syncthreads();
      if (live_io) {
        const long long base = ccio * a.cs + o * a.os + off;
#pragma unroll
        for (int m = 0; m < EPT; ++m) Wr[base + (long long)(tio + m * P) * a.es] = sio[padi(tio + m * P)];
      }
    } else {
      if (live) {
        const long long base = cc * a.cs + o * a.os + off;
#pragma unroll
        for (int m = 0; m < EPT; ++m) Wr[base + (long long)(t + m * P) * a.es] = d[m];
      }
    }
  };

  // the even and odd halves of a line run as two transforms in lockstep,
  // line k of the pair in LDS at s + k sstep
  const int sstep = a.LPW * a.Lp;
  cplx<T> v[2][EPT];
  if constexpr (KIND == HK_FWD_FIELD) {
    const long long fb = (long long)cc * n;
    const double2* xr = x + rhs * a.fstride;
#pragma unroll
    for (int m = 0; m < EPT; ++m) {
      const int e = t + m * P;
      const double2 xv = xr[fb + e];
      const double sc = w2m ? w2m[fb + e] : 1.0;
      v[0][m] = mk<T>((T)(xv.x * sc), (T)(xv.y * sc));
      v[1][m] = cmul(v[0][m], tw[e]);
    }
    const long long wb = (long long)(cc % n) * a.lr + (long long)(cc / n) * a.lr * L;
    fft_half<T, EPT, 2, false>(v, s, sstep, t, P, n, L, a.hr, tw);
    if (live) {
#pragma unroll
      for (int m = 0; m < EPT; ++m) Wr[wb + t + m * P] = v[0][m];
#pragma unroll
      for (int m = 0; m < EPT; ++m) Wr[wb + n + t + m * P] = v[1][m];
    }
  } else if constexpr (KIND == HK_FWD_WORK) {
    load_work(0, v[0], true);
#pragma unroll
    for (int m = 0; m < EPT; ++m) v[1][m] = cmul(v[0][m], tw[t + m * P]);
    fft_half<T, EPT, 2, false>(v, s, sstep, t, P, n, L, a.hr, tw);
    store_work(0, v[0]);
    store_work((long long)n * a.es, v[1]);
  } else if constexpr (KIND == HK_CONV) {
    long long row;
    {
      const int H = n + 1;
      const int c1 = a.d == 2 ? cc : cc % L;
      const int k1 = c1 < n ? 2 * c1 : 2 * (c1 - n) + 1;
      row = fold(k1, L);
      if (a.d == 3) {
        const int c2 = cc / L;
        const int k2 = c2 < n ? 2 * c2 : 2 * (c2 - n) + 1;
        row += (long long)H * fold(k2, L);
      }
    }
    const cplx<T>* sp = spec + row * L;
    load_work(0, v[0], true);
#pragma unroll
    for (int m = 0; m < EPT; ++m) v[1][m] = cmul(v[0][m], tw[t + m * P]);
    fft_half<T, EPT, 2, false>(v, s, sstep, t, P, n, L, a.hr, tw);
#pragma unroll
    for (int m = 0; m < EPT; ++m) { v[0][m] = cmul(v[0][m], sp[t + m * P]); v[1][m] = cmul(v[1][m], sp[n + t + m * P]); }
    fft_half<T, EPT, 2, true>(v, s, sstep, t, P, n, L, a.hr, tw);
#pragma unroll
    for (int m = 0; m < EPT; ++m) v[0][m] = cadd(v[0][m], cmulc(tw[t + m * P], v[1][m]));
    store_work(0, v[0]);
  } else if constexpr (KIND == HK_INV_WORK) {
    load_work(0, v[0], true);
    load_work((long long)n * a.es, v[1], false);
    fft_half<T, EPT, 2, true>(v, s, sstep, t, P, n, L, a.hr, tw);
#pragma unroll
    for (int m = 0; m < EPT; ++m) v[0][m] = cadd(v[0][m], cmulc(tw[t + m * P], v[1][m]));
    store_work(0, v[0]);
  } else {  // HK_INV_FIELD
    const long long wb = (long long)(cc % n) * a.lr + (long long)(cc / n) * a.lr * L;
#pragma unroll
    for (int m = 0; m < EPT; ++m) v[0][m] = Wr[wb + t + m * P];
#pragma unroll
    for (int m = 0; m < EPT; ++m) v[1][m] = Wr[wb + n + t + m * P];
    fft_half<T, EPT, 2, true>(v, s, sstep, t, P, n, L, a.hr, tw);
    if (live) {
      const long long fb = (long long)cc * n;
      const double2* xr = x ? x + rhs * a.fstride : nullptr;
      double2* yr = y + rhs * a.fstride;
#pragma unroll
      for (int m = 0; m < EPT; ++m) {
        const int e = t + m * P;
        double2 r = widen(cadd(v[0][m], cmulc(tw[e], v[1][m])));
        if (xr) { const double2 xv = xr[fb + e]; r.x += xv.x; r.y += xv.y; }
        if (w2m && w2m[fb + e] == 0.0) r = make_double2(0, 0);  // output mask
        yr[fb + e] = r;
      }
    }
  }
}

template <typename T, int EPT, int KIND, bool TIO>
void launch_half_as(const HalfArgs& a, size_t lds, long long blocks, const FftPlanDev<T>& fp, cplx<T>* W,
                    const double2* x, double2* y, const double* w2m, hipStream_t st) {
  LSP_LAUNCH(half_name(KIND), (int)sizeof(cplx<T>), (half_lines_kernel<T, EPT, KIND, TIO>), dim3((unsigned)blocks),
             dim3(a.LPW * a.P), lds, st, W, x, y, w2m, fp.spec, fp.tw, a);
}

template <typename T, int EPT, int KIND>
void launch_half(const FftPlanDev<T>& fp, cplx<T>* W, const double2* x, double2* y, const double* w2m, int ncols,
                 int nout, long long cs, long long os, long long es, int nrhs, hipStream_t st) {
  constexpr int esz = (int)sizeof(cplx<T>);
  constexpr bool field = KIND == HK_FWD_FIELD || KIND == HK_INV_FIELD;
  HalfArgs a;
  a.n = fp.n; a.L = fp.L; a.d = fp.d;
  a.P = fp.n / EPT;
  // transposed IO for a strided axis when a wave's lines would cover less
  // than 64 contiguous bytes per element
  const bool tio = !field && es != 1 && (64 / std::min(a.P, 64)) * esz < 64;
  const int maxthr = kHalfThreads;
  const int lp0 = padi(fp.n - 1) + 1;
  int lpw = 1;
  while (lpw < 64 && lpw * 2 * a.P <= maxthr && (size_t)2 * lpw * 2 * (lp0 + 256 / esz) * esz <= kHalfLds) lpw *= 2;
  // Line stride: the lines of a bank cycle (256 bytes, 256 / esz lanes)
  // tile the banks: with TIO the IO lanes hold 256 / esz / LPW consecutive
  // entries of each line, otherwise (P < 256 / esz) P entries of 256 / esz / P lines.
  const int M = 256 / esz;
  const int X = tio ? std::max(1, M / lpw) : (a.P < M ? a.P : 0);
  int lp = lp0;
  while (lp % M != X % M) ++lp;
  a.Lp = lp;
  a.LPW = lpw;
  a.ncols = ncols; a.nout = nout; a.nrhs = nrhs;
  a.cs = cs; a.os = os; a.es = es;
  a.wstride = fp.wstride; a.fstride = fp.N;
  a.lr = fp.lr;
  a.hr = fp.hrad;
  const long long ncb = (ncols + lpw - 1) / lpw;
  // along a strided axis a block covers LPW adjacent lines' entries of a
  // cache line (128 bytes): GS consecutive blocks complete it
  int gs = 1;
  if (!field && cs == 1)
    while (gs * lpw * esz < 128 && gs < 16) gs *= 2;
  a.ncb = (int)ncb; a.GS = gs;
  const long long blocks = (ncb + gs - 1) / gs * gs * nout * nrhs;
  LSP_REQUIRE(blocks < (1LL << 31), "FFT grid too large");
  const size_t lds = (size_t)2 * lpw * lp * esz;  // two banks of LPW lines
  if (tio) launch_half_as<T, EPT, KIND, !field>(a, lds, blocks, fp, W, x, y, w2m, st);
  else launch_half_as<T, EPT, KIND, false>(a, lds, blocks, fp, W, x, y, w2m, st);
}

template <typename T, int EPT>
void kmatvec_impl(const FftPlanDev<T>& fp, int nrhs, const double2* x, double2* y, const double* w2m,
                  bool add_x, cplx<T>* W, const double* omask, hipStream_t st) {
  const int n = fp.n, L = fp.L;
  const long long LL = (long long)L * L;
  if (fp.d == 2) {
    launch_half<T, EPT, HK_FWD_FIELD>(fp, W, x, y, w2m, n, 1, 0, 0, 1, nrhs, st);
    launch_half<T, EPT, HK_CONV>(fp, W, x, y, w2m, L, 1, 1, 0, fp.lr, nrhs, st);
    launch_half<T, EPT, HK_INV_FIELD>(fp, W, add_x ? x : nullptr, y, omask, n, 1, 0, 0, 1, nrhs, st);
  } else {
    launch_half<T, EPT, HK_FWD_FIELD>(fp, W, x, y, w2m, n * n, 1, 0, 0, 1, nrhs, st);
    // along i2: lines (c1, i3 < n), elements at stride L
    launch_half<T, EPT, HK_FWD_WORK>(fp, W, x, y, w2m, L, n, 1, LL, L, nrhs, st);
    // along i3: lines c1 + L c2, elements at stride L^2
    launch_half<T, EPT, HK_CONV>(fp, W, x, y, w2m, (int)LL, 1, 1, 0, LL, nrhs, st);
    launch_half<T, EPT, HK_INV_WORK>(fp, W, x, y, w2m, L, n, 1, LL, L, nrhs, st);
    launch_half<T, EPT, HK_INV_FIELD>(fp, W, add_x ? x : nullptr, y, omask, n * n, 1, 0, 0, 1, nrhs, st);
  }
}

// ---------------------------------------------------------------- full-length transforms (set-up)

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
    for (int r = 1; r < R; ++r) {
      cplx<T> w = tw[r * k * tstep];
      if (inv) w.y = -w.y;
      v[b][r] = cmul(v[b][r], w);
    }
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

struct LineArgs {
  int L, P, LPW, Lp;
  int ncols;
  long long cs, os, es;
};

// Forward length-L transform of the lines (c, o) of W in place: c in
// [0, ncols) in groups of LPW per workgroup, o over blockIdx.y; element e
// of a line at c cs + o os + e es.
template <typename T, int EPT>
__global__ void __launch_bounds__(1024) full_lines_kernel(cplx<T>* __restrict__ W, const cplx<T>* __restrict__ tw,
                                                          FftRadices rad, LineArgs a) {
  extern __shared__ unsigned char smem_raw[];
  cplx<T>* smem = reinterpret_cast<cplx<T>*>(smem_raw);
  const int tid = threadIdx.x, nthr = blockDim.x;
  const int c0 = blockIdx.x * a.LPW;
  const int nl = min(a.LPW, a.ncols - c0);
  const int L = a.L, Lp = a.Lp;
  const long long obase = (long long)blockIdx.y * a.os;
  for (int idx = tid; idx < a.LPW * L; idx += nthr) {
    const int line = a.es == 1 ? idx / L : idx % a.LPW, e = a.es == 1 ? idx % L : idx / a.LPW;
    smem[line * Lp + e] = line < nl ? W[(long long)(c0 + line) * a.cs + obase + (long long)e * a.es] : mk<T>(0, 0);
  }
  __syncthreads();
  const int line = tid / a.P, t = tid % a.P;
  fft_line<T, EPT>(smem + line * Lp, L, a.P, t, tw, rad, false);
  for (int idx = tid; idx < a.LPW * L; idx += nthr) {
    const int ln = a.es == 1 ? idx / L : idx % a.LPW, e = a.es == 1 ? idx % L : idx / a.LPW;
    if (ln < nl) W[(long long)(c0 + ln) * a.cs + obase + (long long)e * a.es] = smem[ln * Lp + e];
  }
}

template <typename T, int EPT>
void launch_full(const FftPlanDev<T>& fp, cplx<T>* W, int ncols, int nouter, long long cs, long long os,
                 long long es, hipStream_t st) {
  LineArgs a;
  a.L = fp.L; a.P = fp.L / EPT; a.Lp = fp.L + 1;
  const size_t per_line = (size_t)a.Lp * sizeof(cplx<T>);
  int lpw = 1;
  while (lpw < 16 && (size_t)lpw * 2 * per_line <= 64 * 1024 && lpw * 2 * a.P <= 1024) lpw *= 2;
  a.LPW = lpw;
  a.ncols = ncols; a.cs = cs; a.os = os; a.es = es;
  const dim3 grid((ncols + lpw - 1) / lpw, nouter);
  LSP_LAUNCH("fft_full", (int)sizeof(cplx<T>), (full_lines_kernel<T, EPT>), grid, dim3(lpw * a.P),
             (size_t)lpw * per_line, st, W, fp.tw, fp.rad, a);
}

template <typename T, int EPT>
void full_fft_impl(const FftPlanDev<T>& fp, cplx<T>* W, hipStream_t st) {
  const int L = fp.L;
  const long long LL = (long long)L * L;
  if (fp.d == 2) {
    launch_full<T, EPT>(fp, W, L, 1, L, 0, 1, st);
    launch_full<T, EPT>(fp, W, L, 1, 1, 0, L, st);
  } else {
    launch_full<T, EPT>(fp, W, L * L, 1, L, 0, 1, st);
    launch_full<T, EPT>(fp, W, L, L, 1, LL, L, st);
    launch_full<T, EPT>(fp, W, (int)LL, 1, 1, 0, LL, st);
  }
}

}  // namespace

template <typename T>
void kmatvec(const FftPlanDev<T>& fp, int nrhs, const double2* x, double2* y, const double* w2m, bool add_x,
             cplx<T>* W, hipStream_t st, const double* omask) {
  switch (fp.hept) {
    case 12: kmatvec_impl<T, 12>(fp, nrhs, x, y, w2m, add_x, W, omask, st); break;
    case 8: kmatvec_impl<T, 8>(fp, nrhs, x, y, w2m, add_x, W, omask, st); break;
    case 6: kmatvec_impl<T, 6>(fp, nrhs, x, y, w2m, add_x, W, omask, st); break;
    case 4: kmatvec_impl<T, 4>(fp, nrhs, x, y, w2m, add_x, W, omask, st); break;
    case 3: kmatvec_impl<T, 3>(fp, nrhs, x, y, w2m, add_x, W, omask, st); break;
    default: throw Error(LSP_ERR_ARG, "unsupported FFT length");
  }
}

template <typename T>
void full_fft_forward(const FftPlanDev<T>& fp, cplx<T>* W, hipStream_t st) {
  if (fp.ept == 8) full_fft_impl<T, 8>(fp, W, st);
  else if (fp.ept == 12) full_fft_impl<T, 12>(fp, W, st);
  else if (fp.ept == 6) full_fft_impl<T, 6>(fp, W, st);
  else throw Error(LSP_ERR_ARG, "unsupported FFT length");
}

template void kmatvec<double>(const FftPlanDev<double>&, int, const double2*, double2*, const double*, bool,
                              double2*, hipStream_t, const double*);
template void kmatvec<float>(const FftPlanDev<float>&, int, const double2*, double2*, const double*, bool,
                             float2*, hipStream_t, const double*);
template void full_fft_forward<double>(const FftPlanDev<double>&, double2*, hipStream_t);

}  // namespace lsp
