// Blocked triangular sweeps for the tree levels with large fronts.
//
// The multifrontal solve x = M^{-1} z (the preconditioner of eq:PC, with the
// factors of Section 2.2's nested dissection) walks every front twice.  The
// panel-chain kernels give each front one workgroup, which on the upper
// levels (a handful of fronts with thousands of rows) leaves the chip idle
// and streams megabytes of factor through one compute unit.  Here the
// pivots of a front are grouped in super-blocks of SB = 256 rows (8 panels
// of 32), and the sweep becomes a short sequence of wide matrix-vector
// products:
//
//   forward (front rows [I | B], p pivots):
//     gather  v = [z(I); 0] + children's updates
//     for each super-block s = [s0, s1):
//       y_s = W_s v(s0:s1)                       (formed operator, SB x SB)
//       v(s1:m) -= L(s1:m, s0:s1) y_s,  v(s0:s1) = y_s
//   backward:
//     t_I = y_I - U(0:p, p:m) x_B                 (x_B from the solution;
//                                                  columns split in chunks
//                                                  of KC, partial sums added
//                                                  in chunk order)
//     for each super-block s from the last:
//       x_s = V_s t(s0:s1)                        (formed operator)
//       t(0:s0) -= U(0:s0, s0:s1) x_s
//
// W_s and V_s are the panel chains of the super-block (forward: per panel
// y_b = L11_b^{-1} P_b v_b, then the rows below inside the super-block
// updated; backward: x_b = U11_b^{-1} (t_b - U(b, k1:s1) x(k1:s1))) run on
// the unit vectors, once per factorisation, on the formation stream beside
// the upper levels' factorisation.  They are stored SB x SB column-major at
// the front's g_off: the forward operators of its super-blocks, then the
// backward ones.
//
// Every right-hand side's sums run in an order that does not depend on the
// group it is solved in, so a batched right-hand side gets its solo result
// bit for bit.
#include <algorithm>

#include "lsp_common.h"
#include "kernels.h"
#include "mfma.h"

namespace lsp {

namespace {

constexpr int PB = kNbMax;       // panel width
constexpr int SB = kSweepBlock;  // super-block rows (8 panels)
constexpr int KC = kSweepChunk;  // boundary columns per partial sum
constexpr int GR = 64;           // gemv rows per workgroup (one per lane of a wave)
constexpr int GU = 16;           // gemv column loads in flight per lane
constexpr int NF = 8;            // unit vectors per formation workgroup
constexpr int MC = 16;           // right-hand sides per matrix-core product group

// complex accumulator of a 16x16x4 product block (real and imaginary parts)
template <typename T>
struct CAcc {
  typename Mfma<T>::acc_t re, im;
  __device__ void zero() {
#pragma unroll
    for (int v = 0; v < 4; ++v) { re[v] = 0; im[v] = 0; }
  }
  __device__ cplx<T> at(int v) const { return mk<T>(re[v], im[v]); }
};

// c += a b with a from operand A, b from operand B (complex)
template <typename T>
__device__ __forceinline__ void cstep(CAcc<T>& c, const cplx<T> a, const cplx<T> b) {
  c.re = Mfma<T>::step(a.x, b.x, c.re);
  c.re = Mfma<T>::step(-a.y, b.y, c.re);
  c.im = Mfma<T>::step(a.x, b.y, c.im);
  c.im = Mfma<T>::step(a.y, b.x, c.im);
}

// out[k] = sum_j D(i, j) in(k, j) for k < NR, i = tid / 8: eight threads per
// row, each summing every eighth j in two interleaved partial sums, combined
// by an xor butterfly; the order does not depend on NR.
template <typename T, int NR>
__device__ __forceinline__ void tri_apply(const cplx<T> (*D)[PB + 1], const cplx<T> (*in)[PB], const int tid,
                                          cplx<T> (&out)[NR]) {
  constexpr int G = 256 / PB;
  const int i = tid / G, s = tid % G;
  cplx<T> dv[PB / G];
#pragma unroll
  for (int t = 0; t < PB / G; ++t) dv[t] = D[i][s + G * t];
#pragma unroll
  for (int k = 0; k < NR; ++k) {
    cplx<T> a0 = mk<T>(0, 0), a1 = mk<T>(0, 0);
#pragma unroll
    for (int t = 0; t < PB / G; ++t) {
      if (t & 1) a1 = cfma(a1, dv[t], in[k][s + G * t]);
      else a0 = cfma(a0, dv[t], in[k][s + G * t]);
    }
    cplx<T> a = cadd(a0, a1);
#pragma unroll
    for (int off = 1; off < G; off <<= 1) {
      a.x += __shfl_xor(a.x, off, 64);
      a.y += __shfl_xor(a.y, off, 64);
    }
    out[k] = a;
  }
}

// v = [z(I); 0] + children's updates for every row of the level's fronts;
// blockIdx.y the front, blockIdx.z the right-hand side.
template <typename T>
__global__ void __launch_bounds__(256) bsweep_gather_kernel(const FrontDev* __restrict__ fr, const int* __restrict__ idx,
                                                            const int* __restrict__ cpos, const cplx<T>* __restrict__ z,
                                                            cplx<T>* __restrict__ vbuf, int first, long long N,
                                                            long long vstride) {
  const FrontDev f = fr[first + blockIdx.y];
  const int m = f.p + f.q;
  const int r = blockIdx.x * 256 + threadIdx.x;
  if (r >= m) return;
  const int k = blockIdx.z;
  const int* cp = cpos + 2 * f.idx_off;
  const int q0 = f.cidx[0] >= 0 ? cp[2 * r] : -1;
  const int q1 = f.cidx[1] >= 0 ? cp[2 * r + 1] : -1;
  const long long rb = (long long)k * vstride;
  cplx<T> s = r < f.p ? z[(long long)k * N + idx[f.idx_off + r]] : mk<T>(0, 0);
  if (q0 >= 0) s = cadd(s, vbuf[rb + f.cidx[0] + q0]);
  if (q1 >= 0) s = cadd(s, vbuf[rb + f.cidx[1] + q1]);
  vbuf[rb + f.idx_off + r] = s;
}

// ---- formation of the super-block operators

// Forward operator W_s of super-block s = blockIdx.x % nsb of front
// blockIdx.x / nsb: the forward panel chain of the super-block run on the
// unit vectors e_j, j = NF blockIdx.y .. + NF, written as columns j of W_s.
template <typename T>
__global__ void __launch_bounds__(256) bsweep_form_fwd_kernel(const cplx<T>* __restrict__ Fbuf,
                                                              const cplx<T>* __restrict__ Dinv,
                                                              const FrontDev* __restrict__ fr,
                                                              const int* __restrict__ perm, cplx<T>* __restrict__ Gop,
                                                              int first, int nsbmax) {
  __shared__ cplx<T> v[NF][SB];
  __shared__ cplx<T> Li[PB][PB + 1];
  __shared__ cplx<T> tb[NF][PB];
  __shared__ cplx<T> yb[NF][PB];
  const FrontDev f = fr[first + blockIdx.x / nsbmax];
  const int s = blockIdx.x % nsbmax, s0 = s * SB;
  if (f.p <= s0) return;
  const int s1 = min(s0 + SB, f.p), len = s1 - s0;
  const int j0 = blockIdx.y * NF;
  if (j0 >= len) return;
  const int nr = min(NF, len - j0);
  const int m = f.p + f.q;
  const cplx<T>* F = Fbuf + f.f_off;
  const int* pm = perm + f.piv_off;
  const int tid = threadIdx.x;
  for (int e = tid; e < NF * SB; e += 256) {
    const int k = e / SB, r = e % SB;
    v[k][r] = mk<T>(r == j0 + k ? 1 : 0, 0);
  }
  for (int k0 = s0; k0 < s1; k0 += PB) {
    const int kb = min(PB, f.p - k0), k1 = k0 + kb;
    const cplx<T>* Lg = Dinv + f.dinv_off + (long long)(k0 / PB) * 2 * PB * PB;
    const cplx<T> l0 = Lg[tid], l1 = Lg[tid + 256], l2 = Lg[tid + 512], l3 = Lg[tid + 768];
    const int r = k1 + tid;  // rows below this panel inside the super-block, one per thread
    const int rr = min(r, s1 - 1);
    cplx<T> lrow[PB];
#pragma unroll
    for (int j = 0; j < PB; ++j) lrow[j] = F[(long long)(k0 + min(j, kb - 1)) * m + rr];
    __syncthreads();  // the previous panel's updates of v are complete
    Li[tid % PB][tid / PB] = l0;
    Li[tid % PB][tid / PB + 8] = l1;
    Li[tid % PB][tid / PB + 16] = l2;
    Li[tid % PB][tid / PB + 24] = l3;
    {
      const int k = tid / PB, j = tid % PB;  // NF * PB == 256
      tb[k][j] = j < kb ? v[k][pm[k0 + j] - s0] : mk<T>(0, 0);
    }
    __syncthreads();
    {
      cplx<T> y[NF];
      tri_apply<T, NF>(Li, tb, tid, y);
      const int i = tid / 8;
      if (tid % 8 == 0) {
#pragma unroll
        for (int k = 0; k < NF; ++k) {
          yb[k][i] = y[k];
          if (i < kb) v[k][k0 - s0 + i] = y[k];
        }
      }
    }
    __syncthreads();
    if (r < s1) {
#pragma unroll
      for (int k = 0; k < NF; ++k) {
        cplx<T> acc = v[k][r - s0];
#pragma unroll
        for (int j = 0; j < PB; ++j)
          if (j < kb) acc = cfms(acc, lrow[j], yb[k][j]);
        v[k][r - s0] = acc;
      }
    }
  }
  __syncthreads();
  cplx<T>* W = Gop + f.g_off + (long long)s * SB * SB;
  for (int e = tid; e < NF * SB; e += 256) {
    const int k = e / SB, r = e % SB;
    if (k < nr && r < len) W[(long long)(j0 + k) * SB + r] = v[k][r];
  }
}

// Backward operator V_s: the backward panel chain of the super-block on the
// unit vectors, columns j of V_s, stored after the front's forward ones.
template <typename T>
__global__ void __launch_bounds__(256) bsweep_form_bwd_kernel(const cplx<T>* __restrict__ Fbuf,
                                                              const cplx<T>* __restrict__ Dinv,
                                                              const FrontDev* __restrict__ fr, cplx<T>* __restrict__ Gop,
                                                              int first, int nsbmax) {
  constexpr int G = 256 / PB;  // column groups
  __shared__ cplx<T> v[NF][SB];
  __shared__ cplx<T> Ui[PB][PB + 1];
  __shared__ cplx<T> part[G][NF][PB];
  __shared__ cplx<T> rb[NF][PB];
  const FrontDev f = fr[first + blockIdx.x / nsbmax];
  const int s = blockIdx.x % nsbmax, s0 = s * SB;
  if (f.p <= s0) return;
  const int s1 = min(s0 + SB, f.p), len = s1 - s0;
  const int j0 = blockIdx.y * NF;
  if (j0 >= len) return;
  const int nr = min(NF, len - j0);
  const int m = f.p + f.q;
  const cplx<T>* F = Fbuf + f.f_off;
  const int tid = threadIdx.x;
  const int j = tid % PB, grp = tid / PB;
  for (int e = tid; e < NF * SB; e += 256) {
    const int k = e / SB, r = e % SB;
    v[k][r] = mk<T>(r == j0 + k ? 1 : 0, 0);
  }
  const int nb = (len + PB - 1) / PB;
  for (int b = nb - 1; b >= 0; --b) {
    const int k0 = s0 + b * PB, kb = min(PB, f.p - k0), k1 = k0 + kb;
    const cplx<T>* Ug = Dinv + f.dinv_off + (long long)(k0 / PB) * 2 * PB * PB + PB * PB;
    const cplx<T> u0 = Ug[tid], u1 = Ug[tid + 256], u2 = Ug[tid + 512], u3 = Ug[tid + 768];
    // U(k0 + j, c) for this thread's columns c = k1 + grp + 8 t < s1
    constexpr int TU = SB / G;
    cplx<T> ucol[TU];
#pragma unroll
    for (int t = 0; t < TU; ++t) {
      const int c = min(k1 + grp + G * t, m - 1);
      ucol[t] = F[(long long)(k0 + min(j, kb - 1)) + (long long)c * m];
    }
    __syncthreads();  // x(k1:s1) of the previous panel is in v
    Ui[tid % PB][tid / PB] = u0;
    Ui[tid % PB][tid / PB + 8] = u1;
    Ui[tid % PB][tid / PB + 16] = u2;
    Ui[tid % PB][tid / PB + 24] = u3;
    cplx<T> acc[NF];
#pragma unroll
    for (int k = 0; k < NF; ++k) acc[k] = mk<T>(0, 0);
#pragma unroll
    for (int t = 0; t < TU; ++t) {
      const int c = k1 + grp + G * t;
      if (c < s1)
#pragma unroll
        for (int k = 0; k < NF; ++k) acc[k] = cfma(acc[k], ucol[t], v[k][c - s0]);
    }
#pragma unroll
    for (int k = 0; k < NF; ++k) part[grp][k][j] = acc[k];
    __syncthreads();
    {
      const int jj = tid % PB, k = tid / PB;  // NF * PB == 256
      cplx<T> sm = part[0][k][jj];
#pragma unroll
      for (int g = 1; g < G; ++g) sm = cadd(sm, part[g][k][jj]);
      rb[k][jj] = jj < kb ? csub(v[k][k0 - s0 + jj], sm) : mk<T>(0, 0);
    }
    __syncthreads();
    {
      cplx<T> xs[NF];
      tri_apply<T, NF>(Ui, rb, tid, xs);
      const int i = tid / 8;
      if (tid % 8 == 0 && i < kb) {
#pragma unroll
        for (int k = 0; k < NF; ++k) v[k][k0 - s0 + i] = xs[k];
      }
    }
  }
  __syncthreads();
  const int nsb = (f.p + SB - 1) / SB;
  cplx<T>* V = Gop + f.g_off + (long long)(nsb + s) * SB * SB;
  for (int e = tid; e < NF * SB; e += 256) {
    const int k = e / SB, r = e % SB;
    if (k < nr && r < len) V[(long long)(j0 + k) * SB + r] = v[k][r];
  }
}

// ---- the sweeps' matrix-vector products
//
// acc(r) = sum_c A(r, c) in(c) over a rectangle of rows [rlo, rhi) and
// columns [clo, chi) of each front (blockIdx.y), for a group of 16
// right-hand sides (blockIdx.z), on the matrix cores: a workgroup takes 16
// rows (blockIdx.x), its four waves a quarter of each staged chunk of GC
// columns each, as 16x16x4 products of the staged inputs (operand A, the
// right-hand sides as rows) and the matrix entries (operand B, 16
// consecutive rows per load); the four waves' sums are added in wave
// order.  Each output column of the products is its own sum, so a
// right-hand side's result does not depend on the others in its group.
//   MODE_W   forward operator:  rows/columns [s0, s1), A = W_s, in = v (front
//            vector), out: y_s -> ybuf
//   MODE_V   backward operator: rows/columns [s0, s1), A = V_s, in = t, out:
//            x_s -> ybuf, the solution at the pivots' grid points (and xw)
//   MODE_FS  forward step:  rows [s1, m), columns [s0, s1), A = L, in = y_s
//            from ybuf, out: v -= acc; tile 0 also copies y_s into v(s0:s1)
//   MODE_BS  backward step: rows [0, s0), columns [s0, s1), A = U, in = x_s
//            from ybuf, out: t -= acc
//   MODE_BB  backward boundary: rows [0, p), columns [p + KC kc, ...) for
//            the chunk kc = blockIdx.x % kch, A = U, in = x_B from the
//            solution, out: the chunk's partial sums -> pbuf
enum { MODE_W = 0, MODE_V = 1, MODE_FS = 2, MODE_BS = 3, MODE_BB = 4 };

struct GemvArgs {
  int first;         // first front of the level
  int s;             // super-block (MODE_W/V/FS/BS)
  int kch;           // column chunks of MODE_BB
  int maxp;          // the level's largest p (pbuf row stride per front)
  int nrhs;
  long long N, vstride;
  long long ystride;  // ybuf / pbuf elements per right-hand side
};

constexpr int GT = 16;   // rows per workgroup
constexpr int GC = 128;  // columns staged per chunk (32 per wave)

template <typename T, int MODE>
__global__ void __launch_bounds__(256) bsweep_gemv_kernel(const cplx<T>* __restrict__ Fbuf,
                                                          const cplx<T>* __restrict__ Gop,
                                                          const FrontDev* __restrict__ fr, const int* __restrict__ idx,
                                                          cplx<T>* __restrict__ x, cplx<T>* __restrict__ vbuf,
                                                          cplx<T>* __restrict__ ybuf, cplx<T>* __restrict__ pbuf,
                                                          double2* __restrict__ xw, GemvArgs a) {
  __shared__ cplx<T> xin[MC][GC + 1];
  __shared__ cplx<T> part[3][64][4];
  const int fi = blockIdx.y;
  const FrontDev f = fr[a.first + fi];
  const int p = f.p, m = p + f.q;
  const int nsb = (p + SB - 1) / SB;
  const int s0 = a.s * SB, s1 = min(s0 + SB, p);
  int tile = blockIdx.x, kc = 0;
  if constexpr (MODE == MODE_BB) { kc = tile % a.kch; tile /= a.kch; }
  int rlo, rhi, clo, chi;
  if constexpr (MODE == MODE_W || MODE == MODE_V) { rlo = s0; rhi = s1; clo = s0; chi = s1; }
  else if constexpr (MODE == MODE_FS) { rlo = s1; rhi = m; clo = s0; chi = s1; }
  else if constexpr (MODE == MODE_BS) { rlo = 0; rhi = min(s0, p); clo = s0; chi = s1; }
  else { rlo = 0; rhi = p; clo = p + kc * KC; chi = min(m, clo + KC); }
  const int r0 = blockIdx.z * MC, nr = min(MC, a.nrhs - r0);
  const int tid = threadIdx.x, lane = tid % 64, w = tid / 64, li = lane % 16, lk = lane / 16;
  cplx<T>* vg = vbuf + (long long)r0 * a.vstride + f.idx_off;
  cplx<T>* yg = ybuf + (long long)r0 * a.ystride + (long long)fi * SB;  // y_s(c) at yg[c - s0]
  if constexpr (MODE == MODE_FS) {
    if (blockIdx.x == 0)  // y_s into the front vector at the pivot positions
      for (int e = tid; e < MC * SB; e += 256) {
        const int k = e / SB, c = s0 + e % SB;
        if (k < nr && c < s1) vg[(long long)k * a.vstride + c] = yg[(long long)k * a.ystride + c - s0];
      }
  }
  const int row0 = rlo + tile * GT;
  if (row0 >= rhi || clo >= chi) return;
  const int rr = min(row0 + li, rhi - 1);  // this lane's matrix row (clamped in range)
  // entry (r, c) of the rectangle's matrix at A[(c - cb) * ld + r - rb]
  const cplx<T>* A;
  long long ld;
  int rb, cb;
  if constexpr (MODE == MODE_W || MODE == MODE_V) {
    A = Gop + f.g_off + (long long)(MODE == MODE_V ? nsb + a.s : a.s) * SB * SB;
    ld = SB;
    rb = s0;
    cb = s0;
  } else {
    A = Fbuf + f.f_off;
    ld = m;
    rb = 0;
    cb = 0;
  }
  const int* id = idx + f.idx_off;
  CAcc<T> acc;
  acc.zero();
  for (int c0 = clo; c0 < chi; c0 += GC) {
    const int cn = min(GC, chi - c0);
    if (c0 > clo) __syncthreads();  // the previous chunk's reads of xin are done
    for (int e = tid; e < MC * GC; e += 256) {
      const int k = e / GC, jj = e % GC;
      cplx<T> v = mk<T>(0, 0);
      if (k < nr && jj < cn) {
        const int c = c0 + jj;
        if constexpr (MODE == MODE_BB) v = x[(long long)(r0 + k) * a.N + id[c]];
        else if constexpr (MODE == MODE_FS || MODE == MODE_BS) v = yg[(long long)k * a.ystride + c - s0];
        else v = vg[(long long)k * a.vstride + c];
      }
      xin[k][jj] = v;
    }
    __syncthreads();
    // this wave's 32 columns: their matrix entries first, then the products
    const int jw = w * (GC / 4);
    if (jw < cn) {
      cplx<T> av[GC / 16];
#pragma unroll
      for (int s4 = 0; s4 < GC / 16; ++s4) {
        const int jj = min(jw + 4 * s4 + lk, cn - 1);
        av[s4] = A[(long long)(c0 + jj - cb) * ld + (rr - rb)];
      }
#pragma unroll
      for (int s4 = 0; s4 < GC / 16; ++s4) {
        const int jj = jw + 4 * s4 + lk;
        cstep(acc, xin[li][min(jj, GC - 1)], jj < cn ? av[s4] : mk<T>(0, 0));
      }
    }
  }
  if (w > 0) {
#pragma unroll
    for (int v = 0; v < 4; ++v) part[w - 1][lane][v] = acc.at(v);
  }
  __syncthreads();
  if (w > 0) return;
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    cplx<T> sm = acc.at(v);
#pragma unroll
    for (int q = 0; q < 3; ++q) sm = cadd(sm, part[q][lane][v]);
    // the product's row v of this lane's block: right-hand side k, matrix row rw
    const int k = Mfma<T>::row(lk, v), rw = row0 + li;
    if (k < nr && rw < rhi) {
      if constexpr (MODE == MODE_W) {
        yg[(long long)k * a.ystride + rw - s0] = sm;
      } else if constexpr (MODE == MODE_V) {
        yg[(long long)k * a.ystride + rw - s0] = sm;
        const long long gi = id[rw];
        x[(long long)(r0 + k) * a.N + gi] = sm;
        if (xw) xw[(long long)(r0 + k) * a.N + gi] = widen(sm);
      } else if constexpr (MODE == MODE_BB) {
        pbuf[((long long)kc * a.nrhs + r0 + k) * a.ystride + (long long)fi * a.maxp + rw] = sm;
      } else {
        cplx<T>* o = vg + (long long)k * a.vstride + rw;
        *o = csub(*o, sm);
      }
    }
  }
}

// t(r) = t(r) - sum over the boundary column chunks (in chunk order) of the
// partial sums; one thread per (pivot row, front, right-hand side).
template <typename T>
__global__ void __launch_bounds__(256) bsweep_bb_reduce_kernel(const FrontDev* __restrict__ fr,
                                                               cplx<T>* __restrict__ vbuf,
                                                               const cplx<T>* __restrict__ pbuf, GemvArgs a) {
  const int fi = blockIdx.y;
  const FrontDev f = fr[a.first + fi];
  const int r = blockIdx.x * 256 + threadIdx.x;
  if (r >= f.p || f.q == 0) return;
  const int k = blockIdx.z;
  const int kch = (f.q + KC - 1) / KC;
  cplx<T> sm = pbuf[((long long)0 * a.nrhs + k) * a.ystride + (long long)fi * a.maxp + r];
  for (int c = 1; c < kch; ++c) sm = cadd(sm, pbuf[((long long)c * a.nrhs + k) * a.ystride + (long long)fi * a.maxp + r]);
  cplx<T>* o = vbuf + (long long)k * a.vstride + f.idx_off + r;
  *o = csub(*o, sm);
}

template <typename T, int MODE>
void gemv_launch(const MfDev<T>& mf, const Plan& plan, int l, int s, int nrows, int kch, int nrhs, cplx<T>* x,
                 cplx<T>* vbuf, const SweepBufs<T>& sb, double2* xw, hipStream_t st) {
  if (nrows <= 0) return;
  const int first = plan.level_ptr[l];
  const int cnt = plan.level_ptr[l + 1] - first;
  const int groups = (nrhs + MC - 1) / MC;
  GemvArgs a{first, s, kch, plan.level_maxp[l], nrhs, (long long)plan.N, (long long)plan.sum_pq, sb.ystride};
  LSP_LAUNCH("bsweep_gemv", (int)sizeof(cplx<T>), (bsweep_gemv_kernel<T, MODE>),
             dim3((nrows + GT - 1) / GT * kch, cnt, groups), dim3(256), 0, st, mf.F, mf.G, mf.fronts, mf.idx, x, vbuf,
             sb.ybuf, sb.pbuf, xw, a);
}

template <typename T>
void blocked_level_fwd(const MfDev<T>& mf, const Plan& plan, int l, int nrhs, const cplx<T>* z, cplx<T>* vbuf,
                       const SweepBufs<T>& sb, hipStream_t st) {
  const int first = plan.level_ptr[l];
  const int cnt = plan.level_ptr[l + 1] - first;
  const int maxm = plan.level_maxpq[l], maxp = plan.level_maxp[l];
  LSP_LAUNCH("bsweep_gather", (int)sizeof(cplx<T>), bsweep_gather_kernel<T>, dim3((maxm + 255) / 256, cnt, nrhs),
             dim3(256), 0, st, mf.fronts, mf.idx, mf.cpos, z, vbuf, first, (long long)plan.N, (long long)plan.sum_pq);
  const int nsb = (maxp + SB - 1) / SB;
  for (int s = 0; s < nsb; ++s) {
    const int s0 = s * SB;
    gemv_launch<T, MODE_W>(mf, plan, l, s, std::min(SB, maxp - s0), 1, nrhs, nullptr, vbuf, sb, nullptr, st);
    int rows = 0;  // rows below the super-block, the most over the level's fronts
    for (int i = first; i < first + cnt; ++i) {
      const FrontDev& f = plan.fronts[i];
      if (f.p > s0) rows = std::max(rows, f.p + f.q - std::min(s0 + SB, f.p));
    }
    // at least one tile, so that tile 0 copies y_s into the front vector
    gemv_launch<T, MODE_FS>(mf, plan, l, s, std::max(rows, 1), 1, nrhs, nullptr, vbuf, sb, nullptr, st);
  }
}

template <typename T>
void blocked_level_bwd(const MfDev<T>& mf, const Plan& plan, int l, int nrhs, cplx<T>* x, cplx<T>* vbuf,
                       const SweepBufs<T>& sb, hipStream_t st, double2* xw) {
  const int first = plan.level_ptr[l];
  const int cnt = plan.level_ptr[l + 1] - first;
  const int maxp = plan.level_maxp[l];
  int maxq = 0;
  for (int i = first; i < first + cnt; ++i) maxq = std::max(maxq, plan.fronts[i].q);
  if (maxq > 0) {
    const int kch = (maxq + KC - 1) / KC;
    gemv_launch<T, MODE_BB>(mf, plan, l, 0, maxp, kch, nrhs, x, vbuf, sb, nullptr, st);
    GemvArgs a{first, 0, kch, maxp, nrhs, (long long)plan.N, (long long)plan.sum_pq, sb.ystride};
    LSP_LAUNCH("bsweep_bb_reduce", (int)sizeof(cplx<T>), bsweep_bb_reduce_kernel<T>,
               dim3((maxp + 255) / 256, cnt, nrhs), dim3(256), 0, st, mf.fronts, vbuf, sb.pbuf, a);
  }
  const int nsb = (maxp + SB - 1) / SB;
  for (int s = nsb - 1; s >= 0; --s) {
    const int s0 = s * SB;
    gemv_launch<T, MODE_V>(mf, plan, l, s, std::min(SB, maxp - s0), 1, nrhs, x, vbuf, sb, xw, st);
    gemv_launch<T, MODE_BS>(mf, plan, l, s, s0, 1, nrhs, nullptr, vbuf, sb, nullptr, st);
  }
}

// ---- small-front levels: panel chains on the matrix cores (Plan::level_mchain)
//
// Fronts of at most two panels (p <= 64) and 256 rows, many per level.  One
// wave per (front, group of 16 right-hand sides) runs the front's panel
// chain with the right-hand sides as the 16 columns of 16x16x4 MFMA
// products (complex as four real products):
//   forward, per panel b:   y_b = L11_b^{-1} (P_b v_b)       (32 x 32 by 32 x 16)
//                           v(k1:m) -= L21_b y_b              (16-row tiles)
//   backward, per panel from the last:
//                           t_b = y_b - U12_b x(k1:m)         (32 x (m - k1) by (m - k1) x 16)
//                           x_b = U11_b^{-1} t_b
// (the inverse blocks are exactly zero outside their kb x kb part, and the
// operands past kb are zeroed).  The front's vectors stay in LDS, V[row][16].
// Each output column of an MFMA is its own sum, so a right-hand side's
// result does not depend on the others in its group: batched and solo solves
// agree bit for bit.
constexpr int MCP = 64;   // largest p of a matrix-core chain level
constexpr int MCM = 256;  // largest m

template <typename T>
__device__ __forceinline__ cplx<T> front_input(const FrontDev& f, const int* __restrict__ id,
                                               const int* __restrict__ cp, const cplx<T>* __restrict__ z,
                                               const cplx<T>* __restrict__ vbuf, const int r, const int k,
                                               const long long N, const long long vstride) {
  const long long rb = (long long)k * vstride;
  cplx<T> s = r < f.p ? z[(long long)k * N + id[r]] : mk<T>(0, 0);
  const int q0 = f.cidx[0] >= 0 ? cp[2 * r] : -1, q1 = f.cidx[1] >= 0 ? cp[2 * r + 1] : -1;
  if (q0 >= 0) s = cadd(s, vbuf[rb + f.cidx[0] + q0]);
  if (q1 >= 0) s = cadd(s, vbuf[rb + f.cidx[1] + q1]);
  return s;
}

// W waves per front (levels with fewer fronts take more): the gathers and
// the stores are shared, the update's 16-row tiles go round-robin to the
// waves, the inverse-block products' two tiles to waves 0 and 1 (wave 0
// alone when W = 1), and the backward sweep's U12 columns in chunks of 32
// to the waves, whose partial sums wave 0 and 1 add in wave order.  The
// order of every sum depends on W only, which depends on the level's front
// count, not on the right-hand sides.
template <typename T, int W>
__global__ void __launch_bounds__(64 * W) mchain_fwd_kernel(const cplx<T>* __restrict__ Fbuf,
                                                            const cplx<T>* __restrict__ Dinv,
                                                            const FrontDev* __restrict__ fr,
                                                            const int* __restrict__ idx, const int* __restrict__ cpos,
                                                            const int* __restrict__ perm,
                                                            const cplx<T>* __restrict__ z, cplx<T>* __restrict__ vbuf,
                                                            int first, int nrhs, long long N, long long vstride) {
  extern __shared__ unsigned char smem_raw[];
  cplx<T>* V = reinterpret_cast<cplx<T>*>(smem_raw);  // V[r * MC + k]
  const FrontDev f = fr[first + blockIdx.x];
  const int p = f.p, m = p + f.q;
  const int r0 = blockIdx.y * MC, nr = min(MC, nrhs - r0);
  const int tid = threadIdx.x, wave = tid / 64, lane = tid % 64, li = lane % 16, lk = lane / 16;
  const cplx<T>* F = Fbuf + f.f_off;
  const int* id = idx + f.idx_off;
  const int* cp = cpos + 2 * f.idx_off;
  const int* pm = perm + f.piv_off;
  // v = [z(I); 0] + children's updates: a row per thread, the row's index
  // loads first, then its 16 right-hand sides' loads together
  for (int r = tid; r < m; r += 64 * W) {
    const int gi = id[min(r, p - 1)];
    const int q0 = f.cidx[0] >= 0 ? cp[2 * r] : -1, q1 = f.cidx[1] >= 0 ? cp[2 * r + 1] : -1;
    cplx<T> val[MC];
#pragma unroll
    for (int k = 0; k < MC; ++k) {
      const cplx<T> zv = z[(long long)(r0 + min(k, nr - 1)) * N + gi];
      val[k] = k < nr && r < p ? zv : mk<T>(0, 0);
    }
    if (q0 >= 0) {
#pragma unroll
      for (int k = 0; k < MC; ++k) {
        const cplx<T> c = vbuf[(long long)(r0 + min(k, nr - 1)) * vstride + f.cidx[0] + q0];
        if (k < nr) val[k] = cadd(val[k], c);
      }
    }
    if (q1 >= 0) {
#pragma unroll
      for (int k = 0; k < MC; ++k) {
        const cplx<T> c = vbuf[(long long)(r0 + min(k, nr - 1)) * vstride + f.cidx[1] + q1];
        if (k < nr) val[k] = cadd(val[k], c);
      }
    }
#pragma unroll
    for (int k = 0; k < MC; ++k) V[r * MC + k] = val[k];
  }
  for (int k0 = 0; k0 < p; k0 += PB) {
    const int kb = min(PB, p - k0), k1 = k0 + kb, nb = m - k1;
    const int nh = (kb + 15) / 16, ns = (kb + 3) / 4;  // nonzero tiles and k-steps
    const cplx<T>* Lg = Dinv + f.dinv_off + (long long)(k0 / PB) * 2 * PB * PB;
    __syncthreads();  // v is complete
    // y_b = L11^{-1} P_b v_b: operand A the inverse block (column-major),
    // operand B the gathered rows; tile h on wave h (wave 0 both if W = 1);
    // L11^{-1} is lower triangular, so tile 0's k-steps past column 16 are
    // exact zeros and skipped
    CAcc<T> y[W == 1 ? 2 : 1];
#pragma unroll
    for (int u = 0; u < (W == 1 ? 2 : 1); ++u) {
      y[u].zero();
      const int h = W == 1 ? u : wave;
      if (h < nh) {
#pragma unroll
        for (int s4 = 0; s4 < PB / 4; ++s4) {
          if (s4 < ns && !(h == 0 && 4 * s4 >= 16)) {
            const int j = 4 * s4 + lk;
            const int src = pm[k0 + min(j, kb - 1)];
            const cplx<T> tv = V[src * MC + li];
            cstep(y[u], Lg[(16 * h + li) + PB * j], j < kb ? tv : mk<T>(0, 0));
          }
        }
      }
    }
    __syncthreads();  // every gather of the panel's rows is done
#pragma unroll
    for (int u = 0; u < (W == 1 ? 2 : 1); ++u) {
      const int h = W == 1 ? u : wave;
      if (h < nh) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int i = 16 * h + Mfma<T>::row(lk, v);
          if (i < kb) V[(k0 + i) * MC + li] = y[u].at(v);
        }
      }
    }
    __syncthreads();
    // v(k1:m) -= L21 y_b, 16 rows at a time (tiles round-robin over the
    // waves): operand A the rows of L21, operand B y_b (held for all tiles);
    // each tile's L21 entries are loaded a tile ahead
    const int ntile = (nb + 15) / 16;
    if (wave < ntile) {
      cplx<T> yb[PB / 4];
#pragma unroll
      for (int s4 = 0; s4 < PB / 4; ++s4) {
        const int j = 4 * s4 + lk;
        const cplx<T> yv = V[(k0 + min(j, kb - 1)) * MC + li];
        yb[s4] = j < kb ? yv : mk<T>(0, 0);
      }
      cplx<T> lc[PB / 4];
      auto load_tile = [&](const int t, cplx<T>(&dst)[PB / 4]) {
        const int rr = k1 + min(16 * t + li, nb - 1);
#pragma unroll
        for (int s4 = 0; s4 < PB / 4; ++s4)
          if (s4 < ns) dst[s4] = F[(long long)(k0 + min(4 * s4 + lk, kb - 1)) * m + rr];
      };
      load_tile(wave, lc);
      for (int t = wave; t < ntile; t += W) {
        cplx<T> ln[PB / 4];
        if (t + W < ntile) load_tile(t + W, ln);
        CAcc<T> u;
        u.zero();
#pragma unroll
        for (int s4 = 0; s4 < PB / 4; ++s4)
          if (s4 < ns) cstep(u, 4 * s4 + lk < kb ? lc[s4] : mk<T>(0, 0), yb[s4]);
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int r = 16 * t + Mfma<T>::row(lk, v);
          if (r < nb) {
            const cplx<T> o = V[(k1 + r) * MC + li];
            V[(k1 + r) * MC + li] = csub(o, u.at(v));
          }
        }
        if (t + W < ntile) {
#pragma unroll
          for (int s4 = 0; s4 < PB / 4; ++s4) lc[s4] = ln[s4];
        }
      }
    }
  }
  __syncthreads();
  for (int e = tid; e < m * nr; e += 64 * W) {
    const int r = e % m, k = e / m;
    vbuf[(long long)(r0 + k) * vstride + f.idx_off + r] = V[r * MC + k];
  }
}

// The backward sweep gathers the boundary rows' solution from the point-
// major copy xpm (a grid point's 16 right-hand sides in one 128-byte line,
// where the [nrhs][N] layout spreads them over 16 lines) and stores its
// pivots' solution there for the levels below (if any), into xw when given (the
// widened solution, mixed path) and into x unless store_x is 0 (x is not
// needed when xw is the output and every level below is a matrix-core one).
template <typename T, int W>
__global__ void __launch_bounds__(64 * W) mchain_bwd_kernel(const cplx<T>* __restrict__ Fbuf,
                                                            const cplx<T>* __restrict__ Dinv,
                                                            const FrontDev* __restrict__ fr,
                                                            const int* __restrict__ idx, cplx<T>* __restrict__ x,
                                                            const cplx<T>* __restrict__ vbuf, int first, int nrhs,
                                                            long long N, long long vstride,
                                                            double2* __restrict__ xw, int maxm,
                                                            cplx<T>* __restrict__ xpm, int store_x, int store_pm) {
  extern __shared__ unsigned char smem_raw[];
  cplx<T>* V = reinterpret_cast<cplx<T>*>(smem_raw);  // V[r * MC + k]
  cplx<T>* part = V + (long long)maxm * MC;           // part[(w - 1) * 2 + h][64 lanes][4]: waves 1.. partial sums
  const FrontDev f = fr[first + blockIdx.x];
  const int p = f.p, m = p + f.q;
  const int r0 = blockIdx.y * MC, nr = min(MC, nrhs - r0);
  const int tid = threadIdx.x, wave = tid / 64, lane = tid % 64, li = lane % 16, lk = lane / 16;
  const cplx<T>* F = Fbuf + f.f_off;
  const int* id = idx + f.idx_off;
  // v = [y(I) from the forward sweep; x(B) from the ancestors]: a row per
  // thread, its 16 right-hand sides' loads together
  for (int r = tid; r < m; r += 64 * W) {
    cplx<T> val[MC];
    if (r < p) {
#pragma unroll
      for (int k = 0; k < MC; ++k) val[k] = vbuf[(long long)(r0 + min(k, nr - 1)) * vstride + f.idx_off + r];
    } else {
      const cplx<T>* src = xpm + ((long long)blockIdx.y * N + id[r]) * MC;
#pragma unroll
      for (int k = 0; k < MC; ++k) val[k] = src[k];
    }
#pragma unroll
    for (int k = 0; k < MC; ++k) V[r * MC + k] = k < nr ? val[k] : mk<T>(0, 0);
  }
  const int nblk = (p + PB - 1) / PB;
  for (int b = nblk - 1; b >= 0; --b) {
    const int k0 = b * PB, kb = min(PB, p - k0), k1 = k0 + kb, nc = m - k1;
    const int nh = (kb + 15) / 16, ns = (kb + 3) / 4;
    const cplx<T>* Ug = Dinv + f.dinv_off + (long long)b * 2 * PB * PB + PB * PB;
    __syncthreads();  // x of the later panels is in place
    // s = U12 x(k1:m): operand A the panel's rows of U12; wave w takes the
    // column chunks 32 w, 32 (w + W), ..., each chunk's loads issued first
    CAcc<T> sa[2];
    sa[0].zero();
    sa[1].zero();
    for (int c0 = 32 * wave; c0 < nc; c0 += 32 * W) {
      // k-steps of the chunk inside the front (a chunk past the last column
      // contributes exact zeros, so its empty steps are skipped)
      const int n8 = min(8, (nc - c0 + 3) / 4);
      cplx<T> ua[8][2];
#pragma unroll
      for (int s8 = 0; s8 < 8; ++s8) {
        if (s8 >= n8) break;
        const long long col = (long long)(k1 + min(c0 + 4 * s8 + lk, nc - 1)) * m;
#pragma unroll
        for (int h = 0; h < 2; ++h)
          if (h < nh) ua[s8][h] = F[(k0 + min(16 * h + li, kb - 1)) + col];
      }
#pragma unroll
      for (int s8 = 0; s8 < 8; ++s8) {
        if (s8 >= n8) break;
        const int c = c0 + 4 * s8 + lk;
        const cplx<T> xv = V[(k1 + min(c, nc - 1)) * MC + li];
        const cplx<T> b4 = c < nc ? xv : mk<T>(0, 0);
#pragma unroll
        for (int h = 0; h < 2; ++h)
          if (h < nh) cstep(sa[h], 16 * h + li < kb && c < nc ? ua[s8][h] : mk<T>(0, 0), b4);
      }
    }
    // t_b = y_b - s, s the partial sums added in wave order by wave 0
    if constexpr (W > 1) {
      if (wave > 0) {
#pragma unroll
        for (int h = 0; h < 2; ++h)
#pragma unroll
          for (int v = 0; v < 4; ++v) part[(((wave - 1) * 2 + h) * 64 + lane) * 4 + v] = sa[h].at(v);
      }
      __syncthreads();
    }
    if (wave == 0) {
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        if (h < nh) {
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            cplx<T> sv = sa[h].at(v);
#pragma unroll
            for (int w = 1; w < W; ++w) sv = cadd(sv, part[(((w - 1) * 2 + h) * 64 + lane) * 4 + v]);
            const int i = 16 * h + Mfma<T>::row(lk, v);
            if (i < kb) V[(k0 + i) * MC + li] = csub(V[(k0 + i) * MC + li], sv);
          }
        }
      }
    }
    __syncthreads();
    // x_b = U11^{-1} t_b (upper triangular: tile 1's k-steps before column
    // 16 are exact zeros and skipped)
    CAcc<T> xa[W == 1 ? 2 : 1];
#pragma unroll
    for (int u = 0; u < (W == 1 ? 2 : 1); ++u) {
      xa[u].zero();
      const int h = W == 1 ? u : wave;
      if (h < nh) {
#pragma unroll
        for (int s4 = 0; s4 < PB / 4; ++s4) {
          if (s4 < ns && !(h == 1 && 4 * s4 < 16)) {
            const int j = 4 * s4 + lk;
            const cplx<T> tv = V[(k0 + min(j, kb - 1)) * MC + li];
            cstep(xa[u], Ug[(16 * h + li) + PB * j], j < kb ? tv : mk<T>(0, 0));
          }
        }
      }
    }
    __syncthreads();  // every read of t_b is done
#pragma unroll
    for (int u = 0; u < (W == 1 ? 2 : 1); ++u) {
      const int h = W == 1 ? u : wave;
      if (h < nh) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int i = 16 * h + Mfma<T>::row(lk, v);
          if (i < kb) V[(k0 + i) * MC + li] = xa[u].at(v);
        }
      }
    }
  }
  __syncthreads();
  if (store_pm) {  // read by the levels below for their boundary rows
    for (int e = tid; e < p * MC; e += 64 * W) {
      const int r = e / MC, k = e % MC;
      xpm[((long long)blockIdx.y * N + id[r]) * MC + k] = V[r * MC + k];
    }
  }
  for (int e = tid; e < p * nr; e += 64 * W) {
    const int r = e % p, k = e / p;
    const cplx<T> v = V[r * MC + k];
    const long long gi = (long long)(r0 + k) * N + id[r];
    if (xw) xw[gi] = widen(v);
    if (store_x) x[gi] = v;
  }
}

// The pivots of the fronts first .. first + gridDim.x - 1 (levels whose
// solution the backward sweep has just computed with other kernels than the
// matrix-core chains), point-major: one workgroup per front, a pivot per
// thread.
template <typename T>
__global__ void __launch_bounds__(256) point_major_kernel(const cplx<T>* __restrict__ x, cplx<T>* __restrict__ xpm,
                                                          const FrontDev* __restrict__ fr,
                                                          const int* __restrict__ idx, int first, int nrhs,
                                                          long long N) {
  const FrontDev f = fr[first + blockIdx.x];
  const int g = blockIdx.y, nr = min(MC, nrhs - g * MC);
  for (int r = threadIdx.x; r < f.p; r += 256) {
    const long long i = idx[f.idx_off + r];
    cplx<T> v[MC];
#pragma unroll
    for (int k = 0; k < MC; ++k) {
      const cplx<T> a = x[(long long)(g * MC + min(k, nr - 1)) * N + i];
      v[k] = k < nr ? a : mk<T>(0, 0);
    }
    cplx<T>* dst = xpm + ((long long)g * N + i) * MC;
#pragma unroll
    for (int k = 0; k < MC; ++k) dst[k] = v[k];
  }
}

}  // namespace

template <typename T>
void blocked_sweep(bool fwd, const MfDev<T>& mf, const Plan& plan, int l, int nrhs, const cplx<T>* z, cplx<T>* x,
                   cplx<T>* vbuf, const SweepBufs<T>& sb, hipStream_t st, double2* xw) {
  if (fwd) blocked_level_fwd<T>(mf, plan, l, nrhs, z, vbuf, sb, st);
  else blocked_level_bwd<T>(mf, plan, l, nrhs, x, vbuf, sb, st, xw);
}

// waves per front: enough fronts' waves to fill the chip (about 16 per CU)
inline int mchain_waves(int cnt) { return cnt >= 4096 ? 1 : (cnt >= 2048 ? 2 : 4); }

template <typename T, int W>
void mchain_launch(bool fwd, const MfDev<T>& mf, const Plan& plan, int l, int nrhs, const cplx<T>* z, cplx<T>* x,
                   cplx<T>* vbuf, hipStream_t st, double2* xw, cplx<T>* xpm) {
  bool below = true;  // every level below l is a matrix-core one
  for (int k = 0; k < l; ++k) below = below && plan.level_mchain[k];
  const int store_x = xw == nullptr || !below;
  const int first = plan.level_ptr[l];
  const int cnt = plan.level_ptr[l + 1] - first;
  const int maxm = plan.level_maxpq[l];
  const dim3 grid(cnt, (nrhs + MC - 1) / MC);
  const size_t vlds = (size_t)maxm * MC * sizeof(cplx<T>);
  if (fwd) {
    LSP_LAUNCH("fwd_mchain", (int)sizeof(cplx<T>), (mchain_fwd_kernel<T, W>), grid, dim3(64 * W), vlds, st, mf.F,
               mf.Dinv, mf.fronts, mf.idx, mf.cpos, mf.perm, z, vbuf, first, nrhs, (long long)plan.N,
               (long long)plan.sum_pq);
  } else {
    const size_t plds = (size_t)(W - 1) * 2 * 64 * 4 * sizeof(cplx<T>);
    LSP_LAUNCH("bwd_mchain", (int)sizeof(cplx<T>), (mchain_bwd_kernel<T, W>), grid, dim3(64 * W), vlds + plds, st,
               mf.F, mf.Dinv, mf.fronts, mf.idx, x, vbuf, first, nrhs, (long long)plan.N, (long long)plan.sum_pq, xw,
               maxm, xpm, store_x, (int)(l > 0));
  }
}

template <typename T>
void mchain_sweep(bool fwd, const MfDev<T>& mf, const Plan& plan, int l, int nrhs, const cplx<T>* z, cplx<T>* x,
                  cplx<T>* vbuf, hipStream_t st, double2* xw, cplx<T>* xpm) {
  LSP_REQUIRE(plan.level_maxp[l] <= MCP && plan.level_maxpq[l] <= MCM, "matrix-core chain level exceeds its bounds");
  const int W = mchain_waves(plan.level_ptr[l + 1] - plan.level_ptr[l]);
  if (W == 1) mchain_launch<T, 1>(fwd, mf, plan, l, nrhs, z, x, vbuf, st, xw, xpm);
  else if (W == 2) mchain_launch<T, 2>(fwd, mf, plan, l, nrhs, z, x, vbuf, st, xw, xpm);
  else mchain_launch<T, 4>(fwd, mf, plan, l, nrhs, z, x, vbuf, st, xw, xpm);
}

template <typename T>
void launch_point_major(const MfDev<T>& mf, const Plan& plan, int lo, int hi, const cplx<T>* x, cplx<T>* xpm,
                        int nrhs, hipStream_t st) {
  const int first = plan.level_ptr[lo];
  const int cnt = plan.level_ptr[hi] - first;
  if (cnt == 0) return;
  LSP_LAUNCH("point_major", (int)sizeof(cplx<T>), point_major_kernel<T>,
             dim3((unsigned)cnt, (unsigned)((nrhs + MC - 1) / MC)), dim3(256), 0, st, x, xpm, mf.fronts, mf.idx, first,
             nrhs, (long long)plan.N);
}

template <typename T>
void blocked_form(const MfDev<T>& mf, const Plan& plan, int l, hipStream_t st) {
  const int first = plan.level_ptr[l];
  const int cnt = plan.level_ptr[l + 1] - first;
  const int nsbmax = (plan.level_maxp[l] + SB - 1) / SB;
  const int ncol = (std::min(SB, plan.level_maxp[l]) + NF - 1) / NF;
  LSP_LAUNCH("bsweep_form_fwd", (int)sizeof(cplx<T>), bsweep_form_fwd_kernel<T>, dim3(cnt * nsbmax, ncol), dim3(256),
             0, st, mf.F, mf.Dinv, mf.fronts, mf.perm, mf.G, first, nsbmax);
  LSP_LAUNCH("bsweep_form_bwd", (int)sizeof(cplx<T>), bsweep_form_bwd_kernel<T>, dim3(cnt * nsbmax, ncol), dim3(256),
             0, st, mf.F, mf.Dinv, mf.fronts, mf.G, first, nsbmax);
}

template void blocked_sweep<double>(bool, const MfDev<double>&, const Plan&, int, int, const double2*, double2*,
                                    double2*, const SweepBufs<double>&, hipStream_t, double2*);
template void blocked_sweep<float>(bool, const MfDev<float>&, const Plan&, int, int, const float2*, float2*, float2*,
                                   const SweepBufs<float>&, hipStream_t, double2*);
template void mchain_sweep<double>(bool, const MfDev<double>&, const Plan&, int, int, const double2*, double2*,
                                   double2*, hipStream_t, double2*, double2*);
template void mchain_sweep<float>(bool, const MfDev<float>&, const Plan&, int, int, const float2*, float2*, float2*,
                                  hipStream_t, double2*, float2*);
template void launch_point_major<double>(const MfDev<double>&, const Plan&, int, int, const double2*, double2*,
                                         int, hipStream_t);
template void launch_point_major<float>(const MfDev<float>&, const Plan&, int, int, const float2*, float2*, int,
                                        hipStream_t);
template void blocked_form<double>(const MfDev<double>&, const Plan&, int, hipStream_t);
template void blocked_form<float>(const MfDev<float>&, const Plan&, int, hipStream_t);

}  // namespace lsp
