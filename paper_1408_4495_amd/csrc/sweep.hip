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

namespace lsp {

namespace {

constexpr int PB = kNbMax;       // panel width
constexpr int SB = kSweepBlock;  // super-block rows (8 panels)
constexpr int KC = kSweepChunk;  // boundary columns per partial sum
constexpr int GR = 64;           // gemv rows per workgroup (one per lane of a wave)
constexpr int GU = 16;           // gemv column loads in flight per lane
constexpr int NF = 8;            // unit vectors per formation workgroup

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
// columns [clo, chi) of each front (blockIdx.y), right-hand sides r0 ..
// r0 + NR (blockIdx.z), 64-row tiles (blockIdx.x): lane l of wave w owns row
// row0 + l and sums the columns w, w + 4, ... of each staged chunk of GC
// columns; the four waves' sums are added in wave order.
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

template <typename T, int NR, int MODE>
__global__ void __launch_bounds__(256) bsweep_gemv_kernel(const cplx<T>* __restrict__ Fbuf,
                                                          const cplx<T>* __restrict__ Gop,
                                                          const FrontDev* __restrict__ fr, const int* __restrict__ idx,
                                                          cplx<T>* __restrict__ x, cplx<T>* __restrict__ vbuf,
                                                          cplx<T>* __restrict__ ybuf, cplx<T>* __restrict__ pbuf,
                                                          double2* __restrict__ xw, GemvArgs a) {
  constexpr int GC = NR >= 16 ? 128 : 256;  // columns staged per chunk
  __shared__ cplx<T> xin[NR][GC];
  __shared__ cplx<T> part[4][NR][GR];
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
  const int r0 = blockIdx.z * NR, nr = min(NR, a.nrhs - r0);
  const int tid = threadIdx.x, lane = tid % 64, w = tid / 64;
  cplx<T>* vg = vbuf + (long long)r0 * a.vstride + f.idx_off;
  cplx<T>* yg = ybuf + (long long)r0 * a.ystride + (long long)fi * SB;  // y_s(c) at yg[c - s0]
  if constexpr (MODE == MODE_FS) {
    if (blockIdx.x == 0)  // y_s into the front vector at the pivot positions
      for (int e = tid; e < NR * SB; e += 256) {
        const int k = e / SB, c = s0 + e % SB;
        if (k < nr && c < s1) vg[(long long)k * a.vstride + c] = yg[(long long)k * a.ystride + c - s0];
      }
  }
  const int row0 = rlo + tile * GR;
  if (row0 >= rhi || clo >= chi) return;
  const int r = min(row0 + lane, rhi - 1);
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
  cplx<T> acc[NR];
#pragma unroll
  for (int k = 0; k < NR; ++k) acc[k] = mk<T>(0, 0);
  for (int c0 = clo; c0 < chi; c0 += GC) {
    const int cn = min(GC, chi - c0);
    if (c0 > clo) __syncthreads();  // the previous chunk's reads of xin are done
    for (int e = tid; e < NR * GC; e += 256) {
      const int k = e / GC, jj = e % GC;
      if (k < nr && jj < cn) {
        const int c = c0 + jj;
        if constexpr (MODE == MODE_BB) xin[k][jj] = x[(long long)(r0 + k) * a.N + id[c]];
        else if constexpr (MODE == MODE_FS || MODE == MODE_BS) xin[k][jj] = yg[(long long)k * a.ystride + c - s0];
        else xin[k][jj] = vg[(long long)k * a.vstride + c];
      }
    }
    __syncthreads();
    for (int t0 = 0; t0 < GC / 4; t0 += GU) {
      if (w + 4 * t0 >= cn) break;
      cplx<T> av[GU];
#pragma unroll
      for (int u = 0; u < GU; ++u) {
        const int jj = min(w + 4 * (t0 + u), cn - 1);
        av[u] = A[(long long)(c0 + jj - cb) * ld + (r - rb)];
      }
#pragma unroll
      for (int u = 0; u < GU; ++u) {
        const int jj = w + 4 * (t0 + u);
        if (jj < cn)
#pragma unroll
          for (int k = 0; k < NR; ++k) acc[k] = cfma(acc[k], av[u], xin[min(k, nr - 1)][jj]);
      }
    }
  }
#pragma unroll
  for (int k = 0; k < NR; ++k) part[w][k][lane] = acc[k];
  __syncthreads();
  for (int e = tid; e < NR * GR; e += 256) {
    const int k = e / GR, rl = e % GR, rr = row0 + rl;
    if (k < nr && rr < rhi) {
      const cplx<T> sm = cadd(cadd(part[0][k][rl], part[1][k][rl]), cadd(part[2][k][rl], part[3][k][rl]));
      if constexpr (MODE == MODE_W) {
        yg[(long long)k * a.ystride + rr - s0] = sm;
      } else if constexpr (MODE == MODE_V) {
        yg[(long long)k * a.ystride + rr - s0] = sm;
        const long long gi = id[rr];
        x[(long long)(r0 + k) * a.N + gi] = sm;
        if (xw) xw[(long long)(r0 + k) * a.N + gi] = widen(sm);
      } else if constexpr (MODE == MODE_BB) {
        pbuf[((long long)kc * a.nrhs + r0 + k) * a.ystride + (long long)fi * a.maxp + rr] = sm;
      } else {
        cplx<T>* o = vg + (long long)k * a.vstride + rr;
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

template <typename T, int NR, int MODE>
void gemv_launch(const MfDev<T>& mf, const Plan& plan, int l, int s, int nrows, int kch, int nrhs, cplx<T>* x,
                 cplx<T>* vbuf, const SweepBufs<T>& sb, double2* xw, hipStream_t st) {
  if (nrows <= 0) return;
  const int first = plan.level_ptr[l];
  const int cnt = plan.level_ptr[l + 1] - first;
  const int groups = (nrhs + NR - 1) / NR;
  GemvArgs a{first, s, kch, plan.level_maxp[l], nrhs, (long long)plan.N, (long long)plan.sum_pq, sb.ystride};
  LSP_LAUNCH("bsweep_gemv", (int)sizeof(cplx<T>), (bsweep_gemv_kernel<T, NR, MODE>),
             dim3((nrows + GR - 1) / GR * kch, cnt, groups), dim3(256), 0, st, mf.F, mf.G, mf.fronts, mf.idx, x, vbuf,
             sb.ybuf, sb.pbuf, xw, a);
}

template <typename T, int NR>
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
    gemv_launch<T, NR, MODE_W>(mf, plan, l, s, std::min(SB, maxp - s0), 1, nrhs, nullptr, vbuf, sb, nullptr, st);
    int rows = 0;  // rows below the super-block, the most over the level's fronts
    for (int i = first; i < first + cnt; ++i) {
      const FrontDev& f = plan.fronts[i];
      if (f.p > s0) rows = std::max(rows, f.p + f.q - std::min(s0 + SB, f.p));
    }
    // at least one tile, so that tile 0 copies y_s into the front vector
    gemv_launch<T, NR, MODE_FS>(mf, plan, l, s, std::max(rows, 1), 1, nrhs, nullptr, vbuf, sb, nullptr, st);
  }
}

template <typename T, int NR>
void blocked_level_bwd(const MfDev<T>& mf, const Plan& plan, int l, int nrhs, cplx<T>* x, cplx<T>* vbuf,
                       const SweepBufs<T>& sb, hipStream_t st, double2* xw) {
  const int first = plan.level_ptr[l];
  const int cnt = plan.level_ptr[l + 1] - first;
  const int maxp = plan.level_maxp[l];
  int maxq = 0;
  for (int i = first; i < first + cnt; ++i) maxq = std::max(maxq, plan.fronts[i].q);
  if (maxq > 0) {
    const int kch = (maxq + KC - 1) / KC;
    gemv_launch<T, NR, MODE_BB>(mf, plan, l, 0, maxp, kch, nrhs, x, vbuf, sb, nullptr, st);
    GemvArgs a{first, 0, kch, maxp, nrhs, (long long)plan.N, (long long)plan.sum_pq, sb.ystride};
    LSP_LAUNCH("bsweep_bb_reduce", (int)sizeof(cplx<T>), bsweep_bb_reduce_kernel<T>,
               dim3((maxp + 255) / 256, cnt, nrhs), dim3(256), 0, st, mf.fronts, vbuf, sb.pbuf, a);
  }
  const int nsb = (maxp + SB - 1) / SB;
  for (int s = nsb - 1; s >= 0; --s) {
    const int s0 = s * SB;
    gemv_launch<T, NR, MODE_V>(mf, plan, l, s, std::min(SB, maxp - s0), 1, nrhs, x, vbuf, sb, xw, st);
    gemv_launch<T, NR, MODE_BS>(mf, plan, l, s, s0, 1, nrhs, nullptr, vbuf, sb, nullptr, st);
  }
}

// ---- small-front levels with formed operators (Plan::level_sdense)
//
// Fronts of at most 64 pivots and 256 rows, many per level: the forward
// sweep of a front is [0; v_B] + Gf v_I (Gf = m x p, the forward panel chain
// run on the unit vectors, column-major at g_off) and the backward one
// x_I = Gb [y_I; x_B] (Gb^T = m x p column-major after Gf), so a front's
// sweep is one product with no sequential chain.  One workgroup per (front,
// group of NR right-hand sides); a right-hand side's sums run over the
// columns in order, whatever the group.
constexpr int SDP = 64;   // largest p of a small dense level
constexpr int SDM = 256;  // largest m

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

template <typename T, int NR, int TPB>
__global__ void __launch_bounds__(TPB) sdense_fwd_kernel(const cplx<T>* __restrict__ Gop,
                                                         const FrontDev* __restrict__ fr, const int* __restrict__ idx,
                                                         const int* __restrict__ cpos, const cplx<T>* __restrict__ z,
                                                         cplx<T>* __restrict__ vbuf, int first, int nrhs, long long N,
                                                         long long vstride) {
  __shared__ cplx<T> vin[NR][SDP];
  const FrontDev f = fr[first + blockIdx.x];
  const int p = f.p, m = p + f.q;
  const int r0 = blockIdx.y * NR, nr = min(NR, nrhs - r0);
  const int* id = idx + f.idx_off;
  const int* cp = cpos + 2 * f.idx_off;
  const int tid = threadIdx.x;
  for (int e = tid; e < NR * SDP; e += TPB) {
    const int k = e / SDP, c = e % SDP;
    if (k < nr && c < p) vin[k][c] = front_input<T>(f, id, cp, z, vbuf, c, r0 + k, N, vstride);
  }
  __syncthreads();
  const cplx<T>* G = Gop + f.g_off;
  for (int r = tid; r < m; r += TPB) {
    cplx<T> acc[NR];
#pragma unroll
    for (int k = 0; k < NR; ++k) acc[k] = mk<T>(0, 0);
    for (int c0 = 0; c0 < p; c0 += 16) {
      cplx<T> g[16];
#pragma unroll
      for (int u = 0; u < 16; ++u) g[u] = G[(long long)min(c0 + u, p - 1) * m + r];
#pragma unroll
      for (int u = 0; u < 16; ++u)
        if (c0 + u < p)
#pragma unroll
          for (int k = 0; k < NR; ++k) acc[k] = cfma(acc[k], g[u], vin[min(k, nr - 1)][c0 + u]);
    }
#pragma unroll
    for (int k = 0; k < NR; ++k) {
      if (k >= nr) break;
      const cplx<T> out = r >= p ? cadd(front_input<T>(f, id, cp, z, vbuf, r, r0 + k, N, vstride), acc[k]) : acc[k];
      vbuf[(long long)(r0 + k) * vstride + f.idx_off + r] = out;
    }
  }
}

// Four lanes per pivot row i (lane j4 sums the columns j = j4 + 4u), the
// partial sums combined by an xor butterfly (every lane ends with the same
// value).
template <typename T, int NR>
__global__ void __launch_bounds__(256) sdense_bwd_kernel(const cplx<T>* __restrict__ Gop,
                                                         const FrontDev* __restrict__ fr, const int* __restrict__ idx,
                                                         cplx<T>* __restrict__ x, const cplx<T>* __restrict__ vbuf,
                                                         int first, int nrhs, long long N, long long vstride,
                                                         double2* __restrict__ xw) {
  __shared__ cplx<T> vin[NR][SDM];
  const FrontDev f = fr[first + blockIdx.x];
  const int p = f.p, m = p + f.q;
  const int r0 = blockIdx.y * NR, nr = min(NR, nrhs - r0);
  const int* id = idx + f.idx_off;
  const int tid = threadIdx.x;
  for (int e = tid; e < NR * SDM; e += 256) {
    const int k = e / SDM, j = e % SDM;
    if (k < nr && j < m)
      vin[k][j] = j < p ? vbuf[(long long)(r0 + k) * vstride + f.idx_off + j] : x[(long long)(r0 + k) * N + id[j]];
  }
  __syncthreads();
  const int i = tid / 4, j4 = tid % 4;
  const int ii = min(i, p - 1);
  const cplx<T>* G = Gop + f.g_off + (long long)m * p + (long long)ii * m;  // row ii of Gb
  cplx<T> acc[NR];
#pragma unroll
  for (int k = 0; k < NR; ++k) acc[k] = mk<T>(0, 0);
  for (int j0 = 0; j0 < m; j0 += 4 * 16) {
    cplx<T> g[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) g[u] = G[min(j0 + j4 + 4 * u, m - 1)];
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int j = j0 + j4 + 4 * u;
      if (j < m)
#pragma unroll
        for (int k = 0; k < NR; ++k) acc[k] = cfma(acc[k], g[u], vin[min(k, nr - 1)][j]);
    }
  }
#pragma unroll
  for (int k = 0; k < NR; ++k) {
#pragma unroll
    for (int off = 1; off < 4; off <<= 1) {
      acc[k].x += __shfl_xor(acc[k].x, off, 64);
      acc[k].y += __shfl_xor(acc[k].y, off, 64);
    }
  }
  if (j4 == 0 && i < p) {
    const long long gi = id[i];
#pragma unroll
    for (int k = 0; k < NR; ++k) {
      if (k < nr) {
        x[(long long)(r0 + k) * N + gi] = acc[k];
        if (xw) xw[(long long)(r0 + k) * N + gi] = widen(acc[k]);
      }
    }
  }
}

// Formation of a small front's operators: the forward panel chain (TRANS:
// the transposed backward chain, U^T in place of P^T L, whose output for e_i
// is row i of Gb) run on ncol unit vectors at once (columns c0 .. c0 + ncol
// of the identity, blockIdx.y the chunk), the m x ncol block V in LDS (row
// stride ncol + 1).  Per panel: the gathered rows times the inverted
// diagonal block, then the rows below updated with the panel's L21 rows
// (U12 columns), staged in LDS; thread t updates column t % ncol of the rows
// t / ncol, t / ncol + 256 / ncol, ...  Written as columns of Gf (TRANS: of
// Gb^T).
constexpr int SFR = 128;  // rows of a staged panel chunk in the formation

template <typename T, bool TRANS>
__global__ void __launch_bounds__(256) sdense_form_kernel(const cplx<T>* __restrict__ Fbuf,
                                                          const cplx<T>* __restrict__ Dinv,
                                                          const FrontDev* __restrict__ fr, const int* __restrict__ perm,
                                                          cplx<T>* __restrict__ Gop, int first, int ncol) {
  extern __shared__ unsigned char smem_raw[];
  const FrontDev f = fr[first + blockIdx.x];
  const int p = f.p, m = p + f.q;
  const int c0 = blockIdx.y * ncol;
  if (c0 >= p) return;
  const int nc = min(ncol, p - c0), ldv = ncol + 1;
  cplx<T>* V = reinterpret_cast<cplx<T>*>(smem_raw);  // V[r * ldv + c]
  cplx<T>* tb = V + (long long)m * ldv;               // tb[j * ncol + c]
  cplx<T>(*Li)[PB + 1] = reinterpret_cast<cplx<T>(*)[PB + 1]>(tb + PB * ncol);
  cplx<T>* Lp = reinterpret_cast<cplx<T>*>(Li + PB);  // Lp[r' * (PB + 1) + j], r' = r - k1
  const cplx<T>* F = Fbuf + f.f_off;
  const int* pm = perm + f.piv_off;
  const int tid = threadIdx.x;
  const int cc = tid % ncol, rg = tid / ncol, ng = 256 / ncol;
  for (int e = tid; e < m * ncol; e += 256) {
    const int r = e / ncol, c = e % ncol;
    V[r * ldv + c] = mk<T>(r == c0 + c ? 1 : 0, 0);
  }
  for (int k0 = 0; k0 < p; k0 += PB) {
    const int kb = min(PB, p - k0), k1 = k0 + kb, nb = m - k1;
    const cplx<T>* Lg = Dinv + f.dinv_off + (long long)(k0 / PB) * 2 * PB * PB + (TRANS ? PB * PB : 0);
    __syncthreads();  // the previous panel's updates of V and reads of Lp are complete
    for (int e = tid; e < PB * PB; e += 256) {
      const int i = e % PB, j = e / PB;  // entry (i, j) of the column-major block
      if constexpr (TRANS) Li[j][i] = Lg[e];
      else Li[i][j] = Lg[e];
    }
    for (int e = tid; e < PB * ncol; e += 256) {
      const int j = e / ncol, c = e % ncol;
      const int src = j < kb ? (TRANS ? k0 + j : pm[k0 + j]) : k0;
      tb[e] = j < kb ? V[src * ldv + c] : mk<T>(0, 0);
    }
    __syncthreads();
    for (int e = tid; e < PB * ncol; e += 256) {
      const int i = e / ncol, c = e % ncol;
      if (i < kb) {
        // the inverse block is zero outside its kb x kb part and tb's rows
        // past kb are zero, so all 32 terms are summed (exact zeros beyond)
        cplx<T> acc = mk<T>(0, 0);
#pragma unroll
        for (int j = 0; j < PB; ++j) acc = cfma(acc, Li[i][j], tb[j * ncol + c]);
        V[(k0 + i) * ldv + c] = acc;
      }
    }
    // the rows below in chunks of SFR: the panel's entries there, L(r, k0 + j)
    // (TRANS: U(k0 + j, r)), staged in LDS along the matrix's contiguous
    // direction, then the update
    for (int rc = 0; rc < nb; rc += SFR) {
      const int nrw = min(SFR, nb - rc);
      __syncthreads();  // the previous chunk's reads of Lp (and the Y rows above) are complete
      for (int e = tid; e < nrw * kb; e += 256) {
        int rr, j;
        if constexpr (TRANS) { rr = e / kb; j = e % kb; }
        else { rr = e % nrw; j = e / nrw; }
        const int r = k1 + rc + rr;
        Lp[rr * (PB + 1) + j] = TRANS ? F[(long long)(k0 + j) + (long long)r * m] : F[(long long)(k0 + j) * m + r];
      }
      __syncthreads();
      for (int rr = rg; rr < nrw; rr += ng) {
        const int r = k1 + rc + rr;
        cplx<T> acc = V[r * ldv + cc];
#pragma unroll
        for (int j = 0; j < PB; ++j)
          if (j < kb) acc = cfms(acc, Lp[rr * (PB + 1) + j], V[(k0 + j) * ldv + cc]);
        V[r * ldv + cc] = acc;
      }
    }
  }
  __syncthreads();
  cplx<T>* G = Gop + f.g_off + (TRANS ? (long long)m * p : 0LL);
  for (int e = tid; e < m * nc; e += 256) {
    const int c = e / m, r = e % m;
    G[(long long)(c0 + c) * m + r] = V[r * ldv + c];
  }
}

template <typename T, int NR>
void sdense_dispatch(bool fwd, const MfDev<T>& mf, const Plan& plan, int l, int nrhs, const cplx<T>* z, cplx<T>* x,
                     cplx<T>* vbuf, hipStream_t st, double2* xw) {
  const int first = plan.level_ptr[l];
  const int cnt = plan.level_ptr[l + 1] - first;
  const int groups = (nrhs + NR - 1) / NR;
  if (fwd) {
    if (plan.level_maxpq[l] <= 128)
      LSP_LAUNCH("fwd_sdense", (int)sizeof(cplx<T>), (sdense_fwd_kernel<T, NR, 128>), dim3(cnt, groups), dim3(128),
                 0, st, mf.G, mf.fronts, mf.idx, mf.cpos, z, vbuf, first, nrhs, (long long)plan.N,
                 (long long)plan.sum_pq);
    else
      LSP_LAUNCH("fwd_sdense", (int)sizeof(cplx<T>), (sdense_fwd_kernel<T, NR, 256>), dim3(cnt, groups), dim3(256),
                 0, st, mf.G, mf.fronts, mf.idx, mf.cpos, z, vbuf, first, nrhs, (long long)plan.N,
                 (long long)plan.sum_pq);
  } else {
    LSP_LAUNCH("bwd_sdense", (int)sizeof(cplx<T>), (sdense_bwd_kernel<T, NR>), dim3(cnt, groups), dim3(256), 0, st,
               mf.G, mf.fronts, mf.idx, x, vbuf, first, nrhs, (long long)plan.N, (long long)plan.sum_pq, xw);
  }
}

}  // namespace

template <typename T>
void blocked_sweep(bool fwd, const MfDev<T>& mf, const Plan& plan, int l, int nrhs, const cplx<T>* z, cplx<T>* x,
                   cplx<T>* vbuf, const SweepBufs<T>& sb, hipStream_t st, double2* xw) {
#define LSP_BLOCKED(NR)                                               \
  do {                                                                \
    if (fwd) blocked_level_fwd<T, NR>(mf, plan, l, nrhs, z, vbuf, sb, st); \
    else blocked_level_bwd<T, NR>(mf, plan, l, nrhs, x, vbuf, sb, st, xw); \
  } while (0)
  if (nrhs >= 16) LSP_BLOCKED(16);
  else if (nrhs >= 8) LSP_BLOCKED(8);
  else if (nrhs >= 4) LSP_BLOCKED(4);
  else if (nrhs >= 2) LSP_BLOCKED(2);
  else LSP_BLOCKED(1);
#undef LSP_BLOCKED
}

template <typename T>
void sdense_sweep(bool fwd, const MfDev<T>& mf, const Plan& plan, int l, int nrhs, const cplx<T>* z, cplx<T>* x,
                  cplx<T>* vbuf, hipStream_t st, double2* xw) {
  LSP_REQUIRE(plan.level_maxp[l] <= SDP && plan.level_maxpq[l] <= SDM, "small dense level exceeds its bounds");
  if (nrhs >= 8) sdense_dispatch<T, 8>(fwd, mf, plan, l, nrhs, z, x, vbuf, st, xw);
  else if (nrhs >= 4) sdense_dispatch<T, 4>(fwd, mf, plan, l, nrhs, z, x, vbuf, st, xw);
  else if (nrhs >= 2) sdense_dispatch<T, 2>(fwd, mf, plan, l, nrhs, z, x, vbuf, st, xw);
  else sdense_dispatch<T, 1>(fwd, mf, plan, l, nrhs, z, x, vbuf, st, xw);
}

template <typename T>
void sdense_form(const MfDev<T>& mf, const Plan& plan, int l, hipStream_t st) {
  const int first = plan.level_ptr[l];
  const int cnt = plan.level_ptr[l + 1] - first;
  const int maxm = plan.level_maxpq[l], maxp = plan.level_maxp[l];
  // unit vectors per workgroup: the most (64 .. 8) whose block fits 48 KB
  int ncol = 64;
  while (ncol > 8 && (size_t)maxm * (ncol + 1) * sizeof(cplx<T>) > 48 * 1024) ncol /= 2;
  const size_t lds = ((size_t)maxm * (ncol + 1) + (size_t)PB * ncol + (size_t)PB * (PB + 1) +
                      (size_t)SFR * (PB + 1)) * sizeof(cplx<T>);
  const dim3 grid(cnt, (maxp + ncol - 1) / ncol);
  LSP_LAUNCH("sdense_form_fwd", (int)sizeof(cplx<T>), (sdense_form_kernel<T, false>), grid, dim3(256), lds, st, mf.F,
             mf.Dinv, mf.fronts, mf.perm, mf.G, first, ncol);
  LSP_LAUNCH("sdense_form_bwd", (int)sizeof(cplx<T>), (sdense_form_kernel<T, true>), grid, dim3(256), lds, st, mf.F,
             mf.Dinv, mf.fronts, mf.perm, mf.G, first, ncol);
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
template void sdense_sweep<double>(bool, const MfDev<double>&, const Plan&, int, int, const double2*, double2*,
                                   double2*, hipStream_t, double2*);
template void sdense_sweep<float>(bool, const MfDev<float>&, const Plan&, int, int, const float2*, float2*, float2*,
                                  hipStream_t, double2*);
template void sdense_form<double>(const MfDev<double>&, const Plan&, int, hipStream_t);
template void sdense_form<float>(const MfDev<float>&, const Plan&, int, hipStream_t);
template void blocked_form<double>(const MfDev<double>&, const Plan&, int, hipStream_t);
template void blocked_form<float>(const MfDev<float>&, const Plan&, int, hipStream_t);

}  // namespace lsp
