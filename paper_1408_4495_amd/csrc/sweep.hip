// Blocked triangular sweeps for the tree levels with large fronts.
//
// The multifrontal solve x = M^{-1} z (the preconditioner of eq:PC, with the
// factors of Section 2.2's nested dissection) walks every front twice.  The
// panel-chain kernels give each front one workgroup, which on the upper
// levels (a handful of fronts with thousands of rows) leaves the chip idle
// and streams megabytes of factor through one compute unit.  Here a front's
// sweep is split into a short sequential part and wide parallel parts:
//
// forward, front rows [I | B], p pivots, panels of 32 grouped in super-blocks
// of SB = 256 rows:
//   gather   v = [z(I); 0] + children's updates             (one launch)
//   for each super-block s = [s0, s1):
//     chain  the panels of s on their own rows:              (one workgroup
//            y_b = L11_b^{-1} (P_b v_b),                      per front and
//            v(k1:s1) -= L(k1:s1, b) y_b                      right-hand-side
//                                                             group)
//     gemv   v(s1:m) -= L(s1:m, s0:s1) y_s                   (64-row tiles)
// backward:
//   gemv     t_I = y_I - U(0:p, p:m) x_B, x_B read from the solution
//   for each super-block s from the last:
//     chain  x_b = U11_b^{-1} (t_b - U(b, k1:s1) x(k1:s1))
//     gemv   t(0:s0) -= U(0:s0, s0:s1) x_s
//
// The arithmetic is the panel chain's, regrouped: every factor entry is read
// once per right-hand-side group and each right-hand side's sums run in an
// order that does not depend on the group, so a right-hand side solved in a
// batch gets its solo result bit for bit.
#include <algorithm>

#include "lsp_common.h"
#include "kernels.h"

namespace lsp {

namespace {

constexpr int PB = kNbMax;   // panel width
constexpr int SB = kSweepBlock;  // super-block rows (8 panels)
constexpr int GR = 64;       // gemv rows per workgroup (one per lane of a wave)
constexpr int GU = 16;       // gemv column loads in flight per lane

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

// Forward chain over the panels of super-block [s0, s1) of each front
// (blockIdx.x), right-hand sides r0 .. r0 + NR (blockIdx.y), the rows of the
// super-block staged in LDS.
template <typename T, int NR>
__global__ void __launch_bounds__(256) bsweep_fwd_chain_kernel(const cplx<T>* __restrict__ Fbuf,
                                                               const cplx<T>* __restrict__ Dinv,
                                                               const FrontDev* __restrict__ fr,
                                                               const int* __restrict__ perm, cplx<T>* __restrict__ vbuf,
                                                               int first, int s0, int nrhs, long long vstride) {
  __shared__ cplx<T> v[NR][SB];
  __shared__ cplx<T> Li[PB][PB + 1];
  __shared__ cplx<T> tb[NR][PB];
  __shared__ cplx<T> yb[NR][PB];
  const FrontDev f = fr[first + blockIdx.x];
  if (f.p <= s0) return;
  const int s1 = min(s0 + SB, f.p), len = s1 - s0;
  const int m = f.p + f.q;
  const int r0 = blockIdx.y * NR, nr = min(NR, nrhs - r0);
  const cplx<T>* F = Fbuf + f.f_off;
  const int* pm = perm + f.piv_off;
  cplx<T>* vg = vbuf + (long long)r0 * vstride + f.idx_off;
  const int tid = threadIdx.x;
  for (int e = tid; e < NR * SB; e += 256) {
    const int k = e / SB, r = e % SB;
    if (k < nr && r < len) v[k][r] = vg[(long long)k * vstride + s0 + r];
  }
  for (int k0 = s0; k0 < s1; k0 += PB) {
    const int kb = min(PB, f.p - k0), k1 = k0 + kb;
    const cplx<T>* Lg = Dinv + f.dinv_off + (long long)(k0 / PB) * 2 * PB * PB;
    const cplx<T> l0 = Lg[tid], l1 = Lg[tid + 256], l2 = Lg[tid + 512], l3 = Lg[tid + 768];
    // the rows below this panel inside the super-block: one row per thread
    const int r = k1 + tid;
    const int rr = min(r, s1 - 1);
    cplx<T> lrow[PB];
#pragma unroll
    for (int j = 0; j < PB; ++j) lrow[j] = F[(long long)(k0 + min(j, kb - 1)) * m + rr];
    __syncthreads();  // the previous panel's updates of v are complete
    Li[tid % PB][tid / PB] = l0;
    Li[tid % PB][tid / PB + 8] = l1;
    Li[tid % PB][tid / PB + 16] = l2;
    Li[tid % PB][tid / PB + 24] = l3;
    if (tid < NR * PB) {
      const int k = tid / PB, j = tid % PB;
      tb[k][j] = (k < nr && j < kb) ? v[k][pm[k0 + j] - s0] : mk<T>(0, 0);
    }
    __syncthreads();
    {
      cplx<T> y[NR];
      tri_apply<T, NR>(Li, tb, tid, y);
      const int i = tid / 8;
      if (tid % 8 == 0) {
#pragma unroll
        for (int k = 0; k < NR; ++k) {
          yb[k][i] = y[k];
          if (k < nr && i < kb) v[k][k0 - s0 + i] = y[k];
        }
      }
    }
    __syncthreads();
    if (r < s1) {
#pragma unroll
      for (int k = 0; k < NR; ++k) {
        if (k >= nr) break;
        cplx<T> acc = v[k][r - s0];
#pragma unroll
        for (int j = 0; j < PB; ++j)
          if (j < kb) acc = cfms(acc, lrow[j], yb[k][j]);
        v[k][r - s0] = acc;
      }
    }
  }
  __syncthreads();
  for (int e = tid; e < NR * SB; e += 256) {
    const int k = e / SB, r = e % SB;
    if (k < nr && r < len) vg[(long long)k * vstride + s0 + r] = v[k][r];
  }
}

// Backward chain over the panels of super-block [s0, s1), from the last:
// x_b = U11_b^{-1} (t_b - U(b, k1:s1) x(k1:s1)); x goes to the front vector,
// to the solution at the pivots' grid points and, when xw is given, widened
// to complex128 there too.
template <typename T, int NR>
__global__ void __launch_bounds__(256) bsweep_bwd_chain_kernel(const cplx<T>* __restrict__ Fbuf,
                                                               const cplx<T>* __restrict__ Dinv,
                                                               const FrontDev* __restrict__ fr,
                                                               const int* __restrict__ idx, cplx<T>* __restrict__ x,
                                                               cplx<T>* __restrict__ vbuf, int first, int s0, int nrhs,
                                                               long long N, long long vstride,
                                                               double2* __restrict__ xw) {
  constexpr int G = 256 / PB;  // column groups
  __shared__ cplx<T> v[NR][SB];
  __shared__ cplx<T> Ui[PB][PB + 1];
  __shared__ cplx<T> part[G][NR][PB];
  __shared__ cplx<T> rb[NR][PB];
  const FrontDev f = fr[first + blockIdx.x];
  if (f.p <= s0) return;
  const int s1 = min(s0 + SB, f.p), len = s1 - s0;
  const int m = f.p + f.q;
  const int r0 = blockIdx.y * NR, nr = min(NR, nrhs - r0);
  const cplx<T>* F = Fbuf + f.f_off;
  const int* id = idx + f.idx_off;
  cplx<T>* vg = vbuf + (long long)r0 * vstride + f.idx_off;
  const int tid = threadIdx.x;
  const int j = tid % PB, grp = tid / PB;
  for (int e = tid; e < NR * SB; e += 256) {
    const int k = e / SB, r = e % SB;
    if (k < nr && r < len) v[k][r] = vg[(long long)k * vstride + s0 + r];
  }
  const int nb = (len + PB - 1) / PB;
  for (int b = nb - 1; b >= 0; --b) {
    const int k0 = s0 + b * PB, kb = min(PB, f.p - k0), k1 = k0 + kb;
    const cplx<T>* Ug = Dinv + f.dinv_off + (long long)(k0 / PB) * 2 * PB * PB + PB * PB;
    const cplx<T> u0 = Ug[tid], u1 = Ug[tid + 256], u2 = Ug[tid + 512], u3 = Ug[tid + 768];
    // U(k0 + j, c) for this thread's columns c = k1 + grp + 8 t < s1 (at most 28)
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
    cplx<T> acc[NR];
#pragma unroll
    for (int k = 0; k < NR; ++k) acc[k] = mk<T>(0, 0);
#pragma unroll
    for (int t = 0; t < TU; ++t) {
      const int c = k1 + grp + G * t;
      if (c < s1)
#pragma unroll
        for (int k = 0; k < NR; ++k) acc[k] = cfma(acc[k], ucol[t], v[min(k, nr - 1)][c - s0]);
    }
#pragma unroll
    for (int k = 0; k < NR; ++k) part[grp][k][j] = acc[k];
    __syncthreads();
    for (int e = tid; e < NR * PB; e += 256) {
      const int jj = e % PB, k = e / PB;
      cplx<T> s = part[0][k][jj];
#pragma unroll
      for (int g = 1; g < G; ++g) s = cadd(s, part[g][k][jj]);
      rb[k][jj] = (k < nr && jj < kb) ? csub(v[k][k0 - s0 + jj], s) : mk<T>(0, 0);
    }
    __syncthreads();
    {
      cplx<T> xs[NR];
      tri_apply<T, NR>(Ui, rb, tid, xs);
      const int i = tid / 8;
      if (tid % 8 == 0 && i < kb) {
        const long long gi = id[k0 + i];
#pragma unroll
        for (int k = 0; k < NR; ++k) {
          if (k < nr) {
            v[k][k0 - s0 + i] = xs[k];
            x[(long long)(r0 + k) * N + gi] = xs[k];
            if (xw) xw[(long long)(r0 + k) * N + gi] = widen(xs[k]);
          }
        }
      }
    }
  }
  __syncthreads();
  for (int e = tid; e < NR * SB; e += 256) {
    const int k = e / SB, r = e % SB;
    if (k < nr && r < len) vg[(long long)k * vstride + s0 + r] = v[k][r];
  }
}

// out(r) -= sum_c F(r, c) in(c) over a rectangle of each front's matrix
// (column-major, leading dimension m), for the right-hand sides r0 .. r0+NR:
//   MODE 0 (forward step):  rows [s1, m), columns [s0, s1), in = y in the
//                           front vector;
//   MODE 2 (backward B):    rows [0, p),  columns [p, m),  in = x_B read
//                           from the solution at the front's grid points;
//   MODE 3 (backward step): rows [0, s0), columns [s0, s1), in = x in the
//                           front vector;
// with s1 = min(s0 + SB, p).  Workgroup (64-row tile, front, group): lane l
// of wave w owns row row0 + l and sums the columns w, w + 4, ... of each
// staged chunk of GC columns; the four waves' sums are added in wave order.
template <typename T, int NR, int MODE>
__global__ void __launch_bounds__(256) bsweep_gemv_kernel(const cplx<T>* __restrict__ Fbuf,
                                                          const FrontDev* __restrict__ fr, const int* __restrict__ idx,
                                                          const cplx<T>* __restrict__ x, cplx<T>* __restrict__ vbuf,
                                                          int first, int s0, int nrhs, long long N,
                                                          long long vstride) {
  constexpr int GC = NR >= 16 ? 128 : 256;  // columns staged per chunk
  __shared__ cplx<T> xin[NR][GC];
  __shared__ cplx<T> part[4][NR][GR];
  const FrontDev f = fr[first + blockIdx.y];
  const int p = f.p, m = p + f.q;
  const int s1 = min(s0 + SB, p);
  int rlo, rhi, clo, chi;
  if constexpr (MODE == 0) { rlo = s1; rhi = m; clo = s0; chi = s1; }
  else if constexpr (MODE == 2) { rlo = 0; rhi = p; clo = p; chi = m; }
  else { rlo = 0; rhi = min(s0, p); clo = s0; chi = s1; }
  const int row0 = rlo + blockIdx.x * GR;
  if (row0 >= rhi || clo >= chi) return;
  const int r0 = blockIdx.z * NR, nr = min(NR, nrhs - r0);
  const int tid = threadIdx.x, lane = tid % 64, w = tid / 64;
  const int r = min(row0 + lane, rhi - 1);
  const cplx<T>* F = Fbuf + f.f_off;
  const int* id = idx + f.idx_off;
  cplx<T>* vg = vbuf + (long long)r0 * vstride + f.idx_off;
  cplx<T> acc[NR];
#pragma unroll
  for (int k = 0; k < NR; ++k) acc[k] = mk<T>(0, 0);
  for (int c0 = clo; c0 < chi; c0 += GC) {
    const int cn = min(GC, chi - c0);
    if (c0 > clo) __syncthreads();  // the previous chunk's reads of xin are done
    for (int e = tid; e < NR * GC; e += 256) {
      const int k = e / GC, jj = e % GC;
      if (k < nr && jj < cn) {
        if constexpr (MODE == 2) xin[k][jj] = x[(long long)(r0 + k) * N + id[c0 + jj]];
        else xin[k][jj] = vg[(long long)k * vstride + c0 + jj];
      }
    }
    __syncthreads();
    for (int t0 = 0; t0 < GC / 4; t0 += GU) {
      if (w + 4 * t0 >= cn) break;
      cplx<T> a[GU];
#pragma unroll
      for (int u = 0; u < GU; ++u) {
        const int jj = min(w + 4 * (t0 + u), cn - 1);
        a[u] = F[(long long)(c0 + jj) * m + r];
      }
#pragma unroll
      for (int u = 0; u < GU; ++u) {
        const int jj = w + 4 * (t0 + u);
        if (jj < cn)
#pragma unroll
          for (int k = 0; k < NR; ++k) acc[k] = cfma(acc[k], a[u], xin[min(k, nr - 1)][jj]);
      }
    }
  }
#pragma unroll
  for (int k = 0; k < NR; ++k) part[w][k][lane] = acc[k];
  __syncthreads();
  for (int e = tid; e < NR * GR; e += 256) {
    const int k = e / GR, rl = e % GR, rr = row0 + rl;
    if (k < nr && rr < rhi) {
      cplx<T> s = cadd(cadd(part[0][k][rl], part[1][k][rl]), cadd(part[2][k][rl], part[3][k][rl]));
      cplx<T>* o = vg + (long long)k * vstride + rr;
      *o = csub(*o, s);
    }
  }
}

template <typename T, int NR, int MODE>
void gemv_launch(const MfDev<T>& mf, const Plan& plan, int l, int s0, int nrows, int nrhs, const cplx<T>* x,
                 cplx<T>* vbuf, hipStream_t st) {
  if (nrows <= 0) return;
  const int first = plan.level_ptr[l];
  const int cnt = plan.level_ptr[l + 1] - first;
  const int groups = (nrhs + NR - 1) / NR;
  LSP_LAUNCH("bsweep_gemv", (int)sizeof(cplx<T>), (bsweep_gemv_kernel<T, NR, MODE>),
             dim3((nrows + GR - 1) / GR, cnt, groups), dim3(256), 0, st, mf.F, mf.fronts, mf.idx, x, vbuf, first, s0,
             nrhs, (long long)plan.N, (long long)plan.sum_pq);
}

template <typename T, int NR>
void blocked_level_fwd(const MfDev<T>& mf, const Plan& plan, int l, int nrhs, const cplx<T>* z, cplx<T>* vbuf,
                       hipStream_t st) {
  constexpr int NG = NR > 8 ? 8 : NR;  // chain right-hand sides per workgroup
  const int first = plan.level_ptr[l];
  const int cnt = plan.level_ptr[l + 1] - first;
  const int maxm = plan.level_maxpq[l], maxp = plan.level_maxp[l];
  LSP_LAUNCH("bsweep_gather", (int)sizeof(cplx<T>), bsweep_gather_kernel<T>, dim3((maxm + 255) / 256, cnt, nrhs),
             dim3(256), 0, st, mf.fronts, mf.idx, mf.cpos, z, vbuf, first, (long long)plan.N, (long long)plan.sum_pq);
  const int cgroups = (nrhs + NG - 1) / NG;
  for (int s0 = 0; s0 < maxp; s0 += SB) {
    LSP_LAUNCH("bsweep_fwd_chain", (int)sizeof(cplx<T>), (bsweep_fwd_chain_kernel<T, NG>), dim3(cnt, cgroups),
               dim3(256), 0, st, mf.F, mf.Dinv, mf.fronts, mf.perm, vbuf, first, s0, nrhs, (long long)plan.sum_pq);
    // rows below the super-block, the most over the level's fronts
    int rows = 0;
    for (int i = first; i < first + cnt; ++i) {
      const FrontDev& f = plan.fronts[i];
      if (f.p > s0) rows = std::max(rows, f.p + f.q - std::min(s0 + SB, f.p));
    }
    gemv_launch<T, NR, 0>(mf, plan, l, s0, rows, nrhs, nullptr, vbuf, st);
  }
}

template <typename T, int NR>
void blocked_level_bwd(const MfDev<T>& mf, const Plan& plan, int l, int nrhs, cplx<T>* x, cplx<T>* vbuf,
                       hipStream_t st, double2* xw) {
  constexpr int NG = NR > 8 ? 8 : NR;
  const int first = plan.level_ptr[l];
  const int cnt = plan.level_ptr[l + 1] - first;
  const int maxp = plan.level_maxp[l];
  gemv_launch<T, NR, 2>(mf, plan, l, 0, maxp, nrhs, x, vbuf, st);
  const int cgroups = (nrhs + NG - 1) / NG;
  const int nsb = (maxp + SB - 1) / SB;
  for (int s = nsb - 1; s >= 0; --s) {
    const int s0 = s * SB;
    LSP_LAUNCH("bsweep_bwd_chain", (int)sizeof(cplx<T>), (bsweep_bwd_chain_kernel<T, NG>), dim3(cnt, cgroups),
               dim3(256), 0, st, mf.F, mf.Dinv, mf.fronts, mf.idx, x, vbuf, first, s0, nrhs, (long long)plan.N,
               (long long)plan.sum_pq, xw);
    gemv_launch<T, NR, 3>(mf, plan, l, s0, s0, nrhs, nullptr, vbuf, st);
  }
}

template <typename T, int NR>
void blocked_dispatch(bool fwd, const MfDev<T>& mf, const Plan& plan, int l, int nrhs, const cplx<T>* z, cplx<T>* x,
                      cplx<T>* vbuf, hipStream_t st, double2* xw) {
  if (fwd) blocked_level_fwd<T, NR>(mf, plan, l, nrhs, z, vbuf, st);
  else blocked_level_bwd<T, NR>(mf, plan, l, nrhs, x, vbuf, st, xw);
}

}  // namespace

template <typename T>
void blocked_sweep(bool fwd, const MfDev<T>& mf, const Plan& plan, int l, int nrhs, const cplx<T>* z, cplx<T>* x,
                   cplx<T>* vbuf, hipStream_t st, double2* xw) {
  if (nrhs >= 16) blocked_dispatch<T, 16>(fwd, mf, plan, l, nrhs, z, x, vbuf, st, xw);
  else if (nrhs >= 8) blocked_dispatch<T, 8>(fwd, mf, plan, l, nrhs, z, x, vbuf, st, xw);
  else if (nrhs >= 4) blocked_dispatch<T, 4>(fwd, mf, plan, l, nrhs, z, x, vbuf, st, xw);
  else if (nrhs >= 2) blocked_dispatch<T, 2>(fwd, mf, plan, l, nrhs, z, x, vbuf, st, xw);
  else blocked_dispatch<T, 1>(fwd, mf, plan, l, nrhs, z, x, vbuf, st, xw);
}

template void blocked_sweep<double>(bool, const MfDev<double>&, const Plan&, int, int, const double2*, double2*,
                                    double2*, hipStream_t, double2*);
template void blocked_sweep<float>(bool, const MfDev<float>&, const Plan&, int, int, const float2*, float2*, float2*,
                                   hipStream_t, double2*);

}  // namespace lsp
