// Device kernels of restarted right-preconditioned GMRES (the iterative
// solver of Section 3.3), run as one independent Krylov process per
// right-hand side.  Vectors are complex128 blocks; a basis is stored as
// [k][nrhs][N] so that vector k of every right-hand side is one contiguous
// [nrhs][N] block.  Reductions are two-stage with a fixed block count and a
// fixed summation order, so a right-hand side's arithmetic does not depend
// on which other right-hand sides share the batch.
//
// Arnoldi uses classical Gram-Schmidt applied twice (CGS2): h = V^H w,
// w -= V h, h2 = V^H w, w -= V h2, H(:,k) = h + h2, H(k+1,k) = ||w||.  The
// Hessenberg matrix is reduced by Givens rotations as it grows (the
// rotation that zeroes H(k+1,k) is c = |a|/r, s = (a/|a|) conj(b)/r with
// a = H(k,k), b = H(k+1,k), r = sqrt(|a|^2+|b|^2)); |gamma(k+1)| is the
// residual estimate.
#include "lsp_common.h"
#include "krylov.h"

namespace lsp {

namespace {

constexpr int KB = 256;  // threads per block of the reduction kernels

__device__ inline double2 wave_sum(double2 v) {
  for (int off = 32; off > 0; off >>= 1) {
    v.x += __shfl_down(v.x, off, 64);
    v.y += __shfl_down(v.y, off, 64);
  }
  return v;
}

// partial[rhs][blk][i] = sum over this block's chunk of conj(V_i) w, i < nvec.
// V_i of rhs r is at V + (i * nrhs + r) * N.
template <int NV>
__global__ void __launch_bounds__(KB) dots_partial_kernel(const double2* __restrict__ V, const double2* __restrict__ w,
                                                          double2* __restrict__ partial, int nvec, long long N,
                                                          int nrhs, const int* __restrict__ active) {
  const int r = blockIdx.y, blk = blockIdx.x, nblk = gridDim.x;
  if (active && !active[r]) return;
  const long long e0 = N * blk / nblk, e1 = N * (blk + 1) / nblk;
  double2 acc[NV];
#pragma unroll
  for (int i = 0; i < NV; ++i) acc[i] = make_double2(0, 0);
  const double2* wr = w + (long long)r * N;
  // four elements per thread per pass, their loads issued together
  for (long long eb = e0 + threadIdx.x; eb < e1; eb += 4 * KB) {
    double2 we[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) we[u] = eb + u * KB < e1 ? wr[eb + u * KB] : make_double2(0, 0);
#pragma unroll
    for (int i = 0; i < NV; ++i) {
      if (i < nvec) {
        const double2* Vi = V + ((long long)i * nrhs + r) * N;
        double2 ve[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) ve[u] = eb + u * KB < e1 ? Vi[eb + u * KB] : make_double2(0, 0);
#pragma unroll
        for (int u = 0; u < 4; ++u) acc[i] = cadd(acc[i], cmulc(ve[u], we[u]));
      }
    }
  }
  __shared__ double2 ws[KB / 64][kMaxVec];
  const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
#pragma unroll
  for (int i = 0; i < NV; ++i) {
    if (i < nvec) {
      double2 s = wave_sum(acc[i]);
      if (lane == 0) ws[wave][i] = s;
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i < nvec; i += KB) {
    double2 s = ws[0][i];
    for (int k = 1; k < KB / 64; ++k) s = cadd(s, ws[k][i]);
    partial[((long long)r * nblk + blk) * kMaxVec + i] = s;
  }
}

// h[rhs][i] = sum_blk partial; mode 0: H(i,k) = h, mode 1: H(i,k) += h,
// mode 2: norm -> H(k+1,k) = sqrt(re h0), inv[r] = 1/that (0 if zero).
// 256 threads: thread (s, i) sums the partials of blocks s, s+8, ... of
// vector i with all its loads in flight at once; the eight slice sums are
// then combined in slice order, so the result depends only on nblk.
constexpr int kFinSlices = 8;
__global__ void __launch_bounds__(kFinSlices * kMaxVec) dots_final_kernel(
    const double2* __restrict__ partial, double2* __restrict__ h, double2* __restrict__ H, double* __restrict__ scal,
    int nvec, int nblk, int k, int restart, int mode, const int* __restrict__ active) {
  const int r = blockIdx.x;
  if (active && !active[r]) return;
  const int i = threadIdx.x % kMaxVec, sl = threadIdx.x / kMaxVec;
  __shared__ double2 red[kFinSlices][kMaxVec];
  double2 acc = make_double2(0, 0);
  if (i < nvec) {
    const double2* pr = partial + (long long)r * nblk * kMaxVec + i;
    double2 v[8];
    for (int b0 = sl; b0 < nblk; b0 += 8 * kFinSlices) {
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int b = b0 + u * kFinSlices;
        v[u] = b < nblk ? pr[(long long)b * kMaxVec] : make_double2(0, 0);
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) acc = cadd(acc, v[u]);
    }
  }
  red[sl][i] = acc;
  __syncthreads();
  if (sl != 0 || i >= nvec) return;
  double2 s = red[0][i];
#pragma unroll
  for (int q = 1; q < kFinSlices; ++q) s = cadd(s, red[q][i]);
  h[(long long)r * kMaxVec + i] = s;
  double2* Hr = H + (long long)r * (restart + 1) * restart;
  if (mode == 0) Hr[i + (restart + 1) * k] = s;
  else if (mode == 1) Hr[i + (restart + 1) * k] = cadd(Hr[i + (restart + 1) * k], s);
  else {
    double nrm = sqrt(fmax(s.x, 0.0));
    if (k >= 0) Hr[(k + 1) + (restart + 1) * k] = make_double2(nrm, 0.0);
    scal[r * kScal + S_NORM] = nrm;
    scal[r * kScal + S_INV] = nrm > 0 ? 1.0 / nrm : 0.0;
  }
}

// ---- fused Arnoldi orthogonalisation (CGS2 and the norm, five launches per
// step instead of ten): a kernel that consumes a reduction forms its final
// sums itself, identically in every block (fixed order), instead of a
// separate final launch.

// hs[i] = sum over blocks of pin[r][blk][i], i < nvec: thread (i, sl) sums
// blocks sl, sl + 8, ... with its loads in flight together; the eight slice
// sums are then added in slice order.  256 threads; ends with a barrier.
__device__ void final_sums(const double2* __restrict__ pin, int r, int nblk, int nvec, double2* hs,
                           double2 (*red)[kMaxVec]) {
  const int i = threadIdx.x % kMaxVec, sl = threadIdx.x / kMaxVec;
  double2 acc = make_double2(0, 0);
  if (i < nvec) {
    const double2* pr = pin + (long long)r * nblk * kMaxVec + i;
    double2 v[8];
    for (int b0 = sl; b0 < nblk; b0 += 8 * kFinSlices) {
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int b = b0 + u * kFinSlices;
        v[u] = b < nblk ? pr[(long long)b * kMaxVec] : make_double2(0, 0);
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) acc = cadd(acc, v[u]);
    }
  }
  red[sl][i] = acc;
  __syncthreads();
  if (sl == 0 && i < nvec) {
    double2 t = red[0][i];
#pragma unroll
    for (int q = 1; q < kFinSlices; ++q) t = cadd(t, red[q][i]);
    hs[i] = t;
  }
  __syncthreads();
}

// This block's partial sums acc[i], i < nvec, combined over its waves in a
// fixed order and written to pout[r][blk][i].
template <int NV>
__device__ void block_partials(const double2 (&acc)[NV], int nvec, double2* __restrict__ pout, int r, int blk,
                               int nblk) {
  __shared__ double2 ws[KB / 64][kMaxVec];
  const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
#pragma unroll
  for (int i = 0; i < NV; ++i) {
    if (i < nvec) {
      double2 s = wave_sum(acc[i]);
      if (lane == 0) ws[wave][i] = s;
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i < nvec; i += KB) {
    double2 s = ws[0][i];
    for (int q = 1; q < KB / 64; ++q) s = cadd(s, ws[q][i]);
    pout[((long long)r * nblk + blk) * kMaxVec + i] = s;
  }
}

// One Gram-Schmidt pass of Arnoldi step k: h = V^H w from the partial sums
// pin (block 0 records it: mode 0 sets H(0:k, k), mode 1 adds), w -= V h over
// this block's elements, then this block's partial sums of the next
// reduction to pout: V^H w (NEXT == 0) or ||w||^2 (NEXT == 1).  The element
// partition and the per-thread order match dots_partial_kernel.
template <int NEXT, int NV>
__global__ void __launch_bounds__(KB) cgs_kernel(const double2* __restrict__ V, double2* __restrict__ w,
                                                 const double2* __restrict__ pin, double2* __restrict__ pout,
                                                 double2* __restrict__ h, double2* __restrict__ H, int nvec, long long N,
                                                 int nrhs, int k, int restart, int mode,
                                                 const int* __restrict__ active) {
  const int r = blockIdx.y, blk = blockIdx.x, nblk = gridDim.x;
  if (active && !active[r]) return;
  __shared__ double2 hs[kMaxVec];
  __shared__ double2 red[kFinSlices][kMaxVec];
  final_sums(pin, r, nblk, nvec, hs, red);
  if (blk == 0 && threadIdx.x < nvec) {
    const int i = threadIdx.x;
    h[(long long)r * kMaxVec + i] = hs[i];
    double2* Hc = H + (long long)r * (restart + 1) * restart + (restart + 1) * k;
    Hc[i] = mode == 0 ? hs[i] : cadd(Hc[i], hs[i]);
  }
  double2 hv[NV];
#pragma unroll
  for (int i = 0; i < NV; ++i) hv[i] = i < nvec ? hs[i] : make_double2(0, 0);
  const long long e0 = N * blk / nblk, e1 = N * (blk + 1) / nblk;
  constexpr int NA = NEXT == 0 ? NV : 1;
  double2 acc[NA];
#pragma unroll
  for (int i = 0; i < NA; ++i) acc[i] = make_double2(0, 0);
  double2* wr = w + (long long)r * N;
  // EP elements per thread per pass (e, e + KB, ...), their loads issued
  // together; the sums take them in element order.  Up to 8 vectors the
  // loaded V entries are kept for the second product, beyond that they are
  // loaded again (cached), so the registers stay within bounds.
  constexpr int EP = NV <= 4 ? 2 : 1;
  constexpr bool HOLD = NV <= 8;
  for (long long e = e0 + threadIdx.x; e < e1; e += EP * KB) {
    long long ee[EP];
    bool ok[EP];
#pragma unroll
    for (int u = 0; u < EP; ++u) {
      ok[u] = e + u * KB < e1;
      ee[u] = ok[u] ? e + u * KB : e;
    }
    double2 sv[EP];
#pragma unroll
    for (int u = 0; u < EP; ++u) sv[u] = wr[ee[u]];
    double2 vv[HOLD ? NV : 1][EP];
#pragma unroll
    for (int i = 0; i < NV; ++i)
      if (i < nvec) {
#pragma unroll
        for (int u = 0; u < EP; ++u) {
          const double2 v = V[((long long)i * nrhs + r) * N + ee[u]];
          if constexpr (HOLD) vv[i][u] = v;
          sv[u] = cfms(sv[u], hv[i], v);
        }
      }
#pragma unroll
    for (int u = 0; u < EP; ++u)
      if (ok[u]) wr[ee[u]] = sv[u];
#pragma unroll
    for (int u = 0; u < EP; ++u) {
      if (!ok[u]) break;
      if constexpr (NEXT == 0) {
#pragma unroll
        for (int i = 0; i < NV; ++i)
          if (i < nvec) {
            double2 v;
            if constexpr (HOLD) v = vv[i][u];
            else v = V[((long long)i * nrhs + r) * N + ee[u]];
            acc[i] = cadd(acc[i], cmulc(v, sv[u]));
          }
      } else {
        acc[0] = cadd(acc[0], cmulc(sv[u], sv[u]));
      }
    }
  }
  block_partials<NA>(acc, NEXT == 0 ? nvec : 1, pout, r, blk, nblk);
}

// ||w|| from the partial sums pin; block 0 records H(k+1, k) and the
// scalars; every block writes y = w / ||w|| (0 if ||w|| = 0) over its elements.
__global__ void __launch_bounds__(KB) scale_norm_kernel(double2* __restrict__ y, const double2* __restrict__ w,
                                                        const double2* __restrict__ pin, double2* __restrict__ H,
                                                        double* __restrict__ scal, long long N, int k, int restart,
                                                        const int* __restrict__ active) {
  const int r = blockIdx.y, blk = blockIdx.x, nblk = gridDim.x;
  if (active && !active[r]) return;
  __shared__ double2 hs[kMaxVec];
  __shared__ double2 red[kFinSlices][kMaxVec];
  final_sums(pin, r, nblk, 1, hs, red);
  const double nrm = sqrt(fmax(hs[0].x, 0.0));
  const double inv = nrm > 0 ? 1.0 / nrm : 0.0;
  if (blk == 0 && threadIdx.x == 0) {
    if (k >= 0) H[(long long)r * (restart + 1) * restart + (k + 1) + (restart + 1) * k] = make_double2(nrm, 0.0);
    scal[r * kScal + S_NORM] = nrm;
    scal[r * kScal + S_INV] = inv;
  }
  const long long e0 = N * blk / nblk, e1 = N * (blk + 1) / nblk;
  for (long long e = e0 + threadIdx.x; e < e1; e += KB) y[(long long)r * N + e] = cscale(w[(long long)r * N + e], inv);
}

// w -= sum_i h_i V_i
template <int NV>
__global__ void __launch_bounds__(KB) axpy_kernel(const double2* __restrict__ V, double2* __restrict__ w,
                                                  const double2* __restrict__ h, int nvec, long long N, int nrhs,
                                                  const int* __restrict__ active) {
  const int r = blockIdx.y;
  if (active && !active[r]) return;
  double2 hv[NV];
#pragma unroll
  for (int i = 0; i < NV; ++i) hv[i] = i < nvec ? h[(long long)r * kMaxVec + i] : make_double2(0, 0);
  double2* wr = w + (long long)r * N;
  for (long long e = (long long)blockIdx.x * KB + threadIdx.x; e < N; e += (long long)gridDim.x * KB) {
    double2 s = wr[e];
#pragma unroll
    for (int i = 0; i < NV; ++i)
      if (i < nvec) s = cfms(s, hv[i], V[((long long)i * nrhs + r) * N + e]);
    wr[e] = s;
  }
}

// y = x * scal[r][S_INV]
__global__ void scale_kernel(double2* __restrict__ y, const double2* __restrict__ x, const double* __restrict__ scal,
                             long long N, const int* __restrict__ active) {
  const int r = blockIdx.y;
  if (active && !active[r]) return;
  double s = scal[r * kScal + S_INV];
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < N; e += (long long)gridDim.x * blockDim.x)
    y[(long long)r * N + e] = cscale(x[(long long)r * N + e], s);
}

// Counts the right-hand sides still iterating over the block, then stores
// the count and the tag into the host control block (after this thread's
// own host writes: each thread fences them at system scope first).
__device__ void report(int mine, const CtlView& host, unsigned tag) {
  __shared__ int cnt;
  if (threadIdx.x == 0) cnt = 0;
  __threadfence_system();
  __syncthreads();
  if (mine) atomicAdd(&cnt, mine);
  __syncthreads();
  if (threadIdx.x == 0) {
    __hip_atomic_store(&host.hdr->nact, cnt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    __hip_atomic_store(&host.hdr->tag, tag, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
  }
}

// Givens update of column k for one right-hand side.
__device__ void givens_one(double2* __restrict__ H, double2* __restrict__ cs, double2* __restrict__ sn,
                           double2* __restrict__ gam, double* __restrict__ scal, int k, int restart, int r) {
  double2* Hc = H + (long long)r * (restart + 1) * restart + (restart + 1) * k;
  double2* c = cs + (long long)r * restart;
  double2* s = sn + (long long)r * restart;
  double2* g = gam + (long long)r * (restart + 1);
  for (int i = 0; i < k; ++i) {
    double2 t = cadd(cmul(c[i], Hc[i]), cmul(s[i], Hc[i + 1]));
    Hc[i + 1] = csub(cmul(c[i], Hc[i + 1]), cmulc(s[i], Hc[i]));  // -conj(s) H_i + conj(c) H_{i+1}, c real
    Hc[i] = t;
  }
  double2 a = Hc[k], b = Hc[k + 1];
  double aa = sqrt(a.x * a.x + a.y * a.y), bb = sqrt(b.x * b.x + b.y * b.y);
  double den = sqrt(aa * aa + bb * bb);
  double2 ck, sk;
  if (den == 0.0) { ck = make_double2(1, 0); sk = make_double2(0, 0); }
  else if (aa == 0.0) { ck = make_double2(0, 0); sk = make_double2(1, 0); }
  else {
    ck = make_double2(aa / den, 0);
    double2 ph = make_double2(a.x / aa, a.y / aa);
    sk = cscale(cmul(ph, cconj(b)), 1.0 / den);
  }
  c[k] = ck; s[k] = sk;
  Hc[k] = cadd(cmul(ck, a), cmul(sk, b));
  Hc[k + 1] = make_double2(0, 0);
  double2 gk = g[k];
  g[k + 1] = cscale(cmulc(sk, gk), -1.0);   // -conj(s) g_k
  g[k] = cmul(ck, gk);
  double2 gn = g[k + 1];
  scal[r * kScal + S_EST] = sqrt(gn.x * gn.x + gn.y * gn.y);
  scal[r * kScal + S_DEN] = den;
}

// One workgroup, right-hand sides strided over its threads.
__global__ void __launch_bounds__(256) givens_kernel(double2* __restrict__ H, double2* __restrict__ cs,
                                                     double2* __restrict__ sn, double2* __restrict__ gam, int k,
                                                     int restart, int nrhs, GmresState gs, GmresParams gp,
                                                     CtlView host, unsigned tag) {
  int mine = 0;
  for (int r = threadIdx.x; r < nrhs; r += blockDim.x) {
    double* sc = gs.scal + r * kScal;
    if (gs.active[r]) {
      givens_one(H, cs, sn, gam, gs.scal, k, restart, r);
      const int it = gs.iters[r] + 1;
      gs.iters[r] = it;
      gs.ksz[r] = k + 1;
      const double est = sc[S_EST];
      const bool stop = !(est > sc[S_TARGET]) || it >= gp.max_iters || sc[S_DEN] == 0.0;
      if (stop) gs.active[r] = 0;
      else mine += 1;
    }
    host.iters[r] = gs.iters[r];
    host.est[r] = sc[S_EST];
  }
  report(mine, host, tag);
}

// Minimum of v (NaN entries give -1), one workgroup, reported to the host.
__global__ void __launch_bounds__(256) min_report_kernel(const double* __restrict__ v, long long n, CtlView host,
                                                         unsigned tag) {
  __shared__ double red[256];
  double mn = 1e300;
  for (long long i = threadIdx.x; i < n; i += blockDim.x) {
    const double x = v[i];
    mn = x == x ? fmin(mn, x) : -1.0;
  }
  red[threadIdx.x] = mn;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) red[threadIdx.x] = fmin(red[threadIdx.x], red[threadIdx.x + h]);
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    __hip_atomic_store(&host.hdr->value, red[0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    __hip_atomic_store(&host.hdr->tag, tag, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
  }
}

// Start of the solve or end of a cycle (S_NORM from the norm kernel).
__global__ void __launch_bounds__(256) control_kernel(int cycle_end, int nrhs, GmresState gs, GmresParams gp,
                                                      CtlView host, unsigned tag) {
  int mine = 0;
  for (int r = threadIdx.x; r < nrhs; r += blockDim.x) {
    double* sc = gs.scal + r * kScal;
    const double nrm = sc[S_NORM];
    if (!cycle_end) {
      sc[S_GNORM] = nrm;
      sc[S_BETA] = nrm;
      sc[S_EST] = 0.0;
      gs.iters[r] = 0;
      gs.done[r] = nrm == 0.0 || nrm <= gp.tol * nrm;
    } else if (!gs.done[r]) {
      sc[S_BETA] = nrm;
      if (nrm <= gp.tol * sc[S_GNORM]) gs.done[r] = 1;
    }
    const int act = !gs.done[r] && gs.iters[r] < gp.max_iters;
    gs.active[r] = act;
    gs.ksz[r] = 0;
    sc[S_TARGET] = fmax(gp.tol * sc[S_GNORM], gp.eta * sc[S_BETA]);
    mine += act;
    host.iters[r] = gs.iters[r];
    host.est[r] = sc[S_EST];
    host.beta[r] = sc[S_BETA];
    host.gnorm[r] = sc[S_GNORM];
  }
  report(mine, host, tag);
}

// y = triu(H(0:k,0:k))^{-1} gam(0:k); ksz[r] = number of steps of rhs r.
__global__ void backsolve_kernel(const double2* __restrict__ H, const double2* __restrict__ gam, double2* __restrict__ y,
                                 const int* __restrict__ ksz, int restart, int nrhs) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= nrhs) return;
  const int k = ksz[r];
  const double2* Hr = H + (long long)r * (restart + 1) * restart;
  double2* yr = y + (long long)r * kMaxVec;
  for (int i = 0; i < kMaxVec; ++i) yr[i] = make_double2(0, 0);
  for (int i = k - 1; i >= 0; --i) {
    double2 s = gam[(long long)r * (restart + 1) + i];
    for (int j = i + 1; j < k; ++j) s = cfms(s, Hr[i + (restart + 1) * j], yr[j]);
    yr[i] = cdiv(s, Hr[i + (restart + 1) * i]);
  }
}

// x += sum_{j < ksz[r]} y_j Z_j
template <int NV>
__global__ void update_kernel(double2* __restrict__ x, const double2* __restrict__ Z, const double2* __restrict__ y,
                              const int* __restrict__ ksz, long long N, int nrhs) {
  const int r = blockIdx.y;
  const int k = ksz[r];
  if (k == 0) return;
  double2 yv[NV];
#pragma unroll
  for (int i = 0; i < NV; ++i) yv[i] = i < k ? y[(long long)r * kMaxVec + i] : make_double2(0, 0);
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < N; e += (long long)gridDim.x * blockDim.x) {
    double2 s = x[(long long)r * N + e];
#pragma unroll
    for (int i = 0; i < NV; ++i)
      if (i < k) s = cfma(s, yv[i], Z[((long long)i * nrhs + r) * N + e]);
    x[(long long)r * N + e] = s;
  }
}

// r = g - t
__global__ void sub_kernel(double2* __restrict__ r, const double2* __restrict__ g, const double2* __restrict__ t,
                           long long count) {
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < count; e += (long long)gridDim.x * blockDim.x)
    r[e] = csub(g[e], t[e]);
}

// start a cycle: gam = [beta, 0...], clear H, V_0 = r / beta
__global__ void cycle_init_kernel(double2* __restrict__ H, double2* __restrict__ gam, const double* __restrict__ scal,
                                  int restart, int nrhs) {
  const int r = blockIdx.x;
  for (int i = threadIdx.x; i < (restart + 1) * restart; i += blockDim.x)
    H[(long long)r * (restart + 1) * restart + i] = make_double2(0, 0);
  for (int i = threadIdx.x; i <= restart; i += blockDim.x)
    gam[(long long)r * (restart + 1) + i] = make_double2(i == 0 ? scal[r * kScal + S_NORM] : 0.0, 0.0);
}

__global__ void narrow_kernel(float2* __restrict__ y, const double2* __restrict__ x, long long count) {
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < count; e += (long long)gridDim.x * blockDim.x)
    y[e] = to_c64(x[e]);
}
__global__ void scale_rhs_kernel(double2* __restrict__ y, const double2* __restrict__ x, double s, long long count) {
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < count; e += (long long)gridDim.x * blockDim.x)
    y[e] = cscale(x[e], s);
}

inline unsigned grid1(long long count, int bs = 256, long long cap = 8192) {
  long long g = (count + bs - 1) / bs;
  return (unsigned)std::max<long long>(1, std::min(g, cap));
}

// launches kernel<NV> with the smallest vector-count bucket NV >= nv
#define LSP_NV_DISPATCH(nv, CALL)                 \
  do {                                            \
    if ((nv) <= 4) { constexpr int NV = 4; CALL; }        \
    else if ((nv) <= 8) { constexpr int NV = 8; CALL; }   \
    else if ((nv) <= 16) { constexpr int NV = 16; CALL; } \
    else { constexpr int NV = kMaxVec; CALL; }            \
  } while (0)

}  // namespace

int dot_blocks(long long N) {
  long long b = (N + 1023) / 1024;
  return (int)std::max<long long>(1, std::min<long long>(b, 256));
}

void k_dots(const double2* V, const double2* w, double2* partial, double2* h, double2* H, double* scal, int nvec,
            int k, int restart, int mode, long long N, int nrhs, const int* active, hipStream_t st) {
  int nblk = dot_blocks(N);
  LSP_NV_DISPATCH(nvec, LSP_LAUNCH("dots_partial", 0, dots_partial_kernel<NV>, dim3(nblk, nrhs), dim3(KB), 0, st, V, w,
                                    partial, nvec, N, nrhs, active));
  LSP_LAUNCH("dots_final", 0, dots_final_kernel, dim3(nrhs), dim3(kFinSlices * kMaxVec), 0, st, partial, h, H, scal, nvec, nblk, k, restart, mode,
                     active);
}

void k_norm(const double2* w, double2* partial, double2* h, double2* H, double* scal, int k, int restart, long long N,
            int nrhs, const int* active, hipStream_t st) {
  // ||w||^2 = sum conj(w) w: the dot kernel with V = w and nrhs-strided layout
  int nblk = dot_blocks(N);
  LSP_LAUNCH("dots_partial", 0, dots_partial_kernel<4>, dim3(nblk, nrhs), dim3(KB), 0, st, w, w, partial, 1, N, nrhs, active);
  LSP_LAUNCH("dots_final", 0, dots_final_kernel, dim3(nrhs), dim3(kFinSlices * kMaxVec), 0, st, partial, h, H, scal, 1, nblk, k, restart, 2,
                     active);
}

void k_arnoldi_orth(const double2* V, double2* w, double2* pA, double2* pB, double2* h, double2* H, double* scal,
                    double2* vnext, int k, int restart, long long N, int nrhs, const int* active, hipStream_t st) {
  const int nblk = dot_blocks(N), nvec = k + 1;
  LSP_NV_DISPATCH(nvec, {
    LSP_LAUNCH("dots_partial", 0, dots_partial_kernel<NV>, dim3(nblk, nrhs), dim3(KB), 0, st, V, w, pA, nvec, N, nrhs,
               active);
    LSP_LAUNCH("cgs", 0, (cgs_kernel<0, NV>), dim3(nblk, nrhs), dim3(KB), 0, st, V, w, pA, pB, h, H, nvec, N, nrhs, k,
               restart, 0, active);
    LSP_LAUNCH("cgs", 0, (cgs_kernel<1, NV>), dim3(nblk, nrhs), dim3(KB), 0, st, V, w, pB, pA, h, H, nvec, N, nrhs, k,
               restart, 1, active);
  });
  LSP_LAUNCH("scale_norm", 0, scale_norm_kernel, dim3(nblk, nrhs), dim3(KB), 0, st, vnext, w, pA, H, scal, N, k, restart,
             active);
}

void k_axpy(const double2* V, double2* w, const double2* h, int nvec, long long N, int nrhs, const int* active,
            hipStream_t st) {
  LSP_NV_DISPATCH(nvec, LSP_LAUNCH("axpy", 0, axpy_kernel<NV>, dim3(grid1(N, KB, 1024), nrhs), dim3(KB), 0, st, V, w, h,
                                    nvec, N, nrhs, active));
}

void k_scale(double2* y, const double2* x, const double* scal, long long N, int nrhs, const int* active,
             hipStream_t st) {
  LSP_LAUNCH("scale", 0, scale_kernel, dim3(grid1(N, 256, 1024), nrhs), dim3(256), 0, st, y, x, scal, N, active);
}

void k_givens(double2* H, double2* cs, double2* sn, double2* gam, int k, int restart, int nrhs, const GmresState& gs,
              const GmresParams& gp, const CtlView& host, unsigned tag, hipStream_t st) {
  LSP_LAUNCH("givens", 0, givens_kernel, dim3(1), dim3(256), 0, st, H, cs, sn, gam, k, restart, nrhs, gs, gp, host, tag);
}

void k_min_report(const double* v, long long n, const CtlView& host, unsigned tag, hipStream_t st) {
  LSP_LAUNCH("min_report", 0, min_report_kernel, dim3(1), dim3(256), 0, st, v, n, host, tag);
}

void k_gmres_control(bool cycle_end, int nrhs, const GmresState& gs, const GmresParams& gp, const CtlView& host,
                     unsigned tag, hipStream_t st) {
  LSP_LAUNCH("gmres_control", 0, control_kernel, dim3(1), dim3(256), 0, st, cycle_end ? 1 : 0, nrhs, gs, gp, host, tag);
}

void k_backsolve_update(const double2* H, const double2* gam, double2* y, const int* ksz, double2* x, const double2* Z,
                        int restart, int kmax, long long N, int nrhs, hipStream_t st) {
  LSP_LAUNCH("backsolve", 0, backsolve_kernel, dim3((nrhs + 63) / 64), dim3(64), 0, st, H, gam, y, ksz, restart, nrhs);
  LSP_NV_DISPATCH(kmax, LSP_LAUNCH("update", 0, update_kernel<NV>, dim3(grid1(N, 256, 1024), nrhs), dim3(256), 0, st, x,
                                   Z, y, ksz, N, nrhs));
}

void k_sub(double2* r, const double2* g, const double2* t, long long count, hipStream_t st) {
  LSP_LAUNCH("sub", 0, sub_kernel, dim3(grid1(count)), dim3(256), 0, st, r, g, t, count);
}

void k_cycle_init(double2* H, double2* gam, const double* scal, int restart, int nrhs, hipStream_t st) {
  LSP_LAUNCH("cycle_init", 0, cycle_init_kernel, dim3(nrhs), dim3(256), 0, st, H, gam, scal, restart, nrhs);
}

void launch_narrow(float2* y, const double2* x, long long count, hipStream_t st) {
  LSP_LAUNCH("narrow", 0, narrow_kernel, dim3(grid1(count)), dim3(256), 0, st, y, x, count);
}
void launch_scale_rhs(double2* y, const double2* x, double s, long long count, hipStream_t st) {
  LSP_LAUNCH("scale_rhs", 0, scale_rhs_kernel, dim3(grid1(count)), dim3(256), 0, st, y, x, s, count);
}

}  // namespace lsp

namespace lsp {
namespace {
__global__ void fill_zero_kernel(unsigned int* __restrict__ p, long long words) {
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < words; e += (long long)gridDim.x * blockDim.x)
    p[e] = 0u;
}
__global__ void fill_double_kernel(double* __restrict__ p, double v, long long count) {
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < count; e += (long long)gridDim.x * blockDim.x)
    p[e] = v;
}
__global__ void w2m_kernel(double* __restrict__ out, const double* __restrict__ m, double w2, long long N) {
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < N; e += (long long)gridDim.x * blockDim.x)
    out[e] = w2 * m[e];
}
inline unsigned grid_cap(long long count) {
  long long g = (count + 255) / 256;
  return (unsigned)std::max<long long>(1, std::min<long long>(g, 8192));
}
}  // namespace

void k_fill_zero(void* p, long long bytes, hipStream_t st) {
  long long words = bytes / 4;
  if (words <= 0) return;
  LSP_LAUNCH("fill_zero", 0, fill_zero_kernel, dim3(grid_cap(words)), dim3(256), 0, st, (unsigned int*)p, words);
}
void k_fill_double(double* p, double v, long long count, hipStream_t st) {
  if (count <= 0) return;
  LSP_LAUNCH("fill_double", 0, fill_double_kernel, dim3(grid_cap(count)), dim3(256), 0, st, p, v, count);
}
void k_w2m(double* out, const double* m, double w2, long long N, hipStream_t st) {
  LSP_LAUNCH("w2m", 0, w2m_kernel, dim3(grid_cap(N)), dim3(256), 0, st, out, m, w2, N);
}
}  // namespace lsp
