// Multifrontal LU of the sparse stencil matrix M = [A + C w^2 m; B] and its
// triangular solves (Section 2.2 names nested dissection with the
// multifrontal method; Section 3.2 gives their costs).
//
// Fronts of one elimination-tree level are processed together.  A front is
// a dense column-major matrix of order m = p + q over its index list [I | B]:
//   F = [F_II F_IB; F_BI F_BB],
// assembled from M's entries whose row or column is in I plus the children's
// Schur complements (extend-add, written as a gather so no atomics are used).
// The partial LU eliminates I in panels of width kb:
//   1. LU of the kb x kb diagonal block with partial pivoting inside it,
//   2. U12 = L11^{-1} P F12 (rows of the panel, all columns to the right) and
//      L21 = F21 U11^{-1} (all rows below, panel columns),
//   3. trailing update F22 -= L21 U12 on MFMA (complex as four real products).
// Pivoting is restricted to the panel's diagonal block (the paper leaves the
// pivoting strategy open); each front records the smallest ratio
// |u_jj| / max |column j of the block| it met, and the host rejects zero
// pivots.  After the last panel F_BB holds the Schur complement S handed to
// the parent.  Row swaps are not applied to columns left of a panel; the
// forward solve applies each panel's permutation when it reaches the panel.
#include "lsp_common.h"
#include "kernels.h"

namespace lsp {

namespace {

// ---------------------------------------------------------------- assembly
template <typename T>
__global__ void __launch_bounds__(256) assemble_front_kernel(cplx<T>* __restrict__ Fbuf, const FrontDev* __restrict__ fr,
                                                             const int* __restrict__ idx, const int* __restrict__ cpos,
                                                             const double2* __restrict__ Mval, int first, int n,
                                                             int d) {
  const FrontDev f = fr[first + blockIdx.y];
  const int m = f.p + f.q;
  const long long mm = (long long)m * m;
  const int ns = d == 2 ? 9 : 27;
  cplx<T>* F = Fbuf + f.f_off;
  const int* id = idx + f.idx_off;
  const int* cp = cpos + 2 * f.idx_off;
  FrontDev ch[2];
  const cplx<T>* Fc[2] = {nullptr, nullptr};
  int mc[2] = {0, 0};
  if (f.child0 >= 0) { ch[0] = fr[f.child0]; Fc[0] = Fbuf + ch[0].f_off; mc[0] = ch[0].p + ch[0].q; }
  if (f.child1 >= 0) { ch[1] = fr[f.child1]; Fc[1] = Fbuf + ch[1].f_off; mc[1] = ch[1].p + ch[1].q; }
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < mm; e += (long long)gridDim.x * blockDim.x) {
    int r = (int)(e % m), c = (int)(e / m);
    double2 v = make_double2(0, 0);
    if (r < f.p || c < f.p) {
      int gi = id[r], gj = id[c];
      int slot = 0, m3 = 1;
      bool near = true;
      int ai = gi, aj = gj;
      for (int a = 0; a < d; ++a) {
        int di = aj % n - ai % n;
        near = near && di >= -1 && di <= 1;
        slot += (di + 1) * m3;
        m3 *= 3;
        ai /= n; aj /= n;
      }
      if (near) v = Mval[(long long)gi * ns + slot];
    }
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      if (!Fc[k]) continue;
      int pr = cp[2 * r + k], pc = cp[2 * c + k];
      if (pr >= 0 && pc >= 0) v = cadd(v, widen(Fc[k][pr + (long long)pc * mc[k]]));
    }
    F[e] = from_c128<cplx<T>>(v);
  }
}

// ---------------------------------------------------------------- diagonal block LU
template <typename T>
__global__ void __launch_bounds__(256) diag_lu_kernel(cplx<T>* __restrict__ Fbuf, const FrontDev* __restrict__ fr,
                                                      int* __restrict__ piv, int* __restrict__ perm,
                                                      double* __restrict__ pivstat, int first, int k0, int nb) {
  __shared__ cplx<T> Bk[kNbMax][kNbMax + 1];
  __shared__ T redv[256];
  __shared__ int redi[256];
  __shared__ int permb[kNbMax];
  const FrontDev f = fr[first + blockIdx.x];
  if (f.p <= k0) return;
  const int kb = min(nb, f.p - k0);
  const int m = f.p + f.q;
  cplx<T>* F = Fbuf + f.f_off;
  const int tid = threadIdx.x;
  for (int e = tid; e < kb * kb; e += blockDim.x) {
    int r = e % kb, c = e / kb;
    Bk[r][c] = F[(k0 + r) + (long long)(k0 + c) * m];
  }
  if (tid < kb) permb[tid] = tid;
  __syncthreads();
  double worst = 1e300;
  for (int j = 0; j < kb; ++j) {
    T best = (T)-1;
    int bi = j;
    for (int r = j + tid; r < kb; r += blockDim.x) {
      T a = cabs1(Bk[r][j]);
      if (a > best) { best = a; bi = r; }
    }
    redv[tid] = best; redi[tid] = bi;
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
      if (tid < s) {
        if (redv[tid + s] > redv[tid] || (redv[tid + s] == redv[tid] && redi[tid + s] < redi[tid])) {
          redv[tid] = redv[tid + s]; redi[tid] = redi[tid + s];
        }
      }
      __syncthreads();
    }
    const int pr = redi[0];
    const T colmax = redv[0];
    __syncthreads();
    if (pr != j) {
      for (int c = tid; c < kb; c += blockDim.x) {
        cplx<T> t = Bk[j][c]; Bk[j][c] = Bk[pr][c]; Bk[pr][c] = t;
      }
      if (tid == 0) { int t = permb[j]; permb[j] = permb[pr]; permb[pr] = t; }
    }
    if (tid == 0) piv[f.piv_off + k0 + j] = k0 + pr;
    __syncthreads();
    cplx<T> dj = Bk[j][j];
    T dmag = cabs1(dj);
    double ratio = colmax > 0 ? (double)dmag / (double)colmax : 0.0;
    worst = fmin(worst, dmag > 0 ? ratio : 0.0);
    cplx<T> inv = dmag > 0 ? cdiv(mk<T>(1, 0), dj) : mk<T>(0, 0);
    for (int r = j + 1 + tid; r < kb; r += blockDim.x) Bk[r][j] = cmul(Bk[r][j], inv);
    __syncthreads();
    for (int e = tid; e < (kb - j - 1) * (kb - j - 1); e += blockDim.x) {
      int r = j + 1 + e % (kb - j - 1), c = j + 1 + e / (kb - j - 1);
      Bk[r][c] = cfms(Bk[r][c], Bk[r][j], Bk[j][c]);
    }
    __syncthreads();
  }
  for (int e = tid; e < kb * kb; e += blockDim.x) {
    int r = e % kb, c = e / kb;
    F[(k0 + r) + (long long)(k0 + c) * m] = Bk[r][c];
  }
  if (tid < kb) perm[f.piv_off + k0 + tid] = k0 + permb[tid];
  if (tid == 0) pivstat[first + blockIdx.x] = fmin(pivstat[first + blockIdx.x], worst);
}

// ---------------------------------------------------------------- panel triangular solves
// blockIdx.z == 0: U12 = L11^{-1} P F12, one thread per column c >= k1.
// blockIdx.z == 1: L21 = F21 U11^{-1}, one thread per row r >= k1.
template <typename T>
__global__ void __launch_bounds__(256) panel_trsm_kernel(cplx<T>* __restrict__ Fbuf, const FrontDev* __restrict__ fr,
                                                         const int* __restrict__ perm, int first, int k0, int nb) {
  __shared__ cplx<T> D[kNbMax][kNbMax + 1];
  __shared__ int pb[kNbMax];
  const FrontDev f = fr[first + blockIdx.y];
  if (f.p <= k0) return;
  const int kb = min(nb, f.p - k0);
  const int k1 = k0 + kb;
  const int m = f.p + f.q;
  if (k1 >= m) return;
  cplx<T>* F = Fbuf + f.f_off;
  for (int e = threadIdx.x; e < kb * kb; e += blockDim.x) {
    int r = e % kb, c = e / kb;
    D[r][c] = F[(k0 + r) + (long long)(k0 + c) * m];
  }
  if (threadIdx.x < kb) pb[threadIdx.x] = perm[f.piv_off + k0 + threadIdx.x];
  __syncthreads();
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= m - k1) return;
  cplx<T> x[kNbMax];
  if (blockIdx.z == 0) {
    const long long c = k1 + t;
    for (int j = 0; j < kb; ++j) x[j] = F[pb[j] + c * m];
    for (int j = 0; j < kb; ++j)
      for (int i = j + 1; i < kb; ++i) x[i] = cfms(x[i], D[i][j], x[j]);
    for (int j = 0; j < kb; ++j) F[(k0 + j) + c * m] = x[j];
  } else {
    const long long r = k1 + t;
    for (int j = 0; j < kb; ++j) x[j] = F[r + (long long)(k0 + j) * m];
    for (int j = 0; j < kb; ++j) {
      cplx<T> s = x[j];
      for (int i = 0; i < j; ++i) s = cfms(s, x[i], D[i][j]);
      x[j] = cdiv(s, D[j][j]);
    }
    for (int j = 0; j < kb; ++j) F[r + (long long)(k0 + j) * m] = x[j];
  }
}

// ---------------------------------------------------------------- trailing update on MFMA
// C (m-k1 x m-k1 block at (k1,k1)) -= A (panel rows below, m-k1 x kb) * B (kb x m-k1).
// 64x64 output tile per workgroup of 4 waves; each wave owns 32x32 as 2x2
// MFMA 16x16 blocks with separate real and imaginary accumulators.
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

template <typename T>
__global__ void __launch_bounds__(256) gemm_update_kernel(cplx<T>* __restrict__ Fbuf, const FrontDev* __restrict__ fr,
                                                          int first, int k0, int nb) {
  constexpr int TM = 64, TN = 64, KMAX = kNbMax;
  __shared__ T Ar[KMAX][TM], Ai[KMAX][TM], Br[KMAX][TN], Bi[KMAX][TN];
  const FrontDev f = fr[first + blockIdx.z];
  if (f.p <= k0) return;
  const int kb = min(nb, f.p - k0);
  const int k1 = k0 + kb;
  const int m = f.p + f.q;
  const int rem = m - k1;
  const int row0 = blockIdx.y * TM, col0 = blockIdx.x * TN;
  if (row0 >= rem || col0 >= rem) return;
  cplx<T>* F = Fbuf + f.f_off;
  const int tid = threadIdx.x;
  // stage A (rows k1+row0.., cols k0..k1) and B (rows k0..k1, cols k1+col0..)
  for (int e = tid; e < TM * kb; e += 256) {
    int r = e % TM, kk = e / TM;
    cplx<T> v = mk<T>(0, 0);
    if (row0 + r < rem) v = F[(k1 + row0 + r) + (long long)(k0 + kk) * m];
    Ar[kk][r] = v.x; Ai[kk][r] = v.y;
  }
  for (int e = tid; e < TN * kb; e += 256) {
    int kk = e % kb, c = e / kb;
    cplx<T> v = mk<T>(0, 0);
    if (col0 + c < rem) v = F[(k0 + kk) + (long long)(k1 + col0 + c) * m];
    Br[kk][c] = v.x; Bi[kk][c] = v.y;
  }
  const int kpad = (kb + 3) & ~3;
  for (int e = tid; e < TM * (kpad - kb); e += 256) {
    int r = e % TM, kk = kb + e / TM;
    Ar[kk][r] = 0; Ai[kk][r] = 0; Br[kk][r] = 0; Bi[kk][r] = 0;
  }
  __syncthreads();
  using acc_t = typename Mfma<T>::acc_t;
  const int wave = tid / 64, lane = tid % 64;
  const int wr = (wave / 2) * 32, wc = (wave % 2) * 32;
  acc_t accr[2][2], acci[2][2];
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j)
      for (int v = 0; v < 4; ++v) { accr[i][j][v] = 0; acci[i][j][v] = 0; }
  const int li = lane % 16, lk = lane / 16;
  for (int k4 = 0; k4 < kpad; k4 += 4) {
    T ar[2], ai[2], br[2], bi[2];
    for (int i = 0; i < 2; ++i) { ar[i] = Ar[k4 + lk][wr + 16 * i + li]; ai[i] = Ai[k4 + lk][wr + 16 * i + li]; }
    for (int j = 0; j < 2; ++j) { br[j] = Br[k4 + lk][wc + 16 * j + li]; bi[j] = Bi[k4 + lk][wc + 16 * j + li]; }
    for (int i = 0; i < 2; ++i)
      for (int j = 0; j < 2; ++j) {
        accr[i][j] = Mfma<T>::step(ar[i], br[j], accr[i][j]);
        accr[i][j] = Mfma<T>::step(-ai[i], bi[j], accr[i][j]);
        acci[i][j] = Mfma<T>::step(ar[i], bi[j], acci[i][j]);
        acci[i][j] = Mfma<T>::step(ai[i], br[j], acci[i][j]);
      }
  }
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j) {
      int col = col0 + wc + 16 * j + li;
      if (col >= rem) continue;
      for (int v = 0; v < 4; ++v) {
        int row = row0 + wr + 16 * i + Mfma<T>::row(lk, v);
        if (row >= rem) continue;
        long long e = (k1 + row) + (long long)(k1 + col) * m;
        cplx<T> c = F[e];
        c.x -= accr[i][j][v];
        c.y -= acci[i][j][v];
        F[e] = c;
      }
    }
}

// ---------------------------------------------------------------- solves
// Forward sweep of one front for one right-hand side (blockIdx.y):
//   v = [z(I); 0] + children's updates; per panel: v_b <- P_b v_b,
//   y_b = L11^{-1} v_b, v(k1:m) -= L21 y_b.  v lives in the per-front vector
//   buffer; afterwards v(0:p) = y_I and v(p:m) = update for the parent.
template <typename T>
__global__ void __launch_bounds__(256) fwd_kernel(const cplx<T>* __restrict__ Fbuf, const FrontDev* __restrict__ fr,
                                                  const int* __restrict__ idx, const int* __restrict__ cpos,
                                                  const int* __restrict__ perm, const cplx<T>* __restrict__ z,
                                                  cplx<T>* __restrict__ vbuf, int first, int nb, long long N,
                                                  long long vstride) {
  __shared__ cplx<T> yb[kNbMax];
  const FrontDev f = fr[first + blockIdx.x];
  const int rhs = blockIdx.y;
  const int m = f.p + f.q;
  const cplx<T>* F = Fbuf + f.f_off;
  const int* id = idx + f.idx_off;
  const int* cp = cpos + 2 * f.idx_off;
  cplx<T>* v = vbuf + rhs * vstride + f.idx_off;
  const cplx<T>* zr = z + rhs * N;
  const cplx<T>* vc[2] = {nullptr, nullptr};
  int pc[2] = {0, 0};
  if (f.child0 >= 0) { FrontDev c = fr[f.child0]; vc[0] = vbuf + rhs * vstride + c.idx_off; pc[0] = c.p; }
  if (f.child1 >= 0) { FrontDev c = fr[f.child1]; vc[1] = vbuf + rhs * vstride + c.idx_off; pc[1] = c.p; }
  const int tid = threadIdx.x;
  for (int r = tid; r < m; r += blockDim.x) {
    cplx<T> s = r < f.p ? zr[id[r]] : mk<T>(0, 0);
    for (int k = 0; k < 2; ++k) {
      if (!vc[k]) continue;
      int q = cp[2 * r + k];
      if (q >= 0) s = cadd(s, vc[k][q]);
    }
    v[r] = s;
  }
  __syncthreads();
  for (int k0 = 0; k0 < f.p; k0 += nb) {
    const int kb = min(nb, f.p - k0);
    const int k1 = k0 + kb;
    if (tid < 64) {
      cplx<T> val = mk<T>(0, 0);
      if (tid < kb) val = v[perm[f.piv_off + k0 + tid]];
      // unit lower solve with the diagonal block, one wave
      for (int j = 0; j < kb; ++j) {
        T yr = __shfl(val.x, j), yi = __shfl(val.y, j);
        if (tid > j && tid < kb) val = cfms(val, F[(k0 + tid) + (long long)(k0 + j) * m], mk<T>(yr, yi));
      }
      if (tid < kb) yb[tid] = val;
    }
    __syncthreads();
    if (tid < kb) v[k0 + tid] = yb[tid];
    for (int r = k1 + tid; r < m; r += blockDim.x) {
      cplx<T> s = v[r];
      for (int j = 0; j < kb; ++j) s = cfms(s, F[r + (long long)(k0 + j) * m], yb[j]);
      v[r] = s;
    }
    __syncthreads();
  }
}

// Backward sweep: x_B from the global solution, then per panel from the last:
//   x_b = U11^{-1} (y_b - U12 x(k1:m)).  Writes x at the front's grid points.
template <typename T>
__global__ void __launch_bounds__(256) bwd_kernel(const cplx<T>* __restrict__ Fbuf, const FrontDev* __restrict__ fr,
                                                  const int* __restrict__ idx, cplx<T>* __restrict__ x,
                                                  cplx<T>* __restrict__ vbuf, int first, int nb, long long N,
                                                  long long vstride) {
  __shared__ cplx<T> part[256];
  __shared__ cplx<T> xb[kNbMax];
  const FrontDev f = fr[first + blockIdx.x];
  const int rhs = blockIdx.y;
  const int m = f.p + f.q;
  const cplx<T>* F = Fbuf + f.f_off;
  const int* id = idx + f.idx_off;
  cplx<T>* v = vbuf + rhs * vstride + f.idx_off;
  cplx<T>* xr = x + rhs * N;
  const int tid = threadIdx.x;
  for (int r = f.p + tid; r < m; r += blockDim.x) v[r] = xr[id[r]];
  __syncthreads();
  const int nblk = (f.p + nb - 1) / nb;
  for (int b = nblk - 1; b >= 0; --b) {
    const int k0 = b * nb;
    const int kb = min(nb, f.p - k0);
    const int k1 = k0 + kb;
    // partial sums of U12 x over column groups
    const int j = tid % 64, grp = tid / 64;
    cplx<T> acc = mk<T>(0, 0);
    if (j < kb)
      for (int c = k1 + grp; c < m; c += 4) acc = cfma(acc, F[(k0 + j) + (long long)c * m], v[c]);
    part[tid] = acc;
    __syncthreads();
    if (tid < 64) {
      cplx<T> val = mk<T>(0, 0);
      if (tid < kb) {
        cplx<T> s = cadd(cadd(part[tid], part[tid + 64]), cadd(part[tid + 128], part[tid + 192]));
        val = csub(v[k0 + tid], s);
      }
      // upper solve, backwards, one wave
      for (int jj = kb - 1; jj >= 0; --jj) {
        cplx<T> dj = F[(k0 + jj) + (long long)(k0 + jj) * m];
        if (tid == jj) val = cdiv(val, dj);
        T xr_ = __shfl(val.x, jj), xi_ = __shfl(val.y, jj);
        if (tid < jj) val = cfms(val, F[(k0 + tid) + (long long)(k0 + jj) * m], mk<T>(xr_, xi_));
      }
      if (tid < kb) xb[tid] = val;
    }
    __syncthreads();
    if (tid < kb) {
      v[k0 + tid] = xb[tid];
      xr[id[k0 + tid]] = xb[tid];
    }
    __syncthreads();
  }
}

}  // namespace

template <typename T>
void mf_factor(const MfDev<T>& mf, const Plan& plan, int nb, hipStream_t st) {
  for (int l = 0; l < plan.nlevels; ++l) {
    const int first = plan.level_ptr[l];
    const int cnt = plan.level_ptr[l + 1] - first;
    const int maxm = plan.level_maxpq[l];
    const int maxp = plan.level_maxp[l];
    long long mm = (long long)maxm * maxm;
    int gx = (int)std::min<long long>((mm + 255) / 256, 64);
    hipLaunchKernelGGL(assemble_front_kernel<T>, dim3(gx, cnt), dim3(256), 0, st, mf.F, mf.fronts, mf.idx, mf.cpos,
                       mf.Mval, first, plan.n, plan.d);
    LSP_HIP(hipGetLastError());
    for (int k0 = 0; k0 < maxp; k0 += nb) {
      hipLaunchKernelGGL(diag_lu_kernel<T>, dim3(cnt), dim3(256), 0, st, mf.F, mf.fronts, mf.piv, mf.perm,
                         mf.pivstat, first, k0, nb);
      LSP_HIP(hipGetLastError());
      int rem = maxm - k0 - 1;
      if (rem <= 0) continue;
      hipLaunchKernelGGL(panel_trsm_kernel<T>, dim3((rem + 255) / 256, cnt, 2), dim3(256), 0, st, mf.F, mf.fronts,
                         mf.perm, first, k0, nb);
      LSP_HIP(hipGetLastError());
      int tiles = (rem + 63) / 64;
      hipLaunchKernelGGL(gemm_update_kernel<T>, dim3(tiles, tiles, cnt), dim3(256), 0, st, mf.F, mf.fronts, first, k0,
                         nb);
      LSP_HIP(hipGetLastError());
    }
  }
}

template <typename T>
void mf_solve(const MfDev<T>& mf, const Plan& plan, int nb, int nrhs, const cplx<T>* z, cplx<T>* x, cplx<T>* vbuf,
              hipStream_t st) {
  const long long vstride = plan.sum_pq;
  for (int l = 0; l < plan.nlevels; ++l) {
    const int first = plan.level_ptr[l];
    const int cnt = plan.level_ptr[l + 1] - first;
    hipLaunchKernelGGL(fwd_kernel<T>, dim3(cnt, nrhs), dim3(256), 0, st, mf.F, mf.fronts, mf.idx, mf.cpos, mf.perm, z,
                       vbuf, first, nb, (long long)plan.N, vstride);
    LSP_HIP(hipGetLastError());
  }
  for (int l = plan.nlevels - 1; l >= 0; --l) {
    const int first = plan.level_ptr[l];
    const int cnt = plan.level_ptr[l + 1] - first;
    hipLaunchKernelGGL(bwd_kernel<T>, dim3(cnt, nrhs), dim3(256), 0, st, mf.F, mf.fronts, mf.idx, x, vbuf, first, nb,
                       (long long)plan.N, vstride);
    LSP_HIP(hipGetLastError());
  }
}

template void mf_factor<double>(const MfDev<double>&, const Plan&, int, hipStream_t);
template void mf_factor<float>(const MfDev<float>&, const Plan&, int, hipStream_t);
template void mf_solve<double>(const MfDev<double>&, const Plan&, int, int, const double2*, double2*, double2*,
                               hipStream_t);
template void mf_solve<float>(const MfDev<float>&, const Plan&, int, int, const float2*, float2*, float2*, hipStream_t);

}  // namespace lsp
