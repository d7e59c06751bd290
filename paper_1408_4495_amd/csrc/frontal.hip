// Multifrontal LU of the sparse stencil matrix M = [A + C w^2 m; B] and its
// triangular solves (Section 2.2 names nested dissection with the
// multifrontal method; Section 3.2 gives their costs).
//
// Fronts of one elimination-tree level are processed together.  A front is
// a dense column-major matrix of order m = p + q over its index list [I | B]:
//   F = [F_II F_IB; F_BI F_BB],
// assembled from M's entries whose row or column is in I plus the children's
// Schur complements (extend-add, written as a gather so no atomics are used).
// The partial LU eliminates I in panels of width kb <= NB:
//   1. LU of the kb x kb diagonal block with partial pivoting inside it, and
//      the inverses L11^{-1}, U11^{-1} of its triangular factors (kept),
//   2. U12 = L11^{-1} P F12 and L21 = F21 U11^{-1} as small dense products,
//   3. trailing update F22 -= L21 U12 on MFMA (complex as four real products).
// Pivoting is restricted to the panel's diagonal block (the paper leaves the
// pivoting strategy open); each diagonal block records the smallest pivot
// modulus |re| + |im| divided by the largest (NaN when a pivot is NaN), and
// the host rejects the factorisation when the least ratio is tiny or NaN.  After the last panel F_BB holds the Schur complement S handed to
// the parent.  Row swaps are not applied to columns left of a panel; the
// forward solve applies each panel's permutation when it reaches the panel.
// The kept inverses turn every panel step of the triangular solves into a
// small matrix-vector product, so no step has a sequential dependency chain.
#include <climits>

#include "lsp_common.h"
#include "kernels.h"
#include "mfma.h"

namespace lsp {

namespace {

constexpr int NB = kNbMax;
constexpr size_t kVecLds = 80 * 1024;  // LDS for a front's working vectors in the sweeps

// ---------------------------------------------------------------- assembly
// F = the rows / columns of M of the front's pivots (entry (r, c) with r or
// c a pivot: M(i, j) when grid point j is a stencil neighbour of i, read
// from the [N][3^d] stencil values) plus the children's Schur complements
// (extend-add through their positions in this front).  One entry per thread,
// 32-bit entry indices (the plan bounds m^2), neighbour test and stencil
// slot from packed grid coordinates (no division by n).
template <typename T>
__global__ void __launch_bounds__(256) assemble_front_kernel(cplx<T>* __restrict__ Fbuf, const FrontDev* __restrict__ fr,
                                                             const int* __restrict__ idx,
                                                             const unsigned* __restrict__ gpos,
                                                             const int* __restrict__ cpos,
                                                             const double2* __restrict__ Mval, int first, int d) {
  const FrontDev f = fr[first + blockIdx.y];
  const int m = f.p + f.q;
  const int mm = m * m;
  const int ns = d == 2 ? 9 : 27;
  const int sh = d == 2 ? 16 : 10;
  const unsigned mask = (1u << sh) - 1;
  cplx<T>* F = Fbuf + f.f_off;
  const int* id = idx + f.idx_off;
  const unsigned* gp = gpos + f.idx_off;
  const int* cp = cpos + 2 * f.idx_off;
  const cplx<T>* Fc0 = Fbuf + (f.cfoff[0] >= 0 ? f.cfoff[0] : 0);
  const cplx<T>* Fc1 = Fbuf + (f.cfoff[1] >= 0 ? f.cfoff[1] : 0);
  const bool h0 = f.cfoff[0] >= 0, h1 = f.cfoff[1] >= 0;
  const int mc0 = f.cm[0], mc1 = f.cm[1];
  const float rm = 1.0f / (float)m;
  // four entries per thread and step, all their loads issued before any
  // entry is combined and stored
  constexpr int U = 4;
  const int stride = gridDim.x * blockDim.x;
  for (int e0 = blockIdx.x * blockDim.x + threadIdx.x; e0 < mm; e0 += U * stride) {
    int rr[U], cc[U];
    bool live[U];
    double2 mv[U], c0v[U], c1v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int e = e0 + u * stride;
      live[u] = e < mm;
      const int ee = live[u] ? e : 0;
      // (c, r) = divmod(e, m) from a float estimate of e / m instead of an
      // integer division: its relative error is below 2e-7 and e / m < m <
      // 46341 (the plan bounds m^2 by 2^31), so it is off by at most one
      int c = (int)((float)ee * rm), r = ee - c * m;
      if (r < 0) { --c; r += m; } else if (r >= m) { ++c; r -= m; }
      rr[u] = r;
      cc[u] = c;
      mv[u] = c0v[u] = c1v[u] = make_double2(0, 0);
      if (r < f.p || c < f.p) {
        const unsigned pi = gp[r], pj = gp[c];
        int slot = 0, m3 = 1;
        bool near = true;
        for (int a = 0; a < d; ++a) {
          const int di = (int)((pj >> (sh * a)) & mask) - (int)((pi >> (sh * a)) & mask);
          near = near && di >= -1 && di <= 1;
          slot += (di + 1) * m3;
          m3 *= 3;
        }
        if (near) mv[u] = Mval[(long long)id[r] * ns + slot];
      }
      if (h0) {
        const int pr = cp[2 * r], pc = cp[2 * c];
        if (pr >= 0 && pc >= 0) c0v[u] = widen(Fc0[pr + pc * mc0]);
      }
      if (h1) {
        const int pr = cp[2 * r + 1], pc = cp[2 * c + 1];
        if (pr >= 0 && pc >= 0) c1v[u] = widen(Fc1[pr + pc * mc1]);
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u)
      if (live[u]) F[e0 + u * stride] = from_c128<cplx<T>>(cadd(cadd(mv[u], c0v[u]), c1v[u]));
  }
}

// ---------------------------------------------------------------- diagonal block LU
// LU with partial pivoting of a panel's NB x NB diagonal block (padded with
// the identity when kb < NB, which leaves the kb x kb LU unchanged), plus the
// inverses L11^{-1} (unit lower) and U11^{-1} of its triangular factors,
// written to the front's inverse store: panel b keeps [Linv | Uinv], each
// NB x NB column-major, zero outside the kb x kb block.
//
// The elimination is one wave's work (the first wave of the workgroup).
// Elimination is row per lane pair: lane r holds the
// even columns of row r and lane 32 + r the odd ones, so each step updates
// at most 16 columns per lane.  Pivoting is by relabelling: a row keeps its
// lanes and records the step that chose it, so nothing moves.  Each step
// reduces a 32-bit key over the candidate rows with DPP (the magnitude
// |re| + |im| as a float, its five low mantissa bits replaced by 31 - row, so
// the largest wins and ties go to the lowest row: the chosen pivot is within
// a factor 1 - 2^-18 of the column maximum), reads the pivot row from a
// write-through LDS copy of the rows, and updates every row with a
// multiplier that is zero for rows that are already pivotal.  The two
// triangular inverses are then formed by the whole workgroup, blockwise
// with 8 x 8 blocks, for L and for R, the row- and column-reversed U (lower
// triangular): first the four diagonal blocks (forward substitution), then
// the blocks at distance 1, 2 and 3 below the diagonal, each from the
// blocks nearer the diagonal.  Only the inverses and the permutation are
// stored: no later step reads the diagonal block of F itself.

// Largest key over the 64 lanes (lane 63 ends with it): prefix maxima over
// each 16-lane row by right shifts, then row maxima broadcast forward.
__device__ __forceinline__ int lane_max64(int k) {
  k = max(k, __builtin_amdgcn_update_dpp(INT_MIN, k, 0x111, 0xf, 0xf, false));  // row_shr:1
  k = max(k, __builtin_amdgcn_update_dpp(INT_MIN, k, 0x112, 0xf, 0xf, false));  // row_shr:2
  k = max(k, __builtin_amdgcn_update_dpp(INT_MIN, k, 0x114, 0xf, 0xf, false));  // row_shr:4
  k = max(k, __builtin_amdgcn_update_dpp(INT_MIN, k, 0x118, 0xf, 0xf, false));  // row_shr:8
  k = max(k, __builtin_amdgcn_update_dpp(INT_MIN, k, 0x142, 0xa, 0xf, false));  // row_bcast:15
  k = max(k, __builtin_amdgcn_update_dpp(INT_MIN, k, 0x143, 0xc, 0xf, false));  // row_bcast:31
  return __builtin_amdgcn_readlane(k, 63);
}

template <typename T>
struct DiagLds {
  cplx<T> m[2][NB][NB + 1];  // the block's rows, then the factors L and R
  cplx<T> x[2][NB][NB + 1];  // L^{-1} and R^{-1}
  cplx<T> p[2][3][8][8];     // partial products of the blockwise inversion
  int src[NB];               // src[j]: the block row chosen as the j-th pivot
};

// The block factorisation runs in one wave.  LDS operations of a wave are
// performed in issue order, so a wave-scope fence (which only keeps the
// compiler from moving memory operations across it) makes one lane's LDS
// writes visible to the other lanes' later reads.
struct WaveSync {
  __device__ void operator()() const {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
  }
};

// Elimination.  Lane (h, r) holds columns c = 2i + h of row r in rowh[i];
// column J is held by half J % 2 at index J / 2.  Pivot key of a candidate
// entry: its magnitude |re| + |im| as a float with the five low mantissa
// bits replaced by 31 - row.
template <typename T>
__device__ __forceinline__ int pivot_key(const cplx<T>& v, int r) {
  return (__float_as_int((float)cabs1(v)) & 0x7fffffe0) | (NB - 1 - r);
}

__device__ __forceinline__ float lane_value(float v, int src) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), src));
}
__device__ __forceinline__ double lane_value(double v, int src) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffff), src);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), src);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// 1 / den for den > 0 (0 otherwise): hardware reciprocal refined by Newton
// steps (one in single, two in double precision)
__device__ __forceinline__ float recip(float den) {
  float r = __builtin_amdgcn_rcpf(den);
  r = fmaf(r, fmaf(-den, r, 1.0f), r);
  return den > 0.0f ? r : 0.0f;
}
__device__ __forceinline__ double recip(double den) {
  double r = __builtin_amdgcn_rcp(den);
  r = fma(r, fma(-den, r, 1.0), r);
  r = fma(r, fma(-den, r, 1.0), r);
  return den > 0.0 ? r : 0.0;
}

// Step J with the pivot already chosen: pivot row pl, pivot value d, and aJ
// the column-J entry of this lane's row.  The pivot row's entries are read
// from the LDS copy first; column J + 1 is updated before the others, so the
// next pivot (a DPP maximum of the keys, then the pivot value read from its
// lane) is found while the remaining columns are updated and written back.
template <typename T, int J>
__device__ __forceinline__ void diag_elim(cplx<T> (&rowh)[NB / 2], int& rlog, cplx<T>& myinv, T& dmin, T& dmax,
                                          DiagLds<T>& S, const int r, const int h, const int kb, const int pl,
                                          const cplx<T> d, const cplx<T> aJ) {
  if constexpr (J < NB) {
    const WaveSync sync;
    constexpr int hJ = J & 1, iJ = J >> 1;
    constexpr int i0 = (J + 1) / 2;  // first index holding a column > J (in some half)
    constexpr int NP = NB / 2 - i0 > 0 ? NB / 2 - i0 : 1;
    cplx<T> prow[NP];
#pragma unroll
    for (int i = i0; i < NB / 2; ++i) prow[i - i0] = S.m[0][pl][2 * i + h];
    const T rden = recip(d.x * d.x + d.y * d.y);
    const cplx<T> inv = mk<T>(d.x * rden, -d.y * rden);
    if (J < kb) {
      // a NaN pivot makes dmin NaN for the rest of the block (fmin alone
      // would skip it), so the block's ratio is NaN and the factorisation
      // reports a singular pivot
      const T mag = cabs1(d);
      dmin = (dmin != dmin || mag != mag) ? mag + dmin : fmin(dmin, mag);
      dmax = fmax(dmax, mag);
    }
    const bool upd = rlog < 0 && r != pl;
    if (r == pl) { rlog = J; myinv = inv; }
    const cplx<T> l0 = cmul(aJ, inv);
    const cplx<T> l = upd ? l0 : mk<T>(0, 0);
    if (h == hJ && upd) rowh[iJ] = l0;  // the multiplier
    if constexpr (J + 1 < NB) {
      constexpr int h1 = (J + 1) & 1, i1 = (J + 1) >> 1;
      static_assert(i1 == i0, "column J + 1 sits at the first updated index");
      // index i1: column J + 1 in half h1; in the other half column J (even
      // J: the multiplier, coefficient zero) or J + 2
      const cplx<T> c1 = ((J & 1) == 0 && h == 0) ? mk<T>(0, 0) : l;
      rowh[i1] = cfms(rowh[i1], c1, prow[0]);
      S.m[0][r][2 * i1 + h] = rowh[i1];
      const int key = (h == h1 && rlog < 0) ? pivot_key<T>(rowh[i1], r) : -1;
      const int pln = NB - 1 - (lane_max64(key) & (NB - 1));
      const int src = pln + NB * h1;
      cplx<T> dn;
      dn.x = lane_value(rowh[i1].x, src);
      dn.y = lane_value(rowh[i1].y, src);
      cplx<T> other;
      other.x = __shfl_xor(rowh[i1].x, 32, 64);
      other.y = __shfl_xor(rowh[i1].y, 32, 64);
      const cplx<T> an = h == h1 ? rowh[i1] : other;
#pragma unroll
      for (int i = i1 + 1; i < NB / 2; ++i) {
        rowh[i] = cfms(rowh[i], l, prow[i - i0]);
        S.m[0][r][2 * i + h] = rowh[i];
      }
      sync();  // the rows written above are what the next step reads
      diag_elim<T, J + 1>(rowh, rlog, myinv, dmin, dmax, S, r, h, kb, pln, dn, an);
    }
  }
}

// First pivot, then the 32 steps.
template <typename T>
__device__ __forceinline__ void diag_eliminate(cplx<T> (&rowh)[NB / 2], int& rlog, cplx<T>& myinv, T& dmin, T& dmax,
                                               DiagLds<T>& S, const int r, const int h, const int kb) {
  const int key = h == 0 ? pivot_key<T>(rowh[0], r) : -1;
  const int pl = NB - 1 - (lane_max64(key) & (NB - 1));
  cplx<T> d;
  d.x = lane_value(rowh[0].x, pl);
  d.y = lane_value(rowh[0].y, pl);
  cplx<T> other;
  other.x = __shfl_xor(rowh[0].x, 32, 64);
  other.y = __shfl_xor(rowh[0].y, 32, 64);
  const cplx<T> a0 = h == 0 ? rowh[0] : other;
  diag_elim<T, 0>(rowh, rlog, myinv, dmin, dmax, S, r, h, kb, pl, d, a0);
}

// Inverse of the lower-triangular T (T = L, or R = reversed U) held in M
// with the reciprocals of its diagonal on the diagonal, into X (entries on
// and below the diagonal; blocks above it are not written).  Blockwise with
// KB = 8: X_bb = T_bb^{-1} by forward substitution, then for d = 1, 2, 3
// X_ij = -X_ii sum_{k=j..i-1} T_ik X_kj with i = j + d.  Called by all 256
// threads of the workgroup for both matrices at once (mat = 0, 1).
constexpr int KB = 8;

// Blocks (j + D, j) of both inverses, by NT threads, one entry (matrix,
// block j, row r, column c) per thread at a time: first P = sum over
// k = j..j+D-1 of T_{j+D,k} X_kj into S.p, then X_{j+D,j} = -X_{j+D,j+D} P.
template <typename T, int D, int NT>
__device__ __forceinline__ void inv_level(DiagLds<T>& S, const int tid) {
  constexpr int nbk = 4 - D, E = 2 * nbk * KB * KB;
#pragma unroll 1
  for (int e = tid; e < E; e += NT) {
    const int mat = e / (nbk * KB * KB), q = e % (nbk * KB * KB);
    const int j = q / (KB * KB), r = (q / KB) % KB, c = q % KB, i = j + D;
    cplx<T> ta[KB * D], xb[KB * D];  // all operand reads in flight before the sums
#pragma unroll
    for (int t = 0; t < KB * D; ++t) {
      ta[t] = S.m[mat][KB * i + r][KB * j + t];
      xb[t] = S.x[mat][KB * j + t][KB * j + c];
    }
    cplx<T> a0 = mk<T>(0, 0), a1 = mk<T>(0, 0);
#pragma unroll
    for (int t = 0; t < KB * D; t += 2) {
      a0 = cfma(a0, ta[t], xb[t]);
      a1 = cfma(a1, ta[t + 1], xb[t + 1]);
    }
    S.p[mat][j][r][c] = cadd(a0, a1);
  }
  __syncthreads();
#pragma unroll 1
  for (int e = tid; e < E; e += NT) {
    const int mat = e / (nbk * KB * KB), q = e % (nbk * KB * KB);
    const int j = q / (KB * KB), r = (q / KB) % KB, c = q % KB, i = j + D;
    cplx<T> xa[KB], pb[KB];  // X_ii is exactly zero above its diagonal
#pragma unroll
    for (int t = 0; t < KB; ++t) {
      xa[t] = S.x[mat][KB * i + r][KB * i + t];
      pb[t] = S.p[mat][j][t][c];
    }
    cplx<T> a0 = mk<T>(0, 0), a1 = mk<T>(0, 0);
#pragma unroll
    for (int t = 0; t < KB; t += 2) {
      a0 = cfms(a0, xa[t], pb[t]);
      a1 = cfms(a1, xa[t + 1], pb[t + 1]);
    }
    S.x[mat][KB * i + r][KB * j + c] = cadd(a0, a1);
  }
  __syncthreads();
}

template <typename T, int NT>
__device__ __forceinline__ void tri_inverses(DiagLds<T>& S, const int tid) {
  static_assert(NB == 4 * KB, "four diagonal blocks");
  if (tid < 64) {  // 2 matrices x 4 blocks x 8 columns
    const int mat = tid / 32, base = KB * ((tid / KB) % 4), col = tid % KB;
    const cplx<T>(*M)[NB + 1] = S.m[mat];
    cplx<T> x[KB];
#pragma unroll
    for (int i = 0; i < KB; ++i) x[i] = mk<T>(i == col ? 1 : 0, 0);
#pragma unroll
    for (int k = 0; k < KB; ++k) {
      x[k] = cmul(x[k], M[base + k][base + k]);
#pragma unroll
      for (int i = k + 1; i < KB; ++i) x[i] = cfms(x[i], M[base + i][base + k], x[k]);
    }
#pragma unroll
    for (int i = 0; i < KB; ++i) S.x[mat][base + i][base + col] = x[i];
  }
  __syncthreads();
  inv_level<T, 1, NT>(S, tid);
  inv_level<T, 2, NT>(S, tid);
  inv_level<T, 3, NT>(S, tid);
}

// Pivoted LU of the diagonal block of panel k0 and the inverses of its
// factors, by a workgroup of NT = 64 or 256 threads: on entry S.m[0][r][c]
// holds the updated block, padded with the identity beyond kb (visible to
// the whole workgroup).  The elimination runs in the first wave (lane (h, r)
// holds columns 2i + h of row r), the inverses in all NT threads.  Writes the inverses
// to Dinv, the row order to perm and the block's smallest / largest pivot
// magnitude to its pivstat slot.
template <typename T, int NT>
__device__ __forceinline__ void diag_factor_block(DiagLds<T>& S, const FrontDev& f, const int k0, const int kb,
                                                  cplx<T>* __restrict__ Dinv, int* __restrict__ perm,
                                                  double* __restrict__ pivstat, const bool write = true) {
  const int tid = threadIdx.x;
  const int r = tid & (NB - 1), h = tid / NB;
  int rlog = -1;
  T dmin = (T)INFINITY, dmax = (T)0;
  if (tid < 64) {
    const WaveSync sync;
    cplx<T> rowh[NB / 2];
#pragma unroll
    for (int i = 0; i < NB / 2; ++i) rowh[i] = S.m[0][r][2 * i + h];
    cplx<T> myinv = mk<T>(0, 0);
    diag_eliminate<T>(rowh, rlog, myinv, dmin, dmax, S, r, h, kb);
    rlog &= NB - 1;  // every row is chosen exactly once, so this is already in range
    sync();
#pragma unroll
    for (int i = 0; i < NB / 2; ++i) {
      const int c = 2 * i + h;
      S.m[0][rlog][c] = rowh[i];
      S.m[1][NB - 1 - rlog][NB - 1 - c] = rowh[i];
    }
    if (h == 0) {  // after the row writes above, in issue order
      S.m[0][rlog][rlog] = mk<T>(1, 0);
      S.m[1][NB - 1 - rlog][NB - 1 - rlog] = myinv;
      S.src[rlog] = r;
    }
  }
  __syncthreads();
  tri_inverses<T, NT>(S, tid);
  if (!write) return;
  // global stores only now: a barrier waits for the stores issued before it
  if (tid < NB && rlog < kb) perm[f.piv_off + k0 + rlog] = k0 + r;
  if (tid == 0)  // one slot per diagonal block, in the order of the inverted blocks
    pivstat[f.dinv_off / (2 * NB * NB) + k0 / NB] = dmax > (T)0 ? (double)(dmin / dmax) : 0.0;
  // L^{-1}(a, b) = X_L(a, b) for a >= b; U^{-1}(a, b) = X_R(31-a, 31-b) for a <= b
  cplx<T>* Li = Dinv + f.dinv_off + (long long)(k0 / NB) * 2 * NB * NB;
#pragma unroll
  for (int u = 0; u < NB * NB / NT; ++u) {
    const int e = tid + NT * u;
    const int a = e % NB, b = e / NB;
    const bool in = a < kb && b < kb;
    Li[e] = in && a >= b ? S.x[0][a][b] : mk<T>(0, 0);
    Li[NB * NB + e] = in && a <= b ? S.x[1][NB - 1 - a][NB - 1 - b] : mk<T>(0, 0);
  }
}

// Diagonal block of panel k0 (except those factored inside the previous
// panel's trailing update, gemm_update_kernel with FUSE), one workgroup of
// NT threads per front: 64 on levels with more than two fronts per CU (the
// elimination is one wave's work, so one-wave workgroups spread the fronts
// over all SIMDs), else 256 (the inverses then use four waves).
template <typename T, int NT>
__global__ void __launch_bounds__(NT) diag_lu_kernel(cplx<T>* __restrict__ Fbuf, cplx<T>* __restrict__ Dinv,
                                                      const FrontDev* __restrict__ fr, int* __restrict__ perm,
                                                      double* __restrict__ pivstat, int first, int k0) {
  static_assert(NB == 32, "lane layout assumes 32-wide panels");
  __shared__ DiagLds<T> S;
  const FrontDev f = fr[first + blockIdx.x];
  if (f.p <= k0) return;
  const int kb = min(NB, f.p - k0);
  const int m = f.p + f.q;
  const cplx<T>* F = Fbuf + f.f_off;
  const int tid = threadIdx.x;
  cplx<T> v[NB * NB / NT];
#pragma unroll
  for (int u = 0; u < NB * NB / NT; ++u) {
    const int e = tid + NT * u, r = e % NB, c = e / NB;
    v[u] = F[(k0 + min(r, kb - 1)) + (long long)(k0 + min(c, kb - 1)) * m];
  }
#pragma unroll
  for (int u = 0; u < NB * NB / NT; ++u) {
    const int e = tid + NT * u, r = e % NB, c = e / NB;
    S.m[0][r][c] = r < kb && c < kb ? v[u] : mk<T>(r == c ? 1 : 0, 0);
  }
  __syncthreads();
  diag_factor_block<T, NT>(S, f, k0, kb, Dinv, perm, pivstat);
}

// Runs use(i, load(i)) for i = 0 .. N-1 (N and i compile-time after
// unrolling), loading W items ahead of their use: bounds the registers held
// by LDS reads in flight while still hiding their latency.
template <int N, int W, typename Load, typename Use>
__device__ __forceinline__ void chunked(Load&& load, Use&& use) {
  using V = decltype(load(0));
  constexpr int nq = (N + W - 1) / W;
  V buf[2][W];
#pragma unroll
  for (int j = 0; j < W; ++j)
    if (j < N) buf[0][j] = load(j);
#pragma unroll
  for (int q = 0; q < nq; ++q) {
    if (q + 1 < nq) {
#pragma unroll
      for (int j = 0; j < W; ++j) {
        const int i = (q + 1) * W + j;
        if (i < N) buf[(q + 1) & 1][j] = load(i);
      }
    }
    asm volatile("" ::: "memory");  // keeps IR passes from merging or hoisting loads across chunks
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int j = 0; j < W; ++j) {
      const int i = q * W + j;
      if (i < N) use(i, buf[q & 1][j]);
    }
    asm volatile("" ::: "memory");
    __builtin_amdgcn_sched_barrier(0);
  }
}


// ---------------------------------------------------------------- panel products
// blockIdx.z == 0: U12(:, tile) = L11^{-1} P F12(:, tile), 64 columns per block.
// blockIdx.z == 1: L21(tile, :) = F21(tile, :) U11^{-1}, 64 rows per block.
// Every load is issued before the first LDS store (clamped in-range indices,
// invalid entries zeroed after the load); the products run on the 16x16x4
// MFMAs (complex as four real products; the inverses are exactly zero
// outside their triangle and outside the kb x kb block), each wave one
// 16-wide slice of the tile, and the results go back through LDS so the
// stores are coalesced.
template <typename T>
__global__ void __launch_bounds__(256) panel_trsm_kernel(cplx<T>* __restrict__ Fbuf, const cplx<T>* __restrict__ Dinv,
                                                         const FrontDev* __restrict__ fr, const int* __restrict__ perm,
                                                         int first, int k0) {
  __shared__ T Dr[NB][NB + 1], Dq[NB][NB + 1];  // inverse block [row][col], real / imaginary parts
  __shared__ T Tr[64][NB + 1], Tq[64][NB + 1];  // upper: [c][j] = (P F12)(j, c); lower: [r][i] = F21(r, i)
  const FrontDev f = fr[first + blockIdx.y];
  if (f.p <= k0) return;
  const int kb = min(NB, f.p - k0);
  const int k1 = k0 + kb;
  const int m = f.p + f.q;
  const int t0 = blockIdx.x * 64;
  if (t0 >= m - k1) return;
  const int cnt = min(64, m - k1 - t0);
  cplx<T>* F = Fbuf + f.f_off;
  const cplx<T>* Li = Dinv + f.dinv_off + (long long)(k0 / NB) * 2 * NB * NB;
  const bool upper = blockIdx.z == 0;
  const cplx<T>* Dm = upper ? Li : Li + NB * NB;
  const int tid = threadIdx.x;
  cplx<T> dv[4], tv[8];
#pragma unroll
  for (int u = 0; u < 4; ++u) dv[u] = Dm[tid + 256 * u];
  if (upper) {
    const int j = tid % NB;
    const int pj = perm[f.piv_off + k0 + min(j, kb - 1)];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int c = tid / NB + 8 * u;
      const cplx<T> v = F[pj + (long long)(k1 + t0 + min(c, cnt - 1)) * m];
      tv[u] = j < kb && c < cnt ? v : mk<T>(0, 0);
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      Tr[tid / NB + 8 * u][j] = tv[u].x;
      Tq[tid / NB + 8 * u][j] = tv[u].y;
    }
  } else {
    const int r = tid % 64;
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int i = tid / 64 + 4 * u;
      const cplx<T> v = F[(k1 + t0 + min(r, cnt - 1)) + (long long)(k0 + min(i, kb - 1)) * m];
      tv[u] = r < cnt && i < kb ? v : mk<T>(0, 0);
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      Tr[r][tid / 64 + 4 * u] = tv[u].x;
      Tq[r][tid / 64 + 4 * u] = tv[u].y;
    }
  }
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int e = tid + 256 * u;  // the inverse is stored column-major
    Dr[e % NB][e / NB] = dv[u].x;
    Dq[e % NB][e / NB] = dv[u].y;
  }
  __syncthreads();
  using acc_t = typename Mfma<T>::acc_t;
  const int wave = tid / 64, lane = tid % 64, li = lane % 16, lk = lane / 16;
  acc_t cr[2], ci[2];
#pragma unroll
  for (int blk = 0; blk < 2; ++blk)
#pragma unroll
    for (int v = 0; v < 4; ++v) { cr[blk][v] = 0; ci[blk][v] = 0; }
  if (upper) {
    // U12(i, c) = sum_j Linv(i, j) Tt[c][j]: this wave's columns c = 16 wave + li, rows in two blocks
#pragma unroll
    for (int k4 = 0; k4 < NB; k4 += 4) {
      const int kk = k4 + lk;
      const T br = Tr[16 * wave + li][kk], bi = Tq[16 * wave + li][kk];
#pragma unroll
      for (int blk = 0; blk < 2; ++blk) {
        const T ar = Dr[16 * blk + li][kk], ai = Dq[16 * blk + li][kk];
        cr[blk] = Mfma<T>::step(ar, br, cr[blk]);
        cr[blk] = Mfma<T>::step(-ai, bi, cr[blk]);
        ci[blk] = Mfma<T>::step(ar, bi, ci[blk]);
        ci[blk] = Mfma<T>::step(ai, br, ci[blk]);
      }
    }
  } else {
    // L21(r, j) = sum_i Tt[r][i] Uinv(i, j): this wave's rows r = 16 wave + li, columns in two blocks
#pragma unroll
    for (int k4 = 0; k4 < NB; k4 += 4) {
      const int kk = k4 + lk;
      const T ar = Tr[16 * wave + li][kk], ai = Tq[16 * wave + li][kk];
#pragma unroll
      for (int blk = 0; blk < 2; ++blk) {
        const T br = Dr[kk][16 * blk + li], bi = Dq[kk][16 * blk + li];
        cr[blk] = Mfma<T>::step(ar, br, cr[blk]);
        cr[blk] = Mfma<T>::step(-ai, bi, cr[blk]);
        ci[blk] = Mfma<T>::step(ar, bi, ci[blk]);
        ci[blk] = Mfma<T>::step(ai, br, ci[blk]);
      }
    }
  }
  __syncthreads();  // the tile has been read: its LDS now stages the results
#pragma unroll
  for (int blk = 0; blk < 2; ++blk)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int rr = Mfma<T>::row(lk, v);
      if (upper) {  // result (row 16 blk + rr, column 16 wave + li), staged as [column][row]
        Tr[16 * wave + li][16 * blk + rr] = cr[blk][v];
        Tq[16 * wave + li][16 * blk + rr] = ci[blk][v];
      } else {  // result (row 16 wave + rr, column 16 blk + li), staged as [row][column]
        Tr[16 * wave + rr][16 * blk + li] = cr[blk][v];
        Tq[16 * wave + rr][16 * blk + li] = ci[blk][v];
      }
    }
  __syncthreads();
  if (upper) {
    const int i = tid % NB;
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int c = tid / NB + 8 * u;
      if (i < kb && c < cnt) F[(k0 + i) + (long long)(k1 + t0 + c) * m] = mk<T>(Tr[c][i], Tq[c][i]);
    }
  } else {
    const int r = tid % 64;
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int j = tid / 64 + 4 * u;
      if (r < cnt && j < kb) F[(k1 + t0 + r) + (long long)(k0 + j) * m] = mk<T>(Tr[r][j], Tq[r][j]);
    }
  }
}

// ---------------------------------------------------------------- trailing update on MFMA
// C (m-k1 x m-k1 block at (k1,k1)) -= A (panel rows below, m-k1 x kb) * B (kb x m-k1).
// 64x64 output tile per workgroup of 4 waves; each wave owns 32x32 as 2x2
// MFMA 16x16 blocks with separate real and imaginary accumulators.
template <typename T, int TM>
struct GemmLds {
  T Ar[NB][TM], Ai[NB][TM], Br[NB][TM + 1], Bi[NB][TM + 1];
};

// One TM x TM tile of C -= A B over the block [base, m)^2 of a front's
// trailing matrix: A = the L21 rows (columns k0 .. k0+kb), B = the U12
// columns (rows k0 .. k0+kb) of one panel, or of two adjacent panels
// (kb up to 64, taken as two 32-wide chunks through LDS, the products
// accumulated in registers, so C is read and written once); (row0, col0)
// relative to base; entries with row < skip and column < skip, and rows >=
// rlim or columns >= clim, are left alone.  4 waves in a 2x2 arrangement,
// each wave (TM/2)^2 as BW x BW MFMA 16x16 blocks.
template <typename T, int TM>
__device__ __forceinline__ void update_tile(GemmLds<T, TM>& G, cplx<T>* __restrict__ F, const int k0, const int kb,
                                            const int base, const int m, const int row0, const int col0,
                                            const int skip, const int rlim = INT_MAX, const int clim = INT_MAX) {
  constexpr int BW = TM / 32;
  auto& Ar = G.Ar;
  auto& Ai = G.Ai;
  auto& Br = G.Br;
  auto& Bi = G.Bi;
  const int rem = m - base;
  const int tid = threadIdx.x;
  using acc_t = typename Mfma<T>::acc_t;
  const int wave = tid / 64, lane = tid % 64;
  const int wr = (wave / 2) * (TM / 2), wc = (wave % 2) * (TM / 2);
  acc_t accr[BW][BW], acci[BW][BW];
  for (int i = 0; i < BW; ++i)
    for (int j = 0; j < BW; ++j)
      for (int v = 0; v < 4; ++v) { accr[i][j][v] = 0; acci[i][j][v] = 0; }
  const int li = lane % 16, lk = lane / 16;
  constexpr int LA = TM * NB / 256;
  // a chunk's operand tiles into registers (clamped in-range indices, zero
  // outside the block), then into LDS
  auto load_ops = [&](const int kc, cplx<T>(&va)[LA], cplx<T>(&vb)[LA]) {
    const int kbc = min(NB, kb - kc), kcol = k0 + kc;
#pragma unroll
    for (int u = 0; u < LA; ++u) {
      const int e = tid + 256 * u, r = e % TM, kk = e / TM;
      const cplx<T> v = F[(base + min(row0 + r, rem - 1)) + (long long)(kcol + min(kk, kbc - 1)) * m];
      va[u] = row0 + r < rem && kk < kbc ? v : mk<T>(0, 0);
    }
#pragma unroll
    for (int u = 0; u < LA; ++u) {
      const int e = tid + 256 * u, kk = e % NB, c = e / NB;
      const cplx<T> v = F[(kcol + min(kk, kbc - 1)) + (long long)(base + min(col0 + c, rem - 1)) * m];
      vb[u] = col0 + c < rem && kk < kbc ? v : mk<T>(0, 0);
    }
  };
  auto store_ops = [&](const cplx<T>(&va)[LA], const cplx<T>(&vb)[LA]) {
#pragma unroll
    for (int u = 0; u < LA; ++u) {
      const int e = tid + 256 * u;
      Ar[e / TM][e % TM] = va[u].x;
      Ai[e / TM][e % TM] = va[u].y;
      Br[e % NB][e / NB] = vb[u].x;
      Bi[e % NB][e / NB] = vb[u].y;
    }
  };
  // C's entries of this lane (BW x BW blocks of 4), for tiles of up to 64
  // rows loaded right after the first chunk's operands are in LDS, so that
  // their latency and that of the next chunk's operands pass during the
  // products; wider tiles load them at the end (registers)
  constexpr bool kEarlyC = BW <= 2;
  auto c_index = [&](const int i, const int j, const int v) {
    const int col = min(col0 + wc + 16 * j + Mfma<T>::row(lk, v), rem - 1);
    const int row = min(row0 + wr + 16 * i + li, rem - 1);
    return (long long)(base + row) + (long long)(base + col) * m;
  };
  cplx<T> ce[kEarlyC ? BW : 1][kEarlyC ? BW : 1][4];
  cplx<T> va[LA], vb[LA];
  load_ops(0, va, vb);
  store_ops(va, vb);
  if constexpr (kEarlyC) {
#pragma unroll
    for (int i = 0; i < BW; ++i)
#pragma unroll
      for (int j = 0; j < BW; ++j)
#pragma unroll
        for (int v = 0; v < 4; ++v) ce[i][j][v] = F[c_index(i, j, v)];
  }
  for (int kc = 0; kc < kb; kc += NB) {
    const int kbc = min(NB, kb - kc);
    const int kpad = (kbc + 3) & ~3;
    const bool more = kc + NB < kb;
    if (more) load_ops(kc + NB, va, vb);  // in flight during this chunk's products
    __syncthreads();  // this chunk's operand tiles are in LDS
    // Each 16 x 16 block is computed transposed (the MFMA's first operand is
    // B's column block, its second A's row block): the result lane l then
    // holds C rows 16 i + l % 16, so consecutive lanes address consecutive
    // rows of the column-major front and every load / store of C below covers
    // whole cache lines.
    for (int k4 = 0; k4 < kpad; k4 += 4) {
      T ar[BW], ai[BW], br[BW], bi[BW];
      for (int i = 0; i < BW; ++i) { ar[i] = Ar[k4 + lk][wr + 16 * i + li]; ai[i] = Ai[k4 + lk][wr + 16 * i + li]; }
      for (int j = 0; j < BW; ++j) { br[j] = Br[k4 + lk][wc + 16 * j + li]; bi[j] = Bi[k4 + lk][wc + 16 * j + li]; }
      for (int i = 0; i < BW; ++i)
        for (int j = 0; j < BW; ++j) {
          accr[i][j] = Mfma<T>::step(br[j], ar[i], accr[i][j]);
          accr[i][j] = Mfma<T>::step(bi[j], -ai[i], accr[i][j]);
          acci[i][j] = Mfma<T>::step(bi[j], ar[i], acci[i][j]);
          acci[i][j] = Mfma<T>::step(br[j], ai[i], acci[i][j]);
        }
    }
    if (more) {
      __syncthreads();  // this chunk's reads of the operand tiles are done
      store_ops(va, vb);
    }
  }
  // C -= A B: per 16-row block i (wide tiles: all BW x 4 loads of C first),
  // then the stores
  const int rmax = min(rem, rlim), cmax = min(rem, clim);
#pragma unroll
  for (int i = 0; i < BW; ++i) {
    cplx<T> cv[BW][4];
#pragma unroll
    for (int j = 0; j < BW; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        if constexpr (kEarlyC) cv[j][v] = ce[i][j][v];
        else cv[j][v] = F[c_index(i, j, v)];
      }
#pragma unroll
    for (int j = 0; j < BW; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int col = col0 + wc + 16 * j + Mfma<T>::row(lk, v);
        const int row = row0 + wr + 16 * i + li;
        if (col < cmax && row < rmax && !(row < skip && col < skip)) {
          cplx<T> c = cv[j][v];
          c.x -= accr[i][j][v];
          c.y -= acci[i][j][v];
          F[(base + row) + (long long)(base + col) * m] = c;
        }
      }
  }
}

// Lookahead (FUSE): the next panel's diagonal block depends only on this
// update of its own 32 x 32 entries, so workgroup (0, 0) of each front
// applies that part of the update itself (block = F - L21 U12 over the
// block's rows and columns, a sequential 32-term sum per entry) and then
// factors the block in its first wave, while the other workgroups update
// the rest of the trailing matrix on MFMA, leaving that block alone (no
// later step reads the diagonal blocks of F: the factorisation keeps only
// their inverses and the row order).
template <typename T>
__device__ __forceinline__ void update_and_factor_next(unsigned char* raw, const FrontDev& f, const cplx<T>* F,
                                                       const int k0, const int k1, const int m,
                                                       cplx<T>* __restrict__ Dinv, int* __restrict__ perm,
                                                       double* __restrict__ pivstat) {
  DiagLds<T>& S = *reinterpret_cast<DiagLds<T>*>(raw);
  const int kb = k1 - k0;
  const int kbn = min(NB, f.p - k1);  // > 0: the front has a next panel
  const int tid = threadIdx.x;
  cplx<T> la[4], ub[4], ov[4];
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int e = tid + 256 * u, r = e % NB, c = e / NB;
    const cplx<T> a = F[(k1 + min(r, kbn - 1)) + (long long)(k0 + min(c, kb - 1)) * m];   // L21(r, c)
    const cplx<T> b = F[(k0 + min(r, kb - 1)) + (long long)(k1 + min(c, kbn - 1)) * m];   // U12(r, c)
    const cplx<T> o = F[(k1 + min(r, kbn - 1)) + (long long)(k1 + min(c, kbn - 1)) * m];  // block (r, c)
    la[u] = r < kbn && c < kb ? a : mk<T>(0, 0);
    ub[u] = r < kb && c < kbn ? b : mk<T>(0, 0);
    ov[u] = r < kbn && c < kbn ? o : mk<T>(r == c ? 1 : 0, 0);
  }
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int e = tid + 256 * u, r = e % NB, c = e / NB;
    S.m[0][r][c] = la[u];
    S.m[1][r][c] = ub[u];
  }
  __syncthreads();
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int e = tid + 256 * u, r = e % NB, c = e / NB;
#pragma unroll 8
    for (int kk = 0; kk < NB; ++kk) ov[u] = cfms(ov[u], S.m[0][r][kk], S.m[1][kk][c]);
  }
  __syncthreads();
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int e = tid + 256 * u;
    S.m[0][e % NB][e / NB] = ov[u];
  }
  __syncthreads();
  diag_factor_block<T, 256>(S, f, k1, kbn, Dinv, perm, pivstat);
}

template <typename T, int TM, bool FUSE>
__global__ void __launch_bounds__(256) gemm_update_kernel(cplx<T>* __restrict__ Fbuf, const FrontDev* __restrict__ fr,
                                                          int first, int k0, cplx<T>* __restrict__ Dinv,
                                                          int* __restrict__ perm, double* __restrict__ pivstat) {
  // TM x TM output tiles (update_tile).  With FUSE, block row 0 is the
  // lookahead factorisation of the next diagonal block and the tiles start
  // at row 1.
  constexpr size_t kRaw = FUSE && sizeof(DiagLds<T>) > sizeof(GemmLds<T, TM>) ? sizeof(DiagLds<T>)
                                                                             : sizeof(GemmLds<T, TM>);
  __shared__ __align__(16) unsigned char raw[kRaw];
  GemmLds<T, TM>& G = *reinterpret_cast<GemmLds<T, TM>*>(raw);
  const FrontDev f = fr[first + blockIdx.z];
  if (f.p <= k0) return;
  const int kb = min(NB, f.p - k0);
  const int k1 = k0 + kb;
  const int m = f.p + f.q;
  const int rem = m - k1;
  cplx<T>* F = Fbuf + f.f_off;
  const int brow = FUSE ? (int)blockIdx.y - 1 : (int)blockIdx.y;
  if constexpr (FUSE) {
    if (brow < 0) {
      if (blockIdx.x == 0 && f.p > k1)
        update_and_factor_next<T>(raw, f, F, k0, k1, m, Dinv, perm, pivstat);
      return;
    }
  }
  // entries of the next diagonal block, left to the lookahead workgroup
  const int skip = FUSE ? max(0, min(NB, f.p - k1)) : 0;
  const int row0 = brow * TM, col0 = blockIdx.x * TM;
  if (row0 >= rem || col0 >= rem) return;
  update_tile<T, TM>(G, F, k0, kb, k1, m, row0, col0, skip);
}

// Two-panel (rank-64) trailing updates for the large fronts of the levels
// that run separate launches per panel: panel a = [k0, k0 + 32) is factored,
// its update applied only to panel b's column and row strips (the "cross":
// rows [k1, m) of columns [k1, k2), rows [k1, k2) of columns [k2, m)), panel b
// is factored, and the rest [k2, m)^2 takes both panels' update at once, so
// each tile of the trailing matrix is read and written once per two panels.
// Fronts with no panel b take panel a's update over [k1, m)^2 in the second
// launch.  The cross uses 32-wide tiles: grid x the tile along the strip,
// y = 0 the column strip (its diagonal block left out), y = 1 the row
// strip, y = 2 (x = 0) the lookahead: panel a's update of panel b's
// diagonal block and that block's factorisation, so panel b needs no
// diagonal-block launch of its own.
template <typename T>
__global__ void __launch_bounds__(256) cross_update_kernel(cplx<T>* __restrict__ Fbuf,
                                                           const FrontDev* __restrict__ fr, int first, int k0,
                                                           cplx<T>* __restrict__ Dinv, int* __restrict__ perm,
                                                           double* __restrict__ pivstat) {
  constexpr size_t kRaw =
      sizeof(DiagLds<T>) > sizeof(GemmLds<T, 32>) ? sizeof(DiagLds<T>) : sizeof(GemmLds<T, 32>);
  __shared__ __align__(16) unsigned char raw[kRaw];
  GemmLds<T, 32>& G = *reinterpret_cast<GemmLds<T, 32>*>(raw);
  const FrontDev f = fr[first + blockIdx.z];
  if (f.p <= k0 + NB) return;  // no panel b: the pair update takes panel a's update
  const int k1 = k0 + NB, kbb = min(NB, f.p - k1);
  const int m = f.p + f.q;
  cplx<T>* F = Fbuf + f.f_off;
  if (blockIdx.y == 2) {
    if (blockIdx.x == 0) update_and_factor_next<T>(raw, f, F, k0, k1, m, Dinv, perm, pivstat);
    return;
  }
  const int t = blockIdx.x * 32;
  if (blockIdx.y == 0) {
    if (t >= m - k1) return;
    update_tile<T, 32>(G, F, k0, NB, k1, m, t, 0, kbb, INT_MAX, kbb);
  } else {
    if (kbb + t >= m - k1) return;
    update_tile<T, 32>(G, F, k0, NB, k1, m, 0, kbb + t, 0, kbb, INT_MAX);
  }
}

template <typename T, int TM>
__global__ void __launch_bounds__(256) pair_update_kernel(cplx<T>* __restrict__ Fbuf,
                                                          const FrontDev* __restrict__ fr, int first, int k0) {
  __shared__ __align__(16) GemmLds<T, TM> G;
  const FrontDev f = fr[first + blockIdx.z];
  if (f.p <= k0) return;
  const int m = f.p + f.q;
  const int kb = min(2 * NB, f.p - k0);  // both panels' columns (panel a only when it is the last)
  const int base = k0 + kb;
  const int row0 = blockIdx.y * TM, col0 = blockIdx.x * TM;
  if (row0 >= m - base || col0 >= m - base) return;
  update_tile<T, TM>(G, Fbuf + f.f_off, k0, kb, base, m, row0, col0, 0);
}

// ---------------------------------------------------------------- panel strips
// One launch per panel step on levels where every workgroup of the step is
// resident at once (few fronts, the upper levels).  The step of panel b
// updates the trailing matrix outside panel b+1's rows and columns on MFMA
// tiles, while "strip" workgroups, one per 32-wide chunk of panel b+1's
// column strip (rows below the panel) or row strip (columns right of it),
// each apply panel b's update to their chunk and to panel b+1's diagonal
// block, factor that block (every strip workgroup of the front computes the
// same factorisation, so none waits for another; the first one stores it),
// and solve their chunk: L21 = chunk U11^{-1} or U12 = L11^{-1} P chunk.
// The step of panel b+1 then finds everything it reads in memory.

template <typename T>
struct StripLds {
  DiagLds<T> d;
  cplx<T> a[NB][NB + 1];  // previous panel's L21 rows of this panel  [row][k]
  cplx<T> b[NB][NB + 1];  // previous panel's U12 columns of this panel [k][column]
  cplx<T> t[NB][NB + 1];  // this workgroup's chunk [row][column]
  cplx<T> o[NB][NB + 1];  // the chunk's previous-panel operand, then the solved chunk
};

// (cr, ci) = the wave's 16 x 16 block (row block wave / 2, column block
// wave % 2) of the 32 x 32 product A B, A(i, k) and B(k, j) given by
// accessors; element v of a lane is (16 (wave / 2) + row(lk, v), 16 (wave % 2) + li).
template <typename T, typename FA, typename FB>
__device__ __forceinline__ void cgemm32(FA A, FB B, typename Mfma<T>::acc_t& cr, typename Mfma<T>::acc_t& ci) {
  const int lane = threadIdx.x % 64, li = lane % 16, lk = lane / 16, wave = threadIdx.x / 64;
  const int bi = wave / 2, bj = wave % 2;
#pragma unroll
  for (int v = 0; v < 4; ++v) { cr[v] = 0; ci[v] = 0; }
#pragma unroll
  for (int k4 = 0; k4 < NB; k4 += 4) {
    const int kk = k4 + lk;
    const cplx<T> a = A(16 * bi + li, kk), b = B(kk, 16 * bj + li);
    cr = Mfma<T>::step(a.x, b.x, cr);
    cr = Mfma<T>::step(-a.y, b.y, cr);
    ci = Mfma<T>::step(a.x, b.y, ci);
    ci = Mfma<T>::step(a.y, b.x, ci);
  }
}

// Strip workgroup s of panel kp (kbp = its width) of one front: chunks
// s < nch of the column strip, nch <= s < 2 nch of the row strip; s = 0
// also stores the block factorisation (and, with nch = 0, is the only one).
// PREV: first apply the update of the previous panel kprev (full width).
template <typename T, bool PREV>
__device__ __forceinline__ void strip_work(StripLds<T>& L, const FrontDev& f, cplx<T>* __restrict__ F,
                                           const int kprev, const int kp, const int m, const int s, const int nch,
                                           cplx<T>* __restrict__ Dinv, int* __restrict__ perm,
                                           double* __restrict__ pivstat) {
  const int tid = threadIdx.x;
  const int kbp = min(NB, f.p - kp);
  const int k2 = kp + kbp, rem = m - k2;
  const bool colstrip = s < nch;
  const int t0 = NB * (colstrip ? s : s - nch);
  const int cnt = max(0, min(NB, rem - t0));
  const int cc = max(cnt, 1);
  // every load first (clamped in-range indices, masked after the load)
  cplx<T> vd[4], va[4], vb[4], vt[4], vo[4];
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int e = tid + 256 * u, r = e % NB, c = e / NB;
    const int rp = min(r, kbp - 1), cp_ = min(c, kbp - 1);
    vd[u] = F[(kp + rp) + (long long)(kp + cp_) * m];
    if constexpr (PREV) {
      va[u] = F[(kp + rp) + (long long)(kprev + c) * m];
      vb[u] = F[(kprev + r) + (long long)(kp + cp_) * m];
    }
    // chunk row / column, clamped into the front (an empty chunk has none)
    const int xr = min(k2 + t0 + min(r, cc - 1), m - 1), xc = min(k2 + t0 + min(c, cc - 1), m - 1);
    if (colstrip) {
      vt[u] = F[xr + (long long)(kp + cp_) * m];
      if constexpr (PREV) vo[u] = F[xr + (long long)(kprev + c) * m];
    } else {
      vt[u] = F[(kp + rp) + (long long)xc * m];
      if constexpr (PREV) vo[u] = F[(kprev + r) + (long long)xc * m];
    }
  }
  const cplx<T> zero = mk<T>(0, 0);
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int e = tid + 256 * u, r = e % NB, c = e / NB;
    L.d.m[0][r][c] = r < kbp && c < kbp ? vd[u] : mk<T>(r == c ? 1 : 0, 0);
    if constexpr (PREV) {
      L.a[r][c] = r < kbp ? va[u] : zero;
      L.b[r][c] = c < kbp ? vb[u] : zero;
    }
    if (colstrip) {
      L.t[r][c] = r < cnt && c < kbp ? vt[u] : zero;
      if constexpr (PREV) L.o[r][c] = r < cnt ? vo[u] : zero;
    } else {
      L.t[r][c] = r < kbp && c < cnt ? vt[u] : zero;
      if constexpr (PREV) L.o[r][c] = c < cnt ? vo[u] : zero;
    }
  }
  __syncthreads();
  using acc_t = typename Mfma<T>::acc_t;
  const int lane = tid % 64, li = lane % 16, lk = lane / 16, wave = tid / 64;
  const int orow = 16 * (wave / 2), ocol = 16 * (wave % 2) + li;
  if constexpr (PREV) {
    // block -= A B; chunk -= O B (column strip) or A O (row strip).  Each
    // element is updated by the lane that computed it, and no product reads m or t.
    acc_t dr, di, tr, ti;
    cgemm32<T>([&](int i, int k) { return L.a[i][k]; }, [&](int k, int j) { return L.b[k][j]; }, dr, di);
    if (colstrip)
      cgemm32<T>([&](int i, int k) { return L.o[i][k]; }, [&](int k, int j) { return L.b[k][j]; }, tr, ti);
    else
      cgemm32<T>([&](int i, int k) { return L.a[i][k]; }, [&](int k, int j) { return L.o[k][j]; }, tr, ti);
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int row = orow + Mfma<T>::row(lk, v);
      cplx<T> x = L.d.m[0][row][ocol];
      x.x -= dr[v];
      x.y -= di[v];
      L.d.m[0][row][ocol] = x;
      cplx<T> y = L.t[row][ocol];
      y.x -= tr[v];
      y.y -= ti[v];
      L.t[row][ocol] = y;
    }
    __syncthreads();
  }
  diag_factor_block<T, 256>(L.d, f, kp, kbp, Dinv, perm, pivstat, s == 0);
  if (cnt == 0) return;
  acc_t ur, ui;
  if (colstrip) {
    // L21(row, j) = sum_k chunk(row, k) U^{-1}(k, j), U^{-1}(k, j) = X_R(31-k, 31-j) for k <= j
    cgemm32<T>([&](int i, int k) { return L.t[i][k]; },
               [&](int k, int j) { return k <= j ? L.d.x[1][NB - 1 - k][NB - 1 - j] : mk<T>(0, 0); }, ur, ui);
  } else {
    // U12(i, c) = sum_k L^{-1}(i, k) chunk(src[k], c), L^{-1}(i, k) = X_L(i, k) for i >= k
    cgemm32<T>([&](int i, int k) { return i >= k ? L.d.x[0][i][k] : mk<T>(0, 0); },
               [&](int k, int j) { return L.t[L.d.src[k]][j]; }, ur, ui);
  }
#pragma unroll
  for (int v = 0; v < 4; ++v) L.o[orow + Mfma<T>::row(lk, v)][ocol] = mk<T>(ur[v], ui[v]);
  __syncthreads();
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int e = tid + 256 * u, r = e % NB, c = e / NB;
    if (colstrip) {
      if (r < cnt && c < kbp) F[(k2 + t0 + r) + (long long)(kp + c) * m] = L.o[r][c];
    } else {
      if (r < kbp && c < cnt) F[(kp + r) + (long long)(k2 + t0 + c) * m] = L.o[r][c];
    }
  }
}

// Panel 0 of every front of a level: strip workgroups (blockIdx.x) only.
template <typename T>
__global__ void __launch_bounds__(256) strip_first_kernel(cplx<T>* __restrict__ Fbuf, const FrontDev* __restrict__ fr,
                                                          int first, cplx<T>* __restrict__ Dinv,
                                                          int* __restrict__ perm, double* __restrict__ pivstat) {
  __shared__ StripLds<T> L;
  const FrontDev f = fr[first + blockIdx.y];
  const int m = f.p + f.q;
  const int k2 = min(NB, f.p);
  const int nch = (m - k2 + NB - 1) / NB;
  const int s = blockIdx.x;
  if (s >= max(1, 2 * nch)) return;
  strip_work<T, false>(L, f, Fbuf + f.f_off, 0, 0, m, s, nch, Dinv, perm, pivstat);
}

// Panel step k0: block row 0 holds the strip workgroups of the next panel
// (fronts that have one), rows 1.. the update tiles, over [k2, m)^2 when
// the front has a next panel (k2 = its end) and over [k1, m)^2 otherwise.
template <typename T, int TM>
__global__ void __launch_bounds__(256) panel_step_kernel(cplx<T>* __restrict__ Fbuf, const FrontDev* __restrict__ fr,
                                                         int first, int k0, cplx<T>* __restrict__ Dinv,
                                                         int* __restrict__ perm, double* __restrict__ pivstat) {
  constexpr size_t kRaw = sizeof(StripLds<T>) > sizeof(GemmLds<T, TM>) ? sizeof(StripLds<T>) : sizeof(GemmLds<T, TM>);
  __shared__ __align__(16) unsigned char raw[kRaw];
  const FrontDev f = fr[first + blockIdx.z];
  if (f.p <= k0) return;
  const int kb = min(NB, f.p - k0);
  const int k1 = k0 + kb;
  const int m = f.p + f.q;
  cplx<T>* F = Fbuf + f.f_off;
  const bool next = f.p > k1;
  const int k2 = next ? k1 + min(NB, f.p - k1) : k1;
  if (blockIdx.y == 0) {
    if (!next) return;
    const int nch = (m - k2 + NB - 1) / NB;
    const int s = blockIdx.x;
    if (s >= max(1, 2 * nch)) return;
    strip_work<T, true>(*reinterpret_cast<StripLds<T>*>(raw), f, F, k0, k1, m, s, nch, Dinv, perm, pivstat);
    return;
  }
  const int base = k2;
  const int row0 = ((int)blockIdx.y - 1) * TM, col0 = blockIdx.x * TM;
  if (row0 >= m - base || col0 >= m - base) return;
  update_tile<T, TM>(*reinterpret_cast<GemmLds<T, TM>*>(raw), F, k0, kb, base, m, row0, col0, 0);
}

// ---------------------------------------------------------------- solves
// Right-hand sides are taken in groups of NR per workgroup (blockIdx.y), so
// each factor entry is read once per group; a right-hand side's arithmetic
// does not depend on the group it is in.  The front's working vectors live in
// LDS when the level's largest front fits (VL), else in the per-front
// vector buffer in HBM; either way the per-front vector buffer holds them at
// the end (y_I for the backward sweep, the update for the parent).
//
// Per panel the data-independent loads go out first and stay in flight: the
// panel's off-diagonal block (L21 rows or U12 columns) for the first 256
// rows or columns, and the next panel's inverted diagonal block and
// permutation, which are kept in registers until they can be stored.  The
// 32-wide triangular products use eight threads per row.

// out[k] = sum_j D(i, j) in(k, j) for k < NR, i = tid / 8: eight threads per
// row i each sum every eighth j (s = tid % 8, in j order, two interleaved
// partial sums), and an xor butterfly combines the eight.  The order is the
// same for every NR, so a right-hand side's result does not depend on the
// group it is solved in.
template <typename T, int NR>
__device__ __forceinline__ void tri_apply(const cplx<T> (*D)[NB + 1], const cplx<T> (*in)[NB], const int tid,
                                          cplx<T> (&out)[NR]) {
  constexpr int G = 256 / NB;
  static_assert(G == 8, "256 threads over 32 rows");
  const int i = tid / G, s = tid % G;
  cplx<T> dv[NB / G];
#pragma unroll
  for (int t = 0; t < NB / G; ++t) dv[t] = D[i][s + G * t];
#pragma unroll
  for (int k = 0; k < NR; ++k) {
    cplx<T> a0 = mk<T>(0, 0), a1 = mk<T>(0, 0);
#pragma unroll
    for (int t = 0; t < NB / G; ++t) {
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

// Forward sweep of one front: v = [z(I); 0] + children's updates; per panel:
//   y_b = L11^{-1} (P_b v_b),  v(k1:m) -= L21 y_b.
// FORM: the same chain on the unit vectors e_j, j < p (NR per workgroup,
// blockIdx.y the group), written as the columns of the front's forward
// operator Gf (m x p, column-major, at Gop + g_off): the sweep's output for
// any input is then [0; v_B] + Gf v_I.
// FORM and TRANS: the same chain with U^T in place of P^T L (U11^T is lower
// triangular in the (column, pivot-row) order, no permutation, the block
// inverses transposed, U12^T below), whose output for e_i is row i of the
// backward sweep's operator [U11^{-1}, -U11^{-1} U12]: the rows are written
// as the columns of GbT (m x p, column-major, at Gop + g_off + m p).
template <typename T, int NR, bool VL, int TPB, bool FORM = false, bool TRANS = false>
__global__ void __launch_bounds__(TPB) fwd_kernel(const cplx<T>* __restrict__ Fbuf, const cplx<T>* __restrict__ Dinv,
                                                  const FrontDev* __restrict__ fr, const int* __restrict__ idx,
                                                  const int* __restrict__ cpos, const int* __restrict__ perm,
                                                  const cplx<T>* __restrict__ z, cplx<T>* __restrict__ vbuf, int first,
                                                  int nrhs, long long N, long long vstride, cplx<T>* __restrict__ Gop) {
  static_assert(NR * NB <= 2 * TPB, "at most two gathered panel entries per thread");
  static_assert(TPB == 256 || TPB == 512, "256 or 512 threads");
  static_assert(!FORM || VL, "operators are formed with the vectors in LDS");
  constexpr bool G2 = NR * NB > TPB;  // a second gathered entry, right-hand side gk + TPB / NB
  static_assert(FORM || !TRANS, "the transposed chain only forms operators");
  constexpr int IPT = NB * NB / TPB;  // inverse-block entries per thread
  extern __shared__ unsigned char smem_raw[];
  __shared__ cplx<T> Li[2][NB][NB + 1];
  // entry e of a column-major inverse block (e = tid + k TPB) into LDS,
  // transposed for TRANS
  auto put_inv = [](cplx<T> (*D)[NB + 1], const int e, const cplx<T>& v) {
    if constexpr (TRANS) D[e / NB][e % NB] = v;
    else D[e % NB][e / NB] = v;
  };
  __shared__ cplx<T> tb[NR][NB];
  __shared__ cplx<T> yb[NR][NB];
  const FrontDev f = fr[first + blockIdx.x];
  const int r0 = blockIdx.y * NR;
  if (FORM && r0 >= f.p) return;  // the level's largest front sets the grid
  const int nr = min(NR, (FORM ? f.p : nrhs) - r0);
  const int m = f.p + f.q;
  const cplx<T>* F = Fbuf + f.f_off;
  const int* id = idx + f.idx_off;
  const int* cp = cpos + 2 * f.idx_off;
  const int* pm = perm + f.piv_off;
  const long long coff[2] = {f.cidx[0], f.cidx[1]};
  // HBM copy, stride vstride (FORM: columns r0.. of Gf, stride m)
  cplx<T>* vg = FORM ? Gop + f.g_off + (TRANS ? (long long)m * f.p : 0LL) + (long long)r0 * m
                     : vbuf + (long long)r0 * vstride + f.idx_off;
  const long long gstride = FORM ? m : vstride;
  // a typed LDS or global pointer (a run-time choice would make every access
  // a flat one, with conservative waits)
  cplx<T>* vp;
  if constexpr (VL) vp = reinterpret_cast<cplx<T>*>(smem_raw);
  else vp = vg;
  const long long vs = VL ? m : vstride;
  const int tid = threadIdx.x;
  const int gk = tid / NB, gj = tid % NB;  // gather slot of this thread (tid < NR NB)
  // loads below use clamped in-range indices instead of branches (padded
  // entries meet exact zeros, and padded rows are never stored), so the
  // wait counts stay exact and the prefetches stay in flight
  // The L21 rows are prefetched at the panel start when the registers allow
  // (NR right-hand sides of at most 16 bytes in all); with more right-hand
  // sides each entry carries NR times the arithmetic, and rows are loaded
  // eight entries at a time after the product.  (Loading the next panel's
  // rows during the current panel was measured slower.)
  constexpr bool PRE = sizeof(cplx<T>) * NR <= 16 && (TPB == 256 || sizeof(T) == 4);
  constexpr int LN = PRE ? NB : 1;
  // entry (r, k0 + j) of L21, or of U12^T for TRANS
  auto lentry = [&](const int r, const int kj) {
    if constexpr (TRANS) return F[(long long)r * m + kj];
    else return F[(long long)kj * m + (unsigned)r];
  };
  auto load_l = [&](const int k0p, cplx<T>(&dst)[LN]) {
    if constexpr (PRE) {
      const int kbp = min(NB, f.p - k0p);
      const int rr = min(k0p + kbp + tid, m - 1);
#pragma unroll
      for (int j = 0; j < NB; ++j) dst[j] = lentry(rr, k0p + min(j, kbp - 1));
    }
  };
  cplx<T> lrow[LN];
  load_l(0, lrow);  // panel 0's rows go out before the gather of v below
  int pnext = TRANS ? min(gj, f.p - 1) : pm[min(gj, f.p - 1)];
  const cplx<T>* Lg0 = Dinv + f.dinv_off + (TRANS ? NB * NB : 0);
  const cplx<T> li0 = Lg0[tid], li1 = Lg0[tid + TPB];
  const cplx<T> li2 = IPT > 2 ? Lg0[tid + 2 * TPB] : li0, li3 = IPT > 2 ? Lg0[tid + 3 * TPB] : li0;
  // v = [z(I); 0] + children's updates: four entries per thread per pass,
  // the index loads of all four, then their value loads, in flight together
  if constexpr (FORM)
    for (int e = tid; e < m * nr; e += TPB) {
      const int r = e % m, k = e / m;
      vp[k * vs + r] = mk<T>(r == r0 + k ? 1 : 0, 0);
    }
  else
  for (int e0 = 0; e0 < m * nr; e0 += 4 * TPB) {
    int gidx[4], q0[4], q1[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int e = min(e0 + tid + TPB * u, m * nr - 1), r = e % m;
      gidx[u] = id[min(r, f.p - 1)];
      q0[u] = coff[0] >= 0 ? cp[2 * r] : -1;
      q1[u] = coff[1] >= 0 ? cp[2 * r + 1] : -1;
    }
    cplx<T> sv[4], c0v[4], c1v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int e = min(e0 + tid + TPB * u, m * nr - 1), k = e / m;
      const long long rb = (long long)(r0 + k) * vstride;
      sv[u] = z[(long long)(r0 + k) * N + gidx[u]];
      c0v[u] = vbuf[rb + (q0[u] >= 0 ? coff[0] + q0[u] : 0)];
      c1v[u] = vbuf[rb + (q1[u] >= 0 ? coff[1] + q1[u] : 0)];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int e = e0 + tid + TPB * u;
      if (e < m * nr) {
        const int r = e % m, k = e / m;
        cplx<T> s = r < f.p ? sv[u] : mk<T>(0, 0);
        if (q0[u] >= 0) s = cadd(s, c0v[u]);
        if (q1[u] >= 0) s = cadd(s, c1v[u]);
        vp[k * vs + r] = s;
      }
    }
  }
  put_inv(Li[0], tid, li0);
  put_inv(Li[0], tid + TPB, li1);
  if constexpr (IPT > 2) {
    put_inv(Li[0], tid + 2 * TPB, li2);
    put_inv(Li[0], tid + 3 * TPB, li3);
  }
  __syncthreads();
  auto panel = [&](const int b, cplx<T>(&lc)[LN]) {
    const int k0 = b * NB;
    const int kb = min(NB, f.p - k0);
    const int k1 = k0 + kb;
    const int cur = b & 1;
    const bool more = k1 < f.p;
    // gather P_b v_b (issued before the prefetches, so waiting for it does not wait for them)
    const cplx<T> gv = vp[min(gk, nr - 1) * vs + pnext];
    const cplx<T> g = tid < NR * NB && gk < nr && gj < kb ? gv : mk<T>(0, 0);
    constexpr int GK2 = TPB / NB;
    cplx<T> g2 = mk<T>(0, 0);
    if constexpr (G2) {
      const cplx<T> gv2 = vp[min(gk + GK2, nr - 1) * vs + pnext];
      g2 = gk + GK2 < nr && gj < kb ? gv2 : mk<T>(0, 0);
    }
    __builtin_amdgcn_sched_barrier(0);
    // next panel's L11^{-1} (the last panel reloads its own: unused, but it
    // keeps these loads unconditional so they stay in registers)
    // (named scalars: a small array here is left in scratch by the compiler)
    const cplx<T>* Lg = Dinv + f.dinv_off + (long long)(more ? b + 1 : b) * 2 * NB * NB + (TRANS ? NB * NB : 0);
    const cplx<T> lin0 = Lg[tid], lin1 = Lg[tid + TPB];
    const cplx<T> lin2 = IPT > 2 ? Lg[tid + 2 * TPB] : lin0, lin3 = IPT > 2 ? Lg[tid + 3 * TPB] : lin0;
    pnext = TRANS ? min(k1 + gj, f.p - 1) : pm[min(k1 + gj, f.p - 1)];
    if (b > 0) load_l(k0, lc);
    __builtin_amdgcn_sched_barrier(0);
    if (tid < NR * NB) tb[gk][gj] = g;
    if constexpr (G2) tb[gk + GK2][gj] = g2;
    // Li[cur ^ 1] was last read before the previous panel's final barrier
    put_inv(Li[cur ^ 1], tid, lin0);
    put_inv(Li[cur ^ 1], tid + TPB, lin1);
    if constexpr (IPT > 2) {
      put_inv(Li[cur ^ 1], tid + 2 * TPB, lin2);
      put_inv(Li[cur ^ 1], tid + 3 * TPB, lin3);
    }
    __syncthreads();
    if (tid < 256) {  // the 32-row product uses the first four waves
      cplx<T> y[NR];
      tri_apply<T, NR>(Li[cur], tb, tid, y);
      const int i = tid / 8;
      if (tid % 8 == 0) {
#pragma unroll
        for (int k = 0; k < NR; ++k) {
          yb[k][i] = y[k];
          if (k < nr && i < kb) vp[k * vs + k0 + i] = y[k];
        }
      }
    }
    __syncthreads();
    const int rfirst = k1 + tid;
    if constexpr (PRE) {
      if (rfirst < m) {
        cplx<T> acc[NR];
#pragma unroll
        for (int k = 0; k < NR; ++k) acc[k] = vp[min(k, nr - 1) * vs + rfirst];
        chunked<NB * NR, sizeof(T) == 8 ? 4 : 8>(
            [&](int q) { return yb[q % NR][q / NR]; },
            [&](int q, const cplx<T>& y) { acc[q % NR] = cfms(acc[q % NR], lc[q / NR], y); });
#pragma unroll
        for (int k = 0; k < NR; ++k)
          if (k < nr) vp[k * vs + rfirst] = acc[k];
      }
    }
    for (int r = PRE ? rfirst + TPB : rfirst; r < m; r += TPB) {  // rows not prefetched
      cplx<T> acc[NR];
#pragma unroll
      for (int k = 0; k < NR; ++k) acc[k] = vp[min(k, nr - 1) * vs + r];
#pragma unroll 1
      for (int j0 = 0; j0 < NB; j0 += 8) {
        cplx<T> l8[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) l8[u] = lentry(r, k0 + min(j0 + u, kb - 1));
#pragma unroll
        for (int u = 0; u < 8; ++u)
#pragma unroll
          for (int k = 0; k < NR; ++k) acc[k] = cfms(acc[k], l8[u], yb[k][j0 + u]);
      }
#pragma unroll
      for (int k = 0; k < NR; ++k)
        if (k < nr) vp[k * vs + r] = acc[k];
    }
    __syncthreads();
  };
  const int nblk = (f.p + NB - 1) / NB;
  for (int b = 0; b < nblk; ++b) panel(b, lrow);
  if constexpr (VL)
    for (int e = tid; e < m * nr; e += TPB) {
      int r = e % m, k = e / m;
      vg[(long long)k * gstride + r] = vp[k * vs + r];
    }
}

// Backward sweep: x_B from the global solution, then per panel from the last:
//   x_b = U11^{-1} (y_b - U12 x(k1:m)).  Writes x at the front's grid points.
// Thread (j, grp) = (tid % NB, tid / NB) forms the U12 row j product over
// the columns k1 + grp + 8t; the eight column groups are added in order.
template <typename T, int NR, bool VL, int TPB>
__global__ void __launch_bounds__(TPB) bwd_kernel(const cplx<T>* __restrict__ Fbuf, const cplx<T>* __restrict__ Dinv,
                                                  const FrontDev* __restrict__ fr, const int* __restrict__ idx,
                                                  cplx<T>* __restrict__ x, cplx<T>* __restrict__ vbuf, int first,
                                                  int nrhs, long long N, long long vstride,
                                                  double2* __restrict__ xw) {
  static_assert(TPB == 256 || TPB == 512, "256 or 512 threads");
  constexpr int G = TPB / NB;  // column groups
  constexpr int IPT = NB * NB / TPB;  // inverse-block entries per thread
  // With 512 threads, complex64, one right-hand side and the vectors in LDS
  // the registers allow a second U12 buffer of 24 columns per thread (384
  // per pass): each panel
  // then loads the next (lower) panel's block, so its latency overlaps the
  // current panel.
  constexpr bool DB = TPB == 512 && NR == 1 && sizeof(T) == 4 && VL;
  constexpr int TU = DB ? 24 : (sizeof(T) == 8 ? 16 : 32);  // U12 columns per thread held in flight
  extern __shared__ unsigned char smem_raw[];
  __shared__ cplx<T> Ui[2][NB][NB + 1];
  __shared__ cplx<T> part[G][NR][NB];
  __shared__ cplx<T> rb[NR][NB];
  const FrontDev f = fr[first + blockIdx.x];
  const int r0 = blockIdx.y * NR;
  const int nr = min(NR, nrhs - r0);
  const int m = f.p + f.q;
  const cplx<T>* F = Fbuf + f.f_off;
  const int* id = idx + f.idx_off;
  cplx<T>* vg = vbuf + (long long)r0 * vstride + f.idx_off;
  // a typed LDS or global pointer (a run-time choice would make every access
  // a flat one, with conservative waits)
  cplx<T>* vp;
  if constexpr (VL) vp = reinterpret_cast<cplx<T>*>(smem_raw);
  else vp = vg;
  const long long vs = VL ? m : vstride;
  const int tid = threadIdx.x;
  const int nblk = (f.p + NB - 1) / NB;
  const cplx<T>* Ug0 = Dinv + f.dinv_off + (long long)(nblk - 1) * 2 * NB * NB + NB * NB;
  const cplx<T> ui0 = Ug0[tid], ui1 = Ug0[tid + TPB];
  const cplx<T> ui2 = IPT > 2 ? Ug0[tid + 2 * TPB] : ui0, ui3 = IPT > 2 ? Ug0[tid + 3 * TPB] : ui0;
  const int j = tid % NB, grp = tid / NB;
  // U12 block of a panel (first TU columns of this thread): loaded at the
  // panel start, or with DB one panel ahead (with 256 threads a second
  // buffer would spill)
  auto load_u = [&](const int bp, cplx<T>(&dst)[TU]) {
    const int k0p = bp * NB, kbp = min(NB, f.p - k0p), k1p = k0p + kbp;
#pragma unroll
    for (int t = 0; t < TU; ++t) dst[t] = F[(k0p + min(j, kbp - 1)) + (long long)min(k1p + grp + G * t, m - 1) * m];
  };
  cplx<T> ucol[TU], ucol2[DB ? TU : 1];
  if constexpr (DB) load_u(nblk - 1, ucol);  // before the gathers below, so the two overlap
  // v = [y(I) from the forward sweep; x(B) from the ancestors]
  for (int e = tid; e < m * nr; e += TPB) {
    const int r = e % m, k = e / m;
    if (r >= f.p) vp[k * vs + r] = x[(long long)(r0 + k) * N + id[r]];
    else if constexpr (VL) vp[k * vs + r] = vg[(long long)k * vstride + r];
  }
  {
    const int cb = (nblk - 1) & 1;
    Ui[cb][tid % NB][tid / NB] = ui0;
    Ui[cb][tid % NB][tid / NB + TPB / NB] = ui1;
    if constexpr (IPT > 2) {
      Ui[cb][tid % NB][tid / NB + 2 * TPB / NB] = ui2;
      Ui[cb][tid % NB][tid / NB + 3 * TPB / NB] = ui3;
    }
  }
  auto panel = [&](const int b, cplx<T>(&u)[TU], cplx<T>(&un)[DB ? TU : 1]) {
    const int k0 = b * NB;
    const int kb = min(NB, f.p - k0);
    const int k1 = k0 + kb;
    const int cur = b & 1;
    // next (lower) panel's U11^{-1}, four entries per thread (panel 0
    // reloads its own); named scalars, since a small array here was left in
    // scratch memory by the compiler
    const cplx<T>* Ugn = Dinv + f.dinv_off + (long long)(b > 0 ? b - 1 : 0) * 2 * NB * NB + NB * NB;
    const cplx<T> uin0 = Ugn[tid], uin1 = Ugn[tid + TPB];
    const cplx<T> uin2 = IPT > 2 ? Ugn[tid + 2 * TPB] : uin0, uin3 = IPT > 2 ? Ugn[tid + 3 * TPB] : uin0;
    const int gi = id[k0 + min(tid / 8, kb - 1)];  // grid index of row tid / 8, for writing x
    if constexpr (DB)
      load_u(b > 0 ? b - 1 : b, un);  // unconditional: the last panel reloads its own block (unused)
    else
      load_u(b, u);
    __syncthreads();  // x(k1:m) of the previous panel is in place; Ui[cur ^ 1] is free
    Ui[cur ^ 1][tid % NB][tid / NB] = uin0;
    Ui[cur ^ 1][tid % NB][tid / NB + TPB / NB] = uin1;
    if constexpr (IPT > 2) {
      Ui[cur ^ 1][tid % NB][tid / NB + 2 * TPB / NB] = uin2;
      Ui[cur ^ 1][tid % NB][tid / NB + 3 * TPB / NB] = uin3;
    }
    cplx<T> acc[NR];
#pragma unroll
    for (int k = 0; k < NR; ++k) acc[k] = mk<T>(0, 0);
    auto product = [&](const int c0, const cplx<T>(&uc)[TU]) {
      chunked<TU * NR, (sizeof(T) == 8 && NR >= 4) ? 4 : 8>(
          [&](int q) {
            const int c = c0 + G * (q / NR), k = q % NR;
            const cplx<T> v = vp[min(k, nr - 1) * vs + min(c, m - 1)];
            return c < m && k < nr ? v : mk<T>(0, 0);
          },
          [&](int q, const cplx<T>& xv) { acc[q % NR] = cfma(acc[q % NR], uc[q / NR], xv); });
    };
    if (k1 + grp < m) product(k1 + grp, u);
    for (int c0 = k1 + grp + G * TU; c0 < m; c0 += G * TU) {  // more than 256 columns right of the panel
      cplx<T> u2[TU];
#pragma unroll
      for (int t = 0; t < TU; ++t) u2[t] = F[(k0 + min(j, kb - 1)) + (long long)min(c0 + G * t, m - 1) * m];
      product(c0, u2);
    }
#pragma unroll
    for (int k = 0; k < NR; ++k) part[grp][k][j] = acc[k];
    __syncthreads();
    for (int e = tid; e < NR * NB; e += TPB) {
      int jj = e % NB, k = e / NB;
      cplx<T> s = part[0][k][jj];
      for (int g = 1; g < G; ++g) s = cadd(s, part[g][k][jj]);
      rb[k][jj] = (k < nr && jj < kb) ? csub(vp[k * vs + k0 + jj], s) : mk<T>(0, 0);
    }
    __syncthreads();
    if (tid < 256) {  // the 32-row product uses the first four waves
      cplx<T> xs[NR];
      tri_apply<T, NR>(Ui[cur], rb, tid, xs);
      const int i = tid / 8;
      if (tid % 8 == 0 && i < kb) {
#pragma unroll
        for (int k = 0; k < NR; ++k) {
          if (k < nr) {
            vp[k * vs + k0 + i] = xs[k];
            x[(long long)(r0 + k) * N + gi] = xs[k];
            if (xw) xw[(long long)(r0 + k) * N + gi] = widen(xs[k]);
          }
        }
      }
    }
  };
  if constexpr (DB) {
    for (int b = nblk - 1; b >= 0; b -= 2) {
      panel(b, ucol, ucol2);
      if (b >= 1) panel(b - 1, ucol2, ucol);
    }
  } else {
    for (int b = nblk - 1; b >= 0; --b) panel(b, ucol, ucol2);
  }
}

// ---- Sweeps of the small-front levels (Plan::level_small_sweep): fronts of
// at most two panels whose rows below (columns right of) the first panel
// fit 128 threads.  Every load of a front (both inverse blocks, both
// panels' L21 rows or U12 columns, the row order) is issued at the start,
// so the chain waits for memory once instead of once per panel; vectors in
// LDS.  The arithmetic is that of fwd_kernel / bwd_kernel with 256 threads
// in the same order (gather sums, 32-term row products in j order, column
// groups added in order), so the results are the same bit for bit and the
// choice between them may depend on the group size: these run for groups
// of one right-hand side (the backward one in complex64 only: in complex128
// its registers allow fewer workgroups per CU than the chain kernel's).
constexpr int SM = 160;  // front rows a small-front sweep holds in LDS

// v = [z(I); 0] + children's updates of a front into LDS (k < nr)
template <typename T, int NR>
__device__ __forceinline__ void gather_front_input(cplx<T> (*vl)[SM], const FrontDev& f, const int* __restrict__ id,
                                                   const int* __restrict__ cp, const cplx<T>* __restrict__ z,
                                                   const cplx<T>* __restrict__ vbuf, const int r0, const int nr,
                                                   const long long N, const long long vstride) {
  const int m = f.p + f.q, tid = threadIdx.x;
  for (int e0 = 0; e0 < m * nr; e0 += 2 * 256) {
    int gidx[2], q0[2], q1[2];
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int e = min(e0 + tid + 256 * u, m * nr - 1), r = e % m;
      gidx[u] = id[min(r, f.p - 1)];
      q0[u] = f.cidx[0] >= 0 ? cp[2 * r] : -1;
      q1[u] = f.cidx[1] >= 0 ? cp[2 * r + 1] : -1;
    }
    cplx<T> sv[2], c0v[2], c1v[2];
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int e = min(e0 + tid + 256 * u, m * nr - 1), k = e / m;
      const long long rb = (long long)(r0 + k) * vstride;
      sv[u] = z[(long long)(r0 + k) * N + gidx[u]];
      c0v[u] = vbuf[rb + (q0[u] >= 0 ? f.cidx[0] + q0[u] : 0)];
      c1v[u] = vbuf[rb + (q1[u] >= 0 ? f.cidx[1] + q1[u] : 0)];
    }
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int e = e0 + tid + 256 * u;
      if (e < m * nr) {
        const int r = e % m, k = e / m;
        cplx<T> s = r < f.p ? sv[u] : mk<T>(0, 0);
        if (q0[u] >= 0) s = cadd(s, c0v[u]);
        if (q1[u] >= 0) s = cadd(s, c1v[u]);
        vl[k][r] = s;
      }
    }
  }
}

// Forward sweep of a small front: threads 0-127 hold the L21 rows of panel
// 0 (row kb0 + t), threads 128-255 those of panel 1 (row p + t - 128).
template <typename T, int NR>
__global__ void __launch_bounds__(256) fwd_small_kernel(const cplx<T>* __restrict__ Fbuf,
                                                        const cplx<T>* __restrict__ Dinv,
                                                        const FrontDev* __restrict__ fr, const int* __restrict__ idx,
                                                        const int* __restrict__ cpos, const int* __restrict__ perm,
                                                        const cplx<T>* __restrict__ z, cplx<T>* __restrict__ vbuf,
                                                        int first, int nrhs, long long N, long long vstride) {
  static_assert(NR * NB <= 256, "one gather thread per panel entry");
  __shared__ cplx<T> Li[2][NB][NB + 1];
  __shared__ cplx<T> vl[NR][SM];
  __shared__ cplx<T> tb[NR][NB];
  __shared__ cplx<T> yb[NR][NB];
  const FrontDev f = fr[first + blockIdx.x];
  const int r0 = blockIdx.y * NR, nr = min(NR, nrhs - r0);
  const int m = f.p + f.q, nblk = (f.p + NB - 1) / NB;
  const cplx<T>* F = Fbuf + f.f_off;
  const int* id = idx + f.idx_off;
  const int* cp = cpos + 2 * f.idx_off;
  const int* pm = perm + f.piv_off;
  const int tid = threadIdx.x, half = tid / 128, t = tid % 128;
  const int gk = tid / NB, gj = tid % NB;
  // this thread's L21 row (a front of one panel: the upper half reloads
  // panel 0's rows, unused)
  const int hk0 = min(half, nblk - 1) * NB, hkb = min(NB, f.p - hk0);
  const int hr = min(hk0 + hkb + t, m - 1);
  cplx<T> lr[NB];
#pragma unroll
  for (int j = 0; j < NB; ++j) lr[j] = F[(long long)(hk0 + min(j, hkb - 1)) * m + hr];
  const int pn0 = pm[min(gj, f.p - 1)], pn1 = pm[min(NB + gj, f.p - 1)];
  const cplx<T>* Lg = Dinv + f.dinv_off;
  const cplx<T>* Lg1 = Lg + (nblk > 1 ? 2 * NB * NB : 0);
  cplx<T> l0[4], l1[4];
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    l0[u] = Lg[tid + 256 * u];
    l1[u] = Lg1[tid + 256 * u];
  }
  gather_front_input<T, NR>(vl, f, id, cp, z, vbuf, r0, nr, N, vstride);
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int e = tid + 256 * u;
    Li[0][e % NB][e / NB] = l0[u];
    Li[1][e % NB][e / NB] = l1[u];
  }
  __syncthreads();
  for (int b = 0; b < nblk; ++b) {
    const int k0 = b * NB, kb = min(NB, f.p - k0), k1 = k0 + kb;
    if (tid < NR * NB) tb[gk][gj] = gk < nr && gj < kb ? vl[min(gk, nr - 1)][b ? pn1 : pn0] : mk<T>(0, 0);
    __syncthreads();
    cplx<T> y[NR];
    tri_apply<T, NR>(Li[b], tb, tid, y);
    if (tid % 8 == 0) {
      const int i = tid / 8;
#pragma unroll
      for (int k = 0; k < NR; ++k) {
        yb[k][i] = y[k];
        if (k < nr && i < kb) vl[k][k0 + i] = y[k];
      }
    }
    __syncthreads();
    const int r = k1 + t;
    if (half == b && r < m) {
      cplx<T> acc[NR];
#pragma unroll
      for (int k = 0; k < NR; ++k) acc[k] = vl[min(k, nr - 1)][r];
      chunked<NB * NR, sizeof(T) == 8 ? 4 : 8>(
          [&](int q) { return yb[q % NR][q / NR]; },
          [&](int q, const cplx<T>& yv) { acc[q % NR] = cfms(acc[q % NR], lr[q / NR], yv); });
#pragma unroll
      for (int k = 0; k < NR; ++k)
        if (k < nr) vl[k][r] = acc[k];
    }
    __syncthreads();
  }
  cplx<T>* vg = vbuf + (long long)r0 * vstride + f.idx_off;
  for (int e = tid; e < m * nr; e += 256) {
    const int r = e % m, k = e / m;
    vg[(long long)k * vstride + r] = vl[k][r];
  }
}

// Backward sweep of a small front: thread (j, grp) = (tid % 32, tid / 32)
// holds, for each panel, the U12 row j entries of the columns k1 + grp + 8t
// (t < 16); the eight column groups are added in order.
template <typename T, int NR>
__global__ void __launch_bounds__(256) bwd_small_kernel(const cplx<T>* __restrict__ Fbuf,
                                                        const cplx<T>* __restrict__ Dinv,
                                                        const FrontDev* __restrict__ fr, const int* __restrict__ idx,
                                                        cplx<T>* __restrict__ x, cplx<T>* __restrict__ vbuf, int first,
                                                        int nrhs, long long N, long long vstride,
                                                        double2* __restrict__ xw) {
  constexpr int G = 8, TU = 128 / G;
  __shared__ cplx<T> Ui[2][NB][NB + 1];
  __shared__ cplx<T> vl[NR][SM];
  __shared__ cplx<T> part[G][NR][NB];
  __shared__ cplx<T> rb[NR][NB];
  const FrontDev f = fr[first + blockIdx.x];
  const int r0 = blockIdx.y * NR, nr = min(NR, nrhs - r0);
  const int m = f.p + f.q, nblk = (f.p + NB - 1) / NB;
  const cplx<T>* F = Fbuf + f.f_off;
  const int* id = idx + f.idx_off;
  const int tid = threadIdx.x, j = tid % NB, grp = tid / NB;
  cplx<T> uc[2][TU];
#pragma unroll
  for (int b = 0; b < 2; ++b) {
    const int k0 = min(b, nblk - 1) * NB, kb = min(NB, f.p - k0), k1 = k0 + kb;
#pragma unroll
    for (int t = 0; t < TU; ++t) uc[b][t] = F[(k0 + min(j, kb - 1)) + (long long)min(k1 + grp + G * t, m - 1) * m];
  }
  const cplx<T>* Ug = Dinv + f.dinv_off + NB * NB;
  const cplx<T>* Ug1 = Ug + (nblk > 1 ? 2 * NB * NB : 0);
  cplx<T> u0[4], u1[4];
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    u0[u] = Ug[tid + 256 * u];
    u1[u] = Ug1[tid + 256 * u];
  }
  const int gi0 = id[min(tid / 8, f.p - 1)], gi1 = id[min(NB + tid / 8, f.p - 1)];
  // v = [y(I) from the forward sweep; x(B) from the ancestors]
  const cplx<T>* vg = vbuf + (long long)r0 * vstride + f.idx_off;
  for (int e = tid; e < m * nr; e += 256) {
    const int r = e % m, k = e / m;
    vl[k][r] = r >= f.p ? x[(long long)(r0 + k) * N + id[r]] : vg[(long long)k * vstride + r];
  }
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int e = tid + 256 * u;
    Ui[0][e % NB][e / NB] = u0[u];
    Ui[1][e % NB][e / NB] = u1[u];
  }
  __syncthreads();
#pragma unroll
  for (int b = 1; b >= 0; --b) {  // compile-time b: uc stays in registers
    if (b >= nblk) continue;
    const int k0 = b * NB, kb = min(NB, f.p - k0), k1 = k0 + kb;
    cplx<T> acc[NR];
#pragma unroll
    for (int k = 0; k < NR; ++k) acc[k] = mk<T>(0, 0);
    chunked<TU * NR, (sizeof(T) == 8 && NR >= 4) ? 4 : 8>(
        [&](int q) {
          const int c = k1 + grp + G * (q / NR), k = q % NR;
          const cplx<T> v = vl[min(k, nr - 1)][min(c, m - 1)];
          return c < m && k < nr ? v : mk<T>(0, 0);
        },
        [&](int q, const cplx<T>& xv) { acc[q % NR] = cfma(acc[q % NR], uc[b][q / NR], xv); });
#pragma unroll
    for (int k = 0; k < NR; ++k) part[grp][k][j] = acc[k];
    __syncthreads();
    for (int e = tid; e < NR * NB; e += 256) {
      const int jj = e % NB, k = e / NB;
      cplx<T> s = part[0][k][jj];
      for (int g = 1; g < G; ++g) s = cadd(s, part[g][k][jj]);
      rb[k][jj] = (k < nr && jj < kb) ? csub(vl[k][k0 + jj], s) : mk<T>(0, 0);
    }
    __syncthreads();
    cplx<T> xs[NR];
    tri_apply<T, NR>(Ui[b], rb, tid, xs);
    const int i = tid / 8;
    if (tid % 8 == 0 && i < kb) {
#pragma unroll
      for (int k = 0; k < NR; ++k) {
        if (k < nr) {
          vl[k][k0 + i] = xs[k];
          x[(long long)(r0 + k) * N + (b ? gi1 : gi0)] = xs[k];
          if (xw) xw[(long long)(r0 + k) * N + (b ? gi1 : gi0)] = widen(xs[k]);
        }
      }
    }
    __syncthreads();
  }
}

// ---- Sweeps of the dense levels: the formed operators as matrix-vector
// products.  Workgroup (front, chunk of DR rows, right-hand-side group):
// thread (row tid % DR, column class tid / DR) sums the columns of its class
// (c = class mod DJ) for NR right-hand sides, the input staged through LDS
// DC columns at a time; the DJ class sums are added in class order, so a
// right-hand side's result does not depend on the group it is solved in.
constexpr int DR = 16, DJ = 256 / DR, DC = 256;

// Operator entries of the columns [c0, c0 + cn) of this thread's class for
// row r, stored column-major (ROWS false: entry (r, c) at c ld + r) or
// row-major (ROWS true: at r ld + c): DC / DJ loads per thread (clamped
// columns, multiplied only when in range), issued before the input is
// staged so that the two overlap.
constexpr int DU = DC / DJ;
template <typename T, bool ROWS>
__device__ __forceinline__ void dense_load(const cplx<T>* __restrict__ G, const long long ld, const int r,
                                           const int c0, const int cn, const int jg, cplx<T> (&g)[DU]) {
#pragma unroll
  for (int t = 0; t < DU; ++t) {
    const long long c = c0 + min(jg + DJ * t, cn - 1);
    g[t] = ROWS ? G[(long long)r * ld + c] : G[c * ld + r];
  }
}

// Partial products of the staged columns with the loaded entries.
template <typename T, int NR>
__device__ __forceinline__ void dense_chunk(const cplx<T> (&g)[DU], const int cn, const int jg,
                                            const cplx<T> (*vs)[DC], cplx<T> (&acc)[NR]) {
  constexpr int U = DU;
#pragma unroll
  for (int t = 0; t < U; ++t) {
    const int c = jg + DJ * t;
    if (c < cn)
#pragma unroll
      for (int k = 0; k < NR; ++k) acc[k] = cfma(acc[k], g[t], vs[k][c]);
  }
}

// Forward sweep of a dense level: out = [0; v_B] + Gf v_I with
// v = [z(I); 0] + children's updates, written where the panel chain writes
// its output (y_I in pivot order, then the updated v_B).
template <typename T, int NR>
__global__ void __launch_bounds__(256) fwd_dense_kernel(const cplx<T>* __restrict__ Gop, const FrontDev* __restrict__ fr,
                                                        const int* __restrict__ idx, const int* __restrict__ cpos,
                                                        const cplx<T>* __restrict__ z, cplx<T>* __restrict__ vbuf,
                                                        int first, int chunks, int nrhs, long long N, long long vstride) {
  __shared__ cplx<T> vs[NR][DC];
  __shared__ cplx<T> part[DJ][NR][DR];
  const FrontDev f = fr[first + blockIdx.x / chunks];
  const int m = f.p + f.q;
  const int row0 = (blockIdx.x % chunks) * DR;
  if (row0 >= m) return;  // the level's largest front sets the grid
  const int r0 = blockIdx.y * NR;
  const int nr = min(NR, nrhs - r0);
  const int tid = threadIdx.x, rl = tid % DR, jg = tid / DR;
  const int r = min(row0 + rl, m - 1);  // rows past m compute a copy of row m - 1, never stored
  const int* id = idx + f.idx_off;
  const int* cp = cpos + 2 * f.idx_off;
  const cplx<T>* G = Gop + f.g_off;
  // v at front row j (< p, or >= p without the z term) of right-hand side k
  auto vin = [&](const int j, const int k) {
    const long long rb = (long long)(r0 + k) * vstride;
    cplx<T> s = j < f.p ? z[(long long)(r0 + k) * N + id[j]] : mk<T>(0, 0);
    const int q0 = f.cidx[0] >= 0 ? cp[2 * j] : -1, q1 = f.cidx[1] >= 0 ? cp[2 * j + 1] : -1;
    if (q0 >= 0) s = cadd(s, vbuf[rb + f.cidx[0] + q0]);
    if (q1 >= 0) s = cadd(s, vbuf[rb + f.cidx[1] + q1]);
    return s;
  };
  cplx<T> acc[NR], g[DU];
#pragma unroll
  for (int k = 0; k < NR; ++k) acc[k] = mk<T>(0, 0);
  for (int c0 = 0; c0 < f.p; c0 += DC) {
    const int cn = min(DC, f.p - c0);
    if (c0 > 0) __syncthreads();  // the previous columns' reads are done
    dense_load<T, false>(G, m, r, c0, cn, jg, g);
    for (int e = tid; e < NR * DC; e += 256) {
      const int j = e % DC, k = e / DC;
      if (j < cn && k < nr) vs[k][j] = vin(c0 + j, k);
    }
    __syncthreads();
    dense_chunk<T, NR>(g, cn, jg, vs, acc);
  }
#pragma unroll
  for (int k = 0; k < NR; ++k) part[jg][k][rl] = acc[k];
  __syncthreads();
  if (tid < NR * DR) {
    const int k = tid / DR, rr = row0 + tid % DR;
    if (k < nr && rr < m) {
      cplx<T> s = part[0][k][tid % DR];
      for (int g = 1; g < DJ; ++g) s = cadd(s, part[g][k][tid % DR]);
      if (rr >= f.p) s = cadd(vin(rr, k), s);
      vbuf[(long long)(r0 + k) * vstride + f.idx_off + rr] = s;
    }
  }
}

// Backward sweep of a dense level: x_I = Gb [y_I; x_B], y_I from the
// forward sweep's output, x_B from the ancestors' solution; Gb is stored by
// rows (GbT column-major), so here a thread's column class is tid mod DJ
// and DJ consecutive lanes read one row's consecutive entries.
template <typename T, int NR>
__global__ void __launch_bounds__(256) bwd_dense_kernel(const cplx<T>* __restrict__ Gop, const FrontDev* __restrict__ fr,
                                                        const int* __restrict__ idx, cplx<T>* __restrict__ x,
                                                        const cplx<T>* __restrict__ vbuf, int first, int chunks,
                                                        int nrhs, long long N, long long vstride,
                                                        double2* __restrict__ xw) {
  __shared__ cplx<T> vs[NR][DC];
  __shared__ cplx<T> part[DJ][NR][DR];
  const FrontDev f = fr[first + blockIdx.x / chunks];
  const int m = f.p + f.q;
  const int row0 = (blockIdx.x % chunks) * DR;
  if (row0 >= f.p) return;  // the level's largest front sets the grid
  const int r0 = blockIdx.y * NR;
  const int nr = min(NR, nrhs - r0);
  const int tid = threadIdx.x, rl = tid / DJ, jg = tid % DJ;
  const int i = min(row0 + rl, f.p - 1);  // rows past p compute a copy of row p - 1, never stored
  const int* id = idx + f.idx_off;
  const cplx<T>* G = Gop + f.g_off + (long long)m * f.p;
  cplx<T> acc[NR], g[DU];
#pragma unroll
  for (int k = 0; k < NR; ++k) acc[k] = mk<T>(0, 0);
  for (int c0 = 0; c0 < m; c0 += DC) {
    const int cn = min(DC, m - c0);
    if (c0 > 0) __syncthreads();  // the previous columns' reads are done
    dense_load<T, true>(G, m, i, c0, cn, jg, g);
    for (int e = tid; e < NR * DC; e += 256) {
      const int j = e % DC, k = e / DC, c = c0 + j;
      if (j < cn && k < nr)
        vs[k][j] = c < f.p ? vbuf[(long long)(r0 + k) * vstride + f.idx_off + c] : x[(long long)(r0 + k) * N + id[c]];
    }
    __syncthreads();
    dense_chunk<T, NR>(g, cn, jg, vs, acc);
  }
#pragma unroll
  for (int k = 0; k < NR; ++k) part[jg][k][rl] = acc[k];
  __syncthreads();
  if (tid < NR * DR) {
    const int k = tid / DR, ii = row0 + tid % DR;
    if (k < nr && ii < f.p) {
      cplx<T> s = part[0][k][tid % DR];
      for (int g = 1; g < DJ; ++g) s = cadd(s, part[g][k][tid % DR]);
      x[(long long)(r0 + k) * N + id[ii]] = s;
      if (xw) xw[(long long)(r0 + k) * N + id[ii]] = widen(s);
    }
  }
}

inline bool wide_level(const Plan& plan, int l) { return plan.level_maxpq[l] > 256 + NB; }

constexpr size_t kLdsBytes = 160 * 1024;  // LDS of one workgroup on gfx950

// static LDS of the sweep kernels (inverse blocks, panel vectors, partial sums)
template <typename T, int NR, int TPB>
constexpr size_t fwd_static_lds() {
  return sizeof(cplx<T>) * (2 * NB * (NB + 1) + 2 * NR * NB);
}
template <typename T, int NR, int TPB>
constexpr size_t bwd_static_lds() {
  return sizeof(cplx<T>) * (2 * NB * (NB + 1) + (TPB / NB) * NR * NB + NR * NB);
}

// the front vectors go to LDS when they fit beside the static arrays
inline bool vec_in_lds(size_t vb, size_t stat) { return vb <= kVecLds && vb + stat <= kLdsBytes; }

// Levels whose fronts have more than 256 rows beside the first panel get
// 512-thread workgroups (a thread per row or column, all in flight at the
// panel start).  The choice depends on the level only, never on the number
// of right-hand sides, so a right-hand side's result does not depend on the
// group it is solved in.
template <typename T, int NR, int TPB>
void sweep_fwd(const MfDev<T>& mf, const Plan& plan, int l, int groups, int nrhs, const cplx<T>* z, cplx<T>* vbuf,
               hipStream_t st) {
  const int first = plan.level_ptr[l];
  const int cnt = plan.level_ptr[l + 1] - first;
  const size_t vb = (size_t)plan.level_maxpq[l] * NR * sizeof(cplx<T>);
  constexpr size_t stat = fwd_static_lds<T, NR, TPB>();
  static_assert(stat <= kLdsBytes, "sweep arrays exceed the LDS");
  if (vec_in_lds(vb, stat))
    LSP_LAUNCH("fwd", (int)sizeof(cplx<T>), (fwd_kernel<T, NR, true, TPB>), dim3(cnt, groups), dim3(TPB), vb, st,
               mf.F, mf.Dinv, mf.fronts, mf.idx, mf.cpos, mf.perm, z, vbuf, first, nrhs, (long long)plan.N,
               (long long)plan.sum_pq, mf.G);
  else
    LSP_LAUNCH("fwd", (int)sizeof(cplx<T>), (fwd_kernel<T, NR, false, TPB>), dim3(cnt, groups), dim3(TPB), 0, st,
               mf.F, mf.Dinv, mf.fronts, mf.idx, mf.cpos, mf.perm, z, vbuf, first, nrhs, (long long)plan.N,
               (long long)plan.sum_pq, mf.G);
}

template <typename T, int NR, int TPB>
void sweep_bwd(const MfDev<T>& mf, const Plan& plan, int l, int groups, int nrhs, cplx<T>* x, cplx<T>* vbuf,
               hipStream_t st, double2* xw) {
  const int first = plan.level_ptr[l];
  const int cnt = plan.level_ptr[l + 1] - first;
  const size_t vb = (size_t)plan.level_maxpq[l] * NR * sizeof(cplx<T>);
  constexpr size_t stat = bwd_static_lds<T, NR, TPB>();
  static_assert(stat <= kLdsBytes, "sweep arrays exceed the LDS");
  if (vec_in_lds(vb, stat))
    LSP_LAUNCH("bwd", (int)sizeof(cplx<T>), (bwd_kernel<T, NR, true, TPB>), dim3(cnt, groups), dim3(TPB), vb, st,
               mf.F, mf.Dinv, mf.fronts, mf.idx, x, vbuf, first, nrhs, (long long)plan.N, (long long)plan.sum_pq, xw);
  else
    LSP_LAUNCH("bwd", (int)sizeof(cplx<T>), (bwd_kernel<T, NR, false, TPB>), dim3(cnt, groups), dim3(TPB), 0, st,
               mf.F, mf.Dinv, mf.fronts, mf.idx, x, vbuf, first, nrhs, (long long)plan.N, (long long)plan.sum_pq, xw);
}


// The dense levels' sweeps: one workgroup per (front, DR rows, group).
template <typename T, int NR>
void dense_fwd(const MfDev<T>& mf, const Plan& plan, int l, int groups, int nrhs, const cplx<T>* z, cplx<T>* vbuf,
               hipStream_t st) {
  const int first = plan.level_ptr[l];
  const int cnt = plan.level_ptr[l + 1] - first;
  const int chunks = (plan.level_maxpq[l] + DR - 1) / DR;
  LSP_LAUNCH("fwd_dense", (int)sizeof(cplx<T>), (fwd_dense_kernel<T, NR>), dim3(cnt * chunks, groups), dim3(256), 0,
             st, mf.G, mf.fronts, mf.idx, mf.cpos, z, vbuf, first, chunks, nrhs, (long long)plan.N,
             (long long)plan.sum_pq);
}

template <typename T, int NR>
void dense_bwd(const MfDev<T>& mf, const Plan& plan, int l, int groups, int nrhs, cplx<T>* x, const cplx<T>* vbuf,
               hipStream_t st, double2* xw) {
  const int first = plan.level_ptr[l];
  const int cnt = plan.level_ptr[l + 1] - first;
  const int chunks = (plan.level_maxp[l] + DR - 1) / DR;
  LSP_LAUNCH("bwd_dense", (int)sizeof(cplx<T>), (bwd_dense_kernel<T, NR>), dim3(cnt * chunks, groups), dim3(256), 0,
             st, mf.G, mf.fronts, mf.idx, x, vbuf, first, chunks, nrhs, (long long)plan.N, (long long)plan.sum_pq, xw);
}

// Forms the sweep operators of dense level l from its factor: the forward
// chain and the transposed backward chain run on the unit vectors e_j,
// j < p, NF per workgroup.
template <typename T, int TPB>
void form_level(const MfDev<T>& mf, const Plan& plan, int l, hipStream_t st) {
  constexpr int NF = sizeof(T) == 4 ? 8 : 4;
  const int first = plan.level_ptr[l];
  const int cnt = plan.level_ptr[l + 1] - first;
  const int maxm = plan.level_maxpq[l], maxp = plan.level_maxp[l];
  const size_t vb = (size_t)maxm * NF * sizeof(cplx<T>);
  LSP_REQUIRE(vec_in_lds(vb, fwd_static_lds<T, NF, TPB>()), "dense sweep level exceeds the LDS");
  LSP_LAUNCH("form_fwd", (int)sizeof(cplx<T>), (fwd_kernel<T, NF, true, TPB, true, false>),
             dim3(cnt, (maxp + NF - 1) / NF), dim3(TPB), vb, st, mf.F, mf.Dinv, mf.fronts, mf.idx, mf.cpos, mf.perm,
             nullptr, nullptr, first, 0, (long long)plan.N, 0LL, mf.G);
  LSP_LAUNCH("form_bwd", (int)sizeof(cplx<T>), (fwd_kernel<T, NF, true, TPB, true, true>),
             dim3(cnt, (maxp + NF - 1) / NF), dim3(TPB), vb, st, mf.F, mf.Dinv, mf.fronts, mf.idx, mf.cpos, mf.perm,
             nullptr, nullptr, first, 0, (long long)plan.N, 0LL, mf.G);
}

// Formation of dense level l once its factorisation is enqueued on st.
template <typename T>
void form_after(const MfDev<T>& mf, const Plan& plan, int l, hipStream_t st, const FormStream* fs) {
  if (!plan.level_dense[l] && !plan.level_blocked[l]) return;
  hipStream_t fst = st;
  if (fs) {
    LSP_HIP(hipEventRecord(fs->level, st));
    LSP_HIP(hipStreamWaitEvent(fs->aux, fs->level, 0));
    fst = fs->aux;
  }
  if (plan.level_blocked[l]) blocked_form<T>(mf, plan, l, fst);
  else if (wide_level(plan, l)) form_level<T, 512>(mf, plan, l, fst);
  else form_level<T, 256>(mf, plan, l, fst);
}

template <typename T, int NR>
void solve_levels(const MfDev<T>& mf, const Plan& plan, int nrhs, const cplx<T>* z, cplx<T>* x, cplx<T>* vbuf,
                  const SweepBufs<T>& sb, hipStream_t st, hipEvent_t form_done, double2* xw) {
  const int groups = (nrhs + NR - 1) / NR;
  for (int l = 0; l < plan.nlevels; ++l) {
    if ((plan.level_dense[l] || plan.level_blocked[l]) && form_done) {
      LSP_HIP(hipStreamWaitEvent(st, form_done, 0));
      form_done = nullptr;
    }
    if (plan.level_mchain[l]) {
      mchain_sweep<T>(true, mf, plan, l, nrhs, z, x, vbuf, st, xw, sb.xpm);
      continue;
    }
    if constexpr (NR == 1) {
      if (plan.level_small_sweep[l]) {
        LSP_LAUNCH("fwd", (int)sizeof(cplx<T>), (fwd_small_kernel<T, NR>),
                   dim3(plan.level_ptr[l + 1] - plan.level_ptr[l], groups), dim3(256), 0, st, mf.F, mf.Dinv, mf.fronts,
                   mf.idx, mf.cpos, mf.perm, z, vbuf, plan.level_ptr[l], nrhs, (long long)plan.N,
                   (long long)plan.sum_pq);
        continue;
      }
    }
    if (plan.level_blocked[l]) blocked_sweep<T>(true, mf, plan, l, nrhs, z, x, vbuf, sb, st, xw);
    else if (plan.level_dense[l]) dense_fwd<T, NR>(mf, plan, l, groups, nrhs, z, vbuf, st);
    else if (wide_level(plan, l)) sweep_fwd<T, NR, 512>(mf, plan, l, groups, nrhs, z, vbuf, st);
    else sweep_fwd<T, NR, 256>(mf, plan, l, groups, nrhs, z, vbuf, st);
  }
  // the matrix-core levels gather their boundary rows from xpm: the levels
  // swept by other kernels since the last matrix-core one (from unconv_top
  // down) have their pivots copied there first
  int unconv_top = -1;
  for (int l = plan.nlevels - 1; l >= 0; --l) {
    if (plan.level_mchain[l]) {
      if (unconv_top >= 0) launch_point_major<T>(mf, plan, l + 1, unconv_top + 1, x, sb.xpm, nrhs, st);
      unconv_top = -1;
      mchain_sweep<T>(false, mf, plan, l, nrhs, z, x, vbuf, st, xw, sb.xpm);
      continue;
    }
    if (unconv_top < 0) unconv_top = l;
    if constexpr (sizeof(T) == 4 && NR == 1) {
      if (plan.level_small_sweep[l]) {
        LSP_LAUNCH("bwd", (int)sizeof(cplx<T>), (bwd_small_kernel<T, NR>),
                   dim3(plan.level_ptr[l + 1] - plan.level_ptr[l], groups), dim3(256), 0, st, mf.F, mf.Dinv, mf.fronts,
                   mf.idx, x, vbuf, plan.level_ptr[l], nrhs, (long long)plan.N, (long long)plan.sum_pq, xw);
        continue;
      }
    }
    if (plan.level_blocked[l]) blocked_sweep<T>(false, mf, plan, l, nrhs, z, x, vbuf, sb, st, xw);
    else if (plan.level_dense[l]) dense_bwd<T, NR>(mf, plan, l, groups, nrhs, x, vbuf, st, xw);
    else if (wide_level(plan, l)) sweep_bwd<T, NR, 512>(mf, plan, l, groups, nrhs, x, vbuf, st, xw);
    else sweep_bwd<T, NR, 256>(mf, plan, l, groups, nrhs, x, vbuf, st, xw);
  }
}

}  // namespace

// Trailing update of panel k0 over tiles of TM; with FUSE (see fuse_next)
// also the next panel's diagonal-block factorisation (one extra block row).
template <typename T, int TM>
void update_launch(const MfDev<T>& mf, bool fuse, int rem, int cnt, int first, int k0, hipStream_t st) {
  const int gt = (rem + TM - 1) / TM;
  if (fuse)
    LSP_LAUNCH("update_lu", (int)sizeof(cplx<T>), (gemm_update_kernel<T, TM, true>), dim3(gt, gt + 1, cnt), dim3(256),
               0, st, mf.F, mf.fronts, first, k0, mf.Dinv, mf.perm, mf.pivstat);
  else
    LSP_LAUNCH("gemm_update", (int)sizeof(cplx<T>), (gemm_update_kernel<T, TM, false>), dim3(gt, gt, cnt), dim3(256),
               0, st, mf.F, mf.fronts, first, k0, mf.Dinv, mf.perm, mf.pivstat);
}

// trailing-update tile of level l (complex128 128-wide tiles would need more
// than 256 VGPRs; 64 there)
static int update_tile(const Plan& plan, int l, bool fp64) {
  return (fp64 && plan.level_tile[l] == 128) ? 64 : plan.level_tile[l];
}

// Whether panel k0's trailing update of level l also factors the next
// panel's diagonal block: when some front has a next panel and the update
// has few enough tiles that every workgroup of the launch is resident at
// once (the fused kernel carries the factorisation's register count, so its
// tiles run at low occupancy).
static bool fuse_next(const Plan& plan, int l, int k0, bool fp64) {
  const int cnt = plan.level_ptr[l + 1] - plan.level_ptr[l];
  if (k0 + NB >= plan.level_maxp[l]) return false;
  const int rem = plan.level_maxpq[l] - k0 - 1;  // > NB when a next panel exists
  const int tile = update_tile(plan, l, fp64);
  const long long gt = (rem + tile - 1) / tile;
  return cnt * gt * gt <= 256;
}

// Whether level l runs one launch per panel step (strip workgroups, see
// panel_step_kernel): complex64 factors (the complex128 strip workgroup
// would spill registers), and every workgroup of the level's largest step
// (the first: gt^2 tiles and 2 nch strip chunks per front) resident at once.
static bool strip_level(const Plan& plan, int l, bool fp64) {
  if (fp64) return false;
  const long long cnt = plan.level_ptr[l + 1] - plan.level_ptr[l];
  const int maxm = plan.level_maxpq[l];
  const int tile = update_tile(plan, l, fp64);
  const long long gt = (maxm - 1 + tile - 1) / tile;
  const long long nch = (maxm - 1 + NB - 1) / NB;
  return cnt * (gt * gt + 2 * nch) <= 256;
}

// Whether level l runs the two-panel schedule (cross_update_kernel,
// pair_update_kernel): levels of separate launches per panel (not strip
// levels) whose fronts reach 512 rows.
static bool pair_level(const Plan& plan, int l, bool fp64) {
  return !strip_level(plan, l, fp64) && plan.level_maxpq[l] >= 512;
}

template <typename T>
void diag_launch(const MfDev<T>& mf, int cnt, int first, int k0, hipStream_t st) {
  if (cnt > 512)  // more than two fronts per CU
    LSP_LAUNCH("diag_lu", (int)sizeof(cplx<T>), (diag_lu_kernel<T, 64>), dim3(cnt), dim3(64), 0, st, mf.F, mf.Dinv,
               mf.fronts, mf.perm, mf.pivstat, first, k0);
  else
    LSP_LAUNCH("diag_lu", (int)sizeof(cplx<T>), (diag_lu_kernel<T, 256>), dim3(cnt), dim3(256), 0, st, mf.F, mf.Dinv,
               mf.fronts, mf.perm, mf.pivstat, first, k0);
}

// both panels' update of [k0 + kb, m)^2 (rem = the largest m - k0 - 1)
template <typename T, int TM>
void pair_launch(const MfDev<T>& mf, int rem, int cnt, int first, int k0, hipStream_t st) {
  const int gt = (rem + TM - 1) / TM;
  LSP_LAUNCH("pair_update", (int)sizeof(cplx<T>), (pair_update_kernel<T, TM>), dim3(gt, gt, cnt), dim3(256), 0, st,
             mf.F, mf.fronts, first, k0);
}

// Panel step k0 of a strip level (a later panel exists in some front):
// grid row 0 the strip chunks of the next panel, rows 1.. the update tiles.
template <typename T, int TM>
void step_launch(const MfDev<T>& mf, int rem, int maxm, int cnt, int first, int k0, hipStream_t st) {
  const int gt = (rem + TM - 1) / TM;
  const int nch = (std::max(0, maxm - k0 - NB - 1) + NB - 1) / NB;  // chunks of the largest next panel
  LSP_LAUNCH("panel_step", (int)sizeof(cplx<T>), (panel_step_kernel<T, TM>), dim3(std::max(gt, std::max(1, 2 * nch)), gt + 1, cnt),
             dim3(256), 0, st, mf.F, mf.fronts, first, k0, mf.Dinv, mf.perm, mf.pivstat);
}

// the levels' factorisation launches on st, each dense level's formation
// after its own (on fs->aux when given)
template <typename T>
void mf_factor_levels(const MfDev<T>& mf, const Plan& plan, hipStream_t st, const FormStream* fs);

template <typename T>
void mf_factor(const MfDev<T>& mf, const Plan& plan, hipStream_t st, const FormStream* fs) {
  if (fs) LSP_HIP(hipStreamWaitEvent(st, fs->done, 0));  // the previous formation reads the factors
  try {
    mf_factor_levels(mf, plan, st, fs);
  } catch (...) {
    if (fs) (void)hipEventRecord(fs->done, fs->aux);  // covers whatever formation was enqueued
    throw;
  }
  if (fs) LSP_HIP(hipEventRecord(fs->done, fs->aux));
}

template <typename T>
void mf_factor_levels(const MfDev<T>& mf, const Plan& plan, hipStream_t st, const FormStream* fs) {
  for (int l = 0; l < plan.nlevels; ++l) {
    if (l > 0) form_after(mf, plan, l - 1, st, fs);
    const int first = plan.level_ptr[l];
    const int cnt = plan.level_ptr[l + 1] - first;
    const int maxm = plan.level_maxpq[l];
    const int maxp = plan.level_maxp[l];
    long long mm = (long long)maxm * maxm;
    // four entries per thread and step; about 8192 workgroups over the level
    int gx = (int)std::min<long long>((mm + 1023) / 1024, std::max(1, 8192 / cnt));
    LSP_LAUNCH("assemble_front", (int)sizeof(cplx<T>), assemble_front_kernel<T>, dim3(gx, cnt), dim3(256), 0, st, mf.F,
               mf.fronts, mf.idx, mf.gpos, mf.cpos, mf.Mval, first, plan.d);
    const bool fp64 = sizeof(T) == 8;
    if constexpr (sizeof(T) == 4) {
    if (strip_level(plan, l, fp64)) {
      const int nch0 = (maxm - 1 + NB - 1) / NB;
      LSP_LAUNCH("strip_first", (int)sizeof(cplx<T>), strip_first_kernel<T>, dim3(std::max(1, 2 * nch0), cnt),
                 dim3(256), 0, st, mf.F, mf.fronts, first, mf.Dinv, mf.perm, mf.pivstat);
      for (int k0 = 0; k0 < maxp; k0 += NB) {
        const int rem = maxm - k0 - 1;
        if (rem <= 0) continue;
        const int tile = update_tile(plan, l, fp64);
        const bool next = k0 + NB < maxp;
        if (tile == 32) {
          if (next) step_launch<T, 32>(mf, rem, maxm, cnt, first, k0, st);
          else update_launch<T, 32>(mf, false, rem, cnt, first, k0, st);
        } else if (tile == 128) {
          if (next) step_launch<T, 128>(mf, rem, maxm, cnt, first, k0, st);
          else update_launch<T, 128>(mf, false, rem, cnt, first, k0, st);
        } else {
          if (next) step_launch<T, 64>(mf, rem, maxm, cnt, first, k0, st);
          else update_launch<T, 64>(mf, false, rem, cnt, first, k0, st);
        }
      }
      continue;
    }
    }
    if (pair_level(plan, l, fp64)) {
      const int tile = update_tile(plan, l, fp64);
      for (int k0 = 0; k0 < maxp; k0 += 2 * NB) {
        diag_launch(mf, cnt, first, k0, st);
        const int rem = maxm - k0 - 1;
        if (rem <= 0) continue;
        LSP_LAUNCH("panel_trsm", (int)sizeof(cplx<T>), panel_trsm_kernel<T>, dim3((rem + 63) / 64, cnt, 2), dim3(256),
                   0, st, mf.F, mf.Dinv, mf.fronts, mf.perm, first, k0);
        if (k0 + NB < maxp) {  // some front has a panel b
          LSP_LAUNCH("cross_update", (int)sizeof(cplx<T>), cross_update_kernel<T>,
                     dim3((maxm - k0 - NB + 31) / 32, 3, cnt), dim3(256), 0, st, mf.F, mf.fronts, first, k0, mf.Dinv,
                     mf.perm, mf.pivstat);
          const int rem2 = maxm - k0 - NB - 1;
          if (rem2 > 0)
            LSP_LAUNCH("panel_trsm", (int)sizeof(cplx<T>), panel_trsm_kernel<T>, dim3((rem2 + 63) / 64, cnt, 2),
                       dim3(256), 0, st, mf.F, mf.Dinv, mf.fronts, mf.perm, first, k0 + NB);
        }
        if (tile == 128) {
          if constexpr (sizeof(T) == 4) pair_launch<T, 128>(mf, rem, cnt, first, k0, st);
        } else if (tile == 64) {
          pair_launch<T, 64>(mf, rem, cnt, first, k0, st);
        } else {
          pair_launch<T, 32>(mf, rem, cnt, first, k0, st);
        }
      }
      continue;
    }
    bool factored = false;  // panel k0's diagonal block done by the previous update
    for (int k0 = 0; k0 < maxp; k0 += NB) {
      if (!factored) {
        if (cnt > 512)  // more than two fronts per CU
          LSP_LAUNCH("diag_lu", (int)sizeof(cplx<T>), (diag_lu_kernel<T, 64>), dim3(cnt), dim3(64), 0, st, mf.F,
                     mf.Dinv, mf.fronts, mf.perm, mf.pivstat, first, k0);
        else
          LSP_LAUNCH("diag_lu", (int)sizeof(cplx<T>), (diag_lu_kernel<T, 256>), dim3(cnt), dim3(256), 0, st, mf.F,
                     mf.Dinv, mf.fronts, mf.perm, mf.pivstat, first, k0);
      }
      const int rem = maxm - k0 - 1;
      if (rem <= 0) continue;
      const int tiles = (rem + 63) / 64;
      LSP_LAUNCH("panel_trsm", (int)sizeof(cplx<T>), panel_trsm_kernel<T>, dim3(tiles, cnt, 2), dim3(256), 0, st, mf.F,
                 mf.Dinv, mf.fronts, mf.perm, first, k0);
      const int tile = update_tile(plan, l, fp64);
      factored = fuse_next(plan, l, k0, fp64);
      if (tile == 32) update_launch<T, 32>(mf, factored, rem, cnt, first, k0, st);
      else if (tile == 128) {
        if constexpr (sizeof(T) == 4) update_launch<T, 128>(mf, factored, rem, cnt, first, k0, st);
      }
      else update_launch<T, 64>(mf, factored, rem, cnt, first, k0, st);
    }
  }
  form_after(mf, plan, plan.nlevels - 1, st, fs);
}

FactorSchedule factor_schedule(const Plan& plan, bool fp64) {
  FactorSchedule s;
  for (int l = 0; l < plan.nlevels; ++l) {
    const bool strips = strip_level(plan, l, fp64);
    if (!strips)  // U12 = L11^{-1} P F12 and L21 = F21 U11^{-1}: 2 kb^2 (m - k1) complex multiply-adds per panel
      for (int i = plan.level_ptr[l]; i < plan.level_ptr[l + 1]; ++i) {
        const FrontDev& f = plan.fronts[i];
        for (int k0 = 0; k0 < f.p; k0 += NB) {
          const int kb = std::min(NB, f.p - k0);
          s.trsm_flops += 8.0 * 2.0 * (double)kb * kb * (double)(f.p + f.q - k0 - kb);
        }
      }
    if (pair_level(plan, l, fp64)) {
      // rank-kb products over [k0 + kb, m)^2 (kb = both panels' columns),
      // and panel a's rank-32 update of panel b's column and row strips
      for (int i = plan.level_ptr[l]; i < plan.level_ptr[l + 1]; ++i) {
        const FrontDev& f = plan.fronts[i];
        const double m = (double)(f.p + f.q);
        for (int k0 = 0; k0 < f.p; k0 += 2 * NB) {
          const int kb = std::min(2 * NB, f.p - k0);
          s.pair_update_flops += 8.0 * (m - k0 - kb) * (m - k0 - kb) * kb;
          if (f.p > k0 + NB) {
            const int kbb = std::min(NB, f.p - k0 - NB);
            s.cross_update_flops += 8.0 * NB * kbb * (2.0 * (m - k0 - NB) - kbb);
            s.fused_blocks += 1.0;  // panel b's block, factored by the cross launch
          }
        }
      }
      continue;
    }
    for (int k0 = 0; k0 < plan.level_maxp[l]; k0 += NB) {
      // update launches other than gemm_update: the panel steps of a strip
      // level (all but the last panel) and the lookahead launches
      const bool step = strips ? k0 + NB < plan.level_maxp[l]
                               : (!pair_level(plan, l, fp64) && fuse_next(plan, l, k0, fp64));
      for (int i = plan.level_ptr[l]; i < plan.level_ptr[l + 1]; ++i) {
        const FrontDev& f = plan.fronts[i];
        if (f.p <= k0) continue;
        const int kb = std::min(NB, f.p - k0);
        const double rem = (double)(f.p + f.q - k0 - kb);
        if (strips && k0 == 0) s.fused_blocks += 1.0;  // panel 0 in the first strip launch
        if (!step) continue;
        s.fused_update_flops += 8.0 * rem * rem * kb;
        if (f.p > k0 + kb) s.fused_blocks += 1.0;
      }
    }
  }
  return s;
}

template <typename T>
void mf_solve(const MfDev<T>& mf, const Plan& plan, int nrhs, const cplx<T>* z, cplx<T>* x, cplx<T>* vbuf,
              const SweepBufs<T>& sb, hipStream_t st, hipEvent_t form_done, double2* xw) {
  // groups of at most 8 right-hand sides on the panel-chain levels (16 per
  // workgroup halves the workgroups and their occupancy: measured slower on
  // 2D n = 1024); the blocked levels take up to 16 per product
  if (nrhs >= 8) solve_levels<T, 8>(mf, plan, nrhs, z, x, vbuf, sb, st, form_done, xw);
  else if (nrhs >= 4) solve_levels<T, 4>(mf, plan, nrhs, z, x, vbuf, sb, st, form_done, xw);
  else if (nrhs >= 2) solve_levels<T, 2>(mf, plan, nrhs, z, x, vbuf, sb, st, form_done, xw);
  else solve_levels<T, 1>(mf, plan, nrhs, z, x, vbuf, sb, st, form_done, xw);
}

template void mf_factor<double>(const MfDev<double>&, const Plan&, hipStream_t, const FormStream*);
template void mf_factor<float>(const MfDev<float>&, const Plan&, hipStream_t, const FormStream*);
template void mf_solve<double>(const MfDev<double>&, const Plan&, int, const double2*, double2*, double2*,
                               const SweepBufs<double>&, hipStream_t, hipEvent_t, double2*);
template void mf_solve<float>(const MfDev<float>&, const Plan&, int, const float2*, float2*, float2*,
                              const SweepBufs<float>&, hipStream_t, hipEvent_t, double2*);

}  // namespace lsp
