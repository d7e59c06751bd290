// Sparsifying stencils (Section 2.2 and Section 3.1).
//
// For each of the 3^d position classes c the stencil alpha_c is the unit row
// vector minimising ||alpha X_c||, X_c = K(mu_c(0), F_c) (eq:Fmin, eq:Emin,
// eq:Cmin, and the 3D interior / face / edge / corner sets), i.e. the
// conjugate of the least left singular vector of X_c.  X_c has at most 27
// rows and up to (2n-1)^d columns, generated on the fly from the |t| kernel
// table.  It is reduced in two streamed passes:
//   pass 1: G = X X^H (per-block partial sums, reduced in a fixed order),
//           Jacobi eigen-decomposition G = U1 diag U1^H;
//   pass 2: G2 = (U1^H X)(U1^H X)^H, which is nearly diagonal so the rounding
//           of each entry is relative to its own eigenvalue; Jacobi again
//           gives U2, and U = U1 U2.
// Pass 2 restores full relative accuracy of the smallest singular value,
// which a single Gram pass loses (sigma_min / sigma_max is about 1e-5 .. 1e-3
// at eight points per wavelength).  sigma_k = sqrt(lambda_k).
// Normalisation (a reading: the paper fixes alpha only up to a unit scalar):
// ||alpha|| = 1 and the centre (offset 0) entry real and positive.
//
// Then C_c = alpha_c K(mu_c, mu_c) (Section 2.2), the Q apply (eq:PC) and
// the stencil matrix M = [A + C w^2 m; B] (eq:ABop), stored as [N][3^d].
#include "lsp_common.h"
#include "kernels.h"

namespace lsp {

namespace {

constexpr int S = kMaxStencil;  // padded stencil / matrix order
constexpr int CH = 48;          // far-set columns staged per step

__device__ inline long long ktab_index(int t0, int t1, int t2, int n, int d) {
  long long n1 = n + 1;
  long long r = t0 + n1 * t1;
  if (d == 3) r += n1 * n1 * t2;
  return r;
}

template <bool PASS2>
__global__ void __launch_bounds__(256) gram_kernel(const double2* __restrict__ ktab, int n, int d,
                                                   const ClassGeom* __restrict__ geo,
                                                   const double2* __restrict__ U1, double2* __restrict__ partial,
                                                   int nblk) {
  __shared__ double2 X[S][CH + 1];
  __shared__ double2 Z[PASS2 ? S : 1][CH + 1];
  __shared__ double2 Us[PASS2 ? S * S : 1];
  const int c = blockIdx.y, blk = blockIdx.x, tid = threadIdx.x;
  const ClassGeom& g = geo[c];
  __shared__ int soff[S][3];
  for (int e = tid; e < S * 3; e += blockDim.x) soff[e / 3][e % 3] = g.off[e / 3][e % 3];
  const int s = g.s;
  const long long F = g.F;
  const int flo[3] = {g.flo[0], g.flo[1], g.flo[2]};
  const int fsz[3] = {g.fsz[0], g.fsz[1], g.fsz[2]};
  const int interior = g.interior;
  const long long j0 = F * blk / nblk, j1 = F * (blk + 1) / nblk;
  if (PASS2) {
    for (int e = tid; e < S * S; e += blockDim.x) Us[e] = U1[(long long)c * S * S + e];
  }
  // thread -> (pair, column group): small classes (few pairs) split the
  // staged columns over several groups so that every thread accumulates
  const int npairs = s * (s + 1) / 2;
  const int G = npairs <= 128 ? 256 / npairs : 1;
  const int per = npairs <= 128 ? 1 : 2;
  int pa[2] = {0, 0}, pb[2] = {0, 0};
  bool own[2] = {false, false};
  const int grp = npairs <= 128 ? tid / npairs : 0;
  double2 acc[2] = {make_double2(0, 0), make_double2(0, 0)};
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    if (k >= per) break;
    int p = npairs <= 128 ? tid % npairs : tid + k * blockDim.x;
    if (p < npairs && grp < G) {
      int a = 0, rem = p;
      while (rem >= s - a) { rem -= s - a; ++a; }
      pa[k] = a; pb[k] = a + rem; own[k] = true;
    }
  }
  // Chunks of CHs columns: the staging arrays hold S (CH + 1) entries, used
  // as s rows of stride ld = CHs + 1, so classes with few rows take wider
  // chunks (fewer memory round trips per block).  The next chunk's table
  // entries are loaded while the current one is reduced.  Thread tid stages
  // entries e = tid + 256u (row ea = e / CHs, column ej = e % CHs, both fixed
  // across chunks); the far-set coordinates of column base + ej are kept as
  // mixed-radix digits and advanced by CHs per chunk (no divisions in the
  // loop).  Entries outside the block's range load table entry 0 and are zeroed.
  const int ld = (S * (CH + 1)) / s;
  const int CHs = ld - 1;
  double2* Xf = &X[0][0];
  double2* Zf = &Z[0][0];
  constexpr int EPT = (S * (CH + 1) + 255) / 256;
  int ea[EPT], ej[EPT];
  int dig[EPT][3];
#pragma unroll
  for (int u = 0; u < EPT; ++u) {
    const int e = tid + 256 * u;
    ea[u] = min(e / CHs, s - 1);
    ej[u] = e % CHs;
    unsigned rem = (unsigned)(j0 + ej[u]);
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) {
      dig[u][ax] = ax < d ? (int)(rem % (unsigned)fsz[ax]) : 0;
      if (ax < d) rem /= (unsigned)fsz[ax];
    }
  }
  auto fetch = [&](long long base, double2 (&v)[EPT]) {
#pragma unroll
    for (int u = 0; u < EPT; ++u) {
      const int e = tid + 256 * u;
      const int a = ea[u];
      const bool valid = e < s * CHs && base + ej[u] < j1;
      int t[3] = {0, 0, 0};
      bool near = true;
#pragma unroll
      for (int ax = 0; ax < 3; ++ax) {
        if (ax < d) {
          const int j = flo[ax] + dig[u][ax];
          near = near && (j >= -1 && j <= 1);
          t[ax] = abs(soff[a][ax] - j);
        }
      }
      const double2 kv = ktab[valid ? ktab_index(t[0], t[1], t[2], n, d) : 0];
      v[u] = valid && !(interior && near) ? kv : make_double2(0, 0);
      // advance to the same column of the next chunk
      dig[u][0] += CHs;
#pragma unroll
      for (int ax = 0; ax < 2; ++ax) {
        if (ax + 1 < d) {
          while (dig[u][ax] >= fsz[ax]) { dig[u][ax] -= fsz[ax]; ++dig[u][ax + 1]; }
        }
      }
    }
  };
  double2 vnext[EPT];
  __syncthreads();  // soff staged
  if (j0 < j1) fetch(j0, vnext);  // (an empty block range loads nothing)
  for (long long base = j0; base < j1; base += CHs) {
    __syncthreads();
#pragma unroll
    for (int u = 0; u < EPT; ++u) {
      const int e = tid + 256 * u;
      if (e < s * CHs) Xf[ea[u] * ld + ej[u]] = vnext[u];
    }
    if (base + CHs < j1) fetch(base + CHs, vnext);
    __syncthreads();
    if (PASS2) {
      // Z = U1^H X, three rows of Z per thread so that each staged entry of
      // X is read once for three products (rows past s are computed from
      // U1's padding and not stored); each entry's sum runs over a in order
      const int nk3 = (s + 2) / 3;
      for (int e = tid; e < nk3 * CHs; e += blockDim.x) {
        const int k = 3 * (e / CHs), jj = e % CHs;
        double2 z0 = make_double2(0, 0), z1 = z0, z2 = z0;
        for (int a = 0; a < s; ++a) {
          const double2 xa = Xf[a * ld + jj];
          z0 = cadd(z0, cmulc(Us[a + S * k], xa));
          z1 = cadd(z1, cmulc(Us[a + S * min(k + 1, S - 1)], xa));
          z2 = cadd(z2, cmulc(Us[a + S * min(k + 2, S - 1)], xa));
        }
        Zf[k * ld + jj] = z0;
        if (k + 1 < s) Zf[(k + 1) * ld + jj] = z1;
        if (k + 2 < s) Zf[(k + 2) * ld + jj] = z2;
      }
      __syncthreads();
    }
    const double2* Yf = PASS2 ? Zf : Xf;
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      if (k >= per || !own[k]) continue;
      double2 sum = acc[k];
      for (int jj = grp; jj < CHs; jj += G) {
        const double2 u = Yf[pa[k] * ld + jj];
        const double2 w = Yf[pb[k] * ld + jj];
        sum = cadd(sum, cmulc(w, u));  // u * conj(w)
      }
      acc[k] = sum;
    }
  }
  // reduce the column groups in a fixed order
  __syncthreads();
  double2* red = Xf;  // reuse the staging buffer: G x npairs <= 256 entries
  if (npairs <= 128) {
    if (own[0]) red[grp * npairs + (tid % npairs)] = acc[0];
    __syncthreads();
    if (tid < npairs) {
      double2 sum = red[tid];
      for (int q = 1; q < G; ++q) sum = cadd(sum, red[q * npairs + tid]);
      acc[0] = sum;
    }
  }
  double2* out = partial + ((long long)blk * gridDim.y + c) * S * S;
  const bool writer = npairs <= 128 ? tid < npairs : true;
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    if (k >= per || !own[k] || !writer) continue;
    out[pa[k] + S * pb[k]] = acc[k];
    out[pb[k] + S * pa[k]] = cconj(acc[k]);
  }
}

// G_c = sum over blocks of the partial Gram matrices, for the s x s entries
// of class c only (zero elsewhere).  Thread t works on entry t % s^2 and
// block slice t / s^2 (every slices-th block, eight loads in flight); the
// slice sums are added in slice order.
__global__ void __launch_bounds__(768) gram_reduce_kernel(const double2* __restrict__ partial,
                                                          double2* __restrict__ G, int nblk, int nclass,
                                                          const ClassGeom* __restrict__ geo) {
  __shared__ double2 red[768];
  const int c = blockIdx.x, t = threadIdx.x;
  const int s = geo[c].s;
  const int ne = s * s;
  const int slices = max(1, (int)blockDim.x / ne);
  const int e = t % ne, sl = t / ne;
  const int off = (e % s) + S * (e / s);
  double2 acc = make_double2(0, 0);
  if (sl < slices) {
    for (int b0 = sl; b0 < nblk; b0 += 8 * slices) {
      double2 v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int b = b0 + u * slices;
        v[u] = b < nblk ? partial[((long long)b * nclass + c) * S * S + off] : make_double2(0, 0);
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) acc = cadd(acc, v[u]);
    }
  }
  red[t] = acc;
  __syncthreads();
  if (t < ne) {
    double2 sum = red[t];
    for (int q = 1; q < slices; ++q) sum = cadd(sum, red[q * ne + t]);
    G[(long long)c * S * S + off] = sum;
  }
  for (int z = t; z < S * S; z += blockDim.x)
    if (z % S >= s || z / S >= s) G[(long long)c * S * S + z] = make_double2(0, 0);
}

// Parallel cyclic Jacobi on an s x s Hermitian matrix by one workgroup (the
// class stencils: 256 threads per class, the boundary points of a general
// domain: one wave per point); the first s'/2 threads compute a round's
// rotations, all threads share its column and row updates (each entry's
// arithmetic is the same whichever thread does it).  A and U are
// column-major with leading dimension S.  A sweep is
// s' - 1 rounds (s' = s rounded up to even) of s'/2 disjoint pairs in the
// round-robin order (position 0 fixed, the others shifted by the round; the
// index s, when s is odd, is a dummy that pairs with nobody), all rotated
// at once: their parameters come from A before the round, the column update
// A V and U V touches disjoint column pairs, the row update V^H (A V)
// disjoint row pairs.  Rotation of (p, q): with g = A(p,q) = |g| e^{i phi},
// tau = (A(q,q) - A(p,p)) / (2|g|), t = sign(tau) / (|tau| + sqrt(1 + tau^2)),
// c = 1/sqrt(1+t^2), s = t c, V = [[c, s], [-s e^{-i phi}, c e^{-i phi}]].
// A pair is skipped when |g| <= 1e-17 sqrt(A(p,p) A(q,q)) (relative
// criterion, compared squared); the sweeps stop when a whole sweep rotates
// nothing.
// 1 / sqrt(x), x > 0: the hardware estimate refined by two Newton steps
// r <- r (3 - x r^2) / 2 (each roughly doubles the correct bits).
__device__ __forceinline__ double rsqrt_nr(double x) {
  double r = __builtin_amdgcn_rsq(x);
  r = r * fma(-0.5 * x, r * r, 1.5);
  r = r * fma(-0.5 * x, r * r, 1.5);
  return r;
}

__device__ void jacobi_eigen(double2* A, double2* U, int s, int lane) {
  constexpr int NP = (S + 1) / 2;
  __shared__ int rotated;
  __shared__ int rp[NP], rq[NP], ract[NP];
  __shared__ double rcs[NP], rsn[NP];
  __shared__ double2 rv10[NP], rv11[NP];
  const int sp = s + (s & 1);
  const int npair = sp / 2;
  for (int sweep = 0; sweep < 40; ++sweep) {
    if (lane == 0) rotated = 0;
    __syncthreads();
    for (int r = 0; r < sp - 1; ++r) {
      if (lane < npair) {
        auto who = [&](int pos) { return pos == 0 ? 0 : 1 + (pos - 1 + r) % (sp - 1); };
        int p = who(lane), q = who(sp - 1 - lane);
        if (p > q) { const int t = p; p = q; q = t; }
        int act = 0;
        if (q < s) {
          const double2 gpq = A[p + S * q];
          const double a = A[p + S * p].x, b = A[q + S * q].x;
          const double ag2 = gpq.x * gpq.x + gpq.y * gpq.y;  // |g|^2
          if (ag2 > 1e-34 * fabs(a * b) && ag2 != 0.0) {
            const double ri = rsqrt_nr(ag2);                 // 1 / |g|
            const double ex = gpq.x * ri, ey = gpq.y * ri;  // e^{i phi}
            const double tau = (b - a) * 0.5 * ri;
            const double t = (tau >= 0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
            const double cs = rsqrt_nr(1.0 + t * t), sn = t * cs;
            rcs[lane] = cs;
            rsn[lane] = sn;
            rv10[lane] = make_double2(-sn * ex, sn * ey);  // -s e^{-i phi}
            rv11[lane] = make_double2(cs * ex, -cs * ey);  //  c e^{-i phi}
            act = 1;
            rotated = 1;
          }
        }
        rp[lane] = p;
        rq[lane] = q;
        ract[lane] = act;
      }
      __syncthreads();
      // columns: A(:,p) <- c A(:,p) + v10 A(:,q);  A(:,q) <- s A(:,p) + v11 A(:,q); same for U
      for (int it = lane; it < npair * s; it += blockDim.x) {
        const int k = it / s, i = it % s;
        if (!ract[k]) continue;
        const int p = rp[k], q = rq[k];
        const double cs = rcs[k], sn = rsn[k];
        const double2 v10 = rv10[k], v11 = rv11[k];
        const double2 xp = A[i + S * p], xq = A[i + S * q];
        A[i + S * p] = cadd(cscale(xp, cs), cmul(v10, xq));
        A[i + S * q] = cadd(cscale(xp, sn), cmul(v11, xq));
        const double2 up = U[i + S * p], uq = U[i + S * q];
        U[i + S * p] = cadd(cscale(up, cs), cmul(v10, uq));
        U[i + S * q] = cadd(cscale(up, sn), cmul(v11, uq));
      }
      __syncthreads();
      // rows: A(p,:) <- c A(p,:) + conj(v10) A(q,:);  A(q,:) <- s A(p,:) + conj(v11) A(q,:);
      // the rotated pair's off-diagonal entries are set to zero and its
      // diagonal entries to their real parts by the thread that writes them
      for (int it = lane; it < npair * s; it += blockDim.x) {
        const int k = it / s, j = it % s;
        if (!ract[k]) continue;
        const int p = rp[k], q = rq[k];
        const double cs = rcs[k], sn = rsn[k];
        const double2 v10 = rv10[k], v11 = rv11[k];
        const double2 xp = A[p + S * j], xq = A[q + S * j];
        double2 np = cadd(cscale(xp, cs), cmul(cconj(v10), xq));
        double2 nq = cadd(cscale(xp, sn), cmul(cconj(v11), xq));
        if (j == q) np = make_double2(0, 0);
        if (j == p) { nq = make_double2(0, 0); np.y = 0.0; }
        if (j == q) nq.y = 0.0;
        A[p + S * j] = np;
        A[q + S * j] = nq;
      }
      __syncthreads();
    }
    // every wave reads the flag before the next sweep's reset (several
    // waves: a reset seen early would end some waves' sweeps and not others')
    const int any = rotated;
    __syncthreads();
    if (!any) break;
  }
}

__global__ void __launch_bounds__(256) eigen_kernel(const double2* __restrict__ G, const ClassGeom* __restrict__ geo,
                                                   double2* __restrict__ Uout, const double2* __restrict__ U1,
                                                   const double2* __restrict__ ktab, int n, int d, int final_pass,
                                                   double2* __restrict__ alpha_pad, double2* __restrict__ C_pad,
                                                   double* __restrict__ sigma_pad) {
  __shared__ double2 A[S * S];
  __shared__ double2 U[S * S];
  __shared__ double2 Uf[S * S];
  __shared__ double lam[S];
  __shared__ int order[S];
  __shared__ double2 alpha[S];
  const int c = blockIdx.x, lane = threadIdx.x;
  const ClassGeom& g = geo[c];
  __shared__ int soff[S][3];
  for (int e = lane; e < S * 3; e += blockDim.x) soff[e / 3][e % 3] = g.off[e / 3][e % 3];
  const int s = g.s;
  for (int e = lane; e < S * S; e += blockDim.x) {
    A[e] = G[(long long)c * S * S + e];
    int i = e % S, j = e / S;
    U[e] = make_double2(i == j ? 1.0 : 0.0, 0.0);
  }
  __syncthreads();
  jacobi_eigen(A, U, s, lane);
  if (!final_pass) {
    for (int e = lane; e < S * S; e += blockDim.x) Uout[(long long)c * S * S + e] = U[e];
    return;
  }
  // U_final = U1 U
  for (int e = lane; e < S * S; e += blockDim.x) {
    int i = e % S, j = e / S;
    double2 sum = make_double2(0, 0);
    if (i < s && j < s)
      for (int k = 0; k < s; ++k) sum = cadd(sum, cmul(U1[(long long)c * S * S + i + S * k], U[k + S * j]));
    Uf[e] = sum;
  }
  for (int k = lane; k < S; k += blockDim.x) lam[k] = k < s ? A[k + S * k].x : 0.0;
  __syncthreads();
  if (lane == 0) {
    for (int k = 0; k < s; ++k) order[k] = k;
    for (int i = 1; i < s; ++i) {  // insertion sort, descending
      int v = order[i];
      int j = i - 1;
      while (j >= 0 && lam[order[j]] < lam[v]) { order[j + 1] = order[j]; --j; }
      order[j + 1] = v;
    }
  }
  __syncthreads();
  const int kmin = order[s - 1];
  // alpha = conj(u_min); locate the centre offset
  int centre = 0;
  for (int a = 0; a < s; ++a) {
    bool z = true;
    for (int ax = 0; ax < d; ++ax) z = z && soff[a][ax] == 0;
    if (z) centre = a;
  }
  double2 uc = cconj(Uf[centre + S * kmin]);
  double mag = sqrt(uc.x * uc.x + uc.y * uc.y);
  double2 ph = make_double2(uc.x / mag, -uc.y / mag);  // conj(uc)/|uc|
  double nrm2 = 0.0;
  for (int a = 0; a < s; ++a) { double2 u = Uf[a + S * kmin]; nrm2 += u.x * u.x + u.y * u.y; }
  double inv = 1.0 / sqrt(nrm2);
  for (int a = lane; a < s; a += blockDim.x) alpha[a] = cscale(cmul(cconj(Uf[a + S * kmin]), ph), inv);
  __syncthreads();
  // padded outputs
  for (int e = lane; e < S; e += blockDim.x) {
    alpha_pad[(long long)c * S + e] = make_double2(0, 0);
    C_pad[(long long)c * S + e] = make_double2(0, 0);
    sigma_pad[(long long)c * S + e] = e < s ? sqrt(fmax(lam[order[e]], 0.0)) : 0.0;
  }
  __syncthreads();
  for (int a = lane; a < s; a += blockDim.x) {
    int slot = 0, m3 = 1;
    for (int ax = 0; ax < d; ++ax) { slot += (soff[a][ax] + 1) * m3; m3 *= 3; }
    alpha_pad[(long long)c * S + slot] = alpha[a];
    // C(a') = sum_s alpha(s) k_{|s - a'|}
    double2 sum = make_double2(0, 0);
    for (int b2 = 0; b2 < s; ++b2) {
      int t[3] = {0, 0, 0};
      for (int ax = 0; ax < d; ++ax) t[ax] = abs(soff[b2][ax] - soff[a][ax]);
      sum = cadd(sum, cmul(alpha[b2], ktab[ktab_index(t[0], t[1], t[2], n, d)]));
    }
    C_pad[(long long)c * S + slot] = sum;
  }
}

// ---- general domains (Section 4)
//
// Boundary point b of a general domain (neighbours in Omega: the set bits of
// bslots[b], listed in slot order) takes alpha = the conjugate of the least
// left singular vector of X = T(mu, :), T = (K w^2 m) R the sketch (its r
// columns stored as rows of length N), normalised like the class stencils.
// X is reduced by the same two Gram passes: G = X X^H, Jacobi -> U1; then
// G2 = (U1^H X)(U1^H X)^H, Jacobi -> U2, U = U1 U2 (pass 2 restores the
// relative accuracy of the smallest singular value).  One wave per point;
// the sketch columns are staged BC at a time.  Outputs: alpha slot-padded
// (zero for slots outside Omega) and the singular values, descending.
constexpr int BC = 16;

__global__ void __launch_bounds__(64) bnd_stencil_kernel(const double2* __restrict__ T, int r, long long N,
                                                         const int* __restrict__ bpts,
                                                         const unsigned* __restrict__ bslots, int n, int d,
                                                         double2* __restrict__ balpha, double* __restrict__ bsigma) {
  __shared__ double2 X[S * BC];
  __shared__ double2 Y[S * BC];
  __shared__ double2 A[S * S];
  __shared__ double2 U1[S * S];
  __shared__ double2 U2[S * S];
  __shared__ double2 u[S];
  __shared__ double lam[S];
  __shared__ int order[S];
  __shared__ int sl[S];
  __shared__ long long nbi[S];
  __shared__ int ssz;
  const int b = blockIdx.x, lane = threadIdx.x;
  const int ns = d == 2 ? 9 : 27, centre_slot = ns / 2;
  const long long pt = bpts[b];
  const unsigned bits = bslots[b];
  if (lane == 0) {
    int k = 0;
    for (int q = 0; q < ns; ++q)
      if ((bits >> q) & 1u) sl[k++] = q;
    ssz = k;
  }
  __syncthreads();
  const int s = ssz;
  if (lane < s) {
    const int q = sl[lane];
    const long long o1 = q % 3 - 1, o2 = (q / 3) % 3 - 1, o3 = q / 9 - 1;
    nbi[lane] = pt + o1 + o2 * n + (d == 3 ? o3 * (long long)n * n : 0);
  }
  for (int pass = 0; pass < 2; ++pass) {
    for (int e = lane; e < S * S; e += 64) A[e] = make_double2(0, 0);
    __syncthreads();
    for (int c0 = 0; c0 < r; c0 += BC) {
      const int cols = min(BC, r - c0);
      for (int e = lane; e < s * cols; e += 64) {
        const int a = e % s, c = e / s;
        X[a + S * c] = T[(long long)(c0 + c) * N + nbi[a]];
      }
      __syncthreads();
      const double2* Z = X;
      if (pass == 1) {  // Y = U1^H X
        for (int e = lane; e < s * cols; e += 64) {
          const int a = e % s, c = e / s;
          double2 acc = make_double2(0, 0);
          for (int k = 0; k < s; ++k) acc = cadd(acc, cmul(cconj(U1[k + S * a]), X[k + S * c]));
          Y[a + S * c] = acc;
        }
        __syncthreads();
        Z = Y;
      }
      // A += Z Z^H over this chunk's columns
      for (int e = lane; e < s * s; e += 64) {
        const int i = e % s, j = e / s;
        double2 acc = A[i + S * j];
        for (int c = 0; c < cols; ++c) acc = cadd(acc, cmul(Z[i + S * c], cconj(Z[j + S * c])));
        A[i + S * j] = acc;
      }
      __syncthreads();
    }
    double2* Uc = pass == 0 ? U1 : U2;
    for (int e = lane; e < S * S; e += 64) Uc[e] = make_double2((e % S) == (e / S) ? 1.0 : 0.0, 0.0);
    __syncthreads();
    jacobi_eigen(A, Uc, s, lane);
    __syncthreads();
  }
  for (int k = lane; k < S; k += 64) lam[k] = k < s ? A[k + S * k].x : 0.0;
  __syncthreads();
  if (lane == 0) {
    for (int k = 0; k < s; ++k) order[k] = k;
    for (int i = 1; i < s; ++i) {  // insertion sort, descending
      const int v = order[i];
      int j = i - 1;
      while (j >= 0 && lam[order[j]] < lam[v]) { order[j + 1] = order[j]; --j; }
      order[j + 1] = v;
    }
  }
  __syncthreads();
  const int kmin = order[s - 1];
  // u = U1 U2(:, kmin)
  if (lane < s) {
    double2 acc = make_double2(0, 0);
    for (int k = 0; k < s; ++k) acc = cadd(acc, cmul(U1[lane + S * k], U2[k + S * kmin]));
    u[lane] = acc;
  }
  __syncthreads();
  int centre = 0;
  for (int a = 0; a < s; ++a)
    if (sl[a] == centre_slot) centre = a;
  const double2 uc = cconj(u[centre]);
  const double mag = sqrt(uc.x * uc.x + uc.y * uc.y);
  const double2 ph = make_double2(uc.x / mag, -uc.y / mag);
  double nrm2 = 0.0;
  for (int a = 0; a < s; ++a) nrm2 += u[a].x * u[a].x + u[a].y * u[a].y;
  const double inv = 1.0 / sqrt(nrm2);
  if (lane < S) {
    balpha[(long long)b * S + lane] = make_double2(0, 0);
    bsigma[(long long)b * S + lane] = lane < s ? sqrt(fmax(lam[order[lane]], 0.0)) : 0.0;
  }
  __syncthreads();
  if (lane < s) balpha[(long long)b * S + sl[lane]] = cscale(cmul(cconj(u[lane]), ph), inv);
}

// Rows of M for a general domain: outside Omega the identity row, interior
// points the rectangle's interior row alpha + C w^2 m (class icls), boundary
// points their own alpha (slot-padded, zero outside Omega).  [N][3^d].
__global__ void assemble_general_kernel(double2* __restrict__ Mval, const double2* __restrict__ alpha_pad,
                                        const double2* __restrict__ C_pad, const double* __restrict__ w2m,
                                        const int* __restrict__ ptab, const double2* __restrict__ balpha, int n,
                                        int d, long long N) {
  const long long id = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const int ns = d == 2 ? 9 : 27;
  if (id >= N * ns) return;
  const long long pt = id / ns;
  const int slot = (int)(id % ns);
  const int k = ptab[pt];
  double2 v = make_double2(0, 0);
  if (k == -2) {
    v.x = slot == ns / 2 ? 1.0 : 0.0;
  } else if (k == -1) {
    const int icls = d == 2 ? 4 : 13;
    const long long nb = pt + (slot % 3 - 1) + (long long)((slot / 3) % 3 - 1) * n +
                         (d == 3 ? (long long)(slot / 9 - 1) * n * n : 0);
    v = alpha_pad[icls * S + slot];
    const double2 cc = C_pad[icls * S + slot];
    const double w = w2m[nb];
    v.x += cc.x * w;
    v.y += cc.y * w;
  } else {
    v = balpha[(long long)k * S + slot];
  }
  Mval[id] = v;
}

// T row c = mask .* R row c, widened to complex128 (zero outside Omega);
// dmask = 1 in Omega, 0 outside.
__global__ void sketch_widen_kernel(double2* __restrict__ T, const double* __restrict__ R,
                                    const int* __restrict__ ptab, long long N) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  T[i] = make_double2(ptab[i] != -2 ? R[i] : 0.0, 0.0);
}

__global__ void domain_mask_kernel(double* __restrict__ dmask, const int* __restrict__ ptab, long long N) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < N) dmask[i] = ptab[i] != -2 ? 1.0 : 0.0;
}

__device__ inline int point_class(const int* i, int n, int d) {
  int c = 0, m3 = 1;
  for (int a = 0; a < d; ++a) {
    int ca = i[a] == 0 ? 0 : (i[a] == n - 1 ? 2 : 1);
    c += ca * m3; m3 *= 3;
  }
  return c;
}

// M(i, i+s) = alpha_c(s) + [c interior] C_c(s) w^2 m_{i+s}, as [N][3^d].
__global__ void assemble_kernel(double2* __restrict__ Mval, const double2* __restrict__ alpha_pad,
                                const double2* __restrict__ C_pad, const double* __restrict__ w2m, int n, int d,
                                long long N) {
  long long id = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const int ns = d == 2 ? 9 : 27;
  if (id >= N * ns) return;
  long long pt = id / ns;
  int slot = (int)(id % ns);
  int i[3] = {(int)(pt % n), (int)((pt / n) % n), d == 3 ? (int)(pt / ((long long)n * n)) : 0};
  int c = point_class(i, n, d);
  int icls = d == 2 ? 4 : 13;
  int o[3] = {slot % 3 - 1, (slot / 3) % 3 - 1, slot / 9 - 1};
  bool inside = true;
  long long nb = 0, st = 1;
  for (int a = 0; a < d; ++a) {
    int j = i[a] + o[a];
    inside = inside && j >= 0 && j < n;
    nb += (long long)j * st;
    st *= n;
  }
  double2 v = make_double2(0, 0);
  if (inside) {
    v = alpha_pad[c * S + slot];
    if (c == icls) {
      double2 cc = C_pad[c * S + slot];
      double w = w2m[nb];
      v.x += cc.x * w; v.y += cc.y * w;
    }
  }
  Mval[id] = v;
}

// y_i = sum_s alpha_{c(i)}(s) x_{i+s}, complex128.  Grid: blockIdx.x =
// line (i2 + n i3) times the nb1 blocks of 256 along i1, plus the block;
// blockIdx.y the right-hand side; the 3^D offsets unrolled, neighbours
// outside the grid skipped.
template <typename Cx, int D>
__global__ void __launch_bounds__(256) applyQ_kernel(Cx* __restrict__ y, const double2* __restrict__ x,
                                                     const double2* __restrict__ alpha_pad, int n, long long N,
                                                     int nb1) {
  const int line = blockIdx.x / nb1;
  const int i1 = (blockIdx.x - line * nb1) * 256 + threadIdx.x;
  if (i1 >= n) return;
  const int i2 = D == 2 ? line : line % n, i3 = D == 2 ? 0 : line / n;
  const int i[3] = {i1, i2, i3};
  const int c = point_class(i, n, D);
  const long long rb = (long long)blockIdx.y * N;
  const long long pt = (long long)line * n + i1;
  constexpr int NS = D == 2 ? 9 : 27;
  const double2* al = alpha_pad + c * S;
  double2 acc = make_double2(0, 0);
#pragma unroll
  for (int slot = 0; slot < NS; ++slot) {
    const int o1 = slot % 3 - 1, o2 = (slot / 3) % 3 - 1, o3 = slot / 9 - 1;
    const bool inside = i1 + o1 >= 0 && i1 + o1 < n && i2 + o2 >= 0 && i2 + o2 < n &&
                        (D == 2 || (i3 + o3 >= 0 && i3 + o3 < n));
    if (inside) {
      const long long nb = pt + o1 + (long long)o2 * n + (D == 3 ? (long long)o3 * n * n : 0);
      acc = cadd(acc, cmul(al[slot], x[rb + nb]));
    }
  }
  y[rb + pt] = from_c128<Cx>(acc);
}

// Q apply of a general domain: outside Omega the identity row, interior
// points the interior class stencil, boundary points their own (neighbours
// outside the grid skipped; their alpha is zero).
template <typename Cx, int D>
__global__ void __launch_bounds__(256) applyQ_general_kernel(Cx* __restrict__ y, const double2* __restrict__ x,
                                                             const double2* __restrict__ alpha_pad,
                                                             const int* __restrict__ ptab,
                                                             const double2* __restrict__ balpha, int n, long long N,
                                                             int nb1) {
  const int line = blockIdx.x / nb1;
  const int i1 = (blockIdx.x - line * nb1) * 256 + threadIdx.x;
  if (i1 >= n) return;
  const int i2 = D == 2 ? line : line % n, i3 = D == 2 ? 0 : line / n;
  const long long rb = (long long)blockIdx.y * N;
  const long long pt = (long long)line * n + i1;
  constexpr int NS = D == 2 ? 9 : 27;
  const int k = ptab[pt];
  if (k == -2) {
    y[rb + pt] = from_c128<Cx>(x[rb + pt]);
    return;
  }
  const double2* al = k == -1 ? alpha_pad + (D == 2 ? 4 : 13) * S : balpha + (long long)k * S;
  double2 acc = make_double2(0, 0);
#pragma unroll
  for (int slot = 0; slot < NS; ++slot) {
    const int o1 = slot % 3 - 1, o2 = (slot / 3) % 3 - 1, o3 = slot / 9 - 1;
    const bool inside = i1 + o1 >= 0 && i1 + o1 < n && i2 + o2 >= 0 && i2 + o2 < n &&
                        (D == 2 || (i3 + o3 >= 0 && i3 + o3 < n));
    if (inside) {
      const long long nb = pt + o1 + (long long)o2 * n + (D == 3 ? (long long)o3 * n * n : 0);
      acc = cadd(acc, cmul(al[slot], x[rb + nb]));
    }
  }
  y[rb + pt] = from_c128<Cx>(acc);
}

// The 2D stencil product over row blocks: a workgroup takes 256 columns of
// qrb consecutive rows of one right-hand side and keeps a window of three
// rows of x (with one halo column on each side) in LDS, so every row of x
// is read once per block (plus two halo rows) instead of once per row
// above, at and below; each point's sum runs over the slots in the same
// order as applyQ_kernel's (the same values bit for bit).  qrb is 16 unless
// that leaves fewer than 2048 workgroups (small grids, few right-hand
// sides), then halved until it does not, down to one row per workgroup.
constexpr int QRB = 16;

template <typename Cx>
__global__ void __launch_bounds__(256) applyQ_rows_kernel(Cx* __restrict__ y, const double2* __restrict__ x,
                                                          const double2* __restrict__ alpha_pad, int n, long long N,
                                                          int nb1, int qrb) {
  __shared__ double2 win[3][258];
  __shared__ double2 alp[9 * 9];  // the 9 classes' stencils (9 slots each)
  const int cb = blockIdx.x % nb1, r0 = (blockIdx.x / nb1) * qrb, tid = threadIdx.x;
  if (tid < 81) alp[tid] = alpha_pad[(tid / 9) * S + tid % 9];
  const int c0 = cb * 256, i1 = c0 + tid;
  const long long rb = (long long)blockIdx.y * N;
  const int r1 = min(n, r0 + qrb);
  auto load_row = [&](int j) {  // row j (in the grid) into slot j mod 3
    double2* w = win[(j + 3) % 3];
    for (int e = tid; e < 258; e += 256) {
      const int c = c0 - 1 + e;
      w[e] = (j >= 0 && j < n && c >= 0 && c < n) ? x[rb + (long long)j * n + c] : make_double2(0, 0);
    }
  };
  load_row(r0 - 1);
  load_row(r0);
  for (int j = r0; j < r1; ++j) {
    load_row(j + 1);
    __syncthreads();
    if (i1 < n) {
      const int ii[3] = {i1, j, 0};
      const int c = point_class(ii, n, 2);
      const double2* al = alp + c * 9;
      double2 acc = make_double2(0, 0);
#pragma unroll
      for (int slot = 0; slot < 9; ++slot) {
        const int o1 = slot % 3 - 1, o2 = slot / 3 - 1;
        const bool inside = i1 + o1 >= 0 && i1 + o1 < n && j + o2 >= 0 && j + o2 < n;
        if (inside) acc = cadd(acc, cmul(al[slot], win[(j + o2 + 3) % 3][tid + 1 + o1]));
      }
      y[rb + (long long)j * n + i1] = from_c128<Cx>(acc);
    }
    __syncthreads();  // the slot of row j - 1 is reloaded next
  }
}

}  // namespace

void launch_domain_mask(double* dmask, const int* ptab, long long N, hipStream_t st) {
  LSP_LAUNCH("domain_mask", 0, domain_mask_kernel, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, st, dmask, ptab,
             N);
}

void launch_sketch_widen(double2* T, const double* R, const int* ptab, long long N, hipStream_t st) {
  LSP_LAUNCH("sketch_widen", 0, sketch_widen_kernel, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, st, T, R, ptab,
             N);
}

void launch_bnd_stencils(const double2* T, int r, long long N, const int* bpts, const unsigned* bslots, int nbnd,
                         int n, int d, double2* balpha, double* bsigma, hipStream_t st) {
  if (nbnd == 0) return;
  LSP_LAUNCH("bnd_stencil", 0, bnd_stencil_kernel, dim3(nbnd), dim3(64), 0, st, T, r, N, bpts, bslots, n, d, balpha,
             bsigma);
}

void launch_assemble_general(double2* Mval, const double2* alpha_pad, const double2* C_pad, const double* w2m,
                             const int* ptab, const double2* balpha, int n, int d, long long N, hipStream_t st) {
  const long long total = N * (d == 2 ? 9 : 27);
  LSP_LAUNCH("assemble", 0, assemble_general_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, Mval,
             alpha_pad, C_pad, w2m, ptab, balpha, n, d, N);
}

template <typename Cx>
void launch_applyQ_general(Cx* y, const double2* x, const double2* alpha_pad, const int* ptab, const double2* balpha,
                           int n, int d, long long N, int nrhs, hipStream_t st) {
  const int nb1 = (n + 255) / 256;
  const long long lines = d == 2 ? n : (long long)n * n;
  const dim3 grid((unsigned)(lines * nb1), nrhs);
  if (d == 2)
    LSP_LAUNCH("applyQ", (int)sizeof(Cx), (applyQ_general_kernel<Cx, 2>), grid, dim3(256), 0, st, y, x, alpha_pad,
               ptab, balpha, n, N, nb1);
  else
    LSP_LAUNCH("applyQ", (int)sizeof(Cx), (applyQ_general_kernel<Cx, 3>), grid, dim3(256), 0, st, y, x, alpha_pad,
               ptab, balpha, n, N, nb1);
}

template void launch_applyQ_general<double2>(double2*, const double2*, const double2*, const int*, const double2*,
                                             int, int, long long, int, hipStream_t);
template void launch_applyQ_general<float2>(float2*, const double2*, const double2*, const int*, const double2*, int,
                                            int, long long, int, hipStream_t);

void compute_stencils(const double2* ktab, int n, int d, const ClassGeom* geo_dev, int nclass, long long maxF,
                      double2* partial, int nblk, double2* G, double2* U1, double2* alpha_pad, double2* C_pad,
                      double* sigma_pad, hipStream_t st) {
  (void)maxF;
  dim3 grid(nblk, nclass);
  LSP_LAUNCH("gram", 0, gram_kernel<false>, grid, dim3(256), 0, st, ktab, n, d, geo_dev, (const double2*)nullptr,
                     partial, nblk);
  LSP_LAUNCH("gram_reduce", 0, gram_reduce_kernel, dim3(nclass), dim3(768), 0, st, partial, G, nblk, nclass, geo_dev);
  LSP_LAUNCH("eigen", 0, eigen_kernel, dim3(nclass), dim3(256), 0, st, G, geo_dev, U1, (const double2*)nullptr, ktab, n,
                     d, 0, alpha_pad, C_pad, sigma_pad);
  LSP_LAUNCH("gram", 0, gram_kernel<true>, grid, dim3(256), 0, st, ktab, n, d, geo_dev, U1, partial, nblk);
  LSP_LAUNCH("gram_reduce", 0, gram_reduce_kernel, dim3(nclass), dim3(768), 0, st, partial, G, nblk, nclass, geo_dev);
  LSP_LAUNCH("eigen", 0, eigen_kernel, dim3(nclass), dim3(256), 0, st, G, geo_dev, (double2*)nullptr, U1, ktab, n, d, 1,
                     alpha_pad, C_pad, sigma_pad);
}

void launch_assemble(double2* Mval, const double2* alpha_pad, const double2* C_pad, const double* w2m, int n, int d,
                     long long N, hipStream_t st) {
  long long total = N * (d == 2 ? 9 : 27);
  int bs = 256;
  LSP_LAUNCH("assemble", 0, assemble_kernel, dim3((unsigned)((total + bs - 1) / bs)), dim3(bs), 0, st, Mval, alpha_pad,
                     C_pad, w2m, n, d, N);
}

template <typename Cx>
void launch_applyQ(Cx* y, const double2* x, const double2* alpha_pad, int n, int d, long long N, int nrhs,
                   hipStream_t st) {
  const int nb1 = (n + 255) / 256;
  const long long lines = d == 2 ? n : (long long)n * n;
  const dim3 grid((unsigned)(lines * nb1), nrhs);
  if (d == 2) {
    int qrb = QRB;
    while (qrb > 1 && (long long)((n + qrb - 1) / qrb) * nb1 * nrhs < 2048) qrb /= 2;
    LSP_LAUNCH("applyQ", (int)sizeof(Cx), (applyQ_rows_kernel<Cx>), dim3((unsigned)(((n + qrb - 1) / qrb) * nb1), nrhs),
               dim3(256), 0, st, y, x, alpha_pad, n, N, nb1, qrb);
  } else
    LSP_LAUNCH("applyQ", (int)sizeof(Cx), (applyQ_kernel<Cx, 3>), grid, dim3(256), 0, st, y, x, alpha_pad, n, N, nb1);
}

template void launch_applyQ<double2>(double2*, const double2*, const double2*, int, int, long long, int, hipStream_t);
template void launch_applyQ<float2>(float2*, const double2*, const double2*, int, int, long long, int, hipStream_t);

}  // namespace lsp
