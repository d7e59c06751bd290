// Launch interfaces shared between the kernel translation units and the ABI layer.
#pragma once

#include "lsp_common.h"
#include "plan.h"

namespace lsp {

constexpr int kNbMax = 32;  // widest frontal panel
constexpr int kSweepBlock = kSweepRows;  // rows of a super-block of the blocked sweeps
constexpr int kSweepChunk = kSweepCols;  // boundary columns per partial sum of the blocked backward sweep

// ---- Green's table
void launch_ktable(double2* k, int n, int d, double omega, double2 k0, hipStream_t st);
void launch_embed(double2* E, const double2* k, int n, int d, hipStream_t st);
void launch_split_spectrum(double2* s64, float2* s32, const double2* E, int n, int d, hipStream_t st);

// Scattered field away from the grid (mode 0: at points [npts][d]) or its
// far-field pattern (mode 1: unit directions [npts][d]) from u and u_I
// ([nrhs][N] complex128) and w2m; partial: field_chunks(N) * min(nrhs, 16)
// * npts complex128; out [nrhs][npts].
long long field_chunks(long long N);
void field_eval(int mode, const double2* u, const double2* uI, const double* w2m, const double* pts, int npts,
                int nrhs, int n, int d, double omega, double2 k0, double2* partial, double2* out, hipStream_t st);

// ---- FFT
struct FftRadices {
  int r[16];
  int npass;
};

template <typename T>
struct FftPlanDev {
  int n, d, L, N;
  int ept;                   // elements per thread of the full-length (L-point) transforms
  int hept;                  // elements per thread of the half-length (n-point) transforms
  long long wstride;         // work array elements per right-hand side (L^d)
  long long lr;              // row stride of the K-matvec's work rows (L; L + 16 in 2D, n >= 16)
  FftRadices rad;            // radices of L
  FftRadices hrad;           // radices of n
  const cplx<T>* tw;         // exp(-2 pi i k / L), k < L
  const cplx<T>* spec;       // spectrum rows in split order, (n+1)^(d-1) x L, scaled by 1/L^d
};

// y = [x +] K (w2m .* x), fields complex128 [nrhs][N]; w2m == nullptr means
// no scaling; W is the [nrhs][L^d] work array in precision T; omask (may be
// null): y is set to zero where omask is 0 (a general domain's exterior).
template <typename T>
void kmatvec(const FftPlanDev<T>& fp, int nrhs, const double2* x, double2* y, const double* w2m, bool add_x,
             cplx<T>* W, hipStream_t st, const double* omask = nullptr);
// In-place forward transform of a full L^d array (one right-hand side).
template <typename T>
void full_fft_forward(const FftPlanDev<T>& fp, cplx<T>* W, hipStream_t st);

// ---- stencils
struct ClassGeom {
  int s;             // stencil size
  int off[kMaxStencil][3];
  int flo[3], fsz[3];  // far-set box: start and size per axis
  long long F;       // far-set box volume
  int interior;      // 1 for the all-interior class (mu(0) removed)
};

void compute_stencils(const double2* ktab, int n, int d, const ClassGeom* geo_dev, int nclass, long long maxF,
                      double2* partial, int nblk, double2* G, double2* U1, double2* alpha_pad, double2* C_pad,
                      double* sigma_pad, hipStream_t st);
void launch_assemble(double2* Mval, const double2* alpha_pad, const double2* C_pad, const double* w2m, int n, int d,
                     long long N, hipStream_t st);
template <typename Cx>
void launch_applyQ(Cx* y, const double2* x, const double2* alpha_pad, int n, int d, long long N, int nrhs,
                   hipStream_t st);

// general domains (Section 4); ptab / bpts / bslots as in Plan
void launch_domain_mask(double* dmask, const int* ptab, long long N, hipStream_t st);
void launch_sketch_widen(double2* T, const double* R, const int* ptab, long long N, hipStream_t st);
void launch_bnd_stencils(const double2* T, int r, long long N, const int* bpts, const unsigned* bslots, int nbnd,
                         int n, int d, double2* balpha, double* bsigma, hipStream_t st);
void launch_assemble_general(double2* Mval, const double2* alpha_pad, const double2* C_pad, const double* w2m,
                             const int* ptab, const double2* balpha, int n, int d, long long N, hipStream_t st);
template <typename Cx>
void launch_applyQ_general(Cx* y, const double2* x, const double2* alpha_pad, const int* ptab, const double2* balpha,
                           int n, int d, long long N, int nrhs, hipStream_t st);

// ---- multifrontal
template <typename T>
struct MfDev {
  cplx<T>* F;               // front matrices
  cplx<T>* Dinv;            // inverted diagonal panel blocks
  const FrontDev* fronts;
  const int* idx;
  const unsigned* gpos;     // packed grid coordinates of the idx entries
  const int* cpos;
  const double2* Mval;      // [N][3^d]
  int* perm;                // per panel row: the front row it came from
  double* pivstat;          // per diagonal block: smallest / largest pivot magnitude
  cplx<T>* G;               // formed sweep operators of the dense and blocked levels (FrontDev::g_off)
};

// Work buffers of the blocked sweeps (in the solve workspace): ybuf holds a
// super-block's output per front, [nrhs][ystride]; pbuf the boundary
// columns' partial sums, [chunks][nrhs][ystride] (Plan::bsweep_ystride,
// Plan::bsweep_chunks).
template <typename T>
struct SweepBufs {
  cplx<T>* ybuf;
  cplx<T>* pbuf;
  long long ystride;
  cplx<T>* xpm;  // the solution point-major for the matrix-core levels'
                 // gathers: [groups of 16 right-hand sides][N][16]
};

// Second stream for the dense levels' operator formation: each level's
// formation waits (event `level`) for that level's factorisation on the main
// stream and then runs beside the factorisation of the levels above it;
// `done` is recorded after the last.
struct FormStream {
  hipStream_t aux;
  hipEvent_t level, done;
};

// Numeric factorisation, level by level, and the dense levels' sweep
// operators: on fs->aux when fs is given (the caller makes the sweeps wait
// for fs->done), else on st after the factorisation.  Waits on st for a
// previous formation (all work enqueued on fs->aux), which still reads the
// factors.
template <typename T>
void mf_factor(const MfDev<T>& mf, const Plan& plan, hipStream_t st, const FormStream* fs);

// Of one factorisation: the diagonal blocks not factored by a diagonal-block
// launch of their own (lookahead or panel-strip launches), and the
// trailing-update flops of the update launches that also factor a block.
struct FactorSchedule {
  double fused_blocks = 0.0;
  double fused_update_flops = 0.0;
  double trsm_flops = 0.0;  // real flops of the panel_trsm launches
  double pair_update_flops = 0.0;   // real flops of the two-panel updates (pair_update)
  double cross_update_flops = 0.0;  // real flops of panel a's update of panel b's strips (cross_update)
};
FactorSchedule factor_schedule(const Plan& plan, bool fp64);
// Forward and backward sweeps; form_done (may be null): an event the first
// dense level's sweep waits for (the operators' formation); xw (may be
// null): the solution also written there in complex128.
template <typename T>
void mf_solve(const MfDev<T>& mf, const Plan& plan, int nrhs, const cplx<T>* z, cplx<T>* x, cplx<T>* vbuf,
              const SweepBufs<T>& sb, hipStream_t st, hipEvent_t form_done, double2* xw);

// Blocked forward (fwd) or backward sweep of level l (Plan::level_blocked):
// per 256-row super-block of the pivots its formed operator and a wide
// matrix-vector product over the rest of the front; the backward sweep
// starts with the boundary columns' product.  Same inputs and outputs as the
// panel-chain sweeps of that level.
template <typename T>
void blocked_sweep(bool fwd, const MfDev<T>& mf, const Plan& plan, int l, int nrhs, const cplx<T>* z, cplx<T>* x,
                   cplx<T>* vbuf, const SweepBufs<T>& sb, hipStream_t st, double2* xw);
// Sweep of a small-front level (Plan::level_mchain): per front and group of
// 16 right-hand sides one wave runs the panel chain on the matrix cores.
// Same inputs and outputs as the panel-chain sweeps of that level.
template <typename T>
void mchain_sweep(bool fwd, const MfDev<T>& mf, const Plan& plan, int l, int nrhs, const cplx<T>* z, cplx<T>* x,
                  cplx<T>* vbuf, hipStream_t st, double2* xw, cplx<T>* xpm);
// xpm[g][i][k] = x[16 g + k][i] (zero for k beyond nrhs) for the pivots i of
// levels lo .. hi - 1: the backward sweep's solution of levels swept by other
// kernels, point-major, for the matrix-core levels below them (which store
// their own pivots there themselves).
template <typename T>
void launch_point_major(const MfDev<T>& mf, const Plan& plan, int lo, int hi, const cplx<T>* x, cplx<T>* xpm,
                        int nrhs, hipStream_t st);
// Forms the super-block operators of blocked level l from its factor (the
// panel chains on the unit vectors), into mf.G at each front's g_off.
template <typename T>
void blocked_form(const MfDev<T>& mf, const Plan& plan, int l, hipStream_t st);

// ---- Krylov helpers (complex128 vectors, [nrhs][N] blocks)
void launch_narrow(float2* y, const double2* x, long long count, hipStream_t st);
void launch_scale_rhs(double2* y, const double2* x, double s, long long count, hipStream_t st);

}  // namespace lsp
