// Launch interfaces of the GMRES kernels (complex128, one Krylov process per
// right-hand side, basis layout [k][nrhs][N]).
#pragma once

#include "lsp_common.h"

namespace lsp {

constexpr int kMaxVec = 32;  // restart length limit (basis vectors per cycle)
constexpr int kScal = 8;     // per right-hand-side scalars
// S_GNORM: ||g||; S_BETA: latest true residual norm; S_TARGET: this cycle's
// stopping level of the GMRES estimate
enum { S_NORM = 0, S_INV = 1, S_EST = 2, S_DEN = 3, S_GNORM = 4, S_BETA = 5, S_TARGET = 6 };

// GMRES control decided on the device, reported to the host through pinned,
// coherent host memory: after writing the per-right-hand-side fields and the
// number of right-hand sides still iterating, a kernel stores `tag` (release,
// system scope); the host waits for the tag it expects.
struct HostCtl {
  unsigned tag;
  int nact;
  double value;        // a reduced scalar (k_min_report)
};
struct CtlView {       // device-visible pointers into one pinned allocation
  HostCtl* hdr;
  int* iters;          // [nrhs] Arnoldi steps taken
  double* est;         // [nrhs] latest GMRES residual estimate
  double* beta;        // [nrhs] latest true residual norm
  double* gnorm;       // [nrhs] ||g||
};
struct GmresState {    // device arrays of the solve workspace
  double* scal;        // [nrhs][kScal]
  int* active;         // [nrhs] iterating in this cycle
  int* ksz;            // [nrhs] Krylov size of this cycle
  int* iters;          // [nrhs] Arnoldi steps over all cycles
  int* done;           // [nrhs] converged
};
struct GmresParams {
  double tol;          // relative true-residual tolerance
  double eta;          // cycle stops when the estimate falls below eta * beta
  int max_iters;
};

int dot_blocks(long long N);
void k_dots(const double2* V, const double2* w, double2* partial, double2* h, double2* H, double* scal, int nvec,
            int k, int restart, int mode, long long N, int nrhs, const int* active, hipStream_t st);
void k_norm(const double2* w, double2* partial, double2* h, double2* H, double* scal, int k, int restart, long long N,
            int nrhs, const int* active, hipStream_t st);
void k_axpy(const double2* V, double2* w, const double2* h, int nvec, long long N, int nrhs, const int* active,
            hipStream_t st);
// Arnoldi step k: CGS2 of w against V_0..V_k, H(0:k+1, k), the norm scalars,
// and vnext = w / ||w||; pA, pB: two partial-sum buffers [nrhs][dot_blocks(N)][kMaxVec].
void k_arnoldi_orth(const double2* V, double2* w, double2* pA, double2* pB, double2* h, double2* H, double* scal,
                    double2* vnext, int k, int restart, long long N, int nrhs, const int* active, hipStream_t st);
void k_scale(double2* y, const double2* x, const double* scal, long long N, int nrhs, const int* active,
             hipStream_t st);
// Givens update of column k and the stopping decision of step k: a right-
// hand side stops when its estimate is not above S_TARGET, at max_iters, or
// on a zero column; reports the number still iterating under `tag`.
void k_givens(double2* H, double2* cs, double2* sn, double2* gam, int k, int restart, int nrhs, const GmresState& gs,
              const GmresParams& gp, const CtlView& host, unsigned tag, hipStream_t st);
// Start of the solve (cycle_end false: S_NORM holds ||g||) or end of a cycle
// (S_NORM holds the true residual norm): convergence, then the next cycle's
// active set, Krylov sizes and targets; reports under `tag`.
void k_gmres_control(bool cycle_end, int nrhs, const GmresState& gs, const GmresParams& gp, const CtlView& host,
                     unsigned tag, hipStream_t st);
// (kmax: the most Arnoldi steps any right-hand side took in the cycle)
void k_backsolve_update(const double2* H, const double2* gam, double2* y, const int* ksz, double2* x, const double2* Z,
                        int restart, int kmax, long long N, int nrhs, hipStream_t st);
void k_sub(double2* r, const double2* g, const double2* t, long long count, hipStream_t st);
void k_cycle_init(double2* H, double2* gam, const double* scal, int restart, int nrhs, hipStream_t st);
// host.hdr->value = min over v[0..n) (-1 if any entry is NaN), reported under tag.
void k_min_report(const double* v, long long n, const CtlView& host, unsigned tag, hipStream_t st);
void k_fill_zero(void* p, long long bytes, hipStream_t st);
void k_fill_double(double* p, double v, long long count, hipStream_t st);
void k_w2m(double* out, const double* m, double w2, long long N, hipStream_t st);

}  // namespace lsp
