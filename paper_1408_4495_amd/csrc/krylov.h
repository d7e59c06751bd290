// Launch interfaces of the GMRES kernels (complex128, one Krylov process per
// right-hand side, basis layout [k][nrhs][N]).
#pragma once

#include "lsp_common.h"

namespace lsp {

constexpr int kMaxVec = 32;  // restart length limit (basis vectors per cycle)
constexpr int kScal = 8;     // per right-hand-side scalars
enum { S_NORM = 0, S_INV = 1, S_EST = 2, S_DEN = 3 };

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
void k_givens(double2* H, double2* cs, double2* sn, double2* gam, double* scal, int k, int restart, int nrhs,
              const int* active, hipStream_t st);
void k_backsolve_update(const double2* H, const double2* gam, double2* y, const int* ksz, double2* x, const double2* Z,
                        int restart, long long N, int nrhs, hipStream_t st);
void k_sub(double2* r, const double2* g, const double2* t, long long count, hipStream_t st);
void k_cycle_init(double2* H, double2* gam, const double* scal, int restart, int nrhs, hipStream_t st);
void k_fill_zero(void* p, long long bytes, hipStream_t st);
void k_fill_double(double* p, double v, long long count, hipStream_t st);
void k_w2m(double* out, const double* m, double w2, long long N, hipStream_t st);

}  // namespace lsp
