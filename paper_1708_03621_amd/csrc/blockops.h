// Declarations of the packed-block and small-matrix kernels (blockops.hip).
#pragma once

#include <hip/hip_runtime.h>

#include "internal.h"

namespace dpp {

constexpr int DOT_BLOCKS = 64;  // fixed partial-sum count per block reduction
constexpr int PULAY_MAX = 8;

struct Seg {
    int64_t off;          // element offset of block k in the packed buffer
    int npw;
    int pad;
    const double* kG2;
};

struct DotPairs {
    const double2* a[4];
    const double2* b[4];
};

constexpr int MDOT_BLOCKS = 256;

struct PulayOrder {
    int s[PULAY_MAX];
};

struct PulayPtrs {
    const double* nin[PULAY_MAX];
    const double* res[PULAY_MAX];
};

__global__ void k_seg_axpby(const Seg* seg, int nb, const double* a, const double2* x, const double* b,
                            const double2* y, double2* out);
__global__ void k_seg_precond(const Seg* seg, int nb, double scale, const double2* x, double2* out);
__global__ void k_seg_dots(const Seg* seg, int nk, int nb, int npair, DotPairs pr, double* part);
__global__ void k_seg_dots_reduce(const double* part, int nk, int npair, double* out);
__global__ void k_seg_kinetic(const Seg* seg, int nb, int fstride, const double* f, const double2* psi, double* part);
__global__ void k_seg_weighted_total(const double* part, int nk, const double* wk, double scale, double* out);
__global__ void k_nonlocal_energy(int nk, int nproj, int nb, int fstride, const double2* pi, int64_t pi_stride,
                                  const double* f, const double* wk, double D, double* out);
__global__ void k_sm_scale(int n, int64_t st, int op, double scale, const double* scale_arr, const double2* A,
                           double2* out);
__global__ void k_smm(int n, int opA, int opB, double alpha, const double* alpha_arr, const double2* A, int64_t sa,
                      const double2* B, int64_t sb, double beta, double2* Cm, int64_t sc);
__global__ void k_trace(int n, const double2* A, int64_t sa, double scale, double* out);
__global__ void k_trial_mats(int n, const double* alpha, const double2* U, const double2* X, const double2* Q,
                             const double2* H0, const double2* H1, const double2* H2, double2* Ua, double2* Ha);
__global__ void k_trace_RhHR(int n, const double2* Rinv, const double2* H, double* out);
__global__ void k_band_residual(const Seg* seg, int nb, int fstride, const double* eig, double omega, const double2* Y,
                                const double2* HY, double* out);
__global__ void k_grid_lin3(int64_t N, double a, const double* x, double b, const double* y, double c,
                            const double* z, double* out);
__global__ void k_pulay_combine(int64_t N, int m, PulayPtrs h, const double* c, double alpha, double* out);
__global__ void k_pulay_solve(int m, const double* A, PulayOrder order, double* c, int* status);
__global__ void k_multi_dot(int64_t N, const double* a, PulayPtrs bl, int nb, double* part);
__global__ void k_multi_dot_store(const double* part, int nb, PulayOrder slot, int row, double scale, double* A);

}  // namespace dpp
