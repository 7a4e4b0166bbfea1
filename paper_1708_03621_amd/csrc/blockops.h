// Declarations of the packed-block and small-matrix kernels (blockops.hip).
#pragma once

#include <hip/hip_runtime.h>

#include "internal.h"

namespace dpp {

// Partial sums per item of the block reductions over bands x points: 256 for
// systems of up to three items (one item alone then spreads over every CU),
// 64 for more (whose items together fill the chip; more blocks only add
// near-empty workgroups).  Fixed per system, so the summation order is too.
constexpr int DOT_BLOCKS = 256;  // the most per item (partial buffer size)
inline int dot_blocks(int nitems) { return nitems <= 3 ? DOT_BLOCKS : 64; }
constexpr int PULAY_MAX = 8;

// One work item (a k-point of a cell): where its data sits in the packed
// block buffers, its small matrices, projector overlaps and fillings.
struct Seg {
    int64_t off;          // element offset of the item's block in the packed buffer
    int64_t moff;         // offset of its nb x nb matrices
    int64_t pioff;        // offset of its nproj x nb projector overlaps
    int64_t f_off;        // offset of its fillings / eigenvalues (nb entries)
    const double* kG2;
    double wk;            // k-point weight
    double omega;         // cell volume
    int npw, nb, nproj, cell;
};

struct DotPairs {
    const double2* a[4];
    const double2* b[4];
};

constexpr int MDOT_BLOCKS = 256;
constexpr int AUFBAU_MAX = 1024;       // states (k-points x bands) of one cell
constexpr int AUFBAU_MAX_ITEMS = 64;   // k-points of one cell
constexpr double DEGEN_TOL = 1e-6;     // degenerate-set width of the aufbau fillings (Ha)

// Device arrays of the band-CG state, one entry per work item.
struct CgBState {
    double *at, *gkg, *beta, *d0, *d0r, *step, *step2, *cK, *cD;
    double* stepf;  // the accepted step of the last CG step (0: none)
    int *reset, *stat, *act, *steep, *ok, *ok2, *retry;
};

// Kernels with `nbo`: band count override (> 0) for every item, else seg.nb.
__global__ void k_seg_axpby(const Seg* seg, int nbo, const double* a, const double2* x, const double* b,
                            const double2* y, double2* out);
// Band-CG control fused with the elementwise pass that consumes it (each
// workgroup of an item evaluates the item's control in the same fixed order;
// workgroup 0 writes the state):
//   direction: reduce <g,Kg>, <g_prev,Kg>, <g,D_prev>, set beta, then D = -Kg + beta D_prev;
//   retry:     mark failed CG searches, then D = cK Kg + cD D (D = -Kg for them);
//   finish:    accept the steps (stepf), then Y += a D, HY += a HD, g_prev = g, D_prev = D.
__global__ void k_cgB_direction(const Seg* seg, int nitems, const double* part, double* dots, CgBState s,
                                const double2* Kg, const double2* Dp, double2* Dd, int nblk);
__global__ void k_cgB_retry_axpby(const Seg* seg, const double* dots, CgBState s, const double2* Kg, double2* Dd);
__global__ void k_cgB_finish_update(const Seg* seg, const double* dots, CgBState s, double2* Y, const double2* Dd,
                                    double2* HY, const double2* HD, const double2* g, double2* gp, double2* Dp);
__global__ void k_seg_precond(const Seg* seg, int nbo, double scale, const double2* x, double2* out);
__global__ void k_seg_dots(const Seg* seg, int nitems, int nbo, int npair, DotPairs pr, double* part);
__global__ void k_seg_dots_reduce(const double* part, int nitems, int npair, double* out, int nblk);
__global__ void k_seg_kinetic(const Seg* seg, int nbo, const double* f, const double2* psi, double* part);
__global__ void k_cell_weighted_totals(const double* part, const Seg* seg, const CellDesc* cells, int ncells,
                                       double scale_omega, double* out, int out_stride, int nblk);
__global__ void k_nonlocal_energy(const Seg* seg, const CellDesc* cells, int nbo, const double2* pi, const double* f,
                                  double* out, int out_stride);
__global__ void k_sm_scale(const Seg* seg, int nbo, int op, double scale, int flags, const double2* A,
                           double2* out);
__global__ void k_band_residual(const Seg* seg, const double* eig, const double2* Y, const double2* HY, double* out);
__global__ void k_grid_lin3(int64_t N, double a, const double* x, double b, const double* y, double c,
                            const double* z, double* out);
__global__ void k_fill(int64_t n, double v, double* out);
__global__ void k_copy(int64_t n, const double2* x, double2* out);
__global__ void k_pulay_reset(int* st);
__global__ void k_pulay_begin(int* st);
__global__ void k_pulay_store(int64_t Ntot, const int* st, const double* nin, const double* nout, double* hn,
                              double* hr);
__global__ void k_pulay_dots(int64_t Ntot, const int* st, const CellDesc* cells, const double* hr, double* part);
__global__ void k_pulay_solve_cells(int ncells, const int* st, const CellDesc* cells, const double* part, double* A,
                                    double* coef, int* status);
__global__ void k_pulay_combine_cells(int64_t Ntot, const int* st, const CellDesc* cells, const double* coef,
                                      double alpha, const double* hn, const double* hr, double* nin);
__global__ void k_cgB_reset(int nit, const Seg* seg, CgBState s);
__global__ void k_aufbau(const CellDesc* cells, const Seg* seg, const double* eig, double* f, int* status);
// Fermi-Dirac fillings of width sigma per cell (one workgroup per cell): mu by
// SMEAR_ITERS bisections of [min eps - 40 sigma, max eps + 40 sigma] on the
// electron count (fixed-order sums), f = 2 / (1 + exp((eps - mu) / sigma));
// E[c * stride + 0] = sigma S, E[c * stride + 1] = mu.
constexpr int SMEAR_ITERS = 200;
constexpr double SMEAR_BRACKET = 40.0;
__global__ void k_fermi(const CellDesc* cells, const Seg* seg, const double* eig, double sigma, double* f, double* E,
                        int stride, int* status);

__global__ void k_cg_precond_dots(const Seg* seg, int nitems, const double2* g, const double2* gp,
                                  const double2* Dp, double2* Kg, double* part);
__global__ void k_trace_diag(const Seg* seg, const double2* M, double* out);

// blas.hip: per-item Cholesky inverse, eigensolver, fused line search and
// small-matrix products
__global__ void k_smm_mfma(const Seg* seg, int nbo, int opA, int opB, double alpha0, int alpha_omega,
                           const double2* A, const double2* B, double beta, double2* Cm);
constexpr int EIGW_MAXN = 32;  // largest matrix of the single-wave eigensolver
constexpr int EIG_TILE_MAXN = 128;  // largest matrix of the register-tile kernels (dense.hip)
// A Cholesky pivot R_jj^2 at or below this fraction of the largest diagonal
// entry of U counts as "not positive definite".
constexpr double PIVOT_RTOL = 1e-14;
// Single-wave Cholesky inverse and line search for n <= 32 (false: n larger).
bool cholesky_wave_launch(hipStream_t st, unsigned nblk, int n, int64_t stride, const Seg* seg, int nbo,
                          const double2* U, double2* Rinv, int* status, const int* act);
// Cholesky inverse, U^{-1}, M2 = -Omega U^{-1} H0 U^{-1} and E0 = Re Tr(U^{-1} H0)
// per item in one launch for up to 32 bands (false: larger); with `step`, U
// and H0 are first advanced along the line matrices X, Q, H1, H2.
bool grad_prep_wave_launch(hipStream_t st, unsigned nblk, int nmax, const Seg* seg, double2* U, double2* H0,
                           double2* Rinv, double2* M1, double2* M2, double* E0, int* status, const double* step,
                           const double2* X, const double2* Q, const double2* H1, const double2* H2);
bool linesearch_wave_launch(hipStream_t st, unsigned nblk, int n, const Seg* seg, const double2* U,
                            const double2* X, const double2* Q, const double2* H0, const double2* H1,
                            const double2* H2, const double* E0v, const double* at0, const double* d0v,
                            const int* act, int* ok, double* step, double2* Xs, double2* Ps);
// Single-wave eigensolver for up to 32 bands (false: larger).
bool eigh_wave_launch(hipStream_t st, unsigned nblk, int nmax, const Seg* seg, const double2* H, double* eig,
                      double2* vecs);

// dense.hip: register-tile kernels for 33..128 bands (one workgroup per
// matrix; seg == nullptr: `nmat` matrices of order n0 at stride n0^2).
hipError_t cholesky_tiles_launch(hipStream_t st, unsigned nmat, int nmax, const Seg* seg, int nbo, int n0,
                                 const double2* U, double2* Rinv, int* status, const int* act);
// M1 = U^{-1} and E0 = Re Tr(U^{-1} H0) (no R^{-1}); with `step`, U and H0
// first advanced along the line matrices (as grad_prep_wave_launch).
hipError_t grad_prep_tiles_launch(hipStream_t st, unsigned nit, int nmax, const Seg* seg, double2* U, double2* H0,
                                  double2* M1, double* E0, int* status, const double* step, const double2* X,
                                  const double2* Q, const double2* H1, const double2* H2);
hipError_t linesearch_tiles_launch(hipStream_t st, unsigned nit, int nmax, const Seg* seg, const double2* U,
                                   const double2* X, const double2* Q, const double2* H0, const double2* H1,
                                   const double2* H2, const double* E0v, const double* at0, const double* d0v,
                                   const int* act, int* ok, double* step);
// Eigen-decomposition (ascending eigenvalues, eigenvectors as columns): ws
// holds eigh_tiles_ws_bytes(sum of n^2) bytes (per matrix at 10 * moff
// double2), perm eigh_perm_bytes(nmat).
hipError_t eigh_tiles_launch(hipStream_t st, unsigned nmat, int nmax, const Seg* seg, int n0, const double2* H,
                             double* eig, double2* vecs, double2* ws, int* perm);
size_t eigh_tiles_ws_bytes(int64_t n2sum);
size_t eigh_perm_bytes(int nmat);

}  // namespace dpp
