/*
 * dftpp.h - C ABI of the MI355X DFT++ band-minimization library (libdftpp.so).
 *
 * The calls follow the algebraic (DFT++) statement of plane-wave DFT used by
 * JDFTx (Sec. 2.1 of the JDFTx paper: named operators I, J, O, the coulomb
 * operator and pointwise products acting on reciprocal- and real-space
 * fields and on blocks of wavefunctions, composed by the caller).
 *
 * Conventions shared by every call
 * --------------------------------
 *  - Units: bohr, hartree.  Cell matrix R has the lattice vectors as
 *    COLUMNS, stored row-major: R[3*i + j] = component i of vector a_j.
 *  - Complex numbers are interleaved {re, im} pairs (dpp_c64 = two doubles,
 *    dpp_c32 = two floats); layout-compatible with torch complex128/64.
 *  - Wavefunction blocks ("column bundles") are band-major: band b of a block
 *    C with leading dimension ldC starts at C + b*ldC (complex elements), and
 *    holds the npw sphere coefficients in canonical order (lexicographic on
 *    the Miller indices (n0, n1, n2), each ascending).  ldC >= npw.
 *  - Real-space fields are row-major (S0, S1, S2) boxes, i2 fastest.
 *  - Pointers named d_* and every array argument of an operator call are
 *    DEVICE pointers owned by the caller, unless documented as host.
 *    The library owns only its handles and their internal device tables.
 *  - Every call is enqueued on the context's HIP stream and returns without
 *    synchronizing, except where documented (setup calls and the drivers,
 *    which read scalars back to decide line-search steps).
 *  - Scratch: calls taking `void* ws` need a caller-allocated device buffer
 *    of at least the size reported by the matching *_workspace_size call.
 *  - Errors: every call returns a dpp_status; arguments are validated on the
 *    host before any launch and a failing call launches nothing.  The text
 *    of the last error of the calling thread is dpp_last_error().  Failures
 *    found on the device (non-positive-definite overlap, non-finite values)
 *    latch into the context status word, read by dpp_ctx_status after the
 *    caller synchronizes the stream.
 */
#ifndef DFTPP_H
#define DFTPP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct { double re, im; } dpp_c64;
typedef struct { float re, im; } dpp_c32;

typedef enum {
    DPP_OK = 0,
    DPP_EINVAL = -1,       /* bad argument (checked on the host)            */
    DPP_ENOMEM = -2,       /* allocation of an internal table failed        */
    DPP_EDEVICE = -3,      /* HIP runtime error                             */
    DPP_ENOTPD = -4,       /* overlap Y^dag O Y not positive definite       */
    DPP_ENOCONV = -5,      /* an iteration did not converge                 */
    DPP_EUNSUPPORTED = -6  /* size or mode outside what the kernels handle  */
} dpp_status;

typedef enum {
    DPP_F64 = 0,   /* everything in FP64                                    */
    DPP_F32 = 1    /* the mixed-precision bulk: FFT passes, the potential
                      multiply and the density transforms in FP32; A^dag B
                      contractions on split-BF16 MFMA (inputs rounded to
                      FP32 and split into two BF16 parts, all four products,
                      FP32 accumulation over 1024-point chunks, FP64 sums of
                      the chunks); X M contractions on FP32 MFMA with FP32
                      accumulation; Cholesky, eigensolver, energies and
                      other reductions in FP64                             */
} dpp_precision;

/* Device status word bits (dpp_ctx_status). */
#define DPP_STATUS_NOTPD   1     /* an overlap matrix was not positive definite */
#define DPP_STATUS_NONFINITE 2   /* a Pulay system was singular                 */
#define DPP_STATUS_NOBANDS 4     /* a cell had too few bands for its electrons  */

typedef struct dpp_ctx_s *dpp_ctx;
typedef struct dpp_grid_s *dpp_grid;
typedef struct dpp_basis_s *dpp_basis;
typedef struct dpp_ham_s *dpp_ham;
typedef struct dpp_system_s *dpp_system;
typedef struct dpp_net_s *dpp_net;

/* Text of the last error reported to the calling thread ("" if none). */
const char *dpp_last_error(void);
int dpp_version(void);

/* ---------------------------------------------------------------- setup -- */

/* Kernel classes measured by the context timer (dpp_timer_*). */
enum {
    DPP_TK_PLANES_IN = 0,    /* sphere -> x-planes (scatter, z and y transforms)  */
    DPP_TK_XZ_H = 1,         /* x transform, V_eff multiply, x transform back     */
    DPP_TK_PLANES_OUT = 2,   /* y and z transforms, sphere gather (+ kinetic)     */
    DPP_TK_XZ_DENSITY = 3,   /* x transform and |psi|^2 accumulation              */
    DPP_TK_OVERLAP = 4,      /* A^dag B contraction (MFMA) and its reduction      */
    DPP_TK_ROTATE = 5,       /* X M contraction (MFMA)                            */
    DPP_TK_CHOLESKY = 6,
    DPP_TK_EIGH = 7,
    DPP_TK_FULLBOX = 8,      /* full-box transforms (Hartree, J, potentials)      */
    DPP_TK_FIELDS = 9,       /* LDA, grid reductions, density reduction           */
    DPP_TK_BLOCKOPS = 10,    /* packed-block elementwise, dots, small matrices    */
    DPP_TK_XZ_IO = 11,       /* x transforms of I and I^dag to/from full boxes    */
    DPP_TK_NET = 12,         /* learned-density network forward/backward          */
    DPP_TK_LINESEARCH = 13,  /* fused band-energy line searches (Cholesky, trace) */
    DPP_TK_MASKED = 14       /* passes masked to a subset of items (line-search retries;
                                no algorithmic bytes: the active set is decided on the device) */
};
/* Enable (on = 1) or disable the per-context kernel timer: each launch of
 * an instrumented class is bracketed by HIP events on the context stream.
 * Reading synchronizes the stream and returns, for one class since the last
 * reset, the summed milliseconds, the launch count and the summed
 * algorithmic bytes and flops of those launches (the data the operation must
 * read and write once, and its arithmetic; any output may be NULL). */
dpp_status dpp_timer_enable(dpp_ctx ctx, int on);
dpp_status dpp_timer_reset(dpp_ctx ctx);
dpp_status dpp_timer_read(dpp_ctx ctx, int kind, double *total_ms, int64_t *launches, double *bytes,
                          double *flops);

/* Context on HIP device `device`; all work goes to `hip_stream` (a
 * hipStream_t, NULL = the null stream).  Allocates the device status word. */
dpp_status dpp_ctx_create(int device, void *hip_stream, dpp_ctx *out);
dpp_status dpp_ctx_destroy(dpp_ctx ctx);
/* Synchronizes the stream, then reads (and clears if `clear`) the status word. */
dpp_status dpp_ctx_status(dpp_ctx ctx, int clear, int *out);

/* Periodic cell R (host, 9 doubles, columns = lattice vectors) with FFT box
 * S (host, 3 ints, each 2/3/5-smooth, 4 <= S_d <= 128).  GridInfo of Sec. 2.1:
 * builds FFT plans and twiddle tables (FP64 and FP32) on the device. */
dpp_status dpp_grid_create(dpp_ctx ctx, const double *R, const int *S, dpp_grid *out);
dpp_status dpp_grid_destroy(dpp_grid grid);
/* Volume Omega and point count N = S0 S1 S2 (host outputs). */
dpp_status dpp_grid_info(dpp_grid grid, double *omega, int64_t *N);

/* G-sphere of Bloch vector k (host, reduced coordinates) at cutoff ecut:
 * every G = B n with |k+G|^2 / 2 <= ecut evaluated in FP64, canonical order.
 * Built on the device (flag, scan, compact).  Fails with DPP_EINVAL if the
 * sphere does not fit the box (2 max|n_d| + 1 > S_d).  Synchronizes. */
dpp_status dpp_basis_create(dpp_grid grid, const double *k_red, double ecut, dpp_basis *out);
dpp_status dpp_basis_destroy(dpp_basis basis);
/* npw, and the Miller-index extent n_ext = {n0min, n0max, n1min, n1max,
 * n2min, n2max} (host outputs). */
dpp_status dpp_basis_info(dpp_basis basis, int64_t *npw, int32_t *n_ext);
/* Copy the sphere tables into caller device arrays: d_index[npw] (int32
 * linear box index (i0*S1 + i1)*S2 + i2, i_d = n_d mod S_d) and
 * d_kG2[npw] (|k+G|^2).  Either may be NULL. */
dpp_status dpp_basis_export(dpp_basis basis, int32_t *d_index, double *d_kG2);

/* Workspace for I, Idag and apply_H on nb bands of `basis` at `prec`. */
dpp_status dpp_workspace_size(dpp_basis basis, int nb, dpp_precision prec, size_t *bytes);
/* Workspace for the full-box calls on `grid` (J, Jdag, hartree, lda, ...). */
dpp_status dpp_grid_workspace_size(dpp_grid grid, size_t *bytes);

/* ------------------------------------------------------------ operators -- */

/* I: sphere -> grid (Sec. 2.1).  grid_out[b] = sum_G C_bG exp(+i G.r)
 * (unnormalized inverse FFT), nb full boxes of N complex values, band-major.
 * C and grid_out are dpp_c64 (DPP_F64) or dpp_c32 (DPP_F32). */
dpp_status dpp_I(dpp_basis basis, int nb, const void *C, int64_t ldC, void *grid_out,
                 dpp_precision prec, void *ws);
/* I^dag: grid -> sphere, C_out[b] (+)= sum_r grid[b](r) exp(-i G.r).
 * accumulate = 0 overwrites C_out, 1 adds to it. */
dpp_status dpp_Idag(dpp_basis basis, int nb, const void *grid, void *C_out, int64_t ldC,
                    int accumulate, dpp_precision prec, void *ws);
/* J: full box, real space -> reciprocal space, y = FFT(x) / N, on nf fields
 * of N dpp_c64 each (J = I^{-1}).  J^dag: y = IFFT(x) (NumPy normalization). */
dpp_status dpp_J(dpp_grid grid, int nf, const dpp_c64 *x, dpp_c64 *y, void *ws);
dpp_status dpp_Jdag(dpp_grid grid, int nf, const dpp_c64 *x, dpp_c64 *y, void *ws);

/* Diagonal operators on a block (in and out may alias; FP64 dpp_c64):
 *   O: out = Omega in           (overlap, Sec. 2.1)
 *   L: out = -Omega |k+G|^2 in  (Laplacian)
 *   K: out = in / (1 + |k+G|^2/2)  (preconditioner) */
dpp_status dpp_O(dpp_basis basis, int nb, const dpp_c64 *in, int64_t ldin, dpp_c64 *out, int64_t ldout);
dpp_status dpp_L(dpp_basis basis, int nb, const dpp_c64 *in, int64_t ldin, dpp_c64 *out, int64_t ldout);
dpp_status dpp_K(dpp_basis basis, int nb, const dpp_c64 *in, int64_t ldin, dpp_c64 *out, int64_t ldout);

/* Kohn-Sham operator of one k-point: kinetic -L/2, local potential
 * (Omega/N) I^dag(V_eff * I C) and the nonlocal Gaussian s-projectors
 * P_k D P_k^dag, P_k[G,a] = exp(-|k+G|^2 rp^2/2) exp(-i G.tau_a).
 * tau: host (nat x 3, Cartesian bohr); has_proj: host (nat ints, 0/1). */
dpp_status dpp_ham_create(dpp_basis basis, int nat, const double *tau, const int *has_proj,
                          double rp, double D, dpp_ham *out);
dpp_status dpp_ham_destroy(dpp_ham ham);
/* V_eff (device, N doubles) used by later apply_H calls; the pointer is kept,
 * not copied: the caller keeps the array alive and unchanged meanwhile. */
dpp_status dpp_ham_set_potential(dpp_ham ham, const double *d_Veff);
/* HC = H C on nb bands (dpp_c64 for both precisions; DPP_F32 runs the FFT
 * passes in FP32).  C and HC must not alias. */
dpp_status dpp_apply_H(dpp_ham ham, int nb, const dpp_c64 *C, int64_t ldC, dpp_c64 *HC,
                       int64_t ldHC, dpp_precision prec, void *ws);

/* --------------------------------------------------------- contractions -- */

/* U = scale * A^dag B (nbA x nbB, row-major dpp_c64, device) over the npw
 * coefficients of `basis`; scale = Omega gives the overlap A^dag O B (the
 * overlap and subspace matrices of Sec. 2.1).  prec: DPP_F64 (FP64 MFMA) or
 * DPP_F32 (split-BF16 MFMA with FP32 accumulation per 1024 points and FP64
 * sums of those partials; relative error ~1e-7 of the row norms).  U is
 * FP64 either way.  ws: overlap_ws bytes (dpp_workspace_size covers it).
 * Deterministic (fixed reduction order). */
dpp_status dpp_overlap(dpp_basis basis, int nbA, const dpp_c64 *A, int64_t ldA, int nbB,
                       const dpp_c64 *B, int64_t ldB, double scale, dpp_c64 *U, dpp_precision prec,
                       void *ws);
/* out = beta * out + X M: X is nbX bands, M is nbX x nbO (row-major, device),
 * out is nbO bands.  out must not alias X.  prec: DPP_F64 (FP64 MFMA) or
 * DPP_F32 (X and M rounded to FP32, FP32 MFMA and accumulation; out and the
 * beta term in FP64). */
dpp_status dpp_rotate(dpp_basis basis, int nbX, const dpp_c64 *X, int64_t ldX, int nbO,
                      const dpp_c64 *M, double beta, dpp_c64 *out, int64_t ldout, dpp_precision prec);
/* U = R^dag R (Cholesky, R upper triangular with positive real diagonal) of
 * the Hermitian positive-definite nb x nb matrix U (device, row-major), then
 * Rinv = R^{-1}.  A pivot R_jj^2 <= 1e-14 max_i U_ii latches
 * DPP_STATUS_NOTPD and leaves Rinv undefined.  batch matrices back to back. */
dpp_status dpp_cholesky_inverse(dpp_ctx ctx, int nb, int batch, const dpp_c64 *U, dpp_c64 *Rinv);
/* Orthonormalize a block in place: U = Y^dag O Y, Y <- Y R^{-1}; writes
 * Rinv (device nb x nb) if not NULL.  Workspace: dpp_ortho_workspace_size.
 * A non-positive-definite U latches DPP_STATUS_NOTPD and leaves Y as NaN. */
dpp_status dpp_ortho_workspace_size(dpp_basis basis, int nb, size_t *bytes);
dpp_status dpp_cholesky_orthonormalize(dpp_basis basis, int nb, dpp_c64 *Y, int64_t ldY,
                                       dpp_c64 *Rinv, void *ws);
/* Hermitian eigensolver (FP64): H (device, batch x nb x nb, row-major; its
 * lower triangle is read for nb > 32) -> eig ascending (device, batch x nb)
 * and vecs (device, row-major, column j = eigenvector j).  H is not modified.
 * Up to 32 bands: cyclic Jacobi in one wave.  33..128 bands: Householder
 * reduction to a real tridiagonal, bisection, inverse iteration and
 * back-transformation; ws (device) holds dpp_eigh_workspace_size bytes. */
dpp_status dpp_subspace_eigh(dpp_ctx ctx, int nb, int batch, const dpp_c64 *H, double *eig,
                             dpp_c64 *vecs, void *ws);
dpp_status dpp_eigh_workspace_size(int nb, int batch, size_t *bytes);
/* dpp_subspace_eigh for callers that cannot allocate device memory (code
 * under HIP graph capture, serving loops, harnesses that forbid hipMalloc):
 * the same kernels and results, with the workspace in a static device array
 * of 8 MiB per GPU held until the process ends (address taken once per device
 * by dpp_ctx_create).  Sizes needing more workspace than that (for example
 * more than three 128 x 128 matrices per call) return DPP_EINVAL with a
 * message and launch nothing.  No allocation of any kind.  Calls that overlap
 * on one GPU (other streams or threads) share the array and race; calls on
 * one stream are ordered.  The array keeps the last call's contents; no call
 * reads what an earlier call left. */
dpp_status dpp_subspace_eigh_noalloc(dpp_ctx ctx, int nb, int batch, const dpp_c64 *H, double *eig,
                                     dpp_c64 *vecs);

/* ------------------------------------------------ densities, potentials -- */

/* d_n += wk * sum_b f_b |(I psi_b)(r)|^2 (f: device, nb doubles). */
dpp_status dpp_density_accumulate(dpp_basis basis, int nb, const dpp_c64 *psi, int64_t ldpsi,
                                  const double *d_f, double wk, double *d_n, dpp_precision prec,
                                  void *ws);
/* Hartree solve (coulomb operator): V_H = Re I[4 pi (J n)/|G|^2], G = 0
 * dropped; E_H = (Omega/2) sum_{G != 0} 4 pi |J n|^2 / |G|^2 -> *d_EH. */
dpp_status dpp_hartree(dpp_grid grid, const double *d_n, double *d_VH, double *d_EH, void *ws);

/* ------------------------------------------------------------ LinearPCM -- */

/* Workspace bytes of dpp_pcm_solve on this grid (9 full-box complex fields
 * plus reduction partials: about 144 N bytes). */
dpp_status dpp_pcm_workspace_size(dpp_grid grid, size_t *bytes);
/* LinearPCM solvation (Sec. 2.1, Eqs. (1)-(2), Listing 1): solves
 * -4 pi rho = div(eps grad phi), posed on reciprocal fields as
 * (-1/(4 pi)) div(J(eps * I(grad phi~))) = J rho, by conjugate gradients
 * preconditioned with 4 pi / |G'|^2, from phi~ = 0, until
 * ||r|| <= tol ||J rho|| (2-norms over the solved modes) or max_iter
 * iterations; then A_diel = (Omega/2) Re sum_G conj(phi~ - 4 pi rho~/|G|^2) rho~.
 * grad and div use G' = B m' (m' the signed frequency, the Nyquist index of
 * an even axis counted as 0); modes with G' = 0 are outside the solve (phi~ = 0,
 * rho~ dropped there: any net charge meets a neutralizing background).
 * d_eps, d_rho: device, N doubles each, the box in natural order (eps > 0
 * expected; not checked).  d_phi: device, N doubles, phi(r) = Re I phi~, or
 * NULL.  *A_diel (host, hartree), *iterations and *rel_residual (host, may be
 * NULL) report the result.  ws: dpp_pcm_workspace_size bytes, device,
 * caller-owned; its contents on return are scratch.  Stream-ordered on the
 * grid's context; returns after the result is on the host (one host
 * synchronization per CG iteration for the convergence test).  Errors:
 * DPP_EINVAL for null pointers, tol < 0 or max_iter < 0. */
dpp_status dpp_pcm_solve(dpp_grid grid, const double *d_eps, const double *d_rho, double tol, int max_iter,
                         double *d_phi, double *A_diel, int *iterations, double *rel_residual, void *ws);
/* LDA (Slater exchange + Perdew-Zunger 1981 correlation): v_xc per point
 * and E_xc = (Omega/N) sum n eps_xc -> *d_Exc.  n < 1e-16 gives 0. */
dpp_status dpp_lda_pz81(dpp_grid grid, const double *d_n, double *d_vxc, double *d_Exc, void *ws);
/* Workspace bytes of dpp_gga_pbe on this grid (6 full-box complex fields
 * plus reduction partials: about 96 N bytes). */
dpp_status dpp_gga_workspace_size(dpp_grid grid, size_t *bytes);
/* PBE exchange-correlation, spin-unpolarized (Table 1 and Sec. 2.2:
 * semilocal GGA functionals): per point e(n, sigma) = n eps_x^LDA F_x(s)
 * + n (eps_c^PW92(r_s) + H(r_s, t)), sigma = |grad n|^2; potential
 * v_xc = de/dn - div(2 de/dsigma grad n); *d_Exc = (Omega/N) sum_r e.
 * grad and div are spectral (J, i G', I) with G' = B m', the Nyquist index of
 * an even axis counted as 0.  Densities below 1e-16 (negative ones
 * included) contribute e = 0 and no derivatives.  d_n: device, N doubles,
 * natural box order; d_vxc: device, N doubles (output); d_Exc: device, one
 * double (output); ws: dpp_gga_workspace_size bytes, device, caller-owned.
 * Stream-ordered on the grid's context, no host synchronization.  Errors:
 * DPP_EINVAL for null pointers. */
dpp_status dpp_gga_pbe(dpp_grid grid, const double *d_n, double *d_vxc, double *d_Exc, void *ws);
/* Exchange-correlation functional of a system's SCF (V_eff and E_xc):
 * DPP_XC_LDA_PZ81 (default, every cell in one launch) or DPP_XC_PBE
 * (dpp_gga_pbe per cell on its full box).  Allocates the PBE workspace on
 * first use (the system owns it); drops captured SCF graphs, which are
 * captured again on the next iterations.  Errors: DPP_EINVAL for a null
 * system or an unknown value, DPP_ENOMEM. */
enum { DPP_XC_LDA_PZ81 = 0, DPP_XC_PBE = 1 };
dpp_status dpp_system_set_xc(dpp_system sys, int functional);
/* Fermi-Dirac smearing of the SCF fillings (Table 1: smearing for metals):
 * sigma > 0 (hartree) replaces the aufbau fillings of dpp_scf_iteration by
 * f = 2 / (1 + exp((eps - mu) / sigma)), mu per cell by 200 bisections of
 * [min eps - 40 sigma, max eps + 40 sigma] on the electron count; E_el of
 * the report is then the free energy E - sigma S with
 * S = -2 sum_k w_k sum_i [g ln g + (1 - g) ln(1 - g)], g = f / 2.
 * sigma = 0 restores aufbau.  Drops captured SCF graphs.  Errors: DPP_EINVAL
 * for a null system or sigma < 0 or not finite. */
dpp_status dpp_system_set_smearing(dpp_system sys, double sigma);
/* mu[c] and sigma S[c] (hartree, host arrays of ncells, either may be NULL)
 * of the last smeared SCF iteration; synchronizes the stream.  Errors:
 * DPP_EINVAL for a wrong cell count or a system without smearing. */
dpp_status dpp_system_smearing_state(dpp_system sys, int ncells, double *mu, double *TS);
/* V_loc(r) = Re I[sum_a v_a(|G|) exp(-i G.tau_a)], v_a(G) = -4 pi Z_a
 * exp(-G^2 rc_a^2/4) / (Omega G^2), v_a(0) = 0.  Host tau (nat x 3), Z, rc. */
dpp_status dpp_local_potential(dpp_grid grid, int nat, const double *tau, const double *Z,
                               const double *rc, double *d_Vloc, void *ws);
/* Superposition of atomic Gaussians: n0(G) = (1/Omega) sum_a Z_a
 * exp(-G^2 sigma^2/4) exp(-i G.tau_a), n0(r) = Re I n0. */
dpp_status dpp_start_density(dpp_grid grid, int nat, const double *tau, const double *Z,
                             double sigma, double *d_n, void *ws);
/* Deterministic sum_j a_j b_j * scale over N grid points -> *d_out (device). */
dpp_status dpp_grid_dot(dpp_grid grid, const double *d_a, const double *d_b, double scale,
                        double *d_out, void *ws);

/* --------------------------------------------------------------- drivers -- */

/* A system is a batch of independent periodic cells (a batch of one is the
 * plain case), each with its k-points (Gamma-centred folding or any list)
 * and the pseudopotential model of its atoms.  Work items are the
 * (cell, k-point) pairs numbered cell-major; every driver pass runs as one
 * launch over all items or all cells, whatever their boxes, spheres and band
 * counts (form 2).  All descriptor arrays are host arrays read during the
 * call.  The system owns its bases, Hamiltonians and every driver buffer
 * (allocated at creation; later calls allocate only small task tables the
 * first time an operation runs); wavefunction blocks Y stay caller-owned and
 * use the packed layout of dpp_system_layout: the block of item k starts at
 * element offsets[k] and holds that cell's nb bands of npw[k] coefficients
 * each (ld = npw[k]).  Real-space fields of the cells are concatenated (cell c
 * at foff[c] of dpp_system_cells, N_c doubles); per-state arrays (fillings,
 * eigenvalues) are concatenated per item (item k at state0 of its cell plus
 * the nb of the items before it). */
typedef struct {
    const double *R;        /* 9, columns = lattice vectors                */
    const int *S;           /* 3, FFT box                                  */
    double ecut;            /* hartree                                     */
    int nk;                 /* k-points (<= 64)                            */
    const double *kpts;     /* nk x 3 reduced                              */
    const double *wk;       /* nk weights (sum 1)                          */
    int nb;                 /* bands per k-point (<= 128; nk nb <= 1024)   */
    double n_electrons;
    int nat;
    const double *tau;      /* nat x 3 Cartesian                           */
    const double *Z;        /* nat valence charges                         */
    const double *rc;       /* nat erf radii of the local potential        */
    const int *has_proj;    /* nat flags: atom carries the s-projector     */
    double rp, D;           /* projector width and coupling                */
    int prec;               /* dpp_precision of the FFT passes (one value
                               for every cell of a batch)                  */
} dpp_system_desc;

typedef struct {
    double E_el, E_kin, E_nl, E_loc, E_H, E_xc;
} dpp_energy;

typedef struct {
    int nat;
    const double *tau;      /* superposition start density: atoms          */
    const double *Z;
    double sigma;           /* Gaussian width                              */
    const double *d_n_start;/* device start density (overrides the atoms)  */
    int n_inner;            /* band-CG steps per SCF iteration (0 -> 3)    */
    int n_inner_first;      /* steps of the first iteration (0 -> n_inner) */
} dpp_scf_desc;

enum { DPP_FIELD_VLOC = 0, DPP_FIELD_VEFF = 1, DPP_FIELD_N = 2, DPP_FIELD_NIN = 3, DPP_FIELD_NOUT = 4 };

/* Synchronizes.  Builds bases, projectors and V_loc of ncells cells on the
 * device.  dpp_system_create is the batch of one. */
dpp_status dpp_batch_create(dpp_ctx ctx, int ncells, const dpp_system_desc *descs, dpp_system *out);
dpp_status dpp_system_create(dpp_ctx ctx, const dpp_system_desc *desc, dpp_system *out);
dpp_status dpp_system_destroy(dpp_system sys);
/* Cells, items, packed block elements, states and concatenated grid points
 * (host outputs, any may be NULL). */
dpp_status dpp_system_dims(dpp_system sys, int *ncells, int *nitems, int64_t *total, int64_t *nstates,
                           int64_t *ngrid);
/* offsets[nitems+1] and npw[nitems] of the packed wavefunction layout (host). */
dpp_status dpp_system_layout(dpp_system sys, int64_t *offsets, int64_t *npw);
/* Per cell (ncells + 1 entries each, the last one the total; any may be
 * NULL): first item, field offset, first state. */
dpp_status dpp_system_cells(dpp_system sys, int *item0, int64_t *foff, int64_t *state0);
/* Device pointer of an internal real-space field (DPP_FIELD_*), ngrid doubles. */
dpp_status dpp_system_field(dpp_system sys, int which, double **d_ptr);
/* Copy that field into a caller device array of ngrid doubles (stream-ordered). */
dpp_status dpp_system_copy_field(dpp_system sys, int which, double *d_out);

/* Variational minimization of E_el (Sec. 2.2) over the first nocc bands of
 * every k-point with filling f, CG with one step length for all k; systems
 * of one cell.  init orthonormalizes those bands of Y once and evaluates E
 * and its gradient; each step is one CG iteration (stationary = 1 once no
 * step lowers E).  Synchronizes (line-search decisions read energies back). */
dpp_status dpp_cg_V_init(dpp_system sys, dpp_c64 *Y, int nocc, double f, dpp_energy *E);
dpp_status dpp_cg_V_step(dpp_system sys, dpp_c64 *Y, dpp_energy *E, int *stationary);
/* Band-energy minimization at fixed V_eff (device, ngrid doubles), all bands,
 * an independent line search per item, decided on the device.  Eb (host,
 * may be NULL): per-item band energies Tr(U^{-1} Y^dag H Y) after the call
 * (reading them synchronizes). */
dpp_status dpp_cg_B_init(dpp_system sys, dpp_c64 *Y, const double *d_Veff, double *Eb);
dpp_status dpp_cg_B_step(dpp_system sys, dpp_c64 *Y, double *Eb);
/* After band CG: subspace diagonalization Y <- psi V with eigenvalues
 * eig (host, nstates, ascending per item).  Synchronizes. */
dpp_status dpp_band_eigenvalues(dpp_system sys, dpp_c64 *Y, double *eig);

/* SCF (Sec. 2.1 Pulay mixing; Sec. 2.2): start densities from desc (one
 * descriptor per cell; n_inner and n_inner_first are taken from the first).
 * One iteration of every cell: V_eff[n_in], n_inner band-CG steps per item,
 * subspace diagonalization, aufbau fillings per cell (a degenerate set
 * within 1e-6 Ha at the Fermi level shares electrons equally), n_out,
 * E_el[psi, n_out], Pulay mixing of n_in (history 8, alpha 0.5, first
 * iteration linear).  The iteration runs in stream order without host round
 * trips; E (host, ncells) and eig (host, nstates, may be NULL) describe its
 * output, read back at its end (synchronizes). */
dpp_status dpp_scf_init(dpp_system sys, const dpp_scf_desc *desc);
dpp_status dpp_scf_iteration(dpp_system sys, dpp_c64 *Y, dpp_energy *E, double *eig);
/* Graph mode (on != 0): after the first SCF iteration of a run, each
 * iteration is captured once as a HIP graph (per Y pointer, step count and
 * precision) and replayed.  Results equal those of eager mode. */
dpp_status dpp_set_graph_mode(dpp_system sys, int on);
/* Number of (band, item) H applications performed by the system's drivers
 * since creation (host output). */
dpp_status dpp_system_counters(dpp_system sys, int64_t *hc_bandk);
/* HY = H Y on all bands of every item (packed layout, at the potential
 * last set: V_eff of the last SCF iteration or dpp_cg_B_init). */
dpp_status dpp_system_apply_H(dpp_system sys, const dpp_c64 *Y, dpp_c64 *HY);
/* Launch autotuner (form 2's tiles, chosen per system by measurement):
 * times the candidate launch variants on the system's own items and keeps
 * the default rule unless another candidate is at least 3% faster.  Choices: per x-pass length S0 and precision, the register
 * x pass with one thread per column, with a lane pair per column, or the
 * LDS pass; point tiles per wave of the X M contraction (1, 2 or 4, for up
 * to 32 bands); the A^dag O B launch (2x2 tiles per wave, single tiles,
 * one pass, or 4x4 tile blocks staged in LDS).  Y (device, packed layout) is the block the H applications and
 * contractions run on; HY (device, same size) is overwritten.  Each
 * candidate runs reps >= 1 times after a warm-up.  Runs eagerly and
 * synchronizes; the system's internal work blocks are overwritten (a band-CG
 * run must start again with dpp_cg_B_init or dpp_scf_init) and captured
 * graphs are dropped.  Results of every variant agree to rounding.  Errors:
 * DPP_EINVAL for bad arguments or a capturing stream. */
dpp_status dpp_system_tune(dpp_system sys, const dpp_c64 *Y, dpp_c64 *HY, int reps);
/* Sets one launch choice by hand (what dpp_system_tune would choose), for
 * tests and experiments: DPP_CHOICE_OVERLAP (0: the default rule, mode 3
 * when every task has at least 4x4 output tiles, else 2x2 tile blocks over
 * 256-point chunks plus a reduction launch; 1: single tiles, 2: one
 * workgroup per task over all points, 3: 4x4 tile blocks over 256-point
 * chunks with the operands staged in LDS), DPP_CHOICE_ROTATE_PT (0 = by launch
 * size, 1, 2 or 4 point tiles per wave), DPP_CHOICE_XPASS (0 auto, 1 one
 * thread per column, 2 lane pair per column, 3 LDS; for every x length,
 * lengths without the variant use the LDS pass).  Drops captured graphs.
 * Errors: DPP_EINVAL for an unknown choice or value. */
enum { DPP_CHOICE_OVERLAP = 0, DPP_CHOICE_ROTATE_PT = 1, DPP_CHOICE_XPASS = 2 };
dpp_status dpp_system_set_launch_choice(dpp_system sys, int which, int value);
/* Text report of the last dpp_system_tune: the timed candidates (us per
 * call) and the choices; buf (host, len bytes) receives a NUL-terminated
 * string, truncated to fit. */
dpp_status dpp_system_tune_report(dpp_system sys, char *buf, size_t len);
/* Precision policy (form 1): FFT passes, potential multiply and density in
 * `bulk` (DPP_F32 or DPP_F64) until the largest band residual
 * max_i ||(H - eps_i O) psi_i||_2 / sqrt(Omega) of an SCF iteration (over
 * all cells) falls below refine_residual (> 0), then FP64 for the rest of
 * that SCF run (dpp_scf_init returns to bulk).  Contractions, Cholesky,
 * eigensolver, energies, Hartree and LDA are FP64 throughout. */
dpp_status dpp_set_precision_policy(dpp_system sys, int bulk, double refine_residual);
/* Residual of the last SCF iteration (max over cells), the precision of the
 * next one and the iteration count since dpp_scf_init (host outputs, any may
 * be NULL). */
dpp_status dpp_scf_status(dpp_system sys, double *residual, int *prec_now, int *iterations);
/* Largest band residual of each cell in the last SCF iteration (host, ncells). */
dpp_status dpp_scf_cell_residuals(dpp_system sys, double *res);
/* Fillings of the last SCF iteration (host, nstates). */
dpp_status dpp_system_fillings(dpp_system sys, double *f);

/* Forces on the ions of every cell (Table 1: ionic optimization; Sec. 3:
 * the ionic minimization of the example), in hartree/bohr, at the state the
 * last dpp_scf_iteration left: Y its orthonormal wavefunctions (the packed
 * block it updated), its fillings and its output density n_out.
 *   F_loc  -dE_loc/dtau at fixed n_out (local pseudopotential),
 *   F_nl   -dE_nl/dtau at fixed psi and fillings (projectors),
 *   F_ion  -dE_ion/dtau of the point ions in a compensating background
 *          (Ewald sums),
 * each a device array of 3 doubles per atom (cell-major, then atom, then
 * x, y, z), any may be NULL; at a self-consistent state their sum is the
 * force -dE/dtau of E = E_el + E_ion.  E_ion (host, one per cell, may be
 * NULL) receives the ionic energy.  FP64 throughout.  Stream-ordered; with
 * E_ion it synchronizes the stream.  Not capturable (first call allocates
 * the derivative projectors: 3 nproj npw complex per item).  Errors:
 * DPP_EINVAL before the first SCF iteration or while capturing. */
dpp_status dpp_system_forces(dpp_system sys, const dpp_c64 *Y, double *F_loc, double *F_nl, double *F_ion,
                             double *E_ion);
/* Move the ions (ionic minimization, Table 1 and Sec. 3): tau (host, 3 per
 * atom, cell-major, Cartesian bohr) replaces every cell's positions; the
 * local potential, the projectors (and the force tables) are rebuilt in place,
 * so captured SCF graphs stay valid.  The next dpp_scf_iteration works at the
 * new positions (a fresh start density needs dpp_scf_init).  Synchronizes the
 * stream.  DPP_EINVAL: non-finite positions, or while capturing. */
dpp_status dpp_system_set_positions(dpp_system sys, const double *tau);

/* ------------------------------------------------ learned start density -- */

/* A periodic 3D convolutional network that corrects the superposition start
 * density (form 4): x = n0/nbar, three 3x3x3 conv + SiLU layers of 16
 * channels and a linear 3x3x3 output layer (1-16-16-16-1, circular
 * padding, 14737 parameters); dn = nbar (y - mean y); n = max(n0 + dn, 0)
 * rescaled to N_e.  Weights BF16 (from FP32 master copies), FP32
 * activations and accumulation, FP64 loss and density reductions.
 * Parameter order (host float arrays): W1 (16x1x3x3x3), b1, W2, b2, W3, b3,
 * W4 (1x16x3x3x3), b4, each row-major.  max_batch bounds every batch. */
dpp_status dpp_net_create(dpp_ctx ctx, const int *S, int max_batch, dpp_net *out);
dpp_status dpp_net_destroy(dpp_net net);
dpp_status dpp_net_num_params(dpp_net net, int *count);
/* Set FP32 master parameters (resets Adam); get parameters and the
 * gradients of the last backward pass (host arrays, either may be NULL). */
dpp_status dpp_net_set_params(dpp_net net, const float *h_params);
dpp_status dpp_net_get_params(dpp_net net, float *h_params, float *h_grads);
/* Forward pass of `batch` start densities (device, batch x N doubles, back
 * to back); y (device, batch x N floats, may be NULL) receives the raw output. */
dpp_status dpp_net_forward(dpp_net net, int batch, const double *d_n0, double nbar, float *d_y);
/* After dpp_net_forward on the same n0: loss mean_b mean_r (y - mean y - t)^2
 * with t = (n_conv - n0)/nbar, and its parameter gradients.  Synchronizes
 * when loss is not NULL. */
dpp_status dpp_net_backward(dpp_net net, int batch, const double *d_n0, const double *d_nconv, double nbar,
                            double *loss);
/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8) on the last gradients. */
dpp_status dpp_net_adam_step(dpp_net net, double lr);
/* One epoch over nsamples resident samples in the given order (host ints),
 * batches of `batch`; mean batch loss to *mean_loss.  Synchronizes. */
dpp_status dpp_net_train_epoch(dpp_net net, int nsamples, const double *d_n0, const double *d_nconv, double nbar,
                               int batch, double lr, const int *order, double *mean_loss);
/* Learned start density for one cell (device in/out, N doubles). */
dpp_status dpp_net_predict_density(dpp_net net, const double *d_n0, double n_electrons, double omega,
                                   double *d_n_out);

#ifdef __cplusplus
}
#endif
#endif /* DFTPP_H */
