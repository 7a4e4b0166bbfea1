// Minimization and SCF drivers over one periodic system (a cell with its
// k-points): preconditioned Polak-Ribiere CG for the total energy
// (variational minimization, one shared step length) and for the band
// energy at fixed potential (one line search per k-point), and the SCF
// iteration with subspace diagonalization, aufbau fillings and Pulay mixing.
// (Sec. 2.1: Minimize and Pulay; Sec. 2.2: variational minimization vs SCF.)
//
// The host runs only the control flow of the line searches (comparisons of
// scalar energies read back from the device) and the aufbau bookkeeping; every
// arithmetic step runs in the library's kernels.  Step rules:
//   direction  D = -K g + beta D_prev, beta = max(0, <g - g_prev, K g> / <g_prev, K g_prev>),
//              beta = 0 on the first step and after a failed line search,
//              D = -K g if <g, D> >= 0;  <A, B> = sum_k 2 Re Tr(A_k^dag B_k)
//   line       trial a_t (first 0.3/s, then the last accepted step); fit
//              E0 + d0 a + c a^2 through E(a_t); a* = -d0/(2c) if c > 0 else
//              2 a_t, at most 10 a_t; accept a* if E(a*) <= E0, else a_t if
//              E(a_t) <= E0, else halve a_t (at most 6 tries); on failure one
//              more search along -K g, then stationary.
// Band-energy line searches use H(Y + a D) = HY + a HD: the trial energies
// Tr(U(a)^{-1} Y(a)^dag H Y(a)) come from six nb x nb matrices per k-point.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "blockops.h"
#include "internal.h"
#include "../../include/dftpp.h"

using namespace dpp;

namespace {
constexpr int MAX_TRIES = 6;
constexpr double DEGEN_TOL = 1e-6;
}  // namespace

struct dpp_system_s {
    dpp_ctx ctx;
    dpp_grid grid;
    int nk, nb, nat;
    double ne;
    double D;  // projector coupling
    int nproj;
    std::vector<dpp_basis> bases;
    std::vector<dpp_ham> hams;
    std::vector<double> wk;
    std::vector<int64_t> off, npw;
    int64_t total;  // complex elements of one packed block set (nb bands)
    Seg* d_seg;
    double* d_wk;
    // block buffers (total elements each)
    double2 *HY, *Dd, *HD, *g, *g2, *Kg, *gp, *Kgp, *Dp, *psi, *T1, *T2;
    // small matrices, nk x nb x nb each
    double2 *U, *Rinv, *H0, *X, *Q, *H1, *H2, *Ua, *Ha, *Rt, *M1, *M2, *vecs, *Pi;
    int64_t pi_stride;
    // scalars
    double *d_dots, *d_part, *d_alpha, *d_ones, *d_beta, *d_E, *d_f, *d_eig, *d_trial;
    // grids
    double *Vloc, *VH, *vxc, *Veff, *n, *nin, *nout, *pulayA, *pulayC;
    double* hist_nin[PULAY_MAX];
    double* hist_res[PULAY_MAX];
    int hist_m, hist_head;
    std::vector<double> pulayA_h;  // m x m residual overlaps (host mirror of the device matrix)
    int scf_iter;
    // workspaces
    void* ws;
    size_t ws_bytes;
    void* gws;
    void* eigws;
    // CG state (band energy, per k)
    std::vector<double> bE0, bat, bgkg;
    std::vector<int> breset, bstat;
    // CG state (total energy)
    double vE0, vat, vgkg;
    int vreset, vstat, vnocc;
    double vf;
    std::vector<double> fill;  // host fillings nk x nb
    int n_inner_steps;
    int n_inner_first;
    int64_t hc_bandk;          // H applications counted in (band, k) pairs
    // precision policy: bulk precision of the FFT passes until the band
    // residual falls below refine_res, FP64 afterwards (per SCF run)
    dpp_precision bulk_prec;
    double refine_res;
    double last_res;
    double* d_res;
    dpp_precision prec;
    std::vector<void*> allocs;
    // pinned staging ring for small host -> device uploads; a slot is reused
    // only after a stream synchronization
    double* h_ring;
    int ring_slot, ring_slots;
    size_t ring_len;
    // batched launches: FFT item tables (all nb bands; nocc bands for the
    // total-energy CG), task tables and the overlap partial buffer
    FftItem* d_items_nb;
    FftItem* d_items_occ;
    std::vector<FftItem> h_items_nb, h_items_occ;
    int items_occ_nb;
    char* d_tab;            // device task table region (reused in stream order)
    size_t tab_bytes;
    char* h_tab;            // pinned staging ring for task tables
    int tab_slot, tab_slots;
    double2* ov_part;
    size_t ov_part_elems;
    double* dens_part;
    int dens_nch;
    void* Tplanes;          // plane buffer of every k-point
};

namespace {

dpp_status dalloc(dpp_system_s* s, void** p, size_t bytes) {
    if (hipMalloc(p, std::max<size_t>(bytes, 256)) != hipSuccess)
        return set_error(DPP_ENOMEM, "dpp_system_create: device allocation failed");
    s->allocs.push_back(*p);
    return DPP_OK;
}
template <typename T>
dpp_status dalloc_t(dpp_system_s* s, T** p, size_t count) {
    return dalloc(s, reinterpret_cast<void**>(p), count * sizeof(T));
}

unsigned seg_blocks(const dpp_system_s* s, int nb) {
    int64_t mx = 0;
    for (int k = 0; k < s->nk; ++k) mx = std::max<int64_t>(mx, nb * s->npw[k]);
    return (unsigned)std::min<int64_t>(1024, std::max<int64_t>(1, (mx + 255) / 256));
}

hipStream_t stream(const dpp_system_s* s) { return s->ctx->stream; }

// ---------------------------------------------------------- batched ops ---
dpp_status upload_table(dpp_system_s* s, const void* src, size_t bytes, void** dev) {
    if (bytes > s->tab_bytes) return set_error(DPP_EUNSUPPORTED, "task table too large");
    if (s->tab_slot == s->tab_slots) {
        DPP_HIP(hipStreamSynchronize(stream(s)));
        s->tab_slot = 0;
    }
    char* slot = s->h_tab + (size_t)s->tab_slot * s->tab_bytes;
    s->tab_slot++;
    std::memcpy(slot, src, bytes);
    DPP_HIP(hipMemcpyAsync(s->d_tab, slot, bytes, hipMemcpyHostToDevice, stream(s)));
    *dev = s->d_tab;
    return DPP_OK;
}

struct OvJob {
    int nbA;
    const double2* A;   // packed block set
    int nbB;
    const double2* B;
    double scale;
    double2* out;       // nk matrices at stride nb^2
};

// Several A^dag B contractions over every k-point in one launch.
dpp_status overlap_jobs(dpp_system_s* s, const std::vector<OvJob>& jobs) {
    std::vector<OvTask> t;
    int64_t poff = 0;
    for (const OvJob& j : jobs)
        for (int k = 0; k < s->nk; ++k) {
            OvTask x = make_ov_task((int)s->npw[k], j.nbA, j.A + s->off[k], s->npw[k], j.nbB, j.B + s->off[k],
                                    s->npw[k], j.scale, j.out + (int64_t)k * s->nb * s->nb, j.nbB);
            x.part_off = poff;
            poff += (int64_t)x.nchunk * x.ntiles * 256;
            t.push_back(x);
        }
    if ((size_t)poff > s->ov_part_elems) return set_error(DPP_EUNSUPPORTED, "overlap partial buffer too small");
    void* d = nullptr;
    DPP_TRY(upload_table(s, t.data(), t.size() * sizeof(OvTask), &d));
    return overlap_tasks(s->ctx, t, (const OvTask*)d, s->ov_part);
}

// out_k (stride nb^2) = scale A_k^dag B_k
dpp_status overlap_all(dpp_system_s* s, int nbA, const double2* A, int nbB, const double2* B, double scale,
                       double2* out) {
    return overlap_jobs(s, {OvJob{nbA, A, nbB, B, scale, out}});
}

struct RotJob {
    int nbX;
    const double2* X;
    int nbO;
    const double2* M;   // nk matrices at stride nb^2 (row length nbO)
    double beta;
    double2* out;
};

dpp_status rotate_jobs(dpp_system_s* s, const std::vector<RotJob>& jobs) {
    std::vector<RotTask> t;
    for (const RotJob& j : jobs)
        for (int k = 0; k < s->nk; ++k)
            t.push_back(make_rot_task((int)s->npw[k], j.nbX, j.X + s->off[k], s->npw[k], j.nbO,
                                      j.M + (int64_t)k * s->nb * s->nb, j.nbO, j.beta, j.out + s->off[k], s->npw[k]));
    void* d = nullptr;
    DPP_TRY(upload_table(s, t.data(), t.size() * sizeof(RotTask), &d));
    return rotate_tasks(s->ctx, t, (const RotTask*)d);
}

// out_k = beta out_k + X_k M_k
dpp_status rotate_all(dpp_system_s* s, int nbX, const double2* X, int nbO, const double2* M, double beta,
                      double2* out) {
    return rotate_jobs(s, {RotJob{nbX, X, nbO, M, beta, out}});
}

// FFT item table for `nbands` bands per k-point (planes of all k back to back).
dpp_status item_table(dpp_system_s* s, int nbands, std::vector<FftItem>& h, FftItem** d) {
    h.clear();
    int64_t toff = 0;
    for (int k = 0; k < s->nk; ++k) {
        FftItem it = s->bases[k]->h_item;
        it.nb = nbands;
        it.ld = s->npw[k];
        it.c_off = s->off[k];
        it.t_off = toff;
        it.v_off = 0;
        it.wk = s->wk[k];
        it.f_off = (int64_t)k * s->nb;
        toff += (int64_t)nbands * it.nplanes * it.S1 * it.S2;
        h.push_back(it);
    }
    if (*d == nullptr) DPP_TRY(dalloc_t(s, d, (size_t)s->nk));
    DPP_HIP(hipMemcpy(*d, h.data(), h.size() * sizeof(FftItem), hipMemcpyHostToDevice));
    return DPP_OK;
}

dpp_status items_for(dpp_system_s* s, int nbands, const FftItem** d, const std::vector<FftItem>** h) {
    if (nbands == s->nb) {
        *d = s->d_items_nb;
        *h = &s->h_items_nb;
        return DPP_OK;
    }
    if (s->items_occ_nb != nbands) {
        DPP_TRY(item_table(s, nbands, s->h_items_occ, &s->d_items_occ));
        s->items_occ_nb = nbands;
    }
    *d = s->d_items_occ;
    *h = &s->h_items_occ;
    return DPP_OK;
}

// HX = H X for nbands bands of every k-point: batched FFT passes at the
// potential of the first Hamiltonian (shared by all k of the cell), then the
// projector terms HX += P (D P^dag X) as two batched contractions.
dpp_status apply_H_all(dpp_system_s* s, int nbands, const double2* X, double2* HX) {
    s->hc_bandk += (int64_t)nbands * s->nk;
    const FftItem* d;
    const std::vector<FftItem>* h;
    DPP_TRY(items_for(s, nbands, &d, &h));
    const double* V = s->hams[0]->d_Veff;
    if (!V) return set_error(DPP_EINVAL, "apply_H: no potential set");
    if (s->prec == DPP_F64)
        DPP_TRY(apply_H_local_batched<double>(s->ctx, d, *h, X, HX, V, s->Tplanes));
    else
        DPP_TRY(apply_H_local_batched<float>(s->ctx, d, *h, X, HX, V, s->Tplanes));
    if (s->nproj > 0) {
        std::vector<OvTask> t;
        int64_t poff = 0;
        for (int k = 0; k < s->nk; ++k) {
            OvTask x = make_ov_task((int)s->npw[k], s->nproj, s->hams[k]->d_P, s->npw[k], nbands, X + s->off[k],
                                    s->npw[k], s->D, s->Pi + (int64_t)k * s->pi_stride, nbands);
            x.part_off = poff;
            poff += (int64_t)x.nchunk * x.ntiles * 256;
            t.push_back(x);
        }
        void* dt = nullptr;
        DPP_TRY(upload_table(s, t.data(), t.size() * sizeof(OvTask), &dt));
        DPP_TRY(overlap_tasks(s->ctx, t, (const OvTask*)dt, s->ov_part));
        std::vector<RotTask> r;
        for (int k = 0; k < s->nk; ++k)
            r.push_back(make_rot_task((int)s->npw[k], s->nproj, s->hams[k]->d_P, s->npw[k], nbands,
                                      s->Pi + (int64_t)k * s->pi_stride, nbands, 1.0, HX + s->off[k], s->npw[k]));
        DPP_TRY(upload_table(s, r.data(), r.size() * sizeof(RotTask), &dt));
        DPP_TRY(rotate_tasks(s->ctx, r, (const RotTask*)dt));
    }
    return DPP_OK;
}

// Pi_k = P_k^dag X_k (nproj x nbands, row length nbands) for every k.
dpp_status proj_overlaps(dpp_system_s* s, int nbands, const double2* X) {
    std::vector<OvTask> t;
    int64_t poff = 0;
    for (int k = 0; k < s->nk; ++k) {
        OvTask x = make_ov_task((int)s->npw[k], s->nproj, s->hams[k]->d_P, s->npw[k], nbands, X + s->off[k],
                                s->npw[k], 1.0, s->Pi + (int64_t)k * s->pi_stride, nbands);
        x.part_off = poff;
        poff += (int64_t)x.nchunk * x.ntiles * 256;
        t.push_back(x);
    }
    void* dt = nullptr;
    DPP_TRY(upload_table(s, t.data(), t.size() * sizeof(OvTask), &dt));
    return overlap_tasks(s->ctx, t, (const OvTask*)dt, s->ov_part);
}

// n (+)= sum_k w_k sum_i f_ki |I psi_ki|^2 over nbands bands (fillings at d_f, stride nb).
dpp_status density_all(dpp_system_s* s, int nbands, const double2* psi, double* n, dpp_precision prec) {
    const FftItem* d;
    const std::vector<FftItem>* h;
    DPP_TRY(items_for(s, nbands, &d, &h));
    const int nch = std::min(nbands, s->dens_nch);
    if (prec == DPP_F64)
        return density_batched<double>(s->ctx, d, *h, psi, s->d_f, n, s->Tplanes, s->dens_part, nch);
    return density_batched<float>(s->ctx, d, *h, psi, s->d_f, n, s->Tplanes, s->dens_part, nch);
}

dpp_status axpby_all(dpp_system_s* s, int nb, const double* a, const double2* x, const double* b, const double2* y,
                     double2* out) {
    TimerScope ts_(s->ctx, DPP_TK_BLOCKOPS);
    hipLaunchKernelGGL(k_seg_axpby, dim3(seg_blocks(s, nb), s->nk), dim3(256), 0, stream(s), s->d_seg, nb, a, x, b, y,
                       out);
    DPP_LAUNCHED();
    return DPP_OK;
}

dpp_status precond_all(dpp_system_s* s, int nb, const double2* x, double2* out) {
    TimerScope ts_(s->ctx, DPP_TK_BLOCKOPS);
    hipLaunchKernelGGL(k_seg_precond, dim3(seg_blocks(s, nb), s->nk), dim3(256), 0, stream(s), s->d_seg, nb, 1.0, x,
                       out);
    DPP_LAUNCHED();
    return DPP_OK;
}

// dots[p][k] (k < nk) and totals dots[p][nk] to host
dpp_status dots_all(dpp_system_s* s, int nb, int npair, const double2* const* a, const double2* const* b,
                    std::vector<double>& host) {
    TimerScope ts_(s->ctx, DPP_TK_BLOCKOPS);
    DotPairs pr;
    for (int p = 0; p < 4; ++p) {
        pr.a[p] = p < npair ? a[p] : nullptr;
        pr.b[p] = p < npair ? b[p] : nullptr;
    }
    hipLaunchKernelGGL(k_seg_dots, dim3(DOT_BLOCKS, s->nk), dim3(256), 0, stream(s), s->d_seg, s->nk, nb, npair, pr,
                       s->d_part);
    DPP_LAUNCHED();
    hipLaunchKernelGGL(k_seg_dots_reduce, dim3(npair), dim3(64), 0, stream(s), s->d_part, s->nk, npair, s->d_dots);
    DPP_LAUNCHED();
    host.assign((size_t)npair * (s->nk + 1), 0.0);
    DPP_HIP(hipMemcpyAsync(host.data(), s->d_dots, host.size() * sizeof(double), hipMemcpyDeviceToHost, stream(s)));
    DPP_HIP(hipStreamSynchronize(stream(s)));
    return DPP_OK;
}

dpp_status upload(dpp_system_s* s, double* dst, const std::vector<double>& v) {
    if (v.size() > s->ring_len) return set_error(DPP_EINVAL, "upload: array larger than the staging slot");
    if (s->ring_slot == s->ring_slots) {
        DPP_HIP(hipStreamSynchronize(stream(s)));
        s->ring_slot = 0;
    }
    double* slot = s->h_ring + (size_t)s->ring_slot * s->ring_len;
    s->ring_slot++;
    std::memcpy(slot, v.data(), v.size() * sizeof(double));
    DPP_HIP(hipMemcpyAsync(dst, slot, v.size() * sizeof(double), hipMemcpyHostToDevice, stream(s)));
    return DPP_OK;
}

dpp_status smm(dpp_system_s* s, int n, int opA, int opB, double alpha, const double* alpha_arr, const double2* A,
               const double2* B, double beta, double2* C, int batch) {
    TimerScope ts_(s->ctx, DPP_TK_BLOCKOPS);
    const int64_t st = (int64_t)s->nb * s->nb;
    hipLaunchKernelGGL(k_smm, dim3(batch), dim3(256), 0, stream(s), n, opA, opB, alpha, alpha_arr, A, st, B, st, beta,
                       C, st);
    DPP_LAUNCHED();
    return DPP_OK;
}

dpp_status chol_inv_all(dpp_system_s* s, int n, const double2* Um, double2* Ri, int batch) {
    // matrices at stride nb^2: when n < nb, pack via the stride-n layout the kernel expects
    if (n == s->nb) return dpp_cholesky_inverse(s->ctx, n, batch, (const dpp_c64*)Um, (dpp_c64*)Ri);
    for (int b = 0; b < batch; ++b)
        DPP_TRY(dpp_cholesky_inverse(s->ctx, n, 1, (const dpp_c64*)(Um + (int64_t)b * s->nb * s->nb),
                                     (dpp_c64*)(Ri + (int64_t)b * s->nb * s->nb)));
    return DPP_OK;
}

// ----------------------------------------------------- band energy (B) ---
// Gradient state at the current Y (nb bands): U, Rinv, H0 = Y^dag H Y,
// g = (HY - O Y U^{-1} H0) U^{-1}, E0_k = Tr(U^{-1} H0); requires HY.
dpp_status grad_B(dpp_system_s* s, const double2* Y) {
    const int nb = s->nb, nk = s->nk;
    const double om = s->grid->omega;
    DPP_TRY(overlap_jobs(s, {OvJob{nb, Y, nb, Y, om, s->U}, OvJob{nb, Y, nb, s->HY, 1.0, s->H0}}));
    DPP_TRY(chol_inv_all(s, nb, s->U, s->Rinv, nk));
    // Uinv = Rinv Rinv^dag (M1); Q = Uinv H0 Uinv (M2)
    DPP_TRY(smm(s, nb, 0, 1, 1.0, nullptr, s->Rinv, s->Rinv, 0.0, s->M1, nk));
    DPP_TRY(smm(s, nb, 0, 0, 1.0, nullptr, s->M1, s->H0, 0.0, s->Rt, nk));
    DPP_TRY(smm(s, nb, 0, 0, -om, nullptr, s->Rt, s->M1, 0.0, s->M2, nk));
    DPP_TRY(rotate_all(s, nb, s->HY, nb, s->M1, 0.0, s->g));
    DPP_TRY(rotate_all(s, nb, Y, nb, s->M2, 1.0, s->g));
    hipLaunchKernelGGL(k_trace_RhHR, dim3(nk), dim3(256), 0, stream(s), nb, s->Rinv, s->H0, s->d_E);
    DPP_LAUNCHED();
    s->bE0.assign(nk, 0.0);
    DPP_HIP(hipMemcpyAsync(s->bE0.data(), s->d_E, nk * sizeof(double), hipMemcpyDeviceToHost, stream(s)));
    DPP_HIP(hipStreamSynchronize(stream(s)));
    return DPP_OK;
}

// Trial band energies Tr(U(a)^{-1} H(a)) for a = alpha[k] along the current D.
dpp_status trial_B(dpp_system_s* s, const std::vector<double>& alpha, std::vector<double>& E) {
    const int nb = s->nb, nk = s->nk;
    DPP_TRY(upload(s, s->d_alpha, alpha));
    hipLaunchKernelGGL(k_trial_mats, dim3(nk), dim3(256), 0, stream(s), nb, s->d_alpha, s->U, s->X, s->Q, s->H0, s->H1,
                       s->H2, s->Ua, s->Ha);
    DPP_LAUNCHED();
    DPP_TRY(chol_inv_all(s, nb, s->Ua, s->Rt, nk));
    hipLaunchKernelGGL(k_trace_RhHR, dim3(nk), dim3(256), 0, stream(s), nb, s->Rt, s->Ha, s->d_trial);
    DPP_LAUNCHED();
    E.assign(nk, 0.0);
    DPP_HIP(hipMemcpyAsync(E.data(), s->d_trial, nk * sizeof(double), hipMemcpyDeviceToHost, stream(s)));
    DPP_HIP(hipStreamSynchronize(stream(s)));
    return DPP_OK;
}

// Small matrices of the line along D: X = Y^dag O D, Q = D^dag O D, H1 = Y^dag H D, H2 = D^dag H D.
dpp_status line_mats_B(dpp_system_s* s, const double2* Y) {
    const int nb = s->nb;
    const double om = s->grid->omega;
    DPP_TRY(apply_H_all(s, nb, s->Dd, s->HD));
    DPP_TRY(overlap_jobs(s, {OvJob{nb, Y, nb, s->Dd, om, s->X}, OvJob{nb, s->Dd, nb, s->Dd, om, s->Q},
                             OvJob{nb, Y, nb, s->HD, 1.0, s->H1}, OvJob{nb, s->Dd, nb, s->HD, 1.0, s->H2}}));
    return DPP_OK;
}

// Lockstep line searches over the k-points in `active`; returns accepted steps
// (0 where the search failed) and flags.
dpp_status linemin_B(dpp_system_s* s, const std::vector<double>& d0, std::vector<int>& active,
                     std::vector<double>& step, std::vector<int>& ok) {
    const int nk = s->nk;
    std::vector<double> at(s->bat), Et, Es, as(nk, 0.0);
    std::vector<int> tries(nk, 0);
    ok.assign(nk, 0);
    step.assign(nk, 0.0);
    for (;;) {
        bool any = false;
        for (int k = 0; k < nk; ++k) any |= active[k] && !ok[k] && tries[k] < MAX_TRIES;
        if (!any) break;
        std::vector<double> a1(nk, 0.0);
        for (int k = 0; k < nk; ++k) a1[k] = (active[k] && !ok[k] && tries[k] < MAX_TRIES) ? at[k] : 0.0;
        DPP_TRY(trial_B(s, a1, Et));
        for (int k = 0; k < nk; ++k) {
            if (!(active[k] && !ok[k] && tries[k] < MAX_TRIES)) continue;
            const double c = (Et[k] - s->bE0[k] - d0[k] * at[k]) / (at[k] * at[k]);
            double a = c > 0 ? -d0[k] / (2.0 * c) : 2.0 * at[k];
            as[k] = std::min(a, 10.0 * at[k]);
        }
        std::vector<double> a2(nk, 0.0);
        for (int k = 0; k < nk; ++k) a2[k] = (active[k] && !ok[k] && tries[k] < MAX_TRIES) ? as[k] : 0.0;
        DPP_TRY(trial_B(s, a2, Es));
        for (int k = 0; k < nk; ++k) {
            if (!(active[k] && !ok[k] && tries[k] < MAX_TRIES)) continue;
            if (Es[k] <= s->bE0[k]) {
                ok[k] = 1;
                step[k] = as[k];
            } else if (Et[k] <= s->bE0[k]) {
                ok[k] = 1;
                step[k] = at[k];
            } else {
                at[k] *= 0.5;
                tries[k] += 1;
            }
        }
    }
    return DPP_OK;
}

dpp_status cgB_init(dpp_system_s* s, double2* Y) {
    const int nb = s->nb, nk = s->nk;
    // orthonormalize the starting block: Y <- Y R^{-1}
    DPP_TRY(overlap_all(s, nb, Y, nb, Y, s->grid->omega, s->U));
    DPP_TRY(chol_inv_all(s, nb, s->U, s->Rinv, nk));
    DPP_HIP(hipMemcpyAsync(s->T1, Y, s->total * sizeof(double2), hipMemcpyDeviceToDevice, stream(s)));
    DPP_TRY(rotate_all(s, nb, s->T1, nb, s->Rinv, 0.0, Y));
    DPP_TRY(apply_H_all(s, nb, Y, s->HY));
    DPP_TRY(grad_B(s, Y));
    s->bat.assign(nk, 0.3 / s->grid->omega);
    s->breset.assign(nk, 1);
    s->bstat.assign(nk, 0);
    s->bgkg.assign(nk, 0.0);
    return DPP_OK;
}

dpp_status cgB_step(dpp_system_s* s, double2* Y) {
    const int nb = s->nb, nk = s->nk;
    DPP_TRY(precond_all(s, nb, s->g, s->Kg));
    const double2* pa[3] = {s->g, s->gp, s->g};
    const double2* pb[3] = {s->Kg, s->Kg, s->Dp};
    std::vector<double> dt;
    DPP_TRY(dots_all(s, nb, 3, pa, pb, dt));
    std::vector<double> beta(nk, 0.0), d0(nk, 0.0), mKg(nk, -1.0);
    std::vector<int> steepest(nk, 1), active(nk, 0);
    for (int k = 0; k < nk; ++k) {
        if (s->bstat[k]) continue;
        active[k] = 1;
        const double gkg = dt[0 * (nk + 1) + k], gpkg = dt[1 * (nk + 1) + k], gdp = dt[2 * (nk + 1) + k];
        double b = 0.0;
        if (!s->breset[k]) b = std::max(0.0, (gkg - gpkg) / s->bgkg[k]);
        double dd = -gkg + b * gdp;
        if (b != 0.0 && dd >= 0.0) {
            b = 0.0;
            dd = -gkg;
        }
        beta[k] = b;
        d0[k] = dd;
        steepest[k] = b == 0.0;
    }
    DPP_TRY(upload(s, s->d_alpha, mKg));
    DPP_TRY(upload(s, s->d_beta, beta));
    DPP_TRY(axpby_all(s, nb, s->d_alpha, s->Kg, s->d_beta, s->Dp, s->Dd));
    DPP_TRY(line_mats_B(s, Y));
    std::vector<double> step;
    std::vector<int> ok;
    DPP_TRY(linemin_B(s, d0, active, step, ok));
    // failed CG directions: one more search along -K g
    std::vector<int> retry(nk, 0);
    bool anyretry = false;
    for (int k = 0; k < nk; ++k)
        if (active[k] && !ok[k] && !steepest[k]) retry[k] = 1, anyretry = true;
    if (anyretry) {
        std::vector<double> b0(nk, 0.0), st2;
        std::vector<int> ok2;
        // D <- -K g for the retried k (others keep their D; their step is fixed already)
        std::vector<double> aK(nk), aD(nk);
        for (int k = 0; k < nk; ++k) {
            aK[k] = retry[k] ? -1.0 : 0.0;
            aD[k] = retry[k] ? 0.0 : 1.0;
        }
        DPP_TRY(upload(s, s->d_alpha, aK));
        DPP_TRY(upload(s, s->d_beta, aD));
        DPP_TRY(axpby_all(s, nb, s->d_alpha, s->Kg, s->d_beta, s->Dd, s->Dd));
        DPP_TRY(line_mats_B(s, Y));
        std::vector<double> d0r(d0);
        for (int k = 0; k < nk; ++k)
            if (retry[k]) d0r[k] = -dt[0 * (nk + 1) + k];
        DPP_TRY(linemin_B(s, d0r, retry, st2, ok2));
        for (int k = 0; k < nk; ++k)
            if (retry[k]) ok[k] = ok2[k], step[k] = st2[k];
        // HD of the non-retried k must still match their D: it does, since HD was
        // recomputed from the updated D in line_mats_B for every k.
    }
    std::vector<double> ones(nk, 1.0);
    for (int k = 0; k < nk; ++k) {
        if (!active[k]) continue;
        if (!ok[k]) {
            s->bstat[k] = 1;
            s->breset[k] = 1;
            step[k] = 0.0;
        }
    }
    DPP_TRY(upload(s, s->d_ones, ones));
    DPP_TRY(upload(s, s->d_alpha, step));
    DPP_TRY(axpby_all(s, nb, s->d_ones, Y, s->d_alpha, s->Dd, Y));
    DPP_TRY(axpby_all(s, nb, s->d_ones, s->HY, s->d_alpha, s->HD, s->HY));
    // history
    std::swap(s->gp, s->g);
    std::swap(s->Kgp, s->Kg);
    std::swap(s->Dp, s->Dd);
    for (int k = 0; k < nk; ++k) {
        if (active[k] && ok[k]) {
            s->bgkg[k] = dt[0 * (nk + 1) + k];
            s->bat[k] = step[k];
            s->breset[k] = 0;
        }
    }
    DPP_TRY(grad_B(s, Y));
    return DPP_OK;
}

// --------------------------------------------------- total energy (V) -----
struct Parts {
    double Ekin, Enl, Eloc, EH, Exc;
    double total() const { return Ekin + Enl + Eloc + EH + Exc; }
};

// Density and energy of unorthonormalized Y (nocc bands, filling f): leaves
// psi, U, Rinv, n, V_eff (and the hams' potential) for a following gradient.
dpp_status energy_V(dpp_system_s* s, const double2* Y, Parts& P) {
    const int nb = s->vnocc, nk = s->nk;
    const double om = s->grid->omega;
    const int64_t N = s->grid->N;
    DPP_TRY(overlap_all(s, nb, Y, nb, Y, om, s->U));
    DPP_TRY(chol_inv_all(s, nb, s->U, s->Rinv, nk));
    DPP_TRY(rotate_all(s, nb, Y, nb, s->Rinv, 0.0, s->psi));
    DPP_HIP(hipMemsetAsync(s->n, 0, N * sizeof(double), stream(s)));
    DPP_TRY(density_all(s, nb, s->psi, s->n, DPP_F64));
    // potentials and density terms
    DPP_TRY(dpp_hartree(s->grid, s->n, s->VH, s->d_E + 2, s->gws));
    DPP_TRY(dpp_lda_pz81(s->grid, s->n, s->vxc, s->d_E + 3, s->gws));
    DPP_TRY(dpp_grid_dot(s->grid, s->Vloc, s->n, om / (double)N, s->d_E + 4, s->gws));
    hipLaunchKernelGGL(k_grid_lin3, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, stream(s), N, 1.0, s->Vloc, 1.0,
                       s->VH, 1.0, s->vxc, s->Veff);
    DPP_LAUNCHED();
    // kinetic and nonlocal
    hipLaunchKernelGGL(k_seg_kinetic, dim3(DOT_BLOCKS, nk), dim3(256), 0, stream(s), s->d_seg, nb, s->nb, s->d_f,
                       s->psi, s->d_part);
    DPP_LAUNCHED();
    hipLaunchKernelGGL(k_seg_weighted_total, dim3(1), dim3(1), 0, stream(s), s->d_part, nk, s->d_wk, 0.5 * om, s->d_E);
    DPP_LAUNCHED();
    if (s->nproj > 0) {
        DPP_TRY(proj_overlaps(s, nb, s->psi));
        hipLaunchKernelGGL(k_nonlocal_energy, dim3(1), dim3(256), 0, stream(s), nk, s->nproj, nb, s->nb, s->Pi,
                           s->pi_stride, s->d_f, s->d_wk, s->D, s->d_E + 1);
        DPP_LAUNCHED();
    } else {
        DPP_HIP(hipMemsetAsync(s->d_E + 1, 0, sizeof(double), stream(s)));
    }
    double e[5];
    DPP_HIP(hipMemcpyAsync(e, s->d_E, 5 * sizeof(double), hipMemcpyDeviceToHost, stream(s)));
    DPP_HIP(hipStreamSynchronize(stream(s)));
    P.Ekin = e[0];
    P.Enl = e[1];
    P.EH = e[2];
    P.Exc = e[3];
    P.Eloc = e[4];
    return DPP_OK;
}

// Gradient after energy_V: g = w_k f (H psi - O psi Hsub) Rinv^dag into `gout`.
dpp_status grad_V(dpp_system_s* s, double2* gout) {
    const int nb = s->vnocc, nk = s->nk;
    const double om = s->grid->omega;
    const int64_t st = (int64_t)s->nb * s->nb;
    for (int k = 0; k < nk; ++k) DPP_TRY(dpp_ham_set_potential(s->hams[k], s->Veff));
    DPP_TRY(apply_H_all(s, nb, s->psi, s->T1));
    DPP_TRY(overlap_all(s, nb, s->psi, nb, s->T1, 1.0, s->H0));
    hipLaunchKernelGGL(k_sm_scale, dim3(nk), dim3(256), 0, stream(s), nb, st, 0, -om, (const double*)nullptr, s->H0,
                       s->M2);
    DPP_LAUNCHED();
    DPP_TRY(rotate_all(s, nb, s->psi, nb, s->M2, 1.0, s->T1));
    hipLaunchKernelGGL(k_sm_scale, dim3(nk), dim3(256), 0, stream(s), nb, st, 1, s->vf, (const double*)s->d_wk, s->Rinv,
                       s->M1);
    DPP_LAUNCHED();
    DPP_TRY(rotate_all(s, nb, s->T1, nb, s->M1, 0.0, gout));
    return DPP_OK;
}

dpp_status objective_V(dpp_system_s* s, const double2* Y, double2* gout, Parts& P) {
    DPP_TRY(energy_V(s, Y, P));
    DPP_TRY(grad_V(s, gout));
    return DPP_OK;
}

// T2 = Y + a D (nocc bands)
dpp_status trial_point(dpp_system_s* s, const double2* Y, double a, const double2* D, double2* out) {
    std::vector<double> one(s->nk, 1.0), av(s->nk, a);
    DPP_TRY(upload(s, s->d_ones, one));
    DPP_TRY(upload(s, s->d_alpha, av));
    DPP_TRY(axpby_all(s, s->vnocc, s->d_ones, Y, s->d_alpha, D, out));
    return DPP_OK;
}

dpp_status cgV_init(dpp_system_s* s, double2* Y, int nocc, double f, Parts& P) {
    const int nk = s->nk;
    s->vnocc = nocc;
    s->vf = f;
    std::vector<double> fv((size_t)nk * s->nb, 0.0);
    for (int k = 0; k < nk; ++k)
        for (int i = 0; i < nocc; ++i) fv[(size_t)k * s->nb + i] = f;
    DPP_TRY(upload(s, s->d_f, fv));
    // orthonormalize the starting block once
    DPP_TRY(overlap_all(s, nocc, Y, nocc, Y, s->grid->omega, s->U));
    DPP_TRY(chol_inv_all(s, nocc, s->U, s->Rinv, nk));
    for (int k = 0; k < nk; ++k)
        DPP_HIP(hipMemcpyAsync(s->T1 + s->off[k], Y + s->off[k], (size_t)nocc * s->npw[k] * sizeof(double2),
                               hipMemcpyDeviceToDevice, stream(s)));
    DPP_TRY(rotate_all(s, nocc, s->T1, nocc, s->Rinv, 0.0, Y));
    DPP_TRY(objective_V(s, Y, s->g, P));
    s->vE0 = P.total();
    double wmax = 0;
    for (double w : s->wk) wmax = std::max(wmax, w);
    s->vat = 0.3 / (s->grid->omega * f * wmax);
    s->vreset = 1;
    s->vstat = 0;
    s->vgkg = 0;
    return DPP_OK;
}

// One line minimization along s->Dd from Y; on success Y and g are updated.
dpp_status linemin_V(dpp_system_s* s, double2* Y, double d0, bool& ok, double& step, Parts& P) {
    const double E0 = s->vE0;
    double at = s->vat;
    ok = false;
    for (int t = 0; t < MAX_TRIES; ++t) {
        Parts Pt;
        DPP_TRY(trial_point(s, Y, at, s->Dd, s->T2));
        DPP_TRY(energy_V(s, s->T2, Pt));
        const double Et = Pt.total();
        const double c = (Et - E0 - d0 * at) / (at * at);
        double as = c > 0 ? -d0 / (2.0 * c) : 2.0 * at;
        as = std::min(as, 10.0 * at);
        Parts Ps;
        DPP_TRY(trial_point(s, Y, as, s->Dd, s->T2));
        DPP_TRY(objective_V(s, s->T2, s->g2, Ps));
        if (Ps.total() <= E0) {
            ok = true;
            step = as;
            P = Ps;
            break;
        }
        if (Et <= E0) {
            DPP_TRY(trial_point(s, Y, at, s->Dd, s->T2));
            DPP_TRY(objective_V(s, s->T2, s->g2, P));
            ok = true;
            step = at;
            break;
        }
        at *= 0.5;
    }
    if (ok) {
        for (int k = 0; k < s->nk; ++k)
            DPP_HIP(hipMemcpyAsync(Y + s->off[k], s->T2 + s->off[k], (size_t)s->vnocc * s->npw[k] * sizeof(double2),
                                   hipMemcpyDeviceToDevice, stream(s)));
    }
    return DPP_OK;
}

dpp_status cgV_step(dpp_system_s* s, double2* Y, Parts& P) {
    const int nb = s->vnocc, nk = s->nk;
    if (s->vstat) return DPP_OK;
    DPP_TRY(precond_all(s, nb, s->g, s->Kg));
    const double2* pa[3] = {s->g, s->gp, s->g};
    const double2* pb[3] = {s->Kg, s->Kg, s->Dp};
    std::vector<double> dt;
    DPP_TRY(dots_all(s, nb, 3, pa, pb, dt));
    const double gkg = dt[0 * (nk + 1) + nk], gpkg = dt[1 * (nk + 1) + nk], gdp = dt[2 * (nk + 1) + nk];
    double beta = 0.0;
    if (!s->vreset) beta = std::max(0.0, (gkg - gpkg) / s->vgkg);
    double d0 = -gkg + beta * gdp;
    if (beta != 0.0 && d0 >= 0.0) {
        beta = 0.0;
        d0 = -gkg;
    }
    bool steepest = beta == 0.0;
    std::vector<double> mK(nk, -1.0), bv(nk, beta);
    DPP_TRY(upload(s, s->d_alpha, mK));
    DPP_TRY(upload(s, s->d_beta, bv));
    DPP_TRY(axpby_all(s, nb, s->d_alpha, s->Kg, s->d_beta, s->Dp, s->Dd));
    bool ok = false;
    double step = 0;
    DPP_TRY(linemin_V(s, Y, d0, ok, step, P));
    if (!ok && !steepest) {
        std::vector<double> zero(nk, 0.0);
        DPP_TRY(upload(s, s->d_beta, zero));
        DPP_TRY(axpby_all(s, nb, s->d_alpha, s->Kg, s->d_beta, s->Dp, s->Dd));
        DPP_TRY(linemin_V(s, Y, -gkg, ok, step, P));
    }
    if (!ok) {
        s->vstat = 1;
        s->vreset = 1;
        return DPP_OK;
    }
    std::swap(s->gp, s->g);
    std::swap(s->g, s->g2);   // new gradient (from the accepted objective) becomes g
    std::swap(s->Kgp, s->Kg);
    std::swap(s->Dp, s->Dd);
    s->vgkg = gkg;
    s->vE0 = P.total();
    s->vat = step;
    s->vreset = 0;
    return DPP_OK;
}

// ------------------------------------------------------------------ SCF ---
dpp_status potentials(dpp_system_s* s, const double* n) {
    const int64_t N = s->grid->N;
    DPP_TRY(dpp_hartree(s->grid, n, s->VH, s->d_E + 2, s->gws));
    DPP_TRY(dpp_lda_pz81(s->grid, n, s->vxc, s->d_E + 3, s->gws));
    DPP_TRY(dpp_grid_dot(s->grid, s->Vloc, n, s->grid->omega / (double)N, s->d_E + 4, s->gws));
    hipLaunchKernelGGL(k_grid_lin3, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, stream(s), N, 1.0, s->Vloc, 1.0,
                       s->VH, 1.0, s->vxc, s->Veff);
    DPP_LAUNCHED();
    for (int k = 0; k < s->nk; ++k) DPP_TRY(dpp_ham_set_potential(s->hams[k], s->Veff));
    return DPP_OK;
}

void aufbau(const std::vector<double>& eig, int nk, int nb, const std::vector<double>& wk, double ne,
            std::vector<double>& f) {
    struct St {
        double e;
        int k, i;
    };
    std::vector<St> st;
    for (int k = 0; k < nk; ++k)
        for (int i = 0; i < nb; ++i) st.push_back({eig[(size_t)k * nb + i], k, i});
    std::sort(st.begin(), st.end(), [](const St& a, const St& b) {
        if (a.e != b.e) return a.e < b.e;
        if (a.k != b.k) return a.k < b.k;
        return a.i < b.i;
    });
    f.assign((size_t)nk * nb, 0.0);
    double rem = ne;
    size_t j = 0;
    while (j < st.size() && rem > 1e-12) {
        const double e0 = st[j].e;
        size_t j0 = j;
        ++j;
        while (j < st.size() && st[j].e - e0 < DEGEN_TOL) ++j;
        double cap = 0;
        for (size_t t = j0; t < j; ++t) cap += 2.0 * wk[st[t].k];
        if (cap <= rem + 1e-12) {
            for (size_t t = j0; t < j; ++t) f[(size_t)st[t].k * nb + st[t].i] = 2.0;
            rem -= cap;
        } else {
            const double frac = rem / cap;
            for (size_t t = j0; t < j; ++t) f[(size_t)st[t].k * nb + st[t].i] = 2.0 * frac;
            rem = 0;
        }
    }
}

dpp_status pulay_mix(dpp_system_s* s) {
    const int64_t N = s->grid->N;
    const unsigned nbk = (unsigned)((N + 255) / 256);
    const double dV = s->grid->omega / (double)N;
    // new history entry (ring buffer of PULAY_MAX)
    int slot;
    if (s->hist_m < PULAY_MAX) {
        slot = (s->hist_head + s->hist_m) % PULAY_MAX;
        s->hist_m++;
    } else {
        slot = s->hist_head;
        s->hist_head = (s->hist_head + 1) % PULAY_MAX;
    }
    DPP_HIP(hipMemcpyAsync(s->hist_nin[slot], s->nin, N * sizeof(double), hipMemcpyDeviceToDevice, stream(s)));
    hipLaunchKernelGGL(k_grid_lin3, dim3(nbk), dim3(256), 0, stream(s), N, 1.0, s->nout, -1.0, s->nin, 0.0,
                       (const double*)nullptr, s->hist_res[slot]);
    DPP_LAUNCHED();
    const int m = s->hist_m;
    const double alpha = 0.5;
    if (m == 1) {
        PulayPtrs bl;
        PulayOrder sl;
        for (int i = 0; i < PULAY_MAX; ++i) {
            bl.nin[i] = nullptr;
            bl.res[i] = i == 0 ? s->hist_res[slot] : nullptr;
            sl.s[i] = slot;
        }
        hipLaunchKernelGGL(k_multi_dot, dim3(MDOT_BLOCKS), dim3(256), 0, stream(s), N, (const double*)s->hist_res[slot],
                           bl, 1, s->d_part);
        DPP_LAUNCHED();
        hipLaunchKernelGGL(k_multi_dot_store, dim3(1), dim3(64), 0, stream(s), (const double*)s->d_part, 1, sl, slot,
                           dV, s->pulayA);
        DPP_LAUNCHED();
        hipLaunchKernelGGL(k_grid_lin3, dim3(nbk), dim3(256), 0, stream(s), N, 1.0, s->nin, alpha, s->hist_res[slot],
                           0.0, (const double*)nullptr, s->nin);
        DPP_LAUNCHED();
        return DPP_OK;
    }
    // residual overlaps: the new residual against every stored one (one pass),
    // kept in a slot-indexed matrix; the solve reads it in history order
    std::vector<int> order(m);
    for (int i = 0; i < m; ++i) order[i] = (s->hist_head + i) % PULAY_MAX;
    {
        PulayPtrs bl;
        PulayOrder sl;
        for (int i = 0; i < PULAY_MAX; ++i) {
            bl.nin[i] = nullptr;
            bl.res[i] = i < m ? s->hist_res[order[i]] : nullptr;
            sl.s[i] = i < m ? order[i] : 0;
        }
        TimerScope ts_(s->ctx, DPP_TK_FIELDS);
        hipLaunchKernelGGL(k_multi_dot, dim3(MDOT_BLOCKS), dim3(256), 0, stream(s), N, (const double*)s->hist_res[slot],
                           bl, m, s->d_part);
        DPP_LAUNCHED();
        hipLaunchKernelGGL(k_multi_dot_store, dim3(1), dim3(64), 0, stream(s), (const double*)s->d_part, m, sl, slot,
                           dV, s->pulayA);
        DPP_LAUNCHED();
        PulayOrder ord;
        for (int i = 0; i < PULAY_MAX; ++i) ord.s[i] = i < m ? order[i] : 0;
        hipLaunchKernelGGL(k_pulay_solve, dim3(1), dim3(1), 0, stream(s), m, (const double*)s->pulayA, ord, s->pulayC,
                           s->ctx->d_status);
        DPP_LAUNCHED();
    }
    PulayPtrs h;
    for (int i = 0; i < PULAY_MAX; ++i) {
        h.nin[i] = i < m ? s->hist_nin[order[i]] : nullptr;
        h.res[i] = i < m ? s->hist_res[order[i]] : nullptr;
    }
    hipLaunchKernelGGL(k_pulay_combine, dim3(nbk), dim3(256), 0, stream(s), N, m, h, s->pulayC, alpha, s->nin);
    DPP_LAUNCHED();
    return DPP_OK;
}

}  // namespace

// ============================================================== C ABI =====

extern "C" dpp_status dpp_system_create(dpp_ctx ctx, const dpp_system_desc* d, dpp_system* out) {
    clear_error();
    DPP_REQUIRE(ctx && d && out, "dpp_system_create: null argument");
    DPP_REQUIRE(d->nk >= 1 && d->nb >= 1 && d->nb <= 128 && d->nat >= 0, "dpp_system_create: bad sizes");
    DPP_REQUIRE(d->kpts && d->wk && d->R && d->S, "dpp_system_create: null arrays");
    DPP_REQUIRE(d->nat == 0 || (d->tau && d->Z && d->rc && d->has_proj), "dpp_system_create: null atom arrays");
    DPP_REQUIRE(d->prec == DPP_F64 || d->prec == DPP_F32, "dpp_system_create: bad precision");
    dpp_system_s* s = new dpp_system_s();
    s->ctx = ctx;
    s->nk = d->nk;
    s->nb = d->nb;
    s->nat = d->nat;
    s->ne = d->n_electrons;
    s->D = d->D;
    s->prec = (dpp_precision)d->prec;
    s->bulk_prec = s->prec;
    s->hist_m = s->hist_head = 0;
    s->scf_iter = 0;
    s->n_inner_steps = 3;
    s->n_inner_first = 3;
    s->hc_bandk = 0;
    s->refine_res = 0.0;
    s->last_res = -1.0;
    s->h_ring = nullptr;
    s->h_tab = nullptr;
    s->grid = nullptr;
    s->vnocc = 0;
    auto fail = [&](dpp_status st) {
        std::string msg = dpp_last_error();
        dpp_system_destroy(s);
        return set_error(st, msg);
    };
    dpp_status st = dpp_grid_create(ctx, d->R, d->S, &s->grid);
    if (st != DPP_OK) return fail(st);
    s->total = 0;
    for (int k = 0; k < d->nk; ++k) {
        dpp_basis b = nullptr;
        st = dpp_basis_create(s->grid, d->kpts + 3 * k, d->ecut, &b);
        if (st != DPP_OK) return fail(st);
        s->bases.push_back(b);
        dpp_ham h = nullptr;
        st = dpp_ham_create(b, d->nat, d->tau, d->has_proj, d->rp, d->D, &h);
        if (st != DPP_OK) return fail(st);
        s->hams.push_back(h);
        s->wk.push_back(d->wk[k]);
        s->off.push_back(s->total);
        s->npw.push_back(b->npw);
        s->total += (int64_t)d->nb * b->npw;
        if (b->npw < d->nb) return fail(set_error(DPP_EINVAL, "dpp_system_create: more bands than plane waves"));
    }
    s->off.push_back(s->total);
    s->nproj = s->hams[0]->nproj;
    const int nk = s->nk, nb = s->nb;
    const int64_t N = s->grid->N;
    std::vector<Seg> seg(nk);
    for (int k = 0; k < nk; ++k) seg[k] = Seg{s->off[k], (int)s->npw[k], 0, s->bases[k]->d_kG2};
    size_t wsb = 0;
    for (int k = 0; k < nk; ++k) {
        size_t b1 = 0;
        dpp_workspace_size(s->bases[k], nb, s->prec, &b1);
        wsb = std::max(wsb, b1);
        wsb = std::max(wsb, overlap_ws_bytes((int)s->npw[k], std::max(nb, std::max(s->nproj, 1)), nb));
    }
    s->ws_bytes = wsb;
    size_t gwsb = 0;
    dpp_grid_workspace_size(s->grid, &gwsb);
    size_t ewsb = 0;
    dpp_eigh_workspace_size(nb, nk, &ewsb);
    const size_t blk = (size_t)s->total;
    const size_t sm = (size_t)nk * nb * nb;
    s->pi_stride = (int64_t)std::max(s->nproj, 1) * nb;
    struct {
        double2** p;
        size_t n;
    } blocks[] = {{&s->HY, blk}, {&s->Dd, blk}, {&s->HD, blk}, {&s->g, blk}, {&s->g2, blk}, {&s->Kg, blk},
                  {&s->gp, blk}, {&s->Kgp, blk}, {&s->Dp, blk}, {&s->psi, blk}, {&s->T1, blk}, {&s->T2, blk},
                  {&s->U, sm}, {&s->Rinv, sm}, {&s->H0, sm}, {&s->X, sm}, {&s->Q, sm}, {&s->H1, sm},
                  {&s->H2, sm}, {&s->Ua, sm}, {&s->Ha, sm}, {&s->Rt, sm}, {&s->M1, sm}, {&s->M2, sm},
                  {&s->vecs, sm}, {&s->Pi, (size_t)nk * s->pi_stride}};
    for (auto& b : blocks)
        if ((st = dalloc_t(s, b.p, b.n)) != DPP_OK) return fail(st);
    struct {
        double** p;
        size_t n;
    } reals[] = {{&s->d_dots, 4 * (size_t)(nk + 1)}, {&s->d_part, std::max<size_t>(4 * (size_t)nk * DOT_BLOCKS, (size_t)PULAY_MAX * MDOT_BLOCKS)},
                 {&s->d_alpha, (size_t)nk}, {&s->d_ones, (size_t)nk}, {&s->d_beta, (size_t)nk},
                 {&s->d_E, 16}, {&s->d_f, (size_t)nk * nb}, {&s->d_eig, (size_t)nk * nb},
                 {&s->d_trial, (size_t)nk}, {&s->d_wk, (size_t)nk}, {&s->d_res, (size_t)nk * nb}, {&s->Vloc, (size_t)N}, {&s->VH, (size_t)N},
                 {&s->vxc, (size_t)N}, {&s->Veff, (size_t)N}, {&s->n, (size_t)N}, {&s->nin, (size_t)N},
                 {&s->nout, (size_t)N}, {&s->pulayA, PULAY_MAX * PULAY_MAX}, {&s->pulayC, PULAY_MAX}};
    for (auto& r : reals)
        if ((st = dalloc_t(s, r.p, r.n)) != DPP_OK) return fail(st);
    for (int i = 0; i < PULAY_MAX; ++i) {
        if ((st = dalloc_t(s, &s->hist_nin[i], (size_t)N)) != DPP_OK) return fail(st);
        if ((st = dalloc_t(s, &s->hist_res[i], (size_t)N)) != DPP_OK) return fail(st);
    }
    if ((st = dalloc(s, &s->ws, s->ws_bytes)) != DPP_OK) return fail(st);
    if ((st = dalloc(s, &s->gws, gwsb)) != DPP_OK) return fail(st);
    if ((st = dalloc(s, &s->eigws, ewsb)) != DPP_OK) return fail(st);
    if ((st = dalloc_t(s, &s->d_seg, (size_t)nk)) != DPP_OK) return fail(st);
    // batched-launch resources
    s->d_items_nb = s->d_items_occ = nullptr;
    s->items_occ_nb = -1;
    if ((st = item_table(s, nb, s->h_items_nb, &s->d_items_nb)) != DPP_OK) return fail(st);
    {
        const size_t tel = batched_plane_elems(s->h_items_nb);
        if ((st = dalloc(s, &s->Tplanes, tel * sizeof(double2))) != DPP_OK) return fail(st);
        int maxc = 1;
        for (int k = 0; k < nk; ++k) maxc = std::max(maxc, (int)((s->npw[k] + OV_CHUNK - 1) / OV_CHUNK));
        const int tiles = ((std::max(nb, s->nproj) + 15) / 16) * ((nb + 15) / 16);
        s->ov_part_elems = (size_t)4 * nk * maxc * tiles * 256;
        if ((st = dalloc_t(s, &s->ov_part, s->ov_part_elems)) != DPP_OK) return fail(st);
        s->dens_nch = std::min(nb, 16);
        if ((st = dalloc_t(s, &s->dens_part, (size_t)nk * s->dens_nch * N)) != DPP_OK) return fail(st);
        s->tab_bytes = 256 * 1024;
        s->tab_slots = 16;
        s->tab_slot = 0;
        if ((st = dalloc(s, (void**)&s->d_tab, s->tab_bytes)) != DPP_OK) return fail(st);
        if (hipHostMalloc((void**)&s->h_tab, s->tab_slots * s->tab_bytes, hipHostMallocDefault) != hipSuccess) {
            s->h_tab = nullptr;
            return fail(set_error(DPP_ENOMEM, "dpp_system_create: pinned table staging allocation failed"));
        }
    }
    s->ring_slots = 64;
    s->ring_len = std::max<size_t>(256, (size_t)nk * nb);
    s->ring_slot = 0;
    if (hipHostMalloc((void**)&s->h_ring, s->ring_slots * s->ring_len * sizeof(double), hipHostMallocDefault) !=
        hipSuccess) {
        s->h_ring = nullptr;
        return fail(set_error(DPP_ENOMEM, "dpp_system_create: pinned staging allocation failed"));
    }
    hipStream_t sm_st = stream(s);
    if (hipMemcpyAsync(s->d_seg, seg.data(), nk * sizeof(Seg), hipMemcpyHostToDevice, sm_st) != hipSuccess ||
        hipMemcpyAsync(s->d_wk, s->wk.data(), nk * sizeof(double), hipMemcpyHostToDevice, sm_st) != hipSuccess)
        return fail(set_error(DPP_EDEVICE, "dpp_system_create: upload failed"));
    // clear the whole state once (history buffers are read before written otherwise)
    for (auto& b : blocks) hipMemsetAsync(*b.p, 0, b.n * sizeof(double2), sm_st);
    // local pseudopotential
    st = dpp_local_potential(s->grid, d->nat, d->tau, d->Z, d->rc, s->Vloc, s->gws);
    if (st != DPP_OK) return fail(st);
    if (hipStreamSynchronize(sm_st) != hipSuccess) return fail(set_error(DPP_EDEVICE, "dpp_system_create: sync failed"));
    *out = s;
    return DPP_OK;
}

extern "C" dpp_status dpp_system_destroy(dpp_system s) {
    if (!s) return DPP_OK;
    if (s->ctx) hipStreamSynchronize(s->ctx->stream);
    for (void* p : s->allocs) hipFree(p);
    if (s->h_ring) hipHostFree(s->h_ring);
    if (s->h_tab) hipHostFree(s->h_tab);
    for (dpp_ham h : s->hams) dpp_ham_destroy(h);
    for (dpp_basis b : s->bases) dpp_basis_destroy(b);
    if (s->grid) dpp_grid_destroy(s->grid);
    delete s;
    return DPP_OK;
}

extern "C" dpp_status dpp_system_layout(dpp_system s, int64_t* offsets, int64_t* npw) {
    clear_error();
    DPP_REQUIRE(s, "dpp_system_layout: null system");
    for (int k = 0; k <= s->nk; ++k)
        if (offsets) offsets[k] = s->off[k];
    for (int k = 0; k < s->nk; ++k)
        if (npw) npw[k] = s->npw[k];
    return DPP_OK;
}

extern "C" dpp_status dpp_system_field(dpp_system s, int which, double** d_ptr) {
    clear_error();
    DPP_REQUIRE(s && d_ptr, "dpp_system_field: null argument");
    switch (which) {
        case DPP_FIELD_VLOC: *d_ptr = s->Vloc; break;
        case DPP_FIELD_VEFF: *d_ptr = s->Veff; break;
        case DPP_FIELD_N: *d_ptr = s->n; break;
        case DPP_FIELD_NIN: *d_ptr = s->nin; break;
        case DPP_FIELD_NOUT: *d_ptr = s->nout; break;
        default: return set_error(DPP_EINVAL, "dpp_system_field: unknown field");
    }
    return DPP_OK;
}

extern "C" dpp_status dpp_system_copy_field(dpp_system s, int which, double* d_out) {
    clear_error();
    double* src = nullptr;
    DPP_TRY(dpp_system_field(s, which, &src));
    DPP_REQUIRE(d_out, "dpp_system_copy_field: null output");
    DPP_HIP(hipMemcpyAsync(d_out, src, s->grid->N * sizeof(double), hipMemcpyDeviceToDevice, stream(s)));
    return DPP_OK;
}

extern "C" dpp_status dpp_cg_V_init(dpp_system s, dpp_c64* Y, int nocc, double f, dpp_energy* E) {
    clear_error();
    DPP_REQUIRE(s && Y && nocc >= 1 && nocc <= s->nb, "dpp_cg_V_init: bad arguments");
    Parts P;
    DPP_TRY(cgV_init(s, (double2*)Y, nocc, f, P));
    if (E) *E = dpp_energy{P.total(), P.Ekin, P.Enl, P.Eloc, P.EH, P.Exc};
    return DPP_OK;
}

extern "C" dpp_status dpp_cg_V_step(dpp_system s, dpp_c64* Y, dpp_energy* E, int* stationary) {
    clear_error();
    DPP_REQUIRE(s && Y && s->vnocc >= 1, "dpp_cg_V_step: call dpp_cg_V_init first");
    Parts P{0, 0, 0, 0, 0};
    DPP_TRY(cgV_step(s, (double2*)Y, P));
    if (stationary) *stationary = s->vstat;
    if (E) {
        if (s->vstat)
            *E = dpp_energy{s->vE0, 0, 0, 0, 0, 0};
        else
            *E = dpp_energy{P.total(), P.Ekin, P.Enl, P.Eloc, P.EH, P.Exc};
    }
    return DPP_OK;
}

extern "C" dpp_status dpp_cg_B_init(dpp_system s, dpp_c64* Y, const double* d_Veff, double* Eb) {
    clear_error();
    DPP_REQUIRE(s && Y && d_Veff, "dpp_cg_B_init: null argument");
    for (int k = 0; k < s->nk; ++k) DPP_TRY(dpp_ham_set_potential(s->hams[k], d_Veff));
    DPP_TRY(cgB_init(s, (double2*)Y));
    if (Eb) std::copy(s->bE0.begin(), s->bE0.end(), Eb);
    return DPP_OK;
}

extern "C" dpp_status dpp_cg_B_step(dpp_system s, dpp_c64* Y, double* Eb) {
    clear_error();
    DPP_REQUIRE(s && Y && !s->bE0.empty(), "dpp_cg_B_step: call dpp_cg_B_init first");
    DPP_TRY(cgB_step(s, (double2*)Y));
    if (Eb) std::copy(s->bE0.begin(), s->bE0.end(), Eb);
    return DPP_OK;
}

// Subspace rotation at the current band-CG state: psi = Y R^{-1}, H~ = psi^dag H psi,
// H~ V = V eps; Y <- psi V, HY <- (H psi) V.
static dpp_status subspace_rotate(dpp_system_s* s, double2* Y, double* eig_host) {
    const int nb = s->nb, nk = s->nk;
    DPP_TRY(rotate_jobs(s, {RotJob{nb, Y, nb, s->Rinv, 0.0, s->psi}, RotJob{nb, s->HY, nb, s->Rinv, 0.0, s->T1}}));
    DPP_TRY(overlap_all(s, nb, s->psi, nb, s->T1, 1.0, s->H0));
    DPP_TRY(dpp_subspace_eigh(s->ctx, nb, nk, (const dpp_c64*)s->H0, s->d_eig, (dpp_c64*)s->vecs, s->eigws));
    DPP_TRY(rotate_jobs(s, {RotJob{nb, s->psi, nb, s->vecs, 0.0, Y}, RotJob{nb, s->T1, nb, s->vecs, 0.0, s->HY}}));
    if (eig_host) {
        DPP_HIP(hipMemcpyAsync(eig_host, s->d_eig, (size_t)nk * nb * sizeof(double), hipMemcpyDeviceToHost, stream(s)));
        DPP_HIP(hipStreamSynchronize(stream(s)));
    }
    return DPP_OK;
}

extern "C" dpp_status dpp_band_eigenvalues(dpp_system s, dpp_c64* Y, double* eig) {
    clear_error();
    DPP_REQUIRE(s && Y && eig && !s->bE0.empty(), "dpp_band_eigenvalues: call dpp_cg_B_init first");
    DPP_TRY(subspace_rotate(s, (double2*)Y, eig));
    return DPP_OK;
}

extern "C" dpp_status dpp_scf_init(dpp_system s, const dpp_scf_desc* d) {
    clear_error();
    DPP_REQUIRE(s && d, "dpp_scf_init: null argument");
    DPP_REQUIRE(d->nat >= 0 && (d->nat == 0 || (d->tau && d->Z)), "dpp_scf_init: bad atoms");
    const int64_t N = s->grid->N;
    if (d->d_n_start) {
        DPP_HIP(hipMemcpyAsync(s->nin, d->d_n_start, N * sizeof(double), hipMemcpyDeviceToDevice, stream(s)));
    } else {
        DPP_TRY(dpp_start_density(s->grid, d->nat, d->tau, d->Z, d->sigma, s->nin, s->gws));
    }
    s->hist_m = 0;
    s->hist_head = 0;
    s->scf_iter = 0;
    s->n_inner_steps = d->n_inner > 0 ? d->n_inner : 3;
    s->n_inner_first = d->n_inner_first > 0 ? d->n_inner_first : s->n_inner_steps;
    s->prec = s->bulk_prec;
    s->last_res = -1.0;
    DPP_HIP(hipStreamSynchronize(stream(s)));
    return DPP_OK;
}

extern "C" dpp_status dpp_scf_iteration(dpp_system s, dpp_c64* Yc, dpp_energy* E, double* eig) {
    clear_error();
    DPP_REQUIRE(s && Yc, "dpp_scf_iteration: null argument");
    double2* Y = (double2*)Yc;
    const int nk = s->nk, nb = s->nb;
    const int64_t N = s->grid->N;
    // 1. V_eff[n_in]
    DPP_TRY(potentials(s, s->nin));
    // 2. band-energy CG, restarted, warm-started Y
    DPP_TRY(cgB_init(s, Y));
    const int steps = s->scf_iter == 0 ? s->n_inner_first : s->n_inner_steps;
    for (int i = 0; i < steps; ++i) DPP_TRY(cgB_step(s, Y));
    // 3. subspace diagonalization
    std::vector<double> ev((size_t)nk * nb);
    DPP_TRY(subspace_rotate(s, Y, ev.data()));
    if (eig) std::copy(ev.begin(), ev.end(), eig);
    // band residual (Y orthonormal eigenvectors, HY = H Y): drives the switch
    // from the bulk precision to FP64
    {
        TimerScope ts_(s->ctx, DPP_TK_BLOCKOPS);
        hipLaunchKernelGGL(k_band_residual, dim3(nb, nk), dim3(256), 0, stream(s), s->d_seg, nb, nb, s->d_eig,
                           s->grid->omega, (const double2*)Y, (const double2*)s->HY, s->d_res);
        DPP_LAUNCHED();
        std::vector<double> res((size_t)nk * nb);
        DPP_HIP(hipMemcpyAsync(res.data(), s->d_res, res.size() * sizeof(double), hipMemcpyDeviceToHost, stream(s)));
        DPP_HIP(hipStreamSynchronize(stream(s)));
        s->last_res = *std::max_element(res.begin(), res.end());
    }
    // 4. aufbau fillings
    aufbau(ev, nk, nb, s->wk, s->ne, s->fill);
    DPP_TRY(upload(s, s->d_f, s->fill));
    // 5. n_out and E_el[psi, n_out]
    DPP_HIP(hipMemsetAsync(s->nout, 0, N * sizeof(double), stream(s)));
    DPP_TRY(density_all(s, nb, Y, s->nout, s->prec));
    const double om = s->grid->omega;
    DPP_TRY(dpp_hartree(s->grid, s->nout, s->VH, s->d_E + 2, s->gws));
    DPP_TRY(dpp_lda_pz81(s->grid, s->nout, s->vxc, s->d_E + 3, s->gws));
    DPP_TRY(dpp_grid_dot(s->grid, s->Vloc, s->nout, om / (double)N, s->d_E + 4, s->gws));
    hipLaunchKernelGGL(k_seg_kinetic, dim3(DOT_BLOCKS, nk), dim3(256), 0, stream(s), s->d_seg, nb, nb, s->d_f, Y,
                       s->d_part);
    DPP_LAUNCHED();
    hipLaunchKernelGGL(k_seg_weighted_total, dim3(1), dim3(1), 0, stream(s), s->d_part, nk, s->d_wk, 0.5 * om, s->d_E);
    DPP_LAUNCHED();
    if (s->nproj > 0) {
        DPP_TRY(proj_overlaps(s, nb, Y));
        hipLaunchKernelGGL(k_nonlocal_energy, dim3(1), dim3(256), 0, stream(s), nk, s->nproj, nb, s->nb, s->Pi,
                           s->pi_stride, s->d_f, s->d_wk, s->D, s->d_E + 1);
        DPP_LAUNCHED();
    } else {
        DPP_HIP(hipMemsetAsync(s->d_E + 1, 0, sizeof(double), stream(s)));
    }
    // 6. Pulay mixing of n_in
    DPP_TRY(pulay_mix(s));
    double e[5];
    DPP_HIP(hipMemcpyAsync(e, s->d_E, 5 * sizeof(double), hipMemcpyDeviceToHost, stream(s)));
    DPP_HIP(hipStreamSynchronize(stream(s)));
    if (E) *E = dpp_energy{e[0] + e[1] + e[2] + e[3] + e[4], e[0], e[1], e[4], e[2], e[3]};
    s->scf_iter++;
    if (s->prec != DPP_F64 && s->refine_res > 0.0 && s->last_res >= 0.0 && s->last_res < s->refine_res)
        s->prec = DPP_F64;  // FP64 refinement for the rest of this SCF run
    return DPP_OK;
}

extern "C" dpp_status dpp_set_precision_policy(dpp_system s, int bulk, double refine_residual) {
    clear_error();
    DPP_REQUIRE(s && (bulk == DPP_F64 || bulk == DPP_F32) && refine_residual >= 0.0,
                "dpp_set_precision_policy: bad arguments");
    s->bulk_prec = (dpp_precision)bulk;
    s->prec = s->bulk_prec;
    s->refine_res = refine_residual;
    return DPP_OK;
}

extern "C" dpp_status dpp_scf_status(dpp_system s, double* residual, int* prec_now, int* iterations) {
    clear_error();
    DPP_REQUIRE(s, "dpp_scf_status: null system");
    if (residual) *residual = s->last_res;
    if (prec_now) *prec_now = s->prec;
    if (iterations) *iterations = s->scf_iter;
    return DPP_OK;
}

extern "C" dpp_status dpp_system_counters(dpp_system s, int64_t* hc_bandk) {
    clear_error();
    DPP_REQUIRE(s && hc_bandk, "dpp_system_counters: null argument");
    *hc_bandk = s->hc_bandk;
    return DPP_OK;
}

extern "C" dpp_status dpp_system_apply_H(dpp_system s, const dpp_c64* Y, dpp_c64* HY) {
    clear_error();
    DPP_REQUIRE(s && Y && HY && (const void*)Y != (const void*)HY, "dpp_system_apply_H: bad arguments");
    DPP_TRY(apply_H_all(s, s->nb, (const double2*)Y, (double2*)HY));
    return DPP_OK;
}

extern "C" dpp_status dpp_system_fillings(dpp_system s, double* f) {
    clear_error();
    DPP_REQUIRE(s && f, "dpp_system_fillings: null argument");
    DPP_REQUIRE(!s->fill.empty(), "dpp_system_fillings: no SCF iteration yet");
    std::copy(s->fill.begin(), s->fill.end(), f);
    return DPP_OK;
}
