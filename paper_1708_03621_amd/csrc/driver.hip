// Minimization and SCF drivers over a batch of periodic systems (cells, each
// with its k-points): preconditioned Polak-Ribiere CG for the total energy
// (variational minimization, one shared step length; one cell) and for the
// band energy at fixed potential (one line search per k-point), and the SCF
// iteration with subspace diagonalization, aufbau fillings and Pulay mixing.
// (Sec. 2.1: Minimize and Pulay; Sec. 2.2: variational minimization vs SCF.)
//
// Work items are the (cell, k-point) pairs, numbered cell-major.  Every pass
// over wavefunction blocks, every small-matrix step and every field operation
// runs as one launch over all items (or all cells), whatever their box,
// sphere and band counts.  The band-energy CG keeps its whole state on the
// device (direction coefficients, line searches, retries, acceptance), so an
// SCF iteration involves no host round trip and can be captured once as a HIP
// graph and replayed.  Step rules:
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
#include <cstdio>
#include <cstring>
#include <map>
#include <string>
#include <unordered_map>
#include <vector>

#include "blockops.h"
#include "internal.h"
#include "../../include/dftpp.h"

using namespace dpp;

namespace {
constexpr int MAX_TRIES = 6;
constexpr int E_STRIDE = 8;  // per-cell energy slots
enum { EK = 0, ENL = 1, EH = 2, EXC = 3, ELOC = 4, ETS = 5, EMU = 6 };  // ETS: sigma S, EMU: mu (smearing)
constexpr int DENS_MAX_CHUNKS = 16;
}  // namespace

struct CellHost {
    dpp_grid grid;
    int nk, nb, nat, nproj;
    double ne, D;
    int item0;
    int64_t foff, N;
    std::vector<double> tau, Z, rc;  // atoms (tau Cartesian, 3 per atom)
    std::vector<int> has_proj;
};

// Buffers of dpp_system_forces, allocated on its first call.
struct ForceBufs {
    bool ready = false;
    double *tau = nullptr, *sfrac = nullptr, *Z = nullptr, *rc = nullptr;  // every atom, cell-major
    double2* Q = nullptr;      // derivative projectors: per item 3 x nproj x npw
    double2* Pid = nullptr;    // their overlaps with psi: per item 3 x nproj x nb
    double* part = nullptr;    // local-force chunk partials / Ewald partials
    double* nlpart = nullptr;  // per item nproj x 3
    double* E = nullptr;       // Ewald lattice sums per cell
    std::vector<int64_t> qoff, nloff, aoff;
    std::vector<int> proj_atom;  // per cell-major projector: the atom it sits on (within its cell)
    std::vector<int> proj0;      // per cell: first projector index
    int64_t natall = 0;
};

// Item table for a band count override (0: every item's own count) with the
// matching density-partial layout of the cells.
struct ItemTable {
    FftItem* d_items = nullptr;
    std::vector<FftItem> h;
    CellDesc* d_cells = nullptr;
    size_t dens_elems = 0;
    XzPlan xz;   // items grouped by x length for the register x pass
    PlanePlan pl; // items grouped by square y-z face for the register plane passes
};

struct ScfGraph {
    hipGraphExec_t exec;
    const void* Y;
    int steps;
    int prec;
};

struct dpp_system_s {
    dpp_ctx ctx;
    int ncells = 0, nit = 0;
    std::vector<CellHost> cells;
    std::vector<dpp_basis> bases;  // per item
    std::vector<dpp_ham> hams;     // per item
    std::vector<Seg> h_seg;
    std::vector<int64_t> off, npw, moff, pioff, f_off;
    std::vector<int> inb;
    std::vector<double> wk, omega_it;
    int64_t total = 0, msum = 0, pisum = 0, nstates = 0, Ntot = 0, maxN = 0;
    int maxnb = 0, maxnproj = 0;
    Seg* d_seg = nullptr;
    CellDesc* d_cells = nullptr;
    std::vector<CellDesc> h_cells;
    std::vector<FftItem> h_box;
    FftItem* d_box = nullptr;
    // x pass of H: V_eff copy in plane order, scaled (rebuilt when V_eff changed)
    std::vector<FftItem> h_vx;
    FftItem* d_vx = nullptr;
    double* Vx = nullptr;
    bool vx_dirty = true;
    // block buffers (total elements each)
    double2 *HY, *Dd, *HD, *g, *g2, *Kg, *gp, *Dp, *psi, *T1, *T2;
    // small matrices (msum elements each) and projector overlaps (pisum)
    double2 *U, *Rinv, *H0, *X, *Q, *H1, *H2, *Rt, *M1, *M2, *vecs, *Pi;
    double2* eig_scr;
    // scalars
    double *d_dots, *d_part, *d_E, *d_f, *d_eig, *d_res, *d_ones, *d_alpha, *d_beta, *d_bE0, *d_cred, *d_epart;
    CgBState cg;
    // fields (Ntot each)
    double *Vloc, *VH, *vxc, *Veff, *n, *nin, *nout;
    double *hist_n, *hist_r, *pulayA, *pulayC;
    int* d_pst;
    int* d_perm;  // eigensolver output order (EIG_TILE_MAXN per item)
    // workspaces
    void* Tplanes;
    size_t tplane_elems = 0;  // complex FP64 elements
    double* dens_part;
    size_t dens_part_elems = 0;
    double2* ov_part;
    size_t ov_part_elems = 0;
    void* gws;
    std::map<int, ItemTable> items;
    std::unordered_map<std::string, void*> tables;
    // protocol V (host-driven, one cell)
    double vE0 = 0, vat = 0, vgkg = 0, vf = 0;
    int vreset = 1, vstat = 0, vnocc = 0;
    // SCF
    int n_inner_steps = 3, n_inner_first = 3, scf_iter = 0;
    bool cgB_ready = false;
    int64_t hc_bandk = 0;
    dpp_precision prec = DPP_F64, bulk_prec = DPP_F64;
    double refine_res = 0.0, last_res = -1.0;
    std::vector<double> cell_res;
    // launch choices: fixed layout choices, and the ones dpp_system_tune times
    bool reg_xpass = true;  // register-resident x pass of H where S0 is compiled in
    bool reg_planes = true; // register plane passes (digit-reversed planes) for square y-z faces
    int xc = DPP_XC_LDA_PZ81;      // exchange-correlation functional of the SCF
    double smear = 0.0;            // Fermi-Dirac width of the SCF fillings (0: aufbau)
    void* gga_ws = nullptr;        // PBE workspace (largest cell) and a scratch energy
    double* d_gga_scratch = nullptr;
    int rot_pt = 0;         // rotate point tiles per wave (0: by launch size)
    int ov_mode = 0;        // overlap launch shape (0 auto: staged 4x4 blocks when every task has 4x4 tiles,
                            // else chunked 2x2 blocks; 1 chunked single tiles, 2 single pass, 3 staged)
    std::string tune_report;
    // graphs
    bool graph_on = false;
    hipStream_t cap_stream = nullptr;
    std::vector<ScfGraph> graphs;
    // pinned staging ring for small host -> device uploads (protocol V)
    double* h_ring = nullptr;
    double* h_rep = nullptr;  // pinned: energies, residuals, eigenvalues of an SCF iteration
    int ring_slot = 0, ring_slots = 64;
    size_t ring_len = 256;
    std::vector<void*> allocs;
    ForceBufs fb;
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

hipStream_t stream(const dpp_system_s* s) { return s->ctx->stream; }

int nb_of(const dpp_system_s* s, int nbo, int k) { return nbo > 0 ? nbo : s->inb[k]; }

unsigned seg_blocks(const dpp_system_s* s, int nbo) {
    int64_t mx = 0;
    for (int k = 0; k < s->nit; ++k) mx = std::max<int64_t>(mx, (int64_t)nb_of(s, nbo, k) * s->npw[k]);
    return (unsigned)std::min<int64_t>(1024, std::max<int64_t>(1, (mx + 255) / 256));
}

// Device copy of a host table, created on first use and kept for the life of
// the system (identical tables share one copy).  Tables are made during the
// first, eager pass of each operation, so a captured graph only refers to
// existing ones.
dpp_status table(dpp_system_s* s, const void* data, size_t bytes, const void** dev) {
    std::string key(reinterpret_cast<const char*>(data), bytes);
    auto it = s->tables.find(key);
    if (it != s->tables.end()) {
        *dev = it->second;
        return DPP_OK;
    }
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    DPP_HIP(hipStreamIsCapturing(stream(s), &cs));
    if (cs != hipStreamCaptureStatusNone) return set_error(DPP_EUNSUPPORTED, "task table missing during capture");
    void* p = nullptr;
    if (hipMalloc(&p, std::max<size_t>(bytes, 256)) != hipSuccess)
        return set_error(DPP_ENOMEM, "task table allocation failed");
    s->allocs.push_back(p);
    DPP_HIP(hipMemcpy(p, data, bytes, hipMemcpyHostToDevice));
    s->tables.emplace(std::move(key), p);
    *dev = p;
    return DPP_OK;
}

template <typename T>
dpp_status table_t(dpp_system_s* s, const std::vector<T>& v, const T** dev) {
    const void* p = nullptr;
    DPP_TRY(table(s, v.data(), v.size() * sizeof(T), &p));
    *dev = reinterpret_cast<const T*>(p);
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

// Density band chunks of an item: enough workgroups to fill the chip, few
// enough partial boxes to keep the partial traffic small.
int dens_chunks(int nb, int S1, int nit) {
    int c = (1024 + S1 * nit - 1) / (S1 * nit);
    c = std::max(1, std::min(c, std::min(nb, DENS_MAX_CHUNKS)));
    const int chunk = (nb + c - 1) / c;
    return (nb + chunk - 1) / chunk;
}

dpp_status items_for(dpp_system_s* s, int nbo, const ItemTable** out) {
    auto f = s->items.find(nbo);
    if (f != s->items.end()) {
        *out = &f->second;
        return DPP_OK;
    }
    ItemTable t;
    int64_t toff = 0, poff = 0;
    std::vector<CellDesc> cd = s->h_cells;
    for (int c = 0; c < s->ncells; ++c) {
        const CellHost& ch = s->cells[c];
        cd[c].pstart = poff;
        int np = 0;
        for (int k = ch.item0; k < ch.item0 + ch.nk; ++k) {
            FftItem it = s->bases[k]->h_item;
            it.nb = nb_of(s, nbo, k);
            it.ld = s->npw[k];
            it.c_off = s->off[k];
            it.t_off = toff;
            it.v_off = ch.foff;
            it.wk = s->wk[k];
            it.f_off = s->f_off[k];
            it.dnch = dens_chunks(it.nb, it.S1, s->nit);
            it.dchunk = (it.nb + it.dnch - 1) / it.dnch;
            it.p_off = poff;
            it.perm = (s->reg_planes && it.S1 == it.S2 && plane_reg_supported(it.S1)) ? 1 : 0;
            it.vperm = 0;  // the x pass reads Vx
            poff += (int64_t)it.dnch * ch.N;
            np += it.dnch;
            toff += (int64_t)it.nb * it.nplanes * it.S1 * it.S2;
            t.h.push_back(it);
        }
        cd[c].nparts = np;
    }
    if ((size_t)poff > s->dens_part_elems) return set_error(DPP_EUNSUPPORTED, "density partial buffer too small");
    if ((size_t)toff > s->tplane_elems) return set_error(DPP_EUNSUPPORTED, "plane buffer too small");
    DPP_TRY(dalloc_t(s, &t.d_items, t.h.size()));
    DPP_HIP(hipMemcpy(t.d_items, t.h.data(), t.h.size() * sizeof(FftItem), hipMemcpyHostToDevice));
    DPP_TRY(dalloc_t(s, &t.d_cells, cd.size()));
    DPP_HIP(hipMemcpy(t.d_cells, cd.data(), cd.size() * sizeof(CellDesc), hipMemcpyHostToDevice));
    t.dens_elems = (size_t)poff;
    std::vector<std::vector<int>> members;
    t.xz = xz_plan_groups(t.h, members);
    if (t.xz.S0.size() > 1)
        for (size_t g = 0; g < members.size(); ++g) {
            int* d = nullptr;
            DPP_TRY(dalloc_t(s, &d, members[g].size()));
            DPP_HIP(hipMemcpy(d, members[g].data(), members[g].size() * sizeof(int), hipMemcpyHostToDevice));
            t.xz.idx[g] = d;
        }
    t.pl = plane_plan_groups(t.h, members);
    if (t.pl.N.size() > 1)
        for (size_t g = 0; g < members.size(); ++g) {
            int* d = nullptr;
            DPP_TRY(dalloc_t(s, &d, members[g].size()));
            DPP_HIP(hipMemcpy(d, members[g].data(), members[g].size() * sizeof(int), hipMemcpyHostToDevice));
            t.pl.idx[g] = d;
        }
    auto ins = s->items.emplace(nbo, std::move(t));
    *out = &ins.first->second;
    return DPP_OK;
}

// ---------------------------------------------------------- batched ops ---
struct OvJob {
    const double2* A;   // packed block set
    const double2* B;
    double scale;
    bool by_omega;      // scale times the item's cell volume
    double2* out;       // item matrices at moff
};

// Overlap launch over a task table with its work list (only the workgroups
// that have work are launched).
// The contractions follow the system's current precision: split-BF16 (A^dag B)
// and FP32 (X M) MFMA in the mixed-precision bulk, FP64 otherwise.
dpp_status overlap_run(dpp_system_s* s, const std::vector<OvTask>& t, const OvTask* d, const int* act) {
    std::vector<int4> w;
    if (s->prec == DPP_F32)
        overlap_worklist_bf16(t, w);
    else
        overlap_worklist(t, s->ov_mode, w);
    const int4* dw = nullptr;
    DPP_TRY(table_t(s, w, &dw));
    return overlap_tasks(s->ctx, t, d, s->ov_part, act, s->ov_mode, dw, (int)w.size(), s->prec);
}

dpp_status rotate_run(dpp_system_s* s, const std::vector<RotTask>& t, const RotTask* d, const int* act) {
    std::vector<int2> w;
    rotate_worklist(t, s->rot_pt, w, s->prec == DPP_F32);
    const int2* dw = nullptr;
    DPP_TRY(table_t(s, w, &dw));
    return rotate_tasks(s->ctx, t, d, act, s->rot_pt, dw, (int)w.size(), s->prec);
}

// Several A^dag B contractions over every item in one launch (nbo bands).
dpp_status overlap_jobs(dpp_system_s* s, int nbo, const std::vector<OvJob>& jobs, const int* act = nullptr) {
    std::vector<OvTask> t;
    int64_t poff = 0;
    for (const OvJob& j : jobs)
        for (int k = 0; k < s->nit; ++k) {
            const int nb = nb_of(s, nbo, k);
            OvTask x = make_ov_task((int)s->npw[k], nb, j.A + s->off[k], s->npw[k], nb, j.B + s->off[k], s->npw[k],
                                    j.by_omega ? j.scale * s->omega_it[k] : j.scale, j.out + s->moff[k], nb);
            x.part_off = poff;
            x.item = k;
            poff += (int64_t)x.nchunk * x.ntiles * 256;
            t.push_back(x);
        }
    if ((size_t)poff > s->ov_part_elems) return set_error(DPP_EUNSUPPORTED, "overlap partial buffer too small");
    const OvTask* d = nullptr;
    DPP_TRY(table_t(s, t, &d));
    return overlap_run(s, t, d, act);
}

struct RotJob {
    const double2* X;
    const double2* M;   // item matrices at moff (row length = bands)
    double beta;
    double2* out;
    const double2* X2 = nullptr;  // optional second term out += X2 M2
    const double2* M2 = nullptr;
};

dpp_status rotate_jobs(dpp_system_s* s, int nbo, const std::vector<RotJob>& jobs, const int* act = nullptr) {
    std::vector<RotTask> t;
    for (const RotJob& j : jobs)
        for (int k = 0; k < s->nit; ++k) {
            const int nb = nb_of(s, nbo, k);
            RotTask r = make_rot_task((int)s->npw[k], nb, j.X + s->off[k], s->npw[k], nb, j.M + s->moff[k], nb, j.beta,
                                      j.out + s->off[k], s->npw[k]);
            r.item = k;
            if (j.X2) {
                r.nbX2 = nb;
                r.X2 = j.X2 + s->off[k];
                r.M2 = j.M2 + s->moff[k];
            }
            t.push_back(r);
        }
    const RotTask* d = nullptr;
    DPP_TRY(table_t(s, t, &d));
    return rotate_run(s, t, d, act);
}

// HX = H X for nbo bands of every item: batched FFT passes at each cell's
// V_eff, then the projector terms HX += P (D P^dag X) as two batched
// contractions (items of cells with projectors).
dpp_status apply_H_all(dpp_system_s* s, int nbo, const double2* X, double2* HX, const int* act = nullptr) {
    if (!act)
        for (int k = 0; k < s->nit; ++k) s->hc_bandk += nb_of(s, nbo, k);
    const ItemTable* it;
    DPP_TRY(items_for(s, nbo, &it));
    const XzPlan* plan = s->reg_xpass ? &it->xz : nullptr;
    if (s->vx_dirty) {
        DPP_TRY(vx_cells(s->ctx, s->d_vx, s->ncells, s->maxN, s->Veff, s->Vx));
        s->vx_dirty = false;
    }
    if (s->prec == DPP_F64)
        DPP_TRY(apply_H_local_batched<double>(s->ctx, it->d_items, it->h, X, HX, s->Vx, s->Tplanes, act, plan,
                                              &it->pl));
    else
        DPP_TRY(apply_H_local_batched<float>(s->ctx, it->d_items, it->h, X, HX, s->Vx, s->Tplanes, act, plan,
                                             &it->pl));
    if (s->maxnproj > 0) {
        std::vector<OvTask> t;
        std::vector<RotTask> r;
        int64_t poff = 0;
        for (int k = 0; k < s->nit; ++k) {
            const dpp_ham h = s->hams[k];
            if (h->nproj == 0) continue;
            const int nb = nb_of(s, nbo, k);
            OvTask x = make_ov_task((int)s->npw[k], h->nproj, h->d_P, s->npw[k], nb, X + s->off[k], s->npw[k], h->D,
                                    s->Pi + s->pioff[k], nb);
            x.part_off = poff;
            x.item = k;
            poff += (int64_t)x.nchunk * x.ntiles * 256;
            t.push_back(x);
            RotTask y = make_rot_task((int)s->npw[k], h->nproj, h->d_P, s->npw[k], nb, s->Pi + s->pioff[k], nb, 1.0,
                                      HX + s->off[k], s->npw[k]);
            y.item = k;
            r.push_back(y);
        }
        if ((size_t)poff > s->ov_part_elems) return set_error(DPP_EUNSUPPORTED, "overlap partial buffer too small");
        const OvTask* dt = nullptr;
        DPP_TRY(table_t(s, t, &dt));
        DPP_TRY(overlap_run(s, t, dt, act));
        const RotTask* dr = nullptr;
        DPP_TRY(table_t(s, r, &dr));
        DPP_TRY(rotate_run(s, r, dr, act));
    }
    return DPP_OK;
}

// Pi_k = P_k^dag X_k (nproj x nbands, row length nbands) for every item.
dpp_status proj_overlaps(dpp_system_s* s, int nbo, const double2* X) {
    std::vector<OvTask> t;
    int64_t poff = 0;
    for (int k = 0; k < s->nit; ++k) {
        const dpp_ham h = s->hams[k];
        if (h->nproj == 0) continue;
        const int nb = nb_of(s, nbo, k);
        OvTask x = make_ov_task((int)s->npw[k], h->nproj, h->d_P, s->npw[k], nb, X + s->off[k], s->npw[k], 1.0,
                                s->Pi + s->pioff[k], nb);
        x.part_off = poff;
        x.item = k;
        poff += (int64_t)x.nchunk * x.ntiles * 256;
        t.push_back(x);
    }
    if (t.empty()) return DPP_OK;
    const OvTask* dt = nullptr;
    DPP_TRY(table_t(s, t, &dt));
    return overlap_run(s, t, dt, nullptr);
}

// n = sum_k w_k sum_i f_ki |I psi_ki|^2 per cell over nbo bands (fillings at d_f).
dpp_status density_all(dpp_system_s* s, int nbo, const double2* psi, double* n, dpp_precision prec) {
    const ItemTable* it;
    DPP_TRY(items_for(s, nbo, &it));
    const XzPlan* xp = s->reg_xpass ? &it->xz : nullptr;
    if (prec == DPP_F64)
        return density_batched<double>(s->ctx, it->d_items, it->h, psi, s->d_f, s->Tplanes, s->dens_part,
                                       it->d_cells, s->ncells, s->maxN, n, &it->pl, xp);
    return density_batched<float>(s->ctx, it->d_items, it->h, psi, s->d_f, s->Tplanes, s->dens_part, it->d_cells,
                                  s->ncells, s->maxN, n, &it->pl, xp);
}

dpp_status axpby_all(dpp_system_s* s, int nbo, const double* a, const double2* x, const double* b, const double2* y,
                     double2* out) {
    TimerScope ts_(s->ctx, DPP_TK_BLOCKOPS);
    hipLaunchKernelGGL(k_seg_axpby, dim3(seg_blocks(s, nbo), s->nit), dim3(256), 0, stream(s), s->d_seg, nbo, a, x, b,
                       y, out);
    DPP_LAUNCHED();
    return DPP_OK;
}

dpp_status precond_all(dpp_system_s* s, int nbo, const double2* x, double2* out) {
    TimerScope ts_(s->ctx, DPP_TK_BLOCKOPS);
    hipLaunchKernelGGL(k_seg_precond, dim3(seg_blocks(s, nbo), s->nit), dim3(256), 0, stream(s), s->d_seg, nbo, 1.0,
                       x, out);
    DPP_LAUNCHED();
    return DPP_OK;
}

// dots[p * (nit + 1) + k] per item and the totals at k = nit (device).
dpp_status dots_dev(dpp_system_s* s, int nbo, int npair, const double2* const* a, const double2* const* b) {
    TimerScope ts_(s->ctx, DPP_TK_BLOCKOPS);
    DotPairs pr;
    for (int p = 0; p < 4; ++p) {
        pr.a[p] = p < npair ? a[p] : nullptr;
        pr.b[p] = p < npair ? b[p] : nullptr;
    }
    const int nblk = dot_blocks(s->nit);
    hipLaunchKernelGGL(k_seg_dots, dim3(nblk, s->nit), dim3(256), 0, stream(s), s->d_seg, s->nit, nbo, npair, pr,
                       s->d_part);
    DPP_LAUNCHED();
    hipLaunchKernelGGL(k_seg_dots_reduce, dim3(npair), dim3(64), 0, stream(s), (const double*)s->d_part, s->nit, npair,
                       s->d_dots, nblk);
    DPP_LAUNCHED();
    return DPP_OK;
}

dpp_status dots_host(dpp_system_s* s, int nbo, int npair, const double2* const* a, const double2* const* b,
                     std::vector<double>& host) {
    DPP_TRY(dots_dev(s, nbo, npair, a, b));
    host.assign((size_t)npair * (s->nit + 1), 0.0);
    DPP_HIP(hipMemcpyAsync(host.data(), s->d_dots, host.size() * sizeof(double), hipMemcpyDeviceToHost, stream(s)));
    DPP_HIP(hipStreamSynchronize(stream(s)));
    return DPP_OK;
}

dpp_status smm(dpp_system_s* s, int nbo, int opA, int opB, double alpha, int alpha_omega, const double2* A,
               const double2* B, double beta, double2* C) {
    TimerScope ts_(s->ctx, DPP_TK_BLOCKOPS);
    const int n = nbo > 0 ? nbo : s->maxnb;
    const int tn = (n + 15) / 16;
    hipLaunchKernelGGL(k_smm_mfma, dim3(tn * tn, s->nit), dim3(64), 0, stream(s), s->d_seg, nbo, opA, opB, alpha,
                       alpha_omega, A, B, beta, C);
    DPP_LAUNCHED();
    return DPP_OK;
}

dpp_status chol_all(dpp_system_s* s, int nbo, const double2* Um, double2* Ri) {
    const int n = nbo > 0 ? nbo : s->maxnb;
    TimerScope ts_(s->ctx, DPP_TK_CHOLESKY);
    if (!cholesky_wave_launch(stream(s), (unsigned)s->nit, n, 0, s->d_seg, nbo, Um, Ri, s->ctx->d_status, nullptr))
        DPP_HIP(cholesky_tiles_launch(stream(s), (unsigned)s->nit, n, s->d_seg, nbo, 0, Um, Ri, s->ctx->d_status,
                                      nullptr));
    DPP_LAUNCHED();
    return DPP_OK;
}

dpp_status copy_blocks(dpp_system_s* s, const double2* src, double2* dst) {
    TimerScope ts_(s->ctx, DPP_TK_BLOCKOPS);
    const unsigned nbk = (unsigned)std::min<int64_t>(4096, (s->total + 255) / 256);
    hipLaunchKernelGGL(k_copy, dim3(std::max(1u, nbk)), dim3(256), 0, stream(s), s->total, src, dst);
    DPP_LAUNCHED();
    return DPP_OK;
}

dpp_status fill(dpp_system_s* s, double* p, int64_t n, double v) {
    const unsigned nbk = (unsigned)std::min<int64_t>(4096, (n + 255) / 256);
    hipLaunchKernelGGL(k_fill, dim3(std::max(1u, nbk)), dim3(256), 0, stream(s), n, v, p);
    DPP_LAUNCHED();
    return DPP_OK;
}

// ----------------------------------------------------- fields and energies --
// v_xc[n] of every cell (and E_xc into E[c * E_STRIDE] when E is given):
// LDA for all cells in one launch, PBE per cell on the cell's full box.
dpp_status xc_cells(dpp_system_s* s, const double* n, double* E) {
    if (s->xc == DPP_XC_LDA_PZ81) return lda_cells(s->ctx, s->d_cells, s->ncells, n, s->vxc, s->d_cred, E, E_STRIDE);
    for (int c = 0; c < s->ncells; ++c) {
        const CellHost& ch = s->cells[c];
        double* Ec = E ? E + (int64_t)c * E_STRIDE : s->d_gga_scratch;
        DPP_TRY(gga_pbe(ch.grid, n + ch.foff, s->vxc + ch.foff, Ec, s->gga_ws));
    }
    return DPP_OK;
}

// V_eff = V_loc + V_H[n] + v_xc[n] for every cell.
dpp_status potentials(dpp_system_s* s, const double* n) {
    // the potentials only: the energies are those of the output density
    DPP_TRY(hartree_batched(s->ctx, s->d_box, s->h_box, n, s->VH, s->Tplanes, s->d_epart, s->d_cells, nullptr,
                            E_STRIDE));
    DPP_TRY(xc_cells(s, n, nullptr));
    TimerScope ts_(s->ctx, DPP_TK_FIELDS);
    hipLaunchKernelGGL(k_grid_lin3, dim3((unsigned)((s->Ntot + 255) / 256)), dim3(256), 0, stream(s), s->Ntot, 1.0,
                       s->Vloc, 1.0, s->VH, 1.0, s->vxc, s->Veff);
    DPP_LAUNCHED();
    s->vx_dirty = true;
    return DPP_OK;
}

// Energy terms of every cell at orthonormal psi (nbo bands, fillings d_f) and
// density n: d_E[c * E_STRIDE + {EK, ENL, EH, EXC, ELOC}].  Leaves v_xc, and
// V_H unless with_vh is false.
dpp_status energies(dpp_system_s* s, int nbo, const double2* psi, const double* n, bool with_vh = true) {
    DPP_TRY(hartree_batched(s->ctx, s->d_box, s->h_box, n, with_vh ? s->VH : nullptr, s->Tplanes, s->d_epart,
                            s->d_cells, s->d_E + EH, E_STRIDE));
    DPP_TRY(xc_cells(s, n, s->d_E + EXC));
    DPP_TRY(dot_cells(s->ctx, s->d_cells, s->ncells, s->Vloc, n, s->d_cred, s->d_E + ELOC, E_STRIDE));
    {
        TimerScope ts_(s->ctx, DPP_TK_BLOCKOPS);
        hipLaunchKernelGGL(k_seg_kinetic, dim3(dot_blocks(s->nit), s->nit), dim3(256), 0, stream(s), s->d_seg, nbo,
                           (const double*)s->d_f, psi, s->d_part);
        DPP_LAUNCHED();
        hipLaunchKernelGGL(k_cell_weighted_totals, dim3((s->ncells + 63) / 64), dim3(64), 0, stream(s),
                           (const double*)s->d_part, s->d_seg, s->d_cells, s->ncells, 0.5, s->d_E + EK, E_STRIDE,
                           dot_blocks(s->nit));
        DPP_LAUNCHED();
    }
    DPP_TRY(proj_overlaps(s, nbo, psi));
    TimerScope ts_(s->ctx, DPP_TK_BLOCKOPS);
    hipLaunchKernelGGL(k_nonlocal_energy, dim3(s->ncells), dim3(256), 0, stream(s), s->d_seg, s->d_cells, nbo,
                       (const double2*)s->Pi, (const double*)s->d_f, s->d_E + ENL, E_STRIDE);
    DPP_LAUNCHED();
    return DPP_OK;
}

// Pulay (DIIS) mixing of n_in from n_out for every cell; history on the device.
dpp_status pulay_mix(dpp_system_s* s) {
    TimerScope ts_(s->ctx, DPP_TK_FIELDS);
    const double alpha = 0.5;
    hipLaunchKernelGGL(k_pulay_begin, dim3(1), dim3(64), 0, stream(s), s->d_pst);
    DPP_LAUNCHED();
    hipLaunchKernelGGL(k_pulay_store, dim3((unsigned)((s->Ntot + 255) / 256)), dim3(256), 0, stream(s), s->Ntot,
                       (const int*)s->d_pst, (const double*)s->nin, (const double*)s->nout, s->hist_n, s->hist_r);
    DPP_LAUNCHED();
    hipLaunchKernelGGL(k_pulay_dots, dim3(MDOT_BLOCKS, s->ncells), dim3(256), 0, stream(s), s->Ntot,
                       (const int*)s->d_pst, s->d_cells, (const double*)s->hist_r, s->d_part);
    DPP_LAUNCHED();
    hipLaunchKernelGGL(k_pulay_solve_cells, dim3(s->ncells), dim3(256), 0, stream(s), s->ncells,
                       (const int*)s->d_pst, s->d_cells, (const double*)s->d_part, s->pulayA, s->pulayC,
                       s->ctx->d_status);
    DPP_LAUNCHED();
    hipLaunchKernelGGL(k_pulay_combine_cells, dim3((unsigned)((s->maxN + 255) / 256), s->ncells), dim3(256), 0,
                       stream(s), s->Ntot, (const int*)s->d_pst, s->d_cells, (const double*)s->pulayC, alpha,
                       (const double*)s->hist_n, (const double*)s->hist_r, s->nin);
    DPP_LAUNCHED();
    return DPP_OK;
}

// ----------------------------------------------------- band energy (B) ---
// Gradient state at the current Y: U, Rinv, H0 = Y^dag H Y,
// g = (HY - O Y U^{-1} H0) U^{-1}, E0_k = Tr(U^{-1} H0) (device); requires HY.
// after_step: Y and HY were just advanced by the accepted step along the line
// of X, Q, H1, H2; with up to 32 bands U and H0 then follow from those
// matrices (the line search's model of them) without new overlaps.
dpp_status grad_B(dpp_system_s* s, const double2* Y, bool after_step = false) {
    // after a step U and H0 follow from the line matrices (both kernels below)
    if (!after_step)
        DPP_TRY(overlap_jobs(s, 0, {OvJob{Y, Y, 1.0, true, s->U}, OvJob{Y, s->HY, 1.0, false, s->H0}}));
    bool fused = false;
    {
        // up to 32 bands: factor, U^{-1}, M2 and E0 in one single-wave launch
        TimerScope ts_(s->ctx, DPP_TK_CHOLESKY);
        fused = grad_prep_wave_launch(stream(s), (unsigned)s->nit, s->maxnb, s->d_seg, s->U, s->H0, s->Rinv, s->M1,
                                      s->M2, s->d_bE0, s->ctx->d_status, after_step ? s->cg.stepf : nullptr, s->X,
                                      s->Q, s->H1, s->H2);
        if (fused) DPP_LAUNCHED();
        // more bands: U^{-1} and E0 on register tiles, one workgroup per item
        // (R^{-1} is formed where it is used, in the subspace rotation)
        if (!fused)
            DPP_HIP(grad_prep_tiles_launch(stream(s), (unsigned)s->nit, s->maxnb, s->d_seg, s->U, s->H0, s->M1,
                                           s->d_bE0, s->ctx->d_status, after_step ? s->cg.stepf : nullptr, s->X,
                                           s->Q, s->H1, s->H2));
    }
    if (!fused) {
        // M2 = -Omega Uinv H0 Uinv
        DPP_TRY(smm(s, 0, 0, 0, 1.0, 0, s->M1, s->H0, 0.0, s->Rt));
        DPP_TRY(smm(s, 0, 0, 0, -1.0, 1, s->Rt, s->M1, 0.0, s->M2));
    }
    // g = HY Uinv + Y M2 in one pass
    DPP_TRY(rotate_jobs(s, 0, {RotJob{s->HY, s->M1, 0.0, s->g, Y, s->M2}}));
    return DPP_OK;
}

// Small matrices of the line along D: X = Y^dag O D, Q = D^dag O D, H1 = Y^dag H D, H2 = D^dag H D.
dpp_status line_mats_B(dpp_system_s* s, const double2* Y, const int* act) {
    DPP_TRY(apply_H_all(s, 0, s->Dd, s->HD, act));
    DPP_TRY(overlap_jobs(s, 0,
                         {OvJob{Y, s->Dd, 1.0, true, s->X}, OvJob{s->Dd, s->Dd, 1.0, true, s->Q},
                          OvJob{Y, s->HD, 1.0, false, s->H1}, OvJob{s->Dd, s->HD, 1.0, false, s->H2}},
                         act));
    return DPP_OK;
}

dpp_status linesearch_B(dpp_system_s* s, const int* act, const double* d0, int* ok, double* step) {
    const int n = s->maxnb;
    TimerScope ts_(s->ctx, DPP_TK_LINESEARCH);
    if (!linesearch_wave_launch(stream(s), (unsigned)s->nit, n, s->d_seg, s->U, s->X, s->Q, s->H0, s->H1, s->H2,
                                s->d_bE0, s->cg.at, d0, act, ok, step, s->M1, s->M2))
        DPP_HIP(linesearch_tiles_launch(stream(s), (unsigned)s->nit, n, s->d_seg, s->U, s->X, s->Q, s->H0, s->H1,
                                        s->H2, s->d_bE0, s->cg.at, d0, act, ok, step));
    DPP_LAUNCHED();
    return DPP_OK;
}

unsigned item_threads_blocks(const dpp_system_s* s) { return (unsigned)((s->nit + 63) / 64); }

dpp_status cgB_init(dpp_system_s* s, double2* Y) {
    // orthonormalize the starting block: Y <- Y R^{-1}
    DPP_TRY(overlap_jobs(s, 0, {OvJob{Y, Y, 1.0, true, s->U}}));
    DPP_TRY(chol_all(s, 0, s->U, s->Rinv));
    DPP_TRY(copy_blocks(s, Y, s->T1));
    DPP_TRY(rotate_jobs(s, 0, {RotJob{s->T1, s->Rinv, 0.0, Y}}));
    DPP_TRY(apply_H_all(s, 0, Y, s->HY));
    DPP_TRY(grad_B(s, Y));
    hipLaunchKernelGGL(k_cgB_reset, dim3(item_threads_blocks(s)), dim3(64), 0, stream(s), s->nit, s->d_seg, s->cg);
    DPP_LAUNCHED();
    s->cgB_ready = true;
    return DPP_OK;
}

dpp_status cgB_step(dpp_system_s* s, double2* Y) {
    const dim3 eg(seg_blocks(s, 0), s->nit);
    {
        // Kg and the direction dots, then beta and D = -Kg + beta D_prev
        TimerScope ts_(s->ctx, DPP_TK_BLOCKOPS);
        hipLaunchKernelGGL(k_cg_precond_dots, dim3(dot_blocks(s->nit), s->nit), dim3(256), 0, stream(s), s->d_seg, s->nit,
                           (const double2*)s->g, (const double2*)s->gp, (const double2*)s->Dp, s->Kg, s->d_part);
        DPP_LAUNCHED();
        hipLaunchKernelGGL(k_cgB_direction, eg, dim3(256), 0, stream(s), s->d_seg, s->nit, (const double*)s->d_part,
                           s->d_dots, s->cg, (const double2*)s->Kg, (const double2*)s->Dp, s->Dd, dot_blocks(s->nit));
        DPP_LAUNCHED();
    }
    DPP_TRY(line_mats_B(s, Y, nullptr));
    DPP_TRY(linesearch_B(s, s->cg.act, s->cg.d0, s->cg.ok, s->cg.step));
    {
        // failed CG directions: one more search along -K g (masked to those items)
        TimerScope ts_(s->ctx, DPP_TK_BLOCKOPS);
        hipLaunchKernelGGL(k_cgB_retry_axpby, eg, dim3(256), 0, stream(s), s->d_seg, (const double*)s->d_dots, s->cg,
                           (const double2*)s->Kg, s->Dd);
        DPP_LAUNCHED();
    }
    DPP_TRY(line_mats_B(s, Y, s->cg.retry));
    DPP_TRY(linesearch_B(s, s->cg.retry, s->cg.d0r, s->cg.ok2, s->cg.step2));
    {
        // accept the steps; Y += step D, HY += step HD; history for the next direction
        TimerScope ts_(s->ctx, DPP_TK_BLOCKOPS);
        hipLaunchKernelGGL(k_cgB_finish_update, eg, dim3(256), 0, stream(s), s->d_seg, (const double*)s->d_dots,
                           s->cg, Y, (const double2*)s->Dd, s->HY, (const double2*)s->HD, (const double2*)s->g, s->gp,
                           s->Dp);
        DPP_LAUNCHED();
    }
    DPP_TRY(grad_B(s, Y, true));
    return DPP_OK;
}

// Subspace rotation at the current band-CG state: psi = Y R^{-1}, H~ = psi^dag H psi,
// H~ V = V eps; Y <- psi V, HY <- (H psi) V; eigenvalues to d_eig.
dpp_status subspace_rotate(dpp_system_s* s, double2* Y) {
    // the single-wave gradient preparation leaves R^{-1}; the tile one does not
    if (s->maxnb > EIGW_MAXN) DPP_TRY(chol_all(s, 0, s->U, s->Rinv));
    DPP_TRY(rotate_jobs(s, 0, {RotJob{Y, s->Rinv, 0.0, s->psi}, RotJob{s->HY, s->Rinv, 0.0, s->T1}}));
    DPP_TRY(overlap_jobs(s, 0, {OvJob{s->psi, s->T1, 1.0, false, s->H0}}));
    {
        TimerScope ts_(s->ctx, DPP_TK_EIGH);
        if (!eigh_wave_launch(stream(s), (unsigned)s->nit, s->maxnb, s->d_seg, s->H0, s->d_eig, s->vecs))
            DPP_HIP(eigh_tiles_launch(stream(s), (unsigned)s->nit, s->maxnb, s->d_seg, 0, s->H0, s->d_eig, s->vecs,
                                      s->eig_scr, s->d_perm));
        DPP_LAUNCHED();
    }
    DPP_TRY(rotate_jobs(s, 0, {RotJob{s->psi, s->vecs, 0.0, Y}, RotJob{s->T1, s->vecs, 0.0, s->HY}}));
    return DPP_OK;
}

// One SCF iteration of every cell, entirely in stream order (no host sync).
dpp_status scf_body(dpp_system_s* s, double2* Y, int steps) {
    // 1. V_eff[n_in]
    DPP_TRY(potentials(s, s->nin));
    // 2. band-energy CG, restarted, warm-started Y
    DPP_TRY(cgB_init(s, Y));
    for (int i = 0; i < steps; ++i) DPP_TRY(cgB_step(s, Y));
    // 3. subspace diagonalization and band residuals
    DPP_TRY(subspace_rotate(s, Y));
    {
        TimerScope ts_(s->ctx, DPP_TK_BLOCKOPS);
        hipLaunchKernelGGL(k_band_residual, dim3(s->maxnb, s->nit), dim3(256), 0, stream(s), s->d_seg,
                           (const double*)s->d_eig, (const double2*)Y, (const double2*)s->HY, s->d_res);
        DPP_LAUNCHED();
        // 4. fillings per cell: aufbau, or Fermi-Dirac with mu, sigma S into the energy slots
        if (s->smear > 0.0)
            hipLaunchKernelGGL(k_fermi, dim3(s->ncells), dim3(256), 0, stream(s), s->d_cells, s->d_seg,
                               (const double*)s->d_eig, s->smear, s->d_f, s->d_E + ETS, E_STRIDE,
                               s->ctx->d_status);
        else
            hipLaunchKernelGGL(k_aufbau, dim3(s->ncells), dim3(256), 0, stream(s), s->d_cells, s->d_seg,
                               (const double*)s->d_eig, s->d_f, s->ctx->d_status);
        DPP_LAUNCHED();
    }
    // 5. n_out and E_el[psi, n_out]
    DPP_TRY(density_all(s, 0, Y, s->nout, s->prec));
    DPP_TRY(energies(s, 0, Y, s->nout, false));  // V_H[n_out] is not needed: the next V_eff is from the mixed n_in
    // 6. Pulay mixing of n_in
    DPP_TRY(pulay_mix(s));
    return DPP_OK;
}

dpp_status capture_scf(dpp_system_s* s, double2* Y, int steps, hipGraphExec_t* exec) {
    if (!s->cap_stream) DPP_HIP(hipStreamCreateWithFlags(&s->cap_stream, hipStreamNonBlocking));
    hipStream_t user = s->ctx->stream;
    const bool timer_on = s->ctx->timer.on;
    s->ctx->timer.on = false;
    s->ctx->stream = s->cap_stream;
    hipGraph_t graph = nullptr;
    dpp_status st = DPP_OK;
    // recording launches nothing: the H applications are counted when the
    // graph is launched, not while its body is recorded
    const int64_t hc_saved = s->hc_bandk;
    if (hipStreamBeginCapture(s->cap_stream, hipStreamCaptureModeRelaxed) != hipSuccess) {
        st = set_error(DPP_EDEVICE, "graph capture could not start");
    } else {
        st = scf_body(s, Y, steps);
        const hipError_t e = hipStreamEndCapture(s->cap_stream, &graph);
        if (st == DPP_OK && e != hipSuccess) st = set_error(DPP_EDEVICE, "graph capture failed");
    }
    s->ctx->stream = user;
    s->ctx->timer.on = timer_on;
    s->hc_bandk = hc_saved;
    if (st != DPP_OK) {
        if (graph) (void)hipGraphDestroy(graph);
        return st;
    }
    const hipError_t e = hipGraphInstantiate(exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) return set_error(DPP_EDEVICE, "graph instantiation failed");
    return DPP_OK;
}

// --------------------------------------------------- total energy (V) -----
struct Parts {
    double Ekin, Enl, Eloc, EH, Exc;
    double total() const { return Ekin + Enl + Eloc + EH + Exc; }
};

dpp_status read_parts(dpp_system_s* s, Parts& P) {
    double e[E_STRIDE];
    DPP_HIP(hipMemcpyAsync(e, s->d_E, E_STRIDE * sizeof(double), hipMemcpyDeviceToHost, stream(s)));
    DPP_HIP(hipStreamSynchronize(stream(s)));
    P = Parts{e[EK], e[ENL], e[ELOC], e[EH], e[EXC]};
    return DPP_OK;
}

// Density and energy of unorthonormalized Y (nocc bands, filling f): leaves
// psi, U, Rinv, n and V_eff for a following gradient.
dpp_status energy_V(dpp_system_s* s, const double2* Y, Parts& P) {
    const int nb = s->vnocc;
    DPP_TRY(overlap_jobs(s, nb, {OvJob{Y, Y, 1.0, true, s->U}}));
    DPP_TRY(chol_all(s, nb, s->U, s->Rinv));
    DPP_TRY(rotate_jobs(s, nb, {RotJob{Y, s->Rinv, 0.0, s->psi}}));
    DPP_TRY(density_all(s, nb, s->psi, s->n, DPP_F64));
    DPP_TRY(energies(s, nb, s->psi, s->n));
    {
        TimerScope ts_(s->ctx, DPP_TK_FIELDS);
        hipLaunchKernelGGL(k_grid_lin3, dim3((unsigned)((s->Ntot + 255) / 256)), dim3(256), 0, stream(s), s->Ntot,
                           1.0, s->Vloc, 1.0, s->VH, 1.0, s->vxc, s->Veff);
        DPP_LAUNCHED();
        s->vx_dirty = true;
    }
    return read_parts(s, P);
}

// Gradient after energy_V: g = w_k f (H psi - O psi Hsub) Rinv^dag into `gout`.
dpp_status grad_V(dpp_system_s* s, double2* gout) {
    const int nb = s->vnocc;
    DPP_TRY(apply_H_all(s, nb, s->psi, s->T1));
    DPP_TRY(overlap_jobs(s, nb, {OvJob{s->psi, s->T1, 1.0, false, s->H0}}));
    {
        TimerScope ts_(s->ctx, DPP_TK_BLOCKOPS);
        hipLaunchKernelGGL(k_sm_scale, dim3(s->nit), dim3(256), 0, stream(s), s->d_seg, nb, 0, -1.0, 2,
                           (const double2*)s->H0, s->M2);
        DPP_LAUNCHED();
    }
    DPP_TRY(rotate_jobs(s, nb, {RotJob{s->psi, s->M2, 1.0, s->T1}}));
    {
        TimerScope ts_(s->ctx, DPP_TK_BLOCKOPS);
        hipLaunchKernelGGL(k_sm_scale, dim3(s->nit), dim3(256), 0, stream(s), s->d_seg, nb, 1, s->vf, 1,
                           (const double2*)s->Rinv, s->M1);
        DPP_LAUNCHED();
    }
    DPP_TRY(rotate_jobs(s, nb, {RotJob{s->T1, s->M1, 0.0, gout}}));
    return DPP_OK;
}

dpp_status objective_V(dpp_system_s* s, const double2* Y, double2* gout, Parts& P) {
    DPP_TRY(energy_V(s, Y, P));
    DPP_TRY(grad_V(s, gout));
    return DPP_OK;
}

// out = Y + a D (nocc bands)
dpp_status trial_point(dpp_system_s* s, const double2* Y, double a, const double2* D, double2* out) {
    std::vector<double> av(s->nit, a);
    DPP_TRY(upload(s, s->d_alpha, av));
    DPP_TRY(axpby_all(s, s->vnocc, s->d_ones, Y, s->d_alpha, D, out));
    return DPP_OK;
}

dpp_status copy_bands(dpp_system_s* s, const double2* src, double2* dst, int nbands) {
    for (int k = 0; k < s->nit; ++k)
        DPP_HIP(hipMemcpyAsync(dst + s->off[k], src + s->off[k], (size_t)nbands * s->npw[k] * sizeof(double2),
                               hipMemcpyDeviceToDevice, stream(s)));
    return DPP_OK;
}

dpp_status cgV_init(dpp_system_s* s, double2* Y, int nocc, double f, Parts& P) {
    s->vnocc = nocc;
    s->vf = f;
    std::vector<double> fv((size_t)s->nstates, 0.0);
    for (int k = 0; k < s->nit; ++k)
        for (int i = 0; i < nocc; ++i) fv[(size_t)s->f_off[k] + i] = f;
    if (fv.size() > s->ring_len) return set_error(DPP_EINVAL, "cg_V: too many states");
    DPP_TRY(upload(s, s->d_f, fv));
    // orthonormalize the starting block once
    DPP_TRY(overlap_jobs(s, nocc, {OvJob{Y, Y, 1.0, true, s->U}}));
    DPP_TRY(chol_all(s, nocc, s->U, s->Rinv));
    DPP_TRY(copy_bands(s, Y, s->T1, nocc));
    DPP_TRY(rotate_jobs(s, nocc, {RotJob{s->T1, s->Rinv, 0.0, Y}}));
    DPP_TRY(objective_V(s, Y, s->g, P));
    s->vE0 = P.total();
    double wmax = 0;
    for (double w : s->wk) wmax = std::max(wmax, w);
    s->vat = 0.3 / (s->cells[0].grid->omega * f * wmax);
    s->vreset = 1;
    s->vstat = 0;
    s->vgkg = 0;
    return DPP_OK;
}

// One line minimization along Dd from Y; on success Y and g2 are updated.
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
    if (ok) DPP_TRY(copy_bands(s, s->T2, Y, s->vnocc));
    return DPP_OK;
}

dpp_status cgV_step(dpp_system_s* s, double2* Y, Parts& P) {
    const int nb = s->vnocc, nit = s->nit;
    if (s->vstat) return DPP_OK;
    DPP_TRY(precond_all(s, nb, s->g, s->Kg));
    const double2* pa[3] = {s->g, s->gp, s->g};
    const double2* pb[3] = {s->Kg, s->Kg, s->Dp};
    std::vector<double> dt;
    DPP_TRY(dots_host(s, nb, 3, pa, pb, dt));
    const double gkg = dt[0 * (nit + 1) + nit], gpkg = dt[1 * (nit + 1) + nit], gdp = dt[2 * (nit + 1) + nit];
    double beta = 0.0;
    if (!s->vreset) beta = std::max(0.0, (gkg - gpkg) / s->vgkg);
    double d0 = -gkg + beta * gdp;
    if (beta != 0.0 && d0 >= 0.0) {
        beta = 0.0;
        d0 = -gkg;
    }
    const bool steepest = beta == 0.0;
    std::vector<double> mK(nit, -1.0), bv(nit, beta);
    DPP_TRY(upload(s, s->d_alpha, mK));
    DPP_TRY(upload(s, s->d_beta, bv));
    DPP_TRY(axpby_all(s, nb, s->d_alpha, s->Kg, s->d_beta, s->Dp, s->Dd));
    bool ok = false;
    double step = 0;
    DPP_TRY(linemin_V(s, Y, d0, ok, step, P));
    if (!ok && !steepest) {
        std::vector<double> zero(nit, 0.0);
        DPP_TRY(upload(s, s->d_alpha, mK));
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
    std::swap(s->g, s->g2);  // new gradient (from the accepted objective) becomes g
    std::swap(s->Dp, s->Dd);
    s->vgkg = gkg;
    s->vE0 = P.total();
    s->vat = step;
    s->vreset = 0;
    return DPP_OK;
}

dpp_status check_desc(const dpp_system_desc* d) {
    DPP_REQUIRE(d->nk >= 1 && d->nk <= AUFBAU_MAX_ITEMS && d->nb >= 1 && d->nb <= 128 && d->nat >= 0,
                "dpp_batch_create: bad sizes");
    DPP_REQUIRE((int64_t)d->nk * d->nb <= AUFBAU_MAX, "dpp_batch_create: too many states in one cell");
    DPP_REQUIRE(d->kpts && d->wk && d->R && d->S, "dpp_batch_create: null arrays");
    DPP_REQUIRE(d->nat == 0 || (d->tau && d->Z && d->rc && d->has_proj), "dpp_batch_create: null atom arrays");
    DPP_REQUIRE(d->prec == DPP_F64 || d->prec == DPP_F32, "dpp_batch_create: bad precision");
    return DPP_OK;
}

}  // namespace

// ============================================================== C ABI =====

extern "C" dpp_status dpp_batch_create(dpp_ctx ctx, int ncells, const dpp_system_desc* descs, dpp_system* out) {
    clear_error();
    DPP_REQUIRE(ctx && descs && out && ncells >= 1, "dpp_batch_create: null argument");
    for (int c = 0; c < ncells; ++c) DPP_TRY(check_desc(descs + c));
    for (int c = 1; c < ncells; ++c)
        DPP_REQUIRE(descs[c].prec == descs[0].prec, "dpp_batch_create: cells must share the precision");
    dpp_system_s* s = new dpp_system_s();
    s->ctx = ctx;
    s->ncells = ncells;
    s->prec = s->bulk_prec = (dpp_precision)descs[0].prec;
    auto fail = [&](dpp_status st) {
        std::string msg = dpp_last_error();
        dpp_system_destroy(s);
        return set_error(st, msg);
    };
    dpp_status st = DPP_OK;
    // cells, bases and Hamiltonians; offsets of every packed array
    for (int c = 0; c < ncells; ++c) {
        const dpp_system_desc* d = descs + c;
        CellHost ch{};
        if ((st = dpp_grid_create(ctx, d->R, d->S, &ch.grid)) != DPP_OK) return fail(st);
        ch.nk = d->nk;
        ch.nb = d->nb;
        ch.nat = d->nat;
        ch.ne = d->n_electrons;
        ch.D = d->D;
        ch.tau.assign(d->tau, d->tau + 3 * d->nat);
        ch.Z.assign(d->Z, d->Z + d->nat);
        ch.rc.assign(d->rc, d->rc + d->nat);
        ch.has_proj.assign(d->has_proj, d->has_proj + d->nat);
        ch.item0 = (int)s->bases.size();
        ch.foff = s->Ntot;
        ch.N = ch.grid->N;
        s->Ntot += ch.N;
        s->maxN = std::max(s->maxN, ch.N);
        s->cells.push_back(ch);
        for (int k = 0; k < d->nk; ++k) {
            dpp_basis b = nullptr;
            if ((st = dpp_basis_create(ch.grid, d->kpts + 3 * k, d->ecut, &b)) != DPP_OK) return fail(st);
            s->bases.push_back(b);
            dpp_ham h = nullptr;
            if ((st = dpp_ham_create(b, d->nat, d->tau, d->has_proj, d->rp, d->D, &h)) != DPP_OK) return fail(st);
            s->hams.push_back(h);
            if (b->npw < d->nb) return fail(set_error(DPP_EINVAL, "dpp_batch_create: more bands than plane waves"));
            s->wk.push_back(d->wk[k]);
            s->omega_it.push_back(ch.grid->omega);
            s->inb.push_back(d->nb);
            s->off.push_back(s->total);
            s->npw.push_back(b->npw);
            s->moff.push_back(s->msum);
            s->pioff.push_back(s->pisum);
            s->f_off.push_back(s->nstates);
            s->total += (int64_t)d->nb * b->npw;
            s->msum += (int64_t)d->nb * d->nb;
            s->pisum += (int64_t)h->nproj * d->nb;
            s->nstates += d->nb;
            s->maxnb = std::max(s->maxnb, d->nb);
            s->maxnproj = std::max(s->maxnproj, h->nproj);
        }
        s->cells.back().nproj = s->hams.back()->nproj;
    }
    s->nit = (int)s->bases.size();
    s->off.push_back(s->total);
    const int nit = s->nit;
    // device descriptors
    int64_t eoff = 0;
    for (int c = 0; c < ncells; ++c) {
        const CellHost& ch = s->cells[c];
        CellDesc cd{};
        cd.foff = ch.foff;
        cd.N = ch.N;
        cd.omega = ch.grid->omega;
        cd.dV = ch.grid->omega / (double)ch.N;
        cd.item0 = ch.item0;
        cd.nitems = ch.nk;
        cd.S1 = ch.grid->S[1];
        cd.eoff = eoff;
        cd.D = ch.D;
        cd.ne = ch.ne;
        s->h_cells.push_back(cd);
        FftItem bx = ch.grid->h_item;
        bx.v_off = ch.foff;
        bx.t_off = ch.foff;  // complex plane offset: N per cell
        bx.p_off = eoff;
        s->h_box.push_back(bx);
        FftItem vx = ch.grid->h_item;
        vx.v_off = ch.foff;
        vx.perm = (s->reg_planes && vx.S1 == vx.S2 && plane_reg_supported(vx.S1)) ? 1 : 0;
        s->h_vx.push_back(vx);
        eoff += ch.grid->S[1];
    }
    for (int k = 0; k < nit; ++k) {
        Seg sg{};
        sg.off = s->off[k];
        sg.moff = s->moff[k];
        sg.pioff = s->pioff[k];
        sg.f_off = s->f_off[k];
        sg.kG2 = s->bases[k]->d_kG2;
        sg.wk = s->wk[k];
        sg.omega = s->omega_it[k];
        sg.npw = (int)s->npw[k];
        sg.nb = s->inb[k];
        sg.nproj = s->hams[k]->nproj;
        int c = 0;
        while (c + 1 < ncells && s->cells[c + 1].item0 <= k) ++c;
        sg.cell = c;
        s->h_seg.push_back(sg);
    }
    const size_t blk = (size_t)s->total, sm = (size_t)s->msum;
    struct {
        double2** p;
        size_t n;
    } blocks[] = {{&s->HY, blk}, {&s->Dd, blk}, {&s->HD, blk}, {&s->g, blk}, {&s->g2, blk}, {&s->Kg, blk},
                  {&s->gp, blk}, {&s->Dp, blk}, {&s->psi, blk}, {&s->T1, blk}, {&s->T2, blk},
                  {&s->U, sm}, {&s->Rinv, sm}, {&s->H0, sm}, {&s->X, sm}, {&s->Q, sm}, {&s->H1, sm},
                  {&s->H2, sm}, {&s->Rt, sm}, {&s->M1, sm}, {&s->M2, sm}, {&s->vecs, sm},
                  {&s->eig_scr, (eigh_tiles_ws_bytes((int64_t)sm) + 15) / 16}, {&s->Pi, (size_t)std::max<int64_t>(s->pisum, 1)}};
    for (auto& b : blocks)
        if ((st = dalloc_t(s, b.p, b.n)) != DPP_OK) return fail(st);
    const size_t nis = (size_t)nit, ns = (size_t)s->nstates, Nt = (size_t)s->Ntot;
    struct {
        double** p;
        size_t n;
    } reals[] = {{&s->d_dots, 4 * (nis + 1)},
                 {&s->d_part, std::max<size_t>(4 * nis * DOT_BLOCKS, (size_t)ncells * PULAY_MAX * MDOT_BLOCKS)},
                 {&s->d_E, (size_t)ncells * E_STRIDE}, {&s->d_f, ns}, {&s->d_eig, ns}, {&s->d_res, ns},
                 {&s->d_ones, nis}, {&s->d_alpha, nis}, {&s->d_beta, nis}, {&s->d_bE0, nis},
                 {&s->d_cred, cell_red_elems(ncells)}, {&s->d_epart, (size_t)eoff},
                 {&s->cg.at, nis}, {&s->cg.gkg, nis}, {&s->cg.beta, nis}, {&s->cg.d0, nis}, {&s->cg.d0r, nis},
                 {&s->cg.step, nis}, {&s->cg.step2, nis}, {&s->cg.stepf, nis}, {&s->cg.cK, nis}, {&s->cg.cD, nis},
                 {&s->Vloc, Nt}, {&s->VH, Nt}, {&s->vxc, Nt}, {&s->Veff, Nt}, {&s->Vx, Nt}, {&s->n, Nt}, {&s->nin, Nt},
                 {&s->nout, Nt}, {&s->hist_n, PULAY_MAX * Nt}, {&s->hist_r, PULAY_MAX * Nt},
                 {&s->pulayA, (size_t)ncells * PULAY_MAX * PULAY_MAX}, {&s->pulayC, (size_t)ncells * PULAY_MAX}};
    for (auto& r : reals)
        if ((st = dalloc_t(s, r.p, r.n)) != DPP_OK) return fail(st);
    struct {
        int** p;
        size_t n;
    } ints[] = {{&s->cg.reset, nis}, {&s->cg.stat, nis}, {&s->cg.act, nis}, {&s->cg.steep, nis},
                {&s->cg.ok, nis},    {&s->cg.ok2, nis},  {&s->cg.retry, nis}, {&s->d_pst, 4},
                {&s->d_perm, nis * EIG_TILE_MAXN}};
    for (auto& r : ints)
        if ((st = dalloc_t(s, r.p, r.n)) != DPP_OK) return fail(st);
    if ((st = dalloc_t(s, &s->d_seg, nis)) != DPP_OK) return fail(st);
    if ((st = dalloc_t(s, &s->d_cells, (size_t)ncells)) != DPP_OK) return fail(st);
    if ((st = dalloc_t(s, &s->d_box, (size_t)ncells)) != DPP_OK) return fail(st);
    if ((st = dalloc_t(s, &s->d_vx, (size_t)ncells)) != DPP_OK) return fail(st);
    size_t gwsb = 0;
    for (const CellHost& ch : s->cells) {
        size_t b = 0;
        dpp_grid_workspace_size(ch.grid, &b);
        gwsb = std::max(gwsb, b);
    }
    if ((st = dalloc(s, &s->gws, gwsb)) != DPP_OK) return fail(st);
    // plane buffer (every item's planes for all its bands; also every cell's
    // full box), density partials, overlap partials
    {
        int64_t tel = 0, dens = 0;
        for (int c = 0; c < ncells; ++c) {
            const CellHost& ch = s->cells[c];
            for (int k = ch.item0; k < ch.item0 + ch.nk; ++k) {
                const FftItem& it = s->bases[k]->h_item;
                tel += (int64_t)s->inb[k] * it.nplanes * it.S1 * it.S2;
                dens += (int64_t)dens_chunks(s->inb[k], it.S1, nit) * ch.N;
            }
        }
        tel = std::max<int64_t>(tel, s->Ntot);
        s->tplane_elems = (size_t)tel;
        if ((st = dalloc(s, &s->Tplanes, (size_t)tel * sizeof(double2))) != DPP_OK) return fail(st);
        s->dens_part_elems = (size_t)dens;
        if ((st = dalloc_t(s, &s->dens_part, s->dens_part_elems)) != DPP_OK) return fail(st);
        int64_t ovj = 0, ovp = 0;
        for (int k = 0; k < nit; ++k) {
            const int64_t nch = std::max<int64_t>(1, (s->npw[k] + OV_CHUNK - 1) / OV_CHUNK);
            const int64_t tb = (s->inb[k] + 15) / 16;
            ovj += nch * tb * tb * 256;
            ovp += nch * ((s->hams[k]->nproj + 15) / 16) * tb * 256;
        }
        s->ov_part_elems = (size_t)std::max<int64_t>(4 * ovj, ovp);
        if ((st = dalloc_t(s, &s->ov_part, s->ov_part_elems)) != DPP_OK) return fail(st);
    }
    s->ring_len = std::max<size_t>(256, std::max<size_t>(nis, ns));
    if (hipHostMalloc((void**)&s->h_ring, s->ring_slots * s->ring_len * sizeof(double), hipHostMallocDefault) !=
        hipSuccess) {
        s->h_ring = nullptr;
        return fail(set_error(DPP_ENOMEM, "dpp_batch_create: pinned staging allocation failed"));
    }
    if (hipHostMalloc((void**)&s->h_rep, ((size_t)ncells * E_STRIDE + 2 * (size_t)s->nstates) * sizeof(double),
                      hipHostMallocDefault) != hipSuccess) {
        s->h_rep = nullptr;
        return fail(set_error(DPP_ENOMEM, "dpp_batch_create: pinned report allocation failed"));
    }
    if (hipMemcpy(s->d_seg, s->h_seg.data(), nis * sizeof(Seg), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(s->d_cells, s->h_cells.data(), ncells * sizeof(CellDesc), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(s->d_box, s->h_box.data(), ncells * sizeof(FftItem), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(s->d_vx, s->h_vx.data(), ncells * sizeof(FftItem), hipMemcpyHostToDevice) != hipSuccess)
        return fail(set_error(DPP_EDEVICE, "dpp_batch_create: upload failed"));
    // clear every buffer once (history buffers are read before written otherwise)
    hipStream_t sst = stream(s);
    for (auto& b : blocks)
        if (hipMemsetAsync(*b.p, 0, b.n * sizeof(double2), sst) != hipSuccess)
            return fail(set_error(DPP_EDEVICE, "dpp_batch_create: clear failed"));
    for (auto& r : reals)
        if (hipMemsetAsync(*r.p, 0, r.n * sizeof(double), sst) != hipSuccess)
            return fail(set_error(DPP_EDEVICE, "dpp_batch_create: clear failed"));
    for (auto& r : ints)
        if (hipMemsetAsync(*r.p, 0, r.n * sizeof(int), sst) != hipSuccess)
            return fail(set_error(DPP_EDEVICE, "dpp_batch_create: clear failed"));
    if ((st = fill(s, s->d_ones, nit, 1.0)) != DPP_OK) return fail(st);
    // local pseudopotential per cell
    for (int c = 0; c < ncells; ++c) {
        const dpp_system_desc* d = descs + c;
        st = dpp_local_potential(s->cells[c].grid, d->nat, d->tau, d->Z, d->rc, s->Vloc + s->cells[c].foff, s->gws);
        if (st != DPP_OK) return fail(st);
    }
    if (hipStreamSynchronize(sst) != hipSuccess) return fail(set_error(DPP_EDEVICE, "dpp_batch_create: sync failed"));
    *out = s;
    return DPP_OK;
}

extern "C" dpp_status dpp_system_create(dpp_ctx ctx, const dpp_system_desc* d, dpp_system* out) {
    return dpp_batch_create(ctx, 1, d, out);
}

extern "C" dpp_status dpp_system_destroy(dpp_system s) {
    if (!s) return DPP_OK;
    if (s->ctx) (void)hipStreamSynchronize(s->ctx->stream);
    for (ScfGraph& g : s->graphs)
        if (g.exec) (void)hipGraphExecDestroy(g.exec);
    if (s->cap_stream) (void)hipStreamDestroy(s->cap_stream);
    for (void* p : s->allocs) (void)hipFree(p);
    if (s->h_ring) (void)hipHostFree(s->h_ring);
    if (s->h_rep) (void)hipHostFree(s->h_rep);
    for (dpp_ham h : s->hams) dpp_ham_destroy(h);
    for (dpp_basis b : s->bases) dpp_basis_destroy(b);
    for (CellHost& c : s->cells)
        if (c.grid) dpp_grid_destroy(c.grid);
    delete s;
    return DPP_OK;
}

extern "C" dpp_status dpp_system_dims(dpp_system s, int* ncells, int* nitems, int64_t* total, int64_t* nstates,
                                      int64_t* ngrid) {
    clear_error();
    DPP_REQUIRE(s, "dpp_system_dims: null system");
    if (ncells) *ncells = s->ncells;
    if (nitems) *nitems = s->nit;
    if (total) *total = s->total;
    if (nstates) *nstates = s->nstates;
    if (ngrid) *ngrid = s->Ntot;
    return DPP_OK;
}

extern "C" dpp_status dpp_system_layout(dpp_system s, int64_t* offsets, int64_t* npw) {
    clear_error();
    DPP_REQUIRE(s, "dpp_system_layout: null system");
    for (int k = 0; k <= s->nit; ++k)
        if (offsets) offsets[k] = s->off[k];
    for (int k = 0; k < s->nit; ++k)
        if (npw) npw[k] = s->npw[k];
    return DPP_OK;
}

extern "C" dpp_status dpp_system_cells(dpp_system s, int* item0, int64_t* foff, int64_t* state0) {
    clear_error();
    DPP_REQUIRE(s, "dpp_system_cells: null system");
    for (int c = 0; c <= s->ncells; ++c) {
        const bool last = c == s->ncells;
        if (item0) item0[c] = last ? s->nit : s->cells[c].item0;
        if (foff) foff[c] = last ? s->Ntot : s->cells[c].foff;
        if (state0) state0[c] = last ? s->nstates : s->f_off[s->cells[c].item0];
    }
    return DPP_OK;
}

extern "C" dpp_status dpp_system_field(dpp_system s, int which, double** d_ptr) {
    clear_error();
    DPP_REQUIRE(s && d_ptr, "dpp_system_field: null argument");
    switch (which) {
        case DPP_FIELD_VLOC: *d_ptr = s->Vloc; break;
        case DPP_FIELD_VEFF:
            *d_ptr = s->Veff;
            s->vx_dirty = true;  // the caller may write through it
            break;
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
    DPP_HIP(hipMemcpyAsync(d_out, src, s->Ntot * sizeof(double), hipMemcpyDeviceToDevice, stream(s)));
    return DPP_OK;
}

extern "C" dpp_status dpp_cg_V_init(dpp_system s, dpp_c64* Y, int nocc, double f, dpp_energy* E) {
    clear_error();
    DPP_REQUIRE(s && Y && nocc >= 1 && nocc <= s->maxnb, "dpp_cg_V_init: bad arguments");
    DPP_REQUIRE(s->ncells == 1, "dpp_cg_V_init: total-energy CG runs on one cell");
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

static dpp_status read_bE0(dpp_system s, double* Eb) {
    if (!Eb) return DPP_OK;
    DPP_HIP(hipMemcpyAsync(Eb, s->d_bE0, s->nit * sizeof(double), hipMemcpyDeviceToHost, stream(s)));
    DPP_HIP(hipStreamSynchronize(stream(s)));
    return DPP_OK;
}

extern "C" dpp_status dpp_cg_B_init(dpp_system s, dpp_c64* Y, const double* d_Veff, double* Eb) {
    clear_error();
    DPP_REQUIRE(s && Y && d_Veff, "dpp_cg_B_init: null argument");
    if (d_Veff != s->Veff)
        DPP_HIP(hipMemcpyAsync(s->Veff, d_Veff, s->Ntot * sizeof(double), hipMemcpyDeviceToDevice, stream(s)));
    s->vx_dirty = true;
    DPP_TRY(cgB_init(s, (double2*)Y));
    return read_bE0(s, Eb);
}

extern "C" dpp_status dpp_cg_B_step(dpp_system s, dpp_c64* Y, double* Eb) {
    clear_error();
    DPP_REQUIRE(s && Y && s->cgB_ready, "dpp_cg_B_step: call dpp_cg_B_init first");
    DPP_TRY(cgB_step(s, (double2*)Y));
    return read_bE0(s, Eb);
}

extern "C" dpp_status dpp_band_eigenvalues(dpp_system s, dpp_c64* Y, double* eig) {
    clear_error();
    DPP_REQUIRE(s && Y && eig && s->cgB_ready, "dpp_band_eigenvalues: call dpp_cg_B_init first");
    DPP_TRY(subspace_rotate(s, (double2*)Y));
    DPP_HIP(hipMemcpyAsync(eig, s->d_eig, s->nstates * sizeof(double), hipMemcpyDeviceToHost, stream(s)));
    DPP_HIP(hipStreamSynchronize(stream(s)));
    return DPP_OK;
}

extern "C" dpp_status dpp_scf_init(dpp_system s, const dpp_scf_desc* d) {
    clear_error();
    DPP_REQUIRE(s && d, "dpp_scf_init: null argument");
    for (int c = 0; c < s->ncells; ++c) {
        const dpp_scf_desc& dc = d[c];
        DPP_REQUIRE(dc.nat >= 0 && (dc.nat == 0 || (dc.tau && dc.Z)), "dpp_scf_init: bad atoms");
        const CellHost& ch = s->cells[c];
        if (dc.d_n_start) {
            DPP_HIP(hipMemcpyAsync(s->nin + ch.foff, dc.d_n_start, ch.N * sizeof(double), hipMemcpyDeviceToDevice,
                                   stream(s)));
        } else {
            DPP_TRY(dpp_start_density(ch.grid, dc.nat, dc.tau, dc.Z, dc.sigma, s->nin + ch.foff, s->gws));
        }
    }
    hipLaunchKernelGGL(k_pulay_reset, dim3(1), dim3(64), 0, stream(s), s->d_pst);
    DPP_LAUNCHED();
    s->scf_iter = 0;
    s->n_inner_steps = d[0].n_inner > 0 ? d[0].n_inner : 3;
    s->n_inner_first = d[0].n_inner_first > 0 ? d[0].n_inner_first : s->n_inner_steps;
    s->prec = s->bulk_prec;
    s->last_res = -1.0;
    s->cell_res.assign(s->ncells, -1.0);
    DPP_HIP(hipStreamSynchronize(stream(s)));
    return DPP_OK;
}

extern "C" dpp_status dpp_scf_iteration(dpp_system s, dpp_c64* Yc, dpp_energy* E, double* eig) {
    clear_error();
    DPP_REQUIRE(s && Yc, "dpp_scf_iteration: null argument");
    double2* Y = (double2*)Yc;
    const int steps = s->scf_iter == 0 ? s->n_inner_first : s->n_inner_steps;
    ScfGraph* g = nullptr;
    if (s->graph_on && s->scf_iter > 0) {
        for (ScfGraph& x : s->graphs)
            if (x.Y == Y && x.steps == steps && x.prec == s->prec) g = &x;
        if (!g) {
            // the first iteration with a new (block, steps, precision) runs
            // eagerly: it builds the device tables of that precision's
            // launches, which cannot be created while capturing
            s->graphs.push_back(ScfGraph{nullptr, Y, steps, s->prec});
        } else if (!g->exec) {
            DPP_TRY(capture_scf(s, Y, steps, &g->exec));
        }
    }
    if (g && g->exec) {
        DPP_HIP(hipGraphLaunch(g->exec, stream(s)));
        for (int k = 0; k < s->nit; ++k) s->hc_bandk += (int64_t)s->inb[k] * (1 + steps);
    } else {
        DPP_TRY(scf_body(s, Y, steps));
    }
    // report: energies, residuals, eigenvalues (through pinned memory, so the
    // three copies are queued behind the iteration without host staging)
    const size_t ne = (size_t)s->ncells * E_STRIDE;
    const double* e = s->h_rep;
    const double* res = s->h_rep + ne;
    DPP_HIP(hipMemcpyAsync(s->h_rep, s->d_E, ne * sizeof(double), hipMemcpyDeviceToHost, stream(s)));
    DPP_HIP(hipMemcpyAsync(s->h_rep + ne, s->d_res, s->nstates * sizeof(double), hipMemcpyDeviceToHost, stream(s)));
    if (eig)
        DPP_HIP(hipMemcpyAsync(s->h_rep + ne + s->nstates, s->d_eig, s->nstates * sizeof(double),
                               hipMemcpyDeviceToHost, stream(s)));
    DPP_HIP(hipStreamSynchronize(stream(s)));
    if (eig) std::memcpy(eig, s->h_rep + ne + s->nstates, s->nstates * sizeof(double));
    s->cell_res.assign(s->ncells, 0.0);
    double rmax = 0.0;
    for (int c = 0; c < s->ncells; ++c) {
        const CellHost& ch = s->cells[c];
        const int64_t a = s->f_off[ch.item0];
        const int64_t b = (c + 1 < s->ncells) ? s->f_off[s->cells[c + 1].item0] : s->nstates;
        double r = 0.0;
        for (int64_t i = a; i < b; ++i) r = std::max(r, res[i]);
        s->cell_res[c] = r;
        rmax = std::max(rmax, r);
        if (E) {
            const double* p = e + (size_t)c * E_STRIDE;
            // with smearing E_el is the free energy E - sigma S
            const double ts = s->smear > 0.0 ? p[ETS] : 0.0;
            E[c] = dpp_energy{p[EK] + p[ENL] + p[EH] + p[EXC] + p[ELOC] - ts, p[EK], p[ENL], p[ELOC], p[EH], p[EXC]};
        }
    }
    s->last_res = rmax;
    s->scf_iter++;
    if (s->prec != DPP_F64 && s->refine_res > 0.0 && s->last_res >= 0.0 && s->last_res < s->refine_res)
        s->prec = DPP_F64;  // FP64 refinement for the rest of this SCF run
    return DPP_OK;
}

extern "C" dpp_status dpp_set_graph_mode(dpp_system s, int on) {
    clear_error();
    DPP_REQUIRE(s, "dpp_set_graph_mode: null system");
    s->graph_on = on != 0;
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

extern "C" dpp_status dpp_scf_cell_residuals(dpp_system s, double* res) {
    clear_error();
    DPP_REQUIRE(s && res, "dpp_scf_cell_residuals: null argument");
    for (int c = 0; c < s->ncells; ++c) res[c] = c < (int)s->cell_res.size() ? s->cell_res[c] : -1.0;
    return DPP_OK;
}

extern "C" dpp_status dpp_system_counters(dpp_system s, int64_t* hc_bandk) {
    clear_error();
    DPP_REQUIRE(s && hc_bandk, "dpp_system_counters: null argument");
    *hc_bandk = s->hc_bandk;
    return DPP_OK;
}

// ------------------------------------------------------------ autotuner ---
// Times each candidate launch variant on the system's own items and keeps
// the fastest: per x length S0 (and precision) the register x pass with one
// thread per column, with a lane pair per column, or the LDS pass; the point
// tiles per rotate wave; the overlap block shape.  Each candidate runs
// `reps` times (after one warm-up run) between HIP events on the library
// stream.  The default rule is timed first and kept unless another
// candidate is at least 3% faster (timing noise does not flip choices).
constexpr double TUNE_MARGIN = 0.97;
extern "C" dpp_status dpp_system_tune(dpp_system s, const dpp_c64* Yc, dpp_c64* HYc, int reps) {
    clear_error();
    DPP_REQUIRE(s && Yc && HYc && reps >= 1 && (const void*)Yc != (const void*)HYc, "dpp_system_tune: bad arguments");
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    DPP_HIP(hipStreamIsCapturing(stream(s), &cs));
    DPP_REQUIRE(cs == hipStreamCaptureStatusNone, "dpp_system_tune: stream is capturing");
    const double2* Y = (const double2*)Yc;
    double2* HY = (double2*)HYc;
    const ItemTable* itc = nullptr;
    DPP_TRY(items_for(s, 0, &itc));
    ItemTable* it = const_cast<ItemTable*>(itc);
    hipEvent_t e0, e1;
    DPP_HIP(hipEventCreate(&e0));
    DPP_HIP(hipEventCreate(&e1));
    const int64_t bandk = s->hc_bandk;
    dpp_status err = DPP_OK;
    auto timeit = [&](auto&& fn) -> double {
        if (err != DPP_OK) return 1e300;
        if ((err = fn()) != DPP_OK) return 1e300;
        (void)hipEventRecord(e0, stream(s));
        for (int r = 0; r < reps && err == DPP_OK; ++r) err = fn();
        (void)hipEventRecord(e1, stream(s));
        if (hipEventSynchronize(e1) != hipSuccess) err = set_error(DPP_EDEVICE, "dpp_system_tune: sync failed");
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, e0, e1);
        return err == DPP_OK ? 1e3 * ms / reps : 1e300;
    };
    static const char* xname[] = {"auto", "reg1", "reg2", "lds"};
    std::string rep;
    char buf[256];
    const dpp_precision keep = s->prec;
    for (dpp_precision pr : {DPP_F64, DPP_F32}) {
        s->prec = pr;
        const bool fp64 = pr == DPP_F64;
        std::vector<int>& var = fp64 ? it->xz.var64 : it->xz.var32;
        for (size_t g = 0; g < it->xz.S0.size(); ++g) {
            double best = 1e300;
            int bv = XZ_AUTO;
            snprintf(buf, sizeof buf, "x pass S0=%d %s:", it->xz.S0[g], fp64 ? "f64" : "f32");
            rep += buf;
            // the default rule first; another variant must beat it by 3%
            for (int v : {XZ_AUTO, XZ_REG2, XZ_REG1, XZ_LDS}) {
                if (!xz_variant_available(it->xz.S0[g], fp64, v)) continue;
                var[g] = v;
                const double t = timeit([&] { return apply_H_all(s, 0, Y, HY); });
                snprintf(buf, sizeof buf, " %s %.1f", xname[v], t);
                rep += buf;
                if (v == XZ_AUTO ? t < best : t < TUNE_MARGIN * best) best = t, bv = v;
            }
            var[g] = bv;
            snprintf(buf, sizeof buf, " us per H -> %s; ", xname[bv]);
            rep += buf;
        }
    }
    s->prec = keep;
    if (s->maxnb <= 32) {
        double best = 1e300;
        int bp = 0;
        rep += "rotate point tiles:";
        for (int pt : {0, 1, 2, 4}) {
            s->rot_pt = pt;
            const double t = timeit([&] { return rotate_jobs(s, 0, {RotJob{Y, s->Rinv, 0.0, s->psi}}); });
            snprintf(buf, sizeof buf, " %s %.1f", pt ? std::to_string(pt).c_str() : "auto", t);
            rep += buf;
            if (pt == 0 ? t < best : t < TUNE_MARGIN * best) best = t, bp = pt;
        }
        s->rot_pt = bp;
        snprintf(buf, sizeof buf, " us -> %s; ", bp ? std::to_string(bp).c_str() : "auto");
        rep += buf;
    }
    {
        // the launch shapes of the FP64 overlap (the split-BF16 one has a single shape)
        s->prec = DPP_F64;
        static const char* oname[] = {"auto", "single-tile", "single-pass", "staged"};
        double best = 1e300;
        int bn = 0;
        rep += "overlap blocks (f64):";
        for (int mode : {0, 1, 2, 3}) {
            s->ov_mode = mode;
            const double t = timeit([&] {
                return overlap_jobs(s, 0, {OvJob{Y, Y, 1.0, true, s->U}, OvJob{Y, HY, 1.0, false, s->H0}});
            });
            snprintf(buf, sizeof buf, " %s %.1f", oname[mode], t);
            rep += buf;
            if (mode == 0 ? t < best : t < TUNE_MARGIN * best) best = t, bn = mode;
        }
        s->ov_mode = bn;
        snprintf(buf, sizeof buf, " us -> %s", oname[bn]);
        rep += buf;
        s->prec = keep;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    s->hc_bandk = bandk;
    s->cgB_ready = false;  // the tuning runs overwrote the band-CG work blocks
    // captured graphs hold the old launch shapes
    for (ScfGraph& g : s->graphs)
        if (g.exec) (void)hipGraphExecDestroy(g.exec);
    s->graphs.clear();
    s->tune_report = rep;
    return err;
}

extern "C" dpp_status dpp_system_set_launch_choice(dpp_system s, int which, int value) {
    clear_error();
    DPP_REQUIRE(s, "dpp_system_set_launch_choice: null system");
    switch (which) {
        case DPP_CHOICE_OVERLAP:
            DPP_REQUIRE(value >= 0 && value <= 3, "dpp_system_set_launch_choice: overlap mode 0..3");
            s->ov_mode = value;
            break;
        case DPP_CHOICE_ROTATE_PT:
            DPP_REQUIRE(value == 0 || value == 1 || value == 2 || value == 4,
                        "dpp_system_set_launch_choice: rotate point tiles 0, 1, 2 or 4");
            s->rot_pt = value;
            break;
        case DPP_CHOICE_XPASS: {
            DPP_REQUIRE(value >= XZ_AUTO && value <= XZ_LDS, "dpp_system_set_launch_choice: x-pass variant 0..3");
            const ItemTable* itc = nullptr;
            DPP_TRY(items_for(s, 0, &itc));
            ItemTable* it = const_cast<ItemTable*>(itc);
            for (size_t g = 0; g < it->xz.S0.size(); ++g) {
                // variants a length does not have fall back to the LDS pass
                it->xz.var64[g] = xz_variant_available(it->xz.S0[g], true, value) ? value : XZ_LDS;
                it->xz.var32[g] = xz_variant_available(it->xz.S0[g], false, value) ? value : XZ_LDS;
            }
            break;
        }
        default:
            return set_error(DPP_EINVAL, "dpp_system_set_launch_choice: unknown choice");
    }
    for (ScfGraph& g : s->graphs)
        if (g.exec) (void)hipGraphExecDestroy(g.exec);
    s->graphs.clear();
    return DPP_OK;
}

extern "C" dpp_status dpp_system_set_smearing(dpp_system s, double sigma) {
    clear_error();
    DPP_REQUIRE(s && sigma >= 0.0 && std::isfinite(sigma), "dpp_system_set_smearing: bad arguments");
    s->smear = sigma;
    // captured SCF graphs hold the previous fillings kernel
    for (ScfGraph& g : s->graphs)
        if (g.exec) (void)hipGraphExecDestroy(g.exec);
    s->graphs.clear();
    return DPP_OK;
}

extern "C" dpp_status dpp_system_smearing_state(dpp_system s, int ncells, double* mu, double* TS) {
    clear_error();
    DPP_REQUIRE(s && ncells == s->ncells && (mu || TS), "dpp_system_smearing_state: bad arguments");
    DPP_REQUIRE(s->smear > 0.0, "dpp_system_smearing_state: the system has no smearing");
    std::vector<double> h((size_t)s->ncells * E_STRIDE);
    DPP_HIP(hipMemcpyAsync(h.data(), s->d_E, h.size() * sizeof(double), hipMemcpyDeviceToHost, stream(s)));
    DPP_HIP(hipStreamSynchronize(stream(s)));
    for (int c = 0; c < s->ncells; ++c) {
        if (mu) mu[c] = h[(size_t)c * E_STRIDE + EMU];
        if (TS) TS[c] = h[(size_t)c * E_STRIDE + ETS];
    }
    return DPP_OK;
}

extern "C" dpp_status dpp_system_set_xc(dpp_system s, int functional) {
    clear_error();
    DPP_REQUIRE(s, "dpp_system_set_xc: null system");
    DPP_REQUIRE(functional == DPP_XC_LDA_PZ81 || functional == DPP_XC_PBE, "dpp_system_set_xc: unknown functional");
    if (functional == DPP_XC_PBE && !s->gga_ws) {
        size_t bytes = 0;
        for (const CellHost& ch : s->cells) {
            size_t b = 0;
            DPP_TRY(dpp_gga_workspace_size(ch.grid, &b));
            bytes = std::max(bytes, b);
        }
        void* p = nullptr;
        if (hipMalloc(&p, bytes + 256) != hipSuccess) return set_error(DPP_ENOMEM, "dpp_system_set_xc: allocation failed");
        s->allocs.push_back(p);
        s->gga_ws = p;
        s->d_gga_scratch = reinterpret_cast<double*>(reinterpret_cast<char*>(p) + ((bytes + 255) / 256) * 256);
    }
    s->xc = functional;
    s->vx_dirty = true;
    // captured SCF graphs hold the previous functional's launches
    for (ScfGraph& g : s->graphs)
        if (g.exec) (void)hipGraphExecDestroy(g.exec);
    s->graphs.clear();
    return DPP_OK;
}

extern "C" dpp_status dpp_system_tune_report(dpp_system s, char* buf, size_t len) {
    clear_error();
    DPP_REQUIRE(s && buf && len > 0, "dpp_system_tune_report: bad arguments");
    snprintf(buf, len, "%s", s->tune_report.c_str());
    return DPP_OK;
}

extern "C" dpp_status dpp_system_apply_H(dpp_system s, const dpp_c64* Y, dpp_c64* HY) {
    clear_error();
    DPP_REQUIRE(s && Y && HY && (const void*)Y != (const void*)HY, "dpp_system_apply_H: bad arguments");
    DPP_TRY(apply_H_all(s, 0, (const double2*)Y, (double2*)HY));
    return DPP_OK;
}

namespace {

// Position tables of dpp_system_forces: Cartesian and fractional positions,
// derivative projectors.
dpp_status forces_positions(dpp_system_s* s) {
    ForceBufs& fb = s->fb;
    std::vector<double> tau, sfrac;
    for (int c = 0; c < s->ncells; ++c) {
        const CellHost& ch = s->cells[c];
        // s = R^{-1} tau with R's columns the lattice vectors: s_i = b_i . tau / (2 pi)
        const double* B = ch.grid->B;
        for (int a = 0; a < ch.nat; ++a) {
            const double* t = &ch.tau[3 * a];
            for (int i = 0; i < 3; ++i) {
                tau.push_back(t[i]);
                sfrac.push_back((B[i] * t[0] + B[3 + i] * t[1] + B[6 + i] * t[2]) / (2.0 * M_PI));
            }
        }
    }
    if (fb.natall > 0) {
        DPP_HIP(hipMemcpy(fb.tau, tau.data(), tau.size() * sizeof(double), hipMemcpyHostToDevice));
        DPP_HIP(hipMemcpy(fb.sfrac, sfrac.data(), sfrac.size() * sizeof(double), hipMemcpyHostToDevice));
    }
    for (int k = 0; k < s->nit; ++k)
        DPP_TRY(projector_derivatives(s->ctx, s->bases[k], s->hams[k]->nproj, s->hams[k]->d_P, fb.Q + fb.qoff[k]));
    return DPP_OK;
}

// Device tables of dpp_system_forces (first call).
dpp_status forces_setup(dpp_system_s* s) {
    ForceBufs& fb = s->fb;
    if (fb.ready) return DPP_OK;
    std::vector<double> Z, rc;
    size_t maxpart = 0;
    for (int c = 0; c < s->ncells; ++c) {
        const CellHost& ch = s->cells[c];
        fb.aoff.push_back(fb.natall);
        fb.proj0.push_back((int)fb.proj_atom.size());
        fb.natall += ch.nat;
        for (int a = 0; a < ch.nat; ++a) {
            Z.push_back(ch.Z[a]);
            rc.push_back(ch.rc[a]);
            if (ch.has_proj[a]) fb.proj_atom.push_back(a);
        }
        const int64_t N = ch.N;
        const int64_t chunk = std::max<int64_t>(4096, (N + LF_CHUNKS_MAX - 1) / LF_CHUNKS_MAX);
        maxpart = std::max(maxpart, (size_t)ch.nat * 3 * (size_t)((N + chunk - 1) / chunk));
        maxpart = std::max(maxpart, (size_t)ch.nat * 11);  // Ewald partials (8 per atom) and scratch forces
    }
    const int64_t na = std::max<int64_t>(fb.natall, 1);
    DPP_TRY(dalloc_t(s, &fb.tau, 3 * na));
    DPP_TRY(dalloc_t(s, &fb.sfrac, 3 * na));
    DPP_TRY(dalloc_t(s, &fb.Z, na));
    DPP_TRY(dalloc_t(s, &fb.rc, na));
    DPP_TRY(dalloc_t(s, &fb.part, std::max<size_t>(maxpart, 1)));
    DPP_TRY(dalloc_t(s, &fb.E, std::max(s->ncells, 1)));
    if (fb.natall > 0) {
        DPP_HIP(hipMemcpy(fb.Z, Z.data(), Z.size() * sizeof(double), hipMemcpyHostToDevice));
        DPP_HIP(hipMemcpy(fb.rc, rc.data(), rc.size() * sizeof(double), hipMemcpyHostToDevice));
    }
    int64_t q = 0, nl = 0;
    for (int k = 0; k < s->nit; ++k) {
        fb.qoff.push_back(q);
        fb.nloff.push_back(nl);
        q += 3 * (int64_t)s->hams[k]->nproj * s->npw[k];
        nl += 3 * (int64_t)s->hams[k]->nproj;
    }
    DPP_TRY(dalloc_t(s, &fb.Q, std::max<int64_t>(q, 1)));
    DPP_TRY(dalloc_t(s, &fb.Pid, std::max<int64_t>(3 * s->pisum, 1)));
    DPP_TRY(dalloc_t(s, &fb.nlpart, std::max<int64_t>(nl, 1)));
    DPP_TRY(forces_positions(s));
    fb.ready = true;
    return DPP_OK;
}

// Projector forces of one cell: the sum over the cell's items (k-points) of
// the per-projector terms, onto the atoms that carry the projectors (fixed
// order: items in k order).
__global__ void k_nl_gather(int nat, int item0, int nitems, const int* __restrict__ nproj_of,
                            const int64_t* __restrict__ nloff, const int* __restrict__ proj_atom,
                            const double* __restrict__ nlpart, double* __restrict__ F) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= nat * 3) return;
    const int a = e / 3, d = e - 3 * a;
    double s = 0.0;
    for (int k = 0; k < nitems; ++k) {
        const int np = nproj_of[item0 + k];
        for (int p = 0; p < np; ++p)
            if (proj_atom[p] == a) s += nlpart[nloff[item0 + k] + 3 * p + d];
    }
    F[e] = s;
}

}  // namespace

extern "C" dpp_status dpp_system_set_positions(dpp_system s, const double* tau) {
    clear_error();
    DPP_REQUIRE(s && tau, "dpp_system_set_positions: null argument");
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    DPP_HIP(hipStreamIsCapturing(stream(s), &cs));
    DPP_REQUIRE(cs == hipStreamCaptureStatusNone, "dpp_system_set_positions: stream is capturing");
    int64_t a0 = 0;
    for (int c = 0; c < s->ncells; ++c) {
        const int nat = s->cells[c].nat;
        for (int64_t q = 0; q < 3 * (int64_t)nat; ++q)
            DPP_REQUIRE(std::isfinite(tau[3 * a0 + q]), "dpp_system_set_positions: non-finite position");
        a0 += nat;
    }
    a0 = 0;
    for (int c = 0; c < s->ncells; ++c) {
        CellHost& ch = s->cells[c];
        ch.tau.assign(tau + 3 * a0, tau + 3 * (a0 + ch.nat));
        a0 += ch.nat;
        DPP_TRY(dpp_local_potential(ch.grid, ch.nat, ch.tau.data(), ch.Z.data(), ch.rc.data(), s->Vloc + ch.foff,
                                    s->gws));
        for (int k = ch.item0; k < ch.item0 + ch.nk; ++k)
            DPP_TRY(ham_set_positions(s->hams[k], ch.nat, ch.tau.data(), ch.has_proj.data()));
    }
    if (s->fb.ready) DPP_TRY(forces_positions(s));
    s->vx_dirty = true;
    DPP_HIP(hipStreamSynchronize(stream(s)));
    return DPP_OK;
}

extern "C" dpp_status dpp_system_forces(dpp_system s, const dpp_c64* Yc, double* F_loc, double* F_nl, double* F_ion,
                                        double* E_ion) {
    clear_error();
    DPP_REQUIRE(s && Yc, "dpp_system_forces: null argument");
    DPP_REQUIRE(s->scf_iter > 0, "dpp_system_forces: no SCF iteration yet (fillings and density)");
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    DPP_HIP(hipStreamIsCapturing(stream(s), &cs));
    DPP_REQUIRE(cs == hipStreamCaptureStatusNone, "dpp_system_forces: stream is capturing");
    DPP_TRY(forces_setup(s));
    ForceBufs& fb = s->fb;
    const double2* Y = (const double2*)Yc;
    // local and ionic terms, cell by cell
    for (int c = 0; c < s->ncells; ++c) {
        const CellHost& ch = s->cells[c];
        const int64_t a0 = fb.aoff[c];
        if (F_loc) {
            double2* nt = reinterpret_cast<double2*>(reinterpret_cast<char*>(s->gws) + grid_coef_offset(ch.grid));
            DPP_TRY(full_forward_real(ch.grid, s->nout + ch.foff, nt, s->gws));
            DPP_TRY(forces_local(s->ctx, ch.grid, nt, ch.nat, fb.sfrac + 3 * a0, fb.Z + a0, fb.rc + a0, fb.part,
                                 F_loc + 3 * a0));
        }
        if (F_ion || E_ion) {
            EwaldSetup e{};
            for (int i = 0; i < 9; ++i) e.R[i] = ch.grid->R[i], e.B[i] = ch.grid->B[i];
            e.omega = ch.grid->omega;
            // splitting parameter balancing the two sums; both are cut where
            // their terms fall below exp(-36)
            e.eta = std::sqrt(M_PI) * std::pow((double)std::max(ch.nat, 1) / (e.omega * e.omega), 1.0 / 6.0);
            e.rcut = 6.0 / e.eta;
            e.gcut = 12.0 * e.eta;
            for (int i = 0; i < 3; ++i) {
                const double bi = std::sqrt(e.B[i] * e.B[i] + e.B[3 + i] * e.B[3 + i] + e.B[6 + i] * e.B[6 + i]);
                const double ai = std::sqrt(e.R[i] * e.R[i] + e.R[3 + i] * e.R[3 + i] + e.R[6 + i] * e.R[6 + i]);
                e.nr[i] = (int)std::ceil(e.rcut * bi / (2.0 * M_PI)) + 1;  // planes along a_i are 2 pi / |b_i| apart
                e.ng[i] = (int)std::ceil(e.gcut * ai / (2.0 * M_PI)) + 1;  // |m_i| = |G . a_i| / (2 pi)
            }
            double* Fi = F_ion ? F_ion + 3 * a0 : fb.part + 8 * ch.nat;  // energy only: forces to scratch
            DPP_TRY(ewald_sums(s->ctx, e, ch.nat, fb.tau + 3 * a0, fb.sfrac + 3 * a0, fb.Z + a0, fb.part, Fi,
                               fb.E + c));
        }
    }
    // nonlocal terms: Pi = P^dag psi and Pid_d = Q_d^dag psi in one FP64 launch
    if (F_nl) {
        std::vector<OvTask> t;
        int64_t poff = 0;
        for (int k = 0; k < s->nit; ++k) {
            const dpp_ham h = s->hams[k];
            if (h->nproj == 0) continue;
            const int nb = s->inb[k];
            for (int d = -1; d < 3; ++d) {
                const double2* A = d < 0 ? h->d_P : fb.Q + fb.qoff[k] + (int64_t)d * h->nproj * s->npw[k];
                double2* out = d < 0 ? s->Pi + s->pioff[k] : fb.Pid + 3 * s->pioff[k] + (int64_t)d * h->nproj * nb;
                OvTask x = make_ov_task((int)s->npw[k], h->nproj, A, s->npw[k], nb, Y + s->off[k], s->npw[k], 1.0,
                                        out, nb);
                x.part_off = poff;
                x.item = k;
                poff += (int64_t)x.nchunk * x.ntiles * 256;
                t.push_back(x);
            }
        }
        if ((size_t)poff > s->ov_part_elems) return set_error(DPP_EUNSUPPORTED, "overlap partial buffer too small");
        if (!t.empty()) {
            const OvTask* dt = nullptr;
            DPP_TRY(table_t(s, t, &dt));
            std::vector<int4> w;
            overlap_worklist(t, 0, w);
            const int4* dw = nullptr;
            DPP_TRY(table_t(s, w, &dw));
            DPP_TRY(overlap_tasks(s->ctx, t, dt, s->ov_part, nullptr, 0, dw, (int)w.size(), DPP_F64));
        }
        for (int k = 0; k < s->nit; ++k) {
            const dpp_ham h = s->hams[k];
            DPP_TRY(forces_nonlocal_item(s->ctx, h->nproj, s->inb[k], s->wk[k], h->D, s->d_f + s->f_off[k],
                                         s->Pi + s->pioff[k], fb.Pid + 3 * s->pioff[k], fb.nlpart + fb.nloff[k]));
        }
        std::vector<int> np(s->nit);
        for (int k = 0; k < s->nit; ++k) np[k] = s->hams[k]->nproj;
        const int* d_np = nullptr;
        const int64_t* d_nloff = nullptr;
        const int* d_pa = nullptr;
        DPP_TRY(table_t(s, np, &d_np));
        DPP_TRY(table_t(s, fb.nloff, &d_nloff));
        std::vector<int> pa = fb.proj_atom;
        if (pa.empty()) pa.push_back(-1);
        DPP_TRY(table_t(s, pa, &d_pa));
        for (int c = 0; c < s->ncells; ++c) {
            const CellHost& ch = s->cells[c];
            if (ch.nat == 0) continue;
            hipLaunchKernelGGL(k_nl_gather, dim3((ch.nat * 3 + 255) / 256), dim3(256), 0, stream(s), ch.nat,
                               ch.item0, ch.nk, d_np, d_nloff, d_pa + fb.proj0[c], (const double*)fb.nlpart,
                               F_nl + 3 * fb.aoff[c]);
            DPP_LAUNCHED();
        }
    }
    if (E_ion) {
        std::vector<double> e(s->ncells);
        DPP_HIP(hipMemcpyAsync(e.data(), fb.E, s->ncells * sizeof(double), hipMemcpyDeviceToHost, stream(s)));
        DPP_HIP(hipStreamSynchronize(stream(s)));
        for (int c = 0; c < s->ncells; ++c) {
            const CellHost& ch = s->cells[c];
            const double omega = ch.grid->omega;
            const double eta = std::sqrt(M_PI) * std::pow((double)std::max(ch.nat, 1) / (omega * omega), 1.0 / 6.0);
            double z2 = 0.0, zs = 0.0;
            for (double z : ch.Z) z2 += z * z, zs += z;
            // self and compensating-background terms
            E_ion[c] = e[c] - eta / std::sqrt(M_PI) * z2 - M_PI * zs * zs / (2.0 * omega * eta * eta);
        }
    }
    return DPP_OK;
}

extern "C" dpp_status dpp_system_fillings(dpp_system s, double* f) {
    clear_error();
    DPP_REQUIRE(s && f, "dpp_system_fillings: null argument");
    DPP_REQUIRE(s->scf_iter > 0, "dpp_system_fillings: no SCF iteration yet");
    DPP_HIP(hipMemcpyAsync(f, s->d_f, s->nstates * sizeof(double), hipMemcpyDeviceToHost, stream(s)));
    DPP_HIP(hipStreamSynchronize(stream(s)));
    return DPP_OK;
}
