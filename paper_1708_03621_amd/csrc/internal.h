// Internal declarations of libdftpp (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/dftpp.h"

namespace dpp {

// ------------------------------------------------------------ errors -------
dpp_status set_error(dpp_status st, const std::string& msg);
void clear_error();

#define DPP_REQUIRE(cond, msg)                                    \
    do {                                                          \
        if (!(cond)) return ::dpp::set_error(DPP_EINVAL, (msg));  \
    } while (0)

#define DPP_HIP(call)                                                              \
    do {                                                                           \
        hipError_t e_ = (call);                                                    \
        if (e_ != hipSuccess)                                                      \
            return ::dpp::set_error(DPP_EDEVICE, std::string(#call ": ") +         \
                                                     hipGetErrorString(e_));       \
    } while (0)

#define DPP_TRY(call)                        \
    do {                                     \
        dpp_status s_ = (call);              \
        if (s_ != DPP_OK) return s_;         \
    } while (0)

// Check the launch that was just enqueued.
#define DPP_LAUNCHED() DPP_HIP(hipGetLastError())

// ------------------------------------------------------------ FFT plan -----
constexpr int MAX_RADICES = 8;

struct FftAxis {
    int n;
    int nrad;
    int rad[MAX_RADICES];  // radices in {2,3,4,5}, product n
};

// Per-(basis or full box) descriptor consumed by the FFT pass kernels.  Lives
// in device memory (one array entry per work item).
struct FftItem {
    int S0, S1, S2;
    int nplanes;       // x-planes carrying data (sphere: 2*n0max+1; full box: S0)
    int n0min;         // plane p holds Miller index n0 = n0min + p (i0 = n0 mod S0)
    int npw;
    int nb;            // bands of this item
    int full;          // 1: full-box planes (no sphere tables)
    FftAxis ax[3];
    const double2* tw64[3];
    const float2* tw32[3];
    const int4* planes;   // per plane: {sphere start, count, n1 of first row, nrows}
    const int4* rows;     // per (plane, natural i1): {first point, count, n2 of first point, 0}
    int perm;             // 1: planes stored in digit-reversed (i1, i2) order (register plane passes)
    int vperm;            // x pass of H: 1 = V is natural (digit-reverse the column, times vscale);
                          // 0 = V is already in the plane order and scaled
    const int* poff;      // per sphere point: i1*S2 + i2
    const double* kG2;    // per sphere point |k+G|^2
    int64_t c_off;        // offset (complex elements) of this item's block
    int64_t ld;           // leading dimension of the block
    int64_t t_off;        // offset (complex elements) of this item's plane buffer
    int64_t v_off;        // offset (doubles) of this item's cell field (V_eff, n)
    double omega;
    double vscale;        // Omega / N
    double wk;            // k-point weight (density accumulation)
    int64_t f_off;        // offset of this item's fillings
    int64_t p_off;        // offset (doubles) of this item's partial sums (density boxes, Hartree rows)
    int dnch, dchunk;     // density: band chunks of this item and bands per chunk
    double B[9];          // reciprocal basis, row-major (full-box items: Hartree kernel)
};

// One cell of a batch: where its fields sit in the concatenated field arrays
// and which work items (k-points) and partial sums belong to it.
struct CellDesc {
    int64_t foff;         // offset (doubles) of the cell's fields
    int64_t N;            // grid points
    double omega, dV;     // volume and Omega / N
    int item0, nitems;    // items (k-points) of the cell
    int64_t pstart;       // first density partial (doubles) of the cell
    int nparts;           // density partial boxes of the cell
    int S1;               // rows of Hartree energy partials
    int64_t eoff;         // offset of the Hartree energy partials
    double D;             // projector coupling
    double ne;            // electrons
};

// ------------------------------------------------------------ handles ------
}  // namespace dpp

// Per-context kernel timer: when enabled, launches of the instrumented kernel
// classes are bracketed by HIP events on the context stream; durations are
// summed when the pool fills or when the totals are read (both synchronize).
struct KernelTimer {
    bool on = false;
    int cap = 0, used = 0;
    std::vector<hipEvent_t> ev;   // 2 * cap
    std::vector<int> kind;        // cap
    double total_ms[32] = {};
    int64_t count[32] = {};
    double bytes[32] = {};        // algorithmic bytes of the timed launches
    double flops[32] = {};        // algorithmic flops of the timed launches
};

struct dpp_ctx_s {
    int device;
    hipStream_t stream;
    int* d_status;
    KernelTimer timer;
};

namespace dpp {
// Scope that times the launches enqueued during its lifetime as one `kind`.
// `bytes` / `flops` are the algorithmic HBM bytes and flops of the scope's
// launches (what the operation must move and compute, not what it does move).
struct TimerScope {
    dpp_ctx_s* c;
    int slot;
    TimerScope(dpp_ctx_s* ctx, int kind, double bytes = 0.0, double flops = 0.0);
    ~TimerScope();
};
}  // namespace dpp

struct dpp_grid_s {
    dpp_ctx ctx;
    double R[9];   // row-major, columns are lattice vectors
    double B[9];   // reciprocal basis, columns b_i, row-major
    double omega;
    int S[3];
    int64_t N;
    dpp::FftAxis ax[3];
    double2* d_tw64[3];
    float2* d_tw32[3];
    int4* d_fullplanes;      // plane table for full-box transforms
    dpp::FftItem* d_item;    // full-box FFT item (nb = 1)
    dpp::FftItem h_item;
    double* h_pin = nullptr;  // pinned host scalars for the readbacks of iterative solves (first use)
};

struct dpp_basis_s {
    dpp_grid grid;
    double k[3];
    double ecut;
    int64_t npw;
    int next[6];
    int nplanes, n0min;
    int32_t* d_index;
    int32_t* d_poff;
    int4* d_miller;      // n0, n1, n2, unused
    double* d_kG2;
    int4* d_planes;
    int4* d_rows;        // nplanes x S1 (natural i1): {first point, count, n2 of the first point, 0}
    std::vector<int4> h_planes;
    dpp::FftItem h_item;     // static part (c_off = t_off = v_off = 0, nb = 0)
};

struct dpp_ham_s {
    dpp_basis basis;
    int nproj;
    double D, rp;
    double2* d_P;          // nproj x npw, band-major (projector a at d_P + a*npw)
    const double* d_Veff;
};

namespace dpp {

// FFT geometry helpers (fft.hip)
bool factor_axis(int n, FftAxis* ax);
int fft_threads(int elems);            // 0 if the plane is too large
size_t fft_lds_bytes(int elems, bool fp64);
dpp_status check_fft_shape(int S0, int S1, int S2, bool fp64);
size_t plane_buffer_elems(const dpp_basis_s* b, int nb);   // complex elements of T for nb bands

// Full-box inverse transform of reciprocal coefficients (unnormalized,
// e^{+iG.r}) keeping the real part; coef may live in the grid workspace at
// grid_coef_offset (fft.hip).
dpp_status full_inverse_real(dpp_grid_s* g, const double2* coef, double* out, void* ws);
// Projectors of ham recomputed in place for new atom positions (tau: 3 per
// atom, host; the atoms carrying projectors must be those of dpp_ham_create).
dpp_status ham_set_positions(dpp_ham_s* h, int nat, const double* tau, const int* has_proj);
// y = J n (natural order) of a real field on the grid's box; ws: N complex.
dpp_status full_forward_real(dpp_grid_s* g, const double* n, double2* y, void* ws);
// PBE v_xc and E_xc of a real density on the grid's box (gga.hip); ws:
// dpp_gga_workspace_size bytes.
dpp_status gga_pbe(dpp_grid_s* g, const double* n, double* vxc, double* Exc, void* ws);
// Full-box complex transforms of nf fields (stride N): y = scale * sum_r x e^{sign i G.r}
// (natural order; x may equal y), one launch per pass for all fields; ws: nf N complex.
dpp_status full_complex(dpp_grid_s* g, int nf, const double2* x, double2* y, int sign, double scale, void* ws);

// Forces on the ions (forces.hip).  Positions enter as fractional
// coordinates s = R^{-1} tau (3 per atom).
// Local: F_a = -Omega sum_G G v_a(G) Im[conj(nt(G)) exp(-i G.tau_a)] over the
// full box of one cell (nt = J n), per atom into F (nat x 3, device); part
// holds nat * LF_CHUNKS_MAX * 3 doubles.
dpp_status forces_local(dpp_ctx_s* ctx, const dpp_grid_s* g, const double2* nt, int nat, const double* d_sfrac,
                        const double* d_Z, const double* d_rc, double* part, double* F);
// Derivative projectors Q_d[a][g] = -i G_d P[a][g] (d = x, y, z; each nproj x npw, band-major).
dpp_status projector_derivatives(dpp_ctx_s* ctx, const dpp_basis_s* b, int nproj, const double2* P, double2* Q);
// Nonlocal force terms of one item: out[p * 3 + d] = -w D sum_i f_i 2 Re[conj(Pi_pi) Pid_d,pi],
// Pi (nproj x nb) and Pid (3 blocks of nproj x nb), row length nb.
dpp_status forces_nonlocal_item(dpp_ctx_s* ctx, int nproj, int nb, double w, double D, const double* f,
                                const double2* Pi, const double2* Pid, double* out);
// Ewald energy and forces of point charges in a compensating background;
// E (device, 1) gets the two lattice sums; the position-independent self and
// background terms are the caller's.
struct EwaldSetup {
    double R[9], B[9];  // row-major, columns a_i / b_i
    double eta, rcut, gcut, omega;
    int nr[3], ng[3];
};
// part: 8 nat doubles; F: nat x 3 (device).
dpp_status ewald_sums(dpp_ctx_s* ctx, const EwaldSetup& e, int nat, const double* d_tau, const double* d_sfrac,
                      const double* d_Z, double* part, double* F, double* E);
constexpr int LF_CHUNKS_MAX = 1024;
size_t grid_coef_offset(const dpp_grid_s* g);

// Batched passes over a table of items (one per k-point or cell/k pair);
// h_items mirrors the device table d_items.  Tb holds every item's planes.
// Items of a table grouped by x length S0 (the register x pass is compiled
// per S0): group g holds count[g] items listed in the device array idx[g]
// (nullptr when the group is the whole table in order).
// var64[g] / var32[g]: the x-pass variant of the group in FP64 / FP32
// (XZ_AUTO, XZ_REG1, XZ_REG2, XZ_LDS), set by the launch tuner.
enum XzVariant { XZ_AUTO = 0, XZ_REG1 = 1, XZ_REG2 = 2, XZ_LDS = 3 };
struct XzPlan {
    std::vector<int> S0, count, maxS1S2, nbm;
    std::vector<const int*> idx;
    std::vector<int> var64, var32;
};
// Whether variant v of the x pass exists for length S0 in this precision.
bool xz_variant_available(int S0, bool fp64, int v);
XzPlan xz_plan_groups(const std::vector<FftItem>& h, std::vector<std::vector<int>>& members);

// Items grouped for the plane passes: group g with N[g] > 0 holds items with
// square y-z faces S1 = S2 = N[g] whose planes are stored digit-reversed
// (perm = 1, register plane passes); N[g] = 0 is the LDS group.
// Plane-pass groups: N is the register kernel's face length (digit-reversed
// items), kPlane90Group for 90 x 90 faces in natural order, 0 for the rest
// (generic LDS kernel).
constexpr int kPlane90Group = -90;
struct PlanePlan {
    std::vector<int> N, count, maxP, nbm;
    std::vector<const int*> idx;
};
bool plane_reg_supported(int n);
PlanePlan plane_plan_groups(const std::vector<FftItem>& h, std::vector<std::vector<int>>& members);

// Items may have different boxes: the launch takes the largest workgroup and
// LDS size any item needs.  `act` (nullable) masks items: inactive items do
// nothing.  With `plan`, the x pass runs one register-resident launch per S0
// group where that length is compiled in.
template <typename T>
dpp_status apply_H_local_batched(dpp_ctx_s* ctx, const FftItem* d_items, const std::vector<FftItem>& h_items,
                                 const double2* X, double2* HX, const double* V, void* Tb,
                                 const int* act = nullptr, const XzPlan* plan = nullptr,
                                 const PlanePlan* pplan = nullptr);
// Band-chunk partial densities of every item (item p_off, dnch, dchunk), then
// per cell n[foff + j] = sum of the cell's partials (fixed order).
template <typename T>
dpp_status density_batched(dpp_ctx_s* ctx, const FftItem* d_items, const std::vector<FftItem>& h_items,
                           const double2* psi, const double* fill, void* Tb, double* part,
                           const CellDesc* d_cells, int ncells, int64_t maxN, double* n,
                           const PlanePlan* pplan = nullptr, const XzPlan* xplan = nullptr);
size_t batched_plane_elems(const std::vector<FftItem>& h_items);
// Vx = (Omega/N) V in the plane order of each cell's x pass (one item per
// cell: v_off = field offset, perm, axes); the x pass of H then reads it
// with unit stride (items with vperm = 0).
dpp_status vx_cells(dpp_ctx_s* ctx, const FftItem* d_cell_items, int ncells, int64_t maxN, const double* V,
                    double* Vx);
// Hartree potential and energy of every cell: full-box items (one per cell,
// v_off = field offset, t_off = plane offset, p_off = row-partial offset).
// VH may be NULL (only the energies E_H are formed) or E may be NULL (only
// V_H).
dpp_status hartree_batched(dpp_ctx_s* ctx, const FftItem* d_items, const std::vector<FftItem>& h_items,
                           const double* n, double* VH, void* Tb, double* epart, const CellDesc* d_cells,
                           double* E, int E_stride);

// Cell-batched field reductions (fields.hip): v_xc and E_xc per cell; the
// grid dot (Omega / N) sum a b per cell.  `part` holds cell_red_elems doubles.
dpp_status lda_cells(dpp_ctx_s* ctx, const CellDesc* d_cells, int ncells, const double* n, double* vxc,
                     double* part, double* E, int stride);
dpp_status dot_cells(dpp_ctx_s* ctx, const CellDesc* d_cells, int ncells, const double* a, const double* b,
                     double* part, double* E, int stride);
size_t cell_red_elems(int ncells);

// Launch the local-potential H pipeline etc. (fft.hip)
template <typename T>
dpp_status run_apply_H_local(dpp_ham_s* ham, int nb, const double2* C, int64_t ldC, double2* HC,
                             int64_t ldHC, void* ws);

// blas.hip
constexpr int OV_WAVES = 4;
constexpr int OV_CHUNK = 256;  // sphere points per overlap workgroup
constexpr int RT_WAVES = 4;
constexpr int RT_JT = 8;       // 16-band output tiles held by one rotate wave

// out = scale * A^dag B (nbA x nbB, row-major with row length out_ld)
struct OvTask {
    const double2* A;
    const double2* B;
    double2* out;
    int64_t ldA, ldB;
    int npw, nbA, nbB, out_ld;
    double scale;
    int64_t part_off;  // complex elements into the partial buffer
    int nchunk, tilesB, ntiles;
    int item;          // work item (index into an activity mask)
};
// out = beta * out + X M (M: nbX x nbO row-major with row length M_ld)
struct RotTask {
    const double2* X;
    const double2* M;
    double2* out;
    int64_t ldX, ldout;
    int npw, nbX, nbO, M_ld;
    double beta;
    int item;          // work item (index into an activity mask)
    int nbX2;          // optional second term out += X2 M2 (0: none; same ldX, M_ld)
    const double2* X2;
    const double2* M2;
};
OvTask make_ov_task(int npw, int nbA, const double2* A, int64_t ldA, int nbB, const double2* B, int64_t ldB,
                    double scale, double2* out, int out_ld);
RotTask make_rot_task(int npw, int nbX, const double2* X, int64_t ldX, int nbO, const double2* M, int M_ld,
                      double beta, double2* out, int64_t ldout);
// Batched contractions over a device task table; `act` (nullable) masks
// tasks by their work item: tasks of inactive items do nothing.
// Launch choices (set by the tuner): ov_mode 0 = 2x2 tile blocks per wave over
// 256-point chunks, then a fixed-order reduction of the chunk partials; 1 =
// the same with single 16x16 tiles per wave; 2 = one workgroup per (task,
// tile block) over all points, writing the result directly (one launch).
// rot_pt = 1, 2 or 4 fixes the point tiles per rotate wave for outputs of up
// to 32 bands (0: by the launch size).
// prec = DPP_F32 (the mixed-precision bulk): the overlap runs on split-BF16
// MFMA with FP32 accumulation over 1024-point chunks and FP64 chunk sums (its
// work list from overlap_worklist_bf16; ov_mode does not apply), the rotate on
// FP32 MFMA with FP32 accumulation.
dpp_status overlap_tasks(dpp_ctx ctx, const std::vector<OvTask>& h, const OvTask* d_tasks, double2* part,
                         const int* act = nullptr, int ov_mode = 0, const int4* d_work = nullptr, int nwork = 0,
                         dpp_precision prec = DPP_F64);
// The (task, chunk, block) workgroups with work of a task table in launch
// mode ov_mode, for the work-list form of the overlap launch.
void overlap_worklist(const std::vector<OvTask>& h, int ov_mode, std::vector<int4>& w);
// The same for the split-BF16 overlap, ordered so that the workgroups of one
// (task, chunk) run on one XCD (padding entries have x < 0).
void overlap_worklist_bf16(const std::vector<OvTask>& h, std::vector<int4>& w);
dpp_status rotate_tasks(dpp_ctx ctx, const std::vector<RotTask>& h, const RotTask* d_tasks,
                        const int* act = nullptr, int rot_pt = 0, const int2* d_work = nullptr, int nwork = 0,
                        dpp_precision prec = DPP_F64);
// The (task, block) workgroups with points of a rotate task table for the
// launch shape rot_pt picks, for the work-list form of the launch.
void rotate_worklist(const std::vector<RotTask>& h, int rot_pt, std::vector<int2>& w, bool f32 = false);
dpp_status overlap_single(dpp_ctx ctx, int npw, int nbA, const double2* A, int64_t ldA, int nbB,
                          const double2* B, int64_t ldB, double scale, double2* U, void* ws, size_t ws_bytes,
                          dpp_precision prec = DPP_F64);
size_t overlap_ws_bytes(int npw, int nbA, int nbB);
size_t proj_ws_bytes(const dpp_basis_s* b, int nb);
dpp_status rotate_single(dpp_ctx ctx, int npw, int nbX, const double2* X, int64_t ldX, int nbO,
                         const double2* M, double beta, double2* out, int64_t ldout, dpp_precision prec = DPP_F64);

// Records, for the current device, the address of the eigensolver's static
// workspace (dpp_subspace_eigh_noalloc); called by dpp_ctx_create.
dpp_status eigh_scratch_setup(int device);

}  // namespace dpp
