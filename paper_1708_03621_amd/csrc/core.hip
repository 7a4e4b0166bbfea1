// Context, grid (GridInfo), G-sphere basis builder, Hamiltonian handles and
// the diagonal operators O, L, K.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "internal.h"

namespace dpp {

static thread_local std::string g_last_error;

dpp_status set_error(dpp_status st, const std::string& msg) {
    g_last_error = msg;
    return st;
}
void clear_error() { g_last_error.clear(); }

}  // namespace dpp

using namespace dpp;

extern "C" const char* dpp_last_error(void) { return g_last_error.c_str(); }
extern "C" int dpp_version(void) { return 1; }

// ---------------------------------------------------------------- context --

extern "C" dpp_status dpp_ctx_create(int device, void* hip_stream, dpp_ctx* out) {
    clear_error();
    DPP_REQUIRE(out, "dpp_ctx_create: null output");
    int ndev = 0;
    DPP_HIP(hipGetDeviceCount(&ndev));
    DPP_REQUIRE(device >= 0 && device < ndev, "dpp_ctx_create: no such device");
    DPP_HIP(hipSetDevice(device));
    DPP_TRY(eigh_scratch_setup(device));
    dpp_ctx c = new dpp_ctx_s();
    c->device = device;
    c->stream = reinterpret_cast<hipStream_t>(hip_stream);
    if (hipMalloc(&c->d_status, sizeof(int)) != hipSuccess) {
        delete c;
        return set_error(DPP_ENOMEM, "dpp_ctx_create: status word allocation failed");
    }
    DPP_HIP(hipMemsetAsync(c->d_status, 0, sizeof(int), c->stream));
    DPP_HIP(hipStreamSynchronize(c->stream));
    *out = c;
    return DPP_OK;
}

static void timer_flush(dpp_ctx c) {
    KernelTimer& t = c->timer;
    if (t.used == 0) return;
    hipStreamSynchronize(c->stream);
    for (int u = 0; u < t.used; ++u) {
        float ms = 0.0f;
        if (hipEventElapsedTime(&ms, t.ev[2 * u], t.ev[2 * u + 1]) == hipSuccess) {
            t.total_ms[t.kind[u]] += ms;
            t.count[t.kind[u]] += 1;
        }
    }
    t.used = 0;
}

dpp::TimerScope::TimerScope(dpp_ctx_s* ctx, int kind, double bytes, double flops) : c(ctx), slot(-1) {
    KernelTimer& t = c->timer;
    if (!t.on || kind < 0 || kind >= 32) return;
    if (t.used == t.cap) timer_flush(c);
    slot = t.used++;
    t.kind[slot] = kind;
    t.bytes[kind] += bytes;
    t.flops[kind] += flops;
    hipEventRecord(t.ev[2 * slot], c->stream);
}

dpp::TimerScope::~TimerScope() {
    if (slot >= 0) hipEventRecord(c->timer.ev[2 * slot + 1], c->stream);
}

extern "C" dpp_status dpp_timer_enable(dpp_ctx ctx, int on) {
    clear_error();
    DPP_REQUIRE(ctx, "dpp_timer_enable: null context");
    KernelTimer& t = ctx->timer;
    if (on && t.cap == 0) {
        const int cap = 4096;
        t.ev.resize(2 * cap);
        for (auto& e : t.ev) DPP_HIP(hipEventCreate(&e));
        t.kind.assign(cap, 0);
        t.cap = cap;
    }
    if (!on) timer_flush(ctx);
    t.on = on != 0;
    return DPP_OK;
}

extern "C" dpp_status dpp_timer_reset(dpp_ctx ctx) {
    clear_error();
    DPP_REQUIRE(ctx, "dpp_timer_reset: null context");
    timer_flush(ctx);
    for (int k = 0; k < 32; ++k)
        ctx->timer.total_ms[k] = 0, ctx->timer.count[k] = 0, ctx->timer.bytes[k] = 0, ctx->timer.flops[k] = 0;
    return DPP_OK;
}

extern "C" dpp_status dpp_timer_read(dpp_ctx ctx, int kind, double* total_ms, int64_t* launches, double* bytes,
                                     double* flops) {
    clear_error();
    DPP_REQUIRE(ctx && kind >= 0 && kind < 32, "dpp_timer_read: bad arguments");
    timer_flush(ctx);
    if (total_ms) *total_ms = ctx->timer.total_ms[kind];
    if (launches) *launches = ctx->timer.count[kind];
    if (bytes) *bytes = ctx->timer.bytes[kind];
    if (flops) *flops = ctx->timer.flops[kind];
    return DPP_OK;
}

extern "C" dpp_status dpp_ctx_destroy(dpp_ctx ctx) {
    clear_error();
    if (!ctx) return DPP_OK;
    hipStreamSynchronize(ctx->stream);
    for (auto& e : ctx->timer.ev) hipEventDestroy(e);
    hipFree(ctx->d_status);
    delete ctx;
    return DPP_OK;
}

extern "C" dpp_status dpp_ctx_status(dpp_ctx ctx, int clear, int* out) {
    clear_error();
    DPP_REQUIRE(ctx && out, "dpp_ctx_status: null argument");
    DPP_HIP(hipStreamSynchronize(ctx->stream));
    int v = 0;
    DPP_HIP(hipMemcpy(&v, ctx->d_status, sizeof(int), hipMemcpyDeviceToHost));
    if (clear) DPP_HIP(hipMemset(ctx->d_status, 0, sizeof(int)));
    *out = v;
    return DPP_OK;
}

// ------------------------------------------------------------------- grid --

static void inv3(const double* a, double* inv) {
    // row-major 3x3 inverse
    const double det = a[0] * (a[4] * a[8] - a[5] * a[7]) - a[1] * (a[3] * a[8] - a[5] * a[6]) +
                       a[2] * (a[3] * a[7] - a[4] * a[6]);
    inv[0] = (a[4] * a[8] - a[5] * a[7]) / det;
    inv[1] = (a[2] * a[7] - a[1] * a[8]) / det;
    inv[2] = (a[1] * a[5] - a[2] * a[4]) / det;
    inv[3] = (a[5] * a[6] - a[3] * a[8]) / det;
    inv[4] = (a[0] * a[8] - a[2] * a[6]) / det;
    inv[5] = (a[2] * a[3] - a[0] * a[5]) / det;
    inv[6] = (a[3] * a[7] - a[4] * a[6]) / det;
    inv[7] = (a[1] * a[6] - a[0] * a[7]) / det;
    inv[8] = (a[0] * a[4] - a[1] * a[3]) / det;
}

static bool smooth235(int n) {
    for (int p : {2, 3, 5})
        while (n % p == 0) n /= p;
    return n == 1;
}

static void free_grid(dpp_grid g) {
    for (int a = 0; a < 3; ++a) {
        if (g->d_tw64[a]) hipFree(g->d_tw64[a]);
        if (g->d_tw32[a]) hipFree(g->d_tw32[a]);
    }
    if (g->d_fullplanes) hipFree(g->d_fullplanes);
    if (g->h_pin) hipHostFree(g->h_pin);
    delete g;
}

extern "C" dpp_status dpp_grid_create(dpp_ctx ctx, const double* R, const int* S, dpp_grid* out) {
    clear_error();
    DPP_REQUIRE(ctx && R && S && out, "dpp_grid_create: null argument");
    for (int d = 0; d < 3; ++d) {
        DPP_REQUIRE(S[d] >= 4 && S[d] <= 128 && smooth235(S[d]),
                    "dpp_grid_create: box sizes must be 2/3/5-smooth in [4, 128]");
    }
    DPP_TRY(check_fft_shape(S[0], S[1], S[2], true));
    const double det = R[0] * (R[4] * R[8] - R[5] * R[7]) - R[1] * (R[3] * R[8] - R[5] * R[6]) +
                       R[2] * (R[3] * R[7] - R[4] * R[6]);
    DPP_REQUIRE(std::isfinite(det) && std::fabs(det) > 1e-12, "dpp_grid_create: singular cell");
    dpp_grid g = new dpp_grid_s();
    std::memset(g->d_tw64, 0, sizeof(g->d_tw64));
    std::memset(g->d_tw32, 0, sizeof(g->d_tw32));
    g->d_fullplanes = nullptr;
    g->ctx = ctx;
    std::memcpy(g->R, R, sizeof(double) * 9);
    g->omega = std::fabs(det);
    // B = 2 pi R^{-T}: B[i][j] = 2 pi Rinv[j][i]
    double Ri[9];
    inv3(R, Ri);
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) g->B[3 * i + j] = 2.0 * M_PI * Ri[3 * j + i];
    for (int d = 0; d < 3; ++d) g->S[d] = S[d];
    g->N = (int64_t)S[0] * S[1] * S[2];
    for (int d = 0; d < 3; ++d) {
        if (!factor_axis(S[d], &g->ax[d])) {
            free_grid(g);
            return set_error(DPP_EINVAL, "dpp_grid_create: unsupported box size");
        }
        const int n = S[d];
        std::vector<double2> t64(n);
        std::vector<float2> t32(n);
        for (int m = 0; m < n; ++m) {
            // exp(-2 pi i m / n) with the angle reduced to the first octants for accuracy
            const double ang = -2.0 * M_PI * (double)m / (double)n;
            t64[m] = double2{std::cos(ang), std::sin(ang)};
            t32[m] = float2{(float)t64[m].x, (float)t64[m].y};
        }
        if (hipMalloc(&g->d_tw64[d], n * sizeof(double2)) != hipSuccess ||
            hipMalloc(&g->d_tw32[d], n * sizeof(float2)) != hipSuccess) {
            free_grid(g);
            return set_error(DPP_ENOMEM, "dpp_grid_create: twiddle allocation failed");
        }
        DPP_HIP(hipMemcpy(g->d_tw64[d], t64.data(), n * sizeof(double2), hipMemcpyHostToDevice));
        DPP_HIP(hipMemcpy(g->d_tw32[d], t32.data(), n * sizeof(float2), hipMemcpyHostToDevice));
    }
    std::vector<int4> fp(S[0]);
    for (int p = 0; p < S[0]; ++p) fp[p] = int4{0, 0, 0, S[1]};
    if (hipMalloc(&g->d_fullplanes, S[0] * sizeof(int4)) != hipSuccess) {
        free_grid(g);
        return set_error(DPP_ENOMEM, "dpp_grid_create: allocation failed");
    }
    DPP_HIP(hipMemcpy(g->d_fullplanes, fp.data(), S[0] * sizeof(int4), hipMemcpyHostToDevice));
    FftItem& it = g->h_item;
    std::memset(&it, 0, sizeof(it));
    it.S0 = S[0];
    it.S1 = S[1];
    it.S2 = S[2];
    it.nplanes = S[0];
    it.n0min = 0;
    it.npw = 0;
    it.nb = 1;
    it.full = 1;
    for (int d = 0; d < 3; ++d) {
        it.ax[d] = g->ax[d];
        it.tw64[d] = g->d_tw64[d];
        it.tw32[d] = g->d_tw32[d];
    }
    it.planes = g->d_fullplanes;
    it.omega = g->omega;
    it.vscale = g->omega / (double)g->N;
    it.vperm = 1;
    for (int i = 0; i < 9; ++i) it.B[i] = g->B[i];
    *out = g;
    return DPP_OK;
}

extern "C" dpp_status dpp_grid_destroy(dpp_grid grid) {
    clear_error();
    if (!grid) return DPP_OK;
    hipStreamSynchronize(grid->ctx->stream);
    free_grid(grid);
    return DPP_OK;
}

extern "C" dpp_status dpp_grid_info(dpp_grid grid, double* omega, int64_t* N) {
    clear_error();
    DPP_REQUIRE(grid, "dpp_grid_info: null grid");
    if (omega) *omega = grid->omega;
    if (N) *N = grid->N;
    return DPP_OK;
}

// ------------------------------------------------------------- G-sphere ----
// Enumerate the bounding box of Miller indices lexicographically, flag the
// points inside the sphere, scan the flags (one workgroup), compact.

struct SphereBox {
    int lo0, lo1, lo2, n0, n1, n2;  // range starts and extents
    double k0, k1, k2;
    double B[9];
    double ecut;
};

__global__ void k_sphere_flags(SphereBox sb, int64_t M, int* __restrict__ flags) {
    const int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= M) return;
    const int a2 = (int)(m % sb.n2);
    const int64_t r = m / sb.n2;
    const int a1 = (int)(r % sb.n1);
    const int a0 = (int)(r / sb.n1);
    const double x0 = (double)(sb.lo0 + a0) + sb.k0;
    const double x1 = (double)(sb.lo1 + a1) + sb.k1;
    const double x2 = (double)(sb.lo2 + a2) + sb.k2;
    const double g0 = sb.B[0] * x0 + sb.B[1] * x1 + sb.B[2] * x2;
    const double g1 = sb.B[3] * x0 + sb.B[4] * x1 + sb.B[5] * x2;
    const double g2 = sb.B[6] * x0 + sb.B[7] * x1 + sb.B[8] * x2;
    const double q2 = g0 * g0 + g1 * g1 + g2 * g2;
    flags[m] = (0.5 * q2 <= sb.ecut) ? 1 : 0;
}

// Exclusive scan of flags[0..M) by one workgroup of 1024 threads: each
// thread scans a contiguous segment, segment totals are scanned in LDS.
__global__ void __launch_bounds__(1024) k_scan_1wg(const int* __restrict__ flags, int64_t M,
                                                   int* __restrict__ pos, int* __restrict__ total) {
    __shared__ int sums[1024];
    const int t = threadIdx.x;
    const int64_t seg = (M + 1023) / 1024;
    const int64_t a = t * seg, e = min(M, a + seg);
    int s = 0;
    for (int64_t i = a; i < e; ++i) s += flags[i];
    sums[t] = s;
    __syncthreads();
    if (t == 0) {
        int acc = 0;
        for (int i = 0; i < 1024; ++i) {
            const int v = sums[i];
            sums[i] = acc;
            acc += v;
        }
        *total = acc;
    }
    __syncthreads();
    int run = sums[t];
    for (int64_t i = a; i < e; ++i) {
        pos[i] = run;
        run += flags[i];
    }
}

__global__ void k_sphere_compact(SphereBox sb, int64_t M, const int* __restrict__ flags,
                                 const int* __restrict__ pos, int S0, int S1, int S2,
                                 int32_t* __restrict__ index, int32_t* __restrict__ poff,
                                 int4* __restrict__ miller, double* __restrict__ kG2) {
    const int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= M || !flags[m]) return;
    const int a2 = (int)(m % sb.n2);
    const int64_t r = m / sb.n2;
    const int a1 = (int)(r % sb.n1);
    const int a0 = (int)(r / sb.n1);
    const int n0 = sb.lo0 + a0, n1 = sb.lo1 + a1, n2 = sb.lo2 + a2;
    const double x0 = (double)n0 + sb.k0, x1 = (double)n1 + sb.k1, x2 = (double)n2 + sb.k2;
    const double g0 = sb.B[0] * x0 + sb.B[1] * x1 + sb.B[2] * x2;
    const double g1 = sb.B[3] * x0 + sb.B[4] * x1 + sb.B[5] * x2;
    const double g2 = sb.B[6] * x0 + sb.B[7] * x1 + sb.B[8] * x2;
    const int q = pos[m];
    const int i0 = ((n0 % S0) + S0) % S0, i1 = ((n1 % S1) + S1) % S1, i2 = ((n2 % S2) + S2) % S2;
    index[q] = (i0 * S1 + i1) * S2 + i2;
    poff[q] = i1 * S2 + i2;
    miller[q] = int4{n0, n1, n2, 0};
    kG2[q] = g0 * g0 + g1 * g1 + g2 * g2;
}

static void free_basis(dpp_basis b) {
    if (b->d_index) hipFree(b->d_index);
    if (b->d_poff) hipFree(b->d_poff);
    if (b->d_miller) hipFree(b->d_miller);
    if (b->d_kG2) hipFree(b->d_kG2);
    if (b->d_planes) hipFree(b->d_planes);
    if (b->d_rows) hipFree(b->d_rows);
    delete b;
}

extern "C" dpp_status dpp_basis_create(dpp_grid grid, const double* k_red, double ecut, dpp_basis* out) {
    clear_error();
    DPP_REQUIRE(grid && k_red && out, "dpp_basis_create: null argument");
    DPP_REQUIRE(std::isfinite(ecut) && ecut > 0, "dpp_basis_create: ecut must be positive");
    hipStream_t st = grid->ctx->stream;
    SphereBox sb;
    const double gmax = std::sqrt(2.0 * ecut);
    int lo[3], n[3];
    for (int d = 0; d < 3; ++d) {
        const double a = std::sqrt(grid->R[d] * grid->R[d] + grid->R[3 + d] * grid->R[3 + d] +
                                   grid->R[6 + d] * grid->R[6 + d]);
        const double ext = gmax * a / (2.0 * M_PI);
        lo[d] = (int)std::floor(-ext - k_red[d]) - 1;
        const int hi = (int)std::ceil(ext - k_red[d]) + 1;
        n[d] = hi - lo[d] + 1;
    }
    sb.lo0 = lo[0];
    sb.lo1 = lo[1];
    sb.lo2 = lo[2];
    sb.n0 = n[0];
    sb.n1 = n[1];
    sb.n2 = n[2];
    sb.k0 = k_red[0];
    sb.k1 = k_red[1];
    sb.k2 = k_red[2];
    std::memcpy(sb.B, grid->B, sizeof(sb.B));
    sb.ecut = ecut;
    const int64_t M = (int64_t)n[0] * n[1] * n[2];
    DPP_REQUIRE(M < (int64_t)1 << 30, "dpp_basis_create: cutoff too large");

    int *d_flags = nullptr, *d_pos = nullptr, *d_total = nullptr;
    DPP_HIP(hipMalloc(&d_flags, M * sizeof(int)));
    DPP_HIP(hipMalloc(&d_pos, M * sizeof(int)));
    DPP_HIP(hipMalloc(&d_total, sizeof(int)));
    const unsigned nblk = (unsigned)((M + 255) / 256);
    hipLaunchKernelGGL(k_sphere_flags, dim3(nblk), dim3(256), 0, st, sb, M, d_flags);
    hipLaunchKernelGGL(k_scan_1wg, dim3(1), dim3(1024), 0, st, d_flags, M, d_pos, d_total);
    int npw = 0;
    DPP_HIP(hipMemcpyAsync(&npw, d_total, sizeof(int), hipMemcpyDeviceToHost, st));
    DPP_HIP(hipStreamSynchronize(st));

    dpp_basis b = new dpp_basis_s();
    b->grid = grid;
    std::memcpy(b->k, k_red, sizeof(b->k));
    b->ecut = ecut;
    b->npw = npw;
    b->d_index = b->d_poff = nullptr;
    b->d_miller = nullptr;
    b->d_kG2 = nullptr;
    b->d_planes = nullptr;
    b->d_rows = nullptr;
    const int S0 = grid->S[0], S1 = grid->S[1], S2 = grid->S[2];
    bool ok = npw > 0 && hipMalloc(&b->d_index, npw * sizeof(int32_t)) == hipSuccess &&
              hipMalloc(&b->d_poff, npw * sizeof(int32_t)) == hipSuccess &&
              hipMalloc(&b->d_miller, npw * sizeof(int4)) == hipSuccess &&
              hipMalloc(&b->d_kG2, npw * sizeof(double)) == hipSuccess;
    if (!ok) {
        hipFree(d_flags);
        hipFree(d_pos);
        hipFree(d_total);
        free_basis(b);
        return set_error(npw > 0 ? DPP_ENOMEM : DPP_EINVAL, "dpp_basis_create: empty sphere or allocation failed");
    }
    hipLaunchKernelGGL(k_sphere_compact, dim3(nblk), dim3(256), 0, st, sb, M, d_flags, d_pos, S0, S1, S2,
                       b->d_index, b->d_poff, b->d_miller, b->d_kG2);
    std::vector<int4> mil(npw);
    DPP_HIP(hipMemcpyAsync(mil.data(), b->d_miller, npw * sizeof(int4), hipMemcpyDeviceToHost, st));
    DPP_HIP(hipStreamSynchronize(st));
    hipFree(d_flags);
    hipFree(d_pos);
    hipFree(d_total);

    // extents and per-plane tables (points of one n0 are contiguous)
    int ext[6] = {mil[0].x, mil[0].x, mil[0].y, mil[0].y, mil[0].z, mil[0].z};
    for (const int4& m : mil) {
        ext[0] = std::min(ext[0], m.x), ext[1] = std::max(ext[1], m.x);
        ext[2] = std::min(ext[2], m.y), ext[3] = std::max(ext[3], m.y);
        ext[4] = std::min(ext[4], m.z), ext[5] = std::max(ext[5], m.z);
    }
    if (ext[1] - ext[0] + 1 > S0 || ext[3] - ext[2] + 1 > S1 || ext[5] - ext[4] + 1 > S2) {
        free_basis(b);
        return set_error(DPP_EINVAL, "dpp_basis_create: G-sphere does not fit in the FFT box");
    }
    std::memcpy(b->next, ext, sizeof(ext));
    b->n0min = ext[0];
    b->nplanes = ext[1] - ext[0] + 1;
    b->h_planes.assign(b->nplanes, int4{0, 0, 0, 0});
    {
        int q = 0;
        for (int p = 0; p < b->nplanes; ++p) {
            const int n0 = b->n0min + p;
            const int start = q;
            int lo1 = 1 << 30, hi1 = -(1 << 30);
            while (q < npw && mil[q].x == n0) {
                lo1 = std::min(lo1, mil[q].y);
                hi1 = std::max(hi1, mil[q].y);
                ++q;
            }
            const int cnt = q - start;
            b->h_planes[p] = cnt > 0 ? int4{start, cnt, lo1, hi1 - lo1 + 1} : int4{start, 0, 0, 0};
        }
    }
    if (hipMalloc(&b->d_planes, b->nplanes * sizeof(int4)) != hipSuccess) {
        free_basis(b);
        return set_error(DPP_ENOMEM, "dpp_basis_create: allocation failed");
    }
    DPP_HIP(hipMemcpy(b->d_planes, b->h_planes.data(), b->nplanes * sizeof(int4), hipMemcpyHostToDevice));
    // per (plane, natural row i1): first point, count, n2 of the first point
    // (the points of one (n0, n1) row are contiguous with n2 ascending)
    {
        std::vector<int4> rows((size_t)b->nplanes * S1, int4{0, 0, 0, 0});
        for (int q = 0; q < npw;) {
            const int p = mil[q].x - b->n0min, n1 = mil[q].y;
            const int i1 = ((n1 % S1) + S1) % S1;
            int e = q;
            while (e < npw && mil[e].x == mil[q].x && mil[e].y == n1) ++e;
            rows[(size_t)p * S1 + i1] = int4{q, e - q, mil[q].z, 0};
            q = e;
        }
        if (hipMalloc(&b->d_rows, rows.size() * sizeof(int4)) != hipSuccess) {
            free_basis(b);
            return set_error(DPP_ENOMEM, "dpp_basis_create: allocation failed");
        }
        DPP_HIP(hipMemcpy(b->d_rows, rows.data(), rows.size() * sizeof(int4), hipMemcpyHostToDevice));
    }
    FftItem& it = b->h_item;
    it = grid->h_item;
    it.nplanes = b->nplanes;
    it.n0min = b->n0min;
    it.npw = npw;
    it.nb = 0;
    it.full = 0;
    it.planes = b->d_planes;
    it.rows = b->d_rows;
    it.poff = b->d_poff;
    it.kG2 = b->d_kG2;
    *out = b;
    return DPP_OK;
}

extern "C" dpp_status dpp_basis_destroy(dpp_basis basis) {
    clear_error();
    if (!basis) return DPP_OK;
    hipStreamSynchronize(basis->grid->ctx->stream);
    free_basis(basis);
    return DPP_OK;
}

extern "C" dpp_status dpp_basis_info(dpp_basis basis, int64_t* npw, int32_t* n_ext) {
    clear_error();
    DPP_REQUIRE(basis, "dpp_basis_info: null basis");
    if (npw) *npw = basis->npw;
    if (n_ext)
        for (int i = 0; i < 6; ++i) n_ext[i] = basis->next[i];
    return DPP_OK;
}

extern "C" dpp_status dpp_basis_export(dpp_basis basis, int32_t* d_index, double* d_kG2) {
    clear_error();
    DPP_REQUIRE(basis, "dpp_basis_export: null basis");
    hipStream_t st = basis->grid->ctx->stream;
    if (d_index)
        DPP_HIP(hipMemcpyAsync(d_index, basis->d_index, basis->npw * sizeof(int32_t),
                               hipMemcpyDeviceToDevice, st));
    if (d_kG2)
        DPP_HIP(hipMemcpyAsync(d_kG2, basis->d_kG2, basis->npw * sizeof(double), hipMemcpyDeviceToDevice, st));
    return DPP_OK;
}

// ------------------------------------------------------------ diagonals ----

// mode 0: O (Omega), 1: L (-Omega |k+G|^2), 2: K (1 / (1 + |k+G|^2 / 2))
__global__ void k_diag(int mode, int npw, int nb, double omega, const double* __restrict__ kG2,
                       const double2* in, int64_t ldin, double2* out, int64_t ldout) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    const int b = blockIdx.y;
    if (q >= npw || b >= nb) return;
    double s;
    if (mode == 0)
        s = omega;
    else if (mode == 1)
        s = -omega * kG2[q];
    else
        s = 1.0 / (1.0 + 0.5 * kG2[q]);
    const double2 v = in[(int64_t)b * ldin + q];
    out[(int64_t)b * ldout + q] = double2{s * v.x, s * v.y};
}

static dpp_status diag_op(int mode, dpp_basis b, int nb, const dpp_c64* in, int64_t ldin, dpp_c64* out,
                          int64_t ldout, const char* who) {
    clear_error();
    DPP_REQUIRE(b && nb >= 0, std::string(who) + ": bad arguments");
    DPP_REQUIRE(nb == 0 || (in && out), std::string(who) + ": null block");
    DPP_REQUIRE(ldin >= b->npw && ldout >= b->npw, std::string(who) + ": leading dimension < npw");
    if (nb == 0) return DPP_OK;
    DPP_REQUIRE(nb <= 65535, std::string(who) + ": too many bands");
    hipLaunchKernelGGL(k_diag, dim3((unsigned)((b->npw + 255) / 256), nb), dim3(256), 0, b->grid->ctx->stream,
                       mode, (int)b->npw, nb, b->grid->omega, b->d_kG2, (const double2*)in, ldin,
                       (double2*)out, ldout);
    DPP_LAUNCHED();
    return DPP_OK;
}

extern "C" dpp_status dpp_O(dpp_basis b, int nb, const dpp_c64* in, int64_t ldin, dpp_c64* out, int64_t ldout) {
    return diag_op(0, b, nb, in, ldin, out, ldout, "dpp_O");
}
extern "C" dpp_status dpp_L(dpp_basis b, int nb, const dpp_c64* in, int64_t ldin, dpp_c64* out, int64_t ldout) {
    return diag_op(1, b, nb, in, ldin, out, ldout, "dpp_L");
}
extern "C" dpp_status dpp_K(dpp_basis b, int nb, const dpp_c64* in, int64_t ldin, dpp_c64* out, int64_t ldout) {
    return diag_op(2, b, nb, in, ldin, out, ldout, "dpp_K");
}

// ----------------------------------------------------------- Hamiltonian ---

// P[a][q] = exp(-|k+G|^2 rp^2 / 2) exp(-i G.tau_a), G = B n (without k).
__global__ void k_projectors(int npw, int nproj, const int4* __restrict__ miller,
                             const double* __restrict__ kG2, const double* __restrict__ tau,
                             double B0, double B1, double B2, double B3, double B4, double B5,
                             double B6, double B7, double B8, double rp, double2* __restrict__ P) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    const int a = blockIdx.y;
    if (q >= npw || a >= nproj) return;
    const int4 m = miller[q];
    const double gx = B0 * m.x + B1 * m.y + B2 * m.z;
    const double gy = B3 * m.x + B4 * m.y + B5 * m.z;
    const double gz = B6 * m.x + B7 * m.y + B8 * m.z;
    const double ph = gx * tau[3 * a] + gy * tau[3 * a + 1] + gz * tau[3 * a + 2];
    const double beta = exp(-kG2[q] * rp * rp * 0.5);
    double s, c;
    sincos(ph, &s, &c);
    P[(int64_t)a * npw + q] = double2{beta * c, -beta * s};
}

extern "C" dpp_status dpp_ham_create(dpp_basis basis, int nat, const double* tau, const int* has_proj,
                                     double rp, double D, dpp_ham* out) {
    clear_error();
    DPP_REQUIRE(basis && out && nat >= 0, "dpp_ham_create: bad arguments");
    DPP_REQUIRE(nat == 0 || (tau && has_proj), "dpp_ham_create: null atom arrays");
    DPP_REQUIRE(std::isfinite(rp) && rp > 0 && std::isfinite(D), "dpp_ham_create: bad projector parameters");
    std::vector<double> tp;
    for (int a = 0; a < nat; ++a)
        if (has_proj[a])
            for (int d = 0; d < 3; ++d) tp.push_back(tau[3 * a + d]);
    const int nproj = (int)tp.size() / 3;
    dpp_ham h = new dpp_ham_s();
    h->basis = basis;
    h->nproj = nproj;
    h->D = D;
    h->rp = rp;
    h->d_P = nullptr;
    h->d_Veff = nullptr;
    if (nproj > 0) {
        if (hipMalloc(&h->d_P, (size_t)nproj * basis->npw * sizeof(double2)) != hipSuccess) {
            delete h;
            return set_error(DPP_ENOMEM, "dpp_ham_create: allocation failed");
        }
        const dpp_status st = ham_set_positions(h, nat, tau, has_proj);
        if (st != DPP_OK) {
            hipFree(h->d_P);
            delete h;
            return st;
        }
    }
    *out = h;
    return DPP_OK;
}

dpp_status dpp::ham_set_positions(dpp_ham_s* h, int nat, const double* tau, const int* has_proj) {
    std::vector<double> tp;
    for (int a = 0; a < nat; ++a)
        if (has_proj[a])
            for (int d = 0; d < 3; ++d) tp.push_back(tau[3 * a + d]);
    if ((int)tp.size() != 3 * h->nproj) return set_error(DPP_EINVAL, "projector atoms changed");
    if (h->nproj == 0) return DPP_OK;
    const dpp_basis basis = h->basis;
    double* d_tau = nullptr;
    if (hipMalloc(&d_tau, tp.size() * sizeof(double)) != hipSuccess)
        return set_error(DPP_ENOMEM, "projector positions: allocation failed");
    hipStream_t st = basis->grid->ctx->stream;
    hipError_t e = hipMemcpyAsync(d_tau, tp.data(), tp.size() * sizeof(double), hipMemcpyHostToDevice, st);
    if (e == hipSuccess) {
        const double* B = basis->grid->B;
        hipLaunchKernelGGL(k_projectors, dim3((unsigned)((basis->npw + 255) / 256), h->nproj), dim3(256), 0, st,
                           (int)basis->npw, h->nproj, basis->d_miller, basis->d_kG2, d_tau, B[0], B[1], B[2], B[3],
                           B[4], B[5], B[6], B[7], B[8], h->rp, h->d_P);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    hipFree(d_tau);
    if (e != hipSuccess) return set_error(DPP_EDEVICE, "projector positions: HIP error");
    return DPP_OK;
}

extern "C" dpp_status dpp_ham_destroy(dpp_ham ham) {
    clear_error();
    if (!ham) return DPP_OK;
    hipStreamSynchronize(ham->basis->grid->ctx->stream);
    if (ham->d_P) hipFree(ham->d_P);
    delete ham;
    return DPP_OK;
}

extern "C" dpp_status dpp_ham_set_potential(dpp_ham ham, const double* d_Veff) {
    clear_error();
    DPP_REQUIRE(ham && d_Veff, "dpp_ham_set_potential: null argument");
    ham->d_Veff = d_Veff;
    return DPP_OK;
}
