// Real-space scalar fields: LDA exchange-correlation, local pseudopotential,
// superposition start density and deterministic grid reductions.
#include <hip/hip_runtime.h>

#include <cmath>
#include <vector>

#include "internal.h"

namespace dpp {

// Perdew-Zunger 1981 parametrization of the unpolarized correlation energy
// (Ceperley-Alder data) and Slater exchange.
constexpr double PZ_G = -0.1423, PZ_B1 = 1.0529, PZ_B2 = 0.3334;
constexpr double PZ_A = 0.0311, PZ_B = -0.048, PZ_C = 0.0020, PZ_D = -0.0116;
constexpr double N_FLOOR = 1e-16;

__device__ __forceinline__ void lda_point(double n, double* eps, double* v) {
    if (!(n >= N_FLOOR)) {
        *eps = 0.0;
        *v = 0.0;
        return;
    }
    const double cbn = cbrt(n);
    const double ex = -0.75 * 0.98474502184269641 * cbn;  // (3/pi)^{1/3} = 0.98474502...
    const double vx = (4.0 / 3.0) * ex;
    const double rs = 0.62035049089940009 / cbn;  // (3/(4 pi))^{1/3} / n^{1/3}
    double ec, vc;
    if (rs < 1.0) {
        const double lr = log(rs);
        ec = PZ_A * lr + PZ_B + PZ_C * rs * lr + PZ_D * rs;
        vc = PZ_A * lr + (PZ_B - PZ_A / 3.0) + (2.0 / 3.0) * PZ_C * rs * lr + ((2.0 * PZ_D - PZ_C) / 3.0) * rs;
    } else {
        const double srs = sqrt(rs);
        const double den = 1.0 + PZ_B1 * srs + PZ_B2 * rs;
        ec = PZ_G / den;
        vc = ec * (1.0 + (7.0 / 6.0) * PZ_B1 * srs + (4.0 / 3.0) * PZ_B2 * rs) / den;
    }
    *eps = ex + ec;
    *v = vx + vc;
}

constexpr int RED_BLOCKS = 1024;  // fixed number of partial sums for grid reductions

// v_xc per point; block partial of sum n eps_xc.
__global__ void __launch_bounds__(256)
k_lda(int64_t N, const double* __restrict__ n, double* __restrict__ vxc, double* __restrict__ part) {
    __shared__ double red[256];
    double acc = 0.0;
    for (int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x; j < N; j += (int64_t)gridDim.x * 256) {
        double e, v;
        const double nj = n[j];
        lda_point(nj, &e, &v);
        vxc[j] = v;
        acc += (nj >= N_FLOOR) ? nj * e : 0.0;
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ void __launch_bounds__(256)
k_dot(int64_t N, const double* __restrict__ a, const double* __restrict__ b, double* __restrict__ part) {
    __shared__ double red[256];
    double acc = 0.0;
    for (int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x; j < N; j += (int64_t)gridDim.x * 256)
        acc += a[j] * b[j];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ void k_sum_fixed(const double* __restrict__ part, int n, double scale, double* __restrict__ out) {
    __shared__ double red[256];
    double s = 0.0;
    for (int i = threadIdx.x; i < n; i += 256) s += part[i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = scale * red[0];
}

// ---------------------------------------------------------- many cells -----
// Fields of several cells concatenated (cell c at foff, N points); one row of
// CELL_RED_BLOCKS workgroups per cell, partial sums reduced per cell in fixed
// order.
constexpr int CELL_RED_BLOCKS = 256;

__device__ __forceinline__ double block_sum_256(double v, double* red) {
    red[threadIdx.x] = v;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    return red[0];
}

__global__ void __launch_bounds__(256)
k_lda_cells(const CellDesc* __restrict__ cells, const double* __restrict__ n, double* __restrict__ vxc,
            double* __restrict__ part) {
    __shared__ double red[256];
    const CellDesc c = cells[blockIdx.y];
    double acc = 0.0;
    for (int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x; j < c.N; j += (int64_t)CELL_RED_BLOCKS * 256) {
        double e, v;
        const double nj = n[c.foff + j];
        lda_point(nj, &e, &v);
        vxc[c.foff + j] = v;
        acc += (nj >= N_FLOOR) ? nj * e : 0.0;
    }
    const double t = block_sum_256(acc, red);
    if (threadIdx.x == 0) part[(int64_t)blockIdx.y * CELL_RED_BLOCKS + blockIdx.x] = t;
}

__global__ void __launch_bounds__(256)
k_dot_cells(const CellDesc* __restrict__ cells, const double* __restrict__ a, const double* __restrict__ b,
            double* __restrict__ part) {
    __shared__ double red[256];
    const CellDesc c = cells[blockIdx.y];
    double acc = 0.0;
    for (int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x; j < c.N; j += (int64_t)CELL_RED_BLOCKS * 256)
        acc += a[c.foff + j] * b[c.foff + j];
    const double t = block_sum_256(acc, red);
    if (threadIdx.x == 0) part[(int64_t)blockIdx.y * CELL_RED_BLOCKS + blockIdx.x] = t;
}

// E[c * stride] = (Omega / N)_c * sum of the cell's partials.
__global__ void __launch_bounds__(256)
k_sum_cells(const CellDesc* __restrict__ cells, const double* __restrict__ part, double* __restrict__ E,
            int stride) {
    __shared__ double red[256];
    double s = 0.0;
    for (int i = threadIdx.x; i < CELL_RED_BLOCKS; i += 256) s += part[(int64_t)blockIdx.x * CELL_RED_BLOCKS + i];
    const double t = block_sum_256(s, red);
    if (threadIdx.x == 0) E[(int64_t)blockIdx.x * stride] = cells[blockIdx.x].dV * t;
}

dpp_status lda_cells(dpp_ctx_s* ctx, const CellDesc* d_cells, int ncells, const double* n, double* vxc,
                     double* part, double* E, int stride) {
    TimerScope ts_(ctx, DPP_TK_FIELDS);
    hipLaunchKernelGGL(k_lda_cells, dim3(CELL_RED_BLOCKS, ncells), dim3(256), 0, ctx->stream, d_cells, n, vxc, part);
    DPP_LAUNCHED();
    if (!E) return DPP_OK;  // v_xc only
    hipLaunchKernelGGL(k_sum_cells, dim3(ncells), dim3(256), 0, ctx->stream, d_cells, (const double*)part, E, stride);
    DPP_LAUNCHED();
    return DPP_OK;
}

dpp_status dot_cells(dpp_ctx_s* ctx, const CellDesc* d_cells, int ncells, const double* a, const double* b,
                     double* part, double* E, int stride) {
    TimerScope ts_(ctx, DPP_TK_FIELDS);
    hipLaunchKernelGGL(k_dot_cells, dim3(CELL_RED_BLOCKS, ncells), dim3(256), 0, ctx->stream, d_cells, a, b, part);
    DPP_LAUNCHED();
    hipLaunchKernelGGL(k_sum_cells, dim3(ncells), dim3(256), 0, ctx->stream, d_cells, (const double*)part, E, stride);
    DPP_LAUNCHED();
    return DPP_OK;
}

size_t cell_red_elems(int ncells) { return (size_t)ncells * CELL_RED_BLOCKS; }

// Reciprocal-space field of atom-centred Gaussian-type terms on the full box:
// mode 0 (local pseudopotential): sum_a -4 pi Z_a exp(-G^2 rc_a^2/4) / (Omega G^2), 0 at G = 0
// mode 1 (start density):         sum_a Z_a exp(-G^2 sigma^2/4) / Omega
// each times exp(-i G.tau_a).  Output is the unnormalized coefficient array
// whose inverse FFT (e^{+i}) gives the real-space field.
struct AtomTable {
    int nat;
    const double* tau;  // nat x 3
    const double* Z;
    const double* w;    // rc (mode 0) or sigma (mode 1) per atom
};

__global__ void k_atom_field_G(int S0, int S1, int S2, double B0, double B1, double B2, double B3, double B4,
                               double B5, double B6, double B7, double B8, double omega, int mode,
                               AtomTable at, double2* __restrict__ out) {
    const int64_t N = (int64_t)S0 * S1 * S2;
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= N) return;
    const int i2 = (int)(j % S2);
    const int64_t r = j / S2;
    const int i1 = (int)(r % S1), i0 = (int)(r / S1);
    const int n0 = 2 * i0 < S0 ? i0 : i0 - S0;
    const int n1 = 2 * i1 < S1 ? i1 : i1 - S1;
    const int n2 = 2 * i2 < S2 ? i2 : i2 - S2;
    const double gx = B0 * n0 + B1 * n1 + B2 * n2;
    const double gy = B3 * n0 + B4 * n1 + B5 * n2;
    const double gz = B6 * n0 + B7 * n1 + B8 * n2;
    const double G2 = gx * gx + gy * gy + gz * gz;
    double re = 0.0, im = 0.0;
    if (mode == 1 || G2 > 0.0) {
        for (int a = 0; a < at.nat; ++a) {
            const double wa = at.w[a];
            double amp;
            if (mode == 0)
                amp = -4.0 * M_PI * at.Z[a] * exp(-G2 * wa * wa * 0.25) / (omega * G2);
            else
                amp = at.Z[a] * exp(-G2 * wa * wa * 0.25) / omega;
            const double ph = gx * at.tau[3 * a] + gy * at.tau[3 * a + 1] + gz * at.tau[3 * a + 2];
            double s, c;
            sincos(ph, &s, &c);
            re += amp * c;
            im -= amp * s;
        }
    }
    out[j] = double2{re, im};
}

}  // namespace dpp

using namespace dpp;

extern "C" dpp_status dpp_lda_pz81(dpp_grid grid, const double* d_n, double* d_vxc, double* d_Exc, void* ws) {
    clear_error();
    DPP_REQUIRE(grid && d_n && d_vxc && d_Exc && ws, "dpp_lda_pz81: null argument");
    hipStream_t st = grid->ctx->stream;
    double* part = reinterpret_cast<double*>(ws);
    TimerScope ts_(grid->ctx, DPP_TK_FIELDS);
    hipLaunchKernelGGL(k_lda, dim3(RED_BLOCKS), dim3(256), 0, st, grid->N, d_n, d_vxc, part);
    DPP_LAUNCHED();
    hipLaunchKernelGGL(k_sum_fixed, dim3(1), dim3(256), 0, st, part, RED_BLOCKS, grid->omega / (double)grid->N,
                       d_Exc);
    DPP_LAUNCHED();
    return DPP_OK;
}

extern "C" dpp_status dpp_grid_dot(dpp_grid grid, const double* d_a, const double* d_b, double scale,
                                   double* d_out, void* ws) {
    clear_error();
    DPP_REQUIRE(grid && d_a && d_b && d_out && ws, "dpp_grid_dot: null argument");
    hipStream_t st = grid->ctx->stream;
    double* part = reinterpret_cast<double*>(ws);
    TimerScope ts_(grid->ctx, DPP_TK_FIELDS);
    hipLaunchKernelGGL(k_dot, dim3(RED_BLOCKS), dim3(256), 0, st, grid->N, d_a, d_b, part);
    DPP_LAUNCHED();
    hipLaunchKernelGGL(k_sum_fixed, dim3(1), dim3(256), 0, st, part, RED_BLOCKS, scale, d_out);
    DPP_LAUNCHED();
    return DPP_OK;
}

// Build the reciprocal field in the workspace, then take Re of the inverse
// full-box transform (unnormalized: Jdag times N).
static dpp_status atom_field(dpp_grid g, int nat, const double* tau, const double* Z, const double* w,
                             int mode, double* d_out, void* ws) {
    hipStream_t st = g->ctx->stream;
    std::vector<double> host(5 * (size_t)nat);
    for (int a = 0; a < nat; ++a) {
        for (int d = 0; d < 3; ++d) host[3 * a + d] = tau[3 * a + d];
        host[3 * nat + a] = Z[a];
        host[4 * nat + a] = w[a];
    }
    double* d_tab = nullptr;
    DPP_HIP(hipMalloc(&d_tab, std::max<size_t>(host.size(), 1) * sizeof(double)));
    DPP_HIP(hipMemcpyAsync(d_tab, host.data(), host.size() * sizeof(double), hipMemcpyHostToDevice, st));
    AtomTable at{nat, d_tab, d_tab + 3 * nat, d_tab + 4 * nat};
    double2* coef = reinterpret_cast<double2*>(reinterpret_cast<char*>(ws) + grid_coef_offset(g));
    const double* B = g->B;
    hipLaunchKernelGGL(k_atom_field_G, dim3((unsigned)((g->N + 255) / 256)), dim3(256), 0, st, g->S[0], g->S[1],
                       g->S[2], B[0], B[1], B[2], B[3], B[4], B[5], B[6], B[7], B[8], g->omega, mode, at, coef);
    dpp_status s = DPP_OK;
    if (hipGetLastError() != hipSuccess) s = set_error(DPP_EDEVICE, "atom_field: launch failed");
    if (s == DPP_OK) s = full_inverse_real(g, coef, d_out, ws);
    hipStreamSynchronize(st);
    hipFree(d_tab);
    return s;
}

extern "C" dpp_status dpp_local_potential(dpp_grid grid, int nat, const double* tau, const double* Z,
                                          const double* rc, double* d_Vloc, void* ws) {
    clear_error();
    DPP_REQUIRE(grid && d_Vloc && ws && nat >= 0, "dpp_local_potential: bad arguments");
    DPP_REQUIRE(nat == 0 || (tau && Z && rc), "dpp_local_potential: null atom arrays");
    return atom_field(grid, nat, tau, Z, rc, 0, d_Vloc, ws);
}

extern "C" dpp_status dpp_start_density(dpp_grid grid, int nat, const double* tau, const double* Z, double sigma,
                                        double* d_n, void* ws) {
    clear_error();
    DPP_REQUIRE(grid && d_n && ws && nat >= 0 && sigma > 0, "dpp_start_density: bad arguments");
    DPP_REQUIRE(nat == 0 || (tau && Z), "dpp_start_density: null atom arrays");
    std::vector<double> w(nat, sigma);
    return atom_field(grid, nat, tau, Z, w.data(), 1, d_n, ws);
}
