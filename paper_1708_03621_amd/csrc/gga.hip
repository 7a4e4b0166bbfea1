// GGA exchange-correlation: PBE, spin-unpolarized (Table 1 and Sec. 2.2
// list semilocal functionals), on a full grid in FP64.
//
//   e(n, sigma) = n eps_x^LDA F_x(s) + n (eps_c^PW92(r_s) + H(r_s, t)),
//   sigma = |grad n|^2,  v_xc = de/dn - div(2 de/dsigma grad n),
//   E_xc = (Omega/N) sum_r e.
// F_x = 1 + kappa - kappa / (1 + mu s^2 / kappa), s^2 = sigma / (4 k_F^2 n^2);
// H = gamma ln(1 + (beta/gamma) t^2 (1 + A t^2) / (1 + A t^2 + A^2 t^4)),
// A = (beta/gamma) / (exp(-eps_c / gamma) - 1), t^2 = sigma / (4 k_s^2 n^2);
// PW92 eps_c = -2 a (1 + alpha1 r_s) ln(1 + 1 / (2 a (b1 r_s^{1/2} + b2 r_s
// + b3 r_s^{3/2} + b4 r_s^2))).  Densities below 1e-16 give e = 0.
//
// grad and div are spectral (J, times i G', I), with G' = B m' and the
// Nyquist index of an even axis counted as 0, as in the LinearPCM solve.
// The three gradient components travel through the full-box transforms
// packed as two complex fields (g0 + i g1, g2); the pointwise kernel takes
// de/dn and de/dsigma with dual numbers (value and both partials carried
// through the same formula) and packs h = 2 de/dsigma grad n the same way
// for the divergence.  Six full-box transform launches per call.
#include <hip/hip_runtime.h>

#include <cmath>

#include "internal.h"

namespace dpp {
namespace {

constexpr int GGA_BLOCKS = 1024;
constexpr int GGA_THREADS = 256;
constexpr double GGA_NFLOOR = 1e-16;

// value with partial derivatives along n and sigma
struct Dn {
    double v, a, b;
};
__device__ __forceinline__ Dn operator+(Dn x, Dn y) { return {x.v + y.v, x.a + y.a, x.b + y.b}; }
__device__ __forceinline__ Dn operator-(Dn x, Dn y) { return {x.v - y.v, x.a - y.a, x.b - y.b}; }
__device__ __forceinline__ Dn operator*(Dn x, Dn y) { return {x.v * y.v, x.a * y.v + x.v * y.a, x.b * y.v + x.v * y.b}; }
__device__ __forceinline__ Dn operator/(Dn x, Dn y) {
    const double r = 1.0 / y.v, q = x.v * r;
    return {q, (x.a - q * y.a) * r, (x.b - q * y.b) * r};
}
__device__ __forceinline__ Dn operator+(double c, Dn x) { return {c + x.v, x.a, x.b}; }
__device__ __forceinline__ Dn operator*(double c, Dn x) { return {c * x.v, c * x.a, c * x.b}; }
__device__ __forceinline__ Dn dsqrt(Dn x) {
    const double s = sqrt(x.v), d = 0.5 / s;
    return {s, d * x.a, d * x.b};
}
__device__ __forceinline__ Dn dcbrt(Dn x) {
    const double c = cbrt(x.v), d = c / (3.0 * x.v);
    return {c, d * x.a, d * x.b};
}
__device__ __forceinline__ Dn dlog1p(Dn x) {
    const double d = 1.0 / (1.0 + x.v);
    return {log1p(x.v), d * x.a, d * x.b};
}
__device__ __forceinline__ Dn dexp(Dn x) {
    const double e = exp(x.v);
    return {e, e * x.a, e * x.b};
}

__device__ Dn pbe_energy_density(Dn n, Dn sigma) {
    constexpr double kappa = 0.804, beta = 0.06672455060314922;
    const double pi = M_PI;
    const double mu = beta * pi * pi / 3.0;
    const double gamma = (1.0 - M_LN2) / (pi * pi);
    constexpr double a = 0.031091, alpha1 = 0.21370, b1 = 7.5957, b2 = 3.5876, b3 = 1.6382, b4 = 0.49294;
    const Dn cn = dcbrt(n);                               // n^{1/3}
    const Dn kF = cbrt(3.0 * pi * pi) * cn;               // (3 pi^2 n)^{1/3}
    const Dn rs = Dn{cbrt(3.0 / (4.0 * pi)), 0, 0} / cn;  // (3 / (4 pi n))^{1/3}
    const Dn ks = dsqrt((4.0 / pi) * kF);
    const Dn exlda = (-0.75 * cbrt(3.0 / pi)) * cn;
    const Dn nn = n * n;
    const Dn s2 = sigma / ((4.0 * (kF * kF)) * nn);
    const Dn t2 = sigma / ((4.0 * (ks * ks)) * nn);
    const Dn fx = (1.0 + kappa) + (-kappa) * (Dn{1, 0, 0} / (1.0 + (mu / kappa) * s2));
    const Dn srs = dsqrt(rs);
    const Dn den = (2.0 * a) * (b1 * srs + b2 * rs + b3 * (rs * srs) + b4 * (rs * rs));
    const Dn ec = (-2.0 * a) * ((1.0 + alpha1 * rs) * dlog1p(Dn{1, 0, 0} / den));
    const Dn A = Dn{beta / gamma, 0, 0} / (-1.0 + dexp((-1.0 / gamma) * ec));
    const Dn At2 = A * t2;
    const Dn H = gamma * dlog1p((beta / gamma) * (t2 * (1.0 + At2) / (1.0 + At2 + At2 * At2)));
    return n * (exlda * fx) + n * (ec + H);
}

struct GgaGeom {
    int S0, S1, S2;
    double B[9];
};

__device__ __forceinline__ void gga_Gp(const GgaGeom& g, int64_t idx, double Gp[3]) {
    const int i2 = (int)(idx % g.S2);
    const int64_t q = idx / g.S2;
    const int i1 = (int)(q % g.S1), i0 = (int)(q / g.S1);
    int m[3];
    const int ii[3] = {i0, i1, i2}, SS[3] = {g.S0, g.S1, g.S2};
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const int mm = 2 * ii[d] < SS[d] ? ii[d] : ii[d] - SS[d];
        m[d] = (SS[d] % 2 == 0 && 2 * ii[d] == SS[d]) ? 0 : mm;
    }
#pragma unroll
    for (int d = 0; d < 3; ++d) Gp[d] = g.B[3 * d] * m[0] + g.B[3 * d + 1] * m[1] + g.B[3 * d + 2] * m[2];
}

// U[0] = i G'_0 nt + i (i G'_1 nt), U[1] = i G'_2 nt
__global__ void __launch_bounds__(GGA_THREADS)
k_gga_grad(GgaGeom g, int64_t N, const double2* __restrict__ nt, double2* __restrict__ U) {
    for (int64_t i = (int64_t)blockIdx.x * GGA_THREADS + threadIdx.x; i < N; i += (int64_t)gridDim.x * GGA_THREADS) {
        double Gp[3];
        gga_Gp(g, i, Gp);
        const double2 v = nt[i];
        U[i] = double2{-Gp[0] * v.y - Gp[1] * v.x, Gp[0] * v.x - Gp[1] * v.y};
        U[N + i] = double2{-Gp[2] * v.y, Gp[2] * v.x};
    }
}

// per point: e, de/dn -> v, and U <- packed h = 2 de/dsigma grad n; partial sums of e
__global__ void __launch_bounds__(GGA_THREADS)
k_gga_point(int64_t N, const double* __restrict__ n, double2* __restrict__ U, double* __restrict__ v,
            double* __restrict__ part) {
    double acc = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * GGA_THREADS + threadIdx.x; i < N; i += (int64_t)gridDim.x * GGA_THREADS) {
        const double2 u = U[i], w = U[N + i];
        const double g0 = u.x, g1 = u.y, g2 = w.x;
        const double nv = n[i];
        double e = 0.0, en = 0.0, es = 0.0;
        if (nv >= GGA_NFLOOR) {
            const Dn r = pbe_energy_density(Dn{nv, 1.0, 0.0}, Dn{g0 * g0 + g1 * g1 + g2 * g2, 0.0, 1.0});
            e = r.v;
            en = r.a;
            es = r.b;
        }
        acc += e;
        v[i] = en;
        const double h = 2.0 * es;
        U[i] = double2{h * g0, h * g1};
        U[N + i] = double2{h * g2, 0.0};
    }
    __shared__ double red[GGA_THREADS];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int s = GGA_THREADS / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// D = sum_d i G'_d H_d, with H_0, H_1 separated from Y[0] = J(h0 + i h1) and
// H_2 from Y[1] = J(h2) by Hermitian symmetry
__global__ void __launch_bounds__(GGA_THREADS)
k_gga_div(GgaGeom g, int64_t N, const double2* __restrict__ Y, double2* __restrict__ D) {
    for (int64_t i = (int64_t)blockIdx.x * GGA_THREADS + threadIdx.x; i < N; i += (int64_t)gridDim.x * GGA_THREADS) {
        double Gp[3];
        gga_Gp(g, i, Gp);
        const int i2 = (int)(i % g.S2);
        const int64_t q = i / g.S2;
        const int i1 = (int)(q % g.S1), i0 = (int)(q / g.S1);
        const int j0 = i0 ? g.S0 - i0 : 0, j1 = i1 ? g.S1 - i1 : 0, j2 = i2 ? g.S2 - i2 : 0;
        const int64_t im = ((int64_t)j0 * g.S1 + j1) * g.S2 + j2;
        const double2 a = Y[i], am = Y[im], c = Y[N + i], cm = Y[N + im];
        const double2 w0{0.5 * (a.x + am.x), 0.5 * (a.y - am.y)};
        const double2 w1{0.5 * (a.y + am.y), -0.5 * (a.x - am.x)};
        const double2 w2{0.5 * (c.x + cm.x), 0.5 * (c.y - cm.y)};
        const double sx = Gp[0] * w0.x + Gp[1] * w1.x + Gp[2] * w2.x;
        const double sy = Gp[0] * w0.y + Gp[1] * w1.y + Gp[2] * w2.y;
        D[i] = double2{-sy, sx};
    }
}

// v -= Re(div h)
__global__ void __launch_bounds__(GGA_THREADS)
k_gga_combine(int64_t N, const double2* __restrict__ Dr, double* __restrict__ v) {
    for (int64_t i = (int64_t)blockIdx.x * GGA_THREADS + threadIdx.x; i < N; i += (int64_t)gridDim.x * GGA_THREADS)
        v[i] -= Dr[i].x;
}

__global__ void __launch_bounds__(GGA_THREADS)
k_gga_energy(const double* __restrict__ part, int nparts, double scale, double* __restrict__ out) {
    __shared__ double red[GGA_THREADS];
    double s = 0.0;
    for (int i = threadIdx.x; i < nparts; i += GGA_THREADS) s += part[i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = GGA_THREADS / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = red[0] * scale;
}

size_t gga_ws_bytes(int64_t N) { return (size_t)N * 16 * 6 + (size_t)GGA_BLOCKS * 8 + 256; }

}  // namespace
}  // namespace dpp

using namespace dpp;

extern "C" dpp_status dpp_gga_workspace_size(dpp_grid grid, size_t* bytes) {
    clear_error();
    DPP_REQUIRE(grid && bytes, "dpp_gga_workspace_size: null argument");
    *bytes = gga_ws_bytes(grid->N);
    return DPP_OK;
}

extern "C" dpp_status dpp_gga_pbe(dpp_grid grid, const double* d_n, double* d_vxc, double* d_Exc, void* ws) {
    clear_error();
    DPP_REQUIRE(grid && d_n && d_vxc && d_Exc && ws, "dpp_gga_pbe: null argument");
    return gga_pbe(grid, d_n, d_vxc, d_Exc, ws);
}

dpp_status dpp::gga_pbe(dpp_grid_s* grid, const double* d_n, double* d_vxc, double* d_Exc, void* ws) {
    hipStream_t st = grid->ctx->stream;
    TimerScope ts_(grid->ctx, DPP_TK_FIELDS);
    const int64_t N = grid->N;
    GgaGeom g{grid->S[0], grid->S[1], grid->S[2], {}};
    for (int i = 0; i < 9; ++i) g.B[i] = grid->B[i];
    double2* c = reinterpret_cast<double2*>(ws);
    double2* T = c;          // two plane buffers
    double2* nt = c + 2 * N;
    double2* U = c + 3 * N;  // two packed fields
    double2* D = c + 5 * N;
    double* part = reinterpret_cast<double*>(c + 6 * N);
    const dim3 gb(GGA_BLOCKS), tb(GGA_THREADS);
    DPP_TRY(full_forward_real(grid, d_n, nt, T));
    hipLaunchKernelGGL(k_gga_grad, gb, tb, 0, st, g, N, (const double2*)nt, U);
    DPP_LAUNCHED();
    DPP_TRY(full_complex(grid, 2, U, U, +1, 1.0, T));
    hipLaunchKernelGGL(k_gga_point, gb, tb, 0, st, N, d_n, U, d_vxc, part);
    DPP_LAUNCHED();
    DPP_TRY(full_complex(grid, 2, U, U, -1, 1.0 / (double)N, T));
    hipLaunchKernelGGL(k_gga_div, gb, tb, 0, st, g, N, (const double2*)U, D);
    DPP_LAUNCHED();
    DPP_TRY(full_complex(grid, 1, D, D, +1, 1.0, T));
    hipLaunchKernelGGL(k_gga_combine, gb, tb, 0, st, N, (const double2*)D, d_vxc);
    DPP_LAUNCHED();
    hipLaunchKernelGGL(k_gga_energy, dim3(1), tb, 0, st, (const double*)part, GGA_BLOCKS,
                       grid->omega / (double)N, d_Exc);
    DPP_LAUNCHED();
    return DPP_OK;
}
