// LinearPCM: the dielectric Poisson solve and the electrostatic solvation
// energy (Sec. 2.1, Eqs. (1)-(2), Listing 1).
//
//   hessian(x) = (-1/(4 pi)) div(J(eps * I(grad x))),  solve hessian(phi~) = rho~
//   A_diel     = (1/2) dot(phi~ - coulomb(rho~), O rho~)
//
// Reciprocal fields live on the full box in natural order (FP64 complex).
// grad x -> i G' x and div v -> sum_d i G'_d v_d with G' = B m', m' the signed
// frequency with the Nyquist index of an even axis counted as 0, so the
// gradient of a real field is real; modes with G' = 0 (G = 0, pure Nyquist)
// are outside the solve.  CG is preconditioned by the vacuum inverse
// M = 4 pi / |G'|^2 and starts from phi~ = 0.
//
// One operator application = 4 full-box transforms: the three gradient
// components go back to real space packed as two complex fields
// (u0 + i u1, u2), are multiplied by eps there, come forward packed the same
// way, and the divergence kernel separates the packed components by
// Hermitian symmetry (J of a real field w: W(G) = conj(W(-G))).  Every
// reduction is a fixed-order two-level sum, so a solve is bitwise
// reproducible.
#include <hip/hip_runtime.h>

#include <cmath>

#include "internal.h"

namespace dpp {
namespace {

constexpr int PCM_BLOCKS = 1024;  // partial sums per reduction
constexpr int PCM_THREADS = 256;

struct PcmGeom {
    int S0, S1, S2;
    double B[9];
};

// signed frequency with the Nyquist index of an even axis -> 0 (spectral
// derivative), and the plain signed frequency
__device__ __forceinline__ void pcm_freq(int i, int S, int& m, int& mp) {
    m = 2 * i < S ? i : i - S;
    mp = (S % 2 == 0 && 2 * i == S) ? 0 : m;
}

__device__ __forceinline__ void pcm_index(const PcmGeom& g, int64_t idx, int& i0, int& i1, int& i2) {
    i2 = (int)(idx % g.S2);
    const int64_t q = idx / g.S2;
    i1 = (int)(q % g.S1);
    i0 = (int)(q / g.S1);
}

// G' (spectral) and |G|^2 (plain) of a box index
__device__ __forceinline__ void pcm_G(const PcmGeom& g, int i0, int i1, int i2, double Gp[3], double& G2) {
    int m0, m1, m2, p0, p1, p2;
    pcm_freq(i0, g.S0, m0, p0);
    pcm_freq(i1, g.S1, m1, p1);
    pcm_freq(i2, g.S2, m2, p2);
    double G[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        Gp[d] = g.B[3 * d] * p0 + g.B[3 * d + 1] * p1 + g.B[3 * d + 2] * p2;
        G[d] = g.B[3 * d] * m0 + g.B[3 * d + 1] * m1 + g.B[3 * d + 2] * m2;
    }
    G2 = G[0] * G[0] + G[1] * G[1] + G[2] * G[2];
}

// block sum of v into part[blockIdx.x] (fixed order)
__device__ __forceinline__ void pcm_block_sum(double v, double* part) {
    __shared__ double red[PCM_THREADS];
    red[threadIdx.x] = v;
    __syncthreads();
    for (int w = PCM_THREADS / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// out[k] = sum of nparts partials of series k (one block per series)
__global__ void __launch_bounds__(PCM_THREADS) k_pcm_reduce(const double* __restrict__ part, int nparts,
                                                            double* __restrict__ out) {
    __shared__ double red[PCM_THREADS];
    const double* p = part + (int64_t)blockIdx.x * nparts;
    double s = 0.0;
    for (int i = threadIdx.x; i < nparts; i += PCM_THREADS) s += p[i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = PCM_THREADS / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[blockIdx.x] = red[0];
}

// b = J rho on the solved modes (in place), r = b, x = 0, p = M r;
// partials: |b|^2 and r . M r
__global__ void __launch_bounds__(PCM_THREADS)
k_pcm_init(PcmGeom g, int64_t N, double2* __restrict__ b, double2* __restrict__ r, double2* __restrict__ x,
           double2* __restrict__ p, double* __restrict__ part) {
    double bb = 0.0, rz = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * PCM_THREADS + threadIdx.x; i < N; i += (int64_t)gridDim.x * PCM_THREADS) {
        int i0, i1, i2;
        pcm_index(g, i, i0, i1, i2);
        double Gp[3], G2;
        pcm_G(g, i0, i1, i2, Gp, G2);
        const double G2p = Gp[0] * Gp[0] + Gp[1] * Gp[1] + Gp[2] * Gp[2];
        double2 v = b[i];
        if (!(G2p > 0.0)) v = double2{0.0, 0.0};
        const double M = G2p > 0.0 ? 4.0 * M_PI / G2p : 0.0;
        b[i] = v;
        r[i] = v;
        x[i] = double2{0.0, 0.0};
        p[i] = double2{M * v.x, M * v.y};
        bb += v.x * v.x + v.y * v.y;
        rz += M * (v.x * v.x + v.y * v.y);
    }
    pcm_block_sum(bb, part);
    __syncthreads();
    pcm_block_sum(rz, part + gridDim.x);
}

// U[0] = i G'_0 p + i (i G'_1 p), U[1] = i G'_2 p (packed gradient components)
__global__ void __launch_bounds__(PCM_THREADS)
k_pcm_grad(PcmGeom g, int64_t N, const double2* __restrict__ p, double2* __restrict__ U) {
    for (int64_t i = (int64_t)blockIdx.x * PCM_THREADS + threadIdx.x; i < N; i += (int64_t)gridDim.x * PCM_THREADS) {
        int i0, i1, i2;
        pcm_index(g, i, i0, i1, i2);
        double Gp[3], G2;
        pcm_G(g, i0, i1, i2, Gp, G2);
        const double2 v = p[i];
        // i G0 v = (-G0 v.y, G0 v.x); i * (i G1 v) = -G1 v
        U[i] = double2{-Gp[0] * v.y - Gp[1] * v.x, Gp[0] * v.x - Gp[1] * v.y};
        U[N + i] = double2{-Gp[2] * v.y, Gp[2] * v.x};
    }
}

// real-space packed fields times eps (both parts are real fields)
__global__ void __launch_bounds__(PCM_THREADS)
k_pcm_eps(int64_t N, const double* __restrict__ eps, double2* __restrict__ U) {
    for (int64_t i = (int64_t)blockIdx.x * PCM_THREADS + threadIdx.x; i < N; i += (int64_t)gridDim.x * PCM_THREADS) {
        const double e = eps[i];
        const double2 a = U[i], c = U[N + i];
        U[i] = double2{e * a.x, e * a.y};
        U[N + i] = double2{e * c.x, e * c.y};
    }
}

// q = (-1/(4 pi)) sum_d i G'_d W_d on the solved modes, W_0, W_1 separated
// from Y[0] = J(w0 + i w1) and W_2 from Y[1] = J(w2) by Hermitian symmetry;
// partial p . q
__global__ void __launch_bounds__(PCM_THREADS)
k_pcm_div(PcmGeom g, int64_t N, const double2* __restrict__ Y, const double2* __restrict__ p,
          double2* __restrict__ q, double* __restrict__ part) {
    double pq = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * PCM_THREADS + threadIdx.x; i < N; i += (int64_t)gridDim.x * PCM_THREADS) {
        int i0, i1, i2;
        pcm_index(g, i, i0, i1, i2);
        double Gp[3], G2;
        pcm_G(g, i0, i1, i2, Gp, G2);
        const double G2p = Gp[0] * Gp[0] + Gp[1] * Gp[1] + Gp[2] * Gp[2];
        double2 out{0.0, 0.0};
        if (G2p > 0.0) {
            const int j0 = i0 ? g.S0 - i0 : 0, j1 = i1 ? g.S1 - i1 : 0, j2 = i2 ? g.S2 - i2 : 0;
            const int64_t im = ((int64_t)j0 * g.S1 + j1) * g.S2 + j2;
            const double2 a = Y[i], am = Y[im], c = Y[N + i], cm = Y[N + im];
            // W0 = (a + conj(am)) / 2, W1 = (a - conj(am)) / (2 i), W2 = (c + conj(cm)) / 2
            const double2 w0{0.5 * (a.x + am.x), 0.5 * (a.y - am.y)};
            const double2 w1{0.5 * (a.y + am.y), -0.5 * (a.x - am.x)};
            const double2 w2{0.5 * (c.x + cm.x), 0.5 * (c.y - cm.y)};
            // sum_d i G'_d W_d
            const double sx = Gp[0] * w0.x + Gp[1] * w1.x + Gp[2] * w2.x;
            const double sy = Gp[0] * w0.y + Gp[1] * w1.y + Gp[2] * w2.y;
            const double k = -1.0 / (4.0 * M_PI);
            out = double2{-k * sy, k * sx};
        }
        q[i] = out;
        const double2 pv = p[i];
        pq += pv.x * out.x + pv.y * out.y;
    }
    pcm_block_sum(pq, part);
}

// alpha = rz / pq; x += alpha p; r -= alpha q; partials |r|^2 and r . M r
__global__ void __launch_bounds__(PCM_THREADS)
k_pcm_update(PcmGeom g, int64_t N, const double* __restrict__ sc, double2* __restrict__ x, double2* __restrict__ r,
             const double2* __restrict__ p, const double2* __restrict__ q, double* __restrict__ part) {
    const double alpha = sc[0] / sc[1];
    double rr = 0.0, rz = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * PCM_THREADS + threadIdx.x; i < N; i += (int64_t)gridDim.x * PCM_THREADS) {
        int i0, i1, i2;
        pcm_index(g, i, i0, i1, i2);
        double Gp[3], G2;
        pcm_G(g, i0, i1, i2, Gp, G2);
        const double G2p = Gp[0] * Gp[0] + Gp[1] * Gp[1] + Gp[2] * Gp[2];
        const double M = G2p > 0.0 ? 4.0 * M_PI / G2p : 0.0;
        const double2 pv = p[i], qv = q[i];
        double2 xv = x[i], rv = r[i];
        xv = double2{xv.x + alpha * pv.x, xv.y + alpha * pv.y};
        rv = double2{rv.x - alpha * qv.x, rv.y - alpha * qv.y};
        x[i] = xv;
        r[i] = rv;
        rr += rv.x * rv.x + rv.y * rv.y;
        rz += M * (rv.x * rv.x + rv.y * rv.y);
    }
    pcm_block_sum(rr, part);
    __syncthreads();
    pcm_block_sum(rz, part + gridDim.x);
}

// p = M r + beta p, beta = rz_new / rz_old
__global__ void __launch_bounds__(PCM_THREADS)
k_pcm_dir(PcmGeom g, int64_t N, const double* __restrict__ sc_old, const double* __restrict__ sc_new,
          const double2* __restrict__ r, double2* __restrict__ p) {
    const double beta = sc_new[0] / sc_old[0];
    for (int64_t i = (int64_t)blockIdx.x * PCM_THREADS + threadIdx.x; i < N; i += (int64_t)gridDim.x * PCM_THREADS) {
        int i0, i1, i2;
        pcm_index(g, i, i0, i1, i2);
        double Gp[3], G2;
        pcm_G(g, i0, i1, i2, Gp, G2);
        const double G2p = Gp[0] * Gp[0] + Gp[1] * Gp[1] + Gp[2] * Gp[2];
        const double M = G2p > 0.0 ? 4.0 * M_PI / G2p : 0.0;
        const double2 rv = r[i], pv = p[i];
        p[i] = double2{M * rv.x + beta * pv.x, M * rv.y + beta * pv.y};
    }
}

// partial of Re sum_G conj(x - K b) b over the solved modes (K = 4 pi / |G|^2)
__global__ void __launch_bounds__(PCM_THREADS)
k_pcm_adiel(PcmGeom g, int64_t N, const double2* __restrict__ x, const double2* __restrict__ b,
            double* __restrict__ part) {
    double s = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * PCM_THREADS + threadIdx.x; i < N; i += (int64_t)gridDim.x * PCM_THREADS) {
        int i0, i1, i2;
        pcm_index(g, i, i0, i1, i2);
        double Gp[3], G2;
        pcm_G(g, i0, i1, i2, Gp, G2);
        const double G2p = Gp[0] * Gp[0] + Gp[1] * Gp[1] + Gp[2] * Gp[2];
        if (G2p > 0.0 && G2 > 0.0) {
            const double K = 4.0 * M_PI / G2;
            const double2 xv = x[i], bv = b[i];
            s += (xv.x - K * bv.x) * bv.x + (xv.y - K * bv.y) * bv.y;
        }
    }
    pcm_block_sum(s, part);
}

struct PcmWs {
    double2 *T, *x, *r, *p, *q, *U, *b;
    double *part, *sc;
};

size_t pcm_ws_bytes(int64_t N) { return (size_t)N * 16 * 9 + (size_t)PCM_BLOCKS * 2 * 8 + 64 * 8 + 256; }

PcmWs pcm_layout(void* ws, int64_t N) {
    PcmWs w;
    double2* c = reinterpret_cast<double2*>(ws);
    w.T = c;  // two plane buffers
    w.x = c + 2 * N;
    w.r = c + 3 * N;
    w.p = c + 4 * N;
    w.q = c + 5 * N;
    w.U = c + 6 * N;  // two fields
    w.b = c + 8 * N;
    w.part = reinterpret_cast<double*>(c + 9 * N);
    w.sc = w.part + PCM_BLOCKS * 2;
    return w;
}

}  // namespace
}  // namespace dpp

using namespace dpp;

extern "C" dpp_status dpp_pcm_workspace_size(dpp_grid grid, size_t* bytes) {
    clear_error();
    DPP_REQUIRE(grid && bytes, "dpp_pcm_workspace_size: null argument");
    *bytes = pcm_ws_bytes(grid->N);
    return DPP_OK;
}

extern "C" dpp_status dpp_pcm_solve(dpp_grid grid, const double* d_eps, const double* d_rho, double tol,
                                    int max_iter, double* d_phi, double* A_diel, int* iterations,
                                    double* rel_residual, void* ws) {
    clear_error();
    DPP_REQUIRE(grid && d_eps && d_rho && ws && A_diel, "dpp_pcm_solve: null argument");
    DPP_REQUIRE(tol >= 0.0 && max_iter >= 0, "dpp_pcm_solve: bad tolerance or iteration limit");
    hipStream_t st = grid->ctx->stream;
    const int64_t N = grid->N;
    PcmGeom g{grid->S[0], grid->S[1], grid->S[2], {}};
    for (int i = 0; i < 9; ++i) g.B[i] = grid->B[i];
    PcmWs w = pcm_layout(ws, N);
    const dim3 gb(PCM_BLOCKS), tb(PCM_THREADS);
    // slots of the scalar array: 0 rz, 1 pq, 2 rr, 3 rz_new, 4 bb, 5 A
    double* sc = w.sc;
    DPP_TRY(full_forward_real(grid, d_rho, w.b, w.T));
    hipLaunchKernelGGL(k_pcm_init, gb, tb, 0, st, g, N, w.b, w.r, w.x, w.p, w.part);
    DPP_LAUNCHED();
    hipLaunchKernelGGL(k_pcm_reduce, dim3(2), tb, 0, st, (const double*)w.part, PCM_BLOCKS, sc + 4);
    DPP_LAUNCHED();
    // sc[4] = |b|^2, sc[5] = r.Mr -> move r.Mr to slot 0
    DPP_HIP(hipMemcpyAsync(sc, sc + 5, sizeof(double), hipMemcpyDeviceToDevice, st));
    // the per-iteration readback goes through pinned memory (a pageable
    // destination is staged by the host runtime on every copy)
    if (!grid->h_pin) DPP_HIP(hipHostMalloc((void**)&grid->h_pin, 8 * sizeof(double), hipHostMallocDefault));
    double* host = grid->h_pin;
    host[0] = 0.0;
    DPP_HIP(hipMemcpyAsync(host, sc + 4, sizeof(double), hipMemcpyDeviceToHost, st));
    DPP_HIP(hipStreamSynchronize(st));
    const double bn = std::sqrt(host[0]);
    double rel = bn > 0.0 ? 1.0 : 0.0;
    int it = 0;
    while (it < max_iter && rel > tol) {
        // q = hessian(p)
        hipLaunchKernelGGL(k_pcm_grad, gb, tb, 0, st, g, N, (const double2*)w.p, w.U);
        DPP_LAUNCHED();
        DPP_TRY(full_complex(grid, 2, w.U, w.U, +1, 1.0, w.T));
        hipLaunchKernelGGL(k_pcm_eps, gb, tb, 0, st, N, d_eps, w.U);
        DPP_LAUNCHED();
        DPP_TRY(full_complex(grid, 2, w.U, w.U, -1, 1.0 / (double)N, w.T));
        hipLaunchKernelGGL(k_pcm_div, gb, tb, 0, st, g, N, (const double2*)w.U, (const double2*)w.p, w.q, w.part);
        DPP_LAUNCHED();
        hipLaunchKernelGGL(k_pcm_reduce, dim3(1), tb, 0, st, (const double*)w.part, PCM_BLOCKS, sc + 1);
        DPP_LAUNCHED();
        hipLaunchKernelGGL(k_pcm_update, gb, tb, 0, st, g, N, (const double*)sc, w.x, w.r, (const double2*)w.p,
                           (const double2*)w.q, w.part);
        DPP_LAUNCHED();
        hipLaunchKernelGGL(k_pcm_reduce, dim3(2), tb, 0, st, (const double*)w.part, PCM_BLOCKS, sc + 2);
        DPP_LAUNCHED();
        DPP_HIP(hipMemcpyAsync(host, sc + 2, sizeof(double), hipMemcpyDeviceToHost, st));
        DPP_HIP(hipStreamSynchronize(st));
        ++it;
        rel = std::sqrt(host[0]) / bn;
        if (rel <= tol) break;
        hipLaunchKernelGGL(k_pcm_dir, gb, tb, 0, st, g, N, (const double*)sc, (const double*)(sc + 3),
                           (const double2*)w.r, w.p);
        DPP_LAUNCHED();
        DPP_HIP(hipMemcpyAsync(sc, sc + 3, sizeof(double), hipMemcpyDeviceToDevice, st));
    }
    hipLaunchKernelGGL(k_pcm_adiel, gb, tb, 0, st, g, N, (const double2*)w.x, (const double2*)w.b, w.part);
    DPP_LAUNCHED();
    hipLaunchKernelGGL(k_pcm_reduce, dim3(1), tb, 0, st, (const double*)w.part, PCM_BLOCKS, sc + 5);
    DPP_LAUNCHED();
    if (d_phi) DPP_TRY(full_inverse_real(grid, w.x, d_phi, w.T));
    DPP_HIP(hipMemcpyAsync(host, sc + 5, sizeof(double), hipMemcpyDeviceToHost, st));
    DPP_HIP(hipStreamSynchronize(st));
    *A_diel = 0.5 * grid->omega * host[0];
    if (iterations) *iterations = it;
    if (rel_residual) *rel_residual = rel;
    return DPP_OK;
}
