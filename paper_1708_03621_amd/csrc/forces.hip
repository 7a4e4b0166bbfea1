// Forces on the ions (Table 1: ionic optimization; Sec. 3: the ionic
// minimization of the example), as position derivatives of this model's
// energy terms:
//   local     E_loc = Omega Re sum_G conj(n~(G)) sum_a v_a(G) exp(-i G.tau_a),
//             v_a(G) = -4 pi Z_a exp(-G^2 rc_a^2 / 4) / (Omega G^2), G != 0;
//             F_a = -Omega sum_G G v_a(G) Im[conj(n~(G)) exp(-i G.tau_a)]
//   nonlocal  E_nl = sum_k w_k sum_i f_ki D sum_a |Pi_ai|^2, Pi = P^dag psi;
//             dP[G,a]/dtau_a = -i G P[G,a];
//             F_a = -sum_k w_k sum_i f_ki D 2 Re[conj(Pi_ai) (dP_a^dag psi)_i]
//   ions      Ewald sums of point charges in a compensating background
//             (real-space erfc sum over images, reciprocal Gaussian sum).
// Phases exp(-i G.tau) = exp(-2 pi i m.s) use the fractional coordinates
// s = R^{-1} tau, with m.s reduced modulo 1 before sincospi.  Every sum is
// reduced in a fixed order.
#include <hip/hip_runtime.h>

#include <cmath>

#include "internal.h"

namespace dpp {

namespace {

struct Mat3 {
    double m[9];  // row-major
};

__device__ __forceinline__ int box_freq(int i, int S) { return 2 * i < S ? i : i - S; }

// Fixed-order sum of NV values over a 256-thread block; thread 0 gets them.
template <int NV>
__device__ __forceinline__ void block_sum256(double (&v)[NV], double (*red)[256]) {
#pragma unroll
    for (int q = 0; q < NV; ++q) red[q][threadIdx.x] = v[q];
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
#pragma unroll
            for (int q = 0; q < NV; ++q) red[q][threadIdx.x] += red[q][threadIdx.x + w];
        __syncthreads();
    }
#pragma unroll
    for (int q = 0; q < NV; ++q) v[q] = red[q][0];
}

// ----------------------------------------------------------- local ---------
// Workgroup (chunk, atom): the atom's force over `chunk` box points.
__global__ void __launch_bounds__(256)
k_force_local(const double2* __restrict__ nt, int S0, int S1, int S2, Mat3 B, double omega, int nchunk,
              int64_t chunk, const double* __restrict__ sfrac, const double* __restrict__ Z,
              const double* __restrict__ rc, double* __restrict__ part) {
    __shared__ double red[3][256];
    const int a = blockIdx.y, c = blockIdx.x;
    const int64_t N = (int64_t)S0 * S1 * S2;
    const int64_t j0 = (int64_t)c * chunk, j1 = j0 + chunk < N ? j0 + chunk : N;
    const double s0 = sfrac[3 * a], s1 = sfrac[3 * a + 1], s2 = sfrac[3 * a + 2];
    const double za = Z[a], r2 = 0.25 * rc[a] * rc[a];
    double f[3] = {0.0, 0.0, 0.0};
    for (int64_t j = j0 + threadIdx.x; j < j1; j += 256) {
        const int i2 = (int)(j % S2);
        const int64_t t = j / S2;
        const int i1 = (int)(t % S1), i0 = (int)(t / S1);
        const int m0 = box_freq(i0, S0), m1 = box_freq(i1, S1), m2 = box_freq(i2, S2);
        const double gx = B.m[0] * m0 + B.m[1] * m1 + B.m[2] * m2;
        const double gy = B.m[3] * m0 + B.m[4] * m1 + B.m[5] * m2;
        const double gz = B.m[6] * m0 + B.m[7] * m1 + B.m[8] * m2;
        const double G2 = gx * gx + gy * gy + gz * gz;
        if (G2 == 0.0) continue;
        const double v = -4.0 * M_PI * za * exp(-G2 * r2) / (omega * G2);
        double x = m0 * s0 + m1 * s1 + m2 * s2;
        x -= floor(x);
        double sn, cs;
        sincospi(2.0 * x, &sn, &cs);
        const double2 n = nt[j];
        // Im[conj(n) exp(-i theta)] = -(n_re sin theta + n_im cos theta)
        const double w = omega * v * (n.x * sn + n.y * cs);
        f[0] += w * gx;
        f[1] += w * gy;
        f[2] += w * gz;
    }
    block_sum256<3>(f, red);
    if (threadIdx.x == 0)
        for (int d = 0; d < 3; ++d) part[((int64_t)a * nchunk + c) * 3 + d] = f[d];
}

__global__ void k_force_chunks_sum(int nat, int nchunk, const double* __restrict__ part, double* __restrict__ F) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= nat * 3) return;
    const int a = e / 3, d = e - 3 * a;
    double s = 0.0;
    for (int c = 0; c < nchunk; ++c) s += part[((int64_t)a * nchunk + c) * 3 + d];
    F[e] = s;
}

// -------------------------------------------------------- nonlocal ---------
__global__ void k_projector_derivatives(int npw, int nproj, const int4* __restrict__ miller, Mat3 B,
                                        const double2* __restrict__ P, double2* __restrict__ Q) {
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    const int a = blockIdx.y;
    if (g >= npw) return;
    const int4 n = miller[g];
    const double G[3] = {B.m[0] * n.x + B.m[1] * n.y + B.m[2] * n.z, B.m[3] * n.x + B.m[4] * n.y + B.m[5] * n.z,
                         B.m[6] * n.x + B.m[7] * n.y + B.m[8] * n.z};
    const double2 p = P[(int64_t)a * npw + g];
    for (int d = 0; d < 3; ++d)  // -i G_d p
        Q[((int64_t)d * nproj + a) * npw + g] = double2{G[d] * p.y, -G[d] * p.x};
}

// One wave per projector: out[p * 3 + d] = -w D sum_i f_i 2 Re[conj(Pi_pi) Pid_d,pi].
__global__ void __launch_bounds__(64)
k_force_nonlocal(int nproj, int nb, double w, double D, const double* __restrict__ f, const double2* __restrict__ Pi,
                 const double2* __restrict__ Pid, double* __restrict__ out) {
    const int p = blockIdx.x, lane = threadIdx.x;
    double acc[3] = {0.0, 0.0, 0.0};
    for (int i = lane; i < nb; i += 64) {
        const double fi = f[i];
        const double2 a = Pi[(int64_t)p * nb + i];
        for (int d = 0; d < 3; ++d) {
            const double2 b = Pid[((int64_t)d * nproj + p) * nb + i];
            acc[d] += fi * 2.0 * (a.x * b.x + a.y * b.y);
        }
    }
    for (int d = 0; d < 3; ++d) {
        double v = acc[d];
        for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);  // same tree on every lane
        if (lane == 0) out[p * 3 + d] = -w * D * v;
    }
}

// ----------------------------------------------------------- Ewald ---------
// Workgroup per atom a: real-space sum over (b, image) pairs, then
// part[a * 4 + {x, y, z, E}].
__global__ void __launch_bounds__(256)
k_ewald_real(EwaldSetup e, int nat, const double* __restrict__ tau, const double* __restrict__ Z,
             double* __restrict__ part) {
    __shared__ double red[4][256];
    const int a = blockIdx.x;
    const int n0 = 2 * e.nr[0] + 1, n1 = 2 * e.nr[1] + 1, n2 = 2 * e.nr[2] + 1;
    const int64_t total = (int64_t)nat * n0 * n1 * n2;
    const double ta[3] = {tau[3 * a], tau[3 * a + 1], tau[3 * a + 2]};
    double v[4] = {0.0, 0.0, 0.0, 0.0};
    const double two_eta_sqrtpi = 2.0 * e.eta / sqrt(M_PI);
    for (int64_t q = threadIdx.x; q < total; q += 256) {
        const int b = (int)(q % nat);
        int64_t t = q / nat;
        const int l2 = (int)(t % n2) - e.nr[2];
        t /= n2;
        const int l1 = (int)(t % n1) - e.nr[1];
        const int l0 = (int)(t / n1) - e.nr[0];
        if (b == a && l0 == 0 && l1 == 0 && l2 == 0) continue;
        double d[3];
        for (int r = 0; r < 3; ++r)
            d[r] = ta[r] - tau[3 * b + r] + e.R[3 * r] * l0 + e.R[3 * r + 1] * l1 + e.R[3 * r + 2] * l2;
        const double rr = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
        if (rr > e.rcut) continue;
        const double zz = Z[a] * Z[b];
        const double ec = erfc(e.eta * rr);
        v[3] += 0.5 * zz * ec / rr;
        const double g = (ec / rr + two_eta_sqrtpi * exp(-e.eta * e.eta * rr * rr)) / (rr * rr);
        for (int r = 0; r < 3; ++r) v[r] += zz * g * d[r];
    }
    block_sum256<4>(v, red);
    if (threadIdx.x == 0)
        for (int r = 0; r < 4; ++r) part[a * 4 + r] = v[r];
}

// Workgroup per atom a: reciprocal sum over G = B m (0 < |G| <= gcut) with the
// structure factor S(G) = sum_b Z_b exp(i G.tau_b); atom a's share of the
// energy is (2 pi/Omega) w Re[conj(S) Z_a exp(i G.tau_a)] (the shares add up
// to the whole term).
__global__ void __launch_bounds__(256)
k_ewald_recip(EwaldSetup e, int nat, const double* __restrict__ sfrac, const double* __restrict__ Z,
              double* __restrict__ part) {
    __shared__ double red[4][256];
    const int a = blockIdx.x;
    const int n0 = 2 * e.ng[0] + 1, n1 = 2 * e.ng[1] + 1, n2 = 2 * e.ng[2] + 1;
    const int64_t total = (int64_t)n0 * n1 * n2;
    const double inv4e2 = 1.0 / (4.0 * e.eta * e.eta);
    double v[4] = {0.0, 0.0, 0.0, 0.0};
    for (int64_t q = threadIdx.x; q < total; q += 256) {
        const int m2 = (int)(q % n2) - e.ng[2];
        const int64_t t = q / n2;
        const int m1 = (int)(t % n1) - e.ng[1];
        const int m0 = (int)(t / n1) - e.ng[0];
        const double G[3] = {e.B[0] * m0 + e.B[1] * m1 + e.B[2] * m2, e.B[3] * m0 + e.B[4] * m1 + e.B[5] * m2,
                             e.B[6] * m0 + e.B[7] * m1 + e.B[8] * m2};
        const double G2 = G[0] * G[0] + G[1] * G[1] + G[2] * G[2];
        if (G2 == 0.0 || G2 > e.gcut * e.gcut) continue;
        const double w = exp(-G2 * inv4e2) / G2;
        double Sr = 0.0, Si = 0.0, ar = 0.0, ai = 0.0;
        for (int b = 0; b < nat; ++b) {
            double x = m0 * sfrac[3 * b] + m1 * sfrac[3 * b + 1] + m2 * sfrac[3 * b + 2];
            x -= floor(x);
            double sn, cs;
            sincospi(2.0 * x, &sn, &cs);  // exp(i G.tau_b) = cs + i sn
            Sr += Z[b] * cs;
            Si += Z[b] * sn;
            if (b == a) ar = cs, ai = sn;
        }
        // exp(i G.tau_a) conj(S) = (ar + i ai)(Sr - i Si)
        const double pr = ar * Sr + ai * Si, pi = ai * Sr - ar * Si;
        const double fz = 4.0 * M_PI / e.omega * Z[a] * w * pi;
        for (int r = 0; r < 3; ++r) v[r] += fz * G[r];
        v[3] += 2.0 * M_PI / e.omega * w * Z[a] * pr;
    }
    block_sum256<4>(v, red);
    if (threadIdx.x == 0)
        for (int r = 0; r < 4; ++r) part[(nat + a) * 4 + r] = v[r];
}

__global__ void k_ewald_total(int nat, const double* __restrict__ part, double* __restrict__ F,
                              double* __restrict__ E) {
    const int e = threadIdx.x;
    for (int q = e; q < nat * 3; q += blockDim.x) {
        const int a = q / 3, d = q - 3 * a;
        F[q] = part[a * 4 + d] + part[(nat + a) * 4 + d];
    }
    if (e == 0) {
        double s = 0.0;
        for (int a = 0; a < nat; ++a) s += part[a * 4 + 3];
        for (int a = 0; a < nat; ++a) s += part[(nat + a) * 4 + 3];
        *E = s;
    }
}

Mat3 mat3(const double* m) {
    Mat3 r;
    for (int i = 0; i < 9; ++i) r.m[i] = m[i];
    return r;
}

}  // namespace

dpp_status forces_local(dpp_ctx_s* ctx, const dpp_grid_s* g, const double2* nt, int nat, const double* d_sfrac,
                        const double* d_Z, const double* d_rc, double* part, double* F) {
    if (nat == 0) return DPP_OK;
    const int64_t N = g->N;
    const int64_t chunk = std::max<int64_t>(4096, (N + LF_CHUNKS_MAX - 1) / LF_CHUNKS_MAX);
    const int nchunk = (int)((N + chunk - 1) / chunk);
    TimerScope ts_(ctx, DPP_TK_FIELDS);
    hipLaunchKernelGGL(k_force_local, dim3(nchunk, nat), dim3(256), 0, ctx->stream, nt, g->S[0], g->S[1], g->S[2],
                       mat3(g->B), g->omega, nchunk, chunk, d_sfrac, d_Z, d_rc, part);
    DPP_LAUNCHED();
    hipLaunchKernelGGL(k_force_chunks_sum, dim3((nat * 3 + 255) / 256), dim3(256), 0, ctx->stream, nat, nchunk,
                       (const double*)part, F);
    DPP_LAUNCHED();
    return DPP_OK;
}

dpp_status projector_derivatives(dpp_ctx_s* ctx, const dpp_basis_s* b, int nproj, const double2* P, double2* Q) {
    if (nproj == 0 || b->npw == 0) return DPP_OK;
    hipLaunchKernelGGL(k_projector_derivatives, dim3((unsigned)((b->npw + 255) / 256), nproj), dim3(256), 0,
                       ctx->stream, (int)b->npw, nproj, (const int4*)b->d_miller, mat3(b->grid->B), P, Q);
    DPP_LAUNCHED();
    return DPP_OK;
}

dpp_status forces_nonlocal_item(dpp_ctx_s* ctx, int nproj, int nb, double w, double D, const double* f,
                                const double2* Pi, const double2* Pid, double* out) {
    if (nproj == 0) return DPP_OK;
    hipLaunchKernelGGL(k_force_nonlocal, dim3(nproj), dim3(64), 0, ctx->stream, nproj, nb, w, D, f, Pi, Pid, out);
    DPP_LAUNCHED();
    return DPP_OK;
}

dpp_status ewald_sums(dpp_ctx_s* ctx, const EwaldSetup& e, int nat, const double* d_tau, const double* d_sfrac,
                      const double* d_Z, double* part, double* F, double* E) {
    if (nat == 0) return DPP_OK;
    TimerScope ts_(ctx, DPP_TK_FIELDS);
    hipLaunchKernelGGL(k_ewald_real, dim3(nat), dim3(256), 0, ctx->stream, e, nat, d_tau, d_Z, part);
    DPP_LAUNCHED();
    hipLaunchKernelGGL(k_ewald_recip, dim3(nat), dim3(256), 0, ctx->stream, e, nat, d_sfrac, d_Z, part);
    DPP_LAUNCHED();
    hipLaunchKernelGGL(k_ewald_total, dim3(1), dim3(256), 0, ctx->stream, nat, (const double*)part, F, E);
    DPP_LAUNCHED();
    return DPP_OK;
}

}  // namespace dpp
