// Kernels on packed multi-k wavefunction blocks and on small nb x nb matrices,
// used by the minimization and SCF drivers.
//
// Packed layout: the blocks of all k-points of a system sit back to back,
// block k at element offset off[k] with nb bands of ld = npw[k] each.  A
// segment table gives each block's offset, npw and |k+G|^2 array.
#include <hip/hip_runtime.h>

#include "blockops.h"

namespace dpp {

// ------------------------------------------------------- elementwise -------

// out_k = a_k * x_k + b_k * y_k over every block (alpha arrays per k, device).
__global__ void k_seg_axpby(const Seg* __restrict__ seg, int nb, const double* __restrict__ a,
                            const double2* __restrict__ x, const double* __restrict__ b,
                            const double2* __restrict__ y, double2* __restrict__ out) {
    const int k = blockIdx.y;
    const Seg s = seg[k];
    const int64_t n = (int64_t)nb * s.npw;
    const double ak = a ? a[k] : 0.0, bk = b ? b[k] : 0.0;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t o = s.off + e;
        double2 r = double2{0, 0};
        if (x) {
            const double2 v = x[o];
            r.x = ak * v.x;
            r.y = ak * v.y;
        }
        if (y) {
            const double2 v = y[o];
            r.x += bk * v.x;
            r.y += bk * v.y;
        }
        out[o] = r;
    }
}

// out = scale * K x  (K = 1/(1 + |k+G|^2/2)), per block.
__global__ void k_seg_precond(const Seg* __restrict__ seg, int nb, double scale, const double2* __restrict__ x,
                              double2* __restrict__ out) {
    const int k = blockIdx.y;
    const Seg s = seg[k];
    const int64_t n = (int64_t)nb * s.npw;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
        const int q = (int)(e % s.npw);
        const double kk = scale / (1.0 + 0.5 * s.kG2[q]);
        const double2 v = x[s.off + e];
        out[s.off + e] = double2{kk * v.x, kk * v.y};
    }
}

// Per-block dots 2 Re sum conj(A) B for up to 4 pairs: partial sums per
// (pair, k, block) -> part[(pair * nk + k) * DOT_BLOCKS + blockIdx.x].
__global__ void __launch_bounds__(256)
k_seg_dots(const Seg* __restrict__ seg, int nk, int nb, int npair, DotPairs pr, double* __restrict__ part) {
    __shared__ double red[4][256];
    const int k = blockIdx.y;
    const Seg s = seg[k];
    const int64_t n = (int64_t)nb * s.npw;
    double acc[4] = {0, 0, 0, 0};
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < n; e += (int64_t)DOT_BLOCKS * 256) {
        const int64_t o = s.off + e;
#pragma unroll
        for (int p = 0; p < 4; ++p) {
            if (p < npair) {
                const double2 a = pr.a[p][o], b = pr.b[p][o];
                acc[p] += a.x * b.x + a.y * b.y;
            }
        }
    }
#pragma unroll
    for (int p = 0; p < 4; ++p) red[p][threadIdx.x] = acc[p];
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w)
            for (int p = 0; p < 4; ++p) red[p][threadIdx.x] += red[p][threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x < npair) part[((int64_t)threadIdx.x * nk + k) * DOT_BLOCKS + blockIdx.x] = 2.0 * red[threadIdx.x][0];
}

// Sum partials in fixed order: out[pair * (nk + 1) + k] per k, and the total
// over k at out[pair * (nk + 1) + nk].
__global__ void k_seg_dots_reduce(const double* __restrict__ part, int nk, int npair, double* __restrict__ out) {
    const int p = blockIdx.x;
    if (p >= npair) return;
    __shared__ double tot[64];
    for (int k = threadIdx.x; k < nk; k += blockDim.x) {
        double s = 0;
        for (int b = 0; b < DOT_BLOCKS; ++b) s += part[((int64_t)p * nk + k) * DOT_BLOCKS + b];
        out[p * (nk + 1) + k] = s;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = 0;
        for (int k = 0; k < nk; ++k) s += out[p * (nk + 1) + k];
        out[p * (nk + 1) + nk] = s;
    }
    (void)tot;
}

// Band-weighted kinetic sums: part[k * DOT_BLOCKS + block] of
// sum_i f[k*nb+i] * sum_G |k+G|^2 |psi_Gi|^2.
__global__ void __launch_bounds__(256)
k_seg_kinetic(const Seg* __restrict__ seg, int nb, int fstride, const double* __restrict__ f,
              const double2* __restrict__ psi, double* __restrict__ part) {
    __shared__ double red[256];
    const int k = blockIdx.y;
    const Seg s = seg[k];
    const int64_t n = (int64_t)nb * s.npw;
    double acc = 0;
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < n; e += (int64_t)DOT_BLOCKS * 256) {
        const int b = (int)(e / s.npw);
        const int q = (int)(e - (int64_t)b * s.npw);
        const double2 v = psi[s.off + e];
        acc += f[k * fstride + b] * s.kG2[q] * (v.x * v.x + v.y * v.y);
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[k * DOT_BLOCKS + blockIdx.x] = red[0];
}

// E = sum_k w_k * scale * sum_blocks part[k]  (fixed order), written to *out.
__global__ void k_seg_weighted_total(const double* __restrict__ part, int nk, const double* __restrict__ wk,
                                     double scale, double* __restrict__ out) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double tot = 0;
    for (int k = 0; k < nk; ++k) {
        double s = 0;
        for (int b = 0; b < DOT_BLOCKS; ++b) s += part[k * DOT_BLOCKS + b];
        tot += wk[k] * scale * s;
    }
    *out = tot;
}

// Nonlocal energy from Pi (nproj x nb per k, row-major, at pi + k * pi_stride):
// sum_k w_k D sum_i f_ki sum_a |Pi_ai|^2 -> *out (one thread, fixed order).
__global__ void k_nonlocal_energy(int nk, int nproj, int nb, int fstride, const double2* __restrict__ pi,
                                  int64_t pi_stride, const double* __restrict__ f, const double* __restrict__ wk,
                                  double D, double* __restrict__ out) {
    __shared__ double red[256];
    double tot = 0;
    for (int k = 0; k < nk; ++k) {
        double acc = 0;
        for (int e = threadIdx.x; e < nproj * nb; e += blockDim.x) {
            const int i = e % nb;
            const double2 v = pi[k * pi_stride + e];
            acc += f[k * fstride + i] * (v.x * v.x + v.y * v.y);
        }
        red[threadIdx.x] = acc;
        __syncthreads();
        for (int w = 128; w > 0; w >>= 1) {
            if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
            __syncthreads();
        }
        if (threadIdx.x == 0) tot += wk[k] * D * red[0];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = tot;
}

// ------------------------------------------------------- small matrices ----

// C_b = alpha * op(A_b) op(B_b) + beta * C_b for n x n complex row-major
// matrices, op = N or H (conjugate transpose); batch b = blockIdx.x with
// strides sa, sb, sc (elements).  alpha_arr (per batch, optional) multiplies alpha.
__global__ void k_smm(int n, int opA, int opB, double alpha, const double* __restrict__ alpha_arr,
                      const double2* __restrict__ A, int64_t sa, const double2* __restrict__ B, int64_t sb,
                      double beta, double2* __restrict__ Cm, int64_t sc) {
    const int b = blockIdx.x;
    const double2* Ab = A + b * sa;
    const double2* Bb = B + b * sb;
    double2* Cb = Cm + b * sc;
    const double al = alpha * (alpha_arr ? alpha_arr[b] : 1.0);
    for (int e = threadIdx.x; e < n * n; e += blockDim.x) {
        const int i = e / n, j = e - i * n;
        double sr = 0, si = 0;
        for (int t = 0; t < n; ++t) {
            double2 a = opA ? Ab[t * n + i] : Ab[i * n + t];
            if (opA) a.y = -a.y;
            double2 bb = opB ? Bb[j * n + t] : Bb[t * n + j];
            if (opB) bb.y = -bb.y;
            sr += a.x * bb.x - a.y * bb.y;
            si += a.x * bb.y + a.y * bb.x;
        }
        double2 r = double2{al * sr, al * si};
        if (beta != 0.0) {
            const double2 c = Cb[e];
            r.x += beta * c.x;
            r.y += beta * c.y;
        }
        Cb[e] = r;
    }
}

// out_b = scale * (scale_arr ? scale_arr[b] : 1) * op(A_b), op = N or H; n x n at stride st.
__global__ void k_sm_scale(int n, int64_t st, int op, double scale, const double* __restrict__ scale_arr,
                           const double2* __restrict__ A, double2* __restrict__ out) {
    const int b = blockIdx.x;
    const double sc = scale * (scale_arr ? scale_arr[b] : 1.0);
    for (int e = threadIdx.x; e < n * n; e += blockDim.x) {
        const int i = e / n, j = e - i * n;
        double2 a = op ? A[b * st + j * n + i] : A[b * st + e];
        if (op) a.y = -a.y;
        out[b * st + e] = double2{sc * a.x, sc * a.y};
    }
}

// out[b] = Re Tr(A_b) * scale.
__global__ void k_trace(int n, const double2* __restrict__ A, int64_t sa, double scale, double* __restrict__ out) {
    const int b = blockIdx.x;
    if (threadIdx.x == 0) {
        double s = 0;
        for (int i = 0; i < n; ++i) s += A[b * sa + i * n + i].x;
        out[b] = scale * s;
    }
}

// Trial matrices of a line search along D (batch b over k):
//   U(a) = U + a (X + X^dag) + a^2 Q,   H(a) = H0 + a (H1 + H1^dag) + a^2 H2
__global__ void k_trial_mats(int n, const double* __restrict__ alpha, const double2* __restrict__ U,
                             const double2* __restrict__ X, const double2* __restrict__ Q,
                             const double2* __restrict__ H0, const double2* __restrict__ H1,
                             const double2* __restrict__ H2, double2* __restrict__ Ua, double2* __restrict__ Ha) {
    const int b = blockIdx.x;
    const double a = alpha[b];
    const int64_t o = (int64_t)b * n * n;
    for (int e = threadIdx.x; e < n * n; e += blockDim.x) {
        const int i = e / n, j = e - i * n;
        const double2 x = X[o + e], xt = X[o + j * n + i];
        const double2 h = H1[o + e], ht = H1[o + j * n + i];
        const double2 u = U[o + e], q = Q[o + e], h0 = H0[o + e], h2 = H2[o + e];
        Ua[o + e] = double2{u.x + a * (x.x + xt.x) + a * a * q.x, u.y + a * (x.y - xt.y) + a * a * q.y};
        Ha[o + e] = double2{h0.x + a * (h.x + ht.x) + a * a * h2.x, h0.y + a * (h.y - ht.y) + a * a * h2.y};
    }
}

// Re Tr(Rinv^dag H Rinv) per batch (= Tr(U^{-1} H) for U = R^dag R).
__global__ void __launch_bounds__(256)
k_trace_RhHR(int n, const double2* __restrict__ Rinv, const double2* __restrict__ H, double* __restrict__ out) {
    __shared__ double red[256];
    const int b = blockIdx.x;
    const int64_t o = (int64_t)b * n * n;
    double acc = 0;
    // sum_i sum_a conj(Rinv[a][i]) (H Rinv)[a][i]
    for (int e = threadIdx.x; e < n * n; e += blockDim.x) {
        const int a = e / n, i = e - a * n;
        double wr = 0, wi = 0;
        for (int t = 0; t < n; ++t) {
            const double2 h = H[o + a * n + t], r = Rinv[o + t * n + i];
            wr += h.x * r.x - h.y * r.y;
            wi += h.x * r.y + h.y * r.x;
        }
        const double2 ra = Rinv[o + a * n + i];
        acc += ra.x * wr + ra.y * wi;
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[b] = red[0];
}

// Residual norms ||(H - eps_i O) y_i||_2 / sqrt(Omega) for orthonormal
// eigenvector blocks: one workgroup per (band, k), out[k * fstride + band].
__global__ void __launch_bounds__(256)
k_band_residual(const Seg* __restrict__ seg, int nb, int fstride, const double* __restrict__ eig, double omega,
                const double2* __restrict__ Y, const double2* __restrict__ HY, double* __restrict__ out) {
    __shared__ double red[256];
    const int b = blockIdx.x, k = blockIdx.y;
    const Seg s = seg[k];
    const double e = eig[k * fstride + b] * omega;
    const double2* y = Y + s.off + (int64_t)b * s.npw;
    const double2* h = HY + s.off + (int64_t)b * s.npw;
    double acc = 0;
    for (int q = threadIdx.x; q < s.npw; q += 256) {
        const double rx = h[q].x - e * y[q].x, ry = h[q].y - e * y[q].y;
        acc += rx * rx + ry * ry;
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[k * fstride + b] = sqrt(red[0] / omega);
}

// ------------------------------------------------------------ grids --------

// out = a*x + b*y + c*z (any pointer may be null -> term dropped).
__global__ void k_grid_lin3(int64_t N, double a, const double* __restrict__ x, double b, const double* __restrict__ y,
                            double c, const double* __restrict__ z, double* __restrict__ out) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= N) return;
    double r = 0;
    if (x) r += a * x[j];
    if (y) r += b * y[j];
    if (z) r += c * z[j];
    out[j] = r;
}

// Dots of one grid field with up to PULAY_MAX others in one pass:
// part[j * MDOT_BLOCKS + block] = sum over the block's points of a * b_j.
__global__ void __launch_bounds__(256)
k_multi_dot(int64_t N, const double* __restrict__ a, PulayPtrs bl, int nb, double* __restrict__ part) {
    __shared__ double red[PULAY_MAX][256];
    double acc[PULAY_MAX];
#pragma unroll
    for (int j = 0; j < PULAY_MAX; ++j) acc[j] = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < N; i += (int64_t)MDOT_BLOCKS * 256) {
        const double av = a[i];
#pragma unroll
        for (int j = 0; j < PULAY_MAX; ++j)
            if (j < nb) acc[j] += av * bl.res[j][i];
    }
#pragma unroll
    for (int j = 0; j < PULAY_MAX; ++j) red[j][threadIdx.x] = acc[j];
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w)
            for (int j = 0; j < nb; ++j) red[j][threadIdx.x] += red[j][threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x < nb) part[threadIdx.x * MDOT_BLOCKS + blockIdx.x] = red[threadIdx.x][0];
}

// A[row][slot[j]] = A[slot[j]][row] = scale * sum of the partials of dot j (A is
// PULAY_MAX x PULAY_MAX, indexed by history slot).
__global__ void k_multi_dot_store(const double* __restrict__ part, int nb, PulayOrder slot, int row, double scale,
                                  double* __restrict__ A) {
    const int j = threadIdx.x;
    if (j >= nb) return;
    double s = 0;
    for (int b = 0; b < MDOT_BLOCKS; ++b) s += part[j * MDOT_BLOCKS + b];
    A[row * PULAY_MAX + slot.s[j]] = scale * s;
    A[slot.s[j] * PULAY_MAX + row] = scale * s;
}

// Pulay combination: out = sum_i c_i (nin_i + alpha R_i), histories as arrays of pointers.
__global__ void k_pulay_combine(int64_t N, int m, PulayPtrs h, const double* __restrict__ c, double alpha,
                                double* __restrict__ out) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= N) return;
    double r = 0;
    for (int i = 0; i < m; ++i) r += c[i] * (h.nin[i][j] + alpha * h.res[i][j]);
    out[j] = r;
}

// Solve the (m+1) x (m+1) Pulay system [A 1; 1^T 0][c; l] = [0; 1] by LU with
// partial pivoting (one thread).  A is indexed by history slot; order.s[i] is
// the slot of the i-th oldest entry.
__global__ void k_pulay_solve(int m, const double* __restrict__ A, PulayOrder order, double* __restrict__ c,
                              int* __restrict__ status) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double M[PULAY_MAX + 1][PULAY_MAX + 2];
    const int n = m + 1;
    for (int i = 0; i < n; ++i) {
        for (int j = 0; j < n; ++j)
            M[i][j] = (i < m && j < m) ? A[order.s[i] * PULAY_MAX + order.s[j]]
                                       : ((i == m) != (j == m) ? 1.0 : 0.0);
        M[i][n] = (i == m) ? 1.0 : 0.0;
    }
    for (int col = 0; col < n; ++col) {
        int piv = col;
        for (int r = col + 1; r < n; ++r)
            if (fabs(M[r][col]) > fabs(M[piv][col])) piv = r;
        if (M[piv][col] == 0.0) {
            atomicOr(status, DPP_STATUS_NONFINITE);
            for (int i = 0; i < m; ++i) c[i] = (i == m - 1) ? 1.0 : 0.0;
            return;
        }
        if (piv != col)
            for (int j = 0; j <= n; ++j) {
                const double t = M[col][j];
                M[col][j] = M[piv][j];
                M[piv][j] = t;
            }
        for (int r = col + 1; r < n; ++r) {
            const double fct = M[r][col] / M[col][col];
            for (int j = col; j <= n; ++j) M[r][j] -= fct * M[col][j];
        }
    }
    double x[PULAY_MAX + 1];
    for (int i = n - 1; i >= 0; --i) {
        double s = M[i][n];
        for (int j = i + 1; j < n; ++j) s -= M[i][j] * x[j];
        x[i] = s / M[i][i];
    }
    for (int i = 0; i < m; ++i) c[i] = x[i];
}

}  // namespace dpp
