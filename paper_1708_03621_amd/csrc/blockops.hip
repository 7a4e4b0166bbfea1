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

__device__ __forceinline__ int item_nb(const Seg& s, int nbo) { return nbo > 0 ? nbo : s.nb; }

// out_i = a_i * x_i + b_i * y_i over every item's block (a, b per item, device).
__global__ void k_seg_axpby(const Seg* __restrict__ seg, int nbo, const double* __restrict__ a,
                            const double2* __restrict__ x, const double* __restrict__ b,
                            const double2* __restrict__ y, double2* __restrict__ out) {
    const int k = blockIdx.y;
    const Seg s = seg[k];
    const int64_t n = (int64_t)item_nb(s, nbo) * s.npw;
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

// (band, point) of element e = band * npw + point of a grid-stride loop,
// stepped with the loop instead of divided per element: the first index takes
// one 64-bit division per thread, each step an add and at most one carry.
struct BandPoint {
    int b, q, db, dq, npw;
    __device__ BandPoint(int64_t e0, int64_t stride, int npw_) : npw(npw_) {
        b = (int)(e0 / npw_);
        q = (int)(e0 - (int64_t)b * npw_);
        db = (int)(stride / npw_);
        dq = (int)(stride - (int64_t)db * npw_);
    }
    __device__ __forceinline__ void next() {
        b += db;
        q += dq;
        if (q >= npw) {
            q -= npw;
            ++b;
        }
    }
};

// out = scale * K x  (K = 1/(1 + |k+G|^2/2)), per item.
__global__ void k_seg_precond(const Seg* __restrict__ seg, int nbo, double scale, const double2* __restrict__ x,
                              double2* __restrict__ out) {
    const int k = blockIdx.y;
    const Seg s = seg[k];
    const int64_t n = (int64_t)item_nb(s, nbo) * s.npw;
    const int64_t e0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x, st = (int64_t)gridDim.x * blockDim.x;
    BandPoint bp(e0, st, s.npw);
    for (int64_t e = e0; e < n; e += st, bp.next()) {
        const double kk = scale / (1.0 + 0.5 * s.kG2[bp.q]);
        const double2 v = x[s.off + e];
        out[s.off + e] = double2{kk * v.x, kk * v.y};
    }
}

// Per-item dots 2 Re sum conj(A) B for up to 4 pairs: partial sums per
// (pair, item, block) -> part[(pair * nitems + k) * gridDim.x + blockIdx.x]
// (gridDim.x = dot_blocks of the system).
__global__ void __launch_bounds__(256)
k_seg_dots(const Seg* __restrict__ seg, int nitems, int nbo, int npair, DotPairs pr, double* __restrict__ part) {
    __shared__ double red[4][256];
    const int k = blockIdx.y;
    const Seg s = seg[k];
    const int64_t n = (int64_t)item_nb(s, nbo) * s.npw;
    double acc[4] = {0, 0, 0, 0};
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < n; e += (int64_t)gridDim.x * 256) {
        const int64_t o = s.off + e;
#pragma unroll
        for (int p = 0; p < 4; ++p) {
            if (p < npair) {
                const double2 av = pr.a[p][o], bv = pr.b[p][o];
                acc[p] += av.x * bv.x + av.y * bv.y;
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
    if (threadIdx.x < npair)
        part[((int64_t)threadIdx.x * nitems + k) * gridDim.x + blockIdx.x] = 2.0 * red[threadIdx.x][0];
}

// Fixed-order sums: out[pair * (nitems + 1) + k] per item and the total over
// items at out[pair * (nitems + 1) + nitems].
__global__ void k_seg_dots_reduce(const double* __restrict__ part, int nitems, int npair, double* __restrict__ out,
                                  int nblk) {
    const int p = blockIdx.x;
    if (p >= npair) return;
    for (int k = threadIdx.x; k < nitems; k += blockDim.x) {
        double s = 0;
        for (int b = 0; b < nblk; ++b) s += part[((int64_t)p * nitems + k) * nblk + b];
        out[p * (nitems + 1) + k] = s;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = 0;
        for (int k = 0; k < nitems; ++k) s += out[p * (nitems + 1) + k];
        out[p * (nitems + 1) + nitems] = s;
    }
}

// Band-weighted kinetic sums: part[k * gridDim.x + block] of
// sum_i f_ki * sum_G |k+G|^2 |psi_Gi|^2.
__global__ void __launch_bounds__(256)
k_seg_kinetic(const Seg* __restrict__ seg, int nbo, const double* __restrict__ f, const double2* __restrict__ psi,
              double* __restrict__ part) {
    __shared__ double red[256];
    const int k = blockIdx.y;
    const Seg s = seg[k];
    const int64_t n = (int64_t)item_nb(s, nbo) * s.npw;
    double acc = 0;
    const int64_t e0 = (int64_t)blockIdx.x * 256 + threadIdx.x, st = (int64_t)gridDim.x * 256;
    BandPoint bp(e0, st, s.npw);
    for (int64_t e = e0; e < n; e += st, bp.next()) {
        const double2 v = psi[s.off + e];
        acc += f[s.f_off + bp.b] * s.kG2[bp.q] * (v.x * v.x + v.y * v.y);
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[k * gridDim.x + blockIdx.x] = red[0];
}

// out[c * out_stride] = sum over the cell's items of w_k (scale_omega * Omega)
// * sum_blocks part[k]  (fixed order; one thread per cell).
__global__ void k_cell_weighted_totals(const double* __restrict__ part, const Seg* __restrict__ seg,
                                       const CellDesc* __restrict__ cells, int ncells, double scale_omega,
                                       double* __restrict__ out, int out_stride, int nblk) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= ncells) return;
    const CellDesc cr = cells[c];
    double tot = 0;
    for (int k = cr.item0; k < cr.item0 + cr.nitems; ++k) {
        double s = 0;
        for (int b = 0; b < nblk; ++b) s += part[k * nblk + b];
        tot += seg[k].wk * scale_omega * seg[k].omega * s;
    }
    out[c * out_stride] = tot;
}

// Nonlocal energy per cell: sum_k w_k D sum_i f_ki sum_a |Pi_ai|^2, Pi of item
// k at pi + pioff (nproj x nb row-major).  One workgroup per cell.
__global__ void k_nonlocal_energy(const Seg* __restrict__ seg, const CellDesc* __restrict__ cells, int nbo,
                                  const double2* __restrict__ pi, const double* __restrict__ f,
                                  double* __restrict__ out, int out_stride) {
    __shared__ double red[256];
    const CellDesc cr = cells[blockIdx.x];
    double tot = 0;
    for (int k = cr.item0; k < cr.item0 + cr.nitems; ++k) {
        const Seg s = seg[k];
        const int nb = item_nb(s, nbo);
        double acc = 0;
        for (int e = threadIdx.x; e < s.nproj * nb; e += blockDim.x) {
            const int i = e % nb;
            const double2 v = pi[s.pioff + e];
            acc += f[s.f_off + i] * (v.x * v.x + v.y * v.y);
        }
        red[threadIdx.x] = acc;
        __syncthreads();
        for (int w = 128; w > 0; w >>= 1) {
            if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
            __syncthreads();
        }
        if (threadIdx.x == 0) tot += s.wk * cr.D * red[0];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[blockIdx.x * out_stride] = tot;
}

// ------------------------------------------------------- small matrices ----
// Every item's matrices are n x n row-major at moff (n = nbo or seg.nb).

// out = scale * (w_k if flags & 1) * (Omega if flags & 2) * op(A), op = N or H.
__global__ void k_sm_scale(const Seg* __restrict__ seg, int nbo, int op, double scale, int flags,
                           const double2* __restrict__ A, double2* __restrict__ out) {
    const Seg s = seg[blockIdx.x];
    const int n = item_nb(s, nbo);
    const double sc = scale * ((flags & 1) ? s.wk : 1.0) * ((flags & 2) ? s.omega : 1.0);
    for (int e = threadIdx.x; e < n * n; e += blockDim.x) {
        const int i = e / n, j = e - i * n;
        double2 a = op ? A[s.moff + j * n + i] : A[s.moff + e];
        if (op) a.y = -a.y;
        out[s.moff + e] = double2{sc * a.x, sc * a.y};
    }
}

// Residual norms ||(H - eps_i O) y_i||_2 / sqrt(Omega) for orthonormal
// eigenvector blocks: one workgroup per (band, item), out[f_off + band].
__global__ void __launch_bounds__(256)
k_band_residual(const Seg* __restrict__ seg, const double* __restrict__ eig, const double2* __restrict__ Y,
                const double2* __restrict__ HY, double* __restrict__ out) {
    __shared__ double red[256];
    const int b = blockIdx.x, k = blockIdx.y;
    const Seg s = seg[k];
    if (b >= s.nb) return;
    const double e = eig[s.f_off + b] * s.omega;
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
    if (threadIdx.x == 0) out[s.f_off + b] = sqrt(red[0] / s.omega);
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

__global__ void k_fill(int64_t n, double v, double* __restrict__ out) {
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n; j += (int64_t)gridDim.x * blockDim.x)
        out[j] = v;
}

__global__ void k_copy(int64_t n, const double2* __restrict__ x, double2* __restrict__ out) {
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n; j += (int64_t)gridDim.x * blockDim.x)
        out[j] = x[j];
}

// ------------------------------------------------------------- Pulay -------
// History ring of PULAY_MAX entries shared by every cell, state on the device:
// st[0] = entries m, st[1] = oldest slot, st[2] = slot of the newest entry.
// Entry s of a history array lives at s * Ntot (fields of all cells).

__global__ void k_pulay_reset(int* __restrict__ st) {
    if (threadIdx.x == 0) st[0] = st[1] = st[2] = 0;
}

__global__ void k_pulay_begin(int* __restrict__ st) {
    if (threadIdx.x != 0) return;
    int m = st[0], head = st[1], slot;
    if (m < PULAY_MAX) {
        slot = (head + m) % PULAY_MAX;
        ++m;
    } else {
        slot = head;
        head = (head + 1) % PULAY_MAX;
    }
    st[0] = m;
    st[1] = head;
    st[2] = slot;
}

// New entry: n_in and R = n_out - n_in into the slot st[2] (all cells at once).
__global__ void k_pulay_store(int64_t Ntot, const int* __restrict__ st, const double* __restrict__ nin,
                              const double* __restrict__ nout, double* __restrict__ hn, double* __restrict__ hr) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= Ntot) return;
    const int64_t o = (int64_t)st[2] * Ntot + j;
    hn[o] = nin[j];
    hr[o] = nout[j] - nin[j];
}

// Per cell (blockIdx.y): partial dots of the new residual with the m stored
// residuals, history order i (slot (head + i) mod PULAY_MAX):
// part[(cell * PULAY_MAX + i) * MDOT_BLOCKS + block].
__global__ void __launch_bounds__(256)
k_pulay_dots(int64_t Ntot, const int* __restrict__ st, const CellDesc* __restrict__ cells,
             const double* __restrict__ hr, double* __restrict__ part) {
    __shared__ double red[PULAY_MAX][256];
    const CellDesc c = cells[blockIdx.y];
    const int m = st[0], head = st[1], slot = st[2];
    const double* a = hr + (int64_t)slot * Ntot + c.foff;
    double acc[PULAY_MAX];
#pragma unroll
    for (int i = 0; i < PULAY_MAX; ++i) acc[i] = 0.0;
    for (int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x; j < c.N; j += (int64_t)MDOT_BLOCKS * 256) {
        const double av = a[j];
#pragma unroll
        for (int i = 0; i < PULAY_MAX; ++i)
            if (i < m) acc[i] += av * hr[(int64_t)((head + i) % PULAY_MAX) * Ntot + c.foff + j];
    }
#pragma unroll
    for (int i = 0; i < PULAY_MAX; ++i) red[i][threadIdx.x] = acc[i];
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w)
            for (int i = 0; i < m; ++i) red[i][threadIdx.x] += red[i][threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x < m)
        part[((int64_t)blockIdx.y * PULAY_MAX + threadIdx.x) * MDOT_BLOCKS + blockIdx.x] = red[threadIdx.x][0];
}

// Per cell (one thread): finish the residual overlaps into the cell's
// slot-indexed matrix A (PULAY_MAX^2 per cell, scaled by Omega / N), then the
// mixing coefficients in history order: c = (1) for one entry, else the
// solution of [A 1; 1^T 0][c; l] = [0; 1] (LU with partial pivoting).
__global__ void __launch_bounds__(256)
k_pulay_solve_cells(int ncells, const int* __restrict__ st, const CellDesc* __restrict__ cells,
                    const double* __restrict__ part, double* __restrict__ A, double* __restrict__ coef,
                    int* __restrict__ status) {
    __shared__ double ov[PULAY_MAX];
    __shared__ double M[PULAY_MAX + 1][PULAY_MAX + 2];
    __shared__ int piv_s;
    const int cidx = blockIdx.x;
    const int m = st[0], head = st[1], slot = st[2];
    const int tid = threadIdx.x;
    // overlap i: 32 lanes (one half wave) sum its MDOT_BLOCKS partials in a
    // fixed order (strided lane sums, then a butterfly within the 32 lanes)
    {
        const int g = tid >> 5, l = tid & 31;
        double v = 0.0;
        if (g < m)
            for (int b = l; b < MDOT_BLOCKS; b += 32) v += part[((int64_t)cidx * PULAY_MAX + g) * MDOT_BLOCKS + b];
#pragma unroll
        for (int o = 16; o > 0; o >>= 1) v += __shfl_xor(v, o);
        if (g < m && l == 0) ov[g] = v;
    }
    __syncthreads();
    const double dV = cells[cidx].dV;
    double* Ac = A + (int64_t)cidx * PULAY_MAX * PULAY_MAX;
    double* c = coef + (int64_t)cidx * PULAY_MAX;
    if (tid < m) {
        const int si = (head + tid) % PULAY_MAX;
        Ac[slot * PULAY_MAX + si] = dV * ov[tid];
        Ac[si * PULAY_MAX + slot] = dV * ov[tid];
    }
    if (m == 1) {
        if (tid == 0) c[0] = 1.0;
        return;
    }
    // bordered system [[A, 1], [1^T, 0]] [c; lambda] = [0; 1], Gaussian
    // elimination with partial pivoting: one thread per row
    const int n = m + 1;
    if (tid < n * (n + 1)) {
        const int i = tid / (n + 1), j = tid - i * (n + 1);
        double v;
        if (j == n)
            v = (i == m) ? 1.0 : 0.0;
        else if (i < m && j < m) {
            // the newest row and column from this launch's overlaps, the rest
            // from the stored history
            const int si = (head + i) % PULAY_MAX, sj = (head + j) % PULAY_MAX;
            v = si == slot ? dV * ov[j] : (sj == slot ? dV * ov[i] : Ac[si * PULAY_MAX + sj]);
        }
        else
            v = ((i == m) != (j == m)) ? 1.0 : 0.0;
        M[i][j] = v;
    }
    __syncthreads();
    for (int col = 0; col < n; ++col) {
        if (tid == 0) {
            int piv = col;
            for (int r = col + 1; r < n; ++r)
                if (fabs(M[r][col]) > fabs(M[piv][col])) piv = r;
            piv_s = M[piv][col] == 0.0 ? -1 : piv;
        }
        __syncthreads();
        const int piv = piv_s;
        if (piv < 0) {
            if (tid == 0) {
                atomicOr(status, DPP_STATUS_NONFINITE);
                for (int i = 0; i < m; ++i) c[i] = (i == m - 1) ? 1.0 : 0.0;
            }
            return;  // uniform
        }
        if (piv != col && tid <= n) {
            const double t = M[col][tid];
            M[col][tid] = M[piv][tid];
            M[piv][tid] = t;
        }
        __syncthreads();
        if (tid > col && tid < n) {
            const double fct = M[tid][col] / M[col][col];
            for (int j = col; j <= n; ++j) M[tid][j] -= fct * M[col][j];
        }
        __syncthreads();
    }
    if (tid == 0) {
        double x[PULAY_MAX + 1];
        for (int i = n - 1; i >= 0; --i) {
            double sacc = M[i][n];
            for (int j = i + 1; j < n; ++j) sacc -= M[i][j] * x[j];
            x[i] = sacc / M[i][i];
        }
        for (int i = 0; i < m; ++i) c[i] = x[i];
    }
}

// n_in = sum_i c_i (n_in,i + alpha R_i) per cell (blockIdx.y), history order.
__global__ void k_pulay_combine_cells(int64_t Ntot, const int* __restrict__ st, const CellDesc* __restrict__ cells,
                                      const double* __restrict__ coef, double alpha, const double* __restrict__ hn,
                                      const double* __restrict__ hr, double* __restrict__ nin) {
    const CellDesc c = cells[blockIdx.y];
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= c.N) return;
    const int m = st[0], head = st[1];
    const double* cc = coef + (int64_t)blockIdx.y * PULAY_MAX;
    double r = 0;
    for (int i = 0; i < m; ++i) {
        const int64_t o = (int64_t)((head + i) % PULAY_MAX) * Ntot + c.foff + j;
        r += cc[i] * (hn[o] + alpha * hr[o]);
    }
    nin[c.foff + j] = r;
}

// ---------------------------------------------------- band-CG control ------
// Per-item state of the band-energy CG (protocol B), updated on the device so
// that a whole SCF iteration runs without host round trips.

__global__ void k_cgB_reset(int nit, const Seg* __restrict__ seg, CgBState s) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= nit) return;
    s.at[k] = 0.3 / seg[k].omega;
    s.reset[k] = 1;
    s.stat[k] = 0;
    s.gkg[k] = 0.0;
}

// Fused start of a band-CG step: Kg = K g and, per item, partial sums of
// <g, Kg>, <g_prev, Kg>, <g, D_prev> (2 Re sum conj(a) b) in one pass:
// part[(pair * nitems + k) * gridDim.x + block].
__global__ void __launch_bounds__(256)
k_cg_precond_dots(const Seg* __restrict__ seg, int nitems, const double2* __restrict__ g,
                  const double2* __restrict__ gp, const double2* __restrict__ Dp, double2* __restrict__ Kg,
                  double* __restrict__ part) {
    __shared__ double red[3][256];
    const int k = blockIdx.y;
    const Seg s = seg[k];
    const int64_t n = (int64_t)s.nb * s.npw;
    double a0 = 0, a1 = 0, a2 = 0;
    const int64_t e0 = (int64_t)blockIdx.x * 256 + threadIdx.x, st = (int64_t)gridDim.x * 256;
    BandPoint bp(e0, st, s.npw);
    for (int64_t e = e0; e < n; e += st, bp.next()) {
        const int64_t o = s.off + e;
        const double kk = 1.0 / (1.0 + 0.5 * s.kG2[bp.q]);
        const double2 gv = g[o], gpv = gp[o], dv = Dp[o];
        const double2 kg = double2{kk * gv.x, kk * gv.y};
        Kg[o] = kg;
        a0 += gv.x * kg.x + gv.y * kg.y;
        a1 += gpv.x * kg.x + gpv.y * kg.y;
        a2 += gv.x * dv.x + gv.y * dv.y;
    }
    red[0][threadIdx.x] = a0;
    red[1][threadIdx.x] = a1;
    red[2][threadIdx.x] = a2;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w)
            for (int p = 0; p < 3; ++p) red[p][threadIdx.x] += red[p][threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x < 3) part[((int64_t)threadIdx.x * nitems + k) * gridDim.x + blockIdx.x] = 2.0 * red[threadIdx.x][0];
}

// Per item (one 64-thread workgroup): fixed-order sums of the three dot
// partials into dots[pair * (nitems + 1) + k], then the direction
// coefficients of the item (as k_cgB_direction).
// --- fused control + elementwise passes (see blockops.h) ---

__global__ void __launch_bounds__(256)
k_cgB_direction(const Seg* __restrict__ seg, int nitems, const double* __restrict__ part, double* __restrict__ dots,
                CgBState s, const double2* __restrict__ Kg, const double2* __restrict__ Dp, double2* __restrict__ Dd,
                int nblk) {
    __shared__ double red[3][64];
    __shared__ double coef[2];
    const int k = blockIdx.y;
    if (threadIdx.x < 64) {
        for (int p = 0; p < 3; ++p) {
            double v = 0.0;
            for (int b = threadIdx.x; b < nblk; b += 64) v += part[((int64_t)p * nitems + k) * nblk + b];
            red[p][threadIdx.x] = v;
        }
    }
    __syncthreads();
    for (int w = 32; w > 0; w >>= 1) {
        if (threadIdx.x < w)
            for (int p = 0; p < 3; ++p) red[p][threadIdx.x] += red[p][threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double gkg = red[0][0], gpkg = red[1][0], gdp = red[2][0];
        const bool st = s.stat[k] != 0;
        double b = 0.0, dd = 0.0;
        if (!st) {
            if (!s.reset[k]) b = fmax(0.0, (gkg - gpkg) / s.gkg[k]);
            dd = -gkg + b * gdp;
            if (b != 0.0 && dd >= 0.0) {
                b = 0.0;
                dd = -gkg;
            }
        }
        coef[0] = -1.0;
        coef[1] = b;
        if (blockIdx.x == 0) {
            dots[k] = gkg;
            dots[(nitems + 1) + k] = gpkg;
            dots[2 * (nitems + 1) + k] = gdp;
            s.cK[k] = -1.0;
            s.act[k] = st ? 0 : 1;
            s.beta[k] = b;
            s.d0[k] = dd;
            s.steep[k] = st ? 1 : (b == 0.0);
        }
    }
    __syncthreads();
    const Seg sg = seg[k];
    const int64_t n = (int64_t)sg.nb * sg.npw;
    const double ak = coef[0], bk = coef[1];
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t o = sg.off + e;
        const double2 v = Kg[o], w = Dp[o];
        double2 r = double2{ak * v.x, ak * v.y};
        r.x += bk * w.x;
        r.y += bk * w.y;
        Dd[o] = r;
    }
}

__global__ void __launch_bounds__(256)
k_cgB_retry_axpby(const Seg* __restrict__ seg, const double* __restrict__ dots, CgBState s,
                  const double2* __restrict__ Kg, double2* __restrict__ Dd) {
    const int k = blockIdx.y;
    const int r = s.act[k] && !s.ok[k] && !s.steep[k];
    const double ak = r ? -1.0 : 0.0, bk = r ? 0.0 : 1.0;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        s.retry[k] = r;
        s.cK[k] = ak;
        s.cD[k] = bk;
        s.d0r[k] = r ? -dots[k] : s.d0[k];
    }
    if (!r) return;  // D stays (the unfused form computed 0 Kg + 1 D)
    const Seg sg = seg[k];
    const int64_t n = (int64_t)sg.nb * sg.npw;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t o = sg.off + e;
        const double2 v = Kg[o], w = Dd[o];
        double2 q = double2{ak * v.x, ak * v.y};
        q.x += bk * w.x;
        q.y += bk * w.y;
        Dd[o] = q;
    }
}

__global__ void __launch_bounds__(256)
k_cgB_finish_update(const Seg* __restrict__ seg, const double* __restrict__ dots, CgBState s, double2* __restrict__ Y,
                    const double2* __restrict__ Dd, double2* __restrict__ HY, const double2* __restrict__ HD,
                    const double2* __restrict__ g, double2* __restrict__ gp, double2* __restrict__ Dp) {
    const int k = blockIdx.y;
    // accept the step (inputs act, ok, ok2, retry, step, step2 are not written here)
    double st = 0.0;
    int o = 0;
    if (s.act[k]) {
        o = s.ok[k];
        st = s.step[k];
        if (s.retry[k]) {
            o = s.ok2[k];
            st = s.step2[k];
        }
        if (!o) st = 0.0;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        s.stepf[k] = st;
        if (s.act[k]) {
            if (!o) {
                s.stat[k] = 1;
                s.reset[k] = 1;
            } else {
                s.gkg[k] = dots[k];
                s.at[k] = st;
                s.reset[k] = 0;
            }
        }
    }
    const Seg sg = seg[k];
    const int64_t n = (int64_t)sg.nb * sg.npw;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t q = sg.off + e;
        const double2 d = Dd[q], hd = HD[q], y = Y[q], hy = HY[q];
        Y[q] = double2{y.x + st * d.x, y.y + st * d.y};
        HY[q] = double2{hy.x + st * hd.x, hy.y + st * hd.y};
        gp[q] = g[q];
        Dp[q] = d;
    }
}

// Re Tr(M) per item (fixed order), out[item].
__global__ void __launch_bounds__(64)
k_trace_diag(const Seg* __restrict__ seg, const double2* __restrict__ M, double* __restrict__ out) {
    __shared__ double red[64];
    const Seg s = seg[blockIdx.x];
    double v = 0.0;
    for (int i = threadIdx.x; i < s.nb; i += 64) v += M[s.moff + (int64_t)i * s.nb + i].x;
    red[threadIdx.x] = v;
    __syncthreads();
    for (int w = 32; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[blockIdx.x] = red[0];
}

// ------------------------------------------------------------ aufbau -------
// Fillings of one cell (one workgroup): states (e, k, i) ordered by energy,
// then k-point, then band; groups of states within DEGEN_TOL of the group's
// first energy fill together, each state holding 2 w_k electrons; a group that
// does not fit shares the remaining electrons equally.

// Fermi-Dirac fillings (Table 1: smearing) of every cell; see blockops.h.
__global__ void __launch_bounds__(256)
k_fermi(const CellDesc* __restrict__ cells, const Seg* __restrict__ seg, const double* __restrict__ eig, double sigma,
        double* __restrict__ f, double* __restrict__ E, int stride, int* __restrict__ status) {
    __shared__ double e[AUFBAU_MAX];
    __shared__ double w[AUFBAU_MAX];
    __shared__ int64_t fo[AUFBAU_MAX];
    __shared__ double red[256];
    __shared__ double bounds[2];
    const CellDesc c = cells[blockIdx.x];
    // states of the cell's items in item order
    int ns = 0;
    for (int k = 0; k < c.nitems; ++k) {
        const Seg sk = seg[c.item0 + k];
        for (int i = threadIdx.x; i < sk.nb; i += blockDim.x) {
            e[ns + i] = eig[sk.f_off + i];
            w[ns + i] = sk.wk;
            fo[ns + i] = sk.f_off + i;
        }
        ns += sk.nb;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double lo = e[0], hi = e[0], cap = 0.0;
        for (int t = 0; t < ns; ++t) {
            lo = fmin(lo, e[t]);
            hi = fmax(hi, e[t]);
            cap += 2.0 * w[t];
        }
        bounds[0] = lo - SMEAR_BRACKET * sigma;
        bounds[1] = hi + SMEAR_BRACKET * sigma;
        if (cap < c.ne - 1e-9) atomicOr(status, DPP_STATUS_NOBANDS);
    }
    __syncthreads();
    double lo = bounds[0], hi = bounds[1];
    for (int it = 0; it < SMEAR_ITERS; ++it) {
        const double mid = 0.5 * (lo + hi);
        double s = 0.0;
        for (int t = threadIdx.x; t < ns; t += blockDim.x) s += 2.0 * w[t] / (1.0 + exp((e[t] - mid) / sigma));
        red[threadIdx.x] = s;
        __syncthreads();
        for (int h = 128; h > 0; h >>= 1) {
            if (threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
            __syncthreads();
        }
        const double cnt = red[0];
        __syncthreads();  // every thread has read the count before the next step overwrites red
        if (cnt < c.ne)
            lo = mid;
        else
            hi = mid;
    }
    const double mu = 0.5 * (lo + hi);
    double s = 0.0;
    for (int t = threadIdx.x; t < ns; t += blockDim.x) {
        const double x = (e[t] - mu) / sigma;
        const double g = 1.0 / (1.0 + exp(x)), gc = 1.0 / (1.0 + exp(-x));  // g and 1 - g
        f[fo[t]] = 2.0 * g;
        double tt = 0.0;
        if (g > 0.0) tt += g * log(g);
        if (gc > 0.0) tt += gc * log(gc);
        s -= 2.0 * w[t] * tt;
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        E[(int64_t)blockIdx.x * stride] = sigma * red[0];
        E[(int64_t)blockIdx.x * stride + 1] = mu;
    }
}

__global__ void __launch_bounds__(256)
k_aufbau(const CellDesc* __restrict__ cells, const Seg* __restrict__ seg, const double* __restrict__ eig,
         double* __restrict__ f, int* __restrict__ status) {
    __shared__ double e[AUFBAU_MAX];
    __shared__ double es[AUFBAU_MAX];
    __shared__ double cs[AUFBAU_MAX];
    __shared__ double fs[AUFBAU_MAX];
    __shared__ short kk[AUFBAU_MAX];
    __shared__ short ii[AUFBAU_MAX];
    __shared__ int order[AUFBAU_MAX];
    __shared__ int base[AUFBAU_MAX_ITEMS + 1];
    __shared__ double wks[AUFBAU_MAX_ITEMS];
    __shared__ int64_t foffs[AUFBAU_MAX_ITEMS];
    __shared__ int nbk[AUFBAU_MAX_ITEMS];
    const CellDesc c = cells[blockIdx.x];
    for (int k = threadIdx.x; k < c.nitems; k += blockDim.x) {
        const Seg sk = seg[c.item0 + k];
        wks[k] = sk.wk;
        foffs[k] = sk.f_off;
        nbk[k] = sk.nb;
    }
    __syncthreads();
    // Every state occupied: when all weights are positive and the electron
    // count reaches the capacity sum of 2 w_k over all states (to 1e-13,
    // inside the 1e-12 tolerance of the pass below), every degenerate group
    // fits and the pass would give every state f = 2, so the ordering is
    // skipped.
    __shared__ int all_full;
    if (threadIdx.x == 0) {
        base[0] = 0;
        double cap = 0.0;
        bool pos = true;
        for (int k = 0; k < c.nitems; ++k) {
            base[k + 1] = base[k] + nbk[k];
            cap += 2.0 * wks[k] * nbk[k];
            pos = pos && wks[k] > 0.0;
        }
        all_full = pos && c.ne >= cap - 1e-13;
        if (all_full && c.ne - cap > 1e-9) atomicOr(status, DPP_STATUS_NOBANDS);
    }
    __syncthreads();
    const int ns = base[c.nitems];
    if (all_full) {
        for (int t = threadIdx.x; t < ns; t += blockDim.x) {
            int k = 0;
            while (base[k + 1] <= t) ++k;
            f[foffs[k] + (t - base[k])] = 2.0;
        }
        return;
    }
    for (int t = threadIdx.x; t < ns; t += blockDim.x) {
        int k = 0;
        while (base[k + 1] <= t) ++k;
        const int i = t - base[k];
        e[t] = eig[foffs[k] + i];
        kk[t] = (short)k;
        ii[t] = (short)i;
    }
    __syncthreads();
    for (int t = threadIdx.x; t < ns; t += blockDim.x) {
        int r = 0;
        for (int u = 0; u < ns; ++u) {
            const bool less = e[u] < e[t] || (e[u] == e[t] && (kk[u] < kk[t] || (kk[u] == kk[t] && ii[u] < ii[t])));
            r += less;
        }
        order[r] = t;
    }
    __syncthreads();
    // states in sorted order: energy and capacity 2 w_k (reuse kk/ii-free arrays)
    for (int j = threadIdx.x; j < ns; j += blockDim.x) {
        const int t = order[j];
        es[j] = e[t];
        cs[j] = 2.0 * wks[kk[t]];
        fs[j] = 0.0;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        // One pass over the sorted states, eight at a time from LDS into
        // registers: a group [j0, j) closes at the first state j with
        // e_j - e_j0 >= DEGEN_TOL; its capacity is summed in state order.
        double rem = c.ne;
        bool stop = !(ns > 0 && rem > 1e-12);
        int j0 = 0;
        double e0 = ns > 0 ? es[0] : 0.0, cap = 0.0;
        auto close = [&](int j) {
            const bool fits = cap <= rem + 1e-12;
            const double val = fits ? 2.0 : 2.0 * (rem / cap);
            for (int t = j0; t < j; ++t) fs[t] = val;
            rem = fits ? rem - cap : 0.0;
        };
        for (int jb = 0; jb < ns && !stop; jb += 8) {
            double eb[8], cb[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int j = min(jb + u, ns - 1);
                eb[u] = es[j];
                cb[u] = cs[j];
            }
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int j = jb + u;
                if (stop || j >= ns) continue;
                if (j > j0 && !(eb[u] - e0 < DEGEN_TOL)) {
                    close(j);
                    if (!(rem > 1e-12)) {
                        stop = true;
                        continue;
                    }
                    j0 = j;
                    e0 = eb[u];
                    cap = 0.0;
                }
                cap += cb[u];
            }
        }
        if (!stop) close(ns);
        if (rem > 1e-9) atomicOr(status, DPP_STATUS_NOBANDS);
    }
    __syncthreads();
    for (int j = threadIdx.x; j < ns; j += blockDim.x) {
        const int t = order[j];
        f[foffs[kk[t]] + ii[t]] = fs[j];
    }
}

}  // namespace dpp
