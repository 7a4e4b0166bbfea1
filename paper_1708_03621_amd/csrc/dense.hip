// Small dense FP64 linear algebra for 33 to 128 bands, one workgroup per
// matrix with the matrix held in registers:
//   - Cholesky factor and inverse of the overlap U = R^dag R (orthonormalization),
//   - the band-gradient preparation (R^{-1}, U^{-1}, Tr(U^{-1} H~)),
//   - the band-energy line search along the CG direction,
//   - the subspace eigensolver (Householder reduction to a real tridiagonal,
//     bisection, inverse iteration, back-transformation).
//
// Register tiles: a TD x TD grid of threads (TD = 16 for n <= 64, 32 for
// n <= 128); thread (bi, bj) = (tid / TD, tid % TD) owns the 4 x 4 complex
// tile of rows 4bi..4bi+3 and columns 4bj..4bj+3.  A factorization step moves
// one 4-wide panel through LDS; every other entry stays in its owner's
// registers, so a 128 x 128 factorization reads LDS ~n^3/16 times instead of
// streaming the packed matrix through LDS at every pivot.  Rows and columns
// beyond n are padding: identity for factorizations, zero for the
// eigensolver.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cfloat>

#include "blockops.h"

namespace dpp {
namespace {

using z2 = double2;

__device__ __forceinline__ z2 zmul(z2 a, z2 b) { return z2{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x}; }
// conj(a) * b
__device__ __forceinline__ z2 zcmul(z2 a, z2 b) { return z2{a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x}; }
// a * conj(b)
__device__ __forceinline__ z2 zmulc(z2 a, z2 b) { return z2{a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y}; }
__device__ __forceinline__ z2 zadd(z2 a, z2 b) { return z2{a.x + b.x, a.y + b.y}; }
__device__ __forceinline__ z2 zsub(z2 a, z2 b) { return z2{a.x - b.x, a.y - b.y}; }
__device__ __forceinline__ z2 zconj(z2 a) { return z2{a.x, -a.y}; }
__device__ __forceinline__ z2 zscale(z2 a, double s) { return z2{a.x * s, a.y * s}; }
// Complex multiply-accumulate as four FMAs (acc +- a b, with a or b conjugated):
// written out, since the compiler does not re-associate acc - (a b) into FMAs.
__device__ __forceinline__ z2 zfma(z2 a, z2 b, z2 acc) {  // acc + a b
    return z2{fma(a.x, b.x, fma(-a.y, b.y, acc.x)), fma(a.x, b.y, fma(a.y, b.x, acc.y))};
}
__device__ __forceinline__ z2 zfms(z2 a, z2 b, z2 acc) {  // acc - a b
    return z2{fma(-a.x, b.x, fma(a.y, b.y, acc.x)), fma(-a.x, b.y, fma(-a.y, b.x, acc.y))};
}
__device__ __forceinline__ z2 zcfma(z2 a, z2 b, z2 acc) {  // acc + conj(a) b
    return z2{fma(a.x, b.x, fma(a.y, b.y, acc.x)), fma(a.x, b.y, fma(-a.y, b.x, acc.y))};
}
__device__ __forceinline__ z2 zcfms(z2 a, z2 b, z2 acc) {  // acc - conj(a) b
    return z2{fma(-a.x, b.x, fma(-a.y, b.y, acc.x)), fma(-a.x, b.y, fma(a.y, b.x, acc.y))};
}
__device__ __forceinline__ z2 zfmac(z2 a, z2 b, z2 acc) {  // acc + a conj(b)
    return z2{fma(a.x, b.x, fma(a.y, b.y, acc.x)), fma(a.y, b.x, fma(-a.x, b.y, acc.y))};
}
__device__ __forceinline__ z2 zfmsc(z2 a, z2 b, z2 acc) {  // acc - a conj(b)
    return z2{fma(-a.x, b.x, fma(-a.y, b.y, acc.x)), fma(-a.y, b.x, fma(a.x, b.y, acc.y))};
}

__device__ __forceinline__ double wsum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}
__device__ __forceinline__ double wmax(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
    return v;
}

// Which matrix a workgroup works on: from the item table, or matrix b of a
// uniform batch at stride n0^2.
struct Mat {
    int n;
    int64_t moff, f_off;
    double omega;
};

__device__ __forceinline__ Mat mat_of(const Seg* seg, int nbo, int n0, int b) {
    if (seg) {
        const Seg sg = seg[b];
        return Mat{nbo > 0 ? nbo : sg.nb, sg.moff, sg.f_off, sg.omega};
    }
    return Mat{n0, (int64_t)b * n0 * n0, (int64_t)b * n0, 1.0};
}

// v, hidden from the optimizer: addresses derived from it are computed where
// they are used instead of being hoisted to the kernel start and kept live
// (16 of them would take the registers the tile itself needs).
__device__ __forceinline__ int opaque(int v) {
    asm volatile("" : "+v"(v));
    return v;
}

// 1/sqrt(d): the hardware estimate refined by one Newton step.
__device__ __forceinline__ double rsqrt_nr(double d) {
    double y = __builtin_amdgcn_rsq(d);
    y = y * fma(-0.5 * d * y, y, 1.5);  // one Newton step: relative error ~ eps
    return y;
}


// ------------------------------------------------ Cholesky and inverse ----
// LDS of the factorization (aliases the staging area of the products after it).
// Panels are stored element-major (entry e of tile j at [e][j]): the lanes of
// a wave hold consecutive tile columns, so a panel read by all of them touches
// consecutive 16-byte words instead of one LDS bank 32 times.
template <int TD>
struct CholPanels {
    z2 dinv[TD][16];  // inverses of the diagonal tiles of R (read by broadcast)
    z2 pr[16][TD];    // row panel
    z2 pc[16][TD];    // column panel
};

template <int TD>
struct TileShared {
    double wred[TD * TD / 64];
    int fail;
};

template <int TD>
__device__ __forceinline__ double block_sum(double v, TileShared<TD>& S) {
    v = wsum(v);
    if ((threadIdx.x & 63) == 0) S.wred[threadIdx.x >> 6] = v;
    __syncthreads();
    double t = 0.0;
#pragma unroll
    for (int w = 0; w < TD * TD / 64; ++w) t += S.wred[w];
    __syncthreads();
    return t;
}

template <int TD>
__device__ __forceinline__ double block_max(double v, TileShared<TD>& S) {
    v = wmax(v);
    if ((threadIdx.x & 63) == 0) S.wred[threadIdx.x >> 6] = v;
    __syncthreads();
    double t = 0.0;
#pragma unroll
    for (int w = 0; w < TD * TD / 64; ++w) t = fmax(t, S.wred[w]);
    __syncthreads();
    return t;
}

// U = R^dag R for the Hermitian matrix whose upper tiles the threads hold in
// t (identity beyond n, lower tiles ignored); on success the upper tiles hold
// X = R^{-1} and the lower tiles zero.  Returns 1 (uniformly) when a pivot
// R_jj^2 is not above PIVOT_RTOL times the largest diagonal entry of U.
template <int TD>
__device__ __attribute__((always_inline)) int chol_inv_tiles(int n, z2 (&t)[4][4], CholPanels<TD>& P, TileShared<TD>& S) {
    const int tid = threadIdx.x, bi = tid / TD, bj = tid % TD;
    const int T = (n + 3) >> 2;
    double m = 0.0;
    if (bi == bj && bi < T) {
#pragma unroll
        for (int a = 0; a < 4; ++a)
            if (4 * bi + a < n) m = fmax(m, t[a][a].x);
    }
    if (tid == 0) S.fail = 0;
    const double thr = PIVOT_RTOL * block_max<TD>(m, S);
    if (bi > bj) {
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int c = 0; c < 4; ++c) t[a][c] = z2{0.0, 0.0};
    }
    // right-looking factorization over 4-wide block steps
#pragma unroll 1
    for (int K = 0; K < T; ++K) {
        if (bi == K && bj == K) {
            int f = 0;
            double ri[4];
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                double d = t[r][r].x;
                if (4 * K + r < n && !(d > thr)) f = 1;
                if (!(d > 0.0)) d = 1.0;  // keeps the arithmetic finite after a failure
                const double inv = rsqrt_nr(d);
                ri[r] = inv;
                t[r][r] = z2{d * inv, 0.0};
#pragma unroll
                for (int c = r + 1; c < 4; ++c) t[r][c] = zscale(t[r][c], inv);
#pragma unroll
                for (int s = r + 1; s < 4; ++s)
#pragma unroll
                    for (int c = s; c < 4; ++c) t[s][c] = zcfms(t[r][s], t[r][c], t[s][c]);
#pragma unroll
                for (int s = r + 1; s < 4; ++s) t[s][r] = z2{0.0, 0.0};
            }
            // inverse of the diagonal tile (upper triangular), column by column
            // into LDS: X_ij = -(sum_{i <= k < j} X_ik R_kj) / R_jj
            z2* xd = P.dinv[K];
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const double dj = ri[j];
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    z2 v = z2{0.0, 0.0};
                    if (i == j) {
                        v = z2{dj, 0.0};
                    } else if (i < j) {
#pragma unroll
                        for (int k = i; k < j; ++k) v = zfma(xd[4 * i + k], t[k][j], v);
                        v = zscale(v, -dj);
                    }
                    xd[4 * i + j] = v;
                }
            }
            if (f) S.fail = 1;
        }
        __syncthreads();
        if (S.fail) break;  // uniform: read after the barrier
        if (bi == K && bj > K && bj < T) {
            // row panel R_Kj = R_KK^{-dag} U_Kj, in place from the last row up
            // (row a needs rows b <= a of U_Kj)
#pragma unroll
            for (int a = 3; a >= 0; --a)
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    z2 s = z2{0.0, 0.0};
#pragma unroll
                    for (int b = 0; b <= a; ++b) s = zcfma(P.dinv[K][4 * b + a], t[b][c], s);
                    t[a][c] = s;
                    P.pr[4 * a + c][bj] = s;
                }
        }
        __syncthreads();
        if (bi > K && bi <= bj && bj < T) {
            // trailing update U_ij -= R_Ki^dag R_Kj (one row of R_Ki cached,
            // R_Kj streamed entry by entry)
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                z2 pi[4];
#pragma unroll
                for (int a = 0; a < 4; ++a) pi[a] = P.pr[4 * b + a][bi];
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    const z2 pj = P.pr[4 * b + c][bj];
#pragma unroll
                    for (int a = 0; a < 4; ++a) t[a][c] = zcfms(pi[a], pj, t[a][c]);
                }
                __builtin_amdgcn_sched_barrier(0);
            }
        }
    }
    const int failed = S.fail;
    __syncthreads();
    if (failed) return 1;
    // X = R^{-1} by column blocks: X_iK = -S_iK R_KK^{-1}, S_ij = sum_{k<j} X_ik R_kj
    // accumulated in the owner's registers once R_ij has been published.
#pragma unroll 1
    for (int K = 0; K < T; ++K) {
        if (bi == K && bj > K && bj < T) {
#pragma unroll
            for (int a = 0; a < 4; ++a)
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    P.pr[4 * a + c][bj] = t[a][c];
                    t[a][c] = z2{0.0, 0.0};
                }
        }
        if (bj == K && bi <= K) {
            if (bi == K) {
#pragma unroll
                for (int a = 0; a < 4; ++a)
#pragma unroll
                    for (int c = 0; c < 4; ++c) t[a][c] = P.dinv[K][4 * a + c];
            } else {
                // X_iK = -S_iK R_KK^{-1}, in place from the last column (column c
                // needs columns b <= c of S_iK)
#pragma unroll
                for (int a = 0; a < 4; ++a)
#pragma unroll
                    for (int c = 3; c >= 0; --c) {
                        z2 s = z2{0.0, 0.0};
#pragma unroll
                        for (int b = 0; b <= c; ++b) s = zfma(t[a][b], P.dinv[K][4 * b + c], s);
                        t[a][c] = z2{-s.x, -s.y};
                    }
            }
#pragma unroll
            for (int a = 0; a < 4; ++a)
#pragma unroll
                for (int c = 0; c < 4; ++c) P.pc[4 * a + c][bi] = t[a][c];
        }
        __syncthreads();
        if (bi <= K && K < bj && bj < T) {
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                z2 xc[4];
#pragma unroll
                for (int a = 0; a < 4; ++a) xc[a] = P.pc[4 * a + b][bi];
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    const z2 rr = P.pr[4 * b + c][bj];
#pragma unroll
                    for (int a = 0; a < 4; ++a) t[a][c] = zfma(xc[a], rr, t[a][c]);
                }
                __builtin_amdgcn_sched_barrier(0);
            }
        }
        __syncthreads();
    }
    return 0;
}

// f(a, c, r, col, in) over the tile's entries, one at a time: the scheduling
// barrier keeps the loads of one entry from being hoisted above the previous
// entry's (all of them in flight at once would need the registers the tile
// itself occupies).
template <typename F>
__device__ __forceinline__ void for_tile(int bi, int bj, int n, F f) {
#pragma unroll
    for (int a = 0; a < 4; ++a) {
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const int r = 4 * bi + a, col = 4 * bj + c;
            f(a, c, r, col, r < n && col < n);
            __builtin_amdgcn_sched_barrier(0);
        }
    }
}

template <int TD>
__device__ void store_tile(int n, const z2 (&t)[4][4], z2* __restrict__ out) {
    const int tid = opaque(threadIdx.x);
    const int bi = tid / TD, bj = tid % TD;
    for_tile(bi, bj, n, [&](int a, int c, int r, int col, bool in) {
        if (in) out[(int64_t)r * n + col] = t[a][c];
    });
}

template <int TD>
__device__ void store_nan(int n, z2* __restrict__ out) {
    const int bi = threadIdx.x / TD, bj = threadIdx.x % TD;
    for_tile(bi, bj, n, [&](int a, int c, int r, int col, bool in) {
        if (in) out[(int64_t)r * n + col] = z2{NAN, NAN};
    });
}

// ------------------------------------------- Gauss-Jordan inverse -------
// U^{-1} of a Hermitian positive-definite matrix in place on the register
// tiles, by block Gauss-Jordan elimination with the 4 x 4 diagonal blocks as
// pivots (no pivoting: U is positive definite).  Step K, with P = A_KK:
//   A_KK <- P^{-1},  A_Kj <- P^{-1} A_Kj,  A_iK <- -A_iK P^{-1},
//   A_ij <- A_ij - A_iK P^{-1} A_Kj   (i, j != K).
// One pass of T steps replaces the factorization, the triangular inverse and
// the product R^{-1} R^{-dag}; each step's serial part is one 4 x 4 inverse.
// The diagonal blocks' Cholesky pivots are those of U's own factorization, so
// the positive-definiteness test is the same (R_jj^2 > PIVOT_RTOL max_i U_ii).
template <int TD>
struct GJShared {
    z2 pinv[2][16];   // P^{-1} of the step (double-buffered by step parity)
    z2 cp[2][16][TD]; // column panel A_iK before the step, element-major
    z2 rp[16][TD];    // row panel P^{-1} A_Kj, element-major
};

// In-place P <- P^{-1} for a Hermitian positive-definite 4 x 4 tile (upper
// triangle read); pivots of rows < nvalid are tested against thr.  The
// inverse goes to out (16 entries, row-major); p keeps R^{-1}.
__device__ __forceinline__ int hpd_inv4(z2 (&p)[4][4], double thr, int nvalid, z2* __restrict__ out) {
    int f = 0;
    double ri[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        double d = p[r][r].x;
        if (r < nvalid && !(d > thr)) f = 1;
        if (!(d > 0.0)) d = 1.0;  // keeps the arithmetic finite after a failure
        const double y = rsqrt_nr(d);
        ri[r] = y;
        p[r][r] = z2{d * y, 0.0};
#pragma unroll
        for (int c = r + 1; c < 4; ++c) p[r][c] = zscale(p[r][c], y);
#pragma unroll
        for (int s = r + 1; s < 4; ++s)
#pragma unroll
            for (int c = s; c < 4; ++c) p[s][c] = zcfms(p[r][s], p[r][c], p[s][c]);
    }
    // X = R^{-1} in place, column by column (X_ii = 1 / R_ii)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
#pragma unroll
        for (int i = 0; i < j; ++i) {
            z2 s = zscale(p[i][j], ri[i]);
#pragma unroll
            for (int k = i + 1; k < j; ++k) s = zfma(p[i][k], p[k][j], s);
            p[i][j] = zscale(s, -ri[j]);
        }
        p[j][j] = z2{ri[j], 0.0};
    }
    // P^{-1} = X X^dag
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            z2 s = z2{0.0, 0.0};
#pragma unroll
            for (int k = (a > b ? a : b); k < 4; ++k) s = zfmac(p[a][k], p[b][k], s);
            out[4 * a + b] = s;
        }
    return f;
}

// t: this thread's tile of U (every tile of the T x T grid; identity beyond
// n).  On success t holds its tile of U^{-1}; returns 1 (uniformly) on a
// failed pivot test.
template <int TD>
__device__ __attribute__((always_inline)) int gj_inverse_tiles(int n, z2 (&t)[4][4], GJShared<TD>& G,
                                                               TileShared<TD>& S) {
    const int tid = threadIdx.x, bi = tid / TD, bj = tid % TD;
    const int T = (n + 3) >> 2;
    const bool in = bi < T && bj < T;
    double m = 0.0;
    if (bi == bj && in) {
#pragma unroll
        for (int a = 0; a < 4; ++a)
            if (4 * bi + a < n) m = fmax(m, t[a][a].x);
    }
    if (tid == 0) S.fail = 0;
    const double thr = PIVOT_RTOL * block_max<TD>(m, S);
#pragma unroll 1
    for (int K = 0; K < T; ++K) {
        const int b = K & 1;
        // the pivot block's inverse (its owner), and the column panel
        if (bi == K && bj == K) {
            if (hpd_inv4(t, thr, n - 4 * K, G.pinv[b])) S.fail = 1;
        }
        if (bj == K && bi != K && bi < T) {
#pragma unroll
            for (int a = 0; a < 4; ++a)
#pragma unroll
                for (int c = 0; c < 4; ++c) G.cp[b][4 * a + c][bi] = t[a][c];
        }
        __syncthreads();
        if (S.fail) break;  // uniform: read after the barrier
        // row panel P^{-1} A_Kj (A_KK <- P^{-1})
        if (bi == K && bj < T) {
            if (bj == K) {
#pragma unroll
                for (int a = 0; a < 4; ++a)
#pragma unroll
                    for (int c = 0; c < 4; ++c) t[a][c] = G.pinv[b][4 * a + c];
            } else {
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    // (re-read per column: 16 entries kept live would not fit beside the tile)
                    const z2* pv = G.pinv[b] + opaque(0);
                    z2 o[4];
#pragma unroll
                    for (int a = 0; a < 4; ++a) {
                        z2 s = z2{0.0, 0.0};
#pragma unroll
                        for (int k = 0; k < 4; ++k) s = zfma(pv[4 * a + k], t[k][c], s);
                        o[a] = s;
                    }
#pragma unroll
                    for (int a = 0; a < 4; ++a) {
                        t[a][c] = o[a];
                        G.rp[4 * a + c][bj] = o[a];
                    }
                }
            }
        }
        __syncthreads();
        // elimination in the other block rows
        if (bi != K && in) {
            if (bj != K) {
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    z2 ci[4];
                    const int ob = opaque(0);
#pragma unroll
                    for (int a = 0; a < 4; ++a) ci[a] = G.cp[b][4 * a + k][bi + ob];
#pragma unroll
                    for (int c = 0; c < 4; ++c) {
                        const z2 r = G.rp[4 * k + c][bj];
#pragma unroll
                        for (int a = 0; a < 4; ++a) t[a][c] = zfms(ci[a], r, t[a][c]);
                    }
                    __builtin_amdgcn_sched_barrier(0);
                }
            } else {
#pragma unroll
                for (int a = 0; a < 4; ++a) {
                    const z2* pv = G.pinv[b] + opaque(0);
                    z2 o[4];
#pragma unroll
                    for (int c = 0; c < 4; ++c) {
                        z2 s = z2{0.0, 0.0};
#pragma unroll
                        for (int k = 0; k < 4; ++k) s = zfma(t[a][k], pv[4 * k + c], s);
                        o[c] = s;
                    }
#pragma unroll
                    for (int c = 0; c < 4; ++c) t[a][c] = z2{-o[c].x, -o[c].y};
                }
            }
        }
    }
    const int failed = S.fail;
    __syncthreads();
    return failed;
}

// ---------------------------------------------------------- kernels ---------
// Cholesky inverse Rinv = R^{-1} (upper, zero below) of every matrix.
template <int TD>
__global__ void __launch_bounds__(TD* TD)
k_cholesky_tiles(const Seg* __restrict__ seg, int nbo, int n0, const z2* __restrict__ U, z2* __restrict__ Rinv,
                 int* __restrict__ status, const int* __restrict__ act) {
    if (act && !act[blockIdx.x]) return;
    __shared__ CholPanels<TD> P;
    __shared__ TileShared<TD> S;
    const Mat M = mat_of(seg, nbo, n0, blockIdx.x);
    const int n = M.n;
    const int bi = threadIdx.x / TD, bj = threadIdx.x % TD;
    const z2* Ug = U + M.moff;
    z2 t[4][4];
    for_tile(bi, bj, n, [&](int a, int c, int r, int col, bool in) {
        t[a][c] = (in && bi <= bj) ? Ug[(int64_t)r * n + col] : z2{r == col ? 1.0 : 0.0, 0.0};
    });
    const int f = chol_inv_tiles<TD>(n, t, P, S);
    z2* X = Rinv + M.moff;
    if (f) {
        if (threadIdx.x == 0 && status) atomicOr(status, DPP_STATUS_NOTPD);
        store_nan<TD>(n, X);
        return;
    }
    store_tile<TD>(n, t, X);
}

// Band-gradient preparation per item: (with `step`) U and H0 advanced along
// the line matrices, U <- U + a (X + X^dag) + a^2 Q, H0 <- H0 + a (H1 + H1^dag)
// + a^2 H2, and written back; then M1 = U^{-1} and E0 = Re Tr(U^{-1} H0).
// On a failed pivot test M1 and E0 are NaN and the status word latches
// DPP_STATUS_NOTPD.
template <int TD>
__global__ void __launch_bounds__(TD* TD)
k_grad_prep_tiles(const Seg* __restrict__ seg, z2* __restrict__ U, z2* __restrict__ H0, z2* __restrict__ M1,
                  double* __restrict__ E0, int* __restrict__ status, const double* __restrict__ step,
                  const z2* __restrict__ X, const z2* __restrict__ Q, const z2* __restrict__ H1,
                  const z2* __restrict__ H2) {
    __shared__ GJShared<TD> G;
    __shared__ TileShared<TD> S;
    const Mat M = mat_of(seg, 0, 0, blockIdx.x);
    const int n = M.n;
    const int64_t o = M.moff;
    const int bi = threadIdx.x / TD, bj = threadIdx.x % TD;
    const double al = step ? step[blockIdx.x] : 0.0;
    const bool adv = step && al != 0.0;
    if (adv) {
        for_tile(bi, bj, n, [&](int a, int c, int r, int col, bool in) {
            if (in) {
                const int64_t e = o + (int64_t)r * n + col, et = o + (int64_t)col * n + r;
                const z2 h = H0[e], p = H1[e], pt = H1[et], h2 = H2[e];
                H0[e] = z2{h.x + al * (p.x + pt.x) + al * al * h2.x, h.y + al * (p.y - pt.y) + al * al * h2.y};
            }
        });
    }
    z2 t[4][4];
    for_tile(bi, bj, n, [&](int a, int c, int r, int col, bool in) {
        z2 u = z2{r == col ? 1.0 : 0.0, 0.0};
        if (in) {
            const int64_t e = o + (int64_t)r * n + col, et = o + (int64_t)col * n + r;
            u = U[e];
            if (adv) {
                const z2 x = X[e], xt = X[et], q = Q[e];
                u = z2{u.x + al * (x.x + xt.x) + al * al * q.x, u.y + al * (x.y - xt.y) + al * al * q.y};
                U[e] = u;
            }
        }
        t[a][c] = u;
    });
    if (gj_inverse_tiles<TD>(n, t, G, S)) {
        if (threadIdx.x == 0) {
            if (status) atomicOr(status, DPP_STATUS_NOTPD);
            E0[blockIdx.x] = NAN;
        }
        store_nan<TD>(n, M1 + o);
        return;
    }
    store_tile<TD>(n, t, M1 + o);
    // Re Tr(M1 H0) = sum over entries of Re(conj(M1) H0) (both Hermitian)
    double e = 0.0;
    for_tile(bi, bj, n, [&](int a, int c, int r, int col, bool in) {
        if (in) {
            const z2 h = H0[o + (int64_t)r * n + col];
            e += t[a][c].x * h.x + t[a][c].y * h.y;
        }
    });
    e = block_sum<TD>(e, S);
    if (threadIdx.x == 0) E0[blockIdx.x] = e;
}

// Band-energy line search of every active item (the rule of the single-wave
// kernel): E(a) = Re Tr(U(a)^{-1} H(a)), U(a) = U + a (X + X^dag) + a^2 Q,
// H(a) = H0 + a (H1 + H1^dag) + a^2 H2; trial a_t, fit E0 + d0 a + c a^2,
// a* = -d0 / (2c) if c > 0 else 2 a_t, at most 10 a_t; accept a* if
// E(a*) <= E0, else a_t if E(a_t) <= E0, else halve a_t (LS_TRIES times).
// A trial whose U(a) fails the pivot test has E = NaN and is rejected.
constexpr int LS_TRIES = 6;

template <int TD>
__device__ __attribute__((noinline)) double trial_energy_tiles(const Mat& M, double al, const z2* __restrict__ U,
                                                                    const z2* __restrict__ X,
                                                                    const z2* __restrict__ Q,
                                                                    const z2* __restrict__ H0,
                                                                    const z2* __restrict__ H1,
                                                                    const z2* __restrict__ H2, GJShared<TD>& G,
                                                                    TileShared<TD>& S) {
    const int n = M.n;
    const int64_t o = M.moff;
    const int bi = threadIdx.x / TD, bj = threadIdx.x % TD;
    z2 t[4][4];
    for_tile(bi, bj, n, [&](int a, int c, int r, int col, bool in) {
        z2 u = z2{r == col ? 1.0 : 0.0, 0.0};
        if (in) {
            const int64_t e = o + (int64_t)r * n + col, et = o + (int64_t)col * n + r;
            const z2 x = X[e], xt = X[et], q = Q[e];
            u = U[e];
            u = z2{u.x + al * (x.x + xt.x) + al * al * q.x, u.y + al * (x.y - xt.y) + al * al * q.y};
        }
        t[a][c] = u;
    });
    if (gj_inverse_tiles<TD>(n, t, G, S)) return NAN;
    double e = 0.0;
    for_tile(bi, bj, n, [&](int a, int c, int r, int col, bool in) {
        if (in) {
            const int64_t ei = o + (int64_t)r * n + col, et = o + (int64_t)col * n + r;
            const z2 h0 = H0[ei], p = H1[ei], pt = H1[et], h2 = H2[ei];
            const double hr = h0.x + al * (p.x + pt.x) + al * al * h2.x;
            const double hi = h0.y + al * (p.y - pt.y) + al * al * h2.y;
            e += t[a][c].x * hr + t[a][c].y * hi;
        }
    });
    return block_sum<TD>(e, S);
}

template <int TD>
__global__ void __launch_bounds__(TD* TD)
k_linesearch_tiles(const Seg* __restrict__ seg, const z2* __restrict__ U, const z2* __restrict__ X,
                   const z2* __restrict__ Q, const z2* __restrict__ H0, const z2* __restrict__ H1,
                   const z2* __restrict__ H2, const double* __restrict__ E0v, const double* __restrict__ at0,
                   const double* __restrict__ d0v, const int* __restrict__ act, int* __restrict__ ok,
                   double* __restrict__ step) {
    const int k = blockIdx.x;
    if (!act[k]) return;
    __shared__ GJShared<TD> G;
    __shared__ TileShared<TD> S;
    const Mat M = mat_of(seg, 0, 0, k);
    const double E0 = E0v[k], d0 = d0v[k];
    double at = at0[k];
    int good = 0;
    double st = 0.0;
#pragma unroll 1
    for (int tr = 0; tr < LS_TRIES; ++tr) {
        const double Et = trial_energy_tiles<TD>(M, at, U, X, Q, H0, H1, H2, G, S);
        const double c = (Et - E0 - d0 * at) / (at * at);
        double as = c > 0 ? -d0 / (2.0 * c) : 2.0 * at;
        as = fmin(as, 10.0 * at);
        const double Es = trial_energy_tiles<TD>(M, as, U, X, Q, H0, H1, H2, G, S);
        if (Es <= E0) {
            good = 1;
            st = as;
            break;
        }
        if (Et <= E0) {
            good = 1;
            st = at;
            break;
        }
        at *= 0.5;
    }
    if (threadIdx.x == 0) {
        ok[k] = good;
        step[k] = st;
    }
}

// ------------------------------------------------------ eigensolver -------
// H = Q T Q^dag with T real symmetric tridiagonal: Householder reflectors
// H_k = I - tau_k v_k v_k^dag (v_k zero above k+1, v_k[k+1] = 1) chosen so
// that H_k^dag maps column k below the diagonal onto beta_k e_1 with beta_k
// real (the convention of the standard complex elementary reflector), applied
// two-sided to the trailing block as A <- A - v w^dag - w v^dag with
// w = tau A v - (|tau|^2 / 2)(v^dag A v) v.  The last subdiagonal entry c is
// made real by the phase p = c / |c| on the last row.  T's eigenvalues come
// from bisection on Sturm counts, its eigenvectors Z from inverse iteration
// (Gaussian elimination with partial pivoting, eigenvalues closer than
// 1e-3 ||T|| in a cluster orthogonalized against each other inside the
// iteration), and the eigenvectors of H are Q P Z.
constexpr int EIGH_WS_PER_N2 = 10;  // double2 of workspace per n^2 of matrix
constexpr int BT_COLS = 16;         // columns per back-transformation workgroup
constexpr int BT_CHUNK = 16;        // reflectors staged per LDS pass

struct EighWs {
    z2* refl;     // n x n: row k = v_k
    double* Z;    // n x n column-major: column g = eigenvector g of T
    double *d, *e, *lam, *gl, *gu, *ortol;
    z2* tau;      // n
    z2* ph;       // 1
    int *bs, *be;  // block [bs, be) of each index after splitting
    double* lu;    // 3 n x n: LU rows of the inverse iteration, 3n per eigenvalue index
};

__host__ __device__ inline EighWs eigh_ws(z2* base, int n) {
    EighWs w;
    w.refl = base;
    double* p = reinterpret_cast<double*>(base + (size_t)n * n);
    w.Z = p;
    p += (size_t)n * n;
    w.d = p;
    w.e = p + n;
    w.lam = p + 2 * n;
    w.gl = p + 3 * n;
    w.gu = p + 4 * n;
    w.ortol = p + 5 * n;
    p += 6 * n;
    w.tau = reinterpret_cast<z2*>(p);
    w.ph = w.tau + n;
    int* q = reinterpret_cast<int*>(w.ph + 1);
    w.bs = q;
    w.be = q + n;
    w.lu = reinterpret_cast<double*>(q + 2 * n);
    return w;
}

// Per-matrix base of the workspace.
__device__ __forceinline__ z2* eigh_base(z2* ws, const Seg* seg, int n0, int b) {
    if (seg) return ws + (int64_t)EIGH_WS_PER_N2 * seg[b].moff;
    return ws + (int64_t)EIGH_WS_PER_N2 * b * n0 * n0;
}

// Vectors of length n are stored permuted, row r at (r % 4)(TD + 1) + r / 4:
// the lanes of a wave read entry c of consecutive tiles (rows 4j + c) and
// consecutive rows from consecutive 16-byte words.  The partial products are
// [row][tile column] with a padded row.
template <int TD>
struct TriShared {
    static constexpr int PS = TD + 1;
    z2 xb[2][4 * PS];
    z2 yb[4 * PS];
    z2 vb[4 * PS];
    z2 part[4 * TD][PS];
    double d[4 * TD], e[4 * TD];
    z2 clast;
};

template <int TD>
__device__ __forceinline__ int vperm(int r) { return (r & 3) * (TD + 1) + (r >> 2); }

template <int TD>
__global__ void __launch_bounds__(TD* TD)
k_eigh_tridiag(const Seg* __restrict__ seg, int n0, const z2* __restrict__ H, z2* __restrict__ ws) {
    __shared__ TriShared<TD> L;
    const Mat M = mat_of(seg, 0, n0, blockIdx.x);
    const int n = M.n;
    const int tid = threadIdx.x, lane = tid & 63;
    const int bi = tid / TD, bj = tid % TD;
    const int T = (n + 3) >> 2;
    const EighWs W = eigh_ws(eigh_base(ws, seg, n0, blockIdx.x), n);
    const z2* Hg = H + M.moff;
    // tiles of the Hermitian matrix from its lower triangle (real diagonal)
    z2 t[4][4];
    for_tile(bi, bj, n, [&](int a, int c, int r, int col, bool in) {
        z2 v = z2{0.0, 0.0};
        if (in) {
            if (r > col)
                v = Hg[(int64_t)r * n + col];
            else if (r < col)
                v = zconj(Hg[(int64_t)col * n + r]);
            else
                v = z2{Hg[(int64_t)r * n + col].x, 0.0};
        }
        t[a][c] = v;
    });
#pragma unroll 1
    for (int k = 0; k + 2 < n; ++k) {
        const int kb = k >> 2, kc = k & 3;
        z2* xb = L.xb[k & 1];
        // column k below the diagonal, and d_k
        if (bj == kb && bi < T) {
#pragma unroll
            for (int a = 0; a < 4; ++a) {
                const int r = 4 * bi + a;
                z2 v = z2{0.0, 0.0};
#pragma unroll
                for (int c = 0; c < 4; ++c)
                    if (c == kc) v = t[a][c];
                if (r > k && r < n) xb[vperm<TD>(r)] = v;
                if (r == k) L.d[k] = v.x;
            }
        }
        __syncthreads();
        // the reflector (every wave computes it, identically)
        const z2 al = xb[vperm<TD>(k + 1)];
        double xn2 = 0.0;
        for (int r = k + 2 + lane; r < n; r += 64) {
            const z2 x = xb[vperm<TD>(r)];
            xn2 += x.x * x.x + x.y * x.y;
        }
        xn2 = wsum(xn2);
        z2 tau = z2{0.0, 0.0}, sc = z2{0.0, 0.0};
        double beta = al.x;
        if (!(xn2 == 0.0 && al.y == 0.0)) {
            beta = -copysign(sqrt(al.x * al.x + al.y * al.y + xn2), al.x);
            tau = z2{(beta - al.x) / beta, -al.y / beta};
            const z2 zz = z2{al.x - beta, al.y};
            const double m2 = zz.x * zz.x + zz.y * zz.y;
            sc = z2{zz.x / m2, -zz.y / m2};
        }
        auto vof = [&](int r) -> z2 {
            return r == k + 1 ? z2{1.0, 0.0} : (r > k + 1 && r < n ? zmul(xb[vperm<TD>(r)], sc) : z2{0.0, 0.0});
        };
        if (tid < 64) {
            for (int r = lane; r < n; r += 64) W.refl[(int64_t)k * n + r] = vof(r);
            if (lane == 0) {
                W.tau[k] = tau;
                L.e[k] = beta;
            }
        }
        // partial products of A v over the trailing block
        const bool trail = bi < T && bj < T && 4 * bi + 3 > k && 4 * bj + 3 > k;
        if (trail) {
            z2 vj[4];
#pragma unroll
            for (int c = 0; c < 4; ++c) vj[c] = vof(4 * bj + c);
#pragma unroll
            for (int a = 0; a < 4; ++a) {
                z2 p = z2{0.0, 0.0};
#pragma unroll
                for (int c = 0; c < 4; ++c) p = zfma(t[a][c], vj[c], p);
                L.part[4 * bi + a][bj] = p;
            }
        }
        __syncthreads();
        // y = A v on rows > k: TD/4 lanes per row, four partials each; v and y
        // (zero outside rows k+1..n-1) into LDS for the update
        {
            constexpr int LPR = TD / 4;
            const int r = tid / LPR, s = tid % LPR;
            const bool live = r > k && r < n;
            z2 y = z2{0.0, 0.0};
            if (live) {
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int b = s + LPR * q;
                    if (b < T && 4 * b + 3 > k) y = zadd(y, L.part[r][b]);
                }
            }
#pragma unroll
            for (int o = 1; o < LPR; o <<= 1) {
                y.x += __shfl_xor(y.x, o);
                y.y += __shfl_xor(y.y, o);
            }
            if (s == 0) {
                L.yb[vperm<TD>(r)] = live ? y : z2{0.0, 0.0};
                L.vb[vperm<TD>(r)] = vof(r);
            }
        }
        __syncthreads();
        // A <- A - v w^dag - w v^dag, w = tau y - (|tau|^2/2)(v^dag y) v
        double sv = 0.0;
        for (int r = k + 1 + lane; r < n; r += 64) {
            const z2 v = L.vb[vperm<TD>(r)], y = L.yb[vperm<TD>(r)];
            sv += v.x * y.x + v.y * y.y;
        }
        sv = wsum(sv);
        const double coef = 0.5 * (tau.x * tau.x + tau.y * tau.y) * sv;
        if (trail) {
            z2 vc[4], wc[4];
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                vc[c] = L.vb[vperm<TD>(4 * bj + c)];
                const z2 ty = zmul(tau, L.yb[vperm<TD>(4 * bj + c)]);
                wc[c] = z2{ty.x - coef * vc[c].x, ty.y - coef * vc[c].y};
            }
#pragma unroll
            for (int a = 0; a < 4; ++a) {
                const z2 vr = L.vb[vperm<TD>(4 * bi + a)];
                const z2 ty = zmul(tau, L.yb[vperm<TD>(4 * bi + a)]);
                const z2 wr = z2{ty.x - coef * vr.x, ty.y - coef * vr.y};
#pragma unroll
                for (int c = 0; c < 4; ++c)
                    t[a][c] = zfmsc(wr, vc[c], zfmsc(vr, wc[c], t[a][c]));
            }
        }
    }
    // the last 2 x 2 block
    if (bi < T && bj < T) {
        for_tile(bi, bj, n, [&](int a, int c, int r, int col, bool in) {
            if (in && r == col && r >= n - 2) L.d[r] = t[a][c].x;
            if (in && r == n - 1 && col == n - 2) L.clast = t[a][c];
        });
    }
    __syncthreads();
    if (tid == 0) {
        z2 ph = z2{1.0, 0.0};
        if (n >= 2) {
            const z2 c = L.clast;
            const double ac = sqrt(c.x * c.x + c.y * c.y);
            if (ac > 0.0) ph = z2{c.x / ac, c.y / ac};
            L.e[n - 2] = ac;
        }
        *W.ph = ph;
        // split where e_i^2 is below ulp^2 |d_i d_{i+1}| (+ the smallest
        // normal); per block the Gershgorin interval and the cluster width
        int s = 0;
        for (int i = 0; i < n; ++i) {
            const bool last = i == n - 1 ||
                              L.e[i] * L.e[i] <= DBL_EPSILON * DBL_EPSILON * fabs(L.d[i] * L.d[i + 1]) + DBL_MIN;
            W.d[i] = L.d[i];
            W.e[i] = i < n - 1 ? (last ? 0.0 : L.e[i]) : 0.0;
            if (last) {
                double lo = DBL_MAX, hi = -DBL_MAX, nrm = 0.0;
                for (int j = s; j <= i; ++j) {
                    const double el = j > s ? fabs(L.e[j - 1]) : 0.0, er = j < i ? fabs(L.e[j]) : 0.0;
                    lo = fmin(lo, L.d[j] - el - er);
                    hi = fmax(hi, L.d[j] + el + er);
                    nrm = fmax(nrm, fabs(L.d[j]) + el + er);
                }
                const double pad = 2.0 * (i - s + 1) * DBL_EPSILON * nrm + 4.0 * DBL_MIN;
                for (int j = s; j <= i; ++j) {
                    W.bs[j] = s;
                    W.be[j] = i + 1;
                    W.gl[j] = lo - pad;
                    W.gu[j] = hi + pad;
                    W.ortol[j] = 1e-3 * nrm;
                }
                s = i + 1;
            }
        }
    }
}

// Number of eigenvalues below x of the block's tridiagonal (Sturm count).
__device__ __forceinline__ int sturm_count(int m, const double* d, const double* e2, double x, double pivmin) {
    int c = 0;
    double q = d[0] - x;
    if (fabs(q) < pivmin) q = -pivmin;
    c += q < 0.0;
    for (int j = 1; j < m; ++j) {
        q = (d[j] - x) - e2[j - 1] / q;
        if (fabs(q) < pivmin) q = -pivmin;
        c += q < 0.0;
    }
    return c;
}

// Eigenvalue g of the tridiagonal: the (g - bs)-th smallest of its block, by
// 65-section (each lane counts at one of 64 interior points per pass).
__global__ void __launch_bounds__(64)
k_eigh_bisect(const Seg* __restrict__ seg, int n0, z2* __restrict__ ws) {
    __shared__ double d[EIG_TILE_MAXN], e2[EIG_TILE_MAXN];
    const Mat M = mat_of(seg, 0, n0, blockIdx.y);
    const int n = M.n, g = blockIdx.x, lane = threadIdx.x;
    if (g >= n) return;
    const EighWs W = eigh_ws(eigh_base(ws, seg, n0, blockIdx.y), n);
    const int s = W.bs[g], m = W.be[g] - s, i = g - s;
    double em = 0.0;
    for (int j = lane; j < m; j += 64) {
        d[j] = W.d[s + j];
        const double ev = j + 1 < m ? W.e[s + j] : 0.0;
        e2[j] = ev * ev;
        em = fmax(em, ev * ev);
    }
    const double pivmin = DBL_MIN * fmax(1.0, wmax(em));
    __syncthreads();
    double lo = W.gl[g], hi = W.gu[g];
    for (int it = 0; it < 14; ++it) {
        const double h = (hi - lo) * (1.0 / 65.0);
        const double x = fmin(fmax(lo + (lane + 1) * h, lo), hi);
        const int c = sturm_count(m, d, e2, x, pivmin);
        // lanes counting at most i eigenvalues below their point
        const unsigned long long below = __ballot(c <= i);
        const unsigned long long above = __ballot(c > i);
        double nlo = lo, nhi = hi;
        if (below) nlo = __shfl(x, 63 - __clzll((long long)below));
        if (above) nhi = __shfl(x, __ffsll((long long)above) - 1);
        if (nlo > nhi) nlo = nhi = 0.5 * (nlo + nhi);  // a non-monotone count: stop here
        const bool done = !(nhi - nlo > 2.0 * DBL_EPSILON * fmax(fabs(nlo), fabs(nhi)) + DBL_MIN) ||
                          (nlo == lo && nhi == hi);
        lo = nlo;
        hi = nhi;
        if (done) break;
    }
    if (lane == 0) W.lam[g] = 0.5 * (lo + hi);
}

// Eigenvector(s) of the tridiagonal by inverse iteration, one wave per
// cluster leader; every wave also writes its eigenvalue at its rank in the
// ascending order (ties by index) and the column that holds its vector.
__device__ __forceinline__ double start_value(int r, int m) {
    unsigned h = (unsigned)r * 2654435761u ^ ((unsigned)m + 1u) * 40503u;
    h ^= h >> 15;
    h *= 2246822519u;
    h ^= h >> 13;
    return (double)(h >> 8) * (1.0 / 16777216.0) - 0.5;
}

// (T - lm) x = rhs in place on one block of m rows, by elimination with
// partial pivoting (one thread): row j of the upper factor is (u0, u1, u2) at
// columns j, j+1, j+2.  A zero pivot is replaced by pivmin.
__device__ void tri_solve(int m, const double* __restrict__ d, const double* __restrict__ e, double lm,
                          double pivmin, double* __restrict__ x, double* __restrict__ u0, double* __restrict__ u1,
                          double* __restrict__ u2) {
    double p0 = d[0] - lm, p1 = m > 1 ? e[0] : 0.0, p2 = 0.0;
    double ri = x[0];
    for (int j = 0; j + 1 < m; ++j) {
        double q0 = e[j], q1 = d[j + 1] - lm, q2 = j + 2 < m ? e[j + 1] : 0.0;
        double rn = x[j + 1];
        if (fabs(q0) > fabs(p0)) {
            double tq = p0;
            p0 = q0;
            q0 = tq;
            tq = p1;
            p1 = q1;
            q1 = tq;
            tq = p2;
            p2 = q2;
            q2 = tq;
            tq = ri;
            ri = rn;
            rn = tq;
        }
        if (p0 == 0.0) p0 = pivmin;
        const double mu = q0 / p0;
        u0[j] = p0;
        u1[j] = p1;
        u2[j] = p2;
        x[j] = ri;
        ri = rn - mu * ri;
        p0 = q1 - mu * p1;
        p1 = q2 - mu * p2;
        p2 = 0.0;
    }
    if (fabs(p0) < pivmin) p0 = p0 < 0.0 ? -pivmin : pivmin;
    u0[m - 1] = p0;
    x[m - 1] = ri;
    for (int j = m - 1; j >= 0; --j) {
        double tt = x[j];
        if (j + 1 < m) tt -= u1[j] * x[j + 1];
        if (j + 2 < m) tt -= u2[j] * x[j + 2];
        x[j] = tt / u0[j];
    }
}

// x <- x / |x| over m entries (scaled by the largest entry first), one wave.
__device__ __forceinline__ void wave_normalize(int m, double* __restrict__ x) {
    const int lane = threadIdx.x;
    double xm = 0.0;
    for (int j = lane; j < m; j += 64) xm = fmax(xm, fabs(x[j]));
    xm = wmax(xm);
    const double isc = xm > 0.0 ? 1.0 / xm : 1.0;
    double nr = 0.0;
    for (int j = lane; j < m; j += 64) {
        x[j] *= isc;
        nr += x[j] * x[j];
    }
    nr = wsum(nr);
    const double inr = 1.0 / sqrt(nr);
    for (int j = lane; j < m; j += 64) x[j] *= inr;
}

// Clusters of up to CL_MAX eigenvalues run as a block: every member's inverse
// iteration in its own lane, the block orthonormalized (modified Gram-Schmidt)
// after each iteration, then a Rayleigh-Ritz step: K = X^T T X, K = V diag V^T
// by parallel-order Jacobi, eigenvectors X V in ascending order.
constexpr int CL_MAX = 48;
constexpr int KLD = CL_MAX + 1;
constexpr int XLD = EIG_TILE_MAXN + 1;  // odd row stride: lanes walking their own rows hit different banks

// Real symmetric eigen-decomposition of K (mc x mc, row stride KLD, LDS) in
// one wave: parallel-order cyclic Jacobi (round-robin pairs), V accumulated.
__device__ void jacobi_small(int mc, double* __restrict__ K, double* __restrict__ V, int* __restrict__ rp,
                             double* __restrict__ rc) {
    const int lane = threadIdx.x;
    const int m2 = mc + (mc & 1);
    for (int i = lane; i < mc * KLD; i += 64) V[i] = 0.0;
    __syncthreads();
    for (int i = lane; i < mc; i += 64) V[i * KLD + i] = 1.0;
    __syncthreads();
    for (int sweep = 0; sweep < 30; ++sweep) {
        double off = 0.0, all = 0.0;
        for (int i = lane; i < mc * mc; i += 64) {
            const int r = i / mc, c = i - r * mc;
            const double v = K[r * KLD + c];
            all += v * v;
            if (r != c) off += v * v;
        }
        off = wsum(off);
        all = wsum(all);
        if (!(off > fmax(1e-28, 4e-32 * (double)mc * (double)mc) * all)) break;
        for (int round = 0; round < m2 - 1; ++round) {
            if (lane < m2 / 2) {
                int p, q;
                if (lane == 0) {
                    p = m2 - 1;
                    q = round;
                } else {
                    p = (round + lane) % (m2 - 1);
                    q = (round - lane + (m2 - 1)) % (m2 - 1);
                }
                if (p > q) {
                    const int t = p;
                    p = q;
                    q = t;
                }
                double c = 1.0, sn = 0.0;
                if (q < mc) {
                    const double apq = K[p * KLD + q];
                    if (apq != 0.0) {
                        const double tau = (K[q * KLD + q] - K[p * KLD + p]) / (2.0 * apq);
                        const double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
                        c = 1.0 / sqrt(1.0 + t * t);
                        sn = t * c;
                    }
                } else {
                    q = p;  // paired with the dummy: identity
                }
                rp[2 * lane] = p;
                rp[2 * lane + 1] = q;
                rc[2 * lane] = c;
                rc[2 * lane + 1] = sn;
            }
            __syncthreads();
            // columns: K <- K J and V <- V J (lanes over rows)
            for (int i = lane; i < mc; i += 64) {
                for (int s2 = 0; s2 < m2 / 2; ++s2) {
                    const int p = rp[2 * s2], q = rp[2 * s2 + 1];
                    if (p == q) continue;
                    const double c = rc[2 * s2], sn = rc[2 * s2 + 1];
                    const double kp = K[i * KLD + p], kq = K[i * KLD + q];
                    K[i * KLD + p] = c * kp - sn * kq;
                    K[i * KLD + q] = sn * kp + c * kq;
                    const double vp = V[i * KLD + p], vq = V[i * KLD + q];
                    V[i * KLD + p] = c * vp - sn * vq;
                    V[i * KLD + q] = sn * vp + c * vq;
                }
            }
            __syncthreads();
            // rows: K <- J^T K (lanes over columns)
            for (int i = lane; i < mc; i += 64) {
                for (int s2 = 0; s2 < m2 / 2; ++s2) {
                    const int p = rp[2 * s2], q = rp[2 * s2 + 1];
                    if (p == q) continue;
                    const double c = rc[2 * s2], sn = rc[2 * s2 + 1];
                    const double kp = K[p * KLD + i], kq = K[q * KLD + i];
                    K[p * KLD + i] = c * kp - sn * kq;
                    K[q * KLD + i] = sn * kp + c * kq;
                }
            }
            __syncthreads();
        }
    }
}

__global__ void __launch_bounds__(64)
k_eigh_invit(const Seg* __restrict__ seg, int n0, z2* __restrict__ ws, double* __restrict__ eig,
             int* __restrict__ perm_out) {
    __shared__ double lam[EIG_TILE_MAXN], d[EIG_TILE_MAXN], e[EIG_TILE_MAXN];
    __shared__ double Xs[CL_MAX * XLD];  // cluster vectors, member-major
    __shared__ double Ws[CL_MAX * XLD];  // T X; single-vector LU rows
    __shared__ double KV[2 * CL_MAX * KLD];        // Ritz matrix K and its eigenvectors V
    __shared__ int rp[64];
    __shared__ double rc[64];
    __shared__ int ord[CL_MAX];
    const Mat M = mat_of(seg, 0, n0, blockIdx.y);
    const int n = M.n, g = blockIdx.x, lane = threadIdx.x;
    if (g >= n) return;
    const EighWs W = eigh_ws(eigh_base(ws, seg, n0, blockIdx.y), n);
    for (int j = lane; j < n; j += 64) lam[j] = W.lam[j];
    __syncthreads();
    {
        const double lg = lam[g];
        double rk = 0.0;
        for (int h = lane; h < n; h += 64) rk += (lam[h] < lg || (lam[h] == lg && h < g)) ? 1.0 : 0.0;
        const int r = (int)wsum(rk);
        if (lane == 0) {
            eig[M.f_off + r] = lg;
            perm_out[(int64_t)blockIdx.y * EIG_TILE_MAXN + r] = g;
        }
    }
    const int s = W.bs[g], be = W.be[g];
    const double ortol = W.ortol[g];
    if (!(g == s || lam[g] - lam[g - 1] > ortol)) return;
    // the cluster: g and the following eigenvalues of the block closer than ortol to their predecessor
    int mc = 1;
    while (g + mc < be && lam[g + mc] - lam[g + mc - 1] <= ortol) ++mc;
    const int m = be - s;
    for (int j = lane; j < m; j += 64) {
        d[j] = W.d[s + j];
        e[j] = j + 1 < m ? W.e[s + j] : 0.0;
    }
    double tn = 0.0;
    for (int j = lane; j < m; j += 64) tn = fmax(tn, fabs(d[j]) + (j > 0 ? fabs(e[j - 1]) : 0.0) + fabs(e[j]));
    const double pivmin = DBL_EPSILON * fmax(wmax(tn), DBL_MIN);
    __syncthreads();
    if (mc >= 2 && mc <= CL_MAX) {
        for (int k = 0; k < mc; ++k)
            for (int j = lane; j < m; j += 64) Xs[k * XLD + j] = start_value(j, g + k);
        __syncthreads();
        for (int it = 0; it < 3; ++it) {
            if (lane < mc) {
                // one slice per eigenvalue index: clusters run in separate workgroups at once
                double* lu = W.lu + (int64_t)(g + lane) * 3 * n;
                tri_solve(m, d, e, lam[g + lane], pivmin, Xs + lane * XLD, lu, lu + n, lu + 2 * n);
            }
            __syncthreads();
            for (int pass = 0; pass < (it == 2 ? 2 : 1); ++pass) {
                for (int j = 0; j < mc; ++j) {
                    double* xj = Xs + j * XLD;
                    wave_normalize(m, xj);
                    __syncthreads();
                    if (lane > j && lane < mc) {
                        double* xk = Xs + lane * XLD;
                        double dt = 0.0;
                        for (int r = 0; r < m; ++r) dt += xj[r] * xk[r];
                        for (int r = 0; r < m; ++r) xk[r] -= dt * xj[r];
                    }
                    __syncthreads();
                }
            }
        }
        // Rayleigh-Ritz: Y = T X, then K = X^T Y (symmetrized)
        if (lane < mc) {
            const double* x = Xs + lane * XLD;
            double* y = Ws + lane * XLD;
            for (int r = 0; r < m; ++r) {
                double v = d[r] * x[r];
                if (r > 0) v += e[r - 1] * x[r - 1];
                if (r + 1 < m) v += e[r] * x[r + 1];
                y[r] = v;
            }
        }
        __syncthreads();
        double* K = KV;
        double* V = KV + CL_MAX * KLD;
        if (lane < mc) {
            const double* y = Ws + lane * XLD;
            for (int j = 0; j < mc; ++j) {
                const double* xj = Xs + j * XLD;
                double v = 0.0;
                for (int r = 0; r < m; ++r) v += xj[r] * y[r];
                K[j * KLD + lane] = v;
            }
        }
        __syncthreads();
        for (int i = lane; i < mc * mc; i += 64) {
            const int r = i / mc, c = i - r * mc;
            if (r < c) {
                const double v = 0.5 * (K[r * KLD + c] + K[c * KLD + r]);
                K[r * KLD + c] = v;
                K[c * KLD + r] = v;
            }
        }
        __syncthreads();
        jacobi_small(mc, K, V, rp, rc);
        // ascending order of the Ritz values (ties by index)
        if (lane < mc) {
            const double kv = K[lane * KLD + lane];
            int r = 0;
            for (int j = 0; j < mc; ++j) {
                const double kj = K[j * KLD + j];
                r += (kj < kv || (kj == kv && j < lane)) ? 1 : 0;
            }
            ord[r] = lane;
        }
        __syncthreads();
        // Z[:, g + k] = X V[:, ord[k]] on the block, zero elsewhere
        for (int k = 0; k < mc; ++k) {
            const int c = ord[k];
            double* zc = W.Z + (int64_t)(g + k) * n;
            for (int j = lane; j < n; j += 64) {
                double v = 0.0;
                if (j >= s && j < be)
                    for (int q = 0; q < mc; ++q) v += Xs[q * XLD + (j - s)] * V[q * KLD + c];
                zc[j] = v;
            }
        }
        return;
    }
    // one eigenvalue, or a cluster too large for the block: members in turn,
    // each orthogonalized against the earlier ones inside its iteration
    double* x = Ws;
    double* u0 = Ws + XLD;
    double* u1 = Ws + 2 * XLD;
    double* u2 = Ws + 3 * XLD;
    for (int g2 = g; g2 < g + mc; ++g2) {
        const double lm = lam[g2];
        for (int j = lane; j < m; j += 64) x[j] = start_value(j, g2);
        __syncthreads();
        for (int it = 0; it < 3; ++it) {
            if (lane == 0) tri_solve(m, d, e, lm, pivmin, x, u0, u1, u2);
            __syncthreads();
            for (int p = g; p < g2; ++p) {
                const double* zp = W.Z + (int64_t)p * n + s;
                double dt = 0.0;
                for (int j = lane; j < m; j += 64) dt += zp[j] * x[j];
                dt = wsum(dt);
                for (int j = lane; j < m; j += 64) x[j] -= dt * zp[j];
                __syncthreads();
            }
            wave_normalize(m, x);
            __syncthreads();
        }
        double* zc = W.Z + (int64_t)g2 * n;
        for (int j = lane; j < n; j += 64) zc[j] = (j >= s && j < be) ? x[j - s] : 0.0;
        __syncthreads();
    }
}

// Eigenvectors of H in ascending order of the eigenvalues: column c of the
// output is Q P Z[:, perm[c]], the reflectors applied last to first, BT_CHUNK
// at a time from LDS; 16 lanes per column, each holding rows s, s + 16, ...
__global__ void __launch_bounds__(256)
k_eigh_back(const Seg* __restrict__ seg, int n0, z2* __restrict__ ws, const int* __restrict__ perm,
            z2* __restrict__ vecs) {
    __shared__ z2 vs[BT_CHUNK][EIG_TILE_MAXN];
    __shared__ z2 ts[BT_CHUNK];
    const Mat M = mat_of(seg, 0, n0, blockIdx.y);
    const int n = M.n;
    const int c0 = blockIdx.x * BT_COLS;
    if (c0 >= n) return;
    const EighWs W = eigh_ws(eigh_base(ws, seg, n0, blockIdx.y), n);
    const int cc = threadIdx.x >> 4, s = threadIdx.x & 15;
    const int col = c0 + cc;
    // (clamped: a NaN eigenvalue leaves the ranks no permutation)
    const int g = col < n ? min(max(perm[(int64_t)blockIdx.y * EIG_TILE_MAXN + col], 0), n - 1) : 0;
    constexpr int RPT = EIG_TILE_MAXN / 16;
    z2 w[RPT];
    const z2 ph = *W.ph;
#pragma unroll
    for (int j = 0; j < RPT; ++j) {
        const int r = s + 16 * j;
        const double z = (col < n && r < n) ? W.Z[(int64_t)g * n + r] : 0.0;
        w[j] = r == n - 1 ? zscale(ph, z) : z2{z, 0.0};
    }
    const int nref = n - 2;
    for (int kend = nref; kend > 0; kend -= BT_CHUNK) {
        const int kbeg = max(0, kend - BT_CHUNK);
        __syncthreads();
        for (int e = threadIdx.x; e < BT_CHUNK * EIG_TILE_MAXN; e += 256) {
            const int kk = e / EIG_TILE_MAXN, r = e - kk * EIG_TILE_MAXN;
            const int k = kbeg + kk;
            vs[kk][r] = (k < kend && r < n) ? W.refl[(int64_t)k * n + r] : z2{0.0, 0.0};
        }
        if (threadIdx.x < BT_CHUNK) ts[threadIdx.x] = kbeg + (int)threadIdx.x < kend ? W.tau[kbeg + threadIdx.x] : z2{0.0, 0.0};
        __syncthreads();
        for (int k = kend - 1; k >= kbeg; --k) {
            const int kk = k - kbeg;
            z2 dt = z2{0.0, 0.0};
#pragma unroll
            for (int j = 0; j < RPT; ++j) dt = zcfma(vs[kk][s + 16 * j], w[j], dt);
#pragma unroll
            for (int o = 8; o > 0; o >>= 1) {
                dt.x += __shfl_xor(dt.x, o, 16);
                dt.y += __shfl_xor(dt.y, o, 16);
            }
            const z2 tv = zmul(ts[kk], dt);
#pragma unroll
            for (int j = 0; j < RPT; ++j) w[j] = zfms(vs[kk][s + 16 * j], tv, w[j]);
        }
    }
    if (col < n) {
        z2* V = vecs + M.moff;
#pragma unroll
        for (int j = 0; j < RPT; ++j) {
            const int r = s + 16 * j;
            if (r < n) V[(int64_t)r * n + col] = w[j];
        }
    }
}

}  // namespace

// ----------------------------------------------------------- launches ------
size_t eigh_tiles_ws_bytes(int64_t n2sum) { return (size_t)EIGH_WS_PER_N2 * n2sum * sizeof(z2) + 256; }

size_t eigh_perm_bytes(int nmat) { return (size_t)nmat * EIG_TILE_MAXN * sizeof(int) + 256; }

hipError_t cholesky_tiles_launch(hipStream_t st, unsigned nmat, int nmax, const Seg* seg, int nbo, int n0,
                                 const double2* U, double2* Rinv, int* status, const int* act) {
    if (nmax <= 64)
        hipLaunchKernelGGL(k_cholesky_tiles<16>, dim3(nmat), dim3(256), 0, st, seg, nbo, n0, U, Rinv, status, act);
    else
        hipLaunchKernelGGL(k_cholesky_tiles<32>, dim3(nmat), dim3(1024), 0, st, seg, nbo, n0, U, Rinv, status, act);
    return hipGetLastError();
}

hipError_t grad_prep_tiles_launch(hipStream_t st, unsigned nit, int nmax, const Seg* seg, double2* U, double2* H0,
                                  double2* M1, double* E0, int* status, const double* step, const double2* X,
                                  const double2* Q, const double2* H1, const double2* H2) {
    if (nmax <= 64)
        hipLaunchKernelGGL(k_grad_prep_tiles<16>, dim3(nit), dim3(256), 0, st, seg, U, H0, M1, E0, status, step, X, Q,
                           H1, H2);
    else
        hipLaunchKernelGGL(k_grad_prep_tiles<32>, dim3(nit), dim3(1024), 0, st, seg, U, H0, M1, E0, status, step, X,
                           Q, H1, H2);
    return hipGetLastError();
}

hipError_t linesearch_tiles_launch(hipStream_t st, unsigned nit, int nmax, const Seg* seg, const double2* U,
                                   const double2* X, const double2* Q, const double2* H0, const double2* H1,
                                   const double2* H2, const double* E0v, const double* at0, const double* d0v,
                                   const int* act, int* ok, double* step) {
    if (nmax <= 64)
        hipLaunchKernelGGL(k_linesearch_tiles<16>, dim3(nit), dim3(256), 0, st, seg, U, X, Q, H0, H1, H2, E0v, at0,
                           d0v, act, ok, step);
    else
        hipLaunchKernelGGL(k_linesearch_tiles<32>, dim3(nit), dim3(1024), 0, st, seg, U, X, Q, H0, H1, H2, E0v, at0,
                           d0v, act, ok, step);
    return hipGetLastError();
}

hipError_t eigh_tiles_launch(hipStream_t st, unsigned nmat, int nmax, const Seg* seg, int n0, const double2* H,
                             double* eig, double2* vecs, double2* ws, int* perm) {
    if (nmax <= 64)
        hipLaunchKernelGGL(k_eigh_tridiag<16>, dim3(nmat), dim3(256), 0, st, seg, n0, H, ws);
    else
        hipLaunchKernelGGL(k_eigh_tridiag<32>, dim3(nmat), dim3(1024), 0, st, seg, n0, H, ws);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_eigh_bisect, dim3(nmax, nmat), dim3(64), 0, st, seg, n0, ws);
    hipLaunchKernelGGL(k_eigh_invit, dim3(nmax, nmat), dim3(64), 0, st, seg, n0, ws, eig, perm);
    hipLaunchKernelGGL(k_eigh_back, dim3((nmax + BT_COLS - 1) / BT_COLS, nmat), dim3(256), 0, st, seg, n0, ws,
                       (const int*)perm, vecs);
    return hipGetLastError();
}

}  // namespace dpp
