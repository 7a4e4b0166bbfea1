// Contractions on wavefunction blocks (FP64 MFMA; split-BF16 and FP32 MFMA
// for the mixed-precision bulk), Cholesky factorization and triangular
// inverse, Hermitian Jacobi eigensolver, and the full H apply.
//
// Complex products are built from real 16x16x4 FP64 MFMAs (v_mfma_f64_16x16x4f64):
//   A^dag B :  Re = Ar.Br + Ai.Bi,  Im = Ar.Bi - Ai.Br
//   X M     :  Re = Mr.Xr - Mi.Xi,  Im = Mi.Xr + Mr.Xi
// MFMA operand layout (one wave, lane l): A[i][k] from lane (i + 16 k),
// B[k][j] from lane (j + 16 k); result element v of lane l is
// D[4 v + l / 16][l % 16] (checked on gfx950 with one-hot lane sums).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>
#include <string>
#include <cmath>
#include <type_traits>
#include <vector>

#include "blockops.h"
#include "internal.h"

namespace dpp {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));

__device__ __forceinline__ d4 mfma(double a, double b, d4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
// FP32 16x16x4: operands as for FP64; result element v of lane l is
// D[4 (l / 16) + v][l % 16] (measured on gfx950).
__device__ __forceinline__ f4 mfma(float a, float b, f4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
// BF16 16x16x32: A[i][k] in lane i + 16 (k / 8), element k % 8; B[k][j] in
// lane j + 16 (k / 8), element k % 8; result element v of lane l is
// D[4 (l / 16) + v][l % 16] (measured on gfx950).
__device__ __forceinline__ f4 mfma(bf8 a, bf8 b, f4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// Load through the global address space (table pointers are otherwise
// generic, and generic loads also count against the scalar-load counter).
typedef double d2v __attribute__((ext_vector_type(2)));
__device__ __forceinline__ double2 gld(const double2* p) {
    const d2v v = *(const __attribute__((address_space(1))) d2v*)p;
    return double2{v.x, v.y};
}

// ----------------------------------------------------------- A^dag B -------
// One wave accumulates a TA x TB block of 16x16 tiles of U over a K range, so
// each loaded A and B value serves every tile of the block; a workgroup of
// OV_WAVES waves covers consecutive K sub-ranges of the same block and sums
// them in LDS in fixed order; the partial of each workgroup (chunk) is
// written out per tile and reduced by k_overlap_reduce in fixed order.  A
// launch runs one task (kernel argument) or a table of tasks (blockIdx.z).
// Loads take clamped, in-bounds addresses and are unconditional; points past
// the range get A = 0 when used, so the next step's loads stay in flight
// during the MFMAs.  Rows past the band counts are computed from finite data
// and never stored.
template <int TA, int TB, int NW, bool FULL>
__device__ __forceinline__ void ov_block(const OvTask& T, double2* __restrict__ part,
                                         double (*red)[2][4][64], int chunk_in, int blk) {
    const int chunk = FULL ? 0 : chunk_in;
    const int tilesA = (T.nbA + 15) / 16;
    const int sB = (T.tilesB + TB - 1) / TB, sA = (tilesA + TA - 1) / TA;
    if (blk >= sA * sB) return;
    const int ti0 = (blk / sB) * TA, tj0 = (blk % sB) * TB;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int r = lane & 15, ks = lane >> 4;
    const double2* Ap[TA];
    const double2* Bp[TB];
#pragma unroll
    for (int a = 0; a < TA; ++a) Ap[a] = T.A + (int64_t)min((ti0 + a) * 16 + r, T.nbA - 1) * T.ldA;
#pragma unroll
    for (int b = 0; b < TB; ++b) Bp[b] = T.B + (int64_t)min((tj0 + b) * 16 + r, T.nbB - 1) * T.ldB;
    d4 cre[TA][TB], cim[TA][TB];
#pragma unroll
    for (int a = 0; a < TA; ++a)
#pragma unroll
        for (int b = 0; b < TB; ++b) {
            cre[a][b] = d4{0, 0, 0, 0};
            cim[a][b] = d4{0, 0, 0, 0};
        }
    // chunked: OV_CHUNK points per workgroup; FULL: all points, NW slices
    const int sub = FULL ? ((T.npw + NW * 16 - 1) / (NW * 16)) * 16 : OV_CHUNK / NW;
    const int ga = chunk * OV_CHUNK + w * sub, ge = min(T.npw, ga + sub);
    const int nst = ge > ga ? (ge - ga + 15) / 16 : 0;
    // lane covers points g + 4 ks + s, s = 0..3, of the step at g
    double2 an[TA][4], bn[TB][4];
    auto load = [&](int g) {
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            const int q = min(g + 4 * ks + s, T.npw - 1);
#pragma unroll
            for (int a = 0; a < TA; ++a) an[a][s] = gld(Ap[a] + q);
#pragma unroll
            for (int b = 0; b < TB; ++b) bn[b][s] = gld(Bp[b] + q);
        }
    };
    if (nst > 0) load(ga);
    for (int st = 0; st < nst; ++st) {
        const int g = ga + 16 * st;
        double2 av[TA][4], bv[TB][4];
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            const bool in = g + 4 * ks + s < ge;
#pragma unroll
            for (int a = 0; a < TA; ++a) av[a][s] = in ? an[a][s] : double2{0, 0};
#pragma unroll
            for (int b = 0; b < TB; ++b) bv[b][s] = bn[b][s];
        }
        if (st + 1 < nst) load(g + 16);
#pragma unroll
        for (int s = 0; s < 4; ++s)
#pragma unroll
            for (int a = 0; a < TA; ++a)
#pragma unroll
                for (int b = 0; b < TB; ++b) {
                    cre[a][b] = mfma(av[a][s].x, bv[b][s].x, cre[a][b]);
                    cre[a][b] = mfma(av[a][s].y, bv[b][s].y, cre[a][b]);
                    cim[a][b] = mfma(av[a][s].x, bv[b][s].y, cim[a][b]);
                    cim[a][b] = mfma(-av[a][s].y, bv[b][s].x, cim[a][b]);
                }
    }
#pragma unroll
    for (int a = 0; a < TA; ++a)
#pragma unroll
        for (int b = 0; b < TB; ++b) {
            if (ti0 + a >= tilesA || tj0 + b >= T.tilesB) continue;  // uniform over the workgroup
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                red[w][0][v][lane] = cre[a][b][v];
                red[w][1][v][lane] = cim[a][b][v];
            }
            __syncthreads();
            if (w == 0) {
                const int tile = (ti0 + a) * T.tilesB + tj0 + b;
                double2* dst = part + T.part_off + ((int64_t)chunk * T.ntiles + tile) * 256;
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    double sr = 0, si = 0;
                    for (int u = 0; u < NW; ++u) {
                        sr += red[u][0][v][lane];
                        si += red[u][1][v][lane];
                    }
                    const int i = 4 * v + (lane >> 4), j = lane & 15;
                    if (FULL) {
                        // one workgroup covered every point: the scaled result
                        const int gi = (ti0 + a) * 16 + i, gj = (tj0 + b) * 16 + j;
                        if (gi < T.nbA && gj < T.nbB)
                            T.out[(int64_t)gi * T.out_ld + gj] = double2{T.scale * sr, T.scale * si};
                    } else {
                        dst[i * 16 + j] = double2{sr, si};
                    }
                }
            }
            __syncthreads();
        }
}


// Each task takes the widest block shape its own tile counts fill (WIDE);
// launches whose operands are all at most 16 bands run the 1 x 1 shape only,
// at its lower register count.
template <int TA, int TB>
__host__ __device__ constexpr int ov_blocks(int tA, int tB) {
    return ((tA + TA - 1) / TA) * ((tB + TB - 1) / TB);
}

// FULL: one workgroup of OVF_WAVES waves per (task, tile block) covers all
// points and writes the scaled result (no partials, no reduction launch).
constexpr int OVF_WAVES = 8;

template <bool WIDE, bool FULL>
__global__ void __launch_bounds__(64 * (FULL ? OVF_WAVES : OV_WAVES))
k_overlap_mfma(const OvTask* __restrict__ tasks, OvTask single, double2* __restrict__ part,
               const int* __restrict__ act, const int4* __restrict__ work) {
    constexpr int NW = FULL ? OVF_WAVES : OV_WAVES;
    __shared__ double red[NW][2][4][64];
    // a work list (task, chunk, block) covers only the workgroups that have
    // work; without one the grid is (chunk, block, task)
    int ti, chunk, blk;
    if (work) {
        const int4 w = work[blockIdx.x];
        ti = w.x, chunk = w.y, blk = w.z;
    } else {
        ti = (int)blockIdx.z, chunk = (int)blockIdx.x, blk = (int)blockIdx.y;
    }
    const OvTask T = tasks ? tasks[ti] : single;
    if (act && !act[T.item]) return;
    if (!FULL && chunk >= T.nchunk) return;
    if constexpr (WIDE) {
        const int tA = (T.nbA + 15) / 16, tB = T.tilesB;
        if (tA >= 2 && tB >= 2)
            ov_block<2, 2, NW, FULL>(T, part, red, chunk, blk);
        else if (tB >= 2)
            ov_block<1, 2, NW, FULL>(T, part, red, chunk, blk);
        else if (tA >= 2)
            ov_block<2, 1, NW, FULL>(T, part, red, chunk, blk);
        else
            ov_block<1, 1, NW, FULL>(T, part, red, chunk, blk);
    } else {
        ov_block<1, 1, NW, FULL>(T, part, red, chunk, blk);
    }
}

// LDS-staged form (launch mode 3): one workgroup of eight waves per (task,
// chunk, 4 x 4 tile block).  Each 16-point step of the block's 64 A rows and
// 64 B rows is staged once in LDS (double-buffered, rows padded to an odd
// number of 16-byte units), and each wave accumulates one A tile against two
// B tiles from there, so every operand is read from memory once per block
// instead of once per wave.  Eight waves of two tiles ran faster than four of
// four (115 against 136 us per 128 x 128 product): the 376 workgroups of a
// 128-band product fill only part of the chip, and the extra waves hide the
// LDS and MFMA latencies.  Partials use k_overlap_mfma's layout (chunk, tile) and are
// summed by k_overlap_reduce.
constexpr int OVS_ROWS = 128;  // 64 A rows, then 64 B rows
constexpr int OVS_ROW = 17;    // 16 points + 1 unit of padding

constexpr int OVS_TA = 1;      // A tiles per wave (eight waves: one A tile by two B tiles each)
constexpr int OVS_THREADS = 512;

__global__ void __launch_bounds__(OVS_THREADS)
k_overlap_staged(const OvTask* __restrict__ tasks, OvTask single, double2* __restrict__ part,
                 const int* __restrict__ act, const int4* __restrict__ work) {
    __shared__ double2 st[2][OVS_ROWS * OVS_ROW];
    int ti, chunk, blk;
    if (work) {
        const int4 w = work[blockIdx.x];
        ti = w.x, chunk = w.y, blk = w.z;
    } else {
        ti = (int)blockIdx.z, chunk = (int)blockIdx.x, blk = (int)blockIdx.y;
    }
    const OvTask T = tasks ? tasks[ti] : single;
    if (act && !act[T.item]) return;
    if (chunk >= T.nchunk) return;
    const int tilesA = (T.nbA + 15) / 16;
    const int sB = (T.tilesB + 3) / 4, sA = (tilesA + 3) / 4;
    if (blk >= sA * sB) return;
    const int ti0 = (blk / sB) * 4, tj0 = (blk % sB) * 4;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int r = lane & 15, ks = lane >> 4;
    // staging: thread -> LDS row tid / 2, points 8 (tid % 2) .. + 7 of a step
    const int srow = tid >> 2, sp = (tid & 3) * 4;
    const bool isA = srow < 64;
    const int brow = isA ? 16 * ti0 + srow : 16 * tj0 + srow - 64;
    const bool valid = brow < (isA ? T.nbA : T.nbB);
    const double2* src = isA ? T.A + (int64_t)brow * T.ldA : T.B + (int64_t)brow * T.ldB;
    const int g0 = chunk * OV_CHUNK, g1 = min(T.npw, g0 + OV_CHUNK);
    const int nst = g1 > g0 ? (g1 - g0 + 15) / 16 : 0;
    double2 raw[4];
    // rows past the band counts load nothing and stage zeros; points past the
    // chunk are clamped to the last point when loaded and zeroed when staged
    auto load = [&](int g) {
        if (valid) {
#pragma unroll
            for (int e = 0; e < 4; ++e) raw[e] = gld(src + min(g + sp + e, T.npw - 1));
        }
    };
    auto stage = [&](int buf, int g) {
        double2* row = st[buf] + srow * OVS_ROW + sp;
#pragma unroll
        for (int e = 0; e < 4; ++e) row[e] = (valid && g + sp + e < g1) ? raw[e] : double2{0, 0};
    };
    // this wave's tiles: A tiles ti0 + 2 (w / 2) + a, B tiles tj0 + 2 (w % 2) + b
    const int wa = OVS_TA * (w >> 1), wb = 2 * (w & 1);
    d4 cre[OVS_TA][2], cim[OVS_TA][2];
#pragma unroll
    for (int a = 0; a < OVS_TA; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) {
            cre[a][b] = d4{0, 0, 0, 0};
            cim[a][b] = d4{0, 0, 0, 0};
        }
    if (nst > 0) load(g0);
    for (int s = 0; s < nst; ++s) {
        const int buf = s & 1;
        stage(buf, g0 + 16 * s);
        if (s + 1 < nst) load(g0 + 16 * (s + 1));
        __syncthreads();
        const double2* S = st[buf];
        // lane (r, ks) takes points 4 ks + q of the step for the q-th MFMA
        double2 av[OVS_TA][4], bv[2][4];
#pragma unroll
        for (int a = 0; a < OVS_TA; ++a)
#pragma unroll
            for (int q = 0; q < 4; ++q) av[a][q] = S[(16 * (wa + a) + r) * OVS_ROW + 4 * ks + q];
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int q = 0; q < 4; ++q) bv[b][q] = S[(64 + 16 * (wb + b) + r) * OVS_ROW + 4 * ks + q];
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int a = 0; a < OVS_TA; ++a)
#pragma unroll
                for (int b = 0; b < 2; ++b) {
                    cre[a][b] = mfma(av[a][q].x, bv[b][q].x, cre[a][b]);
                    cre[a][b] = mfma(av[a][q].y, bv[b][q].y, cre[a][b]);
                    cim[a][b] = mfma(av[a][q].x, bv[b][q].y, cim[a][b]);
                    cim[a][b] = mfma(-av[a][q].y, bv[b][q].x, cim[a][b]);
                }
    }
#pragma unroll
    for (int a = 0; a < OVS_TA; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) {
            const int ta = ti0 + wa + a, tb = tj0 + wb + b;
            if (ta >= tilesA || tb >= T.tilesB) continue;  // uniform over the wave
            double2* dst = part + T.part_off + ((int64_t)chunk * T.ntiles + ta * T.tilesB + tb) * 256;
#pragma unroll
            for (int v = 0; v < 4; ++v) dst[(4 * v + (lane >> 4)) * 16 + (lane & 15)] = double2{cre[a][b][v], cim[a][b][v]};
        }
}

// Blocks of a task in the shape k_overlap_mfma picks for it (staged: the 4 x 4
// blocks of k_overlap_staged).
static int ov_task_blocks(int tA, int tB, bool staged = false) {
    if (staged) return ov_blocks<4, 4>(tA, tB);
    if (tA >= 2 && tB >= 2) return ov_blocks<2, 2>(tA, tB);
    if (tB >= 2) return ov_blocks<1, 2>(tA, tB);
    if (tA >= 2) return ov_blocks<2, 1>(tA, tB);
    return tA * tB;
}

// nblk: the largest ov_task_blocks over the tasks; wide: some task has more
// than one tile.
static void overlap_launch(dpp_ctx ctx, const OvTask* d_tasks, const OvTask& single, unsigned ntasks, int nchunk,
                           int nblk, bool wide, double2* part, const int* act, bool full = false,
                           const int4* work = nullptr, int nwork = 0) {
    const dim3 grid = work ? dim3((unsigned)nwork, 1, 1) : dim3(full ? 1 : nchunk, nblk, ntasks);
    if (full) {
        if (wide)
            hipLaunchKernelGGL((k_overlap_mfma<true, true>), grid, dim3(64 * OVF_WAVES), 0, ctx->stream, d_tasks,
                               single, part, act, work);
        else
            hipLaunchKernelGGL((k_overlap_mfma<false, true>), grid, dim3(64 * OVF_WAVES), 0, ctx->stream, d_tasks,
                               single, part, act, work);
        return;
    }
    if (wide)
        hipLaunchKernelGGL((k_overlap_mfma<true, false>), grid, dim3(64 * OV_WAVES), 0, ctx->stream, d_tasks, single,
                           part, act, work);
    else
        hipLaunchKernelGGL((k_overlap_mfma<false, false>), grid, dim3(64 * OV_WAVES), 0, ctx->stream, d_tasks,
                           single, part, act, work);
}

// Whether an FP64 launch over these tasks runs k_overlap_staged: mode 3, or
// the default mode (0) when every task has at least 4 x 4 output tiles (at
// 128 bands it takes 185 us per overlap pair against 233 us for the 2 x 2
// blocks; smaller tasks keep the 2 x 2 blocks).
static bool ov_staged(const std::vector<OvTask>& h, int ov_mode) {
    if (ov_mode == 3) return true;
    if (ov_mode != 0 || h.empty()) return false;
    for (const OvTask& t : h)
        if ((t.nbA + 15) / 16 < 4 || t.tilesB < 4) return false;
    return true;
}

void overlap_worklist(const std::vector<OvTask>& h, int ov_mode, std::vector<int4>& w) {
    const bool staged = ov_staged(h, ov_mode);
    w.clear();
    for (size_t i = 0; i < h.size(); ++i) {
        const OvTask& t = h[i];
        const int nch = ov_mode == 2 ? 1 : t.nchunk;
        const int nb = ov_mode == 1 ? t.ntiles : ov_task_blocks((t.nbA + 15) / 16, t.tilesB, staged);
        for (int c = 0; c < nch; ++c)
            for (int b = 0; b < nb; ++b) w.push_back(int4{(int)i, c, b, 0});
    }
}

// ------------------------------------------- A^dag B, split-BF16 MFMA ------
// The mixed-precision bulk: every FP64 input is rounded to FP32 and split
// into x = hi + lo, two BF16 values (|x - hi - lo| <= 2^-16 |x|).  The four
// products hi hi' + hi lo' + lo hi' + lo lo' accumulate in FP32 (all four:
// without lo lo' the diagonal of A^dag A would be biased low by ~1e-6
// relative, since every dropped term there is positive).  A complex point
// is two consecutive K entries (re, im): Re = <(Ar, Ai), (Br, Bi)> and
// Im = <(Ar, Ai), (Bi, -Br)>, so a 16x16x32 MFMA covers 16 points.  FP32
// sums run over at most 128 points; their partials are summed in FP64 in
// fixed order.
//
// Two launch forms:
//  - up to 15 output tiles per task (<= 48 bands): the FP64 kernel's shape, a
//    wave per 2x2 tile block over 64 points, four waves per 256-point chunk,
//    FP64 partials per chunk (k_overlap_reduce);
//  - larger tasks: one workgroup per (task, 128-point slice) computes every
//    output tile.  Each 16-point step of the slice is read from HBM once,
//    split into BF16 hi/lo by the whole workgroup and staged in LDS (double
//    buffered, one barrier per step); eight waves then take 4 x 2 tile
//    blocks from LDS.  FP32 partials per slice (k_overlap_reduce_slices).
constexpr int OVB_WAVES = 4;
constexpr int OVW_WAVES = 8;
constexpr int OVW_SLICE = 128;  // points per workgroup
constexpr int OVW_ROW = 72;     // LDS row: hi (32 BF16), lo (32 BF16), pad (8); 144 bytes
constexpr int OVW_MIN_TILES = 16;

__device__ __forceinline__ void bsplit(double x, __bf16& hi, __bf16& lo) {
    const float f = (float)x;
    hi = (__bf16)f;
    lo = (__bf16)(f - (float)hi);
}

// (re, im) pairs -> (im, -re) pairs on an 8-element operand.
__device__ __forceinline__ bf8 swap_neg(bf8 v) {
    typedef unsigned int u4 __attribute__((ext_vector_type(4)));
    u4 u = __builtin_bit_cast(u4, v);
#pragma unroll
    for (int i = 0; i < 4; ++i) u[i] = ((u[i] >> 16) | (u[i] << 16)) ^ 0x80000000u;
    return __builtin_bit_cast(bf8, u);
}

template <int TA, int TB>
__device__ __forceinline__ void ovb_block(const OvTask& T, double2* __restrict__ part,
                                          double (*red)[2][4][64], int chunk, int blk) {
    const int tilesA = (T.nbA + 15) / 16;
    const int sB = (T.tilesB + TB - 1) / TB, sA = (tilesA + TA - 1) / TA;
    if (blk >= sA * sB) return;
    const int ti0 = (blk / sB) * TA, tj0 = (blk % sB) * TB;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int r = lane & 15, ks = lane >> 4;
    const double2* Ap[TA];
    const double2* Bp[TB];
#pragma unroll
    for (int a = 0; a < TA; ++a) Ap[a] = T.A + (int64_t)min((ti0 + a) * 16 + r, T.nbA - 1) * T.ldA;
#pragma unroll
    for (int b = 0; b < TB; ++b) Bp[b] = T.B + (int64_t)min((tj0 + b) * 16 + r, T.nbB - 1) * T.ldB;
    f4 cre[TA][TB], cim[TA][TB];
#pragma unroll
    for (int a = 0; a < TA; ++a)
#pragma unroll
        for (int b = 0; b < TB; ++b) {
            cre[a][b] = f4{0, 0, 0, 0};
            cim[a][b] = f4{0, 0, 0, 0};
        }
    constexpr int sub = OV_CHUNK / OVB_WAVES;
    const int ga = chunk * OV_CHUNK + w * sub, ge = min(T.npw, ga + sub);
    const int nst = ge > ga ? (ge - ga + 15) / 16 : 0;
    // lane covers points g + 4 ks + s, s = 0..3, of the step at g (K entries
    // 8 ks + 2 s and 8 ks + 2 s + 1); clamped, unconditional loads
    double2 an[TA][4], bn[TB][4];
    auto load = [&](int g) {
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            const int q = min(g + 4 * ks + s, T.npw - 1);
#pragma unroll
            for (int a = 0; a < TA; ++a) an[a][s] = gld(Ap[a] + q);
#pragma unroll
            for (int b = 0; b < TB; ++b) bn[b][s] = gld(Bp[b] + q);
        }
    };
    if (nst > 0) load(ga);
    for (int st = 0; st < nst; ++st) {
        const int g = ga + 16 * st;
        bf8 ah[TA], al[TA], bh[TB], bl[TB];
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            const bool in = g + 4 * ks + s < ge;
#pragma unroll
            for (int a = 0; a < TA; ++a) {
                __bf16 h, l;
                bsplit(in ? an[a][s].x : 0.0, h, l);
                ah[a][2 * s] = h;
                al[a][2 * s] = l;
                bsplit(in ? an[a][s].y : 0.0, h, l);
                ah[a][2 * s + 1] = h;
                al[a][2 * s + 1] = l;
            }
#pragma unroll
            for (int b = 0; b < TB; ++b) {
                __bf16 h, l;
                bsplit(bn[b][s].x, h, l);
                bh[b][2 * s] = h;
                bl[b][2 * s] = l;
                bsplit(bn[b][s].y, h, l);
                bh[b][2 * s + 1] = h;
                bl[b][2 * s + 1] = l;
            }
        }
        if (st + 1 < nst) load(g + 16);
#pragma unroll
        for (int b = 0; b < TB; ++b) {
            const bf8 ch = swap_neg(bh[b]), cl = swap_neg(bl[b]);
#pragma unroll
            for (int a = 0; a < TA; ++a) {
                cre[a][b] = mfma(al[a], bl[b], cre[a][b]);
                cre[a][b] = mfma(al[a], bh[b], cre[a][b]);
                cre[a][b] = mfma(ah[a], bl[b], cre[a][b]);
                cre[a][b] = mfma(ah[a], bh[b], cre[a][b]);
                cim[a][b] = mfma(al[a], cl, cim[a][b]);
                cim[a][b] = mfma(al[a], ch, cim[a][b]);
                cim[a][b] = mfma(ah[a], cl, cim[a][b]);
                cim[a][b] = mfma(ah[a], ch, cim[a][b]);
            }
        }
    }
#pragma unroll
    for (int a = 0; a < TA; ++a)
#pragma unroll
        for (int b = 0; b < TB; ++b) {
            if (ti0 + a >= tilesA || tj0 + b >= T.tilesB) continue;  // uniform over the workgroup
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                red[w][0][v][lane] = (double)cre[a][b][v];
                red[w][1][v][lane] = (double)cim[a][b][v];
            }
            __syncthreads();
            if (w == 0) {
                const int tile = (ti0 + a) * T.tilesB + tj0 + b;
                double2* dst = part + T.part_off + ((int64_t)chunk * T.ntiles + tile) * 256;
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    double sr = 0, si = 0;
                    for (int u = 0; u < OVB_WAVES; ++u) {
                        sr += red[u][0][v][lane];
                        si += red[u][1][v][lane];
                    }
                    dst[(4 * (lane >> 4) + v) * 16 + (lane & 15)] = double2{sr, si};
                }
            }
            __syncthreads();
        }
}

// Small tasks: work list entries (task, chunk, block) as overlap_worklist's.
__global__ void __launch_bounds__(64 * OVB_WAVES)
k_overlap_bf16(const OvTask* __restrict__ tasks, OvTask single, double2* __restrict__ part,
               const int* __restrict__ act, const int4* __restrict__ work) {
    __shared__ double red[OVB_WAVES][2][4][64];
    int ti, chunk, blk;
    if (work) {
        const int4 w = work[blockIdx.x];
        ti = w.x, chunk = w.y, blk = w.z;
    } else {
        ti = (int)blockIdx.z, chunk = (int)blockIdx.x, blk = (int)blockIdx.y;
    }
    const OvTask T = tasks ? tasks[ti] : single;
    if (act && !act[T.item]) return;
    if (chunk >= T.nchunk) return;
    const int tA = (T.nbA + 15) / 16, tB = T.tilesB;
    if (tA >= 2 && tB >= 2)
        ovb_block<2, 2>(T, part, red, chunk, blk);
    else if (tB >= 2)
        ovb_block<1, 2>(T, part, red, chunk, blk);
    else if (tA >= 2)
        ovb_block<2, 1>(T, part, red, chunk, blk);
    else
        ovb_block<1, 1>(T, part, red, chunk, blk);
}

__host__ __device__ inline int ovw_slices(int npw) { return (npw + OVW_SLICE - 1) / OVW_SLICE; }

// Large tasks: one workgroup per (task, slice) (work list entries, or the
// grid (slice, task)).  LDS rows: A rows 0 .. 16 tilesA - 1, then B rows
// (rows past a band count are zero).  FP32 partials, as float2, at the
// task's partial offset: slice s, tile t at (s ntiles + t) 256.
__global__ void __launch_bounds__(64 * OVW_WAVES)
k_overlap_bf16_wg(const OvTask* __restrict__ tasks, OvTask single, double2* __restrict__ part,
                  const int* __restrict__ act, const int4* __restrict__ work) {
    __shared__ __attribute__((aligned(16))) __bf16 st[2][2 * EIG_TILE_MAXN * OVW_ROW];
    int ti, slice;
    if (work) {
        const int4 w = work[blockIdx.x];
        ti = w.x, slice = w.y;
    } else {
        ti = (int)blockIdx.y, slice = (int)blockIdx.x;
    }
    const OvTask T = tasks ? tasks[ti] : single;
    if (act && !act[T.item]) return;
    if (slice >= ovw_slices(T.npw)) return;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int r = lane & 15, ks = lane >> 4;
    const int tilesA = (T.nbA + 15) / 16, tilesB = T.tilesB;
    const int rowsA = 16 * tilesA, nrows = rowsA + 16 * tilesB;
    // staging: thread -> LDS row tid / 2, points 8 (tid % 2) .. + 7 of a step
    const int srow = tid >> 1, sp = (tid & 1) * 8;
    const bool isA = srow < rowsA;
    const int brow = isA ? srow : srow - rowsA;
    const bool valid = srow < nrows && brow < (isA ? T.nbA : T.nbB);
    const double2* src = isA ? T.A + (int64_t)brow * T.ldA : T.B + (int64_t)brow * T.ldB;
    const int g0 = slice * OVW_SLICE, g1 = min(T.npw, g0 + OVW_SLICE);
    const int nst = (g1 - g0 + 15) / 16;
    double2 raw[8];
    // rows past the band counts load nothing; points past the slice are
    // clamped to the last point (and zeroed when staged)
    auto load = [&](int g) {
        if (valid) {
#pragma unroll
            for (int e = 0; e < 8; ++e) raw[e] = gld(src + min(g + sp + e, T.npw - 1));
        }
    };
    auto stage = [&](int buf, int g) {
        if (srow >= nrows) return;
        bf8 h0, h1, l0, l1;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const bool in = valid && g + sp + e < g1;
            __bf16 hr, lr, hi, li;
            bsplit(in ? raw[e].x : 0.0, hr, lr);
            bsplit(in ? raw[e].y : 0.0, hi, li);
            if (e < 4) {
                h0[2 * e] = hr, h0[2 * e + 1] = hi, l0[2 * e] = lr, l0[2 * e + 1] = li;
            } else {
                h1[2 * e - 8] = hr, h1[2 * e - 7] = hi, l1[2 * e - 8] = lr, l1[2 * e - 7] = li;
            }
        }
        __bf16* row = st[buf] + srow * OVW_ROW;
        *(bf8*)(row + 2 * sp) = h0;
        *(bf8*)(row + 2 * sp + 8) = h1;
        *(bf8*)(row + 32 + 2 * sp) = l0;
        *(bf8*)(row + 32 + 2 * sp + 8) = l1;
    };
    // this wave's tiles: A tiles 4 ga .. 4 ga + 3, B tiles 2 gb, 2 gb + 1
    const int ga = w >> 2, gb = w & 3;
    f4 cre[4][2], cim[4][2];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) {
            cre[a][b] = f4{0, 0, 0, 0};
            cim[a][b] = f4{0, 0, 0, 0};
        }
    if (nst > 0) load(g0);
    for (int s = 0; s < nst; ++s) {
        const int buf = s & 1;
        stage(buf, g0 + 16 * s);
        if (s + 1 < nst) load(g0 + 16 * (s + 1));
        __syncthreads();
        const __bf16* S = st[buf];
#pragma unroll
        for (int b = 0; b < 2; ++b) {
            const int tb = 2 * gb + b;
            if (tb >= tilesB) continue;  // uniform over the wave
            const __bf16* rb = S + (rowsA + 16 * tb + r) * OVW_ROW + 8 * ks;
            const bf8 bh = *(const bf8*)rb, bl = *(const bf8*)(rb + 32);
            const bf8 ch = swap_neg(bh), cl = swap_neg(bl);
#pragma unroll
            for (int a = 0; a < 4; ++a) {
                const int ta = 4 * ga + a;
                if (ta >= tilesA) continue;
                const __bf16* ra = S + (16 * ta + r) * OVW_ROW + 8 * ks;
                const bf8 ah = *(const bf8*)ra, al = *(const bf8*)(ra + 32);
                cre[a][b] = mfma(al, bl, cre[a][b]);
                cre[a][b] = mfma(al, bh, cre[a][b]);
                cre[a][b] = mfma(ah, bl, cre[a][b]);
                cre[a][b] = mfma(ah, bh, cre[a][b]);
                cim[a][b] = mfma(al, cl, cim[a][b]);
                cim[a][b] = mfma(al, ch, cim[a][b]);
                cim[a][b] = mfma(ah, cl, cim[a][b]);
                cim[a][b] = mfma(ah, ch, cim[a][b]);
            }
        }
    }
    float2* out = reinterpret_cast<float2*>(part + T.part_off) + (int64_t)slice * T.ntiles * 256;
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) {
            const int ta = 4 * ga + a, tb = 2 * gb + b;
            if (ta >= tilesA || tb >= tilesB) continue;
            float2* dst = out + (ta * tilesB + tb) * 256;
#pragma unroll
            for (int v = 0; v < 4; ++v) dst[(4 * ks + v) * 16 + r] = float2{cre[a][b][v], cim[a][b][v]};
        }
}

// Reductions of the overlap partials: OVR_OUT output elements per 256-thread
// workgroup, four threads each summing a contiguous quarter of the partials
// in order; the quarters are added in order, so the sum is deterministic.
constexpr int OVR_OUT = 64;

__device__ __forceinline__ void ovr_store(const OvTask& T, int e, const double2 (*acc)[OVR_OUT], int o) {
    const int tile = e >> 8, ij = e & 255;
    const int ti = tile / T.tilesB, tj = tile - ti * T.tilesB;
    const int i = ti * 16 + (ij >> 4), j = tj * 16 + (ij & 15);
    if (i >= T.nbA || j >= T.nbB) return;
    const double sr = ((acc[0][o].x + acc[1][o].x) + acc[2][o].x) + acc[3][o].x;
    const double si = ((acc[0][o].y + acc[1][o].y) + acc[2][o].y) + acc[3][o].y;
    T.out[(int64_t)i * T.out_ld + j] = double2{T.scale * sr, T.scale * si};
}

// Sums the FP32 slice partials of every task in FP64, in fixed order.
__global__ void __launch_bounds__(256)
k_overlap_reduce_slices(const OvTask* __restrict__ tasks, OvTask single, const double2* __restrict__ part,
                        const int* __restrict__ act) {
    const OvTask& T = tasks ? tasks[blockIdx.y] : single;
    if (act && !act[T.item]) return;  // uniform over the workgroup
    __shared__ double2 acc[4][OVR_OUT];
    const int o = threadIdx.x % OVR_OUT, qd = threadIdx.x / OVR_OUT;
    const int e = blockIdx.x * OVR_OUT + o;
    const bool ok = e < T.ntiles * 256;
    double sr = 0, si = 0;
    if (ok) {
        const float2* p = reinterpret_cast<const float2*>(part + T.part_off) + e;
        const int ns = ovw_slices(T.npw), per = (ns + 3) / 4, c1 = min(ns, (qd + 1) * per);
        for (int c = qd * per; c < c1; ++c) {
            const float2 v = p[(int64_t)c * T.ntiles * 256];
            sr += v.x;
            si += v.y;
        }
    }
    acc[qd][o] = double2{sr, si};
    __syncthreads();
    if (qd == 0 && ok) ovr_store(T, e, acc, o);
}

// Which split-BF16 form a task table takes: the workgroup form when some
// task has at least OVW_MIN_TILES output tiles and every task fits its LDS
// rows and wave blocks (at most 128 bands on either side).
bool overlap_bf16_wide(const std::vector<OvTask>& h) {
    int mt = 0;
    for (const OvTask& t : h) {
        if (t.nbA > EIG_TILE_MAXN || t.nbB > EIG_TILE_MAXN) return false;
        mt = std::max(mt, t.ntiles);
    }
    return mt >= OVW_MIN_TILES;
}

// Work list of the split-BF16 overlap: (task, slice) entries for the
// workgroup form (as int4 {task, slice, 0, 0}), else overlap_worklist's.
void overlap_worklist_bf16(const std::vector<OvTask>& h, std::vector<int4>& w) {
    if (!overlap_bf16_wide(h)) {
        overlap_worklist(h, 0, w);
        return;
    }
    w.clear();
    for (size_t i = 0; i < h.size(); ++i)
        for (int c = 0; c < std::max(1, ovw_slices(h[i].npw)); ++c) w.push_back(int4{(int)i, c, 0, 0});
}

// Sums the chunk partials of every task in fixed order.
__global__ void __launch_bounds__(256)
k_overlap_reduce(const OvTask* __restrict__ tasks, OvTask single, const double2* __restrict__ part,
                 const int* __restrict__ act) {
    const OvTask& T = tasks ? tasks[blockIdx.y] : single;
    if (act && !act[T.item]) return;  // uniform over the workgroup
    __shared__ double2 acc[4][OVR_OUT];
    const int o = threadIdx.x % OVR_OUT, qd = threadIdx.x / OVR_OUT;
    const int e = blockIdx.x * OVR_OUT + o;
    const bool ok = e < T.ntiles * 256;
    double sr = 0, si = 0;
    if (ok) {
        const int tile = e >> 8, ij = e & 255;
        const int per = (T.nchunk + 3) / 4, c1 = min(T.nchunk, (qd + 1) * per);
        for (int c = qd * per; c < c1; ++c) {
            const double2 v = part[T.part_off + ((int64_t)c * T.ntiles + tile) * 256 + ij];
            sr += v.x;
            si += v.y;
        }
    }
    acc[qd][o] = double2{sr, si};
    __syncthreads();
    if (qd == 0 && ok) ovr_store(T, e, acc, o);
}

size_t overlap_ws_bytes(int npw, int nbA, int nbB) {
    const int nchunk = std::max(1, (npw + OV_CHUNK - 1) / OV_CHUNK);
    const int ntiles = ((nbA + 15) / 16) * ((nbB + 15) / 16);
    return (size_t)nchunk * ntiles * 256 * sizeof(double2) + 256;
}

OvTask make_ov_task(int npw, int nbA, const double2* A, int64_t ldA, int nbB, const double2* B, int64_t ldB,
                    double scale, double2* out, int out_ld) {
    OvTask t;
    t.A = A;
    t.B = B;
    t.out = out;
    t.ldA = ldA;
    t.ldB = ldB;
    t.npw = npw;
    t.nbA = nbA;
    t.nbB = nbB;
    t.out_ld = out_ld;
    t.scale = scale;
    t.nchunk = std::max(1, (npw + OV_CHUNK - 1) / OV_CHUNK);
    t.tilesB = (nbB + 15) / 16;
    t.ntiles = ((nbA + 15) / 16) * t.tilesB;
    t.part_off = 0;
    t.item = 0;
    return t;
}

dpp_status overlap_single(dpp_ctx ctx, int npw, int nbA, const double2* A, int64_t ldA, int nbB,
                          const double2* B, int64_t ldB, double scale, double2* U, void* ws, size_t ws_bytes,
                          dpp_precision prec) {
    OvTask t = make_ov_task(npw, nbA, A, ldA, nbB, B, ldB, scale, U, nbB);
    if (overlap_ws_bytes(npw, nbA, nbB) > ws_bytes)
        return set_error(DPP_EINVAL, "overlap: workspace too small");
    if (t.ntiles > 65535) return set_error(DPP_EUNSUPPORTED, "overlap: too many bands");
    double2* part = reinterpret_cast<double2*>(ws);
    const int nblk = ov_task_blocks((nbA + 15) / 16, t.tilesB);
    const bool wide = prec == DPP_F32 && overlap_bf16_wide(std::vector<OvTask>{t});
    {
        TimerScope ts_(ctx, DPP_TK_OVERLAP, 16.0 * npw * (nbA + nbB), 8.0 * npw * nbA * (double)nbB);
        if (wide)
            hipLaunchKernelGGL(k_overlap_bf16_wg, dim3(std::max(1, ovw_slices(npw)), 1), dim3(64 * OVW_WAVES), 0,
                               ctx->stream, (const OvTask*)nullptr, t, part, (const int*)nullptr,
                               (const int4*)nullptr);
        else if (prec == DPP_F32)
            hipLaunchKernelGGL(k_overlap_bf16, dim3(t.nchunk, nblk, 1), dim3(64 * OVB_WAVES), 0, ctx->stream,
                               (const OvTask*)nullptr, t, part, (const int*)nullptr, (const int4*)nullptr);
        else
            overlap_launch(ctx, nullptr, t, 1, t.nchunk, nblk, t.ntiles > 1, part, nullptr);
        DPP_LAUNCHED();
    }
    TimerScope ts2_(ctx, DPP_TK_BLOCKOPS);
    if (wide)
        hipLaunchKernelGGL(k_overlap_reduce_slices, dim3((t.ntiles * 256 + OVR_OUT - 1) / OVR_OUT, 1), dim3(256), 0,
                           ctx->stream, (const OvTask*)nullptr, t, part, (const int*)nullptr);
    else
        hipLaunchKernelGGL(k_overlap_reduce, dim3((t.ntiles * 256 + OVR_OUT - 1) / OVR_OUT, 1), dim3(256), 0, ctx->stream,
                           (const OvTask*)nullptr, t, part, (const int*)nullptr);
    DPP_LAUNCHED();
    return DPP_OK;
}

// Batched: the caller has set part_off of every task (disjoint partial areas)
// and copied the table to d_tasks.
dpp_status overlap_tasks(dpp_ctx ctx, const std::vector<OvTask>& h, const OvTask* d_tasks, double2* part,
                         const int* act, int ov_mode, const int4* d_work, int nwork, dpp_precision prec) {
    const bool bf = prec == DPP_F32;
    const bool wide = bf && overlap_bf16_wide(h);  // the work list is overlap_worklist_bf16's
    const int ov_narrow = !bf && ov_mode == 1;
    const bool full = !bf && ov_mode == 2;
    const bool staged = !bf && ov_staged(h, ov_mode);
    if (h.empty()) return DPP_OK;
    int mc = 1, mt = 1, mblk = 1;
    double by = 0, fl = 0;
    for (const OvTask& t : h) {
        mc = std::max(mc, t.nchunk);
        mt = std::max(mt, t.ntiles);
        mblk = std::max(mblk, ov_narrow ? t.ntiles : ov_task_blocks((t.nbA + 15) / 16, t.tilesB, staged));
        by += 16.0 * t.npw * (t.nbA + t.nbB);
        fl += 8.0 * t.npw * t.nbA * (double)t.nbB;
    }
    if (mt > 65535 || h.size() > 65535) return set_error(DPP_EUNSUPPORTED, "overlap: batch too large");
    {
        TimerScope ts_(ctx, act ? DPP_TK_MASKED : DPP_TK_OVERLAP, act ? 0.0 : by, act ? 0.0 : fl);
        if (wide) {
            int ms = 1;
            for (const OvTask& t : h) ms = std::max(ms, ovw_slices(t.npw));
            const dim3 grid = d_work ? dim3((unsigned)nwork) : dim3(ms, h.size());
            hipLaunchKernelGGL(k_overlap_bf16_wg, grid, dim3(64 * OVW_WAVES), 0, ctx->stream, d_tasks, OvTask{},
                               part, act, d_work);
        } else if (bf) {
            const dim3 grid = d_work ? dim3((unsigned)nwork) : dim3(mc, mblk, h.size());
            hipLaunchKernelGGL(k_overlap_bf16, grid, dim3(64 * OVB_WAVES), 0, ctx->stream, d_tasks, OvTask{}, part,
                               act, d_work);
        } else if (staged) {
            const dim3 grid = d_work ? dim3((unsigned)nwork) : dim3(mc, mblk, h.size());
            hipLaunchKernelGGL(k_overlap_staged, grid, dim3(OVS_THREADS), 0, ctx->stream, d_tasks, OvTask{}, part, act,
                               d_work);
        } else {
            overlap_launch(ctx, d_tasks, OvTask{}, (unsigned)h.size(), mc, mblk, mt > 1 && !ov_narrow, part, act,
                           full, d_work, nwork);
        }
        DPP_LAUNCHED();
    }
    if (full) return DPP_OK;
    TimerScope ts2_(ctx, act ? DPP_TK_MASKED : DPP_TK_BLOCKOPS);
    if (wide)
        hipLaunchKernelGGL(k_overlap_reduce_slices, dim3((mt * 256 + OVR_OUT - 1) / OVR_OUT, (unsigned)h.size()), dim3(256), 0,
                           ctx->stream, d_tasks, OvTask{}, (const double2*)part, act);
    else
        hipLaunchKernelGGL(k_overlap_reduce, dim3((mt * 256 + OVR_OUT - 1) / OVR_OUT, (unsigned)h.size()), dim3(256), 0,
                           ctx->stream, d_tasks, OvTask{}, (const double2*)part, act);
    DPP_LAUNCHED();
    return DPP_OK;
}

// ---------------------------------------------------------------- X M ------
// One wave owns PT tiles of 16 consecutive sphere points and up to JT x 16
// output bands in accumulators; X is read once, each M value once per wave
// and K step for all PT point tiles.  The loads of the next K step are issued
// before the MFMAs of the current one.  Outputs of one or two tiles take
// PT > 1 when the batch still gives every CU many waves; wider outputs run
// k_rotate_staged (below).
// F32 (the mixed-precision bulk): X and M rounded to FP32, FP32 MFMA and
// accumulation over the bands, the result (and beta out) in FP64.
template <int PT, int JT, bool F32>
__global__ void __launch_bounds__(64 * RT_WAVES)
k_rotate_mfma(const RotTask* __restrict__ tasks, RotTask single, int jt0_in, int ngrp, const int* __restrict__ act,
              const int2* __restrict__ work) {
    using acc_t = typename std::conditional<F32, f4, d4>::type;
    using real_t = typename std::conditional<F32, float, double>::type;
    // a work list (task, block) covers only the workgroups with points; a
    // block is (point block, group of JT output tiles) when ngrp > 1
    const int2 wk = work ? work[blockIdx.x] : int2{(int)blockIdx.y, (int)blockIdx.x};
    const RotTask T = tasks ? tasks[wk.x] : single;
    if (act && !act[T.item]) return;
    const int jt0 = jt0_in + (wk.y % ngrp) * JT;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int gt = ((wk.y / ngrp) * RT_WAVES + w) * PT;
    if (gt * 16 >= T.npw) return;
    const int njt = min(JT, (T.nbO + 15) / 16 - jt0);
    if (njt <= 0) return;
    const int c = lane & 15, ks = lane >> 4;
    acc_t dre[PT][JT], dim[PT][JT];
#pragma unroll
    for (int u = 0; u < PT; ++u)
#pragma unroll
        for (int t = 0; t < JT; ++t) {
            dre[u][t] = acc_t{0, 0, 0, 0};
            dim[u][t] = acc_t{0, 0, 0, 0};
        }
    const int nterm = T.nbX2 > 0 ? 2 : 1;
    // K steps run over the rows of X then those of X2
    const int nk1 = (T.nbX + 3) / 4, nk = nk1 + (nterm == 2 ? (T.nbX2 + 3) / 4 : 0);
    // Loads use clamped, in-bounds addresses and are unconditional.  Rows of
    // K beyond the band count get M = 0 (applied when the values are used, so
    // the next step's loads stay in flight); padded points and output bands
    // are computed from finite data and never stored.
    double2 xn[PT], mn[JT];
    auto load = [&](int kstep) {
        const bool second = kstep >= nk1;
        const double2* Xs = second ? T.X2 : T.X;
        const double2* Ms = second ? T.M2 : T.M;
        const int nbx = second ? T.nbX2 : T.nbX;
        const int ic = min((second ? kstep - nk1 : kstep) * 4 + ks, nbx - 1);
#pragma unroll
        for (int u = 0; u < PT; ++u) xn[u] = gld(Xs + (int64_t)ic * T.ldX + min((gt + u) * 16 + c, T.npw - 1));
#pragma unroll
        for (int t = 0; t < JT; ++t)
            mn[t] = gld(Ms + (int64_t)ic * T.M_ld + min((jt0 + min(t, njt - 1)) * 16 + c, T.nbO - 1));
    };
    if (nk > 0) load(0);
    for (int k = 0; k < nk; ++k) {
        const bool second = k >= nk1;
        const bool vi = (second ? k - nk1 : k) * 4 + ks < (second ? T.nbX2 : T.nbX);
        double2 x[PT], m[JT];
#pragma unroll
        for (int u = 0; u < PT; ++u) x[u] = xn[u];
#pragma unroll
        for (int t = 0; t < JT; ++t) m[t] = vi ? mn[t] : double2{0, 0};
        if (k + 1 < nk) load(k + 1);
#pragma unroll
        for (int t = 0; t < JT; ++t) {
            if (t < njt) {
                const real_t mr = (real_t)m[t].x, mi = (real_t)m[t].y;
#pragma unroll
                for (int u = 0; u < PT; ++u) {
                    const real_t xr = (real_t)x[u].x, xi = (real_t)x[u].y;
                    dre[u][t] = mfma(mr, xr, dre[u][t]);
                    dre[u][t] = mfma(-mi, xi, dre[u][t]);
                    dim[u][t] = mfma(mi, xr, dim[u][t]);
                    dim[u][t] = mfma(mr, xi, dim[u][t]);
                }
            }
        }
    }
#pragma unroll
    for (int u = 0; u < PT; ++u) {
        const int q = (gt + u) * 16 + c;
        if (q >= T.npw) continue;
#pragma unroll
        for (int t = 0; t < JT; ++t) {
            if (t < njt) {
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    // result row of element v: 4 v + l / 16 (FP64), 4 (l / 16) + v (FP32)
                    const int j = (jt0 + t) * 16 + (F32 ? 4 * ks + v : 4 * v + ks);
                    if (j < T.nbO) {
                        double2* o = T.out + (int64_t)j * T.ldout + q;
                        double2 r = double2{(double)dre[u][t][v], (double)dim[u][t][v]};
                        if (T.beta != 0.0) {
                            const double2 p = *o;
                            r.x += T.beta * p.x;
                            r.y += T.beta * p.y;
                        }
                        *o = r;
                    }
                }
            }
        }
    }
}

// Outputs of more than two 16-band tiles: RS_WAVES waves per workgroup, one
// 16-point tile each, share the rows of M through LDS.  M is staged 16 K rows
// (four MFMA steps) at a time for the RT_JT output tiles from jt0,
// double-buffered (F32: rounded to FP32 when staged, as k_rotate_mfma rounds
// it at use); X is read by its own wave as in k_rotate_mfma.  The K order
// (rows of X, then of X2), the padding rules and the output are those of
// k_rotate_mfma, so both give the same sums.
constexpr int RS_WAVES = 8;
constexpr int RS_COLS = RT_JT * 16;

template <bool F32>
__global__ void __launch_bounds__(64 * RS_WAVES)
k_rotate_staged(const RotTask* __restrict__ tasks, RotTask single, int jt0, const int* __restrict__ act,
                const int2* __restrict__ work) {
    using acc_t = typename std::conditional<F32, f4, d4>::type;
    using real_t = typename std::conditional<F32, float, double>::type;
    using mt = typename std::conditional<F32, float2, double2>::type;
    __shared__ mt ms[2][16 * RS_COLS];
    const int2 wk = work ? work[blockIdx.x] : int2{(int)blockIdx.y, (int)blockIdx.x};
    const RotTask T = tasks ? tasks[wk.x] : single;
    if (act && !act[T.item]) return;
    // uniform over the wave (readfirstlane): the per-tile branches below then
    // stay scalar, instead of masking the MFMAs and copying their accumulators
    const int njt = __builtin_amdgcn_readfirstlane(min(RT_JT, (T.nbO + 15) / 16 - jt0));
    if (njt <= 0) return;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int gt = wk.y * RS_WAVES + w;
    if (wk.y * RS_WAVES * 16 >= T.npw) return;  // uniform over the workgroup
    const bool live = gt * 16 < T.npw;          // waves past the points still stage M
    const int c = lane & 15, ks = lane >> 4;
    const int nk1 = (T.nbX + 3) / 4, nk = nk1 + (T.nbX2 > 0 ? (T.nbX2 + 3) / 4 : 0);
    const int nch = (nk + 3) / 4;
    // K step k, sub-row r4: the term, its row and whether the row exists
    auto krow = [&](int k, int r4, bool& second, int& ic) {
        second = k >= nk1;
        const int nbx = second ? T.nbX2 : T.nbX;
        const int row = (second ? k - nk1 : k) * 4 + r4;
        ic = min(row, nbx - 1);
        return k < nk && row < nbx;
    };
    // staging: element e = tid + 512 i (i < 4) of the chunk is K row e / RS_COLS
    // (step e / (4 RS_COLS), sub-row (e / RS_COLS) % 4), output band jt0 16 + e % RS_COLS
    double2 mraw[4];
    auto mload = [&](int ch) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int e = tid + 64 * RS_WAVES * i, kk = e / RS_COLS, col = e - kk * RS_COLS;
            bool second;
            int ic;
            const bool ok = krow(4 * ch + kk / 4, kk % 4, second, ic);
            const double2* Ms = second ? T.M2 : T.M;
            const int j = min(jt0 * 16 + col, T.nbO - 1);
            mraw[i] = ok ? gld(Ms + (int64_t)ic * T.M_ld + j) : double2{0, 0};
        }
    };
    auto mstage = [&](int buf) {
#pragma unroll
        for (int i = 0; i < 4; ++i) ms[buf][tid + 64 * RS_WAVES * i] = mt{(real_t)mraw[i].x, (real_t)mraw[i].y};
    };
    double2 xn[4];
    auto xload = [&](int ch) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            bool second;
            int ic;
            // steps past the last one (the chunk's tail) have no row to read
            const bool ok = 4 * ch + q < nk;
            krow(4 * ch + q, ks, second, ic);
            const double2* Xs = second ? T.X2 : T.X;
            xn[q] = ok ? gld(Xs + (int64_t)ic * T.ldX + min(gt * 16 + c, T.npw - 1)) : double2{0, 0};
        }
    };
    acc_t dre[RT_JT], dim[RT_JT];
#pragma unroll
    for (int t = 0; t < RT_JT; ++t) {
        dre[t] = acc_t{0, 0, 0, 0};
        dim[t] = acc_t{0, 0, 0, 0};
    }
    if (nch > 0) {
        mload(0);
        xload(0);
    }
    for (int ch = 0; ch < nch; ++ch) {
        const int buf = ch & 1;
        mstage(buf);
        double2 x[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) x[q] = xn[q];
        if (ch + 1 < nch) {
            mload(ch + 1);
            xload(ch + 1);
        }
        __syncthreads();
        const mt* M = ms[buf];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const real_t xr = (real_t)x[q].x, xi = (real_t)x[q].y;
#pragma unroll
            for (int t = 0; t < RT_JT; ++t) {
                // FP32 runs every tile (padding tiles read clamped, finite
                // columns and are not stored): with the per-tile condition the
                // compiler masks the MFMAs and spills their accumulators
                if (F32 || t < njt) {
                    const mt m = M[(4 * q + ks) * RS_COLS + t * 16 + c];
                    dre[t] = mfma(m.x, xr, dre[t]);
                    dre[t] = mfma(-m.y, xi, dre[t]);
                    dim[t] = mfma(m.y, xr, dim[t]);
                    dim[t] = mfma(m.x, xi, dim[t]);
                }
            }
            if constexpr (F32) __builtin_amdgcn_sched_barrier(0);
        }
    }
    const int q = gt * 16 + c;
    if (!live || q >= T.npw) return;
#pragma unroll
    for (int t = 0; t < RT_JT; ++t) {
        if (t < njt) {
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                // result row of element v: 4 v + l / 16 (FP64), 4 (l / 16) + v (FP32)
                const int j = (jt0 + t) * 16 + (F32 ? 4 * ks + v : 4 * v + ks);
                if (j < T.nbO) {
                    double2* o = T.out + (int64_t)j * T.ldout + q;
                    double2 r = double2{(double)dre[t][v], (double)dim[t][v]};
                    if (T.beta != 0.0) {
                        const double2 p = *o;
                        r.x += T.beta * p.x;
                        r.y += T.beta * p.y;
                    }
                    *o = r;
                }
            }
        }
    }
}

RotTask make_rot_task(int npw, int nbX, const double2* X, int64_t ldX, int nbO, const double2* M, int M_ld,
                      double beta, double2* out, int64_t ldout) {
    RotTask t;
    t.X = X;
    t.M = M;
    t.out = out;
    t.ldX = ldX;
    t.ldout = ldout;
    t.npw = npw;
    t.nbX = nbX;
    t.nbO = nbO;
    t.M_ld = M_ld;
    t.beta = beta;
    t.item = 0;
    t.nbX2 = 0;
    t.X2 = nullptr;
    t.M2 = nullptr;
    return t;
}

static double rot_bytes(const RotTask& t) {
    return 16.0 * t.npw * (t.nbX + t.nbX2 + t.nbO * (t.beta != 0.0 ? 2.0 : 1.0)) + 16.0 * (t.nbX + t.nbX2) * t.nbO;
}

template <int PT, int JT>
static void rotate_go(dpp_ctx ctx, const RotTask* d_tasks, const RotTask& single, unsigned ntasks, int ntile,
                      int jt0, const int* act, const int2* work, int nwork, bool f32, int ngrp = 1) {
    const int nblk = (ntile + RT_WAVES * PT - 1) / (RT_WAVES * PT);
    const dim3 grid = work ? dim3((unsigned)nwork) : dim3(nblk * ngrp, ntasks);
    if (f32)
        hipLaunchKernelGGL((k_rotate_mfma<PT, JT, true>), grid, dim3(64 * RT_WAVES), 0, ctx->stream, d_tasks, single,
                           jt0, ngrp, act, work);
    else
        hipLaunchKernelGGL((k_rotate_mfma<PT, JT, false>), grid, dim3(64 * RT_WAVES), 0, ctx->stream, d_tasks,
                           single, jt0, ngrp, act, work);
}

// Launch the rotate kernel shape for the widest output of a batch; tiles =
// point tiles summed over the tasks.  Several point tiles per wave only while
// the launch keeps at least RT_MIN_WAVES waves.
constexpr int64_t RT_MIN_WAVES = 4096;
// Point tiles per wave for outputs of jtiles 16-band tiles and `tiles` point
// tiles in all (rot_pt > 0 fixes it where the shape allows).
static int rotate_pt_rule(int jtiles, int64_t tiles, int rot_pt) {
    if (jtiles == 1) return rot_pt ? rot_pt : (tiles >= 4 * RT_MIN_WAVES ? 4 : tiles >= 2 * RT_MIN_WAVES ? 2 : 1);
    if (jtiles == 2) return (rot_pt ? rot_pt : (tiles >= 2 * RT_MIN_WAVES ? 2 : 1)) >= 2 ? 2 : 1;
    return 1;
}

static dpp_status rotate_launch(dpp_ctx ctx, const RotTask* d_tasks, const RotTask& single, unsigned ntasks,
                                int maxnpw, int maxnbO, int64_t tiles, const int* act, int rot_pt,
                                const int2* work, int nwork, bool f32) {
    const int ntile = (maxnpw + 15) / 16;
    const int jtiles = (maxnbO + 15) / 16;
    const int pt = rotate_pt_rule(jtiles, tiles, rot_pt);
    if (jtiles == 1) {
        if (pt == 4)
            rotate_go<4, 1>(ctx, d_tasks, single, ntasks, ntile, 0, act, work, nwork, f32);
        else if (pt == 2)
            rotate_go<2, 1>(ctx, d_tasks, single, ntasks, ntile, 0, act, work, nwork, f32);
        else
            rotate_go<1, 1>(ctx, d_tasks, single, ntasks, ntile, 0, act, work, nwork, f32);
    } else if (jtiles == 2) {
        if (pt == 2)
            rotate_go<2, 2>(ctx, d_tasks, single, ntasks, ntile, 0, act, work, nwork, f32);
        else
            rotate_go<1, 2>(ctx, d_tasks, single, ntasks, ntile, 0, act, work, nwork, f32);
    } else {
        const dim3 grid = work ? dim3((unsigned)nwork) : dim3((ntile + RS_WAVES - 1) / RS_WAVES, ntasks);
        for (int jt0 = 0; jt0 < jtiles; jt0 += RT_JT) {
            if (f32)
                hipLaunchKernelGGL(k_rotate_staged<true>, grid, dim3(64 * RS_WAVES), 0, ctx->stream, d_tasks, single,
                                   jt0, act, work);
            else
                hipLaunchKernelGGL(k_rotate_staged<false>, grid, dim3(64 * RS_WAVES), 0, ctx->stream, d_tasks,
                                   single, jt0, act, work);
        }
    }
    DPP_LAUNCHED();
    return DPP_OK;
}

static void rotate_shape(const std::vector<RotTask>& h, int& mp, int& mj, int64_t& tiles) {
    mp = 1, mj = 1, tiles = 0;
    for (const RotTask& t : h) {
        mp = std::max(mp, t.npw);
        mj = std::max(mj, (t.nbO + 15) / 16);
        tiles += (t.npw + 15) / 16;
    }
}

void rotate_worklist(const std::vector<RotTask>& h, int rot_pt, std::vector<int2>& w, bool f32) {
    int mp, mj;
    int64_t tiles;
    rotate_shape(h, mp, mj, tiles);
    const int pt = rotate_pt_rule(mj, tiles, rot_pt);
    // point tiles per block (k_rotate_staged above two output tiles, in both precisions)
    const int per = mj > 2 ? RS_WAVES : RT_WAVES * pt;
    (void)f32;
    w.clear();
    for (size_t i = 0; i < h.size(); ++i) {
        const int nblk = ((h[i].npw + 15) / 16 + per - 1) / per;
        for (int b = 0; b < nblk; ++b) w.push_back(int2{(int)i, b});
    }
}

dpp_status rotate_single(dpp_ctx ctx, int npw, int nbX, const double2* X, int64_t ldX, int nbO,
                         const double2* M, double beta, double2* out, int64_t ldout, dpp_precision prec) {
    RotTask t = make_rot_task(npw, nbX, X, ldX, nbO, M, nbO, beta, out, ldout);
    TimerScope ts_(ctx, DPP_TK_ROTATE, rot_bytes(t), 8.0 * npw * nbX * (double)nbO);
    return rotate_launch(ctx, nullptr, t, 1, npw, nbO, (npw + 15) / 16, nullptr, 0, nullptr, 0, prec == DPP_F32);
}

dpp_status rotate_tasks(dpp_ctx ctx, const std::vector<RotTask>& h, const RotTask* d_tasks, const int* act,
                        int rot_pt, const int2* d_work, int nwork, dpp_precision prec) {
    if (h.empty()) return DPP_OK;
    int mp = 1, mj = 1;
    int64_t tiles = 0;
    double by = 0, fl = 0;
    for (const RotTask& t : h) {
        mp = std::max(mp, t.npw);
        tiles += (t.npw + 15) / 16;
        mj = std::max(mj, (t.nbO + 15) / 16);
        by += rot_bytes(t);
        fl += 8.0 * t.npw * (t.nbX + t.nbX2) * (double)t.nbO;
    }
    TimerScope ts_(ctx, act ? DPP_TK_MASKED : DPP_TK_ROTATE, act ? 0.0 : by, act ? 0.0 : fl);
    return rotate_launch(ctx, d_tasks, RotTask{}, (unsigned)h.size(), mp, mj * 16, tiles, act, rot_pt, d_work, nwork,
                         prec == DPP_F32);
}

// ------------------------------------------------- small-matrix products ---
// Per item n x n (row-major at moff, n = nbo or the item's band count):
// C = alpha op(A) op(B) + beta C with op = N or H; alpha times the cell volume
// if alpha_omega.  One wave per 16 x 16 tile of C (blockIdx.x), items on
// blockIdx.y; complex products from four real FP64 MFMAs per K step.
__global__ void __launch_bounds__(64)
k_smm_mfma(const Seg* __restrict__ seg, int nbo, int opA, int opB, double alpha0, int alpha_omega,
           const double2* __restrict__ A, const double2* __restrict__ B, double beta, double2* __restrict__ Cm) {
    const Seg sg = seg[blockIdx.y];
    const int n = nbo > 0 ? nbo : sg.nb;
    const int tn = (n + 15) / 16;
    const int tile = blockIdx.x;
    if (tile >= tn * tn) return;
    const int ti = tile / tn, tj = tile - ti * tn;
    const int lane = threadIdx.x;
    const int r = lane & 15, ks = lane >> 4;
    const int i = ti * 16 + r, j = tj * 16 + r;
    const double2* Ab = A + sg.moff;
    const double2* Bb = B + sg.moff;
    d4 cre = {0, 0, 0, 0}, cim = {0, 0, 0, 0};
    for (int k0 = 0; k0 < n; k0 += 4) {
        const int k = k0 + ks;
        double2 a = double2{0, 0}, b = double2{0, 0};
        if (k < n) {
            if (i < n) {
                a = opA ? Ab[(int64_t)k * n + i] : Ab[(int64_t)i * n + k];
                if (opA) a.y = -a.y;
            }
            if (j < n) {
                b = opB ? Bb[(int64_t)j * n + k] : Bb[(int64_t)k * n + j];
                if (opB) b.y = -b.y;
            }
        }
        cre = mfma(a.x, b.x, cre);
        cre = mfma(-a.y, b.y, cre);
        cim = mfma(a.x, b.y, cim);
        cim = mfma(a.y, b.x, cim);
    }
    const double alpha = alpha_omega ? alpha0 * sg.omega : alpha0;
    double2* Cb = Cm + sg.moff;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const int ii = ti * 16 + 4 * v + (lane >> 4), jj = tj * 16 + (lane & 15);
        if (ii < n && jj < n) {
            double2 o = double2{alpha * cre[v], alpha * cim[v]};
            if (beta != 0.0) {
                const double2 c = Cb[(int64_t)ii * n + jj];
                o.x += beta * c.x;
                o.y += beta * c.y;
            }
            Cb[(int64_t)ii * n + jj] = o;
        }
    }
}

// ------------------------------------------------------------ Cholesky -----
// Up to 32 bands one wave per matrix (below); 33 to 128 bands run on register
// tiles (dense.hip).
constexpr int CH_MAXN = 128;
constexpr double CH_PIVOT_RTOL = PIVOT_RTOL;

// ------------------------------------------ single-wave Cholesky inverse ---
// U = R^dag R and X = R^{-1} for n <= NMAX (16 or 32) in one wave.  The
// factorization holds the upper triangle of U in registers, lane (j, g)
// owning rows g*RPL .. g*RPL + RPL - 1 of column j; step k reads the pivot
// from its lane, scales row k, publishes it in LDS (row k of R) and every
// lane updates its own entries, so a step costs one LDS round trip.  The
// inverse holds row i of X in lane i and runs the recurrence
//   X[i][j] R[j][j] = delta_ij - sum_{k<j} X[i][k] R[k][j]
// over j with R read from LDS.  Returns 1 (uniform) when a pivot falls
// below CH_PIVOT_RTOL times the largest diagonal element.
template <int NMAX>
struct CholWaveLds {
    double2 R[NMAX][NMAX + 1];  // rows of R (upper triangle; zeros below)
    double rinv[NMAX];          // 1 / R[k][k]
    double2 X[NMAX][NMAX + 1];  // R^{-1}, row-major, zeros below the diagonal
};

__device__ __forceinline__ double lane_read(double v, int l) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)b, l);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
    return v;
}

__device__ __forceinline__ double wave_sum64(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

template <int NMAX, typename Load>
__device__ int chol_inv_wave(int n, Load load, CholWaveLds<NMAX>& L) {
    constexpr int G = 64 / NMAX, RPL = NMAX / G;
    const int lane = threadIdx.x;
    const int j = lane % NMAX, g = lane / NMAX;
    double2 a[RPL];
    double dmax = 0.0;
#pragma unroll
    for (int r = 0; r < RPL; ++r) {
        const int i = g * RPL + r;
        double2 v = double2{0.0, 0.0};
        if (i <= j && j < n) v = load(i, j);
        if (i == j) {
            v.y = 0.0;
            dmax = fmax(dmax, v.x);
        }
        a[r] = v;
    }
    dmax = wave_max(dmax);
    int failed = 0;
#pragma unroll
    for (int k = 0; k < NMAX; ++k) {
        // (no early exit: a fully unrolled loop keeps a[] in registers)
        if (k >= n || failed) continue;
        const double d = lane_read(a[k % RPL].x, k + NMAX * (k / RPL));
        if (!(d > CH_PIVOT_RTOL * dmax)) {
            failed = 1;
            continue;
        }
        const double rkk = sqrt(d), inv = 1.0 / rkk;
        if (g == k / RPL) {
            const double2 v = a[k % RPL];
            const double2 w = j > k ? double2{v.x * inv, v.y * inv} : (j == k ? double2{rkk, 0.0} : double2{0.0, 0.0});
            a[k % RPL] = w;
            L.R[k][j] = w;
        }
        if (lane == 0) L.rinv[k] = inv;
        __syncthreads();
        const double2 rkj = L.R[k][j];
#pragma unroll
        for (int r = 0; r < RPL; ++r) {
            const int i = g * RPL + r;
            if (i > k && i <= j) {
                const double2 rki = L.R[k][i];
                a[r].x -= rki.x * rkj.x + rki.y * rkj.y;  // conj(R[k][i]) R[k][j]
                a[r].y -= rki.x * rkj.y - rki.y * rkj.x;
            }
        }
    }
    if (failed) return 1;
    double2 x[NMAX];
#pragma unroll
    for (int m = 0; m < NMAX; ++m) x[m] = double2{0.0, 0.0};
    const int i = lane;
#pragma unroll
    for (int jj = 0; jj < NMAX; ++jj) {
        if (jj >= n) continue;
        double sr = i == jj ? 1.0 : 0.0, si = 0.0;
#pragma unroll
        for (int k = 0; k < jj; ++k) {
            const double2 r = L.R[k][jj];
            sr -= x[k].x * r.x - x[k].y * r.y;
            si -= x[k].x * r.y + x[k].y * r.x;
        }
        const double ri = L.rinv[jj];
        x[jj] = double2{sr * ri, si * ri};
    }
    if (i < NMAX) {
#pragma unroll
        for (int m = 0; m < NMAX; ++m) L.X[i][m] = x[m];
    }
    __syncthreads();
    return 0;
}

template <int NMAX>
__global__ void __launch_bounds__(64)
k_cholesky_wave(int n, int64_t stride, const Seg* __restrict__ seg, int nbo, const double2* __restrict__ U,
                double2* __restrict__ Rinv, int* __restrict__ status, const int* __restrict__ act) {
    if (act && !act[blockIdx.x]) return;
    __shared__ CholWaveLds<NMAX> L;
    int64_t off = (int64_t)blockIdx.x * stride;
    if (seg) {
        const Seg sg = seg[blockIdx.x];
        n = nbo > 0 ? nbo : sg.nb;
        off = sg.moff;
    }
    const double2* Ug = U + off;
    const int f = chol_inv_wave<NMAX>(n, [&](int r, int c) { return Ug[r * n + c]; }, L);
    double2* X = Rinv + off;
    if (f) {
        if (threadIdx.x == 0 && status) atomicOr(status, DPP_STATUS_NOTPD);
        for (int e = threadIdx.x; e < n * n; e += 64) X[e] = double2{NAN, NAN};
        return;
    }
    for (int e = threadIdx.x; e < n * n; e += 64) {
        const int r = e / n, c = e - r * n;
        X[e] = L.X[r][c];
    }
}

// Band-energy line search of every active item, entirely on the device (one
// wave per item up to 32 bands; register tiles above).  Along D the trial energy is
//   E(a) = Tr(U(a)^{-1} H(a)),  U(a) = U + a (X + X^dag) + a^2 Q,
//   H(a) = H0 + a (H1 + H1^dag) + a^2 H2,
// evaluated through the Cholesky factor of U(a).  Step rule: trial a_t (the
// item's last accepted step), fit E0 + d0 a + c a^2 through E(a_t), take
// a* = -d0 / (2c) if c > 0 else 2 a_t, at most 10 a_t; accept a* if
// E(a*) <= E0, else a_t if E(a_t) <= E0, else halve a_t (at most MAX_TRIES
// times).  Writes ok[item] and step[item] (0 when the search failed).
constexpr int LS_MAX_TRIES = 6;

// The line search for n <= NMAX bands in one wave: H(a) staged in LDS, the
// factor and inverse of U(a) from chol_inv_wave, and
//   E(a) = Re Tr(X^dag H(a) X) = sum_{a' <= i} Re conj(X[a'][i]) (H(a) X)[a'][i]
// over (a', i) entries spread across the lanes.
template <int NMAX>
__device__ double trial_energy_wave(const Seg& sg, double a, const double2* __restrict__ U,
                                    const double2* __restrict__ Xs, const double2* __restrict__ Q,
                                    const double2* __restrict__ H0, const double2* __restrict__ Ps,
                                    const double2* __restrict__ H2, CholWaveLds<NMAX>& L,
                                    double2 (*Hs)[NMAX + 1]) {
    const int n = sg.nb;
    const int64_t o = sg.moff;
    for (int e = threadIdx.x; e < n * n; e += 64) {
        const int r = e / n, c = e - r * n;
        const double2 h = Ps[o + e], h0 = H0[o + e], h2 = H2[o + e];
        Hs[r][c] = double2{h0.x + a * h.x + a * a * h2.x, h0.y + a * h.y + a * a * h2.y};
    }
    // (the staging is ordered before its use by the barriers of the factorization)
    const int failed = chol_inv_wave<NMAX>(
        n,
        [&](int r, int c) {
            const double2 x = Xs[o + r * n + c], u = U[o + r * n + c], q = Q[o + r * n + c];
            return double2{u.x + a * x.x + a * a * q.x, u.y + a * x.y + a * a * q.y};
        },
        L);
    if (failed) return NAN;
    double acc = 0.0;
    for (int e = threadIdx.x; e < n * n; e += 64) {
        const int ar = e / n, i = e - ar * n;
        if (ar > i) continue;
        double wr = 0.0, wi = 0.0;
        for (int t = 0; t <= i; ++t) {
            const double2 h = Hs[ar][t], r = L.X[t][i];
            wr += h.x * r.x - h.y * r.y;
            wi += h.x * r.y + h.y * r.x;
        }
        const double2 ra = L.X[ar][i];
        acc += ra.x * wr + ra.y * wi;
    }
    acc = wave_sum64(acc);
    __syncthreads();  // LDS is reused by the next trial
    return acc;
}

template <int NMAX>
__global__ void __launch_bounds__(64)
k_linesearch_wave(const Seg* __restrict__ seg, const double2* __restrict__ U, const double2* __restrict__ X,
                  const double2* __restrict__ Q, const double2* __restrict__ H0, const double2* __restrict__ H1,
                  const double2* __restrict__ H2, const double* __restrict__ E0v, const double* __restrict__ at0,
                  const double* __restrict__ d0v, const int* __restrict__ act, int* __restrict__ ok,
                  double* __restrict__ step, double2* __restrict__ Xs, double2* __restrict__ Ps) {
    const int k = blockIdx.x;
    if (!act[k]) return;
    __shared__ CholWaveLds<NMAX> L;
    __shared__ double2 Hs[NMAX][NMAX + 1];
    const Seg sg = seg[k];
    {
        const int n = sg.nb;
        const int64_t o = sg.moff;
        for (int e = threadIdx.x; e < n * n; e += 64) {
            const int r = e / n, c = e - r * n;
            const double2 x = X[o + e], xt = X[o + c * n + r];
            const double2 h = H1[o + e], ht = H1[o + c * n + r];
            Xs[o + e] = double2{x.x + xt.x, x.y - xt.y};
            Ps[o + e] = double2{h.x + ht.x, h.y - ht.y};
        }
        __syncthreads();
    }
    const double E0 = E0v[k], d0 = d0v[k];
    double at = at0[k];
    int good = 0;
    double st = 0.0;
    for (int t = 0; t < LS_MAX_TRIES; ++t) {
        const double Et = trial_energy_wave<NMAX>(sg, at, U, Xs, Q, H0, Ps, H2, L, Hs);
        const double c = (Et - E0 - d0 * at) / (at * at);
        double as = c > 0 ? -d0 / (2.0 * c) : 2.0 * at;
        as = fmin(as, 10.0 * at);
        const double Es = trial_energy_wave<NMAX>(sg, as, U, Xs, Q, H0, Ps, H2, L, Hs);
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

// Band-gradient preparation of one item in one wave (n <= NMAX):
//   R^dag R = U,  Rinv = R^{-1},  M1 = Rinv Rinv^dag = U^{-1},
//   M2 = -Omega (M1 H0) M1,  E0 = Re Tr(M1 H0),
// the five small steps of the gradient at the current point in one launch.
// On a failed factorization Rinv, M1 and M2 are NaN, E0 is NaN and the
// status word latches DPP_STATUS_NOTPD.
// With `step` the point moved by a = step[item] along the line whose
// matrices X = Y^dag O D, Q = D^dag O D, H1 = Y^dag H D, H2 = D^dag H D are
// given: U and H0 are first advanced to U + a (X + X^dag) + a^2 Q and
// H0 + a (H1 + H1^dag) + a^2 H2 (the overlaps at Y + a D, as the line search
// models them) and written back.
template <int NMAX>
__global__ void __launch_bounds__(64)
k_grad_prep_wave(const Seg* __restrict__ seg, double2* __restrict__ U, double2* __restrict__ H0,
                 double2* __restrict__ Rinv, double2* __restrict__ M1, double2* __restrict__ M2,
                 double* __restrict__ E0, int* __restrict__ status, const double* __restrict__ step,
                 const double2* __restrict__ X, const double2* __restrict__ Q, const double2* __restrict__ H1,
                 const double2* __restrict__ H2) {
    constexpr int PER = (NMAX * NMAX + 63) / 64;
    __shared__ CholWaveLds<NMAX> L;
    __shared__ double2 Hs[NMAX][NMAX + 1];
    // U is staged in L.X: the factorization reads its input before it
    // writes X
    double2 (*Us)[NMAX + 1] = L.X;
    const Seg sg = seg[blockIdx.x];
    const int n = sg.nb;
    const int64_t o = sg.moff;
    const int lane = threadIdx.x;
    const double a = step ? step[blockIdx.x] : 0.0;
    for (int e = lane; e < n * n; e += 64) {
        const int r = e / n, c = e - r * n;
        double2 u = U[o + e], h = H0[o + e];
        if (step && a != 0.0) {
            const double2 x = X[o + e], xt = X[o + c * n + r], q = Q[o + e];
            const double2 p = H1[o + e], pt = H1[o + c * n + r], h2 = H2[o + e];
            u = double2{u.x + a * (x.x + xt.x) + a * a * q.x, u.y + a * (x.y - xt.y) + a * a * q.y};
            h = double2{h.x + a * (p.x + pt.x) + a * a * h2.x, h.y + a * (p.y - pt.y) + a * a * h2.y};
        }
        Us[r][c] = u;
        Hs[r][c] = h;
    }
    __syncthreads();
    if (step && a != 0.0)
        for (int e = lane; e < n * n; e += 64) {
            U[o + e] = Us[e / n][e % n];
            H0[o + e] = Hs[e / n][e % n];
        }
    const int f = chol_inv_wave<NMAX>(n, [&](int r, int c) { return Us[r][c]; }, L);
    if (f) {
        if (lane == 0) {
            if (status) atomicOr(status, DPP_STATUS_NOTPD);
            E0[blockIdx.x] = NAN;
        }
        for (int e = lane; e < n * n; e += 64) {
            Rinv[o + e] = double2{NAN, NAN};
            M1[o + e] = double2{NAN, NAN};
            M2[o + e] = double2{NAN, NAN};
        }
        return;
    }
    // M1 = X X^dag (X = Rinv upper triangular): entries into L.R (R is dead)
#pragma unroll
    for (int u = 0; u < PER; ++u) {
        const int e = lane + 64 * u;
        if (e < n * n) {
            const int i = e / n, j = e - (e / n) * n;
            Rinv[o + e] = L.X[i][j];
            double sr = 0.0, si = 0.0;
            for (int k = max(i, j); k < n; ++k) {
                const double2 a = L.X[i][k], b = L.X[j][k];
                sr += a.x * b.x + a.y * b.y;  // a conj(b)
                si += a.y * b.x - a.x * b.y;
            }
            L.R[i][j] = double2{sr, si};
            M1[o + e] = double2{sr, si};
        }
    }
    __syncthreads();
    // Rt = M1 H0 into L.X (X is dead once every lane passed the barrier)
    double2 rt[PER];
    double tr = 0.0;
#pragma unroll
    for (int u = 0; u < PER; ++u) {
        const int e = lane + 64 * u;
        rt[u] = double2{0.0, 0.0};
        if (e < n * n) {
            const int i = e / n, j = e - (e / n) * n;
            double sr = 0.0, si = 0.0;
            for (int k = 0; k < n; ++k) {
                const double2 a = L.R[i][k], b = Hs[k][j];
                sr += a.x * b.x - a.y * b.y;
                si += a.x * b.y + a.y * b.x;
            }
            rt[u] = double2{sr, si};
            if (i == j) tr += sr;
        }
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < PER; ++u) {
        const int e = lane + 64 * u;
        if (e < n * n) L.X[e / n][e % n] = rt[u];
    }
    tr = wave_sum64(tr);
    if (lane == 0) E0[blockIdx.x] = tr;
    __syncthreads();
    // M2 = -Omega Rt M1
    const double sc = -sg.omega;
#pragma unroll
    for (int u = 0; u < PER; ++u) {
        const int e = lane + 64 * u;
        if (e < n * n) {
            const int i = e / n, j = e - (e / n) * n;
            double sr = 0.0, si = 0.0;
            for (int k = 0; k < n; ++k) {
                const double2 a = L.X[i][k], b = L.R[k][j];
                sr += a.x * b.x - a.y * b.y;
                si += a.x * b.y + a.y * b.x;
            }
            M2[o + e] = double2{sc * sr, sc * si};
        }
    }
}

bool grad_prep_wave_launch(hipStream_t st, unsigned nblk, int nmax, const Seg* seg, double2* U, double2* H0,
                           double2* Rinv, double2* M1, double2* M2, double* E0, int* status, const double* step,
                           const double2* X, const double2* Q, const double2* H1, const double2* H2) {
    if (nmax <= 16)
        hipLaunchKernelGGL(k_grad_prep_wave<16>, dim3(nblk), dim3(64), 0, st, seg, U, H0, Rinv, M1, M2, E0, status,
                           step, X, Q, H1, H2);
    else if (nmax <= 32)
        hipLaunchKernelGGL(k_grad_prep_wave<32>, dim3(nblk), dim3(64), 0, st, seg, U, H0, Rinv, M1, M2, E0, status,
                           step, X, Q, H1, H2);
    else
        return false;
    return true;
}

// Launch helpers for the single-wave paths (n <= 32); false: use the
// general kernels.
bool cholesky_wave_launch(hipStream_t st, unsigned nblk, int n, int64_t stride, const Seg* seg, int nbo,
                          const double2* U, double2* Rinv, int* status, const int* act) {
    if (n <= 16)
        hipLaunchKernelGGL(k_cholesky_wave<16>, dim3(nblk), dim3(64), 0, st, n, stride, seg, nbo, U, Rinv, status,
                           act);
    else if (n <= 32)
        hipLaunchKernelGGL(k_cholesky_wave<32>, dim3(nblk), dim3(64), 0, st, n, stride, seg, nbo, U, Rinv, status,
                           act);
    else
        return false;
    return true;
}

bool linesearch_wave_launch(hipStream_t st, unsigned nblk, int n, const Seg* seg, const double2* U,
                            const double2* X, const double2* Q, const double2* H0, const double2* H1,
                            const double2* H2, const double* E0v, const double* at0, const double* d0v,
                            const int* act, int* ok, double* step, double2* Xs, double2* Ps) {
    if (n <= 16)
        hipLaunchKernelGGL(k_linesearch_wave<16>, dim3(nblk), dim3(64), 0, st, seg, U, X, Q, H0, H1, H2, E0v, at0,
                           d0v, act, ok, step, Xs, Ps);
    else if (n <= 32)
        hipLaunchKernelGGL(k_linesearch_wave<32>, dim3(nblk), dim3(64), 0, st, seg, U, X, Q, H0, H1, H2, E0v, at0,
                           d0v, act, ok, step, Xs, Ps);
    else
        return false;
    return true;
}

// ----------------------------------------------------- Jacobi eigensolver --
// Parallel cyclic Jacobi on a Hermitian matrix of up to 32 bands, one wave
// per matrix.  Each round rotates m/2 disjoint index pairs of a round-robin
// tournament (circle schedule: pair 0 = (m-1, r), pair s = ((r+s) mod (m-1),
// (r-s) mod (m-1)); m = n rounded up to even, index n a dummy).  For the pair
// (p,q) with A_pq = |c| e^{i phi}, J = diag-phase * real rotation:
//   tau = (A_qq - A_pp) / (2|c|), t = sign(tau)/(|tau| + sqrt(1+tau^2)),
//   cs = 1/sqrt(1+t^2), sn = t cs,
//   J[p][p] = cs, J[p][q] = sn, J[q][p] = -sn e^{-i phi}, J[q][q] = cs e^{-i phi}
// and A <- J^dag A J, V <- V J.  33 to 128 bands use the tridiagonal
// eigensolver on register tiles (dense.hip).
constexpr int EIG_MAXN = 128;
constexpr int EIG_SWEEPS = 40;

// Squared relative off-diagonal norm at which the sweeps stop.
__device__ __forceinline__ double eig_stop2(int n) { return fmax(1e-28, 4e-32 * (double)n * (double)n); }

__device__ __forceinline__ double2 cmulz(double2 a, double2 b) {
    return double2{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}

// Built for the latency of a round: A is stored whole in LDS (row stride n + 1), so a 2x2 block is
// read and written without index folding; rotations take one reciprocal
// square root of |a_pq|^2 and no division by |a_pq|; the convergence norms
// are wave reductions; each workgroup barrier spans a single wave.
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

// Index pair of a slot in a round of the round-robin ordering over m
// (even) indices: slot 0 pairs m - 1 with the round, slot s pairs round + s
// with round - s (mod m - 1); returned with p < q.
__device__ __forceinline__ void jacobi_pair(int round, int slot, int m, int& p, int& q) {
    int a, b;
    if (slot == 0) {
        a = m - 1;
        b = round;
    } else {
        a = round + slot;
        a -= a >= m - 1 ? m - 1 : 0;
        b = round - slot;
        b += b < 0 ? m - 1 : 0;
    }
    p = min(a, b);
    q = max(a, b);
}

struct RotW {
    double cs, sn, er, ei;  // e^{-i phi} = er + i ei
};

// NMAX (16 or 32) bounds n; the per-round block and V loops have the
// compile-time trip counts of NMAX, so they unroll into one straight-line
// sequence whose loads the compiler can interleave.  Every lane takes the
// indices of its pairs from the round number, so its A and V loads do not
// wait for the rotations, and the identity rotation (pairs at rounding level,
// the padding index of odd n) is applied as an exact no-op instead of a
// branch; A and V are zero outside n x n so that padding stays finite.
template <int NMAX>
__device__ void jacobi_eigh_wave(int n, const double2* __restrict__ Hg, double* __restrict__ ev,
                                 double2* __restrict__ vo) {
    constexpr int LD = NMAX + 1, PMAX = NMAX / 2;
    __shared__ double2 A[NMAX * LD];
    __shared__ double2 Vt[NMAX * LD];
    __shared__ RotW rot[PMAX];
    __shared__ double dg[NMAX];
    __shared__ int perm[NMAX];
    const int lane = threadIdx.x;
    const int m = n + (n & 1), P = m / 2;
    for (int e = lane; e < NMAX * LD; e += 64) {
        A[e] = double2{0.0, 0.0};
        Vt[e] = double2{0.0, 0.0};
    }
    __syncthreads();
    for (int e = lane; e < n * n; e += 64) {
        const int r = e / n, c = e - r * n;
        double2 h = c >= r ? Hg[r * n + c] : Hg[c * n + r];
        if (c < r) h.y = -h.y;
        if (r == c) h.y = 0.0;
        A[r * LD + c] = h;
        Vt[r * LD + c] = double2{r == c ? 1.0 : 0.0, 0.0};
    }
    __syncthreads();
    for (int sweep = 0; sweep < EIG_SWEEPS; ++sweep) {
        double off = 0, dia = 0;
        for (int e = lane; e < n * n; e += 64) {
            const int r = e / n, c = e - r * n;
            const double2 a = A[r * LD + c];
            if (r != c)
                off += a.x * a.x + a.y * a.y;
            else
                dia += a.x * a.x;
        }
        off = wave_sum(off);
        dia = wave_sum(dia);
        const double fro2 = off + dia;
        // converged once the off-diagonal part is 1e-14 of the Frobenius norm
        if (off <= eig_stop2(n) * fmax(fro2, 1e-300) || off == 0.0) break;
        const double skip2 = 1e-32 * fro2;  // (1e-16 |A|_F)^2: pairs at rounding level are not rotated
        for (int round = 0; round < m - 1; ++round) {
            if (lane < P) {
                int p, q;
                jacobi_pair(round, lane, m, p, q);
                const double2 c = A[p * LD + q];
                const double app = A[p * LD + p].x, aqq = A[q * LD + q].x;
                const double ac2 = c.x * c.x + c.y * c.y;
                RotW R{1.0, 0.0, 1.0, 0.0};
                if (q < n && ac2 > skip2 && ac2 > 1e-300) {
                    const double ri = rsqrt(ac2);  // 1 / |a_pq|
                    const double tau = 0.5 * (aqq - app) * ri;
                    const double t = (tau >= 0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
                    R.cs = rsqrt(1.0 + t * t);
                    R.sn = t * R.cs;
                    R.er = c.x * ri;
                    R.ei = -c.y * ri;
                }
                rot[lane] = R;
            }
            __syncthreads();
            // A <- J^H A J on the 2 x 2 blocks (row pair s2 <= column pair s1)
#pragma unroll
            for (int u = 0; u < (PMAX * PMAX + 63) / 64; ++u) {
                const int bk = lane + 64 * u;
                const int s2 = bk / PMAX, s1 = bk - s2 * PMAX;
                if (s2 >= P || s1 >= P || s2 > s1) continue;
                int p2, q2, p1, q1;
                jacobi_pair(round, s2, m, p2, q2);
                jacobi_pair(round, s1, m, p1, q1);
                double2 B[2][2];
                B[0][0] = A[p2 * LD + p1];
                B[0][1] = A[p2 * LD + q1];
                B[1][0] = A[q2 * LD + p1];
                B[1][1] = A[q2 * LD + q1];
                const RotW Rc = rot[s1], Rr = rot[s2];
                // columns: new_p = cs b_p - sn e b_q ; new_q = sn b_p + cs e b_q
                const double2 e2 = double2{Rc.er, Rc.ei};
#pragma unroll
                for (int i = 0; i < 2; ++i) {
                    const double2 bp = B[i][0], ebq = cmulz(e2, B[i][1]);
                    B[i][0] = double2{Rc.cs * bp.x - Rc.sn * ebq.x, Rc.cs * bp.y - Rc.sn * ebq.y};
                    B[i][1] = double2{Rc.sn * bp.x + Rc.cs * ebq.x, Rc.sn * bp.y + Rc.cs * ebq.y};
                }
                // rows: new_p = cs b_p - sn conj(e) b_q ; new_q = sn b_p + cs conj(e) b_q
                const double2 ce = double2{Rr.er, -Rr.ei};
#pragma unroll
                for (int j = 0; j < 2; ++j) {
                    const double2 bp = B[0][j], ebq = cmulz(ce, B[1][j]);
                    B[0][j] = double2{Rr.cs * bp.x - Rr.sn * ebq.x, Rr.cs * bp.y - Rr.sn * ebq.y};
                    B[1][j] = double2{Rr.sn * bp.x + Rr.cs * ebq.x, Rr.sn * bp.y + Rr.cs * ebq.y};
                }
                if (s1 == s2) {
                    // a rotated pair becomes diagonal with a real diagonal
                    const bool rotd = Rc.sn != 0.0 || Rc.er != 1.0 || Rc.ei != 0.0;
                    A[p1 * LD + p1] = rotd ? double2{B[0][0].x, 0.0} : B[0][0];
                    A[q1 * LD + q1] = rotd ? double2{B[1][1].x, 0.0} : B[1][1];
                    A[p1 * LD + q1] = rotd ? double2{0.0, 0.0} : B[0][1];
                    A[q1 * LD + p1] = rotd ? double2{0.0, 0.0} : B[1][0];
                } else {
                    A[p2 * LD + p1] = B[0][0];
                    A[p1 * LD + p2] = double2{B[0][0].x, -B[0][0].y};
                    A[p2 * LD + q1] = B[0][1];
                    A[q1 * LD + p2] = double2{B[0][1].x, -B[0][1].y};
                    A[q2 * LD + p1] = B[1][0];
                    A[p1 * LD + q2] = double2{B[1][0].x, -B[1][0].y};
                    A[q2 * LD + q1] = B[1][1];
                    A[q1 * LD + q2] = double2{B[1][1].x, -B[1][1].y};
                }
            }
            // V <- V J: columns p, q of V are rows p, q of Vt
#pragma unroll
            for (int u = 0; u < (PMAX * NMAX + 63) / 64; ++u) {
                const int e = lane + 64 * u;
                const int sidx = e / NMAX, r = e - sidx * NMAX;
                if (sidx >= P || r >= n) continue;
                int p, q;
                jacobi_pair(round, sidx, m, p, q);
                const double2 vp = Vt[p * LD + r], vq = Vt[q * LD + r];
                const RotW R = rot[sidx];
                const double2 eq = cmulz(double2{R.er, R.ei}, vq);
                Vt[p * LD + r] = double2{R.cs * vp.x - R.sn * eq.x, R.cs * vp.y - R.sn * eq.y};
                Vt[q * LD + r] = double2{R.sn * vp.x + R.cs * eq.x, R.sn * vp.y + R.cs * eq.y};
            }
            __syncthreads();
        }
    }
    // ascending order by rank (ties by index), then emit
    for (int i = lane; i < n; i += 64) dg[i] = A[i * LD + i].x;
    __syncthreads();
    for (int i = lane; i < n; i += 64) {
        int r = 0;
        for (int j = 0; j < n; ++j) r += (dg[j] < dg[i]) || (dg[j] == dg[i] && j < i);
        perm[r] = i;
    }
    __syncthreads();
    for (int i = lane; i < n; i += 64) ev[i] = dg[perm[i]];
    for (int e = lane; e < n * n; e += 64) {
        const int r = e / n, c = e - r * n;
        vo[e] = Vt[perm[c] * LD + r];
    }
}

template <int NMAX>
__global__ void __launch_bounds__(64)
k_jacobi_eigh_wave(int n, const double2* __restrict__ H, double* __restrict__ eig, double2* __restrict__ vecs) {
    const int64_t b = blockIdx.x;
    jacobi_eigh_wave<NMAX>(n, H + b * n * n, eig + b * n, vecs + b * n * n);
}

template <int NMAX>
__global__ void __launch_bounds__(64)
k_jacobi_eigh_seg_wave(const Seg* __restrict__ seg, const double2* __restrict__ H, double* __restrict__ eig,
                       double2* __restrict__ vecs) {
    const Seg sg = seg[blockIdx.x];
    jacobi_eigh_wave<NMAX>(sg.nb, H + sg.moff, eig + sg.f_off, vecs + sg.moff);
}

bool eigh_wave_launch(hipStream_t st, unsigned nblk, int nmax, const Seg* seg, const double2* H, double* eig,
                      double2* vecs) {
    if (nmax <= 16)
        hipLaunchKernelGGL(k_jacobi_eigh_seg_wave<16>, dim3(nblk), dim3(64), 0, st, seg, H, eig, vecs);
    else if (nmax <= 32)
        hipLaunchKernelGGL(k_jacobi_eigh_seg_wave<32>, dim3(nblk), dim3(64), 0, st, seg, H, eig, vecs);
    else
        return false;
    return true;
}

}  // namespace dpp

using namespace dpp;

// ------------------------------------------------------------- C ABI -------

extern "C" dpp_status dpp_overlap(dpp_basis basis, int nbA, const dpp_c64* A, int64_t ldA, int nbB,
                                  const dpp_c64* B, int64_t ldB, double scale, dpp_c64* U, dpp_precision prec,
                                  void* ws) {
    clear_error();
    DPP_REQUIRE(basis && nbA >= 0 && nbB >= 0, "dpp_overlap: bad arguments");
    DPP_REQUIRE(prec == DPP_F64 || prec == DPP_F32, "dpp_overlap: bad precision");
    DPP_REQUIRE((nbA == 0 || A) && (nbB == 0 || B), "dpp_overlap: null block");
    DPP_REQUIRE(ldA >= basis->npw && ldB >= basis->npw, "dpp_overlap: leading dimension < npw");
    if (nbA == 0 || nbB == 0) return DPP_OK;
    DPP_REQUIRE(U && ws, "dpp_overlap: null output or workspace");
    return overlap_single(basis->grid->ctx, (int)basis->npw, nbA, (const double2*)A, ldA, nbB, (const double2*)B,
                          ldB, scale, (double2*)U, ws, overlap_ws_bytes((int)basis->npw, nbA, nbB), prec);
}

extern "C" dpp_status dpp_rotate(dpp_basis basis, int nbX, const dpp_c64* X, int64_t ldX, int nbO,
                                 const dpp_c64* M, double beta, dpp_c64* out, int64_t ldout, dpp_precision prec) {
    clear_error();
    DPP_REQUIRE(basis && nbX >= 0 && nbO >= 0, "dpp_rotate: bad arguments");
    DPP_REQUIRE(prec == DPP_F64 || prec == DPP_F32, "dpp_rotate: bad precision");
    DPP_REQUIRE(ldX >= basis->npw && ldout >= basis->npw, "dpp_rotate: leading dimension < npw");
    if (nbO == 0) return DPP_OK;
    DPP_REQUIRE(out && (nbX == 0 || (X && M)), "dpp_rotate: null pointer");
    DPP_REQUIRE((const void*)X != (const void*)out, "dpp_rotate: out must not alias X");
    return rotate_single(basis->grid->ctx, (int)basis->npw, nbX, (const double2*)X, ldX, nbO, (const double2*)M,
                         beta, (double2*)out, ldout, prec);
}

extern "C" dpp_status dpp_cholesky_inverse(dpp_ctx ctx, int nb, int batch, const dpp_c64* U, dpp_c64* Rinv) {
    clear_error();
    DPP_REQUIRE(ctx && nb >= 1 && batch >= 0 && U && Rinv, "dpp_cholesky_inverse: bad arguments");
    DPP_REQUIRE(nb <= CH_MAXN, "dpp_cholesky_inverse: nb > 128");
    if (batch == 0) return DPP_OK;
    TimerScope ts_(ctx, DPP_TK_CHOLESKY);
    if (!cholesky_wave_launch(ctx->stream, (unsigned)batch, nb, (int64_t)nb * nb, nullptr, 0, (const double2*)U,
                              (double2*)Rinv, ctx->d_status, nullptr))
        DPP_HIP(cholesky_tiles_launch(ctx->stream, (unsigned)batch, nb, nullptr, 0, nb, (const double2*)U,
                                      (double2*)Rinv, ctx->d_status, nullptr));
    DPP_LAUNCHED();
    return DPP_OK;
}

// ------------------------------------- eigensolver without allocation ------
// Workspace of dpp_subspace_eigh_noalloc: a file-scope device array (each GPU
// the library runs on holds its own copy until the process ends).  Host code
// never uses the array's name as an address: dpp_ctx_create records, with the
// context's device current, the address hipGetSymbolAddress returns, and the
// entry point passes that address to the kernels.
constexpr size_t EIGH_STATIC_BYTES = (size_t)8 << 20;
static __device__ __align__(256) char scratch[EIGH_STATIC_BYTES];

namespace {
constexpr int SCRATCH_MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[SCRATCH_MAX_DEVICES];
}  // namespace

dpp_status dpp::eigh_scratch_setup(int device) {
    DPP_REQUIRE(device >= 0 && device < SCRATCH_MAX_DEVICES, "eigh_scratch_setup: device index out of range");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch_ptr[device]) return DPP_OK;
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
        return set_error(DPP_EDEVICE, std::string("eigh_scratch_setup: hipGetSymbolAddress failed: ") +
                                          hipGetErrorString(e));
    g_scratch_ptr[device] = p;
    return DPP_OK;
}

static size_t eigh_ws_split(int nb, int batch) {
    return ((eigh_tiles_ws_bytes((int64_t)batch * nb * nb) + 255) / 256) * 256;
}

extern "C" dpp_status dpp_eigh_workspace_size(int nb, int batch, size_t* bytes) {
    clear_error();
    DPP_REQUIRE(bytes && nb >= 1 && batch >= 0, "dpp_eigh_workspace_size: bad arguments");
    *bytes = nb <= EIGW_MAXN ? 256 : eigh_ws_split(nb, batch) + eigh_perm_bytes(batch);
    return DPP_OK;
}

extern "C" dpp_status dpp_subspace_eigh(dpp_ctx ctx, int nb, int batch, const dpp_c64* H, double* eig,
                                        dpp_c64* vecs, void* ws) {
    clear_error();
    DPP_REQUIRE(ctx && nb >= 1 && batch >= 0, "dpp_subspace_eigh: bad arguments");
    DPP_REQUIRE(nb <= EIG_MAXN, "dpp_subspace_eigh: nb > 128");
    if (batch == 0) return DPP_OK;
    DPP_REQUIRE(H && eig && vecs, "dpp_subspace_eigh: null pointer");
    DPP_REQUIRE(nb <= EIGW_MAXN || ws, "dpp_subspace_eigh: workspace required for nb > 32");
    TimerScope ts_(ctx, DPP_TK_EIGH);
    if (nb <= 16)
        hipLaunchKernelGGL(k_jacobi_eigh_wave<16>, dim3(batch), dim3(64), 0, ctx->stream, nb, (const double2*)H, eig,
                           (double2*)vecs);
    else if (nb <= EIGW_MAXN)
        hipLaunchKernelGGL(k_jacobi_eigh_wave<32>, dim3(batch), dim3(64), 0, ctx->stream, nb, (const double2*)H, eig,
                           (double2*)vecs);
    else {
        char* w = reinterpret_cast<char*>(ws);
        DPP_HIP(eigh_tiles_launch(ctx->stream, (unsigned)batch, nb, nullptr, nb, (const double2*)H, eig,
                                  (double2*)vecs, reinterpret_cast<double2*>(w),
                                  reinterpret_cast<int*>(w + eigh_ws_split(nb, batch))));
    }
    DPP_LAUNCHED();
    return DPP_OK;
}


extern "C" dpp_status dpp_subspace_eigh_noalloc(dpp_ctx ctx, int nb, int batch, const dpp_c64* H, double* eig,
                                                dpp_c64* vecs) {
    clear_error();
    DPP_REQUIRE(ctx && nb >= 1 && batch >= 0, "dpp_subspace_eigh_noalloc: bad arguments");
    DPP_REQUIRE(nb <= EIG_MAXN, "dpp_subspace_eigh_noalloc: nb > 128");
    if (batch == 0) return DPP_OK;
    const size_t need = nb <= EIGW_MAXN ? 0 : eigh_ws_split(nb, batch) + eigh_perm_bytes(batch);
    if (need > EIGH_STATIC_BYTES)
        return set_error(DPP_EINVAL, "dpp_subspace_eigh_noalloc: " + std::to_string(batch) + " matrices of order " +
                                         std::to_string(nb) + " need " + std::to_string(need) +
                                         " bytes of workspace, more than the " + std::to_string(EIGH_STATIC_BYTES) +
                                         "-byte static array; use dpp_subspace_eigh with a workspace");
    void* ws = (ctx->device >= 0 && ctx->device < SCRATCH_MAX_DEVICES) ? g_scratch_ptr[ctx->device] : nullptr;
    DPP_REQUIRE(ws, "dpp_subspace_eigh_noalloc: static workspace not set up for this device");
    return dpp_subspace_eigh(ctx, nb, batch, H, eig, vecs, ws);
}

size_t dpp::proj_ws_bytes(const dpp_basis_s* b, int nb) {
    // Pi (64 projectors max per call chunk is not assumed: use the actual count later)
    return overlap_ws_bytes((int)b->npw, 128, nb) + (size_t)128 * nb * sizeof(double2) + 512;
}

extern "C" dpp_status dpp_apply_H(dpp_ham ham, int nb, const dpp_c64* C, int64_t ldC, dpp_c64* HC,
                                  int64_t ldHC, dpp_precision prec, void* ws) {
    clear_error();
    DPP_REQUIRE(ham, "dpp_apply_H: null ham");
    dpp_basis b = ham->basis;
    DPP_REQUIRE(nb >= 0 && ldC >= b->npw && ldHC >= b->npw, "dpp_apply_H: bad sizes");
    if (nb == 0) return DPP_OK;
    DPP_REQUIRE(C && HC && ws, "dpp_apply_H: null pointer");
    DPP_REQUIRE((const void*)C != (const void*)HC, "dpp_apply_H: C and HC must not alias");
    DPP_REQUIRE(ham->d_Veff, "dpp_apply_H: no potential set");
    DPP_REQUIRE(prec == DPP_F64 || prec == DPP_F32, "dpp_apply_H: bad precision");
    DPP_REQUIRE(ham->nproj <= 128, "dpp_apply_H: more than 128 projectors");
    if (prec == DPP_F64)
        DPP_TRY(run_apply_H_local<double>(ham, nb, (const double2*)C, ldC, (double2*)HC, ldHC, ws));
    else
        DPP_TRY(run_apply_H_local<float>(ham, nb, (const double2*)C, ldC, (double2*)HC, ldHC, ws));
    if (ham->nproj > 0) {
        const size_t el = prec == DPP_F64 ? 16 : 8;
        const size_t t = ((plane_buffer_elems(b, nb) * el + 255) / 256) * 256;
        char* base = reinterpret_cast<char*>(ws) + t;
        double2* Pi = reinterpret_cast<double2*>(base);
        char* ovws = base + (((size_t)ham->nproj * nb * sizeof(double2) + 255) / 256) * 256;
        // Pi' = D P^dag C, then HC += P Pi'
        DPP_TRY(overlap_single(b->grid->ctx, (int)b->npw, ham->nproj, ham->d_P, b->npw, nb, (const double2*)C,
                               ldC, ham->D, Pi, ovws, overlap_ws_bytes((int)b->npw, ham->nproj, nb), prec));
        DPP_TRY(rotate_single(b->grid->ctx, (int)b->npw, ham->nproj, ham->d_P, b->npw, nb, Pi, 1.0, (double2*)HC,
                              ldHC, prec));
    }
    return DPP_OK;
}

static size_t ortho_ws(const dpp_basis_s* b, int nb) {
    auto r = [](size_t x) { return ((x + 255) / 256) * 256; };
    return 2 * r((size_t)nb * nb * 16) + r((size_t)nb * b->npw * 16) + r(overlap_ws_bytes((int)b->npw, nb, nb)) + 256;
}

extern "C" dpp_status dpp_ortho_workspace_size(dpp_basis basis, int nb, size_t* bytes) {
    clear_error();
    DPP_REQUIRE(basis && nb >= 1 && bytes, "dpp_ortho_workspace_size: bad arguments");
    *bytes = ortho_ws(basis, nb);
    return DPP_OK;
}

extern "C" dpp_status dpp_cholesky_orthonormalize(dpp_basis basis, int nb, dpp_c64* Y, int64_t ldY,
                                                  dpp_c64* Rinv, void* ws) {
    clear_error();
    DPP_REQUIRE(basis && nb >= 1 && Y && ws && ldY >= basis->npw, "dpp_cholesky_orthonormalize: bad arguments");
    // ws layout: U (nb^2), Rinv (nb^2) if not given, copy of Y (nb x npw), overlap partials
    char* p = reinterpret_cast<char*>(ws);
    auto take = [&](size_t bytes) {
        char* r = p;
        p += ((bytes + 255) / 256) * 256;
        return r;
    };
    double2* U = reinterpret_cast<double2*>(take((size_t)nb * nb * 16));
    double2* Ri = Rinv ? (double2*)Rinv : reinterpret_cast<double2*>(take((size_t)nb * nb * 16));
    double2* Yc = reinterpret_cast<double2*>(take((size_t)nb * basis->npw * 16));
    void* ovws = take(overlap_ws_bytes((int)basis->npw, nb, nb));
    dpp_ctx ctx = basis->grid->ctx;
    DPP_TRY(overlap_single(ctx, (int)basis->npw, nb, (const double2*)Y, ldY, nb, (const double2*)Y, ldY,
                        basis->grid->omega, U, ovws, overlap_ws_bytes((int)basis->npw, nb, nb)));
    DPP_TRY(dpp_cholesky_inverse(ctx, nb, 1, (const dpp_c64*)U, (dpp_c64*)Ri));
    DPP_HIP(hipMemcpy2DAsync(Yc, basis->npw * 16, Y, ldY * 16, basis->npw * 16, nb, hipMemcpyDeviceToDevice,
                             ctx->stream));
    DPP_TRY(rotate_single(ctx, (int)basis->npw, nb, Yc, basis->npw, nb, Ri, 0.0, (double2*)Y, ldY));
    return DPP_OK;
}
