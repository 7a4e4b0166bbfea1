// Learned initial density: a periodic 3D convolutional network trained and
// evaluated by the library's own kernels.
//
//   x = n0 / nbar;  h1 = silu(conv1(x)); h2 = silu(conv2(h1)); h3 = silu(conv3(h2));
//   y = conv4(h3);  dn = nbar (y - mean y);  n = max(n0 + dn, 0) rescaled to N_e
// conv: 3x3x3 cross-correlation with circular padding, channels 1-16-16-16-1.
// Weights are stored in BF16 (round to nearest even from FP32 master copies
// kept for Adam); activations, accumulation and gradients are FP32; the loss
// and density reductions are FP64.
//
// Kernels: forward (one thread per voxel computes every output channel, the
// layer's weights staged in LDS), backward-data (transposed correlation),
// backward-weights (split-BF16 MFMA implicit GEMM over voxels, workgroup
// partials reduced in fixed order), SiLU backward, loss, Adam.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <vector>

#include "internal.h"

namespace dpp {

constexpr int NL = 4;
constexpr int CH[NL + 1] = {1, 16, 16, 16, 1};

__device__ __forceinline__ float bf16_to_f32(uint16_t h) {
    return __uint_as_float(((uint32_t)h) << 16);
}

// FP32 -> BF16 with round to nearest, ties to even (NaN kept quiet).
__host__ __device__ inline uint16_t f32_to_bf16(float f) {
    uint32_t u;
    std::memcpy(&u, &f, 4);
    if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x007fffffu)) return (uint16_t)((u >> 16) | 0x40);
    const uint32_t lsb = (u >> 16) & 1u;
    u += 0x7fffu + lsb;
    return (uint16_t)(u >> 16);
}

__device__ __forceinline__ float sigm(float a) { return 1.0f / (1.0f + expf(-a)); }

struct Box {
    int S0, S1, S2;
};

__device__ __forceinline__ int64_t shifted(const Box& b, int r0, int r1, int r2, int d0, int d1, int d2) {
    int a = r0 + d0, c = r1 + d1, e = r2 + d2;
    a += a < 0 ? b.S0 : 0;
    a -= a >= b.S0 ? b.S0 : 0;
    c += c < 0 ? b.S1 : 0;
    c -= c >= b.S1 ? b.S1 : 0;
    e += e < 0 ? b.S2 : 0;
    e -= e >= b.S2 ? b.S2 : 0;
    return ((int64_t)a * b.S1 + c) * b.S2 + e;
}

// pre[b][co][r] = bias[co] + sum_ci sum_d W[co][ci][d] x[b][ci][r + d]; act = silu(pre) if ACT.
template <int CI, int CO, bool ACT>
__global__ void __launch_bounds__(256)
k_conv_fwd(Box bx, int64_t N, const float* __restrict__ x, const uint16_t* __restrict__ W,
           const float* __restrict__ bias, float* __restrict__ pre, float* __restrict__ act) {
    __shared__ float w[CO * CI * 27];
    for (int i = threadIdx.x; i < CO * CI * 27; i += blockDim.x) w[i] = bf16_to_f32(W[i]);
    __syncthreads();
    const int b = blockIdx.y;
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= N) return;
    const int r2 = (int)(r % bx.S2);
    const int64_t q = r / bx.S2;
    const int r1 = (int)(q % bx.S1), r0 = (int)(q / bx.S1);
    float acc[CO];
#pragma unroll
    for (int co = 0; co < CO; ++co) acc[co] = bias[co];
    const float* xb = x + (int64_t)b * CI * N;
    for (int d = 0; d < 27; ++d) {
        const int64_t s = shifted(bx, r0, r1, r2, d / 9 - 1, (d / 3) % 3 - 1, d % 3 - 1);
#pragma unroll
        for (int ci = 0; ci < CI; ++ci) {
            const float xv = xb[(int64_t)ci * N + s];
#pragma unroll
            for (int co = 0; co < CO; ++co) acc[co] += w[(co * CI + ci) * 27 + d] * xv;
        }
    }
#pragma unroll
    for (int co = 0; co < CO; ++co) {
        const int64_t o = ((int64_t)b * CO + co) * N + r;
        pre[o] = acc[co];
        if (ACT) act[o] = acc[co] * sigm(acc[co]);
    }
}

// silu'(a) = s (1 + a (1 - s)), s = sigmoid(a)
__device__ __forceinline__ float dsilu(float a) {
    const float sg = sigm(a);
    return sg * (1.0f + a * (1.0f - sg));
}

// dx[b][ci][s] = silu'(apre[b][ci][s]) sum_co sum_d W[co][ci][d] g[b][co][s - d]
// (the gradient with respect to the pre-activation of the layer below)
template <int CI, int CO>
__global__ void __launch_bounds__(256)
k_conv_bwd_data(Box bx, int64_t N, const float* __restrict__ g, const uint16_t* __restrict__ W,
                const float* __restrict__ apre, float* __restrict__ dx) {
    __shared__ float w[CO * CI * 27];
    for (int i = threadIdx.x; i < CO * CI * 27; i += blockDim.x) w[i] = bf16_to_f32(W[i]);
    __syncthreads();
    const int b = blockIdx.y;
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= N) return;
    const int s2 = (int)(s % bx.S2);
    const int64_t q = s / bx.S2;
    const int s1 = (int)(q % bx.S1), s0 = (int)(q / bx.S1);
    float acc[CI];
#pragma unroll
    for (int ci = 0; ci < CI; ++ci) acc[ci] = 0.0f;
    const float* gb = g + (int64_t)b * CO * N;
    for (int d = 0; d < 27; ++d) {
        const int64_t r = shifted(bx, s0, s1, s2, -(d / 9 - 1), -((d / 3) % 3 - 1), -(d % 3 - 1));
#pragma unroll
        for (int co = 0; co < CO; ++co) {
            const float gv = gb[(int64_t)co * N + r];
#pragma unroll
            for (int ci = 0; ci < CI; ++ci) acc[ci] += w[(co * CI + ci) * 27 + d] * gv;
        }
    }
#pragma unroll
    for (int ci = 0; ci < CI; ++ci) {
        const int64_t o = ((int64_t)b * CI + ci) * N + s;
        dx[o] = acc[ci] * dsilu(apre[o]);
    }
}

typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef float f4 __attribute__((ext_vector_type(4)));

// FP32 -> BF16 hi + BF16 lo (x = hi + lo to about 2^-16 relative)
__device__ __forceinline__ void bsplit(float f, __bf16& hi, __bf16& lo) {
    hi = (__bf16)f;
    lo = (__bf16)(f - (float)hi);
}

// buffer resources over one sample's channels (raw, 32-bit byte offsets)
constexpr int WGM_RSRC_WORD3 = 0x00020000;
constexpr unsigned WGM_OUT_OF_RANGE = 0x80000000u;  // buffer loads there return 0

// v in [-n, 2n) -> v mod n
__device__ __forceinline__ int wrap(int v, int n) {
    v += v < 0 ? n : 0;
    return v - (v >= n ? n : 0);
}

// ------------------------------------- 16 -> 16 layers on MFMA (forward,
// backward-data) --------------------------------------------------------------
// out[m][r] = bias[m] + sum_{k, d} A[m][k][d] src[k][r + s d], an implicit GEMM
// on BF16 MFMA (16x16x32, FP32 accumulation): M = 16 output channels, N = 16
// voxels along z, K = 27 taps x 16 input channels = 432 (14 K steps of 32, the
// last half empty).  Forward: A = W[m][k][d], s = +1 (cross-correlation).
// Backward-data: A = W[k][m][d], s = -1 (dx[ci][s] = sum W[co][ci][d] g[co][s - d]).
// The BF16 weights are the A operand exactly; src (FP32) is split into BF16
// hi + lo, two products per K step.  Workgroup = (sample, plane r0, block of
// RT z-rows): the 3 x (RT + 2) src rows around the block are staged once, one
// barrier, channel-last in LDS (row, channel half, position -1..S2 with the
// periodic halo, 8 channels = one 16-byte operand per lane); each wave then
// runs up to three 16-voxel tiles with independent accumulators.
constexpr int C16_THREADS = 256;
constexpr int C16_TPW = 3;      // tiles per wave
constexpr int C16_KSTEPS = 14;  // K steps of 32 over 27 taps x 16 channels
constexpr int C16_SPT = 3;      // staging tasks per thread per batch of loads

__host__ __device__ inline int c16_tiles(int S2) { return (S2 + 15) / 16; }
// z-rows per workgroup: 4 waves x 3 tiles, at most S1
__host__ __device__ inline int c16_rows(int S1, int S2) {
    const int r = 12 / c16_tiles(S2) < 1 ? 1 : 12 / c16_tiles(S2);
    return r < S1 ? r : S1;
}
// staged positions per row: the tiles plus one halo voxel each side
__host__ __device__ inline int c16_pos(int S2) { return 16 * c16_tiles(S2) + 2; }
inline size_t c16_lds_bytes(int S1, int S2) { return (size_t)3 * (c16_rows(S1, S2) + 2) * 2 * c16_pos(S2) * 8 * 2 * 2; }

// floor(a / b) for 0 <= a < 2^16 and 1 <= b < 2^10 from a float reciprocal:
// (a + 1/2) / b is at least 1/(2b) away from an integer, far above the rounding error
__device__ __forceinline__ int c16_div(int a, float inv_b) { return (int)(((float)a + 0.5f) * inv_b); }

// A operands in MFMA lane order, apack[kk * 64 + lane]: lane (m = lane & 15,
// ks = lane >> 4) holds A[m][8 ks + e] of K step kk, i.e. tap 2 kk + (ks >> 1)
// and channel 8 (ks & 1) + e; zero past tap 26.
template <bool TRANS>
__global__ void __launch_bounds__(C16_KSTEPS * 64) k_pack_a16(const uint16_t* __restrict__ W, bf8* __restrict__ apack) {
    const int i = threadIdx.x, kk = i / 64, lane = i % 64;
    const int m = lane & 15, ks = lane >> 4, tap = 2 * kk + (ks >> 1);
    bf8 v;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        const int ch = 8 * (ks & 1) + e;
        const int idx = (TRANS ? ch * 16 + m : m * 16 + ch) * 27 + (tap < 27 ? tap : 0);
        v[e] = __builtin_bit_cast(__bf16, tap < 27 ? W[idx] : (uint16_t)0);
    }
    apack[i] = v;
}

// Forward: out = pre-activation (+ bias), act = silu(out) if ACT.  Backward-
// data: out = the product times silu'(aux), aux the pre-activation of the
// layer below (the gradient with respect to it).
template <bool TRANS, bool ACT>
__global__ void __launch_bounds__(C16_THREADS)
k_conv16_mfma(Box bx, int64_t N, int nblk, const float* __restrict__ src, const bf8* __restrict__ apack,
              const float* __restrict__ aux, float* __restrict__ out, float* __restrict__ act) {
    extern __shared__ __attribute__((aligned(16))) char c16_smem[];
    const int nt = c16_tiles(bx.S2), RT = c16_rows(bx.S1, bx.S2), P = c16_pos(bx.S2);
    const int nrow = 3 * (RT + 2);
    __bf16* sh = reinterpret_cast<__bf16*>(c16_smem);
    __bf16* sl = sh + nrow * 2 * P * 8;
    // XCD-aware order (workgroups dealt round robin to 8 XCDs): each XCD takes a
    // contiguous run of (sample, plane, row block), row block fastest
    const int total = gridDim.x, L = blockIdx.x, xcd = L % 8, q8 = total / 8, rem = total % 8;
    const int id = xcd * q8 + min(xcd, rem) + L / 8;
    const int blk = id % nblk, r0 = (id / nblk) % bx.S0, b = id / (nblk * bx.S0);
    const int r1a = blk * RT;
    const int lane = threadIdx.x & 63, w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int c = lane & 15, ks = lane >> 4;
    bf8 a[C16_KSTEPS];
#pragma unroll
    for (int kk = 0; kk < C16_KSTEPS; ++kk) a[kk] = apack[kk * 64 + lane];
    // stage src rows (r0 + dl0, r1a - 1 + jj), dl0 = -1..1, jj = 0..RT+1: row
    // q = (dl0 + 1) (RT + 2) + jj, position p = z + 1 (periodic halo)
    const auto sr = __builtin_amdgcn_make_buffer_rsrc(const_cast<float*>(src + (int64_t)b * 16 * N), (short)0,
                                                      (int)(16 * N * 4), WGM_RSRC_WORD3);
    const int np = bx.S2 + 2, ntask = nrow * np;
    const float inv_np = 1.0f / (float)np, inv_rt = 1.0f / (float)(RT + 2);
    for (int t0 = 0; t0 < ntask; t0 += C16_THREADS * C16_SPT) {
        float v[C16_SPT][16];
#pragma unroll
        for (int k = 0; k < C16_SPT; ++k) {
            int t = t0 + threadIdx.x + C16_THREADS * k;
            t = t < ntask ? t : 0;
            const int q = c16_div(t, inv_np), pz = t - q * np;
            const int dq = c16_div(q, inv_rt);  // dl0 + 1
            const int a0 = wrap(r0 + dq - 1, bx.S0);
            const int a1 = wrap(r1a - 1 + q - dq * (RT + 2), bx.S1);  // within [-1, 2 S1) as RT <= S1
            const int z = wrap(pz - 1, bx.S2);
            const unsigned vo = (unsigned)(((a0 * bx.S1 + a1) * bx.S2 + z) * 4);
#pragma unroll
            for (int ch = 0; ch < 16; ++ch)  // the channel offset is scalar
                v[k][ch] = __builtin_bit_cast(float,
                                              __builtin_amdgcn_raw_buffer_load_b32(sr, vo, (int)(ch * N * 4), 0));
        }
#pragma unroll
        for (int k = 0; k < C16_SPT; ++k) {
            const int t = t0 + threadIdx.x + C16_THREADS * k;
            if (t < ntask) {
                const int q = c16_div(t, inv_np), pz = t - q * np;
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    bf8 hi, lo;
#pragma unroll
                    for (int e = 0; e < 8; ++e) {
                        __bf16 x0, x1;
                        bsplit(v[k][8 * h + e], x0, x1);
                        hi[e] = x0;
                        lo[e] = x1;
                    }
                    const int o = ((q * 2 + h) * P + pz) * 8;
                    *reinterpret_cast<bf8*>(sh + o) = hi;
                    *reinterpret_cast<bf8*>(sl + o) = lo;
                }
            }
        }
    }
    __syncthreads();
    // per K step: lane (voxel c, ks) reads 8 channels of tap 2 kk + (ks >> 1)
    constexpr int sg = TRANS ? -1 : 1;
    int off[C16_KSTEPS];
#pragma unroll
    for (int kk = 0; kk < C16_KSTEPS; ++kk) {
        int tap = 2 * kk + (ks >> 1);
        tap = tap < 27 ? tap : 26;  // A is zero there
        const int d0 = tap / 9 - 1, d1 = (tap / 3) % 3 - 1, d2 = tap % 3 - 1;
        const int q = (sg * d0 + 1) * (RT + 2) + sg * d1 + 1;
        off[kk] = ((q * 2 + (ks & 1)) * P + c + sg * d2 + 1) * 8;
    }
    int toff[C16_TPW];
    bool tvalid[C16_TPW];
#pragma unroll
    for (int i = 0; i < C16_TPW; ++i) {
        const int T = w + 4 * i;
        tvalid[i] = T < RT * nt;
        const int j = tvalid[i] ? T / nt : 0, tz = tvalid[i] ? T % nt : 0;
        toff[i] = (j * 2 * P + 16 * tz) * 8;
    }
    f4 ah[C16_TPW], al[C16_TPW];
#pragma unroll
    for (int i = 0; i < C16_TPW; ++i) ah[i] = al[i] = f4{0, 0, 0, 0};
    // every slot runs (a slot without a tile reads tile 0 and is not stored),
    // so the MFMA sequence has no branches
#pragma unroll
    for (int kk = 0; kk < C16_KSTEPS; ++kk) {
#pragma unroll
        for (int i = 0; i < C16_TPW; ++i) {
            const bf8 bh = *reinterpret_cast<const bf8*>(sh + off[kk] + toff[i]);
            const bf8 bl = *reinterpret_cast<const bf8*>(sl + off[kk] + toff[i]);
            ah[i] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[kk], bh, ah[i], 0, 0, 0);
            al[i] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[kk], bl, al[i], 0, 0, 0);
        }
    }
    // D[4 (l / 16) + v][l % 16] = (output channel m, voxel c of the tile)
#pragma unroll
    for (int i = 0; i < C16_TPW; ++i) {
        const int T = w + 4 * i;
        if (!tvalid[i]) continue;
        const int r1 = r1a + T / nt, z = 16 * (T % nt) + c;
        if (r1 >= bx.S1 || z >= bx.S2) continue;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int m = 4 * ks + v;
            float val = ah[i][v] + al[i][v];
            const int64_t o = ((int64_t)b * 16 + m) * N + ((int64_t)r0 * bx.S1 + r1) * bx.S2 + z;
            if (TRANS)
                val *= dsilu(aux[o]);
            else
                val += aux[m];  // bias
            out[o] = val;
            if (ACT) act[o] = val * sigm(val);
        }
    }
}

// ------------------------------------------- weight gradient on MFMA ------
// The weight gradient as an implicit GEMM on split-BF16 MFMA (16x16x32,
// FP32 accumulation): for each tap d = (d0, d1, d2),
//   dW_d[co][ci] = sum_r g[co][r] x[ci][r + d] = sum_s g[co][s - d] x[ci][s],
// K running over the voxels s of x rows.  Inputs are FP32 values split into
// BF16 hi + lo (hi hi + hi lo + lo hi products).
// Workgroup = (g plane r0, sample b, part of the z-rows r1), three waves; wave
// w takes the nine taps with d0 = w - 1.  For the g row (r0, r1) the x rows
// (r0 + d0, r1 + d1) are needed: they live in LDS as BF16 hi/lo in a ring of 4
// row slots (slot R mod 4 holds x rows (r0 + d0, R) for d0 = -1, 0, 1 and
// every input channel), so each z-row stages one new row triple.  The g row is
// staged in 2 slots as three copies shifted by d2 (copy i at position p holds
// g[s - d2], s = zs + p, d2 = i - 1), so the B operand of x row (d0, d1) serves
// the three taps d2 = -1, 0, 1 and every operand read is an aligned 16-byte
// LDS load.  Next rows are prefetched into registers during the current one
// (branch-free buffer loads); one barrier per row.  K steps take 32
// consecutive positions (8 per lane group); g copies are zero past the row
// and past the segment (rows longer than 64 voxels run as 64-voxel segments).
// Channels past CI or CO are zero.  FP32 partials per workgroup: weights
// (co, ci, d) then biases, summed in FP64 in fixed order by
// k_sum_weight_partials.
constexpr int WGM_THREADS = 192;  // three waves
constexpr int WGM_SPLIT = 2;      // workgroups per g plane and sample (parts of the z-rows)
constexpr int WGM_XPF = 2;        // x staging tasks per thread (3 rows * 16 channels * 8 groups / 192)

// x row segment staged at once: the row rounded up to 8 voxels, at most 64
__host__ __device__ inline int wgm_row(int S2) { return S2 > 64 ? 64 : (S2 + 7) / 8 * 8; }
// g row length: whole K steps of 32
__host__ __device__ inline int wgm_arow(int S2) { return (wgm_row(S2) + 31) / 32 * 32; }
// LDS row strides: an odd number of 16-byte units, so the 16 channel rows
// that one 16-byte read spans fall in distinct banks
__host__ __device__ inline int wgm_pad(int len) { return (len / 8) % 2 ? len : len + 8; }
// LDS elements (hi or lo) of the x ring (4 slots x 3 rows x 16 channels, plus
// room for the last K step's reads past the final row, where g is zero) and
// of the g slots (2 slots x 3 shifts x 16 channels)
__host__ __device__ inline int wgm_x_elems(int S2) { return 4 * 3 * 16 * wgm_pad(wgm_row(S2)) + 32; }
__host__ __device__ inline int wgm_g_elems(int S2) { return 2 * 3 * 16 * wgm_pad(wgm_arow(S2)); }
inline size_t wgm_lds_bytes(int S2) { return 2 * (size_t)(wgm_x_elems(S2) + wgm_g_elems(S2)) * 2; }

__device__ __forceinline__ float wgm_load(__amdgpu_buffer_rsrc_t r, unsigned off) {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0));
}

template <int CI, int CO>
struct WgmPipe {
    float xv[WGM_XPF][8];  // x rows (r0 + d0, R): task t = (d0 + 1, ci, 8-voxel group)
    float gv[10];          // g row window: task t = (co, group), gv[j] = g[zs + 8 group - 1 + j]
                           // (row-periodic for every counted position; the others may read
                           // another row, or 0 past the array, and are masked)

    __device__ __forceinline__ void load_x(const Box& bx, int64_t N, __amdgpu_buffer_rsrc_t xr, int r0, int R, int zs,
                                           int ngroups) {
        const int cc = wrap(R, bx.S1);
#pragma unroll
        for (int k = 0; k < WGM_XPF; ++k) {
            int t = threadIdx.x + WGM_THREADS * k;
            t = t < 3 * CI * ngroups ? t : 0;
            const int gq = t % ngroups, q = t / ngroups;
            const int ci = q % CI, d0i = q / CI;
            const int a = wrap(r0 + d0i - 1, bx.S0);
            const int base = ci * (int)N + (a * bx.S1 + cc) * bx.S2;
            if (bx.S2 % 4 == 0) {  // 16-byte aligned halves, each wholly inside or past the row
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    const int z = zs + 8 * gq + 4 * h;
                    const f4 q = __builtin_bit_cast(
                        f4, __builtin_amdgcn_raw_buffer_load_b128(
                                xr, z < bx.S2 ? (unsigned)(base + z) * 4u : WGM_OUT_OF_RANGE, 0, 0));
#pragma unroll
                    for (int e = 0; e < 4; ++e) xv[k][4 * h + e] = q[e];
                }
            } else {
#pragma unroll
                for (int e = 0; e < 8; ++e) {
                    const int z = zs + 8 * gq + e;
                    xv[k][e] = wgm_load(xr, z < bx.S2 ? (unsigned)(base + z) * 4u : WGM_OUT_OF_RANGE);
                }
            }
        }
    }
    __device__ __forceinline__ void store_x(__bf16* xh, __bf16* xl, int xst, int slot, int ngroups) const {
#pragma unroll
        for (int k = 0; k < WGM_XPF; ++k) {
            const int t = threadIdx.x + WGM_THREADS * k;
            if (t < 3 * CI * ngroups) {
                const int gq = t % ngroups, q = t / ngroups;
                const int ci = q % CI, d0i = q / CI;
                bf8 hi, lo;
#pragma unroll
                for (int e = 0; e < 8; ++e) {
                    __bf16 h, l;
                    bsplit(xv[k][e], h, l);
                    hi[e] = h;
                    lo[e] = l;
                }
                const int o = ((slot * 3 + d0i) * 16 + ci) * xst + 8 * gq;
                *reinterpret_cast<bf8*>(xh + o) = hi;
                *reinterpret_cast<bf8*>(xl + o) = lo;
            }
        }
    }
    __device__ __forceinline__ void load_g(const Box& bx, int64_t N, __amdgpu_buffer_rsrc_t gr, int r0, int r1, int zs,
                                           int nga) {
        int t = threadIdx.x;
        t = t < CO * nga ? t : 0;
        const int gq = t % nga, co = t / nga;
        const int base = co * (int)N + (r0 * bx.S1 + r1) * bx.S2;
#pragma unroll
        for (int j = 0; j < 10; ++j) gv[j] = wgm_load(gr, (unsigned)(base + wrap(zs + 8 * gq - 1 + j, bx.S2)) * 4u);
    }
    // copy i (d2 = i - 1) at position p = 8 group + e: g[zs + p - d2] = gv[e + 2 - i],
    // zero unless p < zl and zs + p < S2; bsum gathers the unshifted counted values
    __device__ __forceinline__ void store_g(__bf16* gh, __bf16* gl, int zl, int gst, int slot, int zs, int S2,
                                            int nga, float& bsum) const {
        const int t = threadIdx.x;
        if (t < CO * nga) {
            const int gq = t % nga, co = t / nga;
            bf8 hi[3], lo[3];
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const int p = 8 * gq + e;
                const bool ok = p < zl && zs + p < S2;
                bsum += ok ? gv[e + 1] : 0.0f;
#pragma unroll
                for (int i = 0; i < 3; ++i) {
                    __bf16 h, l;
                    bsplit(ok ? gv[e + 2 - i] : 0.0f, h, l);
                    hi[i][e] = h;
                    lo[i][e] = l;
                }
            }
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                const int o = ((slot * 3 + i) * 16 + co) * gst + 8 * gq;
                *reinterpret_cast<bf8*>(gh + o) = hi[i];
                *reinterpret_cast<bf8*>(gl + o) = lo[i];
            }
        }
    }
};

// One wave's share: the nine taps with d0 = W - 1 (compile-time, so every
// operand offset is static); every wave passes the same barriers.
template <int CI, int CO, int W>
__device__ __forceinline__ void wgm_body(const Box& bx, int64_t N, const float* __restrict__ g,
                                         const float* __restrict__ x, float* __restrict__ part, __bf16* xh,
                                         __bf16* xl, __bf16* gh, __bf16* gl, int r0, int b, int part_i) {
    const int zl = wgm_row(bx.S2), zla = wgm_arow(bx.S2);
    const int xst = wgm_pad(zl), gst = wgm_pad(zla);  // LDS row strides
    const int lane = threadIdx.x & 63;
    const int c = lane & 15, ks = lane >> 4;
    f4 acc[9];
#pragma unroll
    for (int t = 0; t < 9; ++t) acc[t] = f4{0, 0, 0, 0};
    float bsum = 0.0f;
    const auto gr = __builtin_amdgcn_make_buffer_rsrc(const_cast<float*>(g + (int64_t)b * CO * N), (short)0,
                                                      (int)(CO * N * 4), WGM_RSRC_WORD3);
    const auto xr = __builtin_amdgcn_make_buffer_rsrc(const_cast<float*>(x + (int64_t)b * CI * N), (short)0,
                                                      (int)(CI * N * 4), WGM_RSRC_WORD3);
    const int rows = (bx.S1 + WGM_SPLIT - 1) / WGM_SPLIT;
    const int r1a = part_i * rows, r1e = min(bx.S1, r1a + rows);
    const int ngroups = zl / 8, nga = zla / 8, nks = zla / 32;
    const int nseg = (bx.S2 + zl - 1) / zl;
    // two register sets: at row r1 one holds x row r1 + 1 and g row r1 (stored
    // now), the other x row r1 + 2 and g row r1 + 1 (in flight since the
    // previous row); loads run two rows ahead of their use
    WgmPipe<CI, CO> pa, pb;
    for (int seg = 0; seg < nseg && r1a < r1e; ++seg) {
        const int zs = seg * zl;
        auto row = [&](int r1, WgmPipe<CI, CO>& cur) {
            // x slot (r1 + 1) mod 4 and g slot r1 mod 2 were last read for row
            // r1 - 2, before the previous barrier
            cur.store_x(xh, xl, xst, (r1 + 1) & 3, ngroups);
            cur.store_g(gh, gl, zl, gst, r1 & 1, zs, bx.S2, nga, bsum);
            if (r1 + 2 < r1e) {
                cur.load_x(bx, N, xr, r0, r1 + 3, zs, ngroups);
                cur.load_g(bx, N, gr, r0, r1 + 2, zs, nga);
            }
            __syncthreads();
            const int go = ((r1 & 1) * 3 * 16 + c) * gst;  // g slot, copy 0, channel c
            int xo[3];                                      // x slots of rows r1 + d1, d0 = W - 1, channel c
#pragma unroll
            for (int i = 0; i < 3; ++i) xo[i] = ((((r1 + i + 3) & 3) * 3 + W) * 16 + c) * xst;
#pragma unroll
            for (int kk = 0; kk < 2; ++kk) {
                if (kk >= nks) break;
                const int z0 = 8 * (4 * kk + ks);
                bf8 ah[3], al[3];
#pragma unroll
                for (int i = 0; i < 3; ++i) {
                    ah[i] = *reinterpret_cast<const bf8*>(gh + go + i * 16 * gst + z0);
                    al[i] = *reinterpret_cast<const bf8*>(gl + go + i * 16 * gst + z0);
                }
#pragma unroll
                for (int d1i = 0; d1i < 3; ++d1i) {
                    const bf8 bh = *reinterpret_cast<const bf8*>(xh + xo[d1i] + z0);
                    const bf8 bl = *reinterpret_cast<const bf8*>(xl + xo[d1i] + z0);
#pragma unroll
                    for (int i = 0; i < 3; ++i)
                        acc[3 * d1i + i] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[i], bh, acc[3 * d1i + i], 0, 0, 0);
#pragma unroll
                    for (int i = 0; i < 3; ++i)
                        acc[3 * d1i + i] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[i], bl, acc[3 * d1i + i], 0, 0, 0);
#pragma unroll
                    for (int i = 0; i < 3; ++i)
                        acc[3 * d1i + i] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[i], bh, acc[3 * d1i + i], 0, 0, 0);
                }
            }
        };
        // prologue: x rows r1a - 1 and r1a into their slots; x rows r1a + 1,
        // r1a + 2 and g rows r1a, r1a + 1 in registers
        pa.load_x(bx, N, xr, r0, r1a - 1, zs, ngroups);
        pa.store_x(xh, xl, xst, (r1a + 3) & 3, ngroups);
        pa.load_x(bx, N, xr, r0, r1a, zs, ngroups);
        pa.store_x(xh, xl, xst, r1a & 3, ngroups);
        pa.load_x(bx, N, xr, r0, r1a + 1, zs, ngroups);
        pa.load_g(bx, N, gr, r0, r1a, zs, nga);
        if (r1a + 1 < r1e) {
            pb.load_x(bx, N, xr, r0, r1a + 2, zs, ngroups);
            pb.load_g(bx, N, gr, r0, r1a + 1, zs, nga);
        }
        for (int r1 = r1a; r1 < r1e; r1 += 2) {
            row(r1, pa);
            if (r1 + 1 < r1e) row(r1 + 1, pb);
        }
        __syncthreads();  // the segment's reads are done before the next prologue
    }
    const int nw = CO * CI * 27 + CO;
    float* dst = part + ((int64_t)(b * bx.S0 + r0) * WGM_SPLIT + part_i) * nw;
    // result element v of lane l: D[4 (l / 16) + v][l % 16] = (co, ci); tap 9 W + 3 d1i + i
#pragma unroll
    for (int t = 0; t < 9; ++t) {
        const int d = 9 * W + t;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int co = 4 * ks + v;
            if (co < CO && c < CI) dst[(co * CI + c) * 27 + d] = acc[t][v];
        }
    }
    // biases: the g-staging threads' sums (thread t = co * nga + group), per
    // channel in group order; the x ring is free after the last barrier
    float* red = reinterpret_cast<float*>(xh);
    if (threadIdx.x < CO * nga) red[threadIdx.x] = bsum;
    __syncthreads();
    if (threadIdx.x < CO) {
        float sacc = 0.0f;
        for (int q = 0; q < nga; ++q) sacc += red[threadIdx.x * nga + q];
        dst[CO * CI * 27 + threadIdx.x] = sacc;
    }
}

template <int CI, int CO>
__global__ void __launch_bounds__(WGM_THREADS) __attribute__((amdgpu_waves_per_eu(2)))
k_conv_bwd_weight_mfma(Box bx, int64_t N, const float* __restrict__ g, const float* __restrict__ x,
                       float* __restrict__ part) {
    extern __shared__ __attribute__((aligned(16))) char wgm_smem[];
    const int nx = wgm_x_elems(bx.S2), ng = wgm_g_elems(bx.S2);
    __bf16* xh = reinterpret_cast<__bf16*>(wgm_smem);
    __bf16* xl = xh + nx;
    __bf16* gh = xl + nx;
    __bf16* gl = gh + ng;
    // zero once: channels past CI or CO and the tail are never staged
    for (int i = threadIdx.x; i < nx + ng; i += WGM_THREADS) reinterpret_cast<uint32_t*>(wgm_smem)[i] = 0u;
    __syncthreads();
    // XCD-aware order: workgroups are dealt to the 8 XCDs round robin, so the
    // ones on one XCD take a contiguous run of (part, sample, plane) with the
    // plane fastest; neighbouring planes read the same x rows from one L2
    const int total = gridDim.x, L = blockIdx.x, xcd = L % 8, q = total / 8, rem = total % 8;
    const int id = xcd * q + min(xcd, rem) + L / 8;
    const int r0 = id % bx.S0, b = (id / bx.S0) % (total / (bx.S0 * WGM_SPLIT)), part_i = id / (total / WGM_SPLIT);
    // the wave index as a scalar, so each wave branches to its own body only
    switch (__builtin_amdgcn_readfirstlane(threadIdx.x >> 6)) {
        case 0: wgm_body<CI, CO, 0>(bx, N, g, x, part, xh, xl, gh, gl, r0, b, part_i); break;
        case 1: wgm_body<CI, CO, 1>(bx, N, g, x, part, xh, xl, gh, gl, r0, b, part_i); break;
        default: wgm_body<CI, CO, 2>(bx, N, g, x, part, xh, xl, gh, gl, r0, b, part_i); break;
    }
}

// grad[i] = sum over the npart workgroup partials, FP64 in fixed order: 16
// strided partial sums per entry (one wave each), then their sum in order.
__global__ void __launch_bounds__(1024)
k_sum_weight_partials(const float* __restrict__ part, int npart, int nw, float* __restrict__ grad) {
    __shared__ double red[16][64];
    const int i = blockIdx.x * 64 + (threadIdx.x & 63), grp = threadIdx.x >> 6;
    double s = 0.0;
    if (i < nw)
        for (int c = grp; c < npart; c += 16) s += (double)part[(int64_t)c * nw + i];
    red[grp][threadIdx.x & 63] = s;
    __syncthreads();
    if (grp == 0 && i < nw) {
        double t = 0.0;
        for (int k = 0; k < 16; ++k) t += red[k][threadIdx.x];
        grad[i] = (float)t;
    }
}

// x = n0 / nbar (FP64 in, FP32 out)
__global__ void k_net_input(int64_t n, const double* __restrict__ n0, double inv_nbar, float* __restrict__ x) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) x[i] = (float)(n0[i] * inv_nbar);
}

// Per-sample FP64 sums of y (blockIdx.y = sample): part[b][block]
__global__ void __launch_bounds__(256)
k_sample_sum(int64_t N, const float* __restrict__ y, double* __restrict__ part) {
    __shared__ double red[256];
    const int b = blockIdx.y;
    double acc = 0;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < N; i += (int64_t)gridDim.x * 256)
        acc += (double)y[(int64_t)b * N + i];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[b * gridDim.x + blockIdx.x] = red[0];
}

// Loss gradient for every sample: e = y - mean(y) - t, t = (nconv - n0)/nbar;
// g = (2/N) (e - mean(e)) / batch; squared-error partials in FP64.
// ymean[b] and the sums of t (tsum[b]) come from k_sample_sum-style reductions.
__global__ void __launch_bounds__(256)
k_loss_grad(int64_t N, int batch, const float* __restrict__ y, const double* __restrict__ ysum,
            const double* __restrict__ n0, const double* __restrict__ nconv, double inv_nbar,
            const double* __restrict__ tsum, float* __restrict__ g, double* __restrict__ lpart) {
    __shared__ double red[256];
    const int b = blockIdx.y;
    const double ym = ysum[b] / (double)N;
    const double em = -tsum[b] / (double)N;  // mean(e) = -mean(t)
    double acc = 0;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < N; i += (int64_t)gridDim.x * 256) {
        const int64_t o = (int64_t)b * N + i;
        const double t = (nconv[o] - n0[o]) * inv_nbar;
        const double e = (double)y[o] - ym - t;
        acc += e * e;
        g[o] = (float)((2.0 / (double)N) * (e - em) / batch);
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) lpart[b * gridDim.x + blockIdx.x] = red[0];
}

// t sums per sample: sum_i (nconv - n0) * inv_nbar
__global__ void __launch_bounds__(256)
k_target_sum(int64_t N, const double* __restrict__ n0, const double* __restrict__ nconv, double inv_nbar,
             double* __restrict__ part) {
    __shared__ double red[256];
    const int b = blockIdx.y;
    double acc = 0;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < N; i += (int64_t)gridDim.x * 256) {
        const int64_t o = (int64_t)b * N + i;
        acc += (nconv[o] - n0[o]) * inv_nbar;
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[b * gridDim.x + blockIdx.x] = red[0];
}

// Fixed-order sums of per-sample partials: out[b] = sum_j part[b * nblk + j] * scale
// (block b; strided thread sums, then a fixed pairwise tree).
__global__ void __launch_bounds__(256)
k_sample_reduce(const double* __restrict__ part, int nblk, double scale, double* __restrict__ out) {
    __shared__ double red[256];
    const int b = blockIdx.x;
    double s = 0;
    for (int j = threadIdx.x; j < nblk; j += 256) s += part[(int64_t)b * nblk + j];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[b] = red[0] * scale;
}

// acc[0] += sum_b v[b] (one thread, fixed order): the epoch's loss stays on the device
__global__ void k_accumulate(const double* __restrict__ v, int nb, double* __restrict__ acc) {
    double s = 0;
    for (int b = 0; b < nb; ++b) s += v[b];
    acc[0] += s;
}

// dst[j] = src[order[j]] for the batch's samples (n0 and the target), N values each
__global__ void k_gather_samples(const int* __restrict__ order, int64_t N, const double* __restrict__ n0,
                                 const double* __restrict__ nc, double* __restrict__ d0, double* __restrict__ dc) {
    const int j = blockIdx.y;
    const int64_t srcoff = (int64_t)order[j] * N;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += (int64_t)gridDim.x * blockDim.x) {
        d0[(int64_t)j * N + i] = n0[srcoff + i];
        dc[(int64_t)j * N + i] = nc[srcoff + i];
    }
}

// Adam on FP32 master parameters; refreshes the BF16 weight copies.
__global__ void k_adam(int n, float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, float lr, float b1, float b2, float eps, float c1, float c2,
                       uint16_t* __restrict__ pbf, const int* __restrict__ is_weight) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float mh = mi / c1, vh = vi / c2;
    const float pi = p[i] - lr * mh / (sqrtf(vh) + eps);
    p[i] = pi;
    if (is_weight[i] >= 0) pbf[is_weight[i]] = f32_to_bf16(pi);
}

// Inference post-processing: n = max(n0 + nbar (y - mean y), 0); sums for the
// rescale to N_e in FP64 partials.
__global__ void __launch_bounds__(256)
k_predict_density(int64_t N, const double* __restrict__ n0, const float* __restrict__ y, const double* __restrict__ ysum,
                  double nbar, double* __restrict__ n, double* __restrict__ part) {
    __shared__ double red[256];
    const double ym = ysum[0] / (double)N;
    double acc = 0;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < N; i += (int64_t)gridDim.x * 256) {
        const double v = fmax(n0[i] + nbar * ((double)y[i] - ym), 0.0);
        n[i] = v;
        acc += v;
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ void k_scale_density(int64_t N, const double* __restrict__ part, int nblk, double target,
                                double* __restrict__ n) {
    __shared__ double tot;
    if (threadIdx.x == 0) {
        double s = 0;
        for (int j = 0; j < nblk; ++j) s += part[j];
        tot = s;
    }
    __syncthreads();
    const double f = target / tot;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += (int64_t)gridDim.x * blockDim.x)
        n[i] *= f;
}

}  // namespace dpp

using namespace dpp;

struct dpp_net_s {
    dpp_ctx ctx;
    Box bx;
    int64_t N;
    int max_batch;
    int nparam;                 // total parameters (weights + biases)
    int off_w[NL], off_b[NL];   // offsets into the flat FP32 parameter vector
    int woff_bf[NL];            // offsets into the BF16 weight copy
    float *p, *g, *m, *v;       // master params, grads, Adam moments (nparam)
    uint16_t* wbf;              // BF16 weights
    int* is_weight;             // param index -> BF16 index or -1
    float* act[NL + 1];         // act[0] = input x, act[l+1] = output of layer l (post-activation)
    float* pre[NL];             // pre-activations
    float* gbuf[2];             // gradient ping-pong (max_batch * 16 * N)
    float* wpart;               // weight-gradient partials
    bf8* apack;                 // MFMA A operands of the 16 -> 16 layers: [layer 1, 2][forward, transposed]
    double *dpart, *dsum, *tsum, *loss;
    double *stage_n0, *stage_nc;  // batch staging (gathered samples)
    int* d_order = nullptr;       // an epoch's sample order on the device
    int order_cap = 0;
    int adam_t;
    std::vector<void*> allocs;
};

namespace {
constexpr int RB = 256;  // reduction blocks per sample

dpp_status nalloc(dpp_net_s* n, void** p, size_t bytes) {
    if (hipMalloc(p, std::max<size_t>(bytes, 256)) != hipSuccess)
        return set_error(DPP_ENOMEM, "dpp_net_create: allocation failed");
    n->allocs.push_back(*p);
    return DPP_OK;
}

// A operands of layer l (1 or 2) for the forward or transposed product
bf8* apack_of(dpp_net_s* n, int l, bool trans) { return n->apack + ((l - 1) * 2 + (trans ? 1 : 0)) * C16_KSTEPS * 64; }

// 16 -> 16 layer on MFMA: forward (bias, SiLU into act) or backward-data
template <bool TRANS, bool ACT>
dpp_status launch_c16(dpp_net_s* n, int l, int batch, const float* src, const float* b, float* out, float* act) {
    bf8* ap = apack_of(n, l, TRANS);
    hipLaunchKernelGGL((k_pack_a16<TRANS>), dim3(1), dim3(C16_KSTEPS * 64), 0, n->ctx->stream,
                       (const uint16_t*)(n->wbf + n->woff_bf[l]), ap);
    DPP_LAUNCHED();
    const int rt = c16_rows(n->bx.S1, n->bx.S2), nblk = (n->bx.S1 + rt - 1) / rt;
    hipLaunchKernelGGL((k_conv16_mfma<TRANS, ACT>), dim3(n->bx.S0 * nblk * batch), dim3(C16_THREADS),
                       c16_lds_bytes(n->bx.S1, n->bx.S2), n->ctx->stream, n->bx, n->N, nblk, src, (const bf8*)ap, b,
                       out, act);
    DPP_LAUNCHED();
    return DPP_OK;
}

template <int CI, int CO, bool ACT>
dpp_status launch_fwd(dpp_net_s* n, int l, int batch, const float* x, const float* b, float* pre, float* act) {
    if constexpr (CI == 16 && CO == 16) {
        return launch_c16<false, ACT>(n, l, batch, x, b, pre, act);
    } else {
        const unsigned nb = (unsigned)((n->N + 255) / 256);
        hipLaunchKernelGGL((k_conv_fwd<CI, CO, ACT>), dim3(nb, batch), dim3(256), 0, n->ctx->stream, n->bx, n->N, x,
                           (const uint16_t*)(n->wbf + n->woff_bf[l]), b, pre, act);
        DPP_LAUNCHED();
        return DPP_OK;
    }
}

dpp_status net_forward(dpp_net_s* n, int batch) {
    TimerScope ts_(n->ctx, DPP_TK_NET, 0.0, 2.0 * batch * (double)n->N * (16 * 27 + 2 * 16 * 16 * 27 + 16 * 27));
    DPP_TRY((launch_fwd<1, 16, true>(n, 0, batch, n->act[0], n->p + n->off_b[0], n->pre[0], n->act[1])));
    DPP_TRY((launch_fwd<16, 16, true>(n, 1, batch, n->act[1], n->p + n->off_b[1], n->pre[1], n->act[2])));
    DPP_TRY((launch_fwd<16, 16, true>(n, 2, batch, n->act[2], n->p + n->off_b[2], n->pre[2], n->act[3])));
    DPP_TRY((launch_fwd<16, 1, false>(n, 3, batch, n->act[3], n->p + n->off_b[3], n->pre[3], nullptr)));
    return DPP_OK;
}

template <int CI, int CO>
dpp_status layer_backward(dpp_net_s* n, int l, int batch, const float* gin, float* gout, bool need_dx) {
    const unsigned nb = (unsigned)((n->N + 255) / 256);
    const int nw = CO * CI * 27 + CO;
    hipLaunchKernelGGL((k_conv_bwd_weight_mfma<CI, CO>), dim3(n->bx.S0 * batch * WGM_SPLIT), dim3(WGM_THREADS),
                       wgm_lds_bytes(n->bx.S2), n->ctx->stream, n->bx, n->N, gin, (const float*)n->act[l], n->wpart);
    DPP_LAUNCHED();
    // weights then biases are contiguous in the flat vector (off_b = off_w + CO*CI*27)
    hipLaunchKernelGGL(k_sum_weight_partials, dim3((nw + 63) / 64), dim3(1024), 0, n->ctx->stream,
                       (const float*)n->wpart, batch * n->bx.S0 * WGM_SPLIT, nw, n->g + n->off_w[l]);
    DPP_LAUNCHED();
    if (need_dx) {
        if constexpr (CI == 16 && CO == 16) {
            DPP_TRY((launch_c16<true, false>(n, l, batch, gin, n->pre[l - 1], gout, nullptr)));
        } else {
            hipLaunchKernelGGL((k_conv_bwd_data<CI, CO>), dim3(nb, batch), dim3(256), 0, n->ctx->stream, n->bx, n->N,
                               gin, (const uint16_t*)(n->wbf + n->woff_bf[l]), (const float*)n->pre[l - 1], gout);
            DPP_LAUNCHED();
        }
    }
    return DPP_OK;
}

dpp_status net_backward(dpp_net_s* n, int batch) {
    // gbuf[0] holds dL/dy (1 channel); walk the layers down
    TimerScope ts_(n->ctx, DPP_TK_NET, 0.0, 4.0 * batch * (double)n->N * (16 * 27 + 2 * 16 * 16 * 27 + 16 * 27));
    // each backward-data pass applies silu' of the layer below in its epilogue
    DPP_TRY((layer_backward<16, 1>(n, 3, batch, n->gbuf[0], n->gbuf[1], true)));
    DPP_TRY((layer_backward<16, 16>(n, 2, batch, n->gbuf[1], n->gbuf[0], true)));
    DPP_TRY((layer_backward<16, 16>(n, 1, batch, n->gbuf[0], n->gbuf[1], true)));
    DPP_TRY((layer_backward<1, 16>(n, 0, batch, n->gbuf[1], nullptr, false)));
    return DPP_OK;
}

dpp_status set_input(dpp_net_s* n, int batch, const double* d_n0, double nbar) {
    const int64_t tot = (int64_t)batch * n->N;
    hipLaunchKernelGGL(k_net_input, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, n->ctx->stream, tot, d_n0,
                       1.0 / nbar, n->act[0]);
    DPP_LAUNCHED();
    return DPP_OK;
}

dpp_status refresh_bf16(dpp_net_s* n, std::vector<float>& host) {
    std::vector<uint16_t> wb;
    for (int l = 0; l < NL; ++l)
        for (int i = 0; i < CH[l + 1] * CH[l] * 27; ++i) wb.push_back(f32_to_bf16(host[n->off_w[l] + i]));
    DPP_HIP(hipMemcpy(n->wbf, wb.data(), wb.size() * sizeof(uint16_t), hipMemcpyHostToDevice));
    return DPP_OK;
}
}  // namespace

extern "C" dpp_status dpp_net_create(dpp_ctx ctx, const int* S, int max_batch, dpp_net* out) {
    clear_error();
    DPP_REQUIRE(ctx && S && out && max_batch >= 1, "dpp_net_create: bad arguments");
    DPP_REQUIRE(S[0] >= 3 && S[1] >= 3 && S[2] >= 3, "dpp_net_create: box too small");
    // the weight-gradient kernel addresses one sample's 16 channels with 32-bit byte offsets below 2^31
    DPP_REQUIRE((int64_t)S[0] * S[1] * S[2] * 16 * 4 < ((int64_t)1 << 31), "dpp_net_create: box too large");
    // the 16 -> 16 MFMA layers hold 12 z tiles of 16 voxels per workgroup
    DPP_REQUIRE(S[2] <= 192, "dpp_net_create: rows longer than 192 voxels are not supported");
    dpp_net_s* n = new dpp_net_s();
    n->ctx = ctx;
    n->bx = Box{S[0], S[1], S[2]};
    n->N = (int64_t)S[0] * S[1] * S[2];
    n->max_batch = max_batch;
    n->adam_t = 0;
    int off = 0, offbf = 0;
    std::vector<int> isw;
    for (int l = 0; l < NL; ++l) {
        n->off_w[l] = off;
        n->woff_bf[l] = offbf;
        const int nw = CH[l + 1] * CH[l] * 27;
        for (int i = 0; i < nw; ++i) isw.push_back(offbf + i);
        off += nw;
        offbf += nw;
        n->off_b[l] = off;
        for (int i = 0; i < CH[l + 1]; ++i) isw.push_back(-1);
        off += CH[l + 1];
    }
    n->nparam = off;
    auto fail = [&](dpp_status st) {
        std::string msg = dpp_last_error();
        dpp_net_destroy(n);
        return set_error(st, msg);
    };
    dpp_status st;
    const size_t np = n->nparam;
    if ((st = nalloc(n, (void**)&n->p, np * 4)) || (st = nalloc(n, (void**)&n->g, np * 4)) ||
        (st = nalloc(n, (void**)&n->m, np * 4)) || (st = nalloc(n, (void**)&n->v, np * 4)) ||
        (st = nalloc(n, (void**)&n->wbf, offbf * 2)) || (st = nalloc(n, (void**)&n->is_weight, np * 4)))
        return fail(st);
    const size_t a16 = (size_t)max_batch * 16 * n->N * 4;
    const size_t a1 = (size_t)max_batch * n->N * 4;
    if ((st = nalloc(n, (void**)&n->act[0], a1))) return fail(st);
    for (int l = 0; l < NL; ++l) {
        const size_t sz = l < 3 ? a16 : a1;
        if ((st = nalloc(n, (void**)&n->pre[l], sz))) return fail(st);
        if (l < 3 && (st = nalloc(n, (void**)&n->act[l + 1], sz))) return fail(st);
    }
    n->act[4] = n->pre[3];
    if ((st = nalloc(n, (void**)&n->gbuf[0], a16)) || (st = nalloc(n, (void**)&n->gbuf[1], a16)) ||
        (st = nalloc(n, (void**)&n->wpart, (size_t)max_batch * S[0] * WGM_SPLIT * (16 * 16 * 27 + 16) * 4)) ||
        (st = nalloc(n, (void**)&n->apack, (size_t)4 * C16_KSTEPS * 64 * sizeof(bf8))) ||
        (st = nalloc(n, (void**)&n->dpart, (size_t)max_batch * RB * 8 * 2)) ||
        (st = nalloc(n, (void**)&n->dsum, (size_t)max_batch * 8)) ||
        (st = nalloc(n, (void**)&n->tsum, (size_t)max_batch * 8)) || (st = nalloc(n, (void**)&n->loss, 64)) ||
        (st = nalloc(n, (void**)&n->stage_n0, (size_t)max_batch * n->N * 8)) ||
        (st = nalloc(n, (void**)&n->stage_nc, (size_t)max_batch * n->N * 8)))
        return fail(st);
    // dynamic LDS: weight gradient 58 KB for a 40-voxel row (83 KB from 57 voxels up);
    // 16 -> 16 layers 58 KB at 40 voxels, at most 112 KB
    const int lds = (int)wgm_lds_bytes(S[2]);
    if (hipFuncSetAttribute((const void*)k_conv_bwd_weight_mfma<1, 16>, hipFuncAttributeMaxDynamicSharedMemorySize,
                            lds) != hipSuccess ||
        hipFuncSetAttribute((const void*)k_conv_bwd_weight_mfma<16, 16>, hipFuncAttributeMaxDynamicSharedMemorySize,
                            lds) != hipSuccess ||
        hipFuncSetAttribute((const void*)k_conv_bwd_weight_mfma<16, 1>, hipFuncAttributeMaxDynamicSharedMemorySize,
                            lds) != hipSuccess ||
        hipFuncSetAttribute((const void*)k_conv16_mfma<false, true>, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)c16_lds_bytes(S[1], S[2])) != hipSuccess ||
        hipFuncSetAttribute((const void*)k_conv16_mfma<true, false>, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)c16_lds_bytes(S[1], S[2])) != hipSuccess) {
        set_error(DPP_EDEVICE, "dpp_net_create: weight-gradient LDS size not accepted");
        return fail(DPP_EDEVICE);
    }
    if (hipMemcpy(n->is_weight, isw.data(), np * 4, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemset(n->m, 0, np * 4) != hipSuccess || hipMemset(n->v, 0, np * 4) != hipSuccess ||
        hipMemset(n->g, 0, np * 4) != hipSuccess) {
        set_error(DPP_EDEVICE, "dpp_net_create: initialisation copy failed");
        return fail(DPP_EDEVICE);
    }
    *out = n;
    return DPP_OK;
}

extern "C" dpp_status dpp_net_destroy(dpp_net n) {
    if (!n) return DPP_OK;
    (void)hipStreamSynchronize(n->ctx->stream);  // best effort: the net is released regardless
    for (void* p : n->allocs) (void)hipFree(p);
    delete n;
    return DPP_OK;
}

extern "C" dpp_status dpp_net_num_params(dpp_net n, int* count) {
    clear_error();
    DPP_REQUIRE(n && count, "dpp_net_num_params: null argument");
    *count = n->nparam;
    return DPP_OK;
}

extern "C" dpp_status dpp_net_set_params(dpp_net n, const float* h_params) {
    clear_error();
    DPP_REQUIRE(n && h_params, "dpp_net_set_params: null argument");
    std::vector<float> host(h_params, h_params + n->nparam);
    DPP_HIP(hipStreamSynchronize(n->ctx->stream));
    DPP_HIP(hipMemcpy(n->p, host.data(), n->nparam * 4, hipMemcpyHostToDevice));
    DPP_TRY(refresh_bf16(n, host));
    DPP_HIP(hipMemset(n->m, 0, n->nparam * 4));
    DPP_HIP(hipMemset(n->v, 0, n->nparam * 4));
    n->adam_t = 0;
    return DPP_OK;
}

extern "C" dpp_status dpp_net_get_params(dpp_net n, float* h_params, float* h_grads) {
    clear_error();
    DPP_REQUIRE(n, "dpp_net_get_params: null net");
    DPP_HIP(hipStreamSynchronize(n->ctx->stream));
    if (h_params) DPP_HIP(hipMemcpy(h_params, n->p, n->nparam * 4, hipMemcpyDeviceToHost));
    if (h_grads) DPP_HIP(hipMemcpy(h_grads, n->g, n->nparam * 4, hipMemcpyDeviceToHost));
    return DPP_OK;
}

extern "C" dpp_status dpp_net_forward(dpp_net n, int batch, const double* d_n0, double nbar, float* d_y) {
    clear_error();
    DPP_REQUIRE(n && d_n0 && batch >= 1 && batch <= n->max_batch && nbar > 0, "dpp_net_forward: bad arguments");
    DPP_TRY(set_input(n, batch, d_n0, nbar));
    DPP_TRY(net_forward(n, batch));
    if (d_y)
        DPP_HIP(hipMemcpyAsync(d_y, n->pre[3], (size_t)batch * n->N * 4, hipMemcpyDeviceToDevice, n->ctx->stream));
    return DPP_OK;
}

// Loss and gradients for a batch (after dpp_net_forward of the same inputs).
static dpp_status loss_backward(dpp_net_s* n, int batch, const double* d_n0, const double* d_nconv, double nbar) {
    hipStream_t st = n->ctx->stream;
    const double inv = 1.0 / nbar;
    hipLaunchKernelGGL(k_sample_sum, dim3(RB, batch), dim3(256), 0, st, n->N, (const float*)n->pre[3], n->dpart);
    DPP_LAUNCHED();
    hipLaunchKernelGGL(k_sample_reduce, dim3(batch), dim3(256), 0, st, (const double*)n->dpart, RB, 1.0, n->dsum);
    DPP_LAUNCHED();
    hipLaunchKernelGGL(k_target_sum, dim3(RB, batch), dim3(256), 0, st, n->N, d_n0, d_nconv, inv, n->dpart);
    DPP_LAUNCHED();
    hipLaunchKernelGGL(k_sample_reduce, dim3(batch), dim3(256), 0, st, (const double*)n->dpart, RB, 1.0, n->tsum);
    DPP_LAUNCHED();
    hipLaunchKernelGGL(k_loss_grad, dim3(RB, batch), dim3(256), 0, st, n->N, batch, (const float*)n->pre[3],
                       (const double*)n->dsum, d_n0, d_nconv, inv, (const double*)n->tsum, n->gbuf[0], n->dpart);
    DPP_LAUNCHED();
    // loss = mean over samples of mean over points
    hipLaunchKernelGGL(k_sample_reduce, dim3(batch), dim3(256), 0, st, (const double*)n->dpart, RB,
                       1.0 / ((double)n->N * batch), n->dsum);
    DPP_LAUNCHED();
    DPP_TRY(net_backward(n, batch));
    return DPP_OK;
}

extern "C" dpp_status dpp_net_backward(dpp_net n, int batch, const double* d_n0, const double* d_nconv, double nbar,
                                       double* loss) {
    clear_error();
    DPP_REQUIRE(n && d_n0 && d_nconv && batch >= 1 && batch <= n->max_batch && nbar > 0,
                "dpp_net_backward: bad arguments");
    DPP_TRY(loss_backward(n, batch, d_n0, d_nconv, nbar));
    if (loss) {
        std::vector<double> lv(batch);
        DPP_HIP(hipMemcpyAsync(lv.data(), n->dsum, batch * 8, hipMemcpyDeviceToHost, n->ctx->stream));
        DPP_HIP(hipStreamSynchronize(n->ctx->stream));
        double s = 0;
        for (double v : lv) s += v;
        *loss = s;
    }
    return DPP_OK;
}

extern "C" dpp_status dpp_net_adam_step(dpp_net n, double lr) {
    clear_error();
    DPP_REQUIRE(n && lr > 0, "dpp_net_adam_step: bad arguments");
    n->adam_t += 1;
    const float b1 = 0.9f, b2 = 0.999f;
    const float c1 = 1.0f - std::pow(b1, (float)n->adam_t), c2 = 1.0f - std::pow(b2, (float)n->adam_t);
    hipLaunchKernelGGL(k_adam, dim3((n->nparam + 255) / 256), dim3(256), 0, n->ctx->stream, n->nparam, n->p,
                       (const float*)n->g, n->m, n->v, (float)lr, b1, b2, 1e-8f, c1, c2, n->wbf,
                       (const int*)n->is_weight);
    DPP_LAUNCHED();
    return DPP_OK;
}

extern "C" dpp_status dpp_net_predict_density(dpp_net n, const double* d_n0, double n_electrons, double omega,
                                              double* d_n_out) {
    clear_error();
    DPP_REQUIRE(n && d_n0 && d_n_out && n_electrons > 0 && omega > 0, "dpp_net_predict_density: bad arguments");
    const double nbar = n_electrons / omega;
    DPP_TRY(set_input(n, 1, d_n0, nbar));
    DPP_TRY(net_forward(n, 1));
    hipStream_t st = n->ctx->stream;
    hipLaunchKernelGGL(k_sample_sum, dim3(RB, 1), dim3(256), 0, st, n->N, (const float*)n->pre[3], n->dpart);
    DPP_LAUNCHED();
    hipLaunchKernelGGL(k_sample_reduce, dim3(1), dim3(256), 0, st, (const double*)n->dpart, RB, 1.0, n->dsum);
    DPP_LAUNCHED();
    hipLaunchKernelGGL(k_predict_density, dim3(RB), dim3(256), 0, st, n->N, d_n0, (const float*)n->pre[3],
                       (const double*)n->dsum, nbar, d_n_out, n->dpart);
    DPP_LAUNCHED();
    // (Omega/N) sum n = N_e  <=>  sum n = N_e N / Omega
    hipLaunchKernelGGL(k_scale_density, dim3(RB), dim3(256), 0, st, n->N, (const double*)n->dpart, RB,
                       n_electrons * (double)n->N / omega, d_n_out);
    DPP_LAUNCHED();
    return DPP_OK;
}

extern "C" dpp_status dpp_net_train_epoch(dpp_net n, int nsamples, const double* d_n0, const double* d_nconv,
                                          double nbar, int batch, double lr, const int* order, double* mean_loss) {
    clear_error();
    DPP_REQUIRE(n && d_n0 && d_nconv && order && nsamples >= 1 && batch >= 1 && batch <= n->max_batch && nbar > 0 &&
                    lr > 0,
                "dpp_net_train_epoch: bad arguments");
    for (int i = 0; i < nsamples; ++i)
        DPP_REQUIRE(order[i] >= 0 && order[i] < nsamples, "dpp_net_train_epoch: order out of range");
    hipStream_t st = n->ctx->stream;
    if (n->order_cap < nsamples) {
        int* d = nullptr;
        if (hipMalloc((void**)&d, (size_t)nsamples * sizeof(int)) != hipSuccess)
            return set_error(DPP_ENOMEM, "dpp_net_train_epoch: allocation failed");
        n->allocs.push_back(d);
        n->d_order = d;
        n->order_cap = nsamples;
    }
    DPP_HIP(hipMemcpyAsync(n->d_order, order, (size_t)nsamples * sizeof(int), hipMemcpyHostToDevice, st));
    DPP_HIP(hipMemsetAsync(n->loss, 0, sizeof(double), st));
    // the batch losses are summed on the device; one readback per epoch
    int nbt = 0;
    for (int s0 = 0; s0 < nsamples; s0 += batch) {
        const int bsz = std::min(batch, nsamples - s0);
        hipLaunchKernelGGL(k_gather_samples, dim3(64, bsz), dim3(256), 0, st, (const int*)(n->d_order + s0), n->N,
                           d_n0, d_nconv, n->stage_n0, n->stage_nc);
        DPP_LAUNCHED();
        DPP_TRY(set_input(n, bsz, n->stage_n0, nbar));
        DPP_TRY(net_forward(n, bsz));
        DPP_TRY(loss_backward(n, bsz, n->stage_n0, n->stage_nc, nbar));
        hipLaunchKernelGGL(k_accumulate, dim3(1), dim3(1), 0, st, (const double*)n->dsum, bsz, n->loss);
        DPP_LAUNCHED();
        DPP_TRY(dpp_net_adam_step(n, lr));
        ++nbt;
    }
    double tot = 0;
    DPP_HIP(hipMemcpyAsync(&tot, n->loss, sizeof(double), hipMemcpyDeviceToHost, st));
    DPP_HIP(hipStreamSynchronize(st));
    if (mean_loss) *mean_loss = tot / nbt;
    return DPP_OK;
}
