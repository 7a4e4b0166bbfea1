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
// backward-weights (one thread per weight over a voxel chunk, chunk partials
// reduced in fixed order), SiLU backward, loss, Adam.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <vector>

#include "internal.h"

namespace dpp {

constexpr int NL = 4;
constexpr int CH[NL + 1] = {1, 16, 16, 16, 1};
constexpr int WG_CHUNKS = 128;  // voxel chunks of the weight-gradient reduction

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

// dx[b][ci][s] = sum_co sum_d W[co][ci][d] g[b][co][s - d]
template <int CI, int CO>
__global__ void __launch_bounds__(256)
k_conv_bwd_data(Box bx, int64_t N, const float* __restrict__ g, const uint16_t* __restrict__ W,
                float* __restrict__ dx) {
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
    for (int ci = 0; ci < CI; ++ci) dx[((int64_t)b * CI + ci) * N + s] = acc[ci];
}

// Weight-gradient partials: part[chunk][widx] = sum over the chunk's voxels
// (all batch samples) of g[b][co][r] x[b][ci][r + d]; bias partials after the
// weights (widx = CO*CI*27 + co).  One thread per gradient entry.
template <int CI, int CO>
__global__ void __launch_bounds__(256)
k_conv_bwd_weight(Box bx, int64_t N, int batch, const float* __restrict__ g, const float* __restrict__ x,
                  float* __restrict__ part) {
    const int nw = CO * CI * 27 + CO;
    const int widx = blockIdx.x * blockDim.x + threadIdx.x;
    const int chunk = blockIdx.y;
    if (widx >= nw) return;
    const int64_t per = (N + WG_CHUNKS - 1) / WG_CHUNKS;
    const int64_t r_a = chunk * per, r_e = min(N, r_a + per);
    float acc = 0.0f;
    if (widx < CO * CI * 27) {
        const int co = widx / (CI * 27), rem = widx - co * CI * 27;
        const int ci = rem / 27, d = rem - ci * 27;
        const int d0 = d / 9 - 1, d1 = (d / 3) % 3 - 1, d2 = d % 3 - 1;
        for (int b = 0; b < batch; ++b) {
            const float* gb = g + ((int64_t)b * CO + co) * N;
            const float* xb = x + ((int64_t)b * CI + ci) * N;
            for (int64_t r = r_a; r < r_e; ++r) {
                const int r2 = (int)(r % bx.S2);
                const int64_t q = r / bx.S2;
                const int r1 = (int)(q % bx.S1), r0 = (int)(q / bx.S1);
                acc += gb[r] * xb[shifted(bx, r0, r1, r2, d0, d1, d2)];
            }
        }
    } else {
        const int co = widx - CO * CI * 27;
        for (int b = 0; b < batch; ++b) {
            const float* gb = g + ((int64_t)b * CO + co) * N;
            for (int64_t r = r_a; r < r_e; ++r) acc += gb[r];
        }
    }
    part[(int64_t)chunk * nw + widx] = acc;
}

__global__ void k_sum_chunks(const float* __restrict__ part, int nw, float* __restrict__ grad) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nw) return;
    float s = 0.0f;
    for (int c = 0; c < WG_CHUNKS; ++c) s += part[(int64_t)c * nw + i];
    grad[i] = s;
}

// g *= silu'(a)
__global__ void k_silu_bwd(int64_t n, const float* __restrict__ a, float* __restrict__ g) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float s = sigm(a[i]);
    g[i] *= s * (1.0f + a[i] * (1.0f - s));
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

// Fixed-order sums of per-sample partials: out[b] = sum_j part[b * nblk + j] * scale.
__global__ void k_sample_reduce(const double* __restrict__ part, int nblk, int batch, double scale,
                                double* __restrict__ out) {
    const int b = threadIdx.x;
    if (b >= batch) return;
    double s = 0;
    for (int j = 0; j < nblk; ++j) s += part[b * nblk + j];
    out[b] = s * scale;
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
    double *dpart, *dsum, *tsum, *loss;
    double *stage_n0, *stage_nc;  // batch staging (gathered samples)
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

template <int CI, int CO, bool ACT>
dpp_status launch_fwd(dpp_net_s* n, int batch, const float* x, const uint16_t* W, const float* b, float* pre, float* act) {
    const unsigned nb = (unsigned)((n->N + 255) / 256);
    hipLaunchKernelGGL((k_conv_fwd<CI, CO, ACT>), dim3(nb, batch), dim3(256), 0, n->ctx->stream, n->bx, n->N, x, W, b,
                       pre, act);
    DPP_LAUNCHED();
    return DPP_OK;
}

dpp_status net_forward(dpp_net_s* n, int batch) {
    TimerScope ts_(n->ctx, DPP_TK_NET, 0.0, 2.0 * batch * (double)n->N * (16 * 27 + 2 * 16 * 16 * 27 + 16 * 27));
    DPP_TRY((launch_fwd<1, 16, true>(n, batch, n->act[0], n->wbf + n->woff_bf[0], n->p + n->off_b[0], n->pre[0], n->act[1])));
    DPP_TRY((launch_fwd<16, 16, true>(n, batch, n->act[1], n->wbf + n->woff_bf[1], n->p + n->off_b[1], n->pre[1], n->act[2])));
    DPP_TRY((launch_fwd<16, 16, true>(n, batch, n->act[2], n->wbf + n->woff_bf[2], n->p + n->off_b[2], n->pre[2], n->act[3])));
    DPP_TRY((launch_fwd<16, 1, false>(n, batch, n->act[3], n->wbf + n->woff_bf[3], n->p + n->off_b[3], n->pre[3], nullptr)));
    return DPP_OK;
}

template <int CI, int CO>
dpp_status layer_backward(dpp_net_s* n, int l, int batch, const float* gin, float* gout, bool need_dx) {
    const unsigned nb = (unsigned)((n->N + 255) / 256);
    const int nw = CO * CI * 27 + CO;
    hipLaunchKernelGGL((k_conv_bwd_weight<CI, CO>), dim3((nw + 255) / 256, WG_CHUNKS), dim3(256), 0, n->ctx->stream,
                       n->bx, n->N, batch, gin, (const float*)n->act[l], n->wpart);
    DPP_LAUNCHED();
    // weights then biases are contiguous in the flat vector (off_b = off_w + CO*CI*27)
    hipLaunchKernelGGL(k_sum_chunks, dim3((nw + 255) / 256), dim3(256), 0, n->ctx->stream, (const float*)n->wpart, nw,
                       n->g + n->off_w[l]);
    DPP_LAUNCHED();
    if (need_dx) {
        hipLaunchKernelGGL((k_conv_bwd_data<CI, CO>), dim3(nb, batch), dim3(256), 0, n->ctx->stream, n->bx, n->N, gin,
                           (const uint16_t*)(n->wbf + n->woff_bf[l]), gout);
        DPP_LAUNCHED();
    }
    return DPP_OK;
}

dpp_status net_backward(dpp_net_s* n, int batch) {
    // gbuf[0] holds dL/dy (1 channel); walk the layers down
    TimerScope ts_(n->ctx, DPP_TK_NET, 0.0, 4.0 * batch * (double)n->N * (16 * 27 + 2 * 16 * 16 * 27 + 16 * 27));
    const int64_t nb16 = (int64_t)batch * 16 * n->N;
    const unsigned eb = (unsigned)((nb16 + 255) / 256);
    DPP_TRY((layer_backward<16, 1>(n, 3, batch, n->gbuf[0], n->gbuf[1], true)));
    hipLaunchKernelGGL(k_silu_bwd, dim3(eb), dim3(256), 0, n->ctx->stream, nb16, (const float*)n->pre[2], n->gbuf[1]);
    DPP_LAUNCHED();
    DPP_TRY((layer_backward<16, 16>(n, 2, batch, n->gbuf[1], n->gbuf[0], true)));
    hipLaunchKernelGGL(k_silu_bwd, dim3(eb), dim3(256), 0, n->ctx->stream, nb16, (const float*)n->pre[1], n->gbuf[0]);
    DPP_LAUNCHED();
    DPP_TRY((layer_backward<16, 16>(n, 1, batch, n->gbuf[0], n->gbuf[1], true)));
    hipLaunchKernelGGL(k_silu_bwd, dim3(eb), dim3(256), 0, n->ctx->stream, nb16, (const float*)n->pre[0], n->gbuf[1]);
    DPP_LAUNCHED();
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

void refresh_bf16(dpp_net_s* n, std::vector<float>& host) {
    std::vector<uint16_t> wb;
    for (int l = 0; l < NL; ++l)
        for (int i = 0; i < CH[l + 1] * CH[l] * 27; ++i) wb.push_back(f32_to_bf16(host[n->off_w[l] + i]));
    hipMemcpy(n->wbf, wb.data(), wb.size() * sizeof(uint16_t), hipMemcpyHostToDevice);
}
}  // namespace

extern "C" dpp_status dpp_net_create(dpp_ctx ctx, const int* S, int max_batch, dpp_net* out) {
    clear_error();
    DPP_REQUIRE(ctx && S && out && max_batch >= 1, "dpp_net_create: bad arguments");
    DPP_REQUIRE(S[0] >= 3 && S[1] >= 3 && S[2] >= 3, "dpp_net_create: box too small");
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
        (st = nalloc(n, (void**)&n->wpart, (size_t)WG_CHUNKS * (16 * 16 * 27 + 16) * 4)) ||
        (st = nalloc(n, (void**)&n->dpart, (size_t)max_batch * RB * 8 * 2)) ||
        (st = nalloc(n, (void**)&n->dsum, (size_t)max_batch * 8)) ||
        (st = nalloc(n, (void**)&n->tsum, (size_t)max_batch * 8)) || (st = nalloc(n, (void**)&n->loss, 64)) ||
        (st = nalloc(n, (void**)&n->stage_n0, (size_t)max_batch * n->N * 8)) ||
        (st = nalloc(n, (void**)&n->stage_nc, (size_t)max_batch * n->N * 8)))
        return fail(st);
    hipMemcpy(n->is_weight, isw.data(), np * 4, hipMemcpyHostToDevice);
    hipMemset(n->m, 0, np * 4);
    hipMemset(n->v, 0, np * 4);
    hipMemset(n->g, 0, np * 4);
    *out = n;
    return DPP_OK;
}

extern "C" dpp_status dpp_net_destroy(dpp_net n) {
    if (!n) return DPP_OK;
    hipStreamSynchronize(n->ctx->stream);
    for (void* p : n->allocs) hipFree(p);
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
    refresh_bf16(n, host);
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
    hipLaunchKernelGGL(k_sample_reduce, dim3(1), dim3(64), 0, st, (const double*)n->dpart, RB, batch, 1.0, n->dsum);
    DPP_LAUNCHED();
    hipLaunchKernelGGL(k_target_sum, dim3(RB, batch), dim3(256), 0, st, n->N, d_n0, d_nconv, inv, n->dpart);
    DPP_LAUNCHED();
    hipLaunchKernelGGL(k_sample_reduce, dim3(1), dim3(64), 0, st, (const double*)n->dpart, RB, batch, 1.0, n->tsum);
    DPP_LAUNCHED();
    hipLaunchKernelGGL(k_loss_grad, dim3(RB, batch), dim3(256), 0, st, n->N, batch, (const float*)n->pre[3],
                       (const double*)n->dsum, d_n0, d_nconv, inv, (const double*)n->tsum, n->gbuf[0], n->dpart);
    DPP_LAUNCHED();
    // loss = mean over samples of mean over points
    hipLaunchKernelGGL(k_sample_reduce, dim3(1), dim3(64), 0, st, (const double*)n->dpart, RB, batch,
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
    hipLaunchKernelGGL(k_sample_reduce, dim3(1), dim3(64), 0, st, (const double*)n->dpart, RB, 1, 1.0, n->dsum);
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
    const size_t bytes = (size_t)n->N * sizeof(double);
    double tot = 0;
    int nbt = 0;
    for (int s0 = 0; s0 < nsamples; s0 += batch) {
        const int bsz = std::min(batch, nsamples - s0);
        for (int j = 0; j < bsz; ++j) {
            const int64_t src = (int64_t)order[s0 + j] * n->N;
            DPP_HIP(hipMemcpyAsync(n->stage_n0 + (int64_t)j * n->N, d_n0 + src, bytes, hipMemcpyDeviceToDevice, st));
            DPP_HIP(hipMemcpyAsync(n->stage_nc + (int64_t)j * n->N, d_nconv + src, bytes, hipMemcpyDeviceToDevice, st));
        }
        DPP_TRY(set_input(n, bsz, n->stage_n0, nbar));
        DPP_TRY(net_forward(n, bsz));
        double l = 0;
        DPP_TRY(dpp_net_backward(n, bsz, n->stage_n0, n->stage_nc, nbar, &l));
        DPP_TRY(dpp_net_adam_step(n, lr));
        tot += l;
        ++nbt;
    }
    if (mean_loss) *mean_loss = tot / nbt;
    return DPP_OK;
}
