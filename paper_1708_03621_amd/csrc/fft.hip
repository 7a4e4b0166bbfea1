// Sphere <-> grid transforms (I, I^dag), the local part of H, full-box
// transforms (J, J^dag), the Hartree solve and density accumulation.
//
// A 3D transform is split into three passes over an intermediate buffer that
// holds, per band, only the x-planes the G-sphere touches (Miller index n0 in
// [n0min, n0max]):
//   pass 1 (plane kernel)  one workgroup per (item, band, plane): scatter the
//                          plane's sphere points into LDS, transform along z
//                          (only the rows holding points) and along y, store
//                          the S1 x S2 plane.
//   pass 2 (xz kernel)     one workgroup per (item, band, i1): gather the
//                          pruned rows of the x-z plane, zero the others,
//                          transform along x, apply the pointwise operation
//                          (V_eff multiply, |psi|^2, store), transform back,
//                          store the pruned rows.
//   pass 3 (plane kernel)  transform y then z (pruned rows) and gather the
//                          sphere points (plus the kinetic term for H).
// Full-box fields use the same passes with every plane and row present.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "fft_engine.h"
#include "fft_reg.h"
#include "internal.h"

namespace dpp {

bool factor_axis(int n, FftAxis* ax) {
    ax->n = n;
    ax->nrad = 0;
    int m = n;
    while (m % 4 == 0 && ax->nrad < MAX_RADICES) ax->rad[ax->nrad++] = 4, m /= 4;
    while (m % 2 == 0 && ax->nrad < MAX_RADICES) ax->rad[ax->nrad++] = 2, m /= 2;
    while (m % 3 == 0 && ax->nrad < MAX_RADICES) ax->rad[ax->nrad++] = 3, m /= 3;
    while (m % 5 == 0 && ax->nrad < MAX_RADICES) ax->rad[ax->nrad++] = 5, m /= 5;
    return m == 1;
}

// Threads per workgroup for a tile of `elems` complex values: each thread
// holds at most 16 complex values per stage (radix 3 and 5: 15).
int fft_threads(int elems) {
    if (elems <= 15 * 256) return 256;
    if (elems <= 15 * 512) return 512;
    if (elems <= 8 * 1024) return 1024;
    return 0;
}

size_t fft_lds_bytes(int elems, bool fp64) { return (size_t)elems * (fp64 ? 16 : 8); }

dpp_status check_fft_shape(int S0, int S1, int S2, bool fp64) {
    const int e1 = S1 * S2, e2 = S0 * S2;
    const int e = std::max(e1, e2);
    if (fft_threads(e) == 0 || fft_lds_bytes(e, fp64) > 160 * 1024)
        return set_error(DPP_EUNSUPPORTED, "FFT plane too large for one workgroup's LDS");
    return DPP_OK;
}

size_t plane_buffer_elems(const dpp_basis_s* b, int nb) {
    return (size_t)nb * b->nplanes * b->grid->S[1] * b->grid->S[2];
}

template <typename T>
__device__ __forceinline__ const double2* TW64(const FftItem& it, int a) {
    return it.tw64[a];
}

template <typename T>
struct Io;
template <>
struct Io<double> {
    __device__ static double2 from(double2 v) { return v; }
    __device__ static double2 from(float2 v) { return double2{v.x, v.y}; }
    __device__ static double2 to_d(double2 v) { return v; }
};
template <>
struct Io<float> {
    __device__ static float2 from(double2 v) { return float2{(float)v.x, (float)v.y}; }
    __device__ static float2 from(float2 v) { return v; }
    __device__ static double2 to_d(float2 v) { return double2{v.x, v.y}; }
};

template <typename TO>
struct Out;
template <>
struct Out<double2> {
    __device__ static double2 make(double x, double y) { return double2{x, y}; }
};
template <>
struct Out<float2> {
    __device__ static float2 make(double x, double y) { return float2{(float)x, (float)y}; }
};
template <typename TO, typename C>
__device__ __forceinline__ TO store_as(C v) {
    return Out<TO>::make((double)v.x, (double)v.y);
}

// Kernels take the item either by value (one item per launch) or from a device
// table indexed by blockIdx.z (batched launches); the choice is compile-time.
#define DPP_ITEM(items, single) (BATCH ? (items)[blockIdx.z] : (single))

// ------------------------------------------------ 90-point transforms ------
// Square faces of 90 points (the 90^3 box) have dedicated LDS paths.  Each
// 90-point transform is split as 9 x 10 (n = n1 + 10 n2, k = 9 k1 + k2, so
// w^(nk) = w10^(n1 k1) w^(n1 k2) w9^(n2 k2)):
//   step A, per (transform, n1): 9-point DFT over n2 in registers, times
//           w^(n1 k2), stored back to the slots n1 + 10 k2 it read;
//   step B, per (transform, k2): 10-point DFT over n1 of those slots, giving
//           X[9 k1 + k2], stored to slot k1 + 10 k2 (the slots it read).
// Both steps touch only their own slots, so an axis costs two LDS round trips
// and one barrier between them, against one round trip and two barriers per
// radix stage in the generic kernel.  Step B leaves the axis permuted: natural
// index i sits at slot(i) = i / 9 + 10 (i mod 9).  Where a step can read its
// input from, or write its output to, device memory directly (the first and
// last steps of a pass), it does.
namespace p90 {
constexpr int N = 90;
constexpr int NT = 1024;

__device__ __forceinline__ int slot(int i) { return i / 9 + 10 * (i - 9 * (i / 9)); }

// 9-point DFT as 3 x 3: v[3p + q] -> rows q, 3-point DFTs over p, twiddles
// w9^(q c), 3-point DFTs over q, X[c + 3d].
template <typename T, int SIGN>
__device__ __forceinline__ void dft9(typename cx<T>::t* v) {
    using C = typename cx<T>::t;
    const T c1 = T(0.766044443118978), s1 = T(SIGN) * T(0.6427876096865393);
    const T c2 = T(0.17364817766693041), s2 = T(SIGN) * T(0.984807753012208);
    const T c4 = T(-0.9396926207859083), s4 = T(SIGN) * T(0.3420201433256689);
    C a[3][3];
#pragma unroll
    for (int q = 0; q < 3; ++q) {
        a[q][0] = v[q];
        a[q][1] = v[q + 3];
        a[q][2] = v[q + 6];
        Dft<T, 3>::run(a[q], SIGN);
    }
    a[1][1] = cmul(a[1][1], C{c1, s1});
    a[1][2] = cmul(a[1][2], C{c2, s2});
    a[2][1] = cmul(a[2][1], C{c2, s2});
    a[2][2] = cmul(a[2][2], C{c4, s4});
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        C b[3] = {a[0][c], a[1][c], a[2][c]};
        Dft<T, 3>::run(b, SIGN);
        v[c] = b[0];
        v[c + 3] = b[1];
        v[c + 6] = b[2];
    }
}

// 10-point DFT as 5 x 2: 5-point DFTs of the even and odd points, twiddles
// w10^c on the odd ones, X[c] = e + o, X[c + 5] = e - o.
template <typename T, int SIGN>
__device__ __forceinline__ void dft10(typename cx<T>::t* v) {
    using C = typename cx<T>::t;
    const T c1 = T(0.8090169943749475), s1 = T(SIGN) * T(0.5877852522924731);
    const T c2 = T(0.30901699437494745), s2 = T(SIGN) * T(0.9510565162951535);
    C e[5], o[5];
#pragma unroll
    for (int p = 0; p < 5; ++p) {
        e[p] = v[2 * p];
        o[p] = v[2 * p + 1];
    }
    Dft<T, 5>::run(e, SIGN);
    Dft<T, 5>::run(o, SIGN);
    o[1] = cmul(o[1], C{c1, s1});
    o[2] = cmul(o[2], C{c2, s2});
    o[3] = cmul(o[3], C{-c2, s2});
    o[4] = cmul(o[4], C{-c1, s1});
#pragma unroll
    for (int c = 0; c < 5; ++c) {
        v[c] = cadd(e[c], o[c]);
        v[c + 5] = csub(e[c], o[c]);
    }
}

// Step A on the 9 values of one (transform, n1) task: DFT and twiddles.
template <typename T, int SIGN>
__device__ __forceinline__ void step_a(typename cx<T>::t* v, int n1, const double2* tw64, const float2* tw32) {
    dft9<T, SIGN>(v);
#pragma unroll
    for (int k2 = 1; k2 < 9; ++k2) v[k2] = cmul(v[k2], twiddle<T>(tw64, tw32, n1 * k2, SIGN));
}

// Natural row i of the face lies in the plane's data rows [n1lo, n1lo + nrows) (mod 90).
__device__ __forceinline__ bool row_in(int i, int n1lo, int nrows) {
    int d = i - n1lo;
    d += d < 0 ? N : 0;
    d -= d >= N ? N : 0;
    return d < nrows;
}
__device__ __forceinline__ int row_at(int f, int n1lo) {
    int r = n1lo + f;
    r += r < 0 ? N : 0;
    r -= r >= N ? N : 0;
    return r;
}

// Full 90 x 90 face, y then z, in the 9 x 10 steps: y step A reads natural
// element i = row * 90 + col through ld(i), the rows end permuted (natural
// row i at LDS row slot(i)), z runs over every LDS row and leaves the slots
// permuted, and st(i, v) receives natural element i (a coalesced copy out).
template <typename T, int SIGN, typename Ld, typename St>
__device__ __forceinline__ void face(typename cx<T>::t* lds, const double2* ty64, const float2* ty32,
                                     const double2* tz64, const float2* tz32, Ld ld, St st) {
    using Cx = typename cx<T>::t;
    const int t = threadIdx.x;
    if (t < 10 * N) {
        const int n1 = t / N, c = t - N * n1;
        Cx v[9];
#pragma unroll
        for (int j = 0; j < 9; ++j) v[j] = ld((n1 + 10 * j) * N + c);
        step_a<T, SIGN>(v, n1, ty64, ty32);
#pragma unroll
        for (int j = 0; j < 9; ++j) lds[(n1 + 10 * j) * N + c] = v[j];
    }
    __syncthreads();
    if (t < 9 * N) {
        const int k2 = t / N, c = t - N * k2;
        Cx u[10];
#pragma unroll
        for (int j = 0; j < 10; ++j) u[j] = lds[(j + 10 * k2) * N + c];
        dft10<T, SIGN>(u);
#pragma unroll
        for (int j = 0; j < 10; ++j) lds[(j + 10 * k2) * N + c] = u[j];
    }
    __syncthreads();
    if (t < 10 * N) {
        const int r = t / 10, n1 = t - 10 * r;
        Cx* row = lds + r * N;
        Cx v[9];
#pragma unroll
        for (int j = 0; j < 9; ++j) v[j] = row[n1 + 10 * j];
        step_a<T, SIGN>(v, n1, tz64, tz32);
#pragma unroll
        for (int j = 0; j < 9; ++j) row[n1 + 10 * j] = v[j];
    }
    __syncthreads();
    if (t < 9 * N) {
        const int r = t / 9, k2 = t - 9 * r;
        Cx* row = lds + r * N + 10 * k2;
        Cx u[10];
#pragma unroll
        for (int j = 0; j < 10; ++j) u[j] = row[j];
        dft10<T, SIGN>(u);
#pragma unroll
        for (int j = 0; j < 10; ++j) row[j] = u[j];
    }
    __syncthreads();
    for (int i = t; i < N * N; i += NT) {
        const int i1 = i / N;
        st(i, lds[slot(i1) * N + slot(i - N * i1)]);
    }
}
}  // namespace p90

// ------------------------------------------------------------- pass 1 ------
// Sphere coefficients -> inverse transform along z and y -> plane buffer.
template <typename T, typename TIO, int NT, bool BATCH = false>
__global__ void __launch_bounds__(NT)
k_planes_from_sphere(const FftItem* items, FftItem single, const TIO* __restrict__ C,
                     typename cx<T>::t* __restrict__ Tb, const int* __restrict__ act,
                     const int* __restrict__ idx) {
    using Cx = typename cx<T>::t;
    const int item = (BATCH && idx) ? idx[blockIdx.z] : (int)blockIdx.z;
    if (BATCH && act && !act[item]) return;
    const FftItem& it = BATCH ? items[item] : single;
    const int p = blockIdx.x, b = blockIdx.y;
    if (p >= it.nplanes || b >= it.nb) return;
    extern __shared__ char smem_raw[];
    Cx* lds = reinterpret_cast<Cx*>(smem_raw);
    const int S1 = it.S1, S2 = it.S2, np = S1 * S2;
    for (int i = threadIdx.x; i < np; i += blockDim.x) lds[i] = Cx{0, 0};
    const int4 pl = it.planes[p];
    __syncthreads();
    const TIO* src = C + it.c_off + (int64_t)b * it.ld + pl.x;
    const int* poff = it.poff + pl.x;
    for (int q = threadIdx.x; q < pl.y; q += blockDim.x) lds[poff[q]] = Io<T>::from(src[q]);
    __syncthreads();
    fft_axis<T, false, NT>(lds, it.ax[2], pl.w, AddrRowsWrap{S2, pl.z, S1}, it.tw64[2], it.tw32[2], +1);
    fft_axis<T, true, NT>(lds, it.ax[1], S2, AddrLinear{1, S2}, it.tw64[1], it.tw32[1], +1);
    Cx* dst = Tb + it.t_off + ((int64_t)b * it.nplanes + p) * np;
    for (int i = threadIdx.x; i < np; i += blockDim.x) dst[i] = lds[i];
}

// Full-box field plane i0 -> 2D transform (sign) -> plane buffer.
// REAL_IN: input is real (double), else complex (double2).
// Batched (one item per cell, blockIdx.z): the field sits at v_off, the
// planes at t_off.
template <typename T, bool REAL_IN, int NT, bool BATCH = false>
__global__ void __launch_bounds__(NT)
k_planes_from_box(const FftItem* items, FftItem single, const void* __restrict__ in, int64_t field_stride,
                  int sign, typename cx<T>::t* __restrict__ Tb) {
    using Cx = typename cx<T>::t;
    const FftItem& it = DPP_ITEM(items, single);
    const int p = blockIdx.x, f = blockIdx.y;
    if (p >= it.S0) return;
    extern __shared__ char smem_raw[];
    Cx* lds = reinterpret_cast<Cx*>(smem_raw);
    const int S1 = it.S1, S2 = it.S2, np = S1 * S2;
    const int64_t base = it.v_off + (int64_t)f * field_stride + (int64_t)p * np;
    if constexpr (NT == p90::NT) {
        if (S1 == p90::N && S2 == p90::N) {  // 90 x 90 face: the 9 x 10 steps
            Cx* dst = Tb + it.t_off + (int64_t)f * it.S0 * np + (int64_t)p * np;
            auto ld = [&](int i) {
                if (REAL_IN) return Cx{(T)(reinterpret_cast<const double*>(in) + base)[i], (T)0};
                return Io<T>::from((reinterpret_cast<const double2*>(in) + base)[i]);
            };
            auto st = [&](int i, Cx v) { dst[i] = v; };
            if (sign > 0)
                p90::face<T, +1>(lds, it.tw64[1], it.tw32[1], it.tw64[2], it.tw32[2], ld, st);
            else
                p90::face<T, -1>(lds, it.tw64[1], it.tw32[1], it.tw64[2], it.tw32[2], ld, st);
            return;
        }
    }
    if (REAL_IN) {
        const double* src = reinterpret_cast<const double*>(in) + base;
        for (int i = threadIdx.x; i < np; i += blockDim.x) lds[i] = Cx{(T)src[i], (T)0};
    } else {
        const double2* src = reinterpret_cast<const double2*>(in) + base;
        for (int i = threadIdx.x; i < np; i += blockDim.x) lds[i] = Io<T>::from(src[i]);
    }
    __syncthreads();
    fft_axis<T, false, NT>(lds, it.ax[2], S1, AddrLinear{S2, 1}, it.tw64[2], it.tw32[2], sign);
    fft_axis<T, true, NT>(lds, it.ax[1], S2, AddrLinear{1, S2}, it.tw64[1], it.tw32[1], sign);
    Cx* dst = Tb + it.t_off + (int64_t)f * it.S0 * np + (int64_t)p * np;
    for (int i = threadIdx.x; i < np; i += blockDim.x) dst[i] = lds[i];
}

// ------------------------------------------------------------- pass 2 ------
enum XzMode { XZ_H = 0, XZ_TO_BOX = 1, XZ_FROM_BOX = 2 };

__device__ __forceinline__ int wrap(int n, int S) { return n < 0 ? n + S : n; }

// Load the pruned rows of x-z plane (band b, i1) from the plane buffer into
// LDS rows i0 = (n0min + p) mod S0, zeroing the rows without data.
template <typename T>
__device__ __forceinline__ void xz_load_pruned(const FftItem& it, const typename cx<T>::t* Tb,
                                               int b, int i1, typename cx<T>::t* lds) {
    using Cx = typename cx<T>::t;
    const int S0 = it.S0, S1 = it.S1, S2 = it.S2;
    const int np = S1 * S2;
    const int nP = it.nplanes;
    // zero the rows whose Miller index lies outside [n0min, n0min + nplanes)
    for (int i = threadIdx.x; i < S0 * S2; i += blockDim.x) {
        const int i0 = i / S2;
        int d = (i0 - it.n0min) % S0;
        d += d < 0 ? S0 : 0;
        if (d >= nP) lds[i] = Cx{0, 0};
    }
    const Cx* src = Tb + it.t_off + (int64_t)b * nP * np + (int64_t)i1 * S2;
    for (int i = threadIdx.x; i < nP * S2; i += blockDim.x) {
        const int p = i / S2, i2 = i - p * S2;
        const int i0 = wrap(it.n0min + p, S0);
        lds[i0 * S2 + i2] = src[(int64_t)p * np + i2];
    }
}

template <typename T>
__device__ __forceinline__ void xz_store_pruned(const FftItem& it, typename cx<T>::t* Tb, int b,
                                                int i1, const typename cx<T>::t* lds) {
    using Cx = typename cx<T>::t;
    const int S0 = it.S0, S1 = it.S1, S2 = it.S2;
    const int np = S1 * S2;
    const int nP = it.nplanes;
    Cx* dst = Tb + it.t_off + (int64_t)b * nP * np + (int64_t)i1 * S2;
    for (int i = threadIdx.x; i < nP * S2; i += blockDim.x) {
        const int p = i / S2, i2 = i - p * S2;
        const int i0 = wrap(it.n0min + p, S0);
        dst[(int64_t)p * np + i2] = lds[i0 * S2 + i2];
    }
}

template <typename T, int MODE, typename TIO, int NT, bool BATCH = false>
__global__ void __launch_bounds__(NT)
k_xz(const FftItem* items, FftItem single, typename cx<T>::t* __restrict__ Tb,
     const double* __restrict__ V, TIO* __restrict__ box, const int* __restrict__ act,
     const int* __restrict__ idx = nullptr) {
    using Cx = typename cx<T>::t;
    const int item = (BATCH && idx) ? idx[blockIdx.z] : (int)blockIdx.z;
    if (BATCH && act && !act[item]) return;
    const FftItem& it = BATCH ? items[item] : single;
    const int i1 = blockIdx.x, b = blockIdx.y;
    if (i1 >= it.S1 || b >= it.nb) return;
    extern __shared__ char smem_raw[];
    Cx* lds = reinterpret_cast<Cx*>(smem_raw);
    const int S0 = it.S0, S1 = it.S1, S2 = it.S2;
    const int e = S0 * S2;
    const int64_t N = (int64_t)S0 * S1 * S2;
    if (MODE == XZ_FROM_BOX) {
        const TIO* src = box + (int64_t)b * N + (int64_t)i1 * S2;
        for (int i = threadIdx.x; i < e; i += blockDim.x) {
            const int i0 = i / S2, i2 = i - i0 * S2;
            lds[i] = Io<T>::from(src[(int64_t)i0 * S1 * S2 + i2]);
        }
        __syncthreads();
        fft_axis<T, true, NT>(lds, it.ax[0], S2, AddrLinear{1, S2}, it.tw64[0], it.tw32[0], -1);
        xz_store_pruned<T>(it, Tb, b, i1, lds);
        return;
    }
    xz_load_pruned<T>(it, Tb, b, i1, lds);
    __syncthreads();
    fft_axis<T, true, NT>(lds, it.ax[0], S2, AddrLinear{1, S2}, it.tw64[0], it.tw32[0], +1);
    if (MODE == XZ_TO_BOX) {
        TIO* dst = box + (int64_t)b * N + (int64_t)i1 * S2;
        for (int i = threadIdx.x; i < e; i += blockDim.x) {
            const int i0 = i / S2, i2 = i - i0 * S2;
            dst[(int64_t)i0 * S1 * S2 + i2] = store_as<TIO>(lds[i]);
        }
        return;
    }
    // XZ_H: pointwise (Omega/N) V_eff at the natural (i1, i2) of the row
    const int n1 = it.vperm && it.perm ? digit_rev_axis(it.ax[1], i1) : i1;
    const double* Vp = V + it.v_off + (int64_t)n1 * S2;
    const T sc = (T)(it.vperm ? it.vscale : 1.0);
    for (int i = threadIdx.x; i < e; i += blockDim.x) {
        const int i0 = i / S2, i2 = i - i0 * S2;
        const int n2 = it.vperm && it.perm ? digit_rev_axis(it.ax[2], i2) : i2;
        const T v = (T)Vp[(int64_t)i0 * S1 * S2 + n2] * sc;
        lds[i] = Cx{lds[i].x * v, lds[i].y * v};
    }
    __syncthreads();
    fft_axis<T, true, NT>(lds, it.ax[0], S2, AddrLinear{1, S2}, it.tw64[0], it.tw32[0], -1);
    xz_store_pruned<T>(it, Tb, b, i1, lds);
}

// Register plane passes for square y-z faces (S1 = S2 = N): one wave per
// (item, band, plane), or per two planes when N <= 32 (lanes 0-31 and 32-63
// each take one, so fewer lanes idle).  Sphere -> planes: lane r < N owns natural row i1 = r,
// gathers the row's sphere points into registers (each register is one z
// point), transforms along z (decimation in frequency), and writes the row to
// LDS; lane c then owns column c (a digit-reversed z point), transforms along
// y and stores the column, so the plane holds (y, z) in digit-reversed order.
// Planes -> sphere runs the same steps backwards with decimation in time and
// gathers the points with the kinetic term.  One LDS exchange per plane.
template <typename T, int N>
__global__ void __launch_bounds__(64)
k_planes_from_sphere_reg(const FftItem* __restrict__ items, const int* __restrict__ idx,
                         const double2* __restrict__ C, typename cx<T>::t* __restrict__ Tb,
                         const int* __restrict__ act) {
    using Cx = typename cx<T>::t;
    const int item = idx ? idx[blockIdx.z] : (int)blockIdx.z;
    if (act && !act[item]) return;
    const FftItem& it = items[item];
    // faces of up to 32 points: two planes per wave (lanes 0-31 and 32-63)
    constexpr int PPW = N <= 32 ? 2 : 1;
    const int sub = PPW == 2 ? (int)(threadIdx.x >> 5) : 0;
    const int lane = PPW == 2 ? (int)(threadIdx.x & 31) : (int)threadIdx.x;
    const int p = blockIdx.x * PPW + sub, b = blockIdx.y;
    if ((int)blockIdx.x * PPW >= it.nplanes || b >= it.nb) return;  // uniform
    const bool on = p < it.nplanes && lane < N;
    __shared__ Cx ldsb[PPW][N * (N + 1)];
    Cx* lds = ldsb[sub];
    if (on) {
        const int4 rw = it.rows[p * N + lane];
        const double2* src = C + it.c_off + (int64_t)b * it.ld + rw.x;
        Cx x[N];
#pragma unroll
        for (int r2 = 0; r2 < N; ++r2) {
            const int n2 = 2 * r2 < N ? r2 : r2 - N;
            const int q = n2 - rw.z;
            x[r2] = (q >= 0 && q < rw.y) ? Io<T>::from(src[q]) : Cx{0, 0};
        }
        if (rw.y > 0) reg_dif<T, N, +1, 0>(x, it.tw64[2], it.tw32[2]);
#pragma unroll
        for (int c = 0; c < N; ++c) lds[lane * (N + 1) + c] = x[c];
    }
    __syncthreads();
    if (on) {
        Cx x[N];
#pragma unroll
        for (int r = 0; r < N; ++r) x[r] = lds[r * (N + 1) + lane];
        reg_dif<T, N, +1, 0>(x, it.tw64[1], it.tw32[1]);
        Cx* dst = Tb + it.t_off + ((int64_t)b * it.nplanes + p) * (N * N) + lane;
#pragma unroll
        for (int r = 0; r < N; ++r) dst[r * N] = x[r];
    }
}

template <typename T, int N>
__global__ void __launch_bounds__(64)
k_planes_to_sphere_reg(const FftItem* __restrict__ items, const int* __restrict__ idx,
                       const typename cx<T>::t* __restrict__ Tb, const double2* __restrict__ Cin,
                       double2* __restrict__ out, const int* __restrict__ act) {
    using Cx = typename cx<T>::t;
    const int item = idx ? idx[blockIdx.z] : (int)blockIdx.z;
    if (act && !act[item]) return;
    const FftItem& it = items[item];
    constexpr int PPW = N <= 32 ? 2 : 1;
    const int sub = PPW == 2 ? (int)(threadIdx.x >> 5) : 0;
    const int lane = PPW == 2 ? (int)(threadIdx.x & 31) : (int)threadIdx.x;
    const int p = blockIdx.x * PPW + sub, b = blockIdx.y;
    if ((int)blockIdx.x * PPW >= it.nplanes || b >= it.nb) return;  // uniform
    const bool on = p < it.nplanes && lane < N;
    __shared__ Cx ldsb[PPW][N * (N + 1)];
    Cx* lds = ldsb[sub];
    if (on) {
        const Cx* src = Tb + it.t_off + ((int64_t)b * it.nplanes + p) * (N * N) + lane;
        Cx x[N];
#pragma unroll
        for (int r = 0; r < N; ++r) x[r] = src[r * N];
        reg_dit<T, N, -1, 0>(x, it.tw64[1], it.tw32[1]);
#pragma unroll
        for (int r = 0; r < N; ++r) lds[r * (N + 1) + lane] = x[r];
    }
    __syncthreads();
    if (on) {
        const int4 rw = it.rows[p * N + lane];
        if (rw.y > 0) {
            Cx* row = lds + lane * (N + 1);
            {
                Cx x[N];
#pragma unroll
                for (int c = 0; c < N; ++c) x[c] = row[c];
                reg_dit<T, N, -1, 0>(x, it.tw64[2], it.tw32[2]);
                // back to the lane's own LDS row, so the gather below holds
                // only a few points in registers at a time
#pragma unroll
                for (int c = 0; c < N; ++c) row[c] = x[c];
            }
            const int64_t o = it.c_off + (int64_t)b * it.ld + rw.x;
            const double* kG2 = it.kG2 + rw.x;
            const double hk = 0.5 * it.omega;
            // the row's points are contiguous in the sphere: q = 0 .. rw.y - 1
            // at z index n2 = rw.z + q
            for (int q0 = 0; q0 < rw.y; q0 += 8) {
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    const int q = q0 + u;
                    if (q < rw.y) {
                        const int n2 = rw.z + q;
                        const double2 c = Cin[o + q];
                        const double2 v = Io<T>::to_d(row[n2 < 0 ? n2 + N : n2]);
                        const double t = hk * kG2[q];
                        out[o + q] = double2{t * c.x + v.x, t * c.y + v.y};
                    }
                }
            }
        }
    }
}

// Register plane pass lengths (FP64 registers of a column: 2N).
constexpr bool plane_reg_len(int n) {
    return n == 12 || n == 15 || n == 16 || n == 18 || n == 20 || n == 24 || n == 25 || n == 27 || n == 30 ||
           n == 32 || n == 36 || n == 40 || n == 45;
}

template <typename T, int N>
static void planes_reg_launch_one(bool to_sphere, dim3 grid, hipStream_t st, const FftItem* items, const int* idx,
                                  const double2* X, typename cx<T>::t* Tb, double2* HX, const int* act) {
    constexpr int PPW = N <= 32 ? 2 : 1;  // planes per wave (kernels above)
    grid.x = (grid.x + PPW - 1) / PPW;
    if (to_sphere)
        hipLaunchKernelGGL((k_planes_to_sphere_reg<T, N>), grid, dim3(64), 0, st, items, idx,
                           (const typename cx<T>::t*)Tb, X, HX, act);
    else
        hipLaunchKernelGGL((k_planes_from_sphere_reg<T, N>), grid, dim3(64), 0, st, items, idx, X, Tb, act);
}

template <typename T>
static bool planes_reg_launch(int N, bool to_sphere, dim3 grid, hipStream_t st, const FftItem* items,
                              const int* idx, const double2* X, typename cx<T>::t* Tb, double2* HX,
                              const int* act) {
    switch (N) {
#define DPP_PL_REG(n)                                                                      \
    case n:                                                                                \
        planes_reg_launch_one<T, n>(to_sphere, grid, st, items, idx, X, Tb, HX, act);      \
        return true;
        DPP_PL_REG(12) DPP_PL_REG(15) DPP_PL_REG(16) DPP_PL_REG(18) DPP_PL_REG(20) DPP_PL_REG(24)
        DPP_PL_REG(25) DPP_PL_REG(27) DPP_PL_REG(30) DPP_PL_REG(32) DPP_PL_REG(36) DPP_PL_REG(40)
        DPP_PL_REG(45)
#undef DPP_PL_REG
        default:
            return false;
    }
}

// Register-resident x pass of H: one thread per (item, band, i1, i2) column.
// Gather the pruned rows into registers (zeros elsewhere), inverse transform
// along x (decimation in frequency: register p then holds x point
// digit_rev(p)), multiply by (Omega/N) V_eff there, transform back
// (decimation in time: natural order again), store the pruned rows.  No LDS,
// no barriers; every load and store is coalesced across the i2 of a wave.
template <typename T, int S0>
__global__ void __launch_bounds__(256)
k_xz_reg(const FftItem* __restrict__ items, const int* __restrict__ idx, typename cx<T>::t* __restrict__ Tb,
         const double* __restrict__ V, const int* __restrict__ act) {
    using Cx = typename cx<T>::t;
    const int item = idx ? idx[blockIdx.z] : (int)blockIdx.z;
    if (act && !act[item]) return;
    const FftItem& it = items[item];
    const int b = blockIdx.y;
    if (b >= it.nb) return;
    const int np = it.S1 * it.S2;
    const int col = blockIdx.x * 256 + threadIdx.x;
    if (col >= np) return;
    const int nP = it.nplanes;
    Cx* base = Tb + it.t_off + (int64_t)b * nP * np + col;
    Cx x[S0];
#pragma unroll
    for (int i0 = 0; i0 < S0; ++i0) {
        int d = (i0 - it.n0min) % S0;
        d += d < 0 ? S0 : 0;
        x[i0] = d < nP ? base[(int64_t)d * np] : Cx{0, 0};
    }
    const double2* tw64 = it.tw64[0];
    const float2* tw32 = it.tw32[0];
    reg_dif<T, S0, +1, 0>(x, tw64, tw32);
    // natural (i1, i2) of this column (planes may be stored digit-reversed)
    int vcol = col;
    if (it.vperm && it.perm) {
        const int p1 = col / it.S2, p2 = col - p1 * it.S2;
        vcol = digit_rev_axis(it.ax[1], p1) * it.S2 + digit_rev_axis(it.ax[2], p2);
    }
    const double* Vp = V + it.v_off + vcol;
    const T sc = (T)(it.vperm ? it.vscale : 1.0);
#pragma unroll
    for (int p = 0; p < S0; ++p) {
        const int k = reg_digit_rev(S0, p);
        const T v = (T)Vp[(int64_t)k * np] * sc;
        x[p] = Cx{x[p].x * v, x[p].y * v};
    }
    reg_dit<T, S0, -1, 0>(x, tw64, tw32);
#pragma unroll
    for (int i0 = 0; i0 < S0; ++i0) {
        int d = (i0 - it.n0min) % S0;
        d += d < 0 ? S0 : 0;
        if (d < nP) base[(int64_t)d * np] = x[i0];
    }
}

// v, hidden from the optimizer (addresses derived from it are computed where
// they are used instead of being kept live from earlier uses).
__device__ __forceinline__ int xz_opaque(int v) {
    asm volatile("" : "+v"(v));
    return v;
}

// Half-lengths whose register transforms run one butterfly at a time.
constexpr bool XZ2_SER(int m) { return m > 32; }
// Points per group of potential loads.
constexpr int XZ2_VG = 9;

// Buffer resources (raw, stride 0): word 3 of the descriptor for gfx9-family
// devices, and an offset beyond any buffer here (loads there return 0,
// stores there are dropped).
constexpr int XZ2_RSRC_WORD3 = 0x00020000;
constexpr unsigned XZ2_OUT_OF_RANGE = 0x80000000u;

template <typename C>
__device__ __forceinline__ C xz_buf_load(__amdgpu_buffer_rsrc_t r, unsigned off);
template <>
__device__ __forceinline__ double2 xz_buf_load<double2>(__amdgpu_buffer_rsrc_t r, unsigned off) {
    typedef double dv2 __attribute__((ext_vector_type(2)));
    const dv2 v = __builtin_bit_cast(dv2, __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, 0));
    return double2{v.x, v.y};
}
template <>
__device__ __forceinline__ float2 xz_buf_load<float2>(__amdgpu_buffer_rsrc_t r, unsigned off) {
    typedef float fv2 __attribute__((ext_vector_type(2)));
    const fv2 v = __builtin_bit_cast(fv2, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0));
    return float2{v.x, v.y};
}
template <typename C>
__device__ __forceinline__ void xz_buf_store(__amdgpu_buffer_rsrc_t r, unsigned off, C v);
template <>
__device__ __forceinline__ void xz_buf_store<double2>(__amdgpu_buffer_rsrc_t r, unsigned off, double2 v) {
    typedef double dv2 __attribute__((ext_vector_type(2)));
    typedef unsigned u4 __attribute__((ext_vector_type(4)));
    __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u4, dv2{v.x, v.y}), r, off, 0, 0);
}
template <>
__device__ __forceinline__ void xz_buf_store<float2>(__amdgpu_buffer_rsrc_t r, unsigned off, float2 v) {
    typedef float fv2 __attribute__((ext_vector_type(2)));
    typedef unsigned u2 __attribute__((ext_vector_type(2)));
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u2, fv2{v.x, v.y}), r, off, 0, 0);
}

// Value of the other lane of an adjacent pair (lane ^ 1) by a DPP quad
// permutation [1, 0, 3, 2].
__device__ __forceinline__ float pair_swap(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0xB1, 0xF, 0xF, false));
}
__device__ __forceinline__ double pair_swap(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)b, 0xB1, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), 0xB1, 0xF, 0xF, false);
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// The same x pass with each column split over a lane pair (half h holds
// points j + h S0/2, j < S0/2), for half the registers per thread.  With
// M = S0/2 and w = exp(+-2 pi i / S0) the forward transform starts with a
// radix-2 step across the pair: half h forms y_h[j] = (x[j] + (-1)^h
// x[j+M]) w^{h j}, whose M-point transform gives the points 2k + h; the
// inverse ends with the matching step, out[j + h M] = z_0[j] + (-1)^h
// w^{-j} z_1[j].  Everything between stays in the thread's registers.
template <typename T, int S0>
// Two waves per SIMD: the FP64 90-point form needs 266 registers without the
// hint (one wave per SIMD) and 256 plus a 24-byte spill with it, which runs
// faster (386 vs 517 us per config-3 H); every other length fits two waves
// without it.
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2)))
k_xz_reg2(const FftItem* __restrict__ items, const int* __restrict__ idx, typename cx<T>::t* __restrict__ Tb,
          const double* __restrict__ V, const int* __restrict__ act) {
    using Cx = typename cx<T>::t;
    constexpr int M = S0 / 2;
    const int item = idx ? idx[blockIdx.z] : (int)blockIdx.z;
    if (act && !act[item]) return;
    const FftItem& it = items[item];
    // workgroups in dispatch order take the bands of one column tile first,
    // so the tile's V (90 KB at S0 = 90) is reused from L2 across bands
    const int lin = blockIdx.x + gridDim.x * blockIdx.y;
    const int b = lin % gridDim.y;
    if (b >= it.nb) return;
    const int np = it.S1 * it.S2;
    const int col = (lin / gridDim.y) * 128 + (threadIdx.x >> 1);
    const int h = threadIdx.x & 1;
    if (col >= np) return;  // both lanes of a pair leave together
    const int nP = it.nplanes;
    // this band's planes as a buffer: points on planes the sphere does not
    // touch get an offset past the end, where the hardware range check makes
    // loads return 0 and drops stores (no branch per point)
    const auto planes = __builtin_amdgcn_make_buffer_rsrc(Tb + it.t_off + (int64_t)b * nP * np, (short)0,
                                                          (int)(nP * np * (int)sizeof(Cx)), XZ2_RSRC_WORD3);
    // plane of point j + h M: d = (j + h M - n0min) mod S0, stepped from d0
    int d0 = (h * M - it.n0min) % S0;
    d0 += d0 < 0 ? S0 : 0;
    auto plane_off = [&](int j, int dstart, int c) -> unsigned {
        int d = dstart + j;
        d -= d >= S0 ? S0 : 0;
        return d < nP ? (unsigned)((c + d * np) * (int)sizeof(Cx)) : XZ2_OUT_OF_RANGE;
    };
    Cx x[M];
#pragma unroll
    for (int j = 0; j < M; ++j) x[j] = xz_buf_load<Cx>(planes, plane_off(j, d0, col));
#pragma unroll
    for (int j = 0; j < M; ++j) {
        const Cx o = Cx{pair_swap(x[j].x), pair_swap(x[j].y)};
        if (h == 0) {
            x[j] = Cx{x[j].x + o.x, x[j].y + o.y};
        } else {
            const Cx dlt = Cx{o.x - x[j].x, o.y - x[j].y};
            x[j] = j == 0 ? dlt : cmul(dlt, reg_twiddle<T, S0>(j, +1));
        }
    }
    reg_dif<T, M, +1, 0, XZ2_SER(M)>(x, nullptr, nullptr);
    int vcol = col;
    if (it.vperm && it.perm) {
        const int p1 = col / it.S2, p2 = col - p1 * it.S2;
        vcol = digit_rev_axis(it.ax[1], p1) * it.S2 + digit_rev_axis(it.ax[2], p2);
    }
    // V of the item's box as a buffer (32-bit offsets from a uniform base)
    const auto vbuf = __builtin_amdgcn_make_buffer_rsrc(const_cast<double*>(V + it.v_off), (short)0,
                                                        (int)(S0 * np * (int)sizeof(double)), XZ2_RSRC_WORD3);
    const int vbase = vcol + h * np;
    const T sc = (T)(it.vperm ? it.vscale : 1.0);
    // in groups of XZ2_VG points, so that not every load is in flight at once
#pragma unroll
    for (int p0 = 0; p0 < M; p0 += XZ2_VG) {
#pragma unroll
        for (int p = p0; p < (p0 + XZ2_VG < M ? p0 + XZ2_VG : M); ++p) {
            const int k = 2 * reg_digit_rev(M, p);
            const T v = (T)__builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(
                                                          vbuf, (unsigned)((vbase + k * np) * 8), 0, 0)) *
                        sc;
            x[p] = Cx{x[p].x * v, x[p].y * v};
        }
        if constexpr (M > XZ2_VG) __builtin_amdgcn_sched_barrier(0);
    }
    reg_dit<T, M, -1, 0, XZ2_SER(M)>(x, nullptr, nullptr);
#pragma unroll
    for (int j = 0; j < M; ++j) {
        const Cx t = (h == 0 || j == 0) ? x[j] : cmul(x[j], reg_twiddle<T, S0>(j, -1));
        const Cx o = Cx{pair_swap(t.x), pair_swap(t.y)};
        x[j] = h == 0 ? Cx{t.x + o.x, t.y + o.y} : Cx{o.x - t.x, o.y - t.y};
    }
    // offsets recomputed here (from opaque values), not kept live since the loads
    const int d0s = xz_opaque(d0), cols = xz_opaque(col);
#pragma unroll
    for (int j = 0; j < M; ++j) xz_buf_store<Cx>(planes, plane_off(j, d0s, cols), x[j]);
}

template <typename T, int N>
static void xz_reg2_one(dim3 grid, hipStream_t st, const FftItem* items, const int* idx, typename cx<T>::t* Tb,
                        const double* V, const int* act) {
    grid.x = (grid.x * 256 + 127) / 128;
    hipLaunchKernelGGL((k_xz_reg2<T, N>), grid, dim3(256), 0, st, items, idx, Tb, V, act);
}

// Register x pass lengths: one thread per column needs FP64 lengths up to 45
// (FP32: 64); the lane-pair split takes even lengths (up to 90).  XZ_AUTO:
// the split from 24 (FP64) or 36 (FP32) points, where one thread per column
// runs at low occupancy.
template <typename T, int N>
constexpr bool xz_has(int v) {
    const bool reg1 = !(sizeof(T) == 8 && N > 45);
    const bool reg2 = N % 2 == 0;
    return v == XZ_REG1 ? reg1 : v == XZ_REG2 ? reg2 : false;
}
template <typename T, int N>
constexpr int xz_auto() {
    if (N % 2 == 0 && N >= (sizeof(T) == 8 ? 24 : 36)) return XZ_REG2;
    return xz_has<T, N>(XZ_REG1) ? XZ_REG1 : XZ_LDS;
}

template <typename T, int N>
static bool xz_reg_one(dim3 grid, hipStream_t st, const FftItem* items, const int* idx, typename cx<T>::t* Tb,
                       const double* V, const int* act, int variant) {
    const int v = variant == XZ_AUTO ? xz_auto<T, N>() : variant;
    if (v == XZ_REG2 && xz_has<T, N>(XZ_REG2)) {
        if constexpr (N % 2 == 0) xz_reg2_one<T, N>(grid, st, items, idx, Tb, V, act);
        return true;
    }
    if (v == XZ_REG1 && xz_has<T, N>(XZ_REG1)) {
        if constexpr (!(sizeof(T) == 8 && N > 45))
            hipLaunchKernelGGL((k_xz_reg<T, N>), grid, dim3(256), 0, st, items, idx, Tb, V, act);
        return true;
    }
    return false;
}

// Launch the register x pass for one S0 group; false if S0 is not compiled in
// for this precision (the caller then uses the LDS pass).
template <typename T>
static bool xz_reg_launch(int S0, dim3 grid, hipStream_t st, const FftItem* items, const int* idx,
                          typename cx<T>::t* Tb, const double* V, const int* act, int variant) {
    switch (S0) {
#define DPP_XZ_REG(n) \
    case n:           \
        return xz_reg_one<T, n>(grid, st, items, idx, Tb, V, act, variant);
        DPP_XZ_REG(12) DPP_XZ_REG(15) DPP_XZ_REG(16) DPP_XZ_REG(18) DPP_XZ_REG(20) DPP_XZ_REG(24)
        DPP_XZ_REG(25) DPP_XZ_REG(27) DPP_XZ_REG(30) DPP_XZ_REG(32) DPP_XZ_REG(36) DPP_XZ_REG(40)
        DPP_XZ_REG(45) DPP_XZ_REG(48) DPP_XZ_REG(50) DPP_XZ_REG(54) DPP_XZ_REG(60) DPP_XZ_REG(64)
        DPP_XZ_REG(90)
#undef DPP_XZ_REG
        default:
            return false;
    }
}

template <typename T>
static bool xz_available_t(int S0, int v) {
    switch (S0) {
#define DPP_XZ_AV(n) \
    case n:          \
        return v == XZ_LDS || v == XZ_AUTO || xz_has<T, n>(v);
        DPP_XZ_AV(12) DPP_XZ_AV(15) DPP_XZ_AV(16) DPP_XZ_AV(18) DPP_XZ_AV(20) DPP_XZ_AV(24)
        DPP_XZ_AV(25) DPP_XZ_AV(27) DPP_XZ_AV(30) DPP_XZ_AV(32) DPP_XZ_AV(36) DPP_XZ_AV(40)
        DPP_XZ_AV(45) DPP_XZ_AV(48) DPP_XZ_AV(50) DPP_XZ_AV(54) DPP_XZ_AV(60) DPP_XZ_AV(64)
        DPP_XZ_AV(90)
#undef DPP_XZ_AV
        default:
            return v == XZ_LDS || v == XZ_AUTO;
    }
}

// Full-box x pass: plane buffer (all S0 planes) -> transform along x (sign)
// -> multiply by `scale` -> complex output box.
// x transform of one 90 x 90 (x, z) slab of a full box: step A per (column z,
// n1) straight from the plane buffer, one LDS exchange, step B per (z, k2)
// straight to the output rows 9 k1 + k2, times `scale`.
template <typename T, int SIGN>
__device__ __forceinline__ void xz_full90(const FftItem& it, const typename cx<T>::t* src, double2* dst, double scale,
                                          typename cx<T>::t* lds) {
    using Cx = typename cx<T>::t;
    using namespace p90;
    const int64_t rs = (int64_t)it.S1 * it.S2;  // x stride of the box
    const int t = threadIdx.x;
    if (t < 10 * N) {
        const int n1 = t / N, z = t - N * n1;
        Cx v[9];
#pragma unroll
        for (int j = 0; j < 9; ++j) v[j] = src[(n1 + 10 * j) * rs + z];
        step_a<T, SIGN>(v, n1, it.tw64[0], it.tw32[0]);
#pragma unroll
        for (int j = 0; j < 9; ++j) lds[(n1 + 10 * j) * N + z] = v[j];
    }
    __syncthreads();
    if (t < 9 * N) {
        const int k2 = t / N, z = t - N * k2;
        Cx u[10];
#pragma unroll
        for (int j = 0; j < 10; ++j) u[j] = lds[(j + 10 * k2) * N + z];
        dft10<T, SIGN>(u);
#pragma unroll
        for (int j = 0; j < 10; ++j)
            dst[(9 * j + k2) * rs + z] = double2{(double)u[j].x * scale, (double)u[j].y * scale};
    }
}

template <typename T, int NT>
__global__ void __launch_bounds__(NT)
k_xz_full(FftItem it, const typename cx<T>::t* __restrict__ Tb, int sign, double scale,
          double2* __restrict__ out, int64_t field_stride) {
    using Cx = typename cx<T>::t;
    const int i1 = blockIdx.x, f = blockIdx.y;
    if (i1 >= it.S1) return;
    extern __shared__ char smem_raw[];
    Cx* lds = reinterpret_cast<Cx*>(smem_raw);
    const int S0 = it.S0, S1 = it.S1, S2 = it.S2;
    const int e = S0 * S2;
    const int64_t N = (int64_t)S0 * S1 * S2;
    const Cx* src = Tb + (int64_t)f * N + (int64_t)i1 * S2;
    double2* dst = out + (int64_t)f * field_stride + (int64_t)i1 * S2;
    if constexpr (NT == p90::NT) {
        if (S0 == p90::N && S2 == p90::N) {  // 90-point x, 90 columns: the 9 x 10 steps, one LDS exchange
            if (sign > 0)
                xz_full90<T, +1>(it, src, dst, scale, lds);
            else
                xz_full90<T, -1>(it, src, dst, scale, lds);
            return;
        }
    }
    for (int i = threadIdx.x; i < e; i += blockDim.x) {
        const int i0 = i / S2, i2 = i - i0 * S2;
        lds[i] = src[(int64_t)i0 * S1 * S2 + i2];
    }
    __syncthreads();
    fft_axis<T, true, NT>(lds, it.ax[0], S2, AddrLinear{1, S2}, it.tw64[0], it.tw32[0], sign);
    for (int i = threadIdx.x; i < e; i += blockDim.x) {
        const int i0 = i / S2, i2 = i - i0 * S2;
        dst[(int64_t)i0 * S1 * S2 + i2] = double2{lds[i].x * scale, lds[i].y * scale};
    }
}

// Hartree x pass: forward x transform of the (already y,z transformed) density,
// multiply by 4 pi / (|G|^2 N^2) (the J normalization 1/N and the I scale N
// of the way back leave 4 pi / (|G|^2 N)), accumulate the energy partial
// sum_G 4 pi |n~|^2 / |G|^2 for this i1, transform back along x.  Without
// BACK only the energy partial is formed (the plane buffer is left as read).
template <int NT, bool BATCH = false, bool BACK = true>
__global__ void __launch_bounds__(NT)
k_xz_hartree(const FftItem* items, FftItem single, double2* __restrict__ Tbase, double* __restrict__ epart) {
    const FftItem& it = DPP_ITEM(items, single);
    const int i1 = blockIdx.x;
    if (i1 >= it.S1) return;
    double2* Tb = Tbase + it.t_off;
    const double B00 = it.B[0], B01 = it.B[1], B02 = it.B[2], B10 = it.B[3], B11 = it.B[4], B12 = it.B[5],
                 B20 = it.B[6], B21 = it.B[7], B22 = it.B[8];
    extern __shared__ char smem_raw[];
    double2* lds = reinterpret_cast<double2*>(smem_raw);
    __shared__ double red[NT];
    const int S0 = it.S0, S1 = it.S1, S2 = it.S2;
    const int e = S0 * S2;
    const double N = (double)S0 * S1 * S2;
    double2* src = Tb + (int64_t)i1 * S2;
    for (int i = threadIdx.x; i < e; i += blockDim.x) {
        const int i0 = i / S2, i2 = i - i0 * S2;
        lds[i] = src[(int64_t)i0 * S1 * S2 + i2];
    }
    __syncthreads();
    fft_axis<double, true, NT>(lds, it.ax[0], S2, AddrLinear{1, S2}, it.tw64[0], it.tw32[0], -1);
    const int n1 = (2 * i1 < S1) ? i1 : i1 - S1;
    double acc = 0.0;
    for (int i = threadIdx.x; i < e; i += blockDim.x) {
        const int i0 = i / S2, i2 = i - i0 * S2;
        const int n0 = (2 * i0 < S0) ? i0 : i0 - S0;
        const int n2 = (2 * i2 < S2) ? i2 : i2 - S2;
        const double gx = B00 * n0 + B01 * n1 + B02 * n2;
        const double gy = B10 * n0 + B11 * n1 + B12 * n2;
        const double gz = B20 * n0 + B21 * n1 + B22 * n2;
        const double G2 = gx * gx + gy * gy + gz * gz;
        double2 v = lds[i];
        double kern = 0.0;
        if (G2 > 0.0) kern = 4.0 * M_PI / G2;
        const double ntr = v.x / N, nti = v.y / N;
        acc += kern * (ntr * ntr + nti * nti);
        const double s = kern / N;  // V_H(G) = kern * n~ = kern * X / N; I brings no 1/N
        if (BACK) lds[i] = double2{v.x * s, v.y * s};
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) epart[it.p_off + i1] = red[0];
    if constexpr (BACK) {
        fft_axis<double, true, NT>(lds, it.ax[0], S2, AddrLinear{1, S2}, it.tw64[0], it.tw32[0], +1);
        for (int i = threadIdx.x; i < e; i += blockDim.x) {
            const int i0 = i / S2, i2 = i - i0 * S2;
            src[(int64_t)i0 * S1 * S2 + i2] = lds[i];
        }
    }
}

// Density x pass: one workgroup per (item, band chunk, i1) loops over the
// chunk's bands, transforms each along x and accumulates f_b |psi|^2 in
// registers; writes the chunk's partial (times w_k) for this i1 to box
// p_off + c N of the partial buffer (the item has dnch chunks of dchunk bands).
// accumulators per thread: every x-z tile fits (7680 elements at 512 threads, 8192 at 1024)
template <int NT>
struct DensMax {
    static constexpr int v = NT == 1024 ? 8 : NT == 512 ? 15 : 15;
};
constexpr int DENS_CHUNKS = 16;
template <typename T, int NT, bool BATCH = false>
__global__ void __launch_bounds__(NT)
k_xz_density(const FftItem* items, FftItem single, const typename cx<T>::t* __restrict__ Tb,
             const double* __restrict__ fill, double* __restrict__ part, const int* __restrict__ idx) {
    using Cx = typename cx<T>::t;
    const FftItem& it = idx ? items[idx[blockIdx.z]] : DPP_ITEM(items, single);
    const int i1 = blockIdx.x, c = blockIdx.y;
    if (i1 >= it.S1 || c >= it.dnch) return;
    const int b0 = c * it.dchunk;
    const int b1 = min(it.nb, b0 + it.dchunk);
    extern __shared__ char smem_raw[];
    Cx* lds = reinterpret_cast<Cx*>(smem_raw);
    const int S0 = it.S0, S1 = it.S1, S2 = it.S2;
    const int e = S0 * S2;
    constexpr int DM = DensMax<NT>::v;
    double acc[DM];
#pragma unroll
    for (int u = 0; u < DM; ++u) acc[u] = 0.0;
    for (int b = b0; b < b1; ++b) {
        const double fb = fill[it.f_off + b];
        if (fb == 0.0) continue;  // uniform across the workgroup
        xz_load_pruned<T>(it, Tb, b, i1, lds);
        __syncthreads();
        fft_axis<T, true, NT>(lds, it.ax[0], S2, AddrLinear{1, S2}, it.tw64[0], it.tw32[0], +1);
#pragma unroll
        for (int u = 0; u < DM; ++u) {
            const int i = threadIdx.x + u * NT;
            if (i < e) {
                const double x = (double)lds[i].x, y = (double)lds[i].y;
                acc[u] += fb * (x * x + y * y);
            }
        }
        __syncthreads();
    }
    const int64_t N = (int64_t)S0 * S1 * S2;
    const int n1 = it.perm ? digit_rev_axis(it.ax[1], i1) : i1;
    double* dst = part + it.p_off + (int64_t)c * N + (int64_t)n1 * S2;
#pragma unroll
    for (int u = 0; u < DM; ++u) {
        const int i = threadIdx.x + u * NT;
        if (i < e) {
            const int i0 = i / S2, i2 = i - i0 * S2;
            const int n2 = it.perm ? digit_rev_axis(it.ax[2], i2) : i2;
            dst[(int64_t)i0 * S1 * S2 + n2] = it.wk * acc[u];
        }
    }
}

// Sum the band-chunk partial densities in fixed order and add to n.
__global__ void k_density_reduce(const double* __restrict__ part, int nchunk, int64_t N,
                                 double* __restrict__ n) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= N) return;
    double s = 0.0;
    for (int c = 0; c < nchunk; ++c) s += part[(int64_t)c * N + j];
    n[j] += s;
}

// Per cell (blockIdx.y): n[foff + j] = sum of the cell's partial boxes in order.
__global__ void k_density_reduce_cells(const double* __restrict__ part, const CellDesc* __restrict__ cells,
                                       double* __restrict__ n) {
    const CellDesc c = cells[blockIdx.y];
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= c.N) return;
    double s = 0.0;
    for (int p = 0; p < c.nparts; ++p) s += part[c.pstart + (int64_t)p * c.N + j];
    n[c.foff + j] = s;
}

// ------------------------------------------------------------- pass 3 ------
enum GatherMode { G_SET = 0, G_ADD = 1, G_H = 2 };

template <typename T, int MODE, typename TIO, int NT, bool BATCH = false>
__global__ void __launch_bounds__(NT)
k_planes_to_sphere(const FftItem* items, FftItem single, const typename cx<T>::t* __restrict__ Tb,
                   const double2* __restrict__ Cin, TIO* __restrict__ out, int64_t ldout_override,
                   const int* __restrict__ act, const int* __restrict__ idx) {
    using Cx = typename cx<T>::t;
    const int item = (BATCH && idx) ? idx[blockIdx.z] : (int)blockIdx.z;
    if (BATCH && act && !act[item]) return;
    const FftItem& it = BATCH ? items[item] : single;
    const int p = blockIdx.x, b = blockIdx.y;
    if (p >= it.nplanes || b >= it.nb) return;
    extern __shared__ char smem_raw[];
    Cx* lds = reinterpret_cast<Cx*>(smem_raw);
    const int S1 = it.S1, S2 = it.S2, np = S1 * S2;
    const Cx* src = Tb + it.t_off + ((int64_t)b * it.nplanes + p) * np;
    for (int i = threadIdx.x; i < np; i += blockDim.x) lds[i] = src[i];
    __syncthreads();
    const int4 pl = it.planes[p];
    fft_axis<T, true, NT>(lds, it.ax[1], S2, AddrLinear{1, S2}, it.tw64[1], it.tw32[1], -1);
    fft_axis<T, false, NT>(lds, it.ax[2], pl.w, AddrRowsWrap{S2, pl.z, S1}, it.tw64[2], it.tw32[2], -1);
    const int64_t ld = ldout_override > 0 ? ldout_override : it.ld;
    TIO* dst = out + it.c_off + (int64_t)b * ld + pl.x;
    const int* poff = it.poff + pl.x;
    if (MODE == G_H) {
        const double2* cin = Cin + it.c_off + (int64_t)b * it.ld + pl.x;
        const double* kG2 = it.kG2 + pl.x;
        const double hk = 0.5 * it.omega;
        for (int q = threadIdx.x; q < pl.y; q += blockDim.x) {
            const double2 c = cin[q];
            const double2 v = Io<T>::to_d(lds[poff[q]]);
            const double t = hk * kG2[q];
            dst[q] = store_as<TIO>(double2{t * c.x + v.x, t * c.y + v.y});
        }
    } else if (MODE == G_ADD) {
        for (int q = threadIdx.x; q < pl.y; q += blockDim.x) {
            const double2 v = Io<T>::to_d(lds[poff[q]]);
            TIO o = dst[q];
            dst[q] = store_as<TIO>(double2{(double)o.x + v.x, (double)o.y + v.y});
        }
    } else {
        for (int q = threadIdx.x; q < pl.y; q += blockDim.x)
            dst[q] = store_as<TIO>(Io<T>::to_d(lds[poff[q]]));
    }
}

// Plane buffer (full box) -> 2D transform (sign) -> real part (REAL_OUT) or
// complex output box, times `scale`.
template <typename T, bool REAL_OUT, int NT, bool BATCH = false>
__global__ void __launch_bounds__(NT)
k_planes_to_box(const FftItem* items, FftItem single, const typename cx<T>::t* __restrict__ Tb, int sign,
                double scale, void* __restrict__ out, int64_t field_stride) {
    using Cx = typename cx<T>::t;
    const FftItem& it = DPP_ITEM(items, single);
    const int p = blockIdx.x, f = blockIdx.y;
    if (p >= it.S0) return;
    extern __shared__ char smem_raw[];
    Cx* lds = reinterpret_cast<Cx*>(smem_raw);
    const int S1 = it.S1, S2 = it.S2, np = S1 * S2;
    const Cx* src = Tb + it.t_off + (int64_t)f * it.S0 * np + (int64_t)p * np;
    const int64_t base = it.v_off + (int64_t)f * field_stride + (int64_t)p * np;
    if constexpr (NT == p90::NT) {
        if (S1 == p90::N && S2 == p90::N) {  // 90 x 90 face: the 9 x 10 steps
            auto ld = [&](int i) { return src[i]; };
            auto st = [&](int i, Cx v) {
                if (REAL_OUT)
                    (reinterpret_cast<double*>(out) + base)[i] = (double)v.x * scale;
                else
                    (reinterpret_cast<double2*>(out) + base)[i] = double2{(double)v.x * scale, (double)v.y * scale};
            };
            if (sign > 0)
                p90::face<T, +1>(lds, it.tw64[1], it.tw32[1], it.tw64[2], it.tw32[2], ld, st);
            else
                p90::face<T, -1>(lds, it.tw64[1], it.tw32[1], it.tw64[2], it.tw32[2], ld, st);
            return;
        }
    }
    for (int i = threadIdx.x; i < np; i += blockDim.x) lds[i] = src[i];
    __syncthreads();
    fft_axis<T, true, NT>(lds, it.ax[1], S2, AddrLinear{1, S2}, it.tw64[1], it.tw32[1], sign);
    fft_axis<T, false, NT>(lds, it.ax[2], S1, AddrLinear{S2, 1}, it.tw64[2], it.tw32[2], sign);
    if (REAL_OUT) {
        double* dst = reinterpret_cast<double*>(out) + base;
        for (int i = threadIdx.x; i < np; i += blockDim.x) dst[i] = (double)lds[i].x * scale;
    } else {
        double2* dst = reinterpret_cast<double2*>(out) + base;
        for (int i = threadIdx.x; i < np; i += blockDim.x)
            dst[i] = double2{(double)lds[i].x * scale, (double)lds[i].y * scale};
    }
}

// ------------------------------------------------ 90 x 90 plane passes ------
// Sphere -> 90 x 90 planes (sign +1): scatter, z along the data rows, y along
// every column (rows without data read as zero), natural order out.
template <typename T, typename TIO, bool BATCH = false>
__global__ void __launch_bounds__(p90::NT)
k_planes90_from_sphere(const FftItem* items, FftItem single, const TIO* __restrict__ C,
                       typename cx<T>::t* __restrict__ Tb, const int* __restrict__ act,
                       const int* __restrict__ idx) {
    using Cx = typename cx<T>::t;
    using namespace p90;
    const int item = (BATCH && idx) ? idx[blockIdx.z] : (int)blockIdx.z;
    if (BATCH && act && !act[item]) return;
    const FftItem& it = BATCH ? items[item] : single;
    const int p = blockIdx.x, b = blockIdx.y;
    if (p >= it.nplanes || b >= it.nb) return;
    extern __shared__ char smem_raw[];
    Cx* lds = reinterpret_cast<Cx*>(smem_raw);
    const int4 pl = it.planes[p];
    const int t = threadIdx.x;
    for (int i = t; i < pl.w * N; i += NT) {
        const int f = i / N;
        lds[row_at(f, pl.z) * N + (i - f * N)] = Cx{0, 0};
    }
    __syncthreads();
    const TIO* src = C + it.c_off + (int64_t)b * it.ld + pl.x;
    const int* poff = it.poff + pl.x;
    for (int q = t; q < pl.y; q += NT) lds[poff[q]] = Io<T>::from(src[q]);
    __syncthreads();
    const double2* tz64 = it.tw64[2];
    const float2* tz32 = it.tw32[2];
    if (t < pl.w * 10) {  // z, step A: task (row f, n1)
        const int f = t / 10, n1 = t - 10 * f;
        Cx* row = lds + row_at(f, pl.z) * N;
        Cx v[9];
#pragma unroll
        for (int j = 0; j < 9; ++j) v[j] = row[n1 + 10 * j];
        step_a<T, +1>(v, n1, tz64, tz32);
#pragma unroll
        for (int j = 0; j < 9; ++j) row[n1 + 10 * j] = v[j];
    }
    __syncthreads();
    if (t < pl.w * 9) {  // z, step B: task (row f, k2); the row ends permuted
        const int f = t / 9, k2 = t - 9 * f;
        Cx* row = lds + row_at(f, pl.z) * N + 10 * k2;
        Cx u[10];
#pragma unroll
        for (int j = 0; j < 10; ++j) u[j] = row[j];
        dft10<T, +1>(u);
#pragma unroll
        for (int j = 0; j < 10; ++j) row[j] = u[j];
    }
    __syncthreads();
    const double2* ty64 = it.tw64[1];
    const float2* ty32 = it.tw32[1];
    if (t < 10 * N) {  // y, step A: task (column slot c, n1)
        const int n1 = t / N, c = t - N * n1;
        Cx v[9];
#pragma unroll
        for (int j = 0; j < 9; ++j) {
            const int r = n1 + 10 * j;
            v[j] = row_in(r, pl.z, pl.w) ? lds[r * N + c] : Cx{0, 0};
        }
        step_a<T, +1>(v, n1, ty64, ty32);
#pragma unroll
        for (int j = 0; j < 9; ++j) lds[(n1 + 10 * j) * N + c] = v[j];
    }
    __syncthreads();
    if (t < 9 * N) {  // y, step B: task (natural column z, k2), straight to the plane buffer
        const int k2 = t / N, z = t - N * k2;
        const int c = slot(z);
        Cx u[10];
#pragma unroll
        for (int j = 0; j < 10; ++j) u[j] = lds[(j + 10 * k2) * N + c];
        dft10<T, +1>(u);
        Cx* dst = Tb + it.t_off + ((int64_t)b * it.nplanes + p) * (N * N) + z;
#pragma unroll
        for (int j = 0; j < 10; ++j) dst[(9 * j + k2) * N] = u[j];
    }
}

// 90 x 90 planes -> sphere (sign -1): y along every column straight from the
// plane buffer (rows end permuted), z along the data rows (slots end
// permuted), then the gather of the sphere points as in k_planes_to_sphere.
template <typename T, int MODE, typename TIO, bool BATCH = false>
__global__ void __launch_bounds__(p90::NT)
k_planes90_to_sphere(const FftItem* items, FftItem single, const typename cx<T>::t* __restrict__ Tb,
                     const double2* __restrict__ Cin, TIO* __restrict__ out, int64_t ldout_override,
                     const int* __restrict__ act, const int* __restrict__ idx) {
    using Cx = typename cx<T>::t;
    using namespace p90;
    const int item = (BATCH && idx) ? idx[blockIdx.z] : (int)blockIdx.z;
    if (BATCH && act && !act[item]) return;
    const FftItem& it = BATCH ? items[item] : single;
    const int p = blockIdx.x, b = blockIdx.y;
    if (p >= it.nplanes || b >= it.nb) return;
    extern __shared__ char smem_raw[];
    Cx* lds = reinterpret_cast<Cx*>(smem_raw);
    const int4 pl = it.planes[p];
    const int t = threadIdx.x;
    const double2* ty64 = it.tw64[1];
    const float2* ty32 = it.tw32[1];
    if (t < 10 * N) {  // y, step A: task (column c, n1), from the plane buffer
        const int n1 = t / N, c = t - N * n1;
        const Cx* src = Tb + it.t_off + ((int64_t)b * it.nplanes + p) * (N * N) + c;
        Cx v[9];
#pragma unroll
        for (int j = 0; j < 9; ++j) v[j] = src[(n1 + 10 * j) * N];
        step_a<T, -1>(v, n1, ty64, ty32);
#pragma unroll
        for (int j = 0; j < 9; ++j) lds[(n1 + 10 * j) * N + c] = v[j];
    }
    __syncthreads();
    if (t < 9 * N) {  // y, step B: task (column c, k2); natural row i at LDS row slot(i)
        const int k2 = t / N, c = t - N * k2;
        Cx u[10];
#pragma unroll
        for (int j = 0; j < 10; ++j) u[j] = lds[(j + 10 * k2) * N + c];
        dft10<T, -1>(u);
#pragma unroll
        for (int j = 0; j < 10; ++j) lds[(j + 10 * k2) * N + c] = u[j];
    }
    __syncthreads();
    const double2* tz64 = it.tw64[2];
    const float2* tz32 = it.tw32[2];
    if (t < pl.w * 10) {  // z, step A: task (data row f, n1)
        const int f = t / 10, n1 = t - 10 * f;
        Cx* row = lds + slot(row_at(f, pl.z)) * N;
        Cx v[9];
#pragma unroll
        for (int j = 0; j < 9; ++j) v[j] = row[n1 + 10 * j];
        step_a<T, -1>(v, n1, tz64, tz32);
#pragma unroll
        for (int j = 0; j < 9; ++j) row[n1 + 10 * j] = v[j];
    }
    __syncthreads();
    if (t < pl.w * 9) {  // z, step B: task (data row f, k2); natural z at slot(z)
        const int f = t / 9, k2 = t - 9 * f;
        Cx* row = lds + slot(row_at(f, pl.z)) * N + 10 * k2;
        Cx u[10];
#pragma unroll
        for (int j = 0; j < 10; ++j) u[j] = row[j];
        dft10<T, -1>(u);
#pragma unroll
        for (int j = 0; j < 10; ++j) row[j] = u[j];
    }
    __syncthreads();
    const int64_t ld = ldout_override > 0 ? ldout_override : it.ld;
    TIO* dst = out + it.c_off + (int64_t)b * ld + pl.x;
    const int* poff = it.poff + pl.x;
    for (int q = t; q < pl.y; q += NT) {
        const int o = poff[q], i1 = o / N;
        const double2 v = Io<T>::to_d(lds[slot(i1) * N + slot(o - N * i1)]);
        if (MODE == G_H) {
            const double2 c = Cin[it.c_off + (int64_t)b * it.ld + pl.x + q];
            const double tk = 0.5 * it.omega * it.kG2[pl.x + q];
            dst[q] = store_as<TIO>(double2{tk * c.x + v.x, tk * c.y + v.y});
        } else if (MODE == G_ADD) {
            const TIO w = dst[q];
            dst[q] = store_as<TIO>(double2{(double)w.x + v.x, (double)w.y + v.y});
        } else {
            dst[q] = store_as<TIO>(v);
        }
    }
}

// ----------------------------------------------------------- launchers -----
namespace {

struct Launch {
    int threads;
    size_t lds;
};

Launch plane_launch(int S1, int S2, bool fp64) {
    const int e = S1 * S2;
    return Launch{fft_threads(e), fft_lds_bytes(e, fp64)};
}
Launch xz_launch(int S0, int S2, bool fp64) {
    const int e = S0 * S2;
    return Launch{fft_threads(e), fft_lds_bytes(e, fp64)};
}

template <typename K>
dpp_status set_lds(K kernel, size_t bytes) {
    if (bytes > 64 * 1024)
        DPP_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(kernel),
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes));
    return DPP_OK;
}

// Run the statement list with NT_ bound to the workgroup size as a constant.
#define DPP_NT_DISPATCH(nt, ...)                                                         \
    switch (nt) {                                                                       \
        case 256: {                                                                     \
            constexpr int NT_ = 256;                                                    \
            __VA_ARGS__;                                                                \
            break;                                                                      \
        }                                                                               \
        case 512: {                                                                     \
            constexpr int NT_ = 512;                                                    \
            __VA_ARGS__;                                                                \
            break;                                                                      \
        }                                                                               \
        case 1024: {                                                                    \
            constexpr int NT_ = 1024;                                                   \
            __VA_ARGS__;                                                                \
            break;                                                                      \
        }                                                                               \
        default:                                                                        \
            return set_error(DPP_EUNSUPPORTED, "FFT tile too large for one workgroup"); \
    }

// Faces the 90 x 90 kernels take: square 90-point faces in natural order.
bool plane90(const FftItem& it) { return it.S1 == p90::N && it.S2 == p90::N && !it.perm && !it.full; }
size_t plane90_lds(bool fp64) { return (size_t)p90::N * p90::N * (fp64 ? 16 : 8); }

FftItem item_for(const dpp_basis_s* b, int nb, int64_t ld) {
    FftItem it = b->h_item;
    it.nb = nb;
    it.ld = ld;
    it.c_off = 0;
    it.t_off = 0;
    it.v_off = 0;
    return it;
}

}  // namespace

// Sphere -> planes (pass 1) for nb bands.
template <typename T, typename TIO>
static dpp_status pass1(dpp_ctx_s* cx_, const FftItem& it, const TIO* C, typename cx<T>::t* Tb) {
    hipStream_t st = cx_->stream;
    const double pl_ = (double)it.nplanes * it.S1 * it.S2;
    TimerScope ts_(cx_, DPP_TK_PLANES_IN, (double)it.nb * (sizeof(TIO) * (double)it.npw + sizeof(typename cx<T>::t) * pl_));
    const bool fp64 = sizeof(T) == 8;
    if (plane90(it)) {
        auto k = k_planes90_from_sphere<T, TIO>;
        DPP_TRY(set_lds(k, plane90_lds(fp64)));
        hipLaunchKernelGGL(k, dim3(it.nplanes, it.nb, 1), dim3(p90::NT), plane90_lds(fp64), st, nullptr, it, C, Tb,
                           (const int*)nullptr, (const int*)nullptr);
        DPP_LAUNCHED();
        return DPP_OK;
    }
    Launch L = plane_launch(it.S1, it.S2, fp64);
    DPP_NT_DISPATCH(L.threads, auto k = k_planes_from_sphere<T, TIO, NT_>; DPP_TRY(set_lds(k, L.lds));
                    hipLaunchKernelGGL(k, dim3(it.nplanes, it.nb, 1), dim3(NT_), L.lds, st, nullptr, it, C, Tb,
                                       (const int*)nullptr, (const int*)nullptr));
    DPP_LAUNCHED();
    return DPP_OK;
}

template <typename T, int MODE, typename TIO>
static dpp_status pass2(dpp_ctx_s* cx_, const FftItem& it, typename cx<T>::t* Tb, const double* V,
                        TIO* box) {
    hipStream_t st = cx_->stream;
    const double pl_ = (double)it.nplanes * it.S1 * it.S2, N_ = (double)it.S0 * it.S1 * it.S2;
    const double cb_ = sizeof(typename cx<T>::t);
    const double by_ = MODE == XZ_H ? it.nb * 2.0 * cb_ * pl_ + 8.0 * N_ : it.nb * (cb_ * pl_ + sizeof(TIO) * N_);
    TimerScope ts_(cx_, MODE == XZ_H ? DPP_TK_XZ_H : DPP_TK_XZ_IO, by_);
    const bool fp64 = sizeof(T) == 8;
    Launch L = xz_launch(it.S0, it.S2, fp64);
    DPP_NT_DISPATCH(L.threads, auto k = k_xz<T, MODE, TIO, NT_>; DPP_TRY(set_lds(k, L.lds));
                    hipLaunchKernelGGL(k, dim3(it.S1, it.nb, 1), dim3(NT_), L.lds, st, nullptr, it, Tb, V, box,
                                       (const int*)nullptr, (const int*)nullptr));
    DPP_LAUNCHED();
    return DPP_OK;
}

template <typename T, int MODE, typename TIO>
static dpp_status pass3(dpp_ctx_s* cx_, const FftItem& it, const typename cx<T>::t* Tb,
                        const double2* Cin, TIO* out) {
    hipStream_t st = cx_->stream;
    const double pl_ = (double)it.nplanes * it.S1 * it.S2;
    TimerScope ts_(cx_, DPP_TK_PLANES_OUT,
                   (double)it.nb * (sizeof(typename cx<T>::t) * pl_ + sizeof(TIO) * (MODE == G_ADD ? 2.0 : 1.0) * it.npw));
    const bool fp64 = sizeof(T) == 8;
    if (plane90(it)) {
        auto k = k_planes90_to_sphere<T, MODE, TIO>;
        DPP_TRY(set_lds(k, plane90_lds(fp64)));
        hipLaunchKernelGGL(k, dim3(it.nplanes, it.nb, 1), dim3(p90::NT), plane90_lds(fp64), st, nullptr, it, Tb, Cin,
                           out, (int64_t)0, (const int*)nullptr, (const int*)nullptr);
        DPP_LAUNCHED();
        return DPP_OK;
    }
    Launch L = plane_launch(it.S1, it.S2, fp64);
    DPP_NT_DISPATCH(L.threads, auto k = k_planes_to_sphere<T, MODE, TIO, NT_>; DPP_TRY(set_lds(k, L.lds));
                    hipLaunchKernelGGL(k, dim3(it.nplanes, it.nb, 1), dim3(NT_), L.lds, st, nullptr, it, Tb, Cin,
                                       out, (int64_t)0, (const int*)nullptr, (const int*)nullptr));
    DPP_LAUNCHED();
    return DPP_OK;
}

template <typename T>
dpp_status run_apply_H_local(dpp_ham_s* ham, int nb, const double2* C, int64_t ldC, double2* HC,
                             int64_t ldHC, void* ws) {
    dpp_basis_s* b = ham->basis;
    dpp_ctx_s* cx_ = b->grid->ctx;
    hipStream_t st = cx_->stream;
    using Cx = typename cx<T>::t;
    Cx* Tb = reinterpret_cast<Cx*>(ws);
    FftItem it = item_for(b, nb, ldC);
    DPP_TRY((pass1<T, double2>(cx_, it, C, Tb)));
    DPP_TRY((pass2<T, XZ_H, double2>(cx_, it, Tb, ham->d_Veff, nullptr)));
    TimerScope ts_(cx_, DPP_TK_PLANES_OUT,
                   (double)nb * (sizeof(Cx) * (double)it.nplanes * it.S1 * it.S2 + 32.0 * it.npw));
    FftItem ot = it;
    // gather writes HC with its own leading dimension; kinetic term reads C with ldC
    const bool fp64 = sizeof(T) == 8;
    if (plane90(ot)) {
        auto k = k_planes90_to_sphere<T, G_H, double2>;
        DPP_TRY(set_lds(k, plane90_lds(fp64)));
        hipLaunchKernelGGL(k, dim3(ot.nplanes, ot.nb, 1), dim3(p90::NT), plane90_lds(fp64), st, nullptr, ot, Tb, C,
                           HC, ldHC, (const int*)nullptr, (const int*)nullptr);
        DPP_LAUNCHED();
        return DPP_OK;
    }
    Launch L = plane_launch(it.S1, it.S2, fp64);
    DPP_NT_DISPATCH(L.threads, auto k = k_planes_to_sphere<T, G_H, double2, NT_>; DPP_TRY(set_lds(k, L.lds));
                    hipLaunchKernelGGL(k, dim3(ot.nplanes, ot.nb, 1), dim3(NT_), L.lds, st, nullptr, ot, Tb, C, HC,
                                       ldHC, (const int*)nullptr, (const int*)nullptr));
    DPP_LAUNCHED();
    return DPP_OK;
}
template dpp_status run_apply_H_local<double>(dpp_ham_s*, int, const double2*, int64_t, double2*,
                                              int64_t, void*);
template dpp_status run_apply_H_local<float>(dpp_ham_s*, int, const double2*, int64_t, double2*,
                                             int64_t, void*);


size_t batched_plane_elems(const std::vector<FftItem>& h) {
    size_t t = 0;
    for (const FftItem& it : h) t = std::max(t, (size_t)it.t_off + (size_t)it.nb * it.nplanes * it.S1 * it.S2);
    return t;
}

namespace {
// Largest workgroup and LDS any item of a table needs for a plane pass and
// for an x-z pass, and the largest grid extents.
struct BatchShape {
    Launch plane, xz;
    int maxP, maxS1, maxS0, nbm;
};

BatchShape batch_shape(const std::vector<FftItem>& h, bool fp64) {
    BatchShape b{{0, 0}, {0, 0}, 0, 0, 0, 0};
    for (const FftItem& it : h) {
        const Launch p = plane_launch(it.S1, it.S2, fp64), x = xz_launch(it.S0, it.S2, fp64);
        b.plane.threads = std::max(b.plane.threads, p.threads);
        b.plane.lds = std::max(b.plane.lds, p.lds);
        b.xz.threads = std::max(b.xz.threads, x.threads);
        b.xz.lds = std::max(b.xz.lds, x.lds);
        b.maxP = std::max(b.maxP, it.nplanes);
        b.maxS1 = std::max(b.maxS1, it.S1);
        b.maxS0 = std::max(b.maxS0, it.S0);
        b.nbm = std::max(b.nbm, it.nb);
    }
    return b;
}
}  // namespace

// Sphere -> planes (to_sphere = false) or planes -> sphere with the kinetic
// term (to_sphere = true) for every item: one launch per plane group
// (register passes for digit-reversed items, LDS passes for the rest), or a
// single LDS launch without a plan.
template <typename T>
static dpp_status planes_pass(dpp_ctx_s* cx_, bool to_sphere, const BatchShape& bs, const FftItem* d_items,
                              const FftItem& i0, unsigned nit, const PlanePlan* pplan, const double2* X,
                              typename cx<T>::t* Tb, double2* HX, const int* act) {
    using Cx = typename cx<T>::t;
    hipStream_t st = cx_->stream;
    const size_t ng = pplan ? pplan->N.size() : 1;
    for (size_t g = 0; g < ng; ++g) {
        const int N = pplan ? pplan->N[g] : 0;
        const int* idx = pplan ? pplan->idx[g] : nullptr;
        const dim3 grid(pplan ? pplan->maxP[g] : bs.maxP, pplan ? pplan->nbm[g] : bs.nbm,
                        pplan ? pplan->count[g] : nit);
        if (N > 0 && planes_reg_launch<T>(N, to_sphere, grid, st, d_items, idx, X, Tb, HX, act)) {
            DPP_LAUNCHED();
            continue;
        }
        if (N == kPlane90Group) {
            const size_t lds = plane90_lds(sizeof(T) == 8);
            if (to_sphere) {
                auto k = k_planes90_to_sphere<T, G_H, double2, true>;
                DPP_TRY(set_lds(k, lds));
                hipLaunchKernelGGL(k, grid, dim3(p90::NT), lds, st, d_items, i0, (const Cx*)Tb, X, HX, (int64_t)0,
                                   act, idx);
            } else {
                auto k = k_planes90_from_sphere<T, double2, true>;
                DPP_TRY(set_lds(k, lds));
                hipLaunchKernelGGL(k, grid, dim3(p90::NT), lds, st, d_items, i0, X, Tb, act, idx);
            }
            DPP_LAUNCHED();
            continue;
        }
        if (N > 0) return set_error(DPP_EUNSUPPORTED, "plane pass length without a register kernel");
        if (to_sphere) {
            DPP_NT_DISPATCH(bs.plane.threads, auto k = k_planes_to_sphere<T, G_H, double2, NT_, true>;
                            DPP_TRY(set_lds(k, bs.plane.lds));
                            hipLaunchKernelGGL(k, grid, dim3(NT_), bs.plane.lds, st, d_items, i0, (const Cx*)Tb, X,
                                               HX, (int64_t)0, act, idx));
        } else {
            DPP_NT_DISPATCH(bs.plane.threads, auto k = k_planes_from_sphere<T, double2, NT_, true>;
                            DPP_TRY(set_lds(k, bs.plane.lds));
                            hipLaunchKernelGGL(k, grid, dim3(NT_), bs.plane.lds, st, d_items, i0, X, Tb, act, idx));
        }
        DPP_LAUNCHED();
    }
    return DPP_OK;
}

// One launch per pass for every item of the table (items may differ in box,
// sphere and band count).
bool plane_reg_supported(int n) { return plane_reg_len(n); }

PlanePlan plane_plan_groups(const std::vector<FftItem>& h, std::vector<std::vector<int>>& members) {
    PlanePlan p;
    members.clear();
    for (size_t k = 0; k < h.size(); ++k) {
        const FftItem& it = h[k];
        const int key = it.perm ? it.S1 : plane90(it) ? kPlane90Group : 0;
        size_t g = 0;
        while (g < p.N.size() && p.N[g] != key) ++g;
        if (g == p.N.size()) {
            p.N.push_back(key);
            p.count.push_back(0);
            p.maxP.push_back(0);
            p.nbm.push_back(0);
            p.idx.push_back(nullptr);
            members.emplace_back();
        }
        p.count[g]++;
        p.maxP[g] = std::max(p.maxP[g], it.nplanes);
        p.nbm[g] = std::max(p.nbm[g], it.nb);
        members[g].push_back((int)k);
    }
    return p;
}

bool xz_variant_available(int S0, bool fp64, int v) {
    return fp64 ? xz_available_t<double>(S0, v) : xz_available_t<float>(S0, v);
}

XzPlan xz_plan_groups(const std::vector<FftItem>& h, std::vector<std::vector<int>>& members) {
    XzPlan p;
    members.clear();
    for (size_t k = 0; k < h.size(); ++k) {
        const FftItem& it = h[k];
        size_t g = 0;
        while (g < p.S0.size() && p.S0[g] != it.S0) ++g;
        if (g == p.S0.size()) {
            p.S0.push_back(it.S0);
            p.count.push_back(0);
            p.maxS1S2.push_back(0);
            p.nbm.push_back(0);
            p.idx.push_back(nullptr);
            p.var64.push_back(XZ_AUTO);
            p.var32.push_back(XZ_AUTO);
            members.emplace_back();
        }
        p.count[g]++;
        p.maxS1S2[g] = std::max(p.maxS1S2[g], it.S1 * it.S2);
        p.nbm[g] = std::max(p.nbm[g], it.nb);
        members[g].push_back((int)k);
    }
    return p;
}

template <typename T>
dpp_status apply_H_local_batched(dpp_ctx_s* cx_, const FftItem* d_items, const std::vector<FftItem>& h,
                                 const double2* X, double2* HX, const double* V, void* Tbv, const int* act,
                                 const XzPlan* plan, const PlanePlan* pplan) {
    using Cx = typename cx<T>::t;
    if (h.empty()) return DPP_OK;
    Cx* Tb = reinterpret_cast<Cx*>(Tbv);
    hipStream_t st = cx_->stream;
    const bool fp64 = sizeof(T) == 8;
    const BatchShape bs = batch_shape(h, fp64);
    double b1 = 0, b2 = 0, b3 = 0;
    for (const FftItem& it : h) {
        const double pl = (double)it.nplanes * it.S1 * it.S2;
        b1 += it.nb * (16.0 * it.npw + sizeof(Cx) * pl);
        b2 += it.nb * 2.0 * sizeof(Cx) * pl + 8.0 * it.S0 * it.S1 * it.S2;
        b3 += it.nb * (sizeof(Cx) * pl + 32.0 * it.npw);
    }
    const FftItem& i0 = h[0];
    const unsigned nit = (unsigned)h.size();
    // passes masked to a subset of items are timed apart, without bytes
    const bool masked = act != nullptr;
    {
        TimerScope ts_(cx_, masked ? DPP_TK_MASKED : DPP_TK_PLANES_IN, masked ? 0.0 : b1);
        DPP_TRY(planes_pass<T>(cx_, false, bs, d_items, i0, nit, pplan, X, Tb, nullptr, act));
    }
    {
        TimerScope ts_(cx_, masked ? DPP_TK_MASKED : DPP_TK_XZ_H, masked ? 0.0 : b2);
        if (plan) {
            for (size_t g = 0; g < plan->S0.size(); ++g) {
                const dim3 grid((unsigned)((plan->maxS1S2[g] + 255) / 256), (unsigned)plan->nbm[g],
                                (unsigned)plan->count[g]);
                const std::vector<int>& var = fp64 ? plan->var64 : plan->var32;
                const int v = g < var.size() ? var[g] : XZ_AUTO;
                if (!xz_reg_launch<T>(plan->S0[g], grid, st, d_items, plan->idx[g], Tb, V, act, v)) {
                    DPP_NT_DISPATCH(bs.xz.threads, auto k = k_xz<T, XZ_H, double2, NT_, true>;
                                    DPP_TRY(set_lds(k, bs.xz.lds));
                                    hipLaunchKernelGGL(k, dim3(bs.maxS1, plan->nbm[g], plan->count[g]), dim3(NT_),
                                                       bs.xz.lds, st, d_items, i0, Tb, V, (double2*)nullptr, act,
                                                       plan->idx[g]));
                }
                DPP_LAUNCHED();
            }
        } else {
            DPP_NT_DISPATCH(bs.xz.threads, auto k = k_xz<T, XZ_H, double2, NT_, true>; DPP_TRY(set_lds(k, bs.xz.lds));
                            hipLaunchKernelGGL(k, dim3(bs.maxS1, bs.nbm, nit), dim3(NT_), bs.xz.lds, st, d_items, i0,
                                               Tb, V, (double2*)nullptr, act, (const int*)nullptr));
            DPP_LAUNCHED();
        }
    }
    {
        TimerScope ts_(cx_, masked ? DPP_TK_MASKED : DPP_TK_PLANES_OUT, masked ? 0.0 : b3);
        DPP_TRY(planes_pass<T>(cx_, true, bs, d_items, i0, nit, pplan, X, Tb, HX, act));
    }
    return DPP_OK;
}
template dpp_status apply_H_local_batched<double>(dpp_ctx_s*, const FftItem*, const std::vector<FftItem>&,
                                                  const double2*, double2*, const double*, void*, const int*,
                                                  const XzPlan*, const PlanePlan*);
template dpp_status apply_H_local_batched<float>(dpp_ctx_s*, const FftItem*, const std::vector<FftItem>&,
                                                 const double2*, double2*, const double*, void*, const int*,
                                                 const XzPlan*, const PlanePlan*);

__global__ void __launch_bounds__(256)
k_vx_cells(const FftItem* __restrict__ items, const double* __restrict__ V, double* __restrict__ Vx) {
    const FftItem& it = items[blockIdx.y];
    const int np = it.S1 * it.S2;
    const int64_t N = (int64_t)it.S0 * np;
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < N; e += (int64_t)gridDim.x * 256) {
        const int k = (int)(e / np), col = (int)(e - (int64_t)k * np);
        int vcol = col;
        if (it.perm) {
            const int p1 = col / it.S2, p2 = col - p1 * it.S2;
            vcol = digit_rev_axis(it.ax[1], p1) * it.S2 + digit_rev_axis(it.ax[2], p2);
        }
        Vx[it.v_off + e] = it.vscale * V[it.v_off + (int64_t)k * np + vcol];
    }
}

dpp_status vx_cells(dpp_ctx_s* cx_, const FftItem* d_cell_items, int ncells, int64_t maxN, const double* V,
                    double* Vx) {
    if (ncells <= 0) return DPP_OK;
    TimerScope ts_(cx_, DPP_TK_FIELDS);
    const unsigned nbx = (unsigned)std::min<int64_t>(1024, (maxN + 255) / 256);
    hipLaunchKernelGGL(k_vx_cells, dim3(nbx, (unsigned)ncells), dim3(256), 0, cx_->stream, d_cell_items, V, Vx);
    DPP_LAUNCHED();
    return DPP_OK;
}

// Density x pass in registers: a lane pair per (item, band chunk, column)
// as in k_xz_reg2; over the chunk's bands the column is transformed to real
// space along x and w f |psi|^2 accumulated in FP64 registers, then written
// to the chunk's partial box at natural (x, y, z).
template <typename T, int S0>
__global__ void __launch_bounds__(256)
k_xz_dens_reg2(const FftItem* __restrict__ items, const int* __restrict__ idx, const typename cx<T>::t* __restrict__ Tb,
               const double* __restrict__ fill, double* __restrict__ part) {
    using Cx = typename cx<T>::t;
    constexpr int M = S0 / 2;
    const int item = idx ? idx[blockIdx.z] : (int)blockIdx.z;
    const FftItem& it = items[item];
    const int c = blockIdx.y;
    if (c >= it.dnch) return;
    const int np = it.S1 * it.S2;
    const int col = blockIdx.x * 128 + (threadIdx.x >> 1);
    const int h = threadIdx.x & 1;
    if (col >= np) return;  // both lanes of a pair leave together
    const int nP = it.nplanes;
    const int b0 = c * it.dchunk, b1 = min(it.nb, b0 + it.dchunk);
    double acc[M];
#pragma unroll
    for (int p = 0; p < M; ++p) acc[p] = 0.0;
    for (int b = b0; b < b1; ++b) {
        const double fb = fill[it.f_off + b];
        if (fb == 0.0) continue;  // uniform across the workgroup
        const Cx* base = Tb + it.t_off + (int64_t)b * nP * np + col;
        Cx x[M];
#pragma unroll
        for (int j = 0; j < M; ++j) {
            int d = (j + h * M - it.n0min) % S0;
            d += d < 0 ? S0 : 0;
            x[j] = d < nP ? base[(int64_t)d * np] : Cx{0, 0};
        }
#pragma unroll
        for (int j = 0; j < M; ++j) {
            const Cx o = Cx{pair_swap(x[j].x), pair_swap(x[j].y)};
            if (h == 0) {
                x[j] = Cx{x[j].x + o.x, x[j].y + o.y};
            } else {
                const Cx dlt = Cx{o.x - x[j].x, o.y - x[j].y};
                x[j] = j == 0 ? dlt : cmul(dlt, reg_twiddle<T, S0>(j, +1));
            }
        }
        reg_dif<T, M, +1, 0>(x, nullptr, nullptr);
#pragma unroll
        for (int p = 0; p < M; ++p) {
            const double xr = (double)x[p].x, xi = (double)x[p].y;
            acc[p] += fb * (xr * xr + xi * xi);
        }
    }
    int n1 = col / it.S2, n2 = col - (col / it.S2) * it.S2;
    if (it.perm) {
        n1 = digit_rev_axis(it.ax[1], n1);
        n2 = digit_rev_axis(it.ax[2], n2);
    }
    const int64_t N = (int64_t)S0 * np;
    double* dst = part + it.p_off + (int64_t)c * N + (int64_t)n1 * it.S2 + n2;
#pragma unroll
    for (int p = 0; p < M; ++p) dst[(int64_t)(2 * reg_digit_rev(M, p) + h) * np] = it.wk * acc[p];
}

// Register density pass for one x-length group; false if S0 has none.
template <typename T>
static bool dens_reg_launch(int S0, dim3 grid, hipStream_t st, const FftItem* items, const int* idx,
                            const typename cx<T>::t* Tb, const double* fill, double* part) {
    grid.x = (grid.x * 256 + 127) / 128;
    switch (S0) {
#define DPP_DENS_REG(n)                                                                                      \
    case n:                                                                                                  \
        hipLaunchKernelGGL((k_xz_dens_reg2<T, n>), grid, dim3(256), 0, st, items, idx, Tb, fill, part); \
        return true;
        DPP_DENS_REG(12) DPP_DENS_REG(16) DPP_DENS_REG(18) DPP_DENS_REG(20) DPP_DENS_REG(24) DPP_DENS_REG(30)
        DPP_DENS_REG(32) DPP_DENS_REG(36) DPP_DENS_REG(40) DPP_DENS_REG(48) DPP_DENS_REG(50) DPP_DENS_REG(54)
        DPP_DENS_REG(60) DPP_DENS_REG(64) DPP_DENS_REG(90)
#undef DPP_DENS_REG
        default:
            return false;
    }
}

static bool dens_reg_available(int S0) {
    switch (S0) {
        case 12: case 16: case 18: case 20: case 24: case 30: case 32: case 36: case 40:
        case 48: case 50: case 54: case 60: case 64: case 90:
            return true;
        default:
            return false;
    }
}

template <typename T>
dpp_status density_batched(dpp_ctx_s* cx_, const FftItem* d_items, const std::vector<FftItem>& h,
                           const double2* psi, const double* fill, void* Tbv, double* part,
                           const CellDesc* d_cells, int ncells, int64_t maxN, double* n, const PlanePlan* pplan,
                           const XzPlan* xplan) {
    using Cx = typename cx<T>::t;
    if (h.empty()) return DPP_OK;
    Cx* Tb = reinterpret_cast<Cx*>(Tbv);
    hipStream_t st = cx_->stream;
    const bool fp64 = sizeof(T) == 8;
    const BatchShape bs = batch_shape(h, fp64);
    double b1 = 0, b2 = 0;
    int mch = 1;
    for (const FftItem& it : h) {
        const double pl = (double)it.nplanes * it.S1 * it.S2;
        b1 += it.nb * (16.0 * it.npw + sizeof(Cx) * pl);
        b2 += it.nb * sizeof(Cx) * pl + it.dnch * 8.0 * it.S0 * it.S1 * it.S2;
        mch = std::max(mch, it.dnch);
    }
    const FftItem& i0 = h[0];
    const unsigned nit = (unsigned)h.size();
    {
        TimerScope ts_(cx_, DPP_TK_PLANES_IN, b1);
        DPP_TRY(planes_pass<T>(cx_, false, bs, d_items, i0, nit, pplan, psi, Tb, nullptr, nullptr));
    }
    {
        TimerScope ts_(cx_, DPP_TK_XZ_DENSITY, b2);
        // per x-length group: the register pass where the length has one, else
        // the LDS pass over the group's items; without groups the LDS pass
        if (xplan) {
            for (size_t g = 0; g < xplan->S0.size(); ++g) {
                const dim3 grid((unsigned)((xplan->maxS1S2[g] + 255) / 256), (unsigned)mch,
                                (unsigned)xplan->count[g]);
                if (!dens_reg_available(xplan->S0[g]) ||
                    !dens_reg_launch<T>(xplan->S0[g], grid, st, d_items, xplan->idx[g], (const Cx*)Tb, fill, part)) {
                    const int* gidx = xplan->idx[g];
                    DPP_NT_DISPATCH(bs.xz.threads, auto k = k_xz_density<T, NT_, true>; DPP_TRY(set_lds(k, bs.xz.lds));
                                    hipLaunchKernelGGL(k, dim3(bs.maxS1, mch, xplan->count[g]), dim3(NT_), bs.xz.lds,
                                                       st, d_items, i0, (const Cx*)Tb, fill, part, gidx));
                }
                DPP_LAUNCHED();
            }
        } else {
            DPP_NT_DISPATCH(bs.xz.threads, auto k = k_xz_density<T, NT_, true>; DPP_TRY(set_lds(k, bs.xz.lds));
                            hipLaunchKernelGGL(k, dim3(bs.maxS1, mch, nit), dim3(NT_), bs.xz.lds, st, d_items, i0,
                                               (const Cx*)Tb, fill, part, (const int*)nullptr));
            DPP_LAUNCHED();
        }
    }
    TimerScope ts_(cx_, DPP_TK_FIELDS);
    hipLaunchKernelGGL(k_density_reduce_cells, dim3((unsigned)((maxN + 255) / 256), (unsigned)ncells), dim3(256), 0,
                       st, (const double*)part, d_cells, n);
    DPP_LAUNCHED();
    return DPP_OK;
}
template dpp_status density_batched<double>(dpp_ctx_s*, const FftItem*, const std::vector<FftItem>&, const double2*,
                                            const double*, void*, double*, const CellDesc*, int, int64_t, double*,
                                            const PlanePlan*, const XzPlan*);
template dpp_status density_batched<float>(dpp_ctx_s*, const FftItem*, const std::vector<FftItem>&, const double2*,
                                           const double*, void*, double*, const CellDesc*, int, int64_t, double*,
                                           const PlanePlan*, const XzPlan*);

// Per cell: E[c * stride] = (Omega / 2) sum of the cell's Hartree row partials.
__global__ void k_hartree_energy_cells(const double* __restrict__ part, const CellDesc* __restrict__ cells,
                                       int ncells, double* __restrict__ E, int E_stride) {
    __shared__ double red[256];
    const CellDesc c = cells[blockIdx.x];
    double s = 0.0;
    for (int i = threadIdx.x; i < c.S1; i += 256) s += part[c.eoff + i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) E[(int64_t)blockIdx.x * E_stride] = 0.5 * c.omega * red[0];
}

dpp_status hartree_batched(dpp_ctx_s* cx_, const FftItem* d_items, const std::vector<FftItem>& h, const double* n,
                           double* VH, void* Tbv, double* epart, const CellDesc* d_cells, double* E, int E_stride) {
    if (h.empty()) return DPP_OK;
    if (!VH && !E) return DPP_OK;
    double2* Tb = reinterpret_cast<double2*>(Tbv);
    hipStream_t st = cx_->stream;
    const BatchShape bs = batch_shape(h, true);
    const unsigned nc = (unsigned)h.size();
    const FftItem& i0 = h[0];
    TimerScope ts_(cx_, DPP_TK_FULLBOX);
    DPP_NT_DISPATCH(bs.plane.threads, auto kp = k_planes_from_box<double, true, NT_, true>;
                    DPP_TRY(set_lds(kp, bs.plane.lds));
                    hipLaunchKernelGGL(kp, dim3(bs.maxS0, 1, nc), dim3(NT_), bs.plane.lds, st, d_items, i0,
                                       (const void*)n, (int64_t)0, -1, Tb));
    DPP_LAUNCHED();
    if (VH) {
        DPP_NT_DISPATCH(bs.xz.threads, auto kx = k_xz_hartree<NT_, true>; DPP_TRY(set_lds(kx, bs.xz.lds));
                        hipLaunchKernelGGL(kx, dim3(bs.maxS1, 1, nc), dim3(NT_), bs.xz.lds, st, d_items, i0, Tb,
                                           epart));
        DPP_LAUNCHED();
        DPP_NT_DISPATCH(bs.plane.threads, auto kq = k_planes_to_box<double, true, NT_, true>;
                        DPP_TRY(set_lds(kq, bs.plane.lds));
                        hipLaunchKernelGGL(kq, dim3(bs.maxS0, 1, nc), dim3(NT_), bs.plane.lds, st, d_items, i0,
                                           (const double2*)Tb, +1, 1.0, (void*)VH, (int64_t)0));
        DPP_LAUNCHED();
    } else {
        // the energy only: no way back to real space
        DPP_NT_DISPATCH(bs.xz.threads, auto kx = k_xz_hartree<NT_, true, false>; DPP_TRY(set_lds(kx, bs.xz.lds));
                        hipLaunchKernelGGL(kx, dim3(bs.maxS1, 1, nc), dim3(NT_), bs.xz.lds, st, d_items, i0, Tb,
                                           epart));
        DPP_LAUNCHED();
    }
    if (!E) return DPP_OK;  // V_H only
    hipLaunchKernelGGL(k_hartree_energy_cells, dim3(nc), dim3(256), 0, st, (const double*)epart, d_cells, (int)nc, E,
                       E_stride);
    DPP_LAUNCHED();
    return DPP_OK;
}

}  // namespace dpp

using namespace dpp;

// ------------------------------------------------------------- C ABI -------

extern "C" dpp_status dpp_workspace_size(dpp_basis basis, int nb, dpp_precision prec, size_t* bytes) {
    clear_error();
    DPP_REQUIRE(basis && bytes, "dpp_workspace_size: null argument");
    DPP_REQUIRE(nb >= 0, "dpp_workspace_size: nb < 0");
    DPP_REQUIRE(prec == DPP_F64 || prec == DPP_F32, "dpp_workspace_size: bad precision");
    const size_t el = prec == DPP_F64 ? 16 : 8;
    const size_t t = ((plane_buffer_elems(basis, std::max(nb, 1)) * el + 255) / 256) * 256;
    // after the plane buffer: density partials (up to DENS_CHUNKS boxes) or the
    // projector scratch (Pi = P^dag C and its reduction partials)
    const size_t dens = (size_t)std::min(std::max(nb, 1), DENS_CHUNKS) * basis->grid->N * sizeof(double);
    const size_t proj = proj_ws_bytes(basis, std::max(nb, 1));
    *bytes = t + std::max(dens, proj) + 256;
    return DPP_OK;
}

// Grid workspace: [plane buffer: N complex][partial sums: 64 KB][coefficients: N complex]
size_t dpp::grid_coef_offset(const dpp_grid_s* g) { return (size_t)g->N * 16 + 64 * 1024; }

extern "C" dpp_status dpp_grid_workspace_size(dpp_grid grid, size_t* bytes) {
    clear_error();
    DPP_REQUIRE(grid && bytes, "dpp_grid_workspace_size: null argument");
    *bytes = grid_coef_offset(grid) + (size_t)grid->N * 16 + 256;
    return DPP_OK;
}

dpp_status dpp::full_inverse_real(dpp_grid_s* g, const double2* coef, double* out, void* ws) {
    hipStream_t st = g->ctx->stream;
    TimerScope ts_(g->ctx, DPP_TK_FULLBOX);
    const FftItem& it = g->h_item;
    double2* Tb = reinterpret_cast<double2*>(ws);
    Launch Lp = plane_launch(it.S1, it.S2, true);
    Launch Lx = xz_launch(it.S0, it.S2, true);
    DPP_NT_DISPATCH(Lx.threads, auto kx = k_xz_full<double, NT_>; DPP_TRY(set_lds(kx, Lx.lds));
                    hipLaunchKernelGGL(kx, dim3(it.S1, 1, 1), dim3(NT_), Lx.lds, st, it, coef, +1, 1.0, Tb,
                                       (int64_t)0));
    DPP_LAUNCHED();
    DPP_NT_DISPATCH(Lp.threads, auto kq = k_planes_to_box<double, true, NT_>; DPP_TRY(set_lds(kq, Lp.lds));
                    hipLaunchKernelGGL(kq, dim3(it.S0, 1, 1), dim3(NT_), Lp.lds, st, nullptr, it, (const double2*)Tb, +1,
                                       1.0, (void*)out, (int64_t)0));
    DPP_LAUNCHED();
    return DPP_OK;
}

template <typename TIO, typename T>
static dpp_status do_I(dpp_basis b, int nb, const TIO* C, int64_t ldC, TIO* out, void* ws) {
    dpp_ctx_s* cx_ = b->grid->ctx;
    using Cx = typename cx<T>::t;
    Cx* Tb = reinterpret_cast<Cx*>(ws);
    FftItem it = item_for(b, nb, ldC);
    DPP_TRY((pass1<T, TIO>(cx_, it, C, Tb)));
    DPP_TRY((pass2<T, XZ_TO_BOX, TIO>(cx_, it, Tb, nullptr, out)));
    return DPP_OK;
}

template <typename TIO, typename T>
static dpp_status do_Idag(dpp_basis b, int nb, const TIO* grid, TIO* C, int64_t ldC, int acc,
                          void* ws) {
    dpp_ctx_s* cx_ = b->grid->ctx;
    using Cx = typename cx<T>::t;
    Cx* Tb = reinterpret_cast<Cx*>(ws);
    FftItem it = item_for(b, nb, ldC);
    DPP_TRY((pass2<T, XZ_FROM_BOX, TIO>(cx_, it, Tb, nullptr, const_cast<TIO*>(grid))));
    if (acc)
        DPP_TRY((pass3<T, G_ADD, TIO>(cx_, it, Tb, nullptr, C)));
    else
        DPP_TRY((pass3<T, G_SET, TIO>(cx_, it, Tb, nullptr, C)));
    return DPP_OK;
}

static dpp_status check_block(dpp_basis b, int nb, const void* p, int64_t ld, const char* who) {
    DPP_REQUIRE(b, std::string(who) + ": null basis");
    DPP_REQUIRE(nb >= 0, std::string(who) + ": nb < 0");
    DPP_REQUIRE(nb == 0 || p, std::string(who) + ": null block");
    DPP_REQUIRE(ld >= b->npw, std::string(who) + ": leading dimension < npw");
    return DPP_OK;
}

extern "C" dpp_status dpp_I(dpp_basis basis, int nb, const void* C, int64_t ldC, void* grid_out,
                            dpp_precision prec, void* ws) {
    clear_error();
    DPP_TRY(check_block(basis, nb, C, ldC, "dpp_I"));
    DPP_REQUIRE(nb == 0 || (grid_out && ws), "dpp_I: null output or workspace");
    DPP_REQUIRE(prec == DPP_F64 || prec == DPP_F32, "dpp_I: bad precision");
    if (nb == 0) return DPP_OK;
    if (prec == DPP_F64)
        return do_I<double2, double>(basis, nb, (const double2*)C, ldC, (double2*)grid_out, ws);
    return do_I<float2, float>(basis, nb, (const float2*)C, ldC, (float2*)grid_out, ws);
}

extern "C" dpp_status dpp_Idag(dpp_basis basis, int nb, const void* grid, void* C_out, int64_t ldC,
                               int accumulate, dpp_precision prec, void* ws) {
    clear_error();
    DPP_TRY(check_block(basis, nb, C_out, ldC, "dpp_Idag"));
    DPP_REQUIRE(nb == 0 || (grid && ws), "dpp_Idag: null input or workspace");
    DPP_REQUIRE(prec == DPP_F64 || prec == DPP_F32, "dpp_Idag: bad precision");
    if (nb == 0) return DPP_OK;
    if (prec == DPP_F64)
        return do_Idag<double2, double>(basis, nb, (const double2*)grid, (double2*)C_out, ldC,
                                        accumulate, ws);
    return do_Idag<float2, float>(basis, nb, (const float2*)grid, (float2*)C_out, ldC, accumulate, ws);
}

// Full-box complex transform: y = scale * FFT_sign(x).
static dpp_status full_transform(dpp_grid g, int nf, const double2* x, double2* y, int sign,
                                 double scale, void* ws) {
    hipStream_t st = g->ctx->stream;
    TimerScope ts_(g->ctx, DPP_TK_FULLBOX);
    const FftItem& it = g->h_item;
    double2* Tb = reinterpret_cast<double2*>(ws);
    Launch Lp = plane_launch(it.S1, it.S2, true);
    Launch Lx = xz_launch(it.S0, it.S2, true);
    for (int f = 0; f < nf; ++f) {
        DPP_NT_DISPATCH(Lp.threads, auto kp = k_planes_from_box<double, false, NT_>; DPP_TRY(set_lds(kp, Lp.lds));
                        hipLaunchKernelGGL(kp, dim3(it.S0, 1, 1), dim3(NT_), Lp.lds, st, nullptr, it,
                                           (const void*)(x + (int64_t)f * g->N), (int64_t)0, sign, Tb));
        DPP_LAUNCHED();
        DPP_NT_DISPATCH(Lx.threads, auto kx = k_xz_full<double, NT_>; DPP_TRY(set_lds(kx, Lx.lds));
                        hipLaunchKernelGGL(kx, dim3(it.S1, 1, 1), dim3(NT_), Lx.lds, st, it, Tb, sign, scale,
                                           y + (int64_t)f * g->N, (int64_t)0));
        DPP_LAUNCHED();
    }
    return DPP_OK;
}

dpp_status dpp::full_complex(dpp_grid_s* g, int nf, const double2* x, double2* y, int sign, double scale, void* ws) {
    // all nf fields in one launch per pass (blockIdx.y = field); ws holds nf plane buffers
    hipStream_t st = g->ctx->stream;
    TimerScope ts_(g->ctx, DPP_TK_FULLBOX);
    const FftItem& it = g->h_item;
    double2* Tb = reinterpret_cast<double2*>(ws);
    Launch Lp = plane_launch(it.S1, it.S2, true);
    Launch Lx = xz_launch(it.S0, it.S2, true);
    DPP_NT_DISPATCH(Lp.threads, auto kp = k_planes_from_box<double, false, NT_>; DPP_TRY(set_lds(kp, Lp.lds));
                    hipLaunchKernelGGL(kp, dim3(it.S0, nf, 1), dim3(NT_), Lp.lds, st, nullptr, it, (const void*)x,
                                       g->N, sign, Tb));
    DPP_LAUNCHED();
    DPP_NT_DISPATCH(Lx.threads, auto kx = k_xz_full<double, NT_>; DPP_TRY(set_lds(kx, Lx.lds));
                    hipLaunchKernelGGL(kx, dim3(it.S1, nf, 1), dim3(NT_), Lx.lds, st, it, Tb, sign, scale, y, g->N));
    DPP_LAUNCHED();
    return DPP_OK;
}

// y = J n for a real field n on the grid's box (FP64, natural order); ws
// holds the N-point plane buffer.
dpp_status dpp::full_forward_real(dpp_grid_s* g, const double* n, double2* y, void* ws) {
    hipStream_t st = g->ctx->stream;
    TimerScope ts_(g->ctx, DPP_TK_FULLBOX);
    const FftItem& it = g->h_item;
    double2* Tb = reinterpret_cast<double2*>(ws);
    Launch Lp = plane_launch(it.S1, it.S2, true);
    Launch Lx = xz_launch(it.S0, it.S2, true);
    DPP_NT_DISPATCH(Lp.threads, auto kp = k_planes_from_box<double, true, NT_>; DPP_TRY(set_lds(kp, Lp.lds));
                    hipLaunchKernelGGL(kp, dim3(it.S0, 1, 1), dim3(NT_), Lp.lds, st, nullptr, it, (const void*)n,
                                       (int64_t)0, -1, Tb));
    DPP_LAUNCHED();
    DPP_NT_DISPATCH(Lx.threads, auto kx = k_xz_full<double, NT_>; DPP_TRY(set_lds(kx, Lx.lds));
                    hipLaunchKernelGGL(kx, dim3(it.S1, 1, 1), dim3(NT_), Lx.lds, st, it, Tb, -1,
                                       1.0 / (double)g->N, y, (int64_t)0));
    DPP_LAUNCHED();
    return DPP_OK;
}

extern "C" dpp_status dpp_J(dpp_grid grid, int nf, const dpp_c64* x, dpp_c64* y, void* ws) {
    clear_error();
    DPP_REQUIRE(grid && nf >= 0, "dpp_J: bad arguments");
    DPP_REQUIRE(nf == 0 || (x && y && ws), "dpp_J: null pointer");
    return full_transform(grid, nf, (const double2*)x, (double2*)y, -1, 1.0 / (double)grid->N, ws);
}

extern "C" dpp_status dpp_Jdag(dpp_grid grid, int nf, const dpp_c64* x, dpp_c64* y, void* ws) {
    clear_error();
    DPP_REQUIRE(grid && nf >= 0, "dpp_Jdag: bad arguments");
    DPP_REQUIRE(nf == 0 || (x && y && ws), "dpp_Jdag: null pointer");
    return full_transform(grid, nf, (const double2*)x, (double2*)y, +1, 1.0 / (double)grid->N, ws);
}

// Reduce per-i1 partial sums in fixed order: out = scale * sum.
__global__ void k_sum_partials(const double* __restrict__ part, int n, double scale,
                               double* __restrict__ out) {
    __shared__ double red[256];
    double s = 0.0;
    // fixed assignment: thread t sums t, t+256, ... in order
    for (int i = threadIdx.x; i < n; i += 256) s += part[i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = scale * red[0];
}

extern "C" dpp_status dpp_hartree(dpp_grid grid, const double* d_n, double* d_VH, double* d_EH,
                                  void* ws) {
    clear_error();
    DPP_REQUIRE(grid && d_n && d_VH && d_EH && ws, "dpp_hartree: null argument");
    hipStream_t st = grid->ctx->stream;
    TimerScope ts_(grid->ctx, DPP_TK_FULLBOX);
    const FftItem& it = grid->h_item;
    double2* Tb = reinterpret_cast<double2*>(ws);
    double* part = reinterpret_cast<double*>(reinterpret_cast<char*>(ws) + (size_t)grid->N * 16);
    Launch Lp = plane_launch(it.S1, it.S2, true);
    Launch Lx = xz_launch(it.S0, it.S2, true);
    DPP_NT_DISPATCH(Lp.threads, auto kp = k_planes_from_box<double, true, NT_>; DPP_TRY(set_lds(kp, Lp.lds));
                    hipLaunchKernelGGL(kp, dim3(it.S0, 1, 1), dim3(NT_), Lp.lds, st, nullptr, it, (const void*)d_n,
                                       (int64_t)0, -1, Tb));
    DPP_LAUNCHED();
    DPP_NT_DISPATCH(Lx.threads, auto kx = k_xz_hartree<NT_>; DPP_TRY(set_lds(kx, Lx.lds));
                    hipLaunchKernelGGL(kx, dim3(it.S1, 1, 1), dim3(NT_), Lx.lds, st, nullptr, it, Tb, part));
    DPP_LAUNCHED();
    DPP_NT_DISPATCH(Lp.threads, auto kq = k_planes_to_box<double, true, NT_>; DPP_TRY(set_lds(kq, Lp.lds));
                    hipLaunchKernelGGL(kq, dim3(it.S0, 1, 1), dim3(NT_), Lp.lds, st, nullptr, it, (const double2*)Tb, +1,
                                       1.0, (void*)d_VH, (int64_t)0));
    DPP_LAUNCHED();
    hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(256), 0, st, part, it.S1, 0.5 * grid->omega, d_EH);
    DPP_LAUNCHED();
    return DPP_OK;
}

extern "C" dpp_status dpp_density_accumulate(dpp_basis basis, int nb, const dpp_c64* psi,
                                             int64_t ldpsi, const double* d_f, double wk,
                                             double* d_n, dpp_precision prec, void* ws) {
    clear_error();
    DPP_TRY(check_block(basis, nb, psi, ldpsi, "dpp_density_accumulate"));
    DPP_REQUIRE(nb == 0 || (d_f && d_n && ws), "dpp_density_accumulate: null argument");
    DPP_REQUIRE(prec == DPP_F64 || prec == DPP_F32, "dpp_density_accumulate: bad precision");
    if (nb == 0) return DPP_OK;
    hipStream_t st = basis->grid->ctx->stream;
    FftItem it = item_for(basis, nb, ldpsi);
    it.wk = wk;
    it.f_off = 0;
    const int64_t N = basis->grid->N;
    const int nchunk = std::min(nb, DENS_CHUNKS);
    const int chunk = (nb + nchunk - 1) / nchunk;
    const int nch = (nb + chunk - 1) / chunk;
    it.p_off = 0;
    it.dnch = nch;
    it.dchunk = chunk;
    const bool fp64 = prec == DPP_F64;
    // partials live after the plane buffer
    const size_t tbytes = plane_buffer_elems(basis, nb) * (fp64 ? 16 : 8);
    double* part = reinterpret_cast<double*>(reinterpret_cast<char*>(ws) + ((tbytes + 255) / 256) * 256);
    Launch Lx = xz_launch(it.S0, it.S2, fp64);
    dpp_ctx_s* cx_ = basis->grid->ctx;
    if (fp64) {
        DPP_TRY((pass1<double, double2>(cx_, it, (const double2*)psi, (double2*)ws)));
        TimerScope ts_(cx_, DPP_TK_XZ_DENSITY, nb * 16.0 * it.nplanes * it.S1 * it.S2 + nch * 8.0 * N);
        DPP_NT_DISPATCH(Lx.threads, auto k = k_xz_density<double, NT_>; DPP_TRY(set_lds(k, Lx.lds));
                        hipLaunchKernelGGL(k, dim3(it.S1, nch, 1), dim3(NT_), Lx.lds, st, nullptr, it,
                                           (const double2*)ws, d_f, part, (const int*)nullptr));
    } else {
        DPP_TRY((pass1<float, double2>(cx_, it, (const double2*)psi, (float2*)ws)));
        TimerScope ts_(cx_, DPP_TK_XZ_DENSITY, nb * 8.0 * it.nplanes * it.S1 * it.S2 + nch * 8.0 * N);
        DPP_NT_DISPATCH(Lx.threads, auto k = k_xz_density<float, NT_>; DPP_TRY(set_lds(k, Lx.lds));
                        hipLaunchKernelGGL(k, dim3(it.S1, nch, 1), dim3(NT_), Lx.lds, st, nullptr, it,
                                           (const float2*)ws, d_f, part, (const int*)nullptr));
    }
    DPP_LAUNCHED();
    hipLaunchKernelGGL(k_density_reduce, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, st, part, nch,
                       N, d_n);
    DPP_LAUNCHED();
    return DPP_OK;
}
