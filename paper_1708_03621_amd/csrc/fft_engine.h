// Batched mixed-radix (2,3,4,5) FFT along one axis of a tile held in LDS.
//
// Stockham auto-sort formulation (Cooley-Tukey mixed radix without a bit
// reversal pass; cf. Govindaraju et al., "High performance discrete Fourier
// transforms on graphics processors", SC 2008): for stage radix R with Ns the
// product of the radices already applied, butterfly j of a length-n transform
// reads x[j + t n/R] (t < R), multiplies by w^(t k n/(Ns R)) with k = j mod Ns
// and w = exp(sign 2 pi i / n), applies the length-R DFT and writes
// y[(j/Ns) Ns R + k + t Ns].  The tile is updated in place: every thread
// loads all of its butterflies into registers, the workgroup synchronizes,
// and the results are stored to their new slots.
#pragma once

#include <hip/hip_runtime.h>

#include "internal.h"

namespace dpp {

template <typename T>
struct cx;
template <>
struct cx<double> {
    using t = double2;
};
template <>
struct cx<float> {
    using t = float2;
};

template <typename C>
__device__ __forceinline__ C cadd(C a, C b) {
    return C{a.x + b.x, a.y + b.y};
}
template <typename C>
__device__ __forceinline__ C csub(C a, C b) {
    return C{a.x - b.x, a.y - b.y};
}
template <typename C>
__device__ __forceinline__ C cmul(C a, C b) {
    return C{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
// multiply by sign*i
template <typename C>
__device__ __forceinline__ C cmul_si(C a, int sign) {
    return sign > 0 ? C{-a.y, a.x} : C{a.y, -a.x};
}
template <typename C, typename S>
__device__ __forceinline__ C cscale(C a, S s) {
    return C{a.x * s, a.y * s};
}

template <typename T>
__device__ __forceinline__ typename cx<T>::t twiddle(const double2* tw64, const float2* tw32, int m,
                                                     int sign);
template <>
__device__ __forceinline__ double2 twiddle<double>(const double2* tw64, const float2*, int m,
                                                   int sign) {
    double2 w = tw64[m];
    if (sign > 0) w.y = -w.y;
    return w;
}
template <>
__device__ __forceinline__ float2 twiddle<float>(const double2*, const float2* tw32, int m,
                                                 int sign) {
    float2 w = tw32[m];
    if (sign > 0) w.y = -w.y;
    return w;
}

// Length-R DFT in registers, V_m = sum_t v_t exp(sign 2 pi i t m / R).
template <typename T, int R>
struct Dft;

template <typename T>
struct Dft<T, 2> {
    using C = typename cx<T>::t;
    __device__ __forceinline__ static void run(C* v, int) {
        C a = v[0], b = v[1];
        v[0] = cadd(a, b);
        v[1] = csub(a, b);
    }
};

template <typename T>
struct Dft<T, 3> {
    using C = typename cx<T>::t;
    __device__ __forceinline__ static void run(C* v, int sign) {
        const T h = T(0.86602540378443864676);  // sqrt(3)/2
        C t1 = cadd(v[1], v[2]);
        C t2 = csub(v[1], v[2]);
        C m = C{v[0].x - T(0.5) * t1.x, v[0].y - T(0.5) * t1.y};
        C j = cmul_si(cscale(t2, h), sign);
        v[0] = cadd(v[0], t1);
        v[1] = cadd(m, j);
        v[2] = csub(m, j);
    }
};

template <typename T>
struct Dft<T, 4> {
    using C = typename cx<T>::t;
    __device__ __forceinline__ static void run(C* v, int sign) {
        C t0 = cadd(v[0], v[2]);
        C t1 = csub(v[0], v[2]);
        C t2 = cadd(v[1], v[3]);
        C t3 = cmul_si(csub(v[1], v[3]), sign);
        v[0] = cadd(t0, t2);
        v[2] = csub(t0, t2);
        v[1] = cadd(t1, t3);
        v[3] = csub(t1, t3);
    }
};

template <typename T>
struct Dft<T, 5> {
    using C = typename cx<T>::t;
    __device__ __forceinline__ static void run(C* v, int sign) {
        const T c1 = T(0.30901699437494742410);   // cos(2 pi/5)
        const T c2 = T(-0.80901699437494742410);  // cos(4 pi/5)
        const T s1 = T(0.95105651629515357212);   // sin(2 pi/5)
        const T s2 = T(0.58778525229247312917);   // sin(4 pi/5)
        C t1 = cadd(v[1], v[4]);
        C t2 = cadd(v[2], v[3]);
        C t3 = csub(v[1], v[4]);
        C t4 = csub(v[2], v[3]);
        C a1 = C{v[0].x + c1 * t1.x + c2 * t2.x, v[0].y + c1 * t1.y + c2 * t2.y};
        C a2 = C{v[0].x + c2 * t1.x + c1 * t2.x, v[0].y + c2 * t1.y + c1 * t2.y};
        C b1 = cmul_si(C{s1 * t3.x + s2 * t4.x, s1 * t3.y + s2 * t4.y}, sign);
        C b2 = cmul_si(C{s2 * t3.x - s1 * t4.x, s2 * t3.y - s1 * t4.y}, sign);
        v[0] = cadd(v[0], cadd(t1, t2));
        v[1] = cadd(a1, b1);
        v[4] = csub(a1, b1);
        v[2] = cadd(a2, b2);
        v[3] = csub(a2, b2);
    }
};

// Butterflies one thread may hold per stage.  Workgroups of 256 or 512
// threads keep up to 16 complex values per thread (R * MAXB <= 16); 1024-thread
// workgroups (128 VGPRs per lane) keep up to 10.  A tile of E elements fits
// when E <= MAXB * R * NT for every radix of the axis: 3840 elements at 256
// threads, 7680 at 512, 8192 at 1024.
template <int R, int NT>
struct MaxB {
    static constexpr int v = NT <= 512 ? (R == 2 ? 8 : R == 3 ? 5 : R == 4 ? 4 : 3)
                                       : (R == 2 ? 5 : R == 3 ? 3 : R == 4 ? 2 : 2);
};

// Address of element e of transform f inside the LDS tile.
struct AddrLinear {
    int fs, es;
    __device__ __forceinline__ int operator()(int f, int e) const { return f * fs + e * es; }
};
// Rows of a plane starting at Miller index n1lo (wrapping modulo S1); element = column.
struct AddrRowsWrap {
    int pitch, n1lo, S1;
    __device__ __forceinline__ int operator()(int f, int e) const {
        int r = n1lo + f;
        r += (r < 0) ? S1 : 0;
        r -= (r >= S1) ? S1 : 0;
        return r * pitch + e;
    }
};

template <typename T, int R, bool FMAJOR, int NT, typename Addr>
__device__ __forceinline__ void fft_stage(typename cx<T>::t* lds, int n, int nfft, int Ns,
                                          const Addr& addr, const double2* tw64,
                                          const float2* tw32, int sign) {
    using C = typename cx<T>::t;
    constexpr int MB = MaxB<R, NT>::v;
    const int m = n / R;
    const int total = nfft * m;
    const int twmul = n / (Ns * R);
    C v[MB][R];
#pragma unroll
    for (int u = 0; u < MB; ++u) {
        const int bt = threadIdx.x + u * NT;
        if (bt < total) {
            int f, j;
            if (FMAJOR) {
                f = bt % nfft;
                j = bt / nfft;
            } else {
                j = bt % m;
                f = bt / m;
            }
            const int k = j % Ns;
#pragma unroll
            for (int t = 0; t < R; ++t) {
                C a = lds[addr(f, j + t * m)];
                if (t > 0) a = cmul(a, twiddle<T>(tw64, tw32, t * k * twmul, sign));
                v[u][t] = a;
            }
            Dft<T, R>::run(v[u], sign);
        }
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < MB; ++u) {
        const int bt = threadIdx.x + u * NT;
        if (bt < total) {
            int f, j;
            if (FMAJOR) {
                f = bt % nfft;
                j = bt / nfft;
            } else {
                j = bt % m;
                f = bt / m;
            }
            const int k = j % Ns;
            const int base = (j / Ns) * Ns * R + k;
#pragma unroll
            for (int t = 0; t < R; ++t) lds[addr(f, base + t * Ns)] = v[u][t];
        }
    }
    __syncthreads();
}

// All stages of one axis.  sign = +1: exp(+i ...) (inverse, unnormalized);
// sign = -1: exp(-i ...) (forward).
template <typename T, bool FMAJOR, int NT, typename Addr>
__device__ __forceinline__ void fft_axis(typename cx<T>::t* lds, const FftAxis& ax, int nfft, const Addr& addr,
                         const double2* tw64, const float2* tw32, int sign) {
    int Ns = 1;
    for (int s = 0; s < ax.nrad; ++s) {
        const int R = ax.rad[s];
        if (R == 4)
            fft_stage<T, 4, FMAJOR, NT>(lds, ax.n, nfft, Ns, addr, tw64, tw32, sign);
        else if (R == 2)
            fft_stage<T, 2, FMAJOR, NT>(lds, ax.n, nfft, Ns, addr, tw64, tw32, sign);
        else if (R == 3)
            fft_stage<T, 3, FMAJOR, NT>(lds, ax.n, nfft, Ns, addr, tw64, tw32, sign);
        else
            fft_stage<T, 5, FMAJOR, NT>(lds, ax.n, nfft, Ns, addr, tw64, tw32, sign);
        Ns *= R;
    }
}

}  // namespace dpp
