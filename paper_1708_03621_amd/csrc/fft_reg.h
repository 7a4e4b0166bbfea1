// Mixed-radix (2,3,4,5) FFT of a length-N column held entirely in one
// thread's registers, N known at compile time.
//
// Decimation in frequency (natural-order input, digit-reversed output) and
// decimation in time (digit-reversed input, natural-order output), both in
// place.  For the radix sequence R_0, R_1, ... (4s, then 2s, 3s, 5s) stage s
// works on blocks of length n_s = N / (R_0 ... R_{s-1}) with span
// S = n_s / R_s: butterfly (block base, j < S) takes x[base + j + r S],
// r < R_s.  DIF applies the length-R_s DFT and then the twiddles
// w^{(N/n_s) r j}; DIT applies the twiddles first and runs the stages in
// reverse order.  With opposite signs, DIT(-) after DIF(+) is N times the
// identity, so a pointwise operation in the transformed (real-space) domain
// needs no reordering: register p holds the point digit_rev(p).
// Twiddles w[m] = exp(-2 pi i m / N) (conjugated for sign > 0) are
// compile-time constants: an exact rational octant reduction of the angle and
// Taylor series of sin and cos on [0, pi/4] evaluated in constant expressions.
#pragma once

#include <hip/hip_runtime.h>

#include "fft_engine.h"

namespace dpp {

constexpr int reg_num_radices(int n) {
    int k = 0;
    while (n % 4 == 0) n /= 4, ++k;
    while (n % 2 == 0) n /= 2, ++k;
    while (n % 3 == 0) n /= 3, ++k;
    while (n % 5 == 0) n /= 5, ++k;
    return n == 1 ? k : -1;
}

constexpr int reg_radix(int n, int s) {
    int k = 0;
    while (n % 4 == 0) {
        if (k == s) return 4;
        n /= 4, ++k;
    }
    while (n % 2 == 0) {
        if (k == s) return 2;
        n /= 2, ++k;
    }
    while (n % 3 == 0) {
        if (k == s) return 3;
        n /= 3, ++k;
    }
    while (n % 5 == 0) {
        if (k == s) return 5;
        n /= 5, ++k;
    }
    return 1;
}

// Block length at stage s: N divided by the radices of the stages before it.
constexpr int reg_block(int n, int s) {
    int b = n;
    for (int i = 0; i < s; ++i) b /= reg_radix(n, i);
    return b;
}

// Point held by register p after DIF: the digits of p (most significant
// first, radices R_0, R_1, ...) read with R_0 as the least significant digit.
constexpr int reg_digit_rev(int n, int p) {
    int k = 0, m = 1, rem = p, blk = n;
    const int ns = reg_num_radices(n);
    for (int s = 0; s < ns; ++s) {
        const int R = reg_radix(n, s);
        blk /= R;
        const int d = rem / blk;
        rem -= d * blk;
        k += d * m;
        m *= R;
    }
    return k;
}

// sin and cos of x in [0, pi/4] by Taylor series (16 terms: the truncation
// error is below 1e-30 there).
constexpr void reg_sincos_small(double x, double& s, double& c) {
    double ts = x, tc = 1.0;
    s = x;
    c = 1.0;
    for (int k = 1; k < 16; ++k) {
        ts *= -x * x / ((2.0 * k) * (2.0 * k + 1.0));
        tc *= -x * x / ((2.0 * k - 1.0) * (2.0 * k));
        s += ts;
        c += tc;
    }
}

// exp(-2 pi i m / n): the angle 2 pi m / n = (pi / 4) (8m / n) is split into an
// octant o = floor(8m / n) and a remainder fraction r = (8m mod n) / n, both
// exact; sin and cos of (pi/4) r (or of (pi/4)(1 - r) in odd octants) then
// give the value by octant symmetry.
struct RegCs {
    double c, s;
};
constexpr RegCs reg_cis(int m, int n) {
    const long q = 8L * (m % n);
    const int o = (int)(q / n);
    const long rem = q % n;
    const double quarter = 0.78539816339744830962;  // pi / 4
    double sa = 0, ca = 0;
    if (o % 2 == 0)
        reg_sincos_small(quarter * ((double)rem / n), sa, ca);
    else
        reg_sincos_small(quarter * ((double)(n - rem) / n), sa, ca);
    // (cos t, sin t) for t = (pi/4)(o + r)
    double c = 0, s = 0;
    switch (o) {
        case 0: c = ca, s = sa; break;            // t = a
        case 1: c = sa, s = ca; break;            // t = pi/2 - a
        case 2: c = -sa, s = ca; break;           // t = pi/2 + a
        case 3: c = -ca, s = sa; break;           // t = pi - a
        case 4: c = -ca, s = -sa; break;          // t = pi + a
        case 5: c = -sa, s = -ca; break;          // t = 3pi/2 - a
        case 6: c = sa, s = -ca; break;           // t = 3pi/2 + a
        default: c = ca, s = -sa; break;          // t = 2pi - a
    }
    return RegCs{c, -s};  // exp(-i t)
}

template <int N>
struct RegTw {
    double re[N], im[N];
    constexpr RegTw() : re(), im() {
        for (int m = 0; m < N; ++m) {
            const RegCs w = reg_cis(m, N);
            re[m] = w.c;
            im[m] = w.s;
        }
    }
};

template <typename T, int N>
__device__ __forceinline__ typename cx<T>::t reg_twiddle(int m, int sign) {
    constexpr RegTw<N> tw{};
    using C = typename cx<T>::t;
    const double re = tw.re[m], im = tw.im[m];
    return C{(T)re, (T)(sign > 0 ? -im : im)};
}

// SER: the butterflies run one after another: each one's inputs and outputs
// pass through an empty volatile asm (a data dependency the compiler keeps in
// order), so the butterflies of a stage are not interleaved (for long
// transforms, whose interleaved temporaries would not fit the register file
// next to the column).
template <typename C>
__device__ __forceinline__ void reg_pin(C& v) {
    asm volatile("" : "+v"(v.x), "+v"(v.y));
}

template <typename T, int N, int SIGN, int STAGE, bool SER = false>
__device__ __forceinline__ void reg_dif(typename cx<T>::t* x, const double2* tw64, const float2* tw32) {
    using C = typename cx<T>::t;
    if constexpr (STAGE < reg_num_radices(N)) {
        constexpr int R = reg_radix(N, STAGE);
        constexpr int n = reg_block(N, STAGE);
        constexpr int S = n / R;
#pragma unroll
        for (int base = 0; base < N; base += n) {
#pragma unroll
            for (int j = 0; j < S; ++j) {
                C v[R];
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    v[r] = x[base + j + r * S];
                    if constexpr (SER) reg_pin(v[r]);
                }
                Dft<T, R>::run(v, SIGN);
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    const int m = ((N / n) * r * j) % N;
                    x[base + j + r * S] = m == 0 ? v[r] : cmul(v[r], reg_twiddle<T, N>(m, SIGN));
                    if constexpr (SER) reg_pin(x[base + j + r * S]);
                }
            }
        }
        reg_dif<T, N, SIGN, STAGE + 1, SER>(x, tw64, tw32);
    }
}

template <typename T, int N, int SIGN, int STAGE, bool SER = false>
__device__ __forceinline__ void reg_dit(typename cx<T>::t* x, const double2* tw64, const float2* tw32) {
    using C = typename cx<T>::t;
    if constexpr (STAGE < reg_num_radices(N)) {
        reg_dit<T, N, SIGN, STAGE + 1, SER>(x, tw64, tw32);
        constexpr int R = reg_radix(N, STAGE);
        constexpr int n = reg_block(N, STAGE);
        constexpr int S = n / R;
#pragma unroll
        for (int base = 0; base < N; base += n) {
#pragma unroll
            for (int j = 0; j < S; ++j) {
                C v[R];
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    const int m = ((N / n) * r * j) % N;
                    C a = x[base + j + r * S];
                    if constexpr (SER) reg_pin(a);
                    v[r] = m == 0 ? a : cmul(a, reg_twiddle<T, N>(m, SIGN));
                }
                Dft<T, R>::run(v, SIGN);
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    x[base + j + r * S] = v[r];
                    if constexpr (SER) reg_pin(x[base + j + r * S]);
                }
            }
        }
    }
}

// Point held at position p of an axis after decimation in frequency, for a
// runtime axis plan (same radix order as the compile-time plan).
__device__ __forceinline__ int digit_rev_axis(const FftAxis& ax, int p) {
    int blk = ax.n, k = 0, m = 1;
    for (int s = 0; s < ax.nrad; ++s) {
        const int R = ax.rad[s];
        blk /= R;
        const int d = p / blk;
        p -= d * blk;
        k += d * m;
        m *= R;
    }
    return k;
}

}  // namespace dpp
