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
// Twiddles come from the per-axis table w[m] = exp(-2 pi i m / N) (conjugated
// for sign > 0) at compile-time indices: uniform scalar loads.
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

template <typename T, int N, int SIGN, int STAGE>
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
                for (int r = 0; r < R; ++r) v[r] = x[base + j + r * S];
                Dft<T, R>::run(v, SIGN);
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    const int m = ((N / n) * r * j) % N;
                    x[base + j + r * S] = m == 0 ? v[r] : cmul(v[r], twiddle<T>(tw64, tw32, m, SIGN));
                }
            }
        }
        reg_dif<T, N, SIGN, STAGE + 1>(x, tw64, tw32);
    }
}

template <typename T, int N, int SIGN, int STAGE>
__device__ __forceinline__ void reg_dit(typename cx<T>::t* x, const double2* tw64, const float2* tw32) {
    using C = typename cx<T>::t;
    if constexpr (STAGE < reg_num_radices(N)) {
        reg_dit<T, N, SIGN, STAGE + 1>(x, tw64, tw32);
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
                    const C a = x[base + j + r * S];
                    v[r] = m == 0 ? a : cmul(a, twiddle<T>(tw64, tw32, m, SIGN));
                }
                Dft<T, R>::run(v, SIGN);
#pragma unroll
                for (int r = 0; r < R; ++r) x[base + j + r * S] = v[r];
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
