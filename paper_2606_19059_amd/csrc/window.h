// Gaussian window weights and sorted-record accessors shared by P2G and G2P.
#pragma once

#include <cmath>

#include "internal.h"

namespace ewald {

constexpr int kKbDeg = 14;  // degree of the per-offset Kaiser-Bessel weight polynomials

// Per-plan window constants for one precision.  Gaussian: w0(u) = exp(-beta u^2) with u the
// distance to the particle in grid spacings (P2G evaluates it at consecutive points by the
// recurrence w0(u + 1) = w0(u) exp(-beta (2u + 1)), the fast Gaussian gridding factorisation).
// Kaiser-Bessel (kb != nullptr): kb[j * (kKbDeg + 1) + k] are the monomial coefficients, in
// s = 2t - 1, of the weight of stencil offset j as a function of the fraction t in [0, 1).
template <typename T>
struct WinArgs {
    T beta;
    const T* kb;
};

template <typename T>
__device__ inline T kb_weight(const T* __restrict__ c, T s)
{
    T q = c[kKbDeg];
#pragma unroll
    for (int k = kKbDeg - 1; k >= 0; --k) q = fma(q, s, c[k]);
    return q;
}

// The stencil of a particle with fraction t = y/h - floor(y/h) has the P grid points
// floor(y/h) - P/2 + 1 + j, j = 0..P-1, with weights w0(j - (P/2 - 1) - t).  The window's
// support is open: the point at distance exactly P h/2 (t == 0, j = P-1) gets weight 0.
// window_weight_one is the weight of one stencil offset j (0 <= j < P).
template <typename T, int P>
__device__ inline T window_weight_one(int j, T t, const WinArgs<T>& wa)
{
    T wv;
    if (wa.kb) {
        wv = kb_weight<T>(wa.kb + j * (kKbDeg + 1), (T)2 * t - (T)1);
    } else {
        const T uu = (T)(j - (P / 2 - 1)) - t;
        wv = exp(-wa.beta * uu * uu);
    }
    if (j == P - 1 && t == (T)0) wv = (T)0;  // open support
    return wv;
}

// Window constants of a plan in precision T (the KB table lives in the plan's device tables).
template <typename T>
inline WinArgs<T> make_win_args(const Plan& pl)
{
    WinArgs<T> wa;
    wa.beta = (T)pl.beta;
    wa.kb = nullptr;
    if (pl.window_kb) wa.kb = (const T*)(sizeof(T) == 8 ? (const void*)pl.d_kb64 : (const void*)pl.d_kb32);
    return wa;
}

// periodic wrap of a grid index; grid sizes are powers of two (checked when a plan is made)
__device__ inline int wrapi(int a, int M) { return a & (M - 1); }
__device__ inline int floor_div(int a, int b) { return (a >= 0) ? a / b : -((-a + b - 1) / b); }

// Cell, fraction and force of a sorted record, in the kernel's precision T.
template <typename T>
struct RecView;

template <>
struct RecView<double> {
    using Rec = Rec64;
    __device__ static inline void load(const Rec64& r, const Geometry& g, int c[3], double t[3], double f[3])
    {
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            c[d] = r.c[d];
            t[d] = r.x[d] / g.h[d] - (double)r.c[d];
            f[d] = r.f[d];
        }
    }
};

template <>
struct RecView<float> {
    using Rec = Rec64;
    __device__ static inline void load(const Rec64& r, const Geometry& g, int c[3], float t[3], float f[3])
    {
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            c[d] = r.c[d];
            t[d] = (float)(r.x[d] / g.h[d] - (double)r.c[d]);
            f[d] = (float)r.f[d];
        }
    }
};

}  // namespace ewald
