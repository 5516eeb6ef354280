// Gaussian window weights and sorted-record accessors shared by P2G and G2P.
#pragma once

#include "internal.h"

namespace ewald {

constexpr int kMaxP = 16;

// Per-plan window constants for one precision: w0(u) = exp(-beta u^2) with u the
// distance to the particle in grid spacings, and ratio[j] = exp(-beta (2j + 1)).
template <typename T>
struct WinArgs {
    T beta;
    T ratio[kMaxP];
};

// The P weights of the stencil of a particle with fraction t = y/h - floor(y/h):
// w[j] = w0(j - (P/2 - 1) - t), j = 0..P-1 (grid points floor(y/h) - P/2 + 1 + j).
// Uses the recurrence w[j+1] = w[j] * exp(-beta (2j+1)) * exp(2 beta m0), m0 = P/2 - 1 + t
// (two exponentials per particle and axis instead of P; the fast Gaussian gridding
// factorisation).  The window's support is open: the point at distance exactly P h/2
// (t == 0, j = P-1) gets weight 0.
template <typename T, int P>
__device__ inline void window_weights(T t, const WinArgs<T>& wa, T* w)
{
    const T m0 = (T)(P / 2 - 1) + t;
    const T E = exp((T)2 * wa.beta * m0);
    w[0] = exp(-wa.beta * m0 * m0);
#pragma unroll
    for (int j = 0; j + 1 < P; ++j) w[j + 1] = w[j] * (wa.ratio[j] * E);
    if (t == (T)0) w[P - 1] = (T)0;
}

__device__ inline int wrapi(int a, int M) { return ((a % M) + M) % M; }
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
