// G2P + SUM: interpolation of the far-field grid back to the particles, eq. (g2p),
//   u^F(x_i) = h1 h2 h3 sum_l w(x_i - g_l + p) v(g_l)
// (the h^3 factor is folded into the CNV scaling, so here it is a plain weighted sum),
// then u_i = u^N_i + u^F_i - (4 xi/sqrt(pi)) f_i (Algorithm "se", SUM step, with the
// self-term correction), scattered back to the caller's particle order.
//
// One lane per target in cell-sorted order, so a wave's 64 targets are spatially close
// and their P^3 stencils overlap in the L1/L2 caches.  No atomics: each lane owns its
// target.  The far field is accumulated in FP64 in both precision modes.
#include "window.h"

namespace ewald {

namespace {

template <typename T, int P>
__global__ __launch_bounds__(256) void k_g2p(int n, const typename RecView<T>::Rec* __restrict__ rec,
                                             const T* __restrict__ grid, Geometry g, WinArgs<T> wa,
                                             double self_coef, const double* __restrict__ u_near,
                                             const double* __restrict__ f_in, double* __restrict__ u,
                                             double* __restrict__ u_near_out,
                                             double* __restrict__ u_far_out)
{
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    const auto& r = rec[s];
    int c[3];
    T t[3], f[3];
    RecView<T>::load(r, g, c, t, f);
    const int orig = r.orig;
    T wx[P], wy[P], wz[P];
    window_weights<T, P>(t[0], wa, wx);
    window_weights<T, P>(t[1], wa, wy);
    window_weights<T, P>(t[2], wa, wz);
    const int M1 = g.M[0], M2 = g.M[1], M3 = g.M[2];
    int iz[P];
#pragma unroll
    for (int k = 0; k < P; ++k) iz[k] = wrapi(c[2] - P / 2 + 1 + k, M3);
    const int64_t nc = g.ncells;
    double a0 = 0.0, a1 = 0.0, a2 = 0.0;
    for (int i = 0; i < P; ++i) {
        const int gx = wrapi(c[0] - P / 2 + 1 + i, M1);
        T b0 = 0, b1 = 0, b2 = 0;
        for (int j = 0; j < P; ++j) {
            const int gy = wrapi(c[1] - P / 2 + 1 + j, M2);
            const int64_t row = ((int64_t)gx * M2 + gy) * M3;
            T s0 = 0, s1 = 0, s2 = 0;
#pragma unroll
            for (int k = 0; k < P; ++k) {
                const int64_t idx = row + iz[k];
                s0 += wz[k] * grid[idx];
                s1 += wz[k] * grid[nc + idx];
                s2 += wz[k] * grid[2 * nc + idx];
            }
            b0 += wy[j] * s0;
            b1 += wy[j] * s1;
            b2 += wy[j] * s2;
        }
        a0 += (double)(wx[i] * b0);
        a1 += (double)(wx[i] * b1);
        a2 += (double)(wx[i] * b2);
    }
    const int64_t nn = n;
    const double n0 = u_near[s], n1 = u_near[nn + s], n2 = u_near[2 * nn + s];
    if (u) {
        u[orig] = n0 + a0 - self_coef * f_in[orig];
        u[nn + orig] = n1 + a1 - self_coef * f_in[nn + orig];
        u[2 * nn + orig] = n2 + a2 - self_coef * f_in[2 * nn + orig];
    } else {
        u_near_out[orig] = n0;
        u_near_out[nn + orig] = n1;
        u_near_out[2 * nn + orig] = n2;
        u_far_out[orig] = a0;
        u_far_out[nn + orig] = a1;
        u_far_out[2 * nn + orig] = a2;
    }
}

template <typename T>
WinArgs<T> win_args(const Plan& pl)
{
    WinArgs<T> wa;
    wa.beta = (T)pl.beta;
    for (int j = 0; j < kMaxP; ++j) wa.ratio[j] = (T)exp(-pl.beta * (2.0 * j + 1.0));
    return wa;
}

template <typename T, int P>
hipError_t launch_g2p_t(const Plan& pl, const Work& w, int n, const double* f, double* u, double* un,
                        double* uf, hipStream_t s)
{
    const double self_coef = 4.0 * pl.xi / sqrt(M_PI);
    hipLaunchKernelGGL((k_g2p<T, P>), dim3((n + 255) / 256), dim3(256), 0, s, n,
                       (const typename RecView<T>::Rec*)w.rec, (const T*)w.grid, pl.g, win_args<T>(pl),
                       self_coef, w.u_near, f, u, un, uf);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_g2p_p(const Plan& pl, const Work& w, int n, const double* f, double* u, double* un,
                        double* uf, hipStream_t s)
{
    switch (pl.P) {
    case 4: return launch_g2p_t<T, 4>(pl, w, n, f, u, un, uf, s);
    case 6: return launch_g2p_t<T, 6>(pl, w, n, f, u, un, uf, s);
    case 8: return launch_g2p_t<T, 8>(pl, w, n, f, u, un, uf, s);
    case 10: return launch_g2p_t<T, 10>(pl, w, n, f, u, un, uf, s);
    case 12: return launch_g2p_t<T, 12>(pl, w, n, f, u, un, uf, s);
    case 14: return launch_g2p_t<T, 14>(pl, w, n, f, u, un, uf, s);
    case 16: return launch_g2p_t<T, 16>(pl, w, n, f, u, un, uf, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace

hipError_t launch_g2p(const Plan& pl, const Work& w, int n, const double* f, double* u,
                      double* u_near_out, double* u_far_out, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    if (pl.mode == EWALD_FP64) return launch_g2p_p<double>(pl, w, n, f, u, u_near_out, u_far_out, s);
    return launch_g2p_p<float>(pl, w, n, f, u, u_near_out, u_far_out, s);
}

}  // namespace ewald
