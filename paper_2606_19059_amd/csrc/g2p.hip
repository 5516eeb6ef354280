// G2P + SUM: interpolation of the far-field grid back to the particles, eq. (g2p),
//   u^F(x_i) = h1 h2 h3 sum_l w(x_i - g_l + p) v(g_l)
// (the h^3 factor is folded into the CNV scaling, so here it is a plain weighted sum),
// then u_i = u^N_i + u^F_i - (4 xi/sqrt(pi)) f_i (Algorithm "se", SUM step, with the
// self-term correction), scattered back to the caller's particle order.
//
// A wavefront gathers one target's P^3 stencil cooperatively (see k_g2p); consecutive
// targets of a wave are cell-sorted neighbours, so their stencils overlap in L1.  No
// atomics: each target's sum is owned by one wave.
#include "window.h"

namespace ewald {

namespace {

template <typename T>
__device__ inline T wave_sum(T v)
{
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, kWave);
    return v;
}

// One wavefront per group of kG2PPerWave consecutive (cell-sorted) targets, one target at
// a time: lane l covers footprint points (y, z) = (l / P, l % P) (+ 64 per pass) and walks
// the P points along x; z is fastest, so each load instruction reads runs of P consecutive
// grid values (a few cache lines for the whole wave).  The 1D weights of the current
// target are computed once (one lane per weight) and shared through LDS; the wave's
// partial sums are reduced with shuffles, and lane 0 writes the result.
constexpr int kG2PPerWave = 16;

template <typename T, typename TG, int P>
__global__ __launch_bounds__(64) void k_g2p(int n, const typename RecView<T>::Rec* __restrict__ rec,
                                            const TG* __restrict__ grid, Geometry g, WinArgs<T> wa,
                                            double self_coef, const double* __restrict__ u_near,
                                            const double* __restrict__ f_in, double* __restrict__ u,
                                            double* __restrict__ u_near_out,
                                            double* __restrict__ u_far_out)
{
    constexpr int kPass = (P * P + kWave - 1) / kWave;
    __shared__ T sw[3][P];
    const int lane = threadIdx.x;
    const int M1 = g.M[0], M2 = g.M[1], M3 = g.M[2];
    const int64_t nc = g.ncells;
    const int64_t nn = n;
    const int s0 = xcd_remap((int)blockIdx.x, (int)gridDim.x) * kG2PPerWave;
    const int s1 = min(s0 + kG2PPerWave, n);
    for (int s = s0; s < s1; ++s) {
        const auto& r = rec[s];
        int c[3];
        T t[3], f[3];
        RecView<T>::load(r, g, c, t, f);
        if (lane < 3 * P) {
            const int d = lane / P, j = lane - d * P;
            const T td = (d == 0) ? t[0] : (d == 1 ? t[1] : t[2]);
            sw[d][j] = window_weight_one<T, P>(j, td, wa);
        }
        __syncthreads();
        TG a0 = 0, a1 = 0, a2 = 0;
#pragma unroll
        for (int pass = 0; pass < kPass; ++pass) {
            const int yz = pass * kWave + lane;
            if (yz < P * P) {
                const int jy = yz / P, kz = yz - jy * P;
                const T wyz = sw[1][jy] * sw[2][kz];
                const int gy = wrapi(c[1] - P / 2 + 1 + jy, M2);
                const int gz = wrapi(c[2] - P / 2 + 1 + kz, M3);
                const int64_t col = (int64_t)gy * M3 + gz;
                for (int ix = 0; ix < P; ++ix) {
                    const int gx = wrapi(c[0] - P / 2 + 1 + ix, M1);
                    const int64_t idx = (int64_t)gx * M2 * M3 + col;
                    const TG wv = sw[0][ix] * wyz;
                    a0 += wv * grid[idx];
                    a1 += wv * grid[nc + idx];
                    a2 += wv * grid[2 * nc + idx];
                }
            }
        }
        const double b0 = wave_sum((double)a0), b1 = wave_sum((double)a1), b2 = wave_sum((double)a2);
        if (lane == 0) {
            const int orig = r.orig;
            const double n0 = u_near[s], n1 = u_near[nn + s], n2 = u_near[2 * nn + s];
            if (u) {
                u[orig] = n0 + b0 - self_coef * f_in[orig];
                u[nn + orig] = n1 + b1 - self_coef * f_in[nn + orig];
                u[2 * nn + orig] = n2 + b2 - self_coef * f_in[2 * nn + orig];
            } else {
                u_near_out[orig] = n0;
                u_near_out[nn + orig] = n1;
                u_near_out[2 * nn + orig] = n2;
                u_far_out[orig] = b0;
                u_far_out[nn + orig] = b1;
                u_far_out[2 * nn + orig] = b2;
            }
        }
        __syncthreads();
    }
}


template <typename T, typename TG, int P>
hipError_t launch_g2p_t(const Plan& pl, const Work& w, int n, const double* f, double* u, double* un,
                        double* uf, hipStream_t s)
{
    const double self_coef = 4.0 * pl.xi / sqrt(M_PI);
    hipLaunchKernelGGL((k_g2p<T, TG, P>), dim3((n + kG2PPerWave - 1) / kG2PPerWave), dim3(kWave), 0, s, n,
                       (const typename RecView<T>::Rec*)w.rec, (const TG*)w.grid, pl.g, make_win_args<T>(pl),
                       self_coef, w.u_near, f, u, un, uf);
    return hipGetLastError();
}

template <typename T, typename TG>
hipError_t launch_g2p_p(const Plan& pl, const Work& w, int n, const double* f, double* u, double* un,
                        double* uf, hipStream_t s)
{
    switch (pl.P) {
    case 4: return launch_g2p_t<T, TG, 4>(pl, w, n, f, u, un, uf, s);
    case 6: return launch_g2p_t<T, TG, 6>(pl, w, n, f, u, un, uf, s);
    case 8: return launch_g2p_t<T, TG, 8>(pl, w, n, f, u, un, uf, s);
    case 10: return launch_g2p_t<T, TG, 10>(pl, w, n, f, u, un, uf, s);
    case 12: return launch_g2p_t<T, TG, 12>(pl, w, n, f, u, un, uf, s);
    case 14: return launch_g2p_t<T, TG, 14>(pl, w, n, f, u, un, uf, s);
    case 16: return launch_g2p_t<T, TG, 16>(pl, w, n, f, u, un, uf, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace

hipError_t launch_g2p(const Plan& pl, const Work& w, int n, const double* f, double* u,
                      double* u_near_out, double* u_far_out, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    if (pl.mode == EWALD_FP64) return launch_g2p_p<double, double>(pl, w, n, f, u, u_near_out, u_far_out, s);
    if (pl.grid64) return launch_g2p_p<float, double>(pl, w, n, f, u, u_near_out, u_far_out, s);
    return launch_g2p_p<float, float>(pl, w, n, f, u, u_near_out, u_far_out, s);
}

}  // namespace ewald
