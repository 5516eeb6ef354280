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
        double a0 = 0, a1 = 0, a2 = 0;  // FP64 sums in every mode (see below)
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
                    const double wv = (double)(sw[0][ix] * wyz);
                    a0 += wv * (double)grid[idx];
                    a1 += wv * (double)grid[nc + idx];
                    a2 += wv * (double)grid[2 * nc + idx];
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


// All G2P sums accumulate in FP64 (FP32 bulk included: the same VALU rate without packed
// math).  The far field at a particle contains its own screened self-interaction, about
// (4 xi / sqrt(pi)) f, which the self term removes; at large xi (fine grids) and for sparse
// particles that cancellation is large, and FP32 partial sums would set an error floor.
//
// LDS-tiled G2P.  A block of four wavefronts takes kTileTargets consecutive cell-sorted
// targets (a compact group: sort order is tile-major with Morton columns inside a tile),
// stages the union of their P^3 stencils into LDS one grid component at a time (one pass
// over that region, coalesced along z, periodic wrap per element), and every target then
// gathers its stencil from LDS: each grid value read from L2 serves all targets whose
// stencils contain it, and the gathers run at LDS bandwidth.  A block whose region does not
// fit the LDS budget gathers directly from the grid instead (same arithmetic and order of
// summation within a target).  Weights: one lane per (target, axis, offset); partial sums
// reduced per wave with shuffles; lane q of the block writes target q's result.
constexpr int kTileTargets = 32;
constexpr int kTileWaves = 4;

template <typename T, typename TG, int P>
__global__ __launch_bounds__(kTileWaves * 64) void k_g2p_tile(int n, const Rec64* __restrict__ rec,
                                                             const TG* __restrict__ grid, Geometry g,
                                                             WinArgs<T> wa, double self_coef,
                                                             const double* __restrict__ u_near,
                                                             const double* __restrict__ f_in, double* __restrict__ u,
                                                             double* __restrict__ u_near_out,
                                                             double* __restrict__ u_far_out, int max_points)
{
    extern __shared__ unsigned char smem_raw[];
    TG* reg = reinterpret_cast<TG*>(smem_raw);
    __shared__ T sw[kTileTargets][3][P];
    __shared__ int anc[kTileTargets][3];
    __shared__ double res[kTileTargets][3];
    __shared__ int lo_s[3], hi_s[3];
    constexpr int kPass = (P * P + kWave - 1) / kWave;
    const int tid = threadIdx.x, lane = tid & (kWave - 1), wid = tid / kWave;
    const int s0 = xcd_remap((int)blockIdx.x, (int)gridDim.x) * kTileTargets;
    const int cnt = min(kTileTargets, n - s0);
    const int M1 = g.M[0], M2 = g.M[1], M3 = g.M[2];
    const int64_t nc = g.ncells;
    if (tid < 3) {
        lo_s[tid] = 0x7fffffff;
        hi_s[tid] = -0x7fffffff;
    }
    __syncthreads();
    if (tid < cnt) {
        const Rec64& r = rec[s0 + tid];
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            const int a = r.c[d] - P / 2 + 1;  // stencil anchor (unwrapped)
            anc[tid][d] = a;
            atomicMin(&lo_s[d], a);
            atomicMax(&hi_s[d], a);
        }
    }
    for (int k = tid; k < cnt * 3 * P; k += kTileWaves * kWave) {
        const int q = k / (3 * P), d = (k / P) % 3, j = k % P;
        int c[3];
        T t[3], f[3];
        RecView<T>::load(rec[s0 + q], g, c, t, f);
        const T td = (d == 0) ? t[0] : (d == 1 ? t[1] : t[2]);
        sw[q][d][j] = window_weight_one<T, P>(j, td, wa);
    }
    __syncthreads();
    const int E0 = hi_s[0] - lo_s[0] + P, E1 = hi_s[1] - lo_s[1] + P, E2 = hi_s[2] - lo_s[2] + P;
    const int E12 = E1 * E2;
    const int tot = E0 * E12;
    if ((int64_t)3 * tot <= max_points) {
        // the three components fit together: one staging pass, one gather per target
        for (int idx = tid; idx < tot; idx += kTileWaves * kWave) {
            const int ix = idx / E12, rem = idx - ix * E12;
            const int iy = rem / E2, iz = rem - iy * E2;
            const int64_t gi = ((int64_t)wrapi(lo_s[0] + ix, M1) * M2 + wrapi(lo_s[1] + iy, M2)) * M3 +
                               wrapi(lo_s[2] + iz, M3);
            reg[idx] = grid[gi];
            reg[tot + idx] = grid[nc + gi];
            reg[2 * tot + idx] = grid[2 * nc + gi];
        }
        __syncthreads();
        for (int q = wid; q < cnt; q += kTileWaves) {
            const int ox = anc[q][0] - lo_s[0], oy = anc[q][1] - lo_s[1], oz = anc[q][2] - lo_s[2];
            T wx[P];
#pragma unroll
            for (int ix = 0; ix < P; ++ix) wx[ix] = sw[q][0][ix];
            double a0 = 0, a1 = 0, a2 = 0;  // FP64 sums in every mode (see below)
#pragma unroll
            for (int pass = 0; pass < kPass; ++pass) {
                const int yz = pass * kWave + lane;
                if (yz < P * P) {
                    const int jy = yz / P, kz = yz - jy * P;
                    const T wyz = sw[q][1][jy] * sw[q][2][kz];
                    const TG* rp = reg + ox * E12 + (oy + jy) * E2 + oz + kz;
#pragma unroll
                    for (int ix = 0; ix < P; ++ix) {
                        const double wv = (double)(wx[ix] * wyz);
                        a0 += wv * (double)rp[ix * E12];
                        a1 += wv * (double)rp[tot + ix * E12];
                        a2 += wv * (double)rp[2 * tot + ix * E12];
                    }
                }
            }
            const double b0 = wave_sum((double)a0), b1 = wave_sum((double)a1), b2 = wave_sum((double)a2);
            if (lane == 0) {
                res[q][0] = b0;
                res[q][1] = b1;
                res[q][2] = b2;
            }
        }
        __syncthreads();
    } else if (tot <= max_points) {
        for (int comp = 0; comp < 3; ++comp) {
            const TG* gc = grid + comp * nc;
            for (int idx = tid; idx < tot; idx += kTileWaves * kWave) {
                const int ix = idx / E12, rem = idx - ix * E12;
                const int iy = rem / E2, iz = rem - iy * E2;
                const int gx = wrapi(lo_s[0] + ix, M1), gy = wrapi(lo_s[1] + iy, M2), gz = wrapi(lo_s[2] + iz, M3);
                reg[idx] = gc[((int64_t)gx * M2 + gy) * M3 + gz];
            }
            __syncthreads();
            for (int q = wid; q < cnt; q += kTileWaves) {
                const int ox = anc[q][0] - lo_s[0], oy = anc[q][1] - lo_s[1], oz = anc[q][2] - lo_s[2];
                T wx[P];
#pragma unroll
                for (int ix = 0; ix < P; ++ix) wx[ix] = sw[q][0][ix];
                double acc = 0;
#pragma unroll
                for (int pass = 0; pass < kPass; ++pass) {
                    const int yz = pass * kWave + lane;
                    if (yz < P * P) {
                        const int jy = yz / P, kz = yz - jy * P;
                        const T wyz = sw[q][1][jy] * sw[q][2][kz];
                        const TG* rp = reg + ox * E12 + (oy + jy) * E2 + oz + kz;
#pragma unroll
                        for (int ix = 0; ix < P; ++ix) acc += (double)(wx[ix] * wyz) * (double)rp[ix * E12];
                    }
                }
                const double s = wave_sum((double)acc);
                if (lane == 0) res[q][comp] = s;
            }
            __syncthreads();
        }
    } else {
        for (int q = wid; q < cnt; q += kTileWaves) {
            double a0 = 0, a1 = 0, a2 = 0;  // FP64 sums in every mode (see below)
#pragma unroll
            for (int pass = 0; pass < kPass; ++pass) {
                const int yz = pass * kWave + lane;
                if (yz < P * P) {
                    const int jy = yz / P, kz = yz - jy * P;
                    const T wyz = sw[q][1][jy] * sw[q][2][kz];
                    const int64_t col = (int64_t)wrapi(anc[q][1] + jy, M2) * M3 + wrapi(anc[q][2] + kz, M3);
                    for (int ix = 0; ix < P; ++ix) {
                        const int64_t idx = (int64_t)wrapi(anc[q][0] + ix, M1) * M2 * M3 + col;
                        const double wv = (double)(sw[q][0][ix] * wyz);
                        a0 += wv * (double)grid[idx];
                        a1 += wv * (double)grid[nc + idx];
                        a2 += wv * (double)grid[2 * nc + idx];
                    }
                }
            }
            const double b0 = wave_sum((double)a0), b1 = wave_sum((double)a1), b2 = wave_sum((double)a2);
            if (lane == 0) {
                res[q][0] = b0;
                res[q][1] = b1;
                res[q][2] = b2;
            }
        }
        __syncthreads();
    }
    if (tid < cnt) {
        const int s = s0 + tid;
        const int orig = rec[s].orig;
        const int64_t nn = n;
        const double n0 = u_near[s], n1 = u_near[nn + s], n2 = u_near[2 * nn + s];
        if (u) {
            u[orig] = n0 + res[tid][0] - self_coef * f_in[orig];
            u[nn + orig] = n1 + res[tid][1] - self_coef * f_in[nn + orig];
            u[2 * nn + orig] = n2 + res[tid][2] - self_coef * f_in[2 * nn + orig];
        } else {
            u_near_out[orig] = n0;
            u_near_out[nn + orig] = n1;
            u_near_out[2 * nn + orig] = n2;
            u_far_out[orig] = res[tid][0];
            u_far_out[nn + orig] = res[tid][1];
            u_far_out[2 * nn + orig] = res[tid][2];
        }
    }
}

template <typename T, typename TG, int P>
hipError_t launch_g2p_t(const Plan& pl, const Work& w, int n, const double* f, double* u, double* un,
                        double* uf, hipStream_t s)
{
    const double self_coef = 4.0 * pl.xi / sqrt(M_PI);
    // LDS-tiled kernel (region budget: what a workgroup may use beyond its static arrays, at
    // most half of a CU's 160 KB so that two blocks share a CU) for grids above half of the
    // 256 MB Infinity Cache, where the direct gathers of neighbouring targets stop hitting the
    // on-chip caches (measured: c4's 201 MB grid 28.9 -> 19.8 ms); below that the
    // one-wave-per-target kernel's cache hits beat the staging (a 25 MB FP32 grid: 2.6 vs 2.9 ms)
    const int static_bytes = (int)(sizeof(T) * kTileTargets * 3 * P + (sizeof(int) * 3 + sizeof(double) * 3) *
                                   kTileTargets + 64);
    const int budget = std::min(pl.lds_per_block, 80 * 1024) - static_bytes;
    const int max_points = budget / (int)sizeof(TG);
    const double grid_bytes = 3.0 * (double)pl.g.ncells * (double)sizeof(TG);
    if (max_points >= P * P * P && grid_bytes > 128.0 * (1 << 20)) {
        hipLaunchKernelGGL((k_g2p_tile<T, TG, P>), dim3((n + kTileTargets - 1) / kTileTargets),
                           dim3(kTileWaves * kWave), (size_t)max_points * sizeof(TG), s, n, (const Rec64*)w.rec,
                           (const TG*)w.grid, pl.g, make_win_args<T>(pl), self_coef, w.u_near, f, u, un, uf,
                           max_points);
        return hipGetLastError();
    }
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
