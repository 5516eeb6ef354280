// G2P + SUM: interpolation of the far-field grid back to the particles, eq. (g2p),
//   u^F(x_i) = h1 h2 h3 sum_l w(x_i - g_l + p) v(g_l)
// (the h^3 factor is folded into the CNV scaling, so here it is a plain weighted sum),
// then u_i = u^N_i + u^F_i - (4 xi/sqrt(pi)) f_i (Algorithm "se", SUM step, with the
// self-term correction), scattered back to the caller's particle order.
//
// A wavefront gathers the P^3 stencils of 16 consecutive cell-sorted targets together
// (see k_g2p): neighbouring stencils overlap, so each grid line fetched into L1 serves
// several targets.  No atomics: each target's sum is owned by four lanes of one wave.
// All sums accumulate in FP64 (FP32 bulk included: the same VALU rate without packed
// math).  The far field at a particle contains its own screened self-interaction, about
// (4 xi / sqrt(pi)) f, which the self term removes; at large xi (fine grids) and for sparse
// particles that cancellation is large, and FP32 partial sums would set an error floor.
#include "window.h"

namespace ewald {

namespace {

// One wavefront per group of consecutive (cell-sorted) targets, all at once: 16 targets of
// four lanes each for FP64 grids, 32 of two lanes for FP32 grids (measured fastest: FP64 at
// P = 16 and 14 with 16, FP32 at P = 12 and 10 with 32).  A lane item is a footprint row y
// and a run of V consecutive z (one 16-byte load per item and x-plane, 8-byte for FP32
// grids whose P is not a multiple of 4); the lanes of a target step through its P * P / V
// items and walk the P x-planes of each.  The wave's loads of one step touch the union of
// the group's neighbouring footprints, which is a small multiple of one footprint
// (measured at N = 1e6, 128^3, FP64, P = 16: 5.8 ms with one target per wave at a time,
// 3.3 ms with 16).  The 3 x P 1D weights of every target are computed once (one lane per
// weight) and shared through LDS; each target's partial sums are reduced with shuffles.
template <typename TG>
constexpr int g2p_per_wave() { return sizeof(TG) == 4 ? 32 : 16; }

// V consecutive grid values.  Runs start at any element, so the alignment is only that of
// the element; gfx950 global loads accept such multi-dword accesses (the compiler emits
// one 16-byte load for these types).
template <typename TG, int V>
struct GVec;
template <>
struct GVec<double, 2> {
    typedef double type __attribute__((ext_vector_type(2), aligned(8)));
};
template <>
struct GVec<float, 2> {
    typedef float type __attribute__((ext_vector_type(2), aligned(4)));
};
template <>
struct GVec<float, 4> {
    typedef float type __attribute__((ext_vector_type(4), aligned(4)));
};


template <typename T, typename TG, int P>
__global__ __launch_bounds__(64) void k_g2p(int n, const typename RecView<T>::Rec* __restrict__ rec,
                                            const TG* __restrict__ grid, Geometry g, WinArgs<T> wa,
                                            double self_coef, const double* __restrict__ u_near,
                                            const double* __restrict__ f_in, double* __restrict__ u,
                                            double* __restrict__ u_near_out,
                                            double* __restrict__ u_far_out, Batch bt)
{
    // lane items: (footprint row y, run of V consecutive z) -- one 16-byte (8-byte for FP32
    // grids with P not a multiple of 4) load per item and x-plane
    constexpr int V = (sizeof(TG) == 8 || P % 4 != 0) ? 2 : 4;
    constexpr int G = P / V;
    constexpr int kItems = P * G;
    constexpr int kG2PGroup = g2p_per_wave<TG>();  // targets gathered together
    constexpr int kG2PLanes = kWave / kG2PGroup;   // lanes per target
    constexpr int kPass = (kItems + kG2PLanes - 1) / kG2PLanes;
    // x-planes per batch of loads: a divisor of P, 4 where P allows it, else the largest odd
    // divisor up to 7 (more loads in flight: P = 14 measured 6% faster with 7 than with 2)
    constexpr int kU = (P % 4 == 0) ? 4 : (P % 7 == 0) ? 7 : (P % 5 == 0) ? 5 : (P % 3 == 0) ? 3 : 2;
    using VT = typename GVec<TG, V>::type;
    __shared__ T sw[kG2PGroup][3][P];
    __shared__ int anc[kG2PGroup][3];
    const int lane = threadIdx.x;
    const int q = lane / kG2PLanes, ql = lane % kG2PLanes;  // target of the group, lane within it
    static_assert(kWave % kG2PGroup == 0, "whole groups of lanes");
    const int M1 = g.M[0], M2 = g.M[1], M3 = g.M[2];
    const int64_t nc = g.ncells;
    // 32-bit offsets within one component (at most 512^3 points)
    const unsigned plane = (unsigned)M2 * (unsigned)M3;
    const int64_t nn = n;
    const T e2 = exp((T)-2 * wa.beta);  // ratio of consecutive Gaussian recurrence factors
    const int s0 = xcd_remap((int)blockIdx.x, (int)gridDim.x) * kG2PGroup;
    const int s1 = min(s0 + kG2PGroup, n);
    for (int sg = s0; sg < s1; sg += kG2PGroup) {
        // weights and stencil anchors of the group's targets (missing targets repeat the last)
        if (sizeof(T) == 8 && !wa.kb) {
            // FP64 Gaussian: two lanes per (target, axis), each walking P/2 weights away from
            // the peak by the recurrence w(u + s) = w(u) exp(-beta (2 s u + 1)), s = -1 for
            // offsets P/2-1 down to 0 and s = +1 for P/2 up to P-1 (two exponentials per lane)
            for (int k = lane; k < kG2PGroup * 6; k += kWave) {
                const int qq = k / 6, d = (k >> 1) % 3, up = k & 1;
                int c[3];
                T t[3], f[3];
                RecView<T>::load(rec[min(sg + qq, s1 - 1)], g, c, t, f);
                const T td = (d == 0) ? t[0] : (d == 1 ? t[1] : t[2]);
                const T sgn = up ? (T)1 : (T)-1;
                const T u0 = (T)up - td;  // distance of offset P/2 - 1 + up
                T w = exp(-wa.beta * u0 * u0);
                T r = exp(-wa.beta * ((T)2 * sgn * u0 + (T)1));
#pragma unroll
                for (int l = 0; l < P / 2; ++l) {
                    const int jj = up ? P / 2 + l : P / 2 - 1 - l;
                    sw[qq][d][jj] = (jj == P - 1 && td == (T)0) ? (T)0 : w;
                    w *= r;
                    r *= e2;
                }
                if (!up) anc[qq][d] = (d == 0 ? c[0] : (d == 1 ? c[1] : c[2])) - P / 2 + 1;
            }
        } else {
            for (int k = lane; k < kG2PGroup * 3 * P; k += kWave) {
                const int qq = k / (3 * P), d = (k / P) % 3, jj = k % P;
                int c[3];
                T t[3], f[3];
                RecView<T>::load(rec[min(sg + qq, s1 - 1)], g, c, t, f);
                const T td = (d == 0) ? t[0] : (d == 1 ? t[1] : t[2]);
                sw[qq][d][jj] = window_weight_one<T, P>(jj, td, wa);
                if (jj == 0) anc[qq][d] = c[d] - P / 2 + 1;
            }
        }
        __syncthreads();
        const int ax = anc[q][0], ay = anc[q][1], az = anc[q][2];
        // the grid of the target's system (the systems of a batch are consecutive sorted ranges)
        const TG* __restrict__ g0 = grid + (int64_t)3 * batch_system(bt, min(sg + q, s1 - 1)) * nc;
        const TG* __restrict__ g1 = g0 + nc;
        const TG* __restrict__ g2 = g0 + 2 * nc;
        double a0 = 0, a1 = 0, a2 = 0;  // FP64 sums in every mode (see below)
#pragma unroll 1
        for (int pass = 0; pass < kPass; ++pass) {
            const int item = pass * kG2PLanes + ql;
            if (item < kItems) {
                const int jy = item / G, zg = item - jy * G;
                const T wy = sw[q][1][jy];
                T wyz[V];
#pragma unroll
                for (int e = 0; e < V; ++e) wyz[e] = wy * sw[q][2][zg * V + e];
                const int gz = wrapi(az + zg * V, M3);
                const bool wraps = gz + V > M3;  // the run crosses the periodic z boundary
                const unsigned col = (unsigned)wrapi(ay + jy, M2) * (unsigned)M3 + (unsigned)gz;
                // kU x-planes at a time: their loads are in flight together
#pragma unroll 1
                for (int ix0 = 0; ix0 < P; ix0 += kU) {
                    TG v0[kU][V], v1[kU][V], v2[kU][V];
#pragma unroll
                    for (int k = 0; k < kU; ++k) {
                        const unsigned idx = (unsigned)wrapi(ax + ix0 + k, M1) * plane + col;
                        if (!wraps) {
                            const VT q0 = *reinterpret_cast<const VT*>(g0 + idx);
                            const VT q1 = *reinterpret_cast<const VT*>(g1 + idx);
                            const VT q2 = *reinterpret_cast<const VT*>(g2 + idx);
#pragma unroll
                            for (int e = 0; e < V; ++e) {
                                v0[k][e] = q0[e];
                                v1[k][e] = q1[e];
                                v2[k][e] = q2[e];
                            }
                        } else {
#pragma unroll
                            for (int e = 0; e < V; ++e) {
                                const unsigned ie = idx - (unsigned)gz + (unsigned)wrapi(gz + e, M3);
                                v0[k][e] = g0[ie];
                                v1[k][e] = g1[ie];
                                v2[k][e] = g2[ie];
                            }
                        }
                    }
#pragma unroll
                    for (int k = 0; k < kU; ++k) {
                        const T wx = sw[q][0][ix0 + k];
#pragma unroll
                        for (int e = 0; e < V; ++e) {
                            const double wv = (double)(wx * wyz[e]);
                            a0 += wv * (double)v0[k][e];
                            a1 += wv * (double)v1[k][e];
                            a2 += wv * (double)v2[k][e];
                        }
                    }
                }
            }
        }
        // sums over the lanes of each target
#pragma unroll
        for (int o = kG2PLanes / 2; o >= 1; o >>= 1) {
            a0 += __shfl_xor(a0, o, kWave);
            a1 += __shfl_xor(a1, o, kWave);
            a2 += __shfl_xor(a2, o, kWave);
        }
        const int s = sg + q;
        if (ql == 0 && s < s1) {
            const int orig = rec[s].orig;
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
        __syncthreads();
    }
}


template <typename T, typename TG, int P>
hipError_t launch_g2p_t(const Plan& pl, const Work& w, int n, const double* f, double* u, double* un,
                        double* uf, const Batch& b, hipStream_t s)
{
    const double self_coef = pl.info.self_coef;
    constexpr int per_wave = g2p_per_wave<TG>();
    hipLaunchKernelGGL((k_g2p<T, TG, P>), dim3((n + per_wave - 1) / per_wave), dim3(kWave), 0, s, n,
                       (const typename RecView<T>::Rec*)w.rec, (const TG*)w.grid, pl.g, make_win_args<T>(pl),
                       self_coef, w.u_near, f, u, un, uf, b);
    return hipGetLastError();
}

template <typename T, typename TG>
hipError_t launch_g2p_p(const Plan& pl, const Work& w, int n, const double* f, double* u, double* un,
                        double* uf, const Batch& b, hipStream_t s)
{
    switch (pl.P) {
    case 4: return launch_g2p_t<T, TG, 4>(pl, w, n, f, u, un, uf, b, s);
    case 6: return launch_g2p_t<T, TG, 6>(pl, w, n, f, u, un, uf, b, s);
    case 8: return launch_g2p_t<T, TG, 8>(pl, w, n, f, u, un, uf, b, s);
    case 10: return launch_g2p_t<T, TG, 10>(pl, w, n, f, u, un, uf, b, s);
    case 12: return launch_g2p_t<T, TG, 12>(pl, w, n, f, u, un, uf, b, s);
    case 14: return launch_g2p_t<T, TG, 14>(pl, w, n, f, u, un, uf, b, s);
    case 16: return launch_g2p_t<T, TG, 16>(pl, w, n, f, u, un, uf, b, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace

hipError_t launch_g2p(const Plan& pl, const Work& w, int n, const double* f, double* u,
                      double* u_near_out, double* u_far_out, const Batch& b, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    if (pl.mode == EWALD_FP64) return launch_g2p_p<double, double>(pl, w, n, f, u, u_near_out, u_far_out, b, s);
    if (pl.grid64) return launch_g2p_p<float, double>(pl, w, n, f, u, u_near_out, u_far_out, b, s);
    return launch_g2p_p<float, float>(pl, w, n, f, u, u_near_out, u_far_out, b, s);
}

}  // namespace ewald
