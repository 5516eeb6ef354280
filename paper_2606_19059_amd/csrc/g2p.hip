// G2P + SUM: interpolation of the far-field grid back to the particles, eq. (g2p),
//   u^F(x_i) = h1 h2 h3 sum_l w(x_i - g_l + p) v(g_l)
// (the h^3 factor is folded into the CNV scaling, so here it is a plain weighted sum),
// then u_i = u^N_i + u^F_i - (4 xi/sqrt(pi)) f_i (Algorithm "se", SUM step, with the
// self-term correction), scattered back to the caller's particle order.
//
// The sum is separable, so for a group of targets whose stencils share one box of grid points
// it is a matrix product (one grid value serves every target of the group) followed by a short
// weighted sum per target; the product runs on the matrix cores (see k_g2p_mfma).  No
// atomics: each target's result is owned by one lane.  The far field at a particle contains its
// own screened self-interaction, about (4 xi / sqrt(pi)) f, which the self term removes; at large
// xi (fine grids) and for sparse particles that cancellation is large, so FP32 sums over a whole
// stencil would set an error floor.  With an FP64 grid every sum is FP64; with an FP32 grid (the
// FP32 bulk mode) only the matrix product sums in FP32, each of its sums covering one z-column of
// the box over at most U_x U_y points, and the z-weighted sums per target are FP64.
#include "window.h"

#include <type_traits>

namespace ewald {

namespace {

// Window weights and stencil anchors of NG consecutive sorted targets sg, sg + 1, ... (those
// at or past s1 repeat target s1 - 1), by the 64 lanes of one wave: sw[q][d][j] is the weight
// of stencil offset j along axis d of target q, anc[q][d] the (unwrapped) first stencil cell.
template <typename T, int P, int NG>
__device__ inline void stage_weights(const typename RecView<T>::Rec* __restrict__ rec, const Geometry& g,
                                     const WinArgs<T>& wa, int sg, int s1, T (*sw)[3][P], int (*anc)[3],
                                     int lane)
{
    if (sizeof(T) == 8 && !wa.kb) {
        // FP64 Gaussian: two lanes per (target, axis), each walking P/2 weights away from the
        // peak by the recurrence w(u + s) = w(u) exp(-beta (2 s u + 1)), s = -1 for offsets
        // P/2-1 down to 0 and s = +1 for P/2 up to P-1 (two exponentials per lane)
        const T e2 = exp((T)-2 * wa.beta);  // ratio of consecutive recurrence factors
        for (int k = lane; k < NG * 6; k += kWave) {
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
        for (int k = lane; k < NG * 3 * P; k += kWave) {
            const int qq = k / (3 * P), d = (k / P) % 3, jj = k % P;
            int c[3];
            T t[3], f[3];
            RecView<T>::load(rec[min(sg + qq, s1 - 1)], g, c, t, f);
            const T td = (d == 0) ? t[0] : (d == 1 ? t[1] : t[2]);
            sw[qq][d][jj] = window_weight_one<T, P>(jj, td, wa);
            if (jj == 0) anc[qq][d] = c[d] - P / 2 + 1;
        }
    }
}

// u = u^N + u^F - self term at the caller's index (or u^N and u^F apart)
__device__ inline void write_target(int s, int orig, int64_t nn, double a0, double a1, double a2, double self_coef,
                                    const double* __restrict__ u_near, const double* __restrict__ f_in,
                                    double* __restrict__ u, double* __restrict__ u_near_out,
                                    double* __restrict__ u_far_out)
{
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

// ---------------------------------------------------------------- matrix-core form
// For a group of 16 targets of one P2P tile (consecutive in the cell-sorted order, so their
// stencils share most of one box of U_x x U_y x U_z grid points), the gather is a product of
// two matrices followed by a small weighted sum:
//   D[i][(c, z)] = sum_{(x, y)} A[i][(x, y)] F_c[x][y][z],   A[i][(x, y)] = w_x,i(x) w_y,i(y)
//   u^F_i,c = sum_z w_z,i(z) D[i][(c, z)]
// (A is zero off target i's P x P footprint).  The box spans the group's anchors in x and y
// and the whole tile in z (U_z = B + P - 1, so that the 3 U_z columns of D make a fixed number
// NB of 16-column blocks per plan).  The contraction runs over the U_x U_y points of the box in
// steps of 4, one matrix instruction per column block: v_mfma_f64_16x16x4f64 (FP64 in and out),
// or for FP32 grids and weights v_mfma_f32_16x16x4f32, at twice the FP64 instruction's rate on
// gfx950 and with half the registers per operand and accumulator.  Each
// grid value loaded serves all 16 targets of the group, where a per-target gather loads P^3
// values for every target; the 16 lanes of a column block read 16 consecutive z of one grid
// line.  Lane layouts on gfx950: lane l supplies A[l % 16][l / 16] and B[l / 16][l % 16] (both
// instructions) and receives D[4 r + l / 16][l % 16] (FP64) or D[4 (l / 16) + r][l % 16] (FP32),
// r = 0..3.
typedef double g2p_v4d __attribute__((ext_vector_type(4)));
typedef float g2p_v4f __attribute__((ext_vector_type(4)));
__device__ inline g2p_v4d g2p_mfma(double a, double b, g2p_v4d c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }
__device__ inline g2p_v4f g2p_mfma(float a, float b, g2p_v4f c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
// operand and accumulator types: FP32 when both the weights and the grid are FP32
template <typename T, typename TG>
struct G2PMat {
    static constexpr bool f32 = std::is_same<T, float>::value && std::is_same<TG, float>::value;
    typedef typename std::conditional<f32, float, double>::type S;
    typedef typename std::conditional<f32, g2p_v4f, g2p_v4d>::type V4;
};
constexpr int kMG = 16;     // targets per wave (matrix rows)
constexpr int kMWaves = 4;  // waves per block: one 64-target chunk of a tile

// column blocks of a plan: 3 (B + P - 1) columns
constexpr int g2p_mfma_blocks(int B, int P) { return (3 * (B + P - 1) + 15) / 16; }

// Up to five column blocks the FP64 kernel is bounded to 96 VGPRs (five waves per SIMD instead of
// four): the loads of a step wait on L2 most of the time, and the fifth wave hides more of it
// (c3 5.73 -> 5.47 ms, H 0.79 -> 0.77 ms, c2 unchanged); six blocks would spill under that bound.
// The FP32 kernel fits eight waves (64 VGPRs) up to four blocks, and five below P = 16; six
// otherwise.
template <typename T, typename TG, int P, int NB>
constexpr int g2p_waves()
{
    return G2PMat<T, TG>::f32 ? ((NB <= 4 || (NB == 5 && P < 16)) ? 8 : 6) : (NB <= 5 ? 5 : 4);
}
template <typename T, typename TG, int P, int NB>
__global__ __launch_bounds__(kMWaves * 64) __attribute__((amdgpu_waves_per_eu(g2p_waves<T, TG, P, NB>()))) void k_g2p_mfma(const typename RecView<T>::Rec* __restrict__ rec,
                                                           const int* __restrict__ start,
                                                           const int* __restrict__ chunk_off,
                                                           const TG* __restrict__ grid, Geometry g, WinArgs<T> wa,
                                                           double self_coef, const double* __restrict__ u_near,
                                                           const double* __restrict__ f_in, double* __restrict__ u,
                                                           double* __restrict__ u_near_out,
                                                           double* __restrict__ u_far_out, int n)
{
    __shared__ T sw[kMWaves][kMG][3][P];
    __shared__ int anc[kMWaves][kMG][3];
    typedef typename G2PMat<T, TG>::S TM;
    // rows of D held by a lane: 4 r + quarter (FP64 instruction) or 4 quarter + r (FP32)
    constexpr bool kRowsGrouped = G2PMat<T, TG>::f32;
    const int wid = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int nt = g.ntiles * g.nsys;
    const int total = chunk_off[nt];  // 64-target chunks of all tiles of all systems
    if ((int)blockIdx.x >= total) return;
    // blocks are dealt to the 8 XCDs round robin: each XCD takes one contiguous range of chunks
    const int chunk = xcd_remap((int)blockIdx.x, total);
    int lo = 0, hi = nt;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (chunk_off[mid] <= chunk) lo = mid; else hi = mid;
    }
    const int t = lo;
    const int per = 1 << (3 * g.log2B);
    const int t_end = start[(t + 1) * per];
    const int sg = start[t * per] + (chunk - chunk_off[t]) * kWave + wid * kMG;
    if (sg >= t_end) return;  // this wave's part of a short chunk is empty (no block barriers below)
    const int s1 = min(sg + kMG, t_end);
    T (*swq)[3][P] = sw[wid];
    int (*ancq)[3] = anc[wid];
    stage_weights<T, P, kMG>(rec, g, wa, sg, s1, swq, ancq, lane);
    wave_lds_sync();

    // the group's box: x and y from the anchors of its 16 targets (short groups repeat the
    // last), reduced over the 16 lanes of each quarter wave; z from the tile
    const int i = lane & 15, kq = lane >> 4;
    int mn0 = ancq[i][0], mx0 = mn0, mn1 = ancq[i][1], mx1 = mn1;
#pragma unroll
    for (int o = 1; o < 16; o <<= 1) {
        mn0 = min(mn0, __shfl_xor(mn0, o, kWave));
        mx0 = max(mx0, __shfl_xor(mx0, o, kWave));
        mn1 = min(mn1, __shfl_xor(mn1, o, kWave));
        mx1 = max(mx1, __shfl_xor(mx1, o, kWave));
    }
    const int tl = t - (t / g.ntiles) * g.ntiles;
    const int ux = __builtin_amdgcn_readfirstlane(mn0), uy = __builtin_amdgcn_readfirstlane(mn1);
    const int uz = (tl % g.NT[2]) * g.B - P / 2 + 1;
    const int Ux = __builtin_amdgcn_readfirstlane(mx0) - ux + P;
    const int Uy = __builtin_amdgcn_readfirstlane(mx1) - uy + P;
    const int Uzt = g.B + P - 1;
    const int ncol = 3 * Uzt;
    const int steps = (Ux * Uy + 3) >> 2;

    const int M1 = g.M[0], M2 = g.M[1], M3 = g.M[2];
    const unsigned plane = (unsigned)M2 * (unsigned)M3;
    const unsigned nc = (unsigned)g.ncells;
    const TG* __restrict__ gs = grid + (int64_t)3 * (t / g.ntiles) * g.ncells;
    // this lane's column of each block: component c and box z (columns past 3 U_z read a valid
    // point and are ignored)
    unsigned zc[NB];
#pragma unroll
    for (int cb = 0; cb < NB; ++cb) {
        const int col = min(16 * cb + i, ncol - 1);
        const int c = col / Uzt, z = col - c * Uzt;
        zc[cb] = (unsigned)c * nc + (unsigned)((uz + z) & (M3 - 1));
    }
    // this lane's row of A: target i's offsets in the box
    const int dxi = ancq[i][0] - ux, dyi = ancq[i][1] - uy;
    const T* __restrict__ wxi = swq[i][0];
    const T* __restrict__ wyi = swq[i][1];

    // box point (xk, yk) of this lane's k = 4 step + kq (U_y >= P >= 4: one wrap at most).  Steps
    // go in pairs with two operand sets, each loaded one step ahead of its use; steps past the
    // last have x >= U_x, so jx >= P and A = 0, and read valid (wrapped) grid points.
    int xk = 0, yk = kq;
    auto a_of = [&]() {
        const int jx = xk - dxi, jy = yk - dyi;
        const bool in = (unsigned)jx < (unsigned)P && (unsigned)jy < (unsigned)P;
        const T w = wxi[in ? jx : 0] * wyi[in ? jy : 0];
        return in ? (TM)w : (TM)0;
    };
    auto load_b = [&](TM* b) {
        const unsigned xy =
            (unsigned)((ux + xk) & (M1 - 1)) * plane + (unsigned)((uy + yk) & (M2 - 1)) * (unsigned)M3;
#pragma unroll
        for (int cb = 0; cb < NB; ++cb) b[cb] = (TM)gs[xy + zc[cb]];
    };
    auto advance = [&]() {
        yk += 4;
        if (yk >= Uy) {
            yk -= Uy;
            ++xk;
        }
    };
    typename G2PMat<T, TG>::V4 acc[NB];
#pragma unroll
    for (int cb = 0; cb < NB; ++cb)
#pragma unroll
        for (int r = 0; r < 4; ++r) acc[cb][r] = (TM)0;
    TM a0 = a_of(), b0[NB], a1, b1[NB];
    load_b(b0);
#pragma unroll 1
    for (int st = 0; st < steps; st += 2) {
        advance();
        a1 = a_of();
        load_b(b1);
        __builtin_amdgcn_sched_barrier(0);  // the loads go out before this step's instructions
#pragma unroll
        for (int cb = 0; cb < NB; ++cb) acc[cb] = g2p_mfma(a0, b0[cb], acc[cb]);
        advance();
        a0 = a_of();
        load_b(b0);
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int cb = 0; cb < NB; ++cb) acc[cb] = g2p_mfma(a1, b1[cb], acc[cb]);
    }

    // u^F of this lane's four rows: weight each column by w_z of its row's target, sum the 16 columns
    double p[4][3];
#pragma unroll
    for (int r = 0; r < 4; ++r) p[r][0] = p[r][1] = p[r][2] = 0.0;
#pragma unroll
    for (int cb = 0; cb < NB; ++cb) {
        const int col = 16 * cb + i;
        const int c = col / Uzt, z = col - c * Uzt;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int q = kRowsGrouped ? 4 * kq + r : 4 * r + kq;
            const int jz = z + uz - ancq[q][2];
            const bool in = col < ncol && (unsigned)jz < (unsigned)P;
            const double v = in ? (double)swq[q][2][in ? jz : 0] * (double)acc[cb][r] : 0.0;
            p[r][0] += c == 0 ? v : 0.0;
            p[r][1] += c == 1 ? v : 0.0;
            p[r][2] += c == 2 ? v : 0.0;
        }
    }
#pragma unroll
    for (int o = 1; o < 16; o <<= 1) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            p[r][0] += __shfl_xor(p[r][0], o, kWave);
            p[r][1] += __shfl_xor(p[r][1], o, kWave);
            p[r][2] += __shfl_xor(p[r][2], o, kWave);
        }
    }
    if (i < 4) {
        // lane i of quarter kq writes its row r = i
        const int s = sg + (kRowsGrouped ? 4 * kq + i : 4 * i + kq);
        double v0 = p[0][0], v1 = p[0][1], v2 = p[0][2];
#pragma unroll
        for (int r = 1; r < 4; ++r) {
            if (i == r) {
                v0 = p[r][0];
                v1 = p[r][1];
                v2 = p[r][2];
            }
        }
        if (s < s1) write_target(s, rec[s].orig, n, v0, v1, v2, self_coef, u_near, f_in, u, u_near_out, u_far_out);
    }
}

template <typename T, typename TG, int P, int NB>
hipError_t launch_g2p_mfma(const Plan& pl, const Work& w, int n, const double* f, double* u, double* un, double* uf,
                           const Batch& b, hipStream_t s)
{
    Geometry g = pl.g;
    g.nsys = b.count;
    // an upper bound on the chunks (each tile has at most one short chunk); blocks past the
    // actual count exit at once
    const int64_t blocks = (int64_t)g.ntiles * g.nsys + (n + kWave - 1) / kWave;
    hipLaunchKernelGGL((k_g2p_mfma<T, TG, P, NB>), dim3((unsigned)blocks), dim3(kMWaves * kWave), 0, s,
                       (const typename RecView<T>::Rec*)w.rec, w.start, w.chunk_off, (const TG*)w.grid, g,
                       make_win_args<T>(pl), pl.info.self_coef, w.u_near, f, u, un, uf, n);
    return hipGetLastError();
}

template <typename T, typename TG, int P>
hipError_t launch_g2p_t(const Plan& pl, const Work& w, int n, const double* f, double* u, double* un,
                        double* uf, const Batch& b, hipStream_t s)
{
    switch (pl.g.B) {  // tile edge (cells; a power of two up to 16): fixes the matrix's column blocks
    case 2: return launch_g2p_mfma<T, TG, P, g2p_mfma_blocks(2, P)>(pl, w, n, f, u, un, uf, b, s);
    case 4: return launch_g2p_mfma<T, TG, P, g2p_mfma_blocks(4, P)>(pl, w, n, f, u, un, uf, b, s);
    case 8: return launch_g2p_mfma<T, TG, P, g2p_mfma_blocks(8, P)>(pl, w, n, f, u, un, uf, b, s);
    case 16: return launch_g2p_mfma<T, TG, P, g2p_mfma_blocks(16, P)>(pl, w, n, f, u, un, uf, b, s);
    default: return hipErrorInvalidValue;
    }
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
