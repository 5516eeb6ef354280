// P2G: spreading of the 3-vector forces onto the uniform grid, eq. (p2g):
//   phi(g_l) = sum_j sum_p w(g_l - y_j + p) f_j,  w separable, P points per axis.
//
// Atomic-free, owner-computes design for MI355X.  One wavefront owns an 8 x 8 patch of
// grid lines along x (lane (ly, lz) owns line (y0+ly, z0+lz)) over an x-segment
// [x0, x1), and sweeps the particle slabs of constant cell-x in increasing order.  Each
// lane keeps P x-accumulators per component in registers: a particle in cell-x c adds
// w_x[k] * w_y * w_z * f to the lane's points x = c - P/2 + 1 + k; after slab c has been
// processed the point x = c - P/2 + 1 receives nothing more from the segment, so it is
// written once and the register window shifts by one.  The first and last P - 1 points of a
// segment also receive from the neighbouring segment: both segments write their partial
// sums to halo planes, which k_p2g_halo_sum adds into the grid.  Every grid point has one
// writer and a fixed summation order: deterministic, no atomics, no zero-fill.
// The particles of a slab that can reach the patch (a (8+P-1)^2 window of cells) are
// contiguous runs of the cell-sorted arrays; they are staged in LDS with their P x weights
// and, per line of the patch, the y weight and the z weight times f (zero where the line is
// outside the particle's P x P footprint), so a lane's factor for a particle is
// w_y[ly] * (w_z f)[lz], read without any dependent index arithmetic.  The x direction is
// exact (no wasted work); in y and z a lane whose line is outside the footprint multiplies
// by zero.
#include <type_traits>

#include "window.h"

namespace ewald {

namespace {

constexpr int kPatch = 8;     // lines per patch edge (8 x 8 = 64 lanes)
constexpr int kWaves = 4;     // waves per block, all owning the block's lines
constexpr int kPerWave = 32;  // particles staged per wave and round
constexpr int kChunk = kWaves * kPerWave;
constexpr int kMaxRuns = 320; // runs per slab (window rows x z-tile segments)

// T: arithmetic and accumulation precision; TG: grid element type (the FP32 bulk mode
// accumulates in FP64 -- the same VALU rate as FP32 without packed math -- and stores FP32).
// A block of kWaves waves owns one (patch, x-segment): every wave keeps accumulators for
// all 64 lines, takes a contiguous quarter of each slab's particles (staged kPerWave at a
// time: 32 amortises the load and search latency of a staging round, and an even split
// keeps the waves of a block equally busy), and at each output step the waves' partial
// sums are added in a fixed order through LDS.
template <typename T, typename TG, int P>
__global__ __launch_bounds__(kWaves * 64) void k_p2g_sweep(const typename RecView<T>::Rec* __restrict__ rec,
                                                           const int* __restrict__ start, Geometry g,
                                                           WinArgs<T> wa, int seg, int npy, int npz,
                                                           const double* __restrict__ sv, int sv_off,
                                                           TG* __restrict__ grid, double* __restrict__ halo,
                                                           int64_t grid_stride, int64_t halo_stride)
{
    // system blockIdx.y of a batch: its cell list, grid and halo planes
    start += (int64_t)blockIdx.y * g.ncells;
    grid += (int64_t)blockIdx.y * grid_stride;
    if (halo) halo += (int64_t)blockIdx.y * halo_stride;
    constexpr int W = kPatch + P - 1;
    __shared__ int run_start[kMaxRuns];
    __shared__ int run_pre[kMaxRuns + 1];
    __shared__ T swx[kChunk][P];             // x weights of the staged particles
    __shared__ T swy[kChunk][kPatch];        // y weight of each patch line (0 off the footprint)
    __shared__ T swz[kChunk][3][kPatch];     // z weight of each patch line times the 3 sources
    __shared__ T sf[kChunk][3];
    __shared__ T st[kChunk][3];  // in-cell fractions (Kaiser-Bessel weights are computed from them)
    __shared__ int soff[kChunk];
    __shared__ T red[kWaves - 1][3][64];

    const int tid = threadIdx.x;
    const int wid = tid >> 6, lane = tid & 63;
    const int item = blockIdx.x;
    const int pz = item % npz, py = (item / npz) % npy, sx = item / (npz * npy);
    const int M1 = g.M[0], M2 = g.M[1], M3 = g.M[2];
    const int x0 = sx * seg, x1 = min(x0 + seg, M1);
    const int y0 = py * kPatch, z0 = pz * kPatch;
    const int ly = lane >> 3, lz = lane & 7;
    const int B = g.B;

    const T e2 = exp((T)-2 * wa.beta);  // ratio of consecutive Gaussian recurrence factors
    T acc[P][3];
#pragma unroll
    for (int k = 0; k < P; ++k) acc[k][0] = acc[k][1] = acc[k][2] = (T)0;

    const int zlo = z0 - P / 2, zhi = z0 + kPatch - 1 + P / 2 - 1;
    const int zt0 = floor_div(zlo, B), zt1 = floor_div(zhi, B);
    const int nzs = zt1 - zt0 + 1;
    const int R = W * nzs;
    const int64_t nc = g.ncells;

    // Output steps: the partial sums of the waves are added in a fixed order through LDS and
    // the sum of wave 0 goes to dst[0], dst[cs], dst[2 cs] (the three components).
    auto output = [&](T a0, T a1, T a2, auto* dst, int64_t cs) {
        if (wid > 0) {
            red[wid - 1][0][lane] = a0;
            red[wid - 1][1][lane] = a1;
            red[wid - 1][2][lane] = a2;
        }
        __syncthreads();
        if (wid == 0) {
#pragma unroll
            for (int k = 0; k < kWaves - 1; ++k) {
                a0 += red[k][0][lane];
                a1 += red[k][1][lane];
                a2 += red[k][2][lane];
            }
            using D = typename std::remove_pointer<decltype(dst)>::type;
            dst[0] = (D)a0;
            dst[cs] = (D)a1;
            dst[2 * cs] = (D)a2;
        }
    };
    // With halo == nullptr the segment's sweep starts P - 1 slabs early (a warm-up that makes its
    // first points complete).  With a halo buffer it sweeps only its own slabs [x0, x1): its first
    // and last P - 1 points are then partial, and go to the halo's head and tail planes of this
    // segment (head[s][k] and tail[s][k] hold the point x0 - P/2 + 1 + k and x1 - P/2 + 1 + k);
    // k_p2g_halo_sum adds tail[s - 1] to head[s] into the grid.
    const int64_t m23 = (int64_t)M2 * M3;
    const int64_t line = (int64_t)(y0 + ly) * M3 + (z0 + lz);
    const int hk = P - 1;
    double* head = halo ? halo + (int64_t)sx * hk * 3 * m23 + line : nullptr;
    double* tail = halo ? halo + ((int64_t)gridDim.x / (npy * npz) + sx) * hk * 3 * m23 + line : nullptr;
    const int cbeg = halo ? x0 : x0 - P / 2, cend = halo ? x1 - 1 : x1 + P / 2 - 2;
    for (int cxu = cbeg; cxu <= cend; ++cxu) {
        const int cx = wrapi(cxu, M1);
        // runs of this slab: one per (window row, z-tile segment); wave 0 builds the table
        int carry = 0;
        if (wid == 0) {
            for (int r0 = 0; r0 < R; r0 += kWave) {
                const int r = r0 + lane;
                int len = 0;
                if (r < R) {
                    const int iy = r / nzs, zs = r - iy * nzs;
                    const int cy = wrapi(y0 - P / 2 + iy, M2);
                    const int zt = zt0 + zs;
                    const int au = max(zlo, zt * B), bu = min(zhi, zt * B + B - 1);
                    const int k0 = cell_key(cx, cy, wrapi(au, M3), g);
                    const int st = start[k0];
                    len = start[k0 + (bu - au) + 1] - st;
                    run_start[r] = st;
                }
                int inc = len;
#pragma unroll
                for (int o = 1; o < kWave; o <<= 1) {
                    const int y = __shfl_up(inc, o, kWave);
                    if (lane >= o) inc += y;
                }
                if (r < R) run_pre[r + 1] = carry + inc;
                carry += __shfl(inc, kWave - 1, kWave);
            }
            if (lane == 0) run_pre[0] = 0;
        }
        __syncthreads();
        const int total = __builtin_amdgcn_readfirstlane(run_pre[R]);

        // the slab's particles are split evenly over the waves; each wave stages and spreads
        // its share in rounds of kPerWave
        const int share = (total + kWaves - 1) / kWaves;
        const int wend = min(total, (wid + 1) * share);
        const int q0 = wid * kPerWave;
        for (int base = wid * share; base < wend; base += kPerWave) {
            const int cnt = min(kPerWave, wend - base);
            if (lane < cnt) {
                const int flat = base + lane;
                int lo = 0, hi = R;
                while (hi - lo > 1) {
                    const int mid = (lo + hi) >> 1;
                    if (run_pre[mid] <= flat) lo = mid; else hi = mid;
                }
                const int r = lo;
                const int p = run_start[r] + (flat - run_pre[r]);
                int c[3];
                T t[3], f[3];
                RecView<T>::load(rec[p], g, c, t, f);
                if (sv) {  // spread three stresslet components instead of the force
#pragma unroll
                    for (int d = 0; d < 3; ++d) f[d] = (T)sv[6 * (int64_t)p + sv_off + d];
                }
                const int iy = r / nzs, zs = r - iy * nzs;
                const int oy = iy - (P - 1);  // stencil anchor - y0
                const int czu = (zt0 + zs) * B + (c[2] & (B - 1));
                const int oz = czu - P / 2 + 1 - z0;
                const int q = q0 + lane;
                soff[q] = (oy + P) | ((oz + P) << 8);
#pragma unroll
                for (int d = 0; d < 3; ++d) {
                    sf[q][d] = f[d];
                    st[q][d] = t[d];
                }
            }
            wave_lds_sync();
            if (!wa.kb) {
                // Gaussian x weights: two lanes per particle, P/2 consecutive weights each by the
                // same recurrence (two exponentials per lane)
                for (int li = lane; li < 2 * cnt; li += kWave) {
                    const int qq = q0 + (li >> 1), j0 = (li & 1) * (P / 2);
                    const T t = st[qq][0];
                    const T u0 = (T)(j0 - (P / 2 - 1)) - t;
                    T w = exp(-wa.beta * u0 * u0);
                    T r = exp(-wa.beta * ((T)2 * u0 + (T)1));
#pragma unroll
                    for (int l = 0; l < P / 2; ++l) {
                        swx[qq][j0 + l] = (j0 + l == P - 1 && t == (T)0) ? (T)0 : w;
                        w *= r;
                        r *= e2;
                    }
                }
                // y and z weights of the patch's lines, one lane per (particle, axis): line l is at
                // stencil offset j = l - o and distance u0 + l from the particle, and the Gaussian
                // obeys w(u + 1) = w(u) exp(-beta (2u + 1)): two exponentials and 2 x 8 products
                for (int li = lane; li < 2 * cnt; li += kWave) {
                    const int qq = q0 + (li >> 1);
                    const bool isy = (li & 1) == 0;
                    const int off = soff[qq];
                    const int o = (isy ? (off & 255) : (off >> 8)) - P;  // stencil anchor - patch origin
                    const T t = st[qq][isy ? 1 : 2];
                    const T u0 = (T)(-o - (P / 2 - 1)) - t;
                    T w = exp(-wa.beta * u0 * u0);
                    T r = exp(-wa.beta * ((T)2 * u0 + (T)1));
                    T wl[kPatch];
#pragma unroll
                    for (int l = 0; l < kPatch; ++l) {
                        const int j = l - o;
                        const bool in = (unsigned)j < (unsigned)P && !(j == P - 1 && t == (T)0);
                        wl[l] = in ? w : (T)0;
                        w *= r;
                        r *= e2;
                    }
                    if (isy) {
#pragma unroll
                        for (int l = 0; l < kPatch; ++l) swy[qq][l] = wl[l];
                    } else {
                        const T f0 = sf[qq][0], f1 = sf[qq][1], f2 = sf[qq][2];
#pragma unroll
                        for (int l = 0; l < kPatch; ++l) {
                            swz[qq][0][l] = wl[l] * f0;
                            swz[qq][1][l] = wl[l] * f1;
                            swz[qq][2][l] = wl[l] * f2;
                        }
                    }
                }
            } else {
                // Kaiser-Bessel: one polynomial per weight, spread over all lanes of the wave
                for (int k = lane; k < cnt * P; k += kWave) {
                    const int qq = q0 + k / P, j = k % P;
                    swx[qq][j] = window_weight_one<T, P>(j, st[qq][0], wa);
                }
                for (int k = lane; k < cnt * 2 * kPatch; k += kWave) {
                    const int qq = q0 + k / (2 * kPatch), l = k % kPatch;
                    const bool isy = (k / kPatch) % 2 == 0;
                    const int off = soff[qq];
                    const int j = l + P - (isy ? (off & 255) : (off >> 8));  // stencil offset of line l
                    T wv = (T)0;
                    if ((unsigned)j < (unsigned)P) wv = window_weight_one<T, P>(j, st[qq][isy ? 1 : 2], wa);
                    if (isy) {
                        swy[qq][l] = wv;
                    } else {
                        swz[qq][0][l] = wv * sf[qq][0];
                        swz[qq][1][l] = wv * sf[qq][1];
                        swz[qq][2][l] = wv * sf[qq][2];
                    }
                }
            }
            wave_lds_sync();
#pragma unroll 2
            for (int q = q0; q < q0 + cnt; ++q) {
                // single-value LDS loads (a paired load occupies the LDS pipeline twice as long)
                const T wy = ld1(swy[q][ly]);
                const T g0 = wy * ld1(swz[q][0][lz]), g1 = wy * ld1(swz[q][1][lz]), g2 = wy * ld1(swz[q][2][lz]);
#pragma unroll
                for (int k = 0; k < P; ++k) {
                    const T wx = swx[q][k];
                    acc[k][0] += wx * g0;
                    acc[k][1] += wx * g1;
                    acc[k][2] += wx * g2;
                }
            }
            wave_lds_sync();
        }

        const int xo = cxu - P / 2 + 1;
        if (halo && xo < x0 + P / 2)
            output(acc[0][0], acc[0][1], acc[0][2], head + (int64_t)(xo - (x0 - P / 2 + 1)) * 3 * m23, m23);
        else if (xo >= x0)
            output(acc[0][0], acc[0][1], acc[0][2], grid + (int64_t)xo * m23 + line, nc);
#pragma unroll
        for (int k = 0; k + 1 < P; ++k) {
            acc[k][0] = acc[k + 1][0];
            acc[k][1] = acc[k + 1][1];
            acc[k][2] = acc[k + 1][2];
        }
        acc[P - 1][0] = acc[P - 1][1] = acc[P - 1][2] = (T)0;
        __syncthreads();
    }
    if (halo) {
#pragma unroll
        for (int k = 0; k < P - 1; ++k) {
            output(acc[k][0], acc[k][1], acc[k][2], tail + (int64_t)k * 3 * m23, m23);
            __syncthreads();
        }
    }
}

// The points next to the segment boundaries: grid(x0(s) - P/2 + 1 + k) = head[s][k] + tail[s-1][k]
// (periodic in s), for k < P - 1, every line and component; head and tail planes are laid out
// [segment][k][component][line].
template <typename TG>
__global__ __launch_bounds__(256) void k_p2g_halo_sum(const double* __restrict__ halo, int nseg, int seg, int P,
                                                      Geometry g, TG* __restrict__ grid, int64_t grid_stride,
                                                      int64_t halo_stride)
{
    halo += (int64_t)blockIdx.y * halo_stride;
    grid += (int64_t)blockIdx.y * grid_stride;
    const int64_t m23 = (int64_t)g.M[1] * g.M[2];
    const int64_t planes = (int64_t)nseg * (P - 1) * 3;
    const int64_t total = planes * m23;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t yz = i % m23, pl = i / m23;
        const int c = (int)(pl % 3), sk = (int)(pl / 3);
        const int k = sk % (P - 1), sg = sk / (P - 1);
        const int sp = (sg + nseg - 1) % nseg;
        const double v = halo[i] + halo[total + ((int64_t)(sp * (P - 1) + k) * 3 + c) * m23 + yz];
        const int x = wrapi(sg * seg - P / 2 + 1 + k, g.M[0]);
        grid[(int64_t)c * g.ncells + (int64_t)x * m23 + yz] = (TG)v;
    }
}


template <typename TG, int P>
hipError_t launch_p2g_t(const Plan& pl, const Work& w, hipStream_t s, bool st, int nsys)
{
    const Geometry& g = pl.g;
    const int npy = g.M[1] / kPatch, npz = g.M[2] / kPatch;
    const int seg = p2g_segment_length(g.M, P);
    const int nseg = g.M[0] / seg;
    const int blocks = nseg * npy * npz;
    // the halo scheme needs every boundary point to lie in exactly two segments
    double* halo = seg >= P ? w.p2g_halo : nullptr;
    const int64_t halo_n = (int64_t)nseg * (P - 1) * 3 * g.M[1] * g.M[2];
    const int fix_blocks = (int)std::min<int64_t>((halo_n + 255) / 256, 4096);
    // force (3 components); with stresslet sources also the 6 tensor components, three per sweep
    const int passes = st ? 3 : 1;
    const int64_t gstride = (int64_t)(st ? 9 : 3) * g.ncells, hstride = p2g_halo_elems(pl);
    for (int ps = 0; ps < passes; ++ps) {
        TG* grid = (TG*)w.grid + (int64_t)3 * ps * g.ncells;
        hipLaunchKernelGGL((k_p2g_sweep<double, TG, P>), dim3(blocks, nsys), dim3(kWaves * kWave), 0, s,
                           (const Rec64*)w.rec, w.start, g, make_win_args<double>(pl), seg, npy, npz,
                           ps == 0 ? nullptr : w.srec, 3 * (ps - 1), grid, halo, gstride, hstride);
        if (halo)
            hipLaunchKernelGGL((k_p2g_halo_sum<TG>), dim3(fix_blocks, nsys), dim3(256), 0, s, (const double*)halo,
                               nseg, seg, P, g, grid, gstride, hstride);
    }
    return hipGetLastError();
}

template <typename T>
hipError_t launch_p2g_p(const Plan& pl, const Work& w, hipStream_t s, bool st, int nsys)
{
    switch (pl.P) {
    case 4: return launch_p2g_t<T, 4>(pl, w, s, st, nsys);
    case 6: return launch_p2g_t<T, 6>(pl, w, s, st, nsys);
    case 8: return launch_p2g_t<T, 8>(pl, w, s, st, nsys);
    case 10: return launch_p2g_t<T, 10>(pl, w, s, st, nsys);
    case 12: return launch_p2g_t<T, 12>(pl, w, s, st, nsys);
    case 14: return launch_p2g_t<T, 14>(pl, w, s, st, nsys);
    case 16: return launch_p2g_t<T, 16>(pl, w, s, st, nsys);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace

int p2g_max_runs() { return kMaxRuns; }

// x-segment length of the sweep: halved while segments stay longer than 2P (the halo planes
// are then a small share of a segment's points) and the launch has fewer than 2048 blocks
// (measured: c3 P2G 10.3 -> 9.8 ms, c4 4.89 -> 4.76 ms against 4P and 1024 blocks)
int p2g_segment_length(const int M[3], int P)
{
    const int npy = M[1] / kPatch, npz = M[2] / kPatch;
    int seg = M[0];
    while (seg > 2 * P && (int64_t)(M[0] / seg) * npy * npz < 2048) seg >>= 1;
    return seg;
}

int64_t p2g_halo_elems(const Plan& pl)
{
    const int seg = p2g_segment_length(pl.g.M, pl.P);
    if (seg < pl.P) return 0;
    return 2 * (int64_t)(pl.g.M[0] / seg) * (pl.P - 1) * 3 * pl.g.M[1] * pl.g.M[2];
}

hipError_t launch_p2g(const Plan& pl, const Work& w, int n, hipStream_t s, bool st, int nsys)
{
    (void)n;
    if (pl.grid64) return launch_p2g_p<double>(pl, w, s, st, nsys);
    return launch_p2g_p<float>(pl, w, s, st, nsys);
}

}  // namespace ewald
