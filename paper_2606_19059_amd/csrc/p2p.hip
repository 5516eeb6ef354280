// P2P: the near-field sum of Sec. 2.1, eq. (potentials-near) with the screened Stokeslet
// of eq. (g-near),
//   u^N_i = sum_{j,p : 0 < |r| < r_c} G^N(r) f_j,   r = x_i - x_j + p,
//   G^N(r) f = C(r) (f/|r| + r (r.f)/|r|^3) - (4 xi/sqrt(pi)) e^{-xi^2 |r|^2} f,
//   C(r) = erfc(xi |r|) + (2 xi |r|/sqrt(pi)) e^{-xi^2 |r|^2}.
//
// Work decomposition (MI355X): the particles are sorted by tile (a cube of B^3 grid
// cells, edge ~ r_c/2.5); one wavefront takes 64 consecutive targets of one tile, one
// target per lane.  The wave walks the (2S+1)^3 neighbour tiles in unwrapped tile
// coordinates (so each periodic image of a source is met at most once, also when a
// dimension has fewer than 2S+1 tiles), skips tiles farther than r_c from the bounding
// box of its 64 targets, and streams each remaining tile's sources with wave-uniform
// loads (one source per step, broadcast to all lanes through the scalar unit).  Pairs
// with r^2 >= r_c^2 or r^2 == 0 are skipped (the paper skips coincident points).
#include "internal.h"

namespace ewald {

namespace {

struct P2PArgs {
    double xi, rc2;
    double c_two_over_sqrtpi;  // 2/sqrt(pi)
    double c_four_xi_over_sqrtpi;
};

__device__ inline double wave_min(double v)
{
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v = fmin(v, __shfl_xor(v, o, kWave));
    return v;
}

__device__ inline double wave_max(double v)
{
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v = fmax(v, __shfl_xor(v, o, kWave));
    return v;
}

__device__ inline int floor_div(int a, int b) { return (a >= 0) ? a / b : -((-a + b - 1) / b); }

// A value every lane of the wave already holds, made provably uniform for the compiler
// (so that addresses derived from it use scalar loads).
__device__ inline int uniform_i(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ inline double uniform_d(double v)
{
    const unsigned long long b = __double_as_longlong(v);
    const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)(b & 0xffffffffull));
    const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)(b >> 32));
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

__global__ __launch_bounds__(256) void k_p2p64(int n, const Rec64* __restrict__ rec,
                                               const int* __restrict__ start,
                                               const int* __restrict__ chunk_off, Geometry g,
                                               P2PArgs a, double* __restrict__ u_near)
{
    const int wave = uniform_i((int)((blockIdx.x * blockDim.x + threadIdx.x) / kWave));
    const int lane = threadIdx.x & (kWave - 1);
    const int total = chunk_off[g.ntiles];
    if (wave >= total) return;

    // tile of this wave: largest t with chunk_off[t] <= wave
    int lo = 0, hi = g.ntiles;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (chunk_off[mid] <= wave) lo = mid; else hi = mid;
    }
    const int t = lo;
    const int per = 1 << (3 * g.log2B);
    const int t_end = start[(t + 1) * per];
    const int first = start[t * per] + (wave - chunk_off[t]) * kWave;
    const int i = first + lane;
    const bool active = i < t_end;
    const Rec64 me = rec[active ? i : first];

    const int tc[3] = {t / (g.NT[1] * g.NT[2]), (t / g.NT[2]) % g.NT[1], t % g.NT[2]};
    double w[3];
    double blo[3], bhi[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        w[d] = g.B * g.h[d];
        blo[d] = uniform_d(wave_min(me.x[d]));
        bhi[d] = uniform_d(wave_max(me.x[d]));
    }

    double s0 = 0.0, s1 = 0.0, s2 = 0.0;
    for (int dx = -g.S[0]; dx <= g.S[0]; ++dx) {
        const int ux = tc[0] + dx;
        const int wx = ux - floor_div(ux, g.NT[0]) * g.NT[0];
        const double shx = floor_div(ux, g.NT[0]) * g.L[0];
        const double gx = fmax(0.0, fmax(ux * w[0] - bhi[0], blo[0] - (ux + 1) * w[0]));
        for (int dy = -g.S[1]; dy <= g.S[1]; ++dy) {
            const int uy = tc[1] + dy;
            const int wy = uy - floor_div(uy, g.NT[1]) * g.NT[1];
            const double shy = floor_div(uy, g.NT[1]) * g.L[1];
            const double gy = fmax(0.0, fmax(uy * w[1] - bhi[1], blo[1] - (uy + 1) * w[1]));
            if (gx * gx + gy * gy >= a.rc2) continue;
            for (int dz = -g.S[2]; dz <= g.S[2]; ++dz) {
                const int uz = tc[2] + dz;
                const int wz = uz - floor_div(uz, g.NT[2]) * g.NT[2];
                const double shz = floor_div(uz, g.NT[2]) * g.L[2];
                const double gz = fmax(0.0, fmax(uz * w[2] - bhi[2], blo[2] - (uz + 1) * w[2]));
                if (gx * gx + gy * gy + gz * gz >= a.rc2) continue;
                const int nt = (wx * g.NT[1] + wy) * g.NT[2] + wz;
                const int sa = start[nt * per], sb = start[(nt + 1) * per];
                // target relative to the source image frame
                const double px = me.x[0] - shx, py = me.x[1] - shy, pz = me.x[2] - shz;
                for (int s = sa; s < sb; ++s) {
                    const Rec64& src = rec[s];
                    const double rx = px - src.x[0], ry = py - src.x[1], rz = pz - src.x[2];
                    const double r2 = rx * rx + ry * ry + rz * rz;
                    if (r2 < a.rc2 && r2 > 0.0) {
                        const double rinv = rsqrt(r2);
                        const double r = r2 * rinv;
                        const double xr = a.xi * r;
                        const double e = exp(-xr * xr);
                        const double c = erfc(xr) + a.c_two_over_sqrtpi * xr * e;
                        const double a1 = c * rinv - a.c_four_xi_over_sqrtpi * e;
                        const double rf = rx * src.f[0] + ry * src.f[1] + rz * src.f[2];
                        const double a2 = c * rinv * rinv * rinv * rf;
                        s0 += a1 * src.f[0] + a2 * rx;
                        s1 += a1 * src.f[1] + a2 * ry;
                        s2 += a1 * src.f[2] + a2 * rz;
                    }
                }
            }
        }
    }
    if (active) {
        u_near[i] = s0;
        u_near[(int64_t)n + i] = s1;
        u_near[2 * (int64_t)n + i] = s2;
    }
}

}  // namespace

hipError_t launch_p2p(const Plan& pl, const Work& w, int n, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    P2PArgs a;
    a.xi = pl.xi;
    a.rc2 = pl.rc * pl.rc;
    a.c_two_over_sqrtpi = 2.0 / sqrt(M_PI);
    a.c_four_xi_over_sqrtpi = 4.0 * pl.xi / sqrt(M_PI);
    const int64_t waves = (int64_t)pl.g.ntiles + (n + kWave - 1) / kWave;
    const int blocks = (int)((waves * kWave + 255) / 256);
    if (pl.mode == EWALD_FP64) {
        hipLaunchKernelGGL(k_p2p64, dim3(blocks), dim3(256), 0, s, n, (const Rec64*)w.rec, w.start,
                           w.chunk_off, pl.g, a, w.u_near);
        return hipGetLastError();
    }
    return hipErrorNotSupported;
}

}  // namespace ewald
