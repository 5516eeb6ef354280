// P2P: the near-field sum of Sec. 2.1, eq. (potentials-near) with the screened Stokeslet
// of eq. (g-near),
//   u^N_i = sum_{j,p : 0 < |r| < r_c} G^N(r) f_j,   r = x_i - x_j + p,
//   G^N(r) f = C(r) (f/|r| + r (r.f)/|r|^3) - (4 xi/sqrt(pi)) e^{-xi^2 |r|^2} f,
//   C(r) = erfc(xi |r|) + (2 xi |r|/sqrt(pi)) e^{-xi^2 |r|^2}.
// With x = xi |r| and E = e^{-x^2}, C = E (erfcx(x) + 2x/sqrt(pi)), so one exponential, one
// reciprocal square root and one short polynomial (screening.h) give both coefficients
//   a1 = C/|r| - (4 xi/sqrt(pi)) E   (of f)   and   a2 = C/|r|^3   (of r (r.f)).
//
// Work decomposition (MI355X).  Particles are sorted by tile (B^3 grid cells, edge about
// r_c/2.5).  One wavefront takes 64 consecutive targets of one tile, one target per lane,
// and walks the (2S+1)^3 neighbour tiles in unwrapped tile coordinates (each periodic image
// of a source is met at most once, also when a dimension has fewer than 2S+1 tiles),
// skipping tiles farther than r_c from the bounding box of its targets.  Lockstep over
// sources would run the expensive formula for every source that ANY lane accepts (about
// twice the useful pairs); instead:
//   1. the wave loads 64 candidate sources at a time (one per lane), keeps those within
//      r_c of the targets' bounding box and appends them, shifted into the targets'
//      periodic frame, to an LDS ring;
//   2. per 32 ring sources every lane tests its target against each source (r^2 < r_c^2,
//      r^2 > 0) and the accepted (target, source) pairs are appended to an LDS queue in
//      source-major order (ballot + lane-prefix count);
//   3. the queue is drained 64 pairs at a time, one pair per lane, every lane busy; each
//      result is added to its target's FP64 accumulator in LDS with ds_add_f64 (the pairs
//      of one source have distinct targets, so conflicts are few).
#include "internal.h"
#include "screening.h"

namespace ewald {

namespace {

struct PairArgs {
    double xi, xi2, rc2;
    double four_xi_over_sqrtpi;
};

constexpr double kTwoOverSqrtPi = 1.1283791670955125739;

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

// number of set bits of m in the lanes below this one
__device__ inline int lanes_below(unsigned long long m)
{
    return (int)__builtin_amdgcn_mbcnt_hi((unsigned)(m >> 32),
                                          __builtin_amdgcn_mbcnt_lo((unsigned)m, 0u));
}

// erfcx(x) + 2x/sqrt(pi) for 0 <= x <= kScreenXmax (polynomial of screening.h)
__device__ inline double screen_q64(double x)
{
    const double d = x + kScreenK;
    double r = __builtin_amdgcn_rcp(d);
    r = fma(fma(-d, r, 1.0), r, r);
    r = fma(fma(-d, r, 1.0), r, r);
    const double u = fma((x - kScreenK) * r, kScreenA, kScreenB);
    double q = kScreenC64[kScreenDeg64];
#pragma unroll
    for (int k = kScreenDeg64 - 1; k >= 0; --k) q = fma(q, u, kScreenC64[k]);
    return fma(kTwoOverSqrtPi, x, q);
}

// G^N(r) f for 0 < r^2 < r_c^2
__device__ inline void pair64(double rx, double ry, double rz, double r2, double f0, double f1, double f2,
                              const PairArgs& a, double& c0, double& c1, double& c2)
{
    const double rinv = rsqrt(r2);
    const double x = a.xi * r2 * rinv;
    const double e = exp(-a.xi2 * r2);
    const double C = e * screen_q64(x);
    const double a1 = fma(C, rinv, -a.four_xi_over_sqrtpi * e);
    const double rf = rx * f0 + ry * f1 + rz * f2;
    const double b = C * rinv * (rinv * rinv) * rf;
    c0 = fma(a1, f0, b * rx);
    c1 = fma(a1, f1, b * ry);
    c2 = fma(a1, f2, b * rz);
}

// FP32 versions (FP32 bulk mode): hardware reciprocal, rsqrt (+ one Newton step) and exp2,
// degree-11 polynomial.  The exponent -xi^2 r^2 log2(e) reaches ~40, where one FP32 ulp is
// ~4e-6, so it is formed and split into integer and fraction in FP64 (same VALU rate) and
// only 2^fraction is taken in FP32.
__device__ inline float screen_q32(float x)
{
    const float d = x + (float)kScreenK;
    float r = __builtin_amdgcn_rcpf(d);
    r = fmaf(fmaf(-d, r, 1.0f), r, r);
    const float u = fmaf((x - (float)kScreenK) * r, (float)kScreenA, (float)kScreenB);
    float q = (float)kScreenC32[kScreenDeg32];
#pragma unroll
    for (int k = kScreenDeg32 - 1; k >= 0; --k) q = fmaf(q, u, (float)kScreenC32[k]);
    return fmaf((float)kTwoOverSqrtPi, x, q);
}

__device__ inline void pair32(float rx, float ry, float rz, float r2, double r2d, float f0, float f1, float f2,
                              float xi, double xi2_log2e, float four_xi_over_sqrtpi, float& c0, float& c1,
                              float& c2)
{
    const float y = __builtin_amdgcn_rsqf(r2);
    const float rinv = y * fmaf(-0.5f * r2 * y, y, 1.5f);
    const float x = xi * r2 * rinv;
    const double ea = -xi2_log2e * r2d;
    const double en = rint(ea);
    const float e = ldexpf(__builtin_amdgcn_exp2f((float)(ea - en)), (int)en);
    const float C = e * screen_q32(x);
    const float a1 = fmaf(C, rinv, -four_xi_over_sqrtpi * e);
    const float rf = rx * f0 + ry * f1 + rz * f2;
    const float b = C * rinv * (rinv * rinv) * rf;
    c0 = fmaf(a1, f0, b * rx);
    c1 = fmaf(a1, f1, b * ry);
    c2 = fmaf(a1, f2, b * rz);
}

// Pair evaluation in the formula precision TF (double: FP64 path; float: FP32 bulk).
template <typename TF>
struct Pair;

template <>
struct Pair<double> {
    __device__ static inline void eval(double rx, double ry, double rz, double r2, double f0, double f1,
                                       double f2, const PairArgs& a, double& c0, double& c1, double& c2)
    {
        pair64(rx, ry, rz, r2, f0, f1, f2, a, c0, c1, c2);
    }
};

template <>
struct Pair<float> {
    __device__ static inline void eval(double rx, double ry, double rz, double r2, float f0, float f1,
                                       float f2, const PairArgs& a, float& c0, float& c1, float& c2)
    {
        pair32((float)rx, (float)ry, (float)rz, (float)r2, r2, f0, f1, f2, (float)a.xi,
               a.xi2 * 1.4426950408889634, (float)a.four_xi_over_sqrtpi, c0, c1, c2);
    }
};

constexpr int kRing = 128;   // LDS ring of filtered candidate sources
constexpr int kTest = 32;    // sources tested per round (queue <= kTest * 64 pairs)

// TF: precision of the pair formula and of the staged forces; TA: accumulator precision.
// Positions and the r^2 < r_c^2 test are FP64 in both modes (same VALU rate as FP32).
template <typename TF, typename TA>
__global__ __launch_bounds__(64) void k_p2p(int n, const Rec64* __restrict__ rec,
                                            const int* __restrict__ start,
                                            const int* __restrict__ chunk_off, Geometry g,
                                            PairArgs a, double* __restrict__ u_near)
{
    __shared__ double tgt[3][kWave];
    __shared__ TA acc[3][kWave];
    __shared__ double ring[3][kRing];
    __shared__ TF ringf[3][kRing];
    __shared__ unsigned short queue[kTest * kWave];

    const int wave = uniform_i(xcd_remap((int)blockIdx.x, (int)gridDim.x));
    const int lane = threadIdx.x;
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
    double w[3], blo[3], bhi[3], tx[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        w[d] = g.B * g.h[d];
        blo[d] = uniform_d(wave_min(me.x[d]));
        bhi[d] = uniform_d(wave_max(me.x[d]));
        tx[d] = active ? me.x[d] : 1e30;  // an inactive lane accepts no pair
        tgt[d][lane] = tx[d];
        acc[d][lane] = (TA)0;
    }
    __syncthreads();

    int rhead = 0, rcount = 0;

    // test the targets against ring sources [rhead, rhead + cnt), then drain the queue
    auto process = [&](int cnt) {
        int qn = 0;
        for (int j = 0; j < cnt; ++j) {
            const int slot = (rhead + j) & (kRing - 1);
            const double rx = tx[0] - ring[0][slot], ry = tx[1] - ring[1][slot], rz = tx[2] - ring[2][slot];
            const double r2 = rx * rx + ry * ry + rz * rz;
            const bool pass = (r2 < a.rc2) && (r2 > 0.0);
            const unsigned long long b = __ballot(pass);
            if (pass) queue[qn + lanes_below(b)] = (unsigned short)(lane | (j << 6));
            qn += __popcll(b);
        }
        __syncthreads();
        for (int q0 = 0; q0 < qn; q0 += kWave) {
            const int k = q0 + lane;
            if (k < qn) {
                const int e = queue[k];
                const int tt = e & (kWave - 1);
                const int slot = (rhead + (e >> 6)) & (kRing - 1);
                const double rx = tgt[0][tt] - ring[0][slot];
                const double ry = tgt[1][tt] - ring[1][slot];
                const double rz = tgt[2][tt] - ring[2][slot];
                const double r2 = rx * rx + ry * ry + rz * rz;
                TF c0, c1, c2;
                Pair<TF>::eval(rx, ry, rz, r2, ringf[0][slot], ringf[1][slot], ringf[2][slot], a, c0, c1, c2);
                atomicAdd(&acc[0][tt], (TA)c0);
                atomicAdd(&acc[1][tt], (TA)c1);
                atomicAdd(&acc[2][tt], (TA)c2);
            }
        }
        __syncthreads();
    };

    for (int dx = -g.S[0]; dx <= g.S[0]; ++dx) {
        const int ux = tc[0] + dx;
        const int fx = floor_div(ux, g.NT[0]);
        const int wx = ux - fx * g.NT[0];
        const double shx = fx * g.L[0];
        const double gx = fmax(0.0, fmax(ux * w[0] - bhi[0], blo[0] - (ux + 1) * w[0]));
        for (int dy = -g.S[1]; dy <= g.S[1]; ++dy) {
            const int uy = tc[1] + dy;
            const int fy = floor_div(uy, g.NT[1]);
            const int wy = uy - fy * g.NT[1];
            const double shy = fy * g.L[1];
            const double gy = fmax(0.0, fmax(uy * w[1] - bhi[1], blo[1] - (uy + 1) * w[1]));
            if (gx * gx + gy * gy >= a.rc2) continue;
            for (int dz = -g.S[2]; dz <= g.S[2]; ++dz) {
                const int uz = tc[2] + dz;
                const int fz = floor_div(uz, g.NT[2]);
                const int wz = uz - fz * g.NT[2];
                const double shz = fz * g.L[2];
                const double gz = fmax(0.0, fmax(uz * w[2] - bhi[2], blo[2] - (uz + 1) * w[2]));
                if (gx * gx + gy * gy + gz * gz >= a.rc2) continue;
                const int nt = (wx * g.NT[1] + wy) * g.NT[2] + wz;
                const int sa = start[nt * per], sb = start[(nt + 1) * per];
                for (int base = sa; base < sb; base += kWave) {
                    const int s = base + lane;
                    bool keep = false;
                    double sx = 0, sy = 0, sz = 0, f0 = 0, f1 = 0, f2 = 0;
                    if (s < sb) {
                        const Rec64& q = rec[s];
                        sx = q.x[0] + shx;
                        sy = q.x[1] + shy;
                        sz = q.x[2] + shz;
                        f0 = q.f[0];
                        f1 = q.f[1];
                        f2 = q.f[2];
                        const double ex = fmax(0.0, fmax(blo[0] - sx, sx - bhi[0]));
                        const double ey = fmax(0.0, fmax(blo[1] - sy, sy - bhi[1]));
                        const double ez = fmax(0.0, fmax(blo[2] - sz, sz - bhi[2]));
                        keep = ex * ex + ey * ey + ez * ez < a.rc2;
                    }
                    const unsigned long long b = __ballot(keep);
                    if (keep) {
                        const int slot = (rhead + rcount + lanes_below(b)) & (kRing - 1);
                        ring[0][slot] = sx;
                        ring[1][slot] = sy;
                        ring[2][slot] = sz;
                        ringf[0][slot] = (TF)f0;
                        ringf[1][slot] = (TF)f1;
                        ringf[2][slot] = (TF)f2;
                    }
                    rcount += __popcll(b);
                    __syncthreads();
                    while (rcount >= kTest) {
                        process(kTest);
                        rhead = (rhead + kTest) & (kRing - 1);
                        rcount -= kTest;
                    }
                }
            }
        }
    }
    while (rcount > 0) {
        const int c = rcount < kTest ? rcount : kTest;
        process(c);
        rhead = (rhead + c) & (kRing - 1);
        rcount -= c;
    }
    if (active) {
        u_near[i] = (double)acc[0][lane];
        u_near[(int64_t)n + i] = (double)acc[1][lane];
        u_near[2 * (int64_t)n + i] = (double)acc[2][lane];
    }
}

}  // namespace

hipError_t launch_p2p(const Plan& pl, const Work& w, int n, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    PairArgs a;
    a.xi = pl.xi;
    a.xi2 = pl.xi * pl.xi;
    a.rc2 = pl.rc * pl.rc;
    a.four_xi_over_sqrtpi = 4.0 * pl.xi / sqrt(M_PI);
    const int64_t waves = (int64_t)pl.g.ntiles + (n + kWave - 1) / kWave;
    const dim3 grid((unsigned)waves), block(kWave);
    const Rec64* rec = (const Rec64*)w.rec;
    // FP32 bulk accumulates in FP64 as well: LDS atomic adds of FP64 are fast on gfx950,
    // those of FP32 are not (measured: 3x slower kernel)
    if (pl.mode == EWALD_FP64)
        hipLaunchKernelGGL((k_p2p<double, double>), grid, block, 0, s, n, rec, w.start, w.chunk_off, pl.g, a,
                           w.u_near);
    else
        hipLaunchKernelGGL((k_p2p<float, double>), grid, block, 0, s, n, rec, w.start, w.chunk_off, pl.g, a,
                           w.u_near);
    return hipGetLastError();
}

}  // namespace ewald
