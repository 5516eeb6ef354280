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
#include <type_traits>
#include "screening.h"

namespace ewald {

namespace {

// Accuracy levels of the FP64 pair formula (template argument Lv), chosen from the plan's tol so
// that the formula's own error stays 30-40 times below it:
//   0 (tol < 1e-10): degree-16 screening polynomial (|dC| < 5e-15), library exponential, two
//     Newton steps on the hardware reciprocal, third-order rsqrt correction;
//   1 (1e-10 <= tol < 1e-8): degree 12 (|dC| < 4e-12), e^{-y} = 2^z (z = -y log2 e) as 2^n times a
//     degree-8 Chebyshev polynomial of 2^s, z = n + s, n = rint(z) (relative error 1.1e-12; no
//     range checks: -61 < z <= 0 on the P2P range), one Newton step on rcp and on rsqrt;
//   2 (tol >= 1e-8): degree 10 (|dC| < 3e-10) and a degree-7 polynomial of 2^s (5.6e-11), else
//     as level 1: near-field error about 2.5e-10 of the field's max (a CPU model of c2's and of a
//     coarse plan's geometry).
// Both polynomials are stored divided by their leading coefficients (screening.h), so that Horner
// starts with an addition (an FMA cannot take two scalar-register coefficients).  The FP64 pair
// formula therefore returns its coefficients divided by post = lead_screen x lead_exp (lead_exp = 1
// at level 0); the kernels multiply each target's and source's sum by post once, at the end.
constexpr double kLog2e = 1.4426950408889634074;

struct PairArgs {
    double xi, xi2, rc2;
    double four_xi_over_sqrtpi;
    double xi2_log2e;
    // FP64 formula of the launched level: z = zc r^2 (zc = -xi^2 log2 e); monic screening (ms,
    // x coefficient g = (2/sqrt(pi))/lead_s) and exponential (me) polynomials; a1 / post =
    // C'/r - h e' with h = (4 xi/sqrt(pi))/lead_s
    double zc, g, h, post, lead_s, lead_e;
    // polynomials passed by value, so that the coefficients sit in scalar registers (an FMA then
    // takes them as an operand, no per-pair register copies); c32: the FP32 formula's
    double ms[kScreenDeg64];
    double me[kExpDeg1];
    float c32[kScreenDeg32 + 1];
    float zc32;  // FP32 formula: -xi^2 log2 e
    double six_xi_over_sqrtpi, four_xi3_over_sqrtpi;  // stresslet screening
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

// minimum over the wave of v in [0, 63], by six ballots (no cross-lane data movement: the
// shuffle form of this reduction put six dependent LDS round trips into every batch)
__device__ inline int wave_min_small(int v)
{
    int lo = 0;
#pragma unroll
    for (int b = 32; b >= 1; b >>= 1)
        if (__builtin_amdgcn_ballot_w64(v < lo + b) == 0ull) lo += b;
    return lo;
}

// position of the k-th (from 0) set bit of m, for k < popcount(m): five halving steps
__device__ inline int select_bit(unsigned m, int k)
{
    int pos = 0;
#pragma unroll
    for (int s = 16; s >= 1; s >>= 1) {
        const int low = __popc(m & ((1u << s) - 1u));
        const bool up = low <= k;
        k = up ? k - low : k;
        m = up ? m >> s : m;
        pos = up ? pos + s : pos;
    }
    return pos;
}

// v | (v of lane l ^ 16) | (v of lane l ^ 32) | (v of lane l ^ 48), by the lane-swap instructions
// (VALU; a shuffle would take the LDS pipeline, which bounds the P2P kernels)
__device__ inline unsigned or_rows4(unsigned v)
{
    const auto a = __builtin_amdgcn_permlane16_swap(v, v, false, false);
    v = a[0] | a[1];
    const auto b = __builtin_amdgcn_permlane32_swap(v, v, false, false);
    return b[0] | b[1];
}

// number of set bits of m in the lanes below this one
__device__ inline int lanes_below(unsigned long long m)
{
    return (int)__builtin_amdgcn_mbcnt_hi((unsigned)(m >> 32),
                                          __builtin_amdgcn_mbcnt_lo((unsigned)m, 0u));
}

// (erfcx(x) + 2x/sqrt(pi)) / lead_s for 0 <= x <= kScreenXmax: the monic polynomial of screening.h
// in t = (x - K)/(x + K) = 1 - 2K/(x + K), plus g x
template <int Lv>
__device__ inline double screen_q64(double x, const PairArgs& a)
{
    const double d = x + kScreenK;
    double r = __builtin_amdgcn_rcp(d);
    r = fma(fma(-d, r, 1.0), r, r);
    if (Lv == 0) r = fma(fma(-d, r, 1.0), r, r);
    const double t = fma(-2.0 * kScreenK, r, 1.0);
    constexpr int deg = Lv == 0 ? kScreenDeg64 : Lv == 1 ? kScreenDeg64s : kScreenDeg64f;
    const double* m = a.ms;
    double q = t + m[deg - 1];
#pragma unroll
    for (int k = deg - 2; k >= 0; --k) q = fma(q, t, m[k]);
    return fma(a.g, x, q);
}

// 2^z / lead_e for -61 < z <= 0: z = n + s, n = rint(z), |s| <= 1/2 (s exact), 2^s from the monic
// polynomial of screening.h
template <int Lv>
__device__ inline double exp2_lead(double z, const PairArgs& a)
{
    const double n = rint(z);
    const double s = z - n;
    constexpr int deg = Lv == 1 ? kExpDeg1 : kExpDeg2;
    const double* m = a.me;
    double p = s + m[deg - 1];
#pragma unroll
    for (int k = deg - 2; k >= 0; --k) p = fma(p, s, m[k]);
    return ldexp(p, (int)n);
}

// 1/sqrt(r2) for finite r2 > 0: hardware estimate y (error bound 2^29 ulp, ~2^-23
// relative), then with e = 1 - r2 y^2 one third-order correction y (1 + e/2 + 3e^2/8) (full
// FP64), or for levels 1 and 2 one Newton step y (1 + e/2) (relative error ~ 3e^2/8, below
// 1e-13).  No special values.
template <int Lv>
__device__ inline double rsqrt_pos(double r2)
{
    const double y = __builtin_amdgcn_rsq(r2);
    const double e = fma(-r2 * y, y, 1.0);
    if (Lv > 0) return fma(y * e, 0.5, y);
    return fma(y * e, fma(0.375, e, 0.5), y);
}

// Coefficients of G^N(r) f = a1 f + b (r.f) r for 0 < r^2 < r_c^2 (FP64), divided by post:
// a1 = C/r - (4 xi/sqrt(pi)) e, b = C/r^3, with e = e^{-xi^2 r^2} = lead_e e' and C = e Q,
// Q = lead_s Q'
template <int Lv>
__device__ inline void coef64(double r2, const PairArgs& a, double& a1, double& b)
{
    const double rinv = rsqrt_pos<Lv>(r2);
    const double x = a.xi * r2 * rinv;
    const double e = Lv > 0 ? exp2_lead<Lv>(a.zc * r2, a) : exp(-a.xi2 * r2);
    const double Cr = e * screen_q64<Lv>(x, a) * rinv;
    a1 = fma(-a.h, e, Cr);
    b = Cr * (rinv * rinv);
}

// FP32 versions (FP32 bulk mode): hardware reciprocal, rsqrt and exp2 (1 ulp each, used
// as they come: a refinement step would only chase FP32's own rounding), degree-11
// polynomial.  e = 2^z with z = -xi^2 r^2 log2(e) formed in FP32: z reaches -61, where its
// rounding moves 2^z by up to 3e-6 relative, but the absolute error, 2^z |z| ln2 x 2^-24, stays
// below 8e-8 over the whole range (as for FP32 rounding of e itself); e multiplies the field
// terms, so this is the error that counts.
__device__ inline float screen_q32(float x, const PairArgs& a)
{
    const float d = x + (float)kScreenK;
    const float r = __builtin_amdgcn_rcpf(d);  // 1 ulp: no refinement needed in FP32
    const float u = fmaf((x - (float)kScreenK) * r, (float)kScreenA, (float)kScreenB);
    float q = a.c32[kScreenDeg32];
#pragma unroll
    for (int k = kScreenDeg32 - 1; k >= 0; --k) q = fmaf(q, u, a.c32[k]);
    return fmaf((float)kTwoOverSqrtPi, x, q);
}

__device__ inline void coef32(double r2d, const PairArgs& a, float& a1, float& b)
{
    const float r2 = (float)r2d;
    const float rinv = __builtin_amdgcn_rsqf(r2);  // 1 ulp: no refinement needed in FP32
    const float x = (float)a.xi * r2 * rinv;
    const float e = __builtin_amdgcn_exp2f(a.zc32 * r2);
    const float Cr = e * screen_q32(x, a) * rinv;
    a1 = fmaf(-(float)a.four_xi_over_sqrtpi, e, Cr);
    b = Cr * (rinv * rinv);
}

// Pair coefficients in the formula precision TF (double: FP64 path at accuracy level Lv;
// float: FP32 bulk, Lv unused).
template <typename TF, int Lv>
struct Coef;
// post: the factor that the sums of eval's contributions take at the end
template <int Lv>
struct Coef<double, Lv> {
    __device__ static inline void eval(double r2, const PairArgs& a, double& a1, double& b)
    {
        coef64<Lv>(r2, a, a1, b);
    }
    __device__ static inline double post(const PairArgs& a) { return a.post; }
};
template <int Lv>
struct Coef<float, Lv> {
    __device__ static inline void eval(double r2, const PairArgs& a, float& a1, float& b) { coef32(r2, a, a1, b); }
    __device__ static inline double post(const PairArgs&) { return 1.0; }
};

// Stresslet pair (combined single and double layer sources, Sec. 2.3): with the screened
// remainder of T(r) = -6 r r r / |r|^5,
//   T^N_abc(r) S_bc = alpha r_a (r.S r) + beta (2 (S r)_a + tr(S) r_a)   (S symmetric),
//   alpha = -2 |r|^-3 (3 erfc(xi |r|) |r|^-2 + e^{-xi^2 r^2} (6 xi/(sqrt(pi) |r|) + 4 xi^3 |r|/sqrt(pi))),
//   beta = 4 xi^3 e^{-xi^2 r^2} / sqrt(pi).
// Both follow from the same exponential and screening polynomial as G^N:
// erfc(x) = C - (2x/sqrt(pi)) e^{-x^2}.
template <int Lv>
__device__ inline void coef64_st(double r2, const PairArgs& a, double& a1, double& b, double& al, double& be)
{
    const double rinv = rsqrt(r2);
    const double r = r2 * rinv;
    const double x = a.xi * r;
    const double e = Lv > 0 ? a.lead_e * exp2_lead<Lv>(a.zc * r2, a) : exp(-a.xi2 * r2);
    const double C = e * (a.lead_s * screen_q64<Lv>(x, a));
    const double rinv2 = rinv * rinv, rinv3 = rinv2 * rinv;
    a1 = fma(C, rinv, -a.four_xi_over_sqrtpi * e);
    b = C * rinv3;
    const double erfc_x = fma(-kTwoOverSqrtPi * x, e, C);
    al = -2.0 * rinv3 * fma(3.0 * erfc_x, rinv2, e * fma(a.six_xi_over_sqrtpi, rinv, a.four_xi3_over_sqrtpi * r));
    be = a.four_xi3_over_sqrtpi * e;
}

__device__ inline void coef32_st(double r2d, const PairArgs& a, float& a1, float& b, float& al, float& be)
{
    const float r2 = (float)r2d;
    const float rinv = __builtin_amdgcn_rsqf(r2);
    const float r = r2 * rinv;
    const float x = (float)a.xi * r;
    const float e = __builtin_amdgcn_exp2f(a.zc32 * r2);
    const float C = e * screen_q32(x, a);
    const float rinv2 = rinv * rinv, rinv3 = rinv2 * rinv;
    a1 = fmaf(C, rinv, -(float)a.four_xi_over_sqrtpi * e);
    b = C * rinv3;
    const float erfc_x = fmaf(-(float)kTwoOverSqrtPi * x, e, C);
    al = -2.0f * rinv3 *
         fmaf(3.0f * erfc_x, rinv2, e * fmaf((float)a.six_xi_over_sqrtpi, rinv, (float)a.four_xi3_over_sqrtpi * r));
    be = (float)a.four_xi3_over_sqrtpi * e;
}

template <typename TF, int Lv>
struct CoefSt;
template <int Lv>
struct CoefSt<double, Lv> {
    __device__ static inline void eval(double r2, const PairArgs& a, double& a1, double& b, double& al, double& be)
    {
        coef64_st<Lv>(r2, a, a1, b, al, be);
    }
};
template <int Lv>
struct CoefSt<float, Lv> {
    __device__ static inline void eval(double r2, const PairArgs& a, float& a1, float& b, float& al, float& be)
    {
        coef32_st(r2, a, a1, b, al, be);
    }
};

// c += alpha r (r.S r) + beta (2 S r + tr(S) r), S = (s0..s5) = (xx, yy, zz, xy, xz, yz)
template <typename TF>
__device__ inline void apply_st(TF al, TF be, TF rx, TF ry, TF rz, const TF* s, TF& c0, TF& c1, TF& c2)
{
    const TF t0 = s[0] * rx + s[3] * ry + s[4] * rz;
    const TF t1 = s[3] * rx + s[1] * ry + s[5] * rz;
    const TF t2 = s[4] * rx + s[5] * ry + s[2] * rz;
    const TF rsr = rx * t0 + ry * t1 + rz * t2;
    const TF g = al * rsr + be * (s[0] + s[1] + s[2]);
    const TF be2 = be + be;
    c0 += g * rx + be2 * t0;
    c1 += g * ry + be2 * t1;
    c2 += g * rz + be2 * t2;
}

// c = a1 f + b (r.f) r
template <typename TF>
__device__ inline void apply(TF a1, TF b, TF rx, TF ry, TF rz, TF f0, TF f1, TF f2, TF& c0, TF& c1, TF& c2)
{
    const TF rf = (rx * f0 + ry * f1 + rz * f2) * b;
    c0 = a1 * f0 + rf * rx;
    c1 = a1 * f1 + rf * ry;
    c2 = a1 * f2 + rf * rz;
}

constexpr int kRing = 128;   // LDS ring of filtered candidate sources
constexpr int kTest = 32;    // sources tested per round (queue <= kTest * 64 pairs)

// TF: precision of the pair formula and of the staged forces; TA: accumulator precision.
// Positions and the r^2 < r_c^2 test are FP64 in both modes (same VALU rate as FP32).
// Count: no pair formula; the wave only counts its accepted (target, source) pairs and adds
// the count to *pair_count (one integer atomic per wave): the exact number of ordered pairs
// the near-field sum runs over, for measurement.
template <typename TF, typename TA, int Lv, bool Count = false>
__global__ __launch_bounds__(64) void k_p2p(int n, const Rec64* __restrict__ rec,
                                            const int* __restrict__ start,
                                            const int* __restrict__ chunk_off, Geometry g,
                                            PairArgs a, double* __restrict__ u_near,
                                            unsigned long long* __restrict__ pair_count = nullptr)
{
    __shared__ double tgt[3][kWave];
    __shared__ TA acc[3][kWave];
    __shared__ double ring[3][kRing];
    __shared__ TF ringf[3][kRing];
    __shared__ unsigned short queue[kTest * kWave];

    // plain block order: an XCD-aware order (each XCD sweeping a contiguous range) was
    // measured 12% slower here, unlike in G2P
    const int wave = uniform_i((int)blockIdx.x);
    const int lane = threadIdx.x;
    const int total = chunk_off[g.ntiles * g.nsys];  // chunks of all systems
    if (wave >= total) return;

    // tile of this wave: largest t with chunk_off[t] <= wave
    int lo = 0, hi = g.ntiles * g.nsys;
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

    // tile t of system sys (the systems of a batch have consecutive tile ranges)
    const int sys = t / g.ntiles, tl = t - sys * g.ntiles, tbase = sys * g.ntiles;
    const int tc[3] = {tl / (g.NT[1] * g.NT[2]), (tl / g.NT[2]) % g.NT[1], tl % g.NT[2]};
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
    unsigned long long counted = 0;

    // test the targets against ring sources [rhead, rhead + cnt), then drain the queue
    auto process = [&](int cnt) {
        int qn = 0;
        for (int j = 0; j < cnt; ++j) {
            const int slot = (rhead + j) & (kRing - 1);
            const double rx = tx[0] - ld1(ring[0][slot]), ry = tx[1] - ld1(ring[1][slot]), rz = tx[2] - ld1(ring[2][slot]);
            const double r2 = rx * rx + ry * ry + rz * rz;
            const bool pass = (r2 < a.rc2) && (r2 > 0.0);
            const unsigned long long b = __ballot(pass);
            if (!Count && pass) queue[qn + lanes_below(b)] = (unsigned short)(lane | (j << 6));
            qn += __popcll(b);
        }
        if (Count) {
            counted += (unsigned long long)qn;
            __syncthreads();
            return;
        }
        __syncthreads();
        for (int q0 = 0; q0 < qn; q0 += kWave) {
            const int k = q0 + lane;
            if (k < qn) {
                const int e = queue[k];
                const int tt = e & (kWave - 1);
                const int slot = (rhead + (e >> 6)) & (kRing - 1);
                const double rx = ld1(tgt[0][tt]) - ld1(ring[0][slot]);
                const double ry = ld1(tgt[1][tt]) - ld1(ring[1][slot]);
                const double rz = ld1(tgt[2][tt]) - ld1(ring[2][slot]);
                const double r2 = rx * rx + ry * ry + rz * rz;
                TF a1, b, c0, c1, c2;
                Coef<TF, Lv>::eval(r2, a, a1, b);
                apply<TF>(a1, b, (TF)rx, (TF)ry, (TF)rz, ld1(ringf[0][slot]), ld1(ringf[1][slot]), ld1(ringf[2][slot]), c0,
                          c1, c2);
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
                const int nt = tbase + (wx * g.NT[1] + wy) * g.NT[2] + wz;
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
    if (Count) {
        if (lane == 0 && counted > 0) atomicAdd(pair_count, counted);
        return;
    }
    if (active) {
        const double post = Coef<TF, Lv>::post(a);
        u_near[i] = post * (double)acc[0][lane];
        u_near[(int64_t)n + i] = post * (double)acc[1][lane];
        u_near[2 * (int64_t)n + i] = post * (double)acc[2][lane];
    }
}

// ---------------------------------------------------------------- symmetric form
// G^N is even in r, so one evaluation of a pair (i, j) gives both G^N(r) f_j (to u_i) and
// G^N(r) f_i (to u_j).  Every unordered pair is visited once: a wave walks only the upper
// half of the neighbour-tile offsets D (lexicographically D > 0), plus its own tile (D = 0)
// restricted to sources with a larger sorted index than the target; the mirrored offset
// -D carries the same pairs.  The source side accumulates per ring entry in LDS and is
// added to u^N with one FP64 atomic per component and source when the entry retires.
// u^N is zeroed first.  The order of those atomic additions varies between runs, so
// results agree to rounding, not bitwise (the one-sided kernel above is the reproducible
// variant).
//
// Balanced drain.  LDS traffic, not arithmetic, bounded an earlier form that put every
// accepted pair through an LDS queue (six LDS atomics and twelve operand loads per pair), so
// the target side is kept in registers where possible.  Per batch of 32 ring entries each
// lane tests its own target against all of them (a 32-bit mask; all lanes read the same
// entry, an LDS broadcast).  With Q accepted pairs the batch takes R = ceil(Q / 64) rounds
// of one pair per lane; a lane keeps up to R pairs of its own target (summed in registers)
// and puts the rest in a queue, from which lanes with fewer than R pairs take work in their
// spare rounds (target side by LDS atomics, about 15% of the pairs at uniform density).
// Each lane takes its own sources in cyclic order from its (lane mod c)-th accepted one (c its
// pair count), so that the lanes of a half-wave start on different sources also when their
// accepted sets are alike (fewer collisions on the batch's source accumulators).  The ring
// and target slots are read one value per LDS instruction (ld1).  With stresslet sources the
// same schedule carries the stresslet pair terms as well.
//
// Cutoff test on the matrix cores.  The targets' positions t' and the ring's sources s' are taken
// relative to the centre of the targets' bounding box, so that |s' - t'|^2 < r_c^2 can be tested
// in the expanded form |s'|^2 - 2 s'.t' < r_c^2 - |t'|^2 without cancellation beyond a few ulps of
// (box diagonal + r_c)^2.  A full batch past the own tile (32 sources x 64 targets) is eight
// v_mfma_f64_16x16x4f64 (sources as rows with K = (x, y, z, |s'|^2), targets as columns with
// K = (-2x, -2y, -2z, 1)) and 32 comparisons per lane, instead of 32 broadcast LDS reads and six
// FP64 operations per source: c2 P2P 22.9 -> 21.3 ms, H 12.2 -> 11.3 ms.  The own tile, whose
// pairs also need r > 0 and the index order, and the last, shorter batch keep the direct test;
// the direct difference of repeated positions is exactly 0 also in the centred frame.
constexpr int kSymRing = 64;
constexpr int kFar = 1 << 30;  // ring key offset of sources outside the targets' own tile
// Balanced drain: batches of 32 ring entries and one copy of the source
// accumulators (a second copy, for lanes 32-63, was measured 2% slower: the LDS it takes
// costs more occupancy than the atomic collisions it saves).  Queue bound: with c_t <= 32
// pairs per lane, Q = sum c_t and R = ceil(Q / 64) rounds, the excess sum over c_t >= R
// of (c_t - R) is at most Q (32 - R) / 32 <= 2 R (32 - R) <= 512.
constexpr int kBalBatch = 32;
constexpr int kBalExcess = 512;
static_assert(kBalBatch == 32 && kSymRing == 64, "the mask, ring and queue sizes assume 32-entry batches");

// wave ballot of a condition, without materialising it as an integer first
__device__ inline unsigned long long ballot(bool p) { return __builtin_amdgcn_ballot_w64(p); }

__global__ void k_zero_f64(double* __restrict__ p, int64_t count)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) p[i] = 0.0;
}

// ST: stresslet sources too (srec: sorted symmetric tensors, 6 per particle); T^N is odd,
// so the source side of a pair takes -T^N(r) S_target.
template <typename TF, int Lv, bool ST>
__global__ __launch_bounds__(64) void k_p2p_sym(int n, const Rec64* __restrict__ rec,
                                                const double* __restrict__ srec,
                                                const int* __restrict__ start,
                                                const int* __restrict__ chunk_off, Geometry g,
                                                PairArgs a, double* __restrict__ u_near, int nsplit)
{
    constexpr int NS = ST ? 6 : 1;
    __shared__ double tgt[4][kWave];  // t' (x, y, z) and r_c^2 - |t'|^2
    __shared__ TF tgtf[3][kWave];
    __shared__ TF tgts[NS][kWave];
    __shared__ TF rings[NS][kSymRing];
    __shared__ double acc[3][kWave];
    __shared__ double ring[3][kSymRing];
    __shared__ TF ringf[3][kSymRing];
    __shared__ int ringk[kSymRing];
    // batch size and copies of the per-batch source accumulators (per component, copy, entry)
    constexpr int kB = kBalBatch;
    constexpr int kCp = 1;
    __shared__ double racc[3][kCp][kB];
    __shared__ unsigned short queue[kBalExcess];
    static_assert(kSymRing == kWave, "one ring slot per lane");

    // plain block order: an XCD-aware order (each XCD sweeping a contiguous range) was
    // measured 12% slower here, unlike in G2P
    // nsplit waves share a chunk, each taking every nsplit-th of its neighbour tiles (shorter
    // waves: a smaller tail when the last waves of the launch run)
    const int wave = uniform_i((int)blockIdx.x) / nsplit;
    const int part = uniform_i((int)blockIdx.x) % nsplit;
    const int lane = threadIdx.x;
    const int total = chunk_off[g.ntiles * g.nsys];  // chunks of all systems
    if (wave >= total) return;

    int lo = 0, hi = g.ntiles * g.nsys;
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

    // tile t of system sys (the systems of a batch have consecutive tile ranges)
    const int sys = t / g.ntiles, tl = t - sys * g.ntiles, tbase = sys * g.ntiles;
    const int tc[3] = {tl / (g.NT[1] * g.NT[2]), (tl / g.NT[2]) % g.NT[1], tl % g.NT[2]};
    // positions relative to the centre of the targets' bounding box (see the cutoff test above)
    double w[3], blo[3], bhi[3], cen[3], tx[3], oacc[3];
    double tlim = a.rc2;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        w[d] = g.B * g.h[d];
        blo[d] = uniform_d(wave_min(me.x[d]));
        bhi[d] = uniform_d(wave_max(me.x[d]));
        cen[d] = uniform_d(0.5 * (blo[d] + bhi[d]));
        tx[d] = active ? me.x[d] - cen[d] : 1e30;  // an inactive lane accepts no pair
        tlim -= tx[d] * tx[d];
        tgt[d][lane] = tx[d];
        tgtf[d][lane] = (TF)me.f[d];
        acc[d][lane] = 0.0;
        if (lane < kCp * kB) racc[d][lane / kB][lane % kB] = 0.0;
        oacc[d] = 0.0;
    }
    tgt[3][lane] = tlim;
    if (ST) {
        const int ii = active ? i : first;
#pragma unroll
        for (int c = 0; c < NS; ++c) tgts[c][lane] = (TF)srec[6 * (int64_t)ii + c];
    }
    __syncthreads();
    const int mi = lane & 15, mk = lane >> 4;  // lane = 16 mk + mi
    // the stresslet formula (CoefSt) returns its coefficients unscaled
    const double post = ST ? 1.0 : Coef<TF, Lv>::post(a);

    int rhead = 0, rcount = 0;
    int tk = 0;  // neighbour tiles met so far (those within r_c of the targets)

    auto process = [&](int cnt) {
        // 1. test: bit j of m is set when this lane's target pairs with batch entry j (all
        //    lanes read the same entry: LDS broadcast)
        //    Sources of other tiles are never at r = 0 and always follow the wave's own
        //    tile in the ring, so a batch whose first entry is not of the own tile needs
        //    only the cutoff test.
        unsigned m = 0;
        int qn = 0;
        const bool own_tile = uniform_i(ringk[rhead]) < kFar;
        if (own_tile) {
            for (int j = 0; j < cnt; ++j) {
                const int slot = (rhead + j) & (kSymRing - 1);
                const double rx = tx[0] - ld1(ring[0][slot]), ry = tx[1] - ld1(ring[1][slot]), rz = tx[2] - ld1(ring[2][slot]);
                const double r2 = rx * rx + ry * ry + rz * rz;
                const bool pass = (r2 < a.rc2) & (r2 > 0.0) & (ringk[slot] > i);
                m = pass ? (m | (1u << j)) : m;
                qn += __popcll(ballot(pass));
            }
        } else if (cnt == kB) {
            // a full batch past the own tile: |s' - t'|^2 < r_c^2  <=>  |s'|^2 - 2 s'.t' < r_c^2 - |t'|^2,
            // for 32 sources x 64 targets by eight v_mfma_f64_16x16x4f64 (sources as rows, targets
            // as columns).  On gfx950 lane l = 16 kq + i supplies A[i][kq] and B[kq][i] and receives
            // D[4 r + kq][i], r = 0..3.  Batches start at ring slot 0 or 32 (32 entries at a time
            // from a 64-slot ring), so the batch's slots need no wrap.  Source row rho of block mb is
            // loaded from slot 16 mb + 4 (rho % 4) + rho / 4, so that result item r of lane (kq, i)
            // -- row 4 r + kq -- is slot 16 mb + 4 kq + r: a lane's four items are four consecutive
            // bits of the batch mask.
            typedef double v4d __attribute__((ext_vector_type(4)));
            double av[2];
#pragma unroll
            for (int mb = 0; mb < 2; ++mb) {
                const int slot = rhead + 16 * mb + 4 * (mi & 3) + (mi >> 2);
                const double x0 = ld1(ring[0][slot]), x1 = ld1(ring[1][slot]), x2 = ld1(ring[2][slot]);
                av[mb] = mk == 0 ? x0 : mk == 1 ? x1 : mk == 2 ? x2 : fma(x0, x0, fma(x1, x1, x2 * x2));
            }
            // column block nb: targets 16 nb + i; operand B[kq][i] = -2 t'_kq (kq = 3: 1).  The bits of
            // target 16 nb + i are spread over lanes (kq, i), kq = 0..3: OR over the four rows, kept
            // by the lanes of row nb (the target's own lane)
#pragma unroll
            for (int nb = 0; nb < 4; ++nb) {
                const double tk = tgt[mk < 3 ? mk : 0][16 * nb + mi];
                const double bt = mk < 3 ? -2.0 * tk : 1.0;
                const double lim = tgt[3][16 * nb + mi];
                unsigned wv = 0;
#pragma unroll
                for (int mb = 0; mb < 2; ++mb) {
                    const v4d dd = __builtin_amdgcn_mfma_f64_16x16x4f64(av[mb], bt, v4d{0.0, 0.0, 0.0, 0.0}, 0, 0, 0);
                    unsigned nib = 0;
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const bool p = dd[r] < lim;
                        nib |= p ? (1u << r) : 0u;
                        qn += __popcll(ballot(p));
                    }
                    wv |= nib << (16 * mb + 4 * mk);
                }
                wv = or_rows4(wv);
                m = mk == nb ? wv : m;
                __builtin_amdgcn_sched_barrier(0);
            }
        } else {
            for (int j = 0; j < cnt; ++j) {
                const int slot = (rhead + j) & (kSymRing - 1);
                const double rx = tx[0] - ld1(ring[0][slot]), ry = tx[1] - ld1(ring[1][slot]), rz = tx[2] - ld1(ring[2][slot]);
                const bool pass = rx * rx + ry * ry + rz * rz < a.rc2;
                m = pass ? (m | (1u << j)) : m;
                qn += __popcll(ballot(pass));
            }
        }
        const int rounds = (qn + kWave - 1) / kWave;
        // 2. a lane keeps up to `rounds` of its target's pairs, taken in cyclic order from its
        //    (lane mod c)-th accepted source (c: its number of pairs), so that the lanes of a
        //    half-wave start on different sources even when their accepted sets are alike (a
        //    rotation by the lane number alone sent the lanes whose start lies outside a common
        //    band of accepted sources to the band's first source together: same-address LDS
        //    atomics); the excess goes to the queue, for lanes that run out of pairs of their own
        const int c = __popc(m);
        const int rot = c ? select_bit(m, lane % c) : 0;
        const unsigned rm0 = rot ? ((m >> rot) | (m << (kB - rot))) : m;
        unsigned rm = rm0;
        const int own_n = c < rounds ? c : rounds;
        int ex = c - own_n;
        int qx = 0;
        for (;;) {
            const bool wr = ex > 0;
            const unsigned long long bw = ballot(wr);
            if (bw == 0) break;
            if (wr) {
                const int p = 31 - __clz(rm);
                rm ^= 1u << p;
                queue[qx + lanes_below(bw)] = (unsigned short)(lane | (((p + rot) & (kB - 1)) << 6));
                --ex;
            }
            qx += __popcll(bw);
        }
        __syncthreads();
        // 3. `rounds` rounds of one pair per lane; a lane's own target's side is summed in
        //    registers, the source side goes to the batch's source accumulators.
        // The pair (target tt at position p with force tf, ring slot): c = G^N(r) f_source for
        // the target, d = G^N(-r) f_target for the source (r = p - x_source)
        auto pair = [&](double p0, double p1, double p2, TF tf0, TF tf1, TF tf2, int tt, int slot, TF& c0,
                        TF& c1, TF& c2, TF& d0, TF& d1, TF& d2) {
            const double rx = p0 - ld1(ring[0][slot]);
            const double ry = p1 - ld1(ring[1][slot]);
            const double rz = p2 - ld1(ring[2][slot]);
            const double r2 = rx * rx + ry * ry + rz * rz;
            TF a1, b;
            if constexpr (ST) {
                TF al, be;
                CoefSt<TF, Lv>::eval(r2, a, a1, b, al, be);
                apply<TF>(a1, b, (TF)rx, (TF)ry, (TF)rz, ld1(ringf[0][slot]), ld1(ringf[1][slot]), ld1(ringf[2][slot]), c0,
                          c1, c2);
                apply<TF>(a1, b, (TF)rx, (TF)ry, (TF)rz, tf0, tf1, tf2, d0, d1, d2);
                TF ss[6], st[6];
#pragma unroll
                for (int c = 0; c < 6; ++c) {
                    ss[c] = ld1(rings[c][slot]);
                    st[c] = -ld1(tgts[c][tt]);  // T^N(-r) = -T^N(r)
                }
                apply_st<TF>(al, be, (TF)rx, (TF)ry, (TF)rz, ss, c0, c1, c2);
                apply_st<TF>(al, be, (TF)rx, (TF)ry, (TF)rz, st, d0, d1, d2);
            } else {
                Coef<TF, Lv>::eval(r2, a, a1, b);
                apply<TF>(a1, b, (TF)rx, (TF)ry, (TF)rz, ld1(ringf[0][slot]), ld1(ringf[1][slot]), ld1(ringf[2][slot]), c0,
                          c1, c2);
                apply<TF>(a1, b, (TF)rx, (TF)ry, (TF)rz, tf0, tf1, tf2, d0, d1, d2);
            }
        };
        const int rq = lane / (kWave / kCp);
        // 3a. rounds in which every lane still takes a pair of its own target (about a third
        //     at uniform density): no queue, no ballot, and the target's position and force
        //     come from registers
        const int own_all = wave_min_small(own_n);
        // the lane's target (position, force).  At the reduced-cost FP64 levels the all-own rounds
        // sum the target side straight into the FMAs, and a lane that runs out of pairs of its
        // own overwrites these registers with a donated pair's target in the queue rounds (c2
        // P2P -1.4%); at level 0 and in FP32 both cost more registers or time than they save
        constexpr bool kRegTarget = std::is_same<TF, double>::value && Lv > 0;
        double px = tx[0], py = tx[1], pz = tx[2];
        TF mf0 = (TF)me.f[0], mf1 = (TF)me.f[1], mf2 = (TF)me.f[2];
        for (int r = 0; r < own_all; ++r) {
            const int sl = (__builtin_ctz(rm) + rot) & (kB - 1);
            rm &= rm - 1;
            const int slot = rhead + sl;
            if constexpr (!ST && kRegTarget) {
                // the target side summed straight into the FMAs: oacc += a1 f_s + b (r.f_s) r
                const double rx = px - ld1(ring[0][slot]), ry = py - ld1(ring[1][slot]), rz = pz - ld1(ring[2][slot]);
                double a1, b;
                Coef<double, Lv>::eval(rx * rx + ry * ry + rz * rz, a, a1, b);
                const double s0 = ld1(ringf[0][slot]), s1 = ld1(ringf[1][slot]), s2 = ld1(ringf[2][slot]);
                const double rs = (rx * s0 + ry * s1 + rz * s2) * b;
                oacc[0] = fma(rs, rx, fma(a1, s0, oacc[0]));
                oacc[1] = fma(rs, ry, fma(a1, s1, oacc[1]));
                oacc[2] = fma(rs, rz, fma(a1, s2, oacc[2]));
                const double rt = (rx * mf0 + ry * mf1 + rz * mf2) * b;
                atomicAdd(&racc[0][rq][sl], fma(a1, mf0, rt * rx));
                atomicAdd(&racc[1][rq][sl], fma(a1, mf1, rt * ry));
                atomicAdd(&racc[2][rq][sl], fma(a1, mf2, rt * rz));
                continue;
            }
            TF c0, c1, c2, d0, d1, d2;
            pair(px, py, pz, mf0, mf1, mf2, lane, slot, c0, c1, c2, d0, d1, d2);
            oacc[0] += (double)c0;
            oacc[1] += (double)c1;
            oacc[2] += (double)c2;
            atomicAdd(&racc[0][rq][sl], (double)d0);
            atomicAdd(&racc[1][rq][sl], (double)d1);
            atomicAdd(&racc[2][rq][sl], (double)d2);
        }
        // 3b. the remaining rounds, one pair per lane: the lane's own target while it has
        //     pairs, then queue entries in order (target side by LDS atomics)
        int qb = 0;
        for (int r = own_all; r < rounds; ++r) {
            // every lane reads a queue entry (in range, used only by donated lanes)
            const bool own = r < own_n;
            const unsigned long long bi = ballot(!own);
            const int q = qb + lanes_below(bi);
            qb += __popcll(bi);
            const bool don = !own && q < qx;
            const int e = queue[q < qx ? q : 0];
            const int pb = __builtin_ctz(rm);  // used by own lanes only (rm != 0)
            if constexpr (!kRegTarget) rm = own ? (rm & (rm - 1)) : rm;
            const int tt = own ? lane : (e & (kWave - 1));
            const int sl = own ? ((pb + rot) & (kB - 1)) : ((e >> 6) & (kB - 1));
            const int slot = rhead + sl;
            // own lanes take their target from registers, donated lanes from LDS (the volatile
            // loads stay under the branch, so own lanes add no LDS traffic)
            TF c0, c1, c2, d0, d1, d2;
            if constexpr (kRegTarget) {
                // a lane that is not own in this round is not own in any later one: it
                // overwrites its target registers
                if (!own) {
                    px = ld1(tgt[0][tt]);
                    py = ld1(tgt[1][tt]);
                    pz = ld1(tgt[2][tt]);
                    mf0 = ld1(tgtf[0][tt]);
                    mf1 = ld1(tgtf[1][tt]);
                    mf2 = ld1(tgtf[2][tt]);
                }
                pair(px, py, pz, mf0, mf1, mf2, tt, slot, c0, c1, c2, d0, d1, d2);
                if (own) {
                    // an empty volatile asm keeps this a branch (the if-converted form takes
                    // two selects per component)
                    asm volatile("");
                    oacc[0] += (double)c0;
                    oacc[1] += (double)c1;
                    oacc[2] += (double)c2;
                    rm &= rm - 1;
                }
            } else {
                double q0 = px, q1 = py, q2 = pz;
                TF g0 = mf0, g1 = mf1, g2 = mf2;
                if (!own) {
                    q0 = ld1(tgt[0][tt]);
                    q1 = ld1(tgt[1][tt]);
                    q2 = ld1(tgt[2][tt]);
                    g0 = ld1(tgtf[0][tt]);
                    g1 = ld1(tgtf[1][tt]);
                    g2 = ld1(tgtf[2][tt]);
                }
                pair(q0, q1, q2, g0, g1, g2, tt, slot, c0, c1, c2, d0, d1, d2);
                if (own) {
                    oacc[0] += (double)c0;
                    oacc[1] += (double)c1;
                    oacc[2] += (double)c2;
                }
            }
            if (don) {
                atomicAdd(&acc[0][tt], (double)c0);
                atomicAdd(&acc[1][tt], (double)c1);
                atomicAdd(&acc[2][tt], (double)c2);
            }
            if (own || don) {
                atomicAdd(&racc[0][rq][sl], (double)d0);
                atomicAdd(&racc[1][rq][sl], (double)d1);
                atomicAdd(&racc[2][rq][sl], (double)d2);
            }
        }
        __syncthreads();
        // retire the cnt ring sources: their source-side sums go to u^N
        if (lane < cnt) {
            const int slot = (rhead + lane) & (kSymRing - 1);
            double v0 = 0.0, v1 = 0.0, v2 = 0.0;
#pragma unroll
            for (int rq = 0; rq < kCp; ++rq) {
                v0 += racc[0][rq][lane];
                v1 += racc[1][rq][lane];
                v2 += racc[2][rq][lane];
                racc[0][rq][lane] = 0.0;
                racc[1][rq][lane] = 0.0;
                racc[2][rq][lane] = 0.0;
            }
            if (v0 != 0.0 || v1 != 0.0 || v2 != 0.0) {
                const int64_t jj = ringk[slot] & (kFar - 1);
                unsafeAtomicAdd(&u_near[jj], post * v0);
                unsafeAtomicAdd(&u_near[(int64_t)n + jj], post * v1);
                unsafeAtomicAdd(&u_near[2 * (int64_t)n + jj], post * v2);
            }
        }
        __syncthreads();
    };

    for (int dx = 0; dx <= g.S[0]; ++dx) {
        const int ux = tc[0] + dx;
        const int fx = floor_div(ux, g.NT[0]);
        const int wx = ux - fx * g.NT[0];
        const double shx = fx * g.L[0];
        const double gx = fmax(0.0, fmax(ux * w[0] - bhi[0], blo[0] - (ux + 1) * w[0]));
        for (int dy = (dx == 0 ? 0 : -g.S[1]); dy <= g.S[1]; ++dy) {
            const int uy = tc[1] + dy;
            const int fy = floor_div(uy, g.NT[1]);
            const int wy = uy - fy * g.NT[1];
            const double shy = fy * g.L[1];
            const double gy = fmax(0.0, fmax(uy * w[1] - bhi[1], blo[1] - (uy + 1) * w[1]));
            if (gx * gx + gy * gy >= a.rc2) continue;
            for (int dz = (dx == 0 && dy == 0 ? 0 : -g.S[2]); dz <= g.S[2]; ++dz) {
                const int uz = tc[2] + dz;
                const int fz = floor_div(uz, g.NT[2]);
                const int wz = uz - fz * g.NT[2];
                const double shz = fz * g.L[2];
                const double gz = fmax(0.0, fmax(uz * w[2] - bhi[2], blo[2] - (uz + 1) * w[2]));
                if (gx * gx + gy * gy + gz * gz >= a.rc2) continue;
                if (tk++ % nsplit != part) continue;  // another wave of this chunk takes it
                const bool own = (dx == 0 && dy == 0 && dz == 0);
                const int nt = tbase + (wx * g.NT[1] + wy) * g.NT[2] + wz;
                // own tile: sources below the first target can pair with none of them
                const int sa = own ? first : start[nt * per], sb = start[(nt + 1) * per];
                const int koff = own ? 0 : kFar;
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
                        sx -= cen[0];
                        sy -= cen[1];
                        sz -= cen[2];
                    }
                    // append in two halves so the 64-slot ring never holds more than 63
#pragma unroll
                    for (int half = 0; half < 2; ++half) {
                        const bool mine = keep && ((lane >> 5) == half);
                        const unsigned long long bm = __ballot(mine);
                        if (mine) {
                            const int slot = (rhead + rcount + lanes_below(bm)) & (kSymRing - 1);
                            ring[0][slot] = sx;
                            ring[1][slot] = sy;
                            ring[2][slot] = sz;
                            ringf[0][slot] = (TF)f0;
                            ringf[1][slot] = (TF)f1;
                            ringf[2][slot] = (TF)f2;
                            ringk[slot] = koff + s;
                            if (ST) {
#pragma unroll
                                for (int c = 0; c < NS; ++c) rings[c][slot] = (TF)srec[6 * (int64_t)s + c];
                            }
                        }
                        rcount += __popcll(bm);
                        __syncthreads();
                        while (rcount >= kB) {
                            process(kB);
                            rhead = (rhead + kB) & (kSymRing - 1);
                            rcount -= kB;
                        }
                    }
                }
            }
        }
    }
    while (rcount > 0) {
        const int c = rcount < kB ? rcount : kB;
        process(c);
        rhead = (rhead + c) & (kSymRing - 1);
        rcount -= c;
    }
    if (active) {
        unsafeAtomicAdd(&u_near[i], post * (acc[0][lane] + oacc[0]));
        unsafeAtomicAdd(&u_near[(int64_t)n + i], post * (acc[1][lane] + oacc[1]));
        unsafeAtomicAdd(&u_near[2 * (int64_t)n + i], post * (acc[2][lane] + oacc[2]));
    }
}

}  // namespace

namespace {

PairArgs pair_args(const Plan& pl, int lv)
{
    PairArgs a;
    a.xi = pl.xi;
    a.xi2 = pl.xi * pl.xi;
    a.rc2 = pl.rc * pl.rc;
    a.four_xi_over_sqrtpi = 4.0 * pl.xi / sqrt(M_PI);
    a.xi2_log2e = a.xi2 * kLog2e;
    a.six_xi_over_sqrtpi = 6.0 * pl.xi / sqrt(M_PI);
    a.four_xi3_over_sqrtpi = 4.0 * pl.xi * pl.xi * pl.xi / sqrt(M_PI);
    const double* ms = lv == 2 ? kScreenM64f : lv == 1 ? kScreenM64s : kScreenM64;
    const int ds = lv == 2 ? kScreenDeg64f : lv == 1 ? kScreenDeg64s : kScreenDeg64;
    for (int k = 0; k < kScreenDeg64; ++k) a.ms[k] = k < ds ? ms[k] : 0.0;
    a.lead_s = lv == 2 ? kScreenLead64f : lv == 1 ? kScreenLead64s : kScreenLead64;
    const double* me = lv == 2 ? kExpM2 : kExpM1;
    const int de = lv == 2 ? kExpDeg2 : kExpDeg1;
    for (int k = 0; k < kExpDeg1; ++k) a.me[k] = k < de ? me[k] : 0.0;
    a.lead_e = lv == 0 ? 1.0 : lv == 2 ? kExpLead2 : kExpLead1;
    a.zc = -a.xi2 * kLog2e;
    a.zc32 = (float)a.zc;
    a.g = kTwoOverSqrtPi / a.lead_s;
    a.h = a.four_xi_over_sqrtpi / a.lead_s;
    a.post = a.lead_s * a.lead_e;
    for (int k = 0; k <= kScreenDeg32; ++k) a.c32[k] = (float)kScreenC32[k];
    return a;
}

__global__ void k_zero_u64(unsigned long long* p) { *p = 0ull; }

}  // namespace

hipError_t launch_count_pairs(const Plan& pl, const Work& w, int n, unsigned long long* count, hipStream_t s,
                              int nsys)
{
    hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(1), 0, s, count);
    if (n > 0) {
        const PairArgs a = pair_args(pl, 0);
        Geometry g = pl.g;
        g.nsys = nsys;
        const int64_t waves = (int64_t)g.ntiles * nsys + (n + kWave - 1) / kWave;
        hipLaunchKernelGGL((k_p2p<double, double, 0, true>), dim3((unsigned)waves), dim3(kWave), 0, s, n,
                           (const Rec64*)w.rec, w.start, w.chunk_off, g, a, nullptr, count);
    }
    return hipGetLastError();
}

// the FP64 pair formula's accuracy level for a plan's tolerance (see PairArgs)
static int pair_level(double tol) { return tol >= 1e-8 ? 2 : tol >= 1e-10 ? 1 : 0; }

template <typename TF, int Lv>
void launch_p2p_det(const Plan& pl, const Work& w, int n, hipStream_t s, const Geometry& g, const PairArgs& a,
                    dim3 grid)
{
    hipLaunchKernelGGL((k_p2p<TF, double, Lv>), grid, dim3(kWave), 0, s, n, (const Rec64*)w.rec, w.start,
                       w.chunk_off, g, a, w.u_near);
}

template <typename TF, int Lv, bool ST>
void launch_p2p_sym(const Work& w, int n, hipStream_t s, const Geometry& g, const PairArgs& a, dim3 grid, int split)
{
    hipLaunchKernelGGL((k_p2p_sym<TF, Lv, ST>), grid, dim3(kWave), 0, s, n, (const Rec64*)w.rec, w.srec, w.start,
                       w.chunk_off, g, a, w.u_near, split);
}

hipError_t launch_p2p(const Plan& pl, const Work& w, int n, hipStream_t s, bool st, int nsys)
{
    if (n <= 0) return hipSuccess;
    const bool f64 = pl.mode == EWALD_FP64;
    const int lv = f64 ? pair_level(pl.p.tol) : -1;  // -1: the FP32 formula
    const PairArgs a = pair_args(pl, lv < 0 ? 0 : lv);
    Geometry g = pl.g;
    g.nsys = nsys;
    const int64_t waves = (int64_t)g.ntiles * nsys + (n + kWave - 1) / kWave;
    const dim3 grid((unsigned)waves);
    if (pl.deterministic && !st) {
        // FP32 bulk accumulates in FP64 as well: LDS atomic adds of FP64 are fast on
        // gfx950, those of FP32 are not (measured: 3x slower kernel)
        switch (lv) {
        case 0: launch_p2p_det<double, 0>(pl, w, n, s, g, a, grid); break;
        case 1: launch_p2p_det<double, 1>(pl, w, n, s, g, a, grid); break;
        case 2: launch_p2p_det<double, 2>(pl, w, n, s, g, a, grid); break;
        default: launch_p2p_det<float, 0>(pl, w, n, s, g, a, grid); break;
        }
        return hipGetLastError();
    }
    // Symmetric kernel: three waves per chunk (each taking every third neighbour tile) shorten the
    // waves and so the launch's tail.  Measured P2P ms for 1 / 2 / 3 / 4 / 6 waves per chunk: c2
    // (17k chunks) 20.1 / 18.7 / 18.5 / 19.5 / 18.7; H 10.8 / 10.4 / 10.1 / 11.6 / 10.4; c4 (63k)
    // 51.7 / 51.4 / 50.9 / 55.6 / 52.1; clustered c3 (160k) 172.7 / 177.6 / 172.2 / 231.8 / 182.2.
    // With fewer chunks than wave slots, six (c1, N = 1e3: 0.158 / 0.093 / 0.098 / 0.072 / 0.063).
    const int kSplit = waves < 2048 ? 6 : 3;
    const dim3 sgrid((unsigned)(waves * kSplit));
    const int64_t cnt = 3 * (int64_t)n;
    hipLaunchKernelGGL(k_zero_f64, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, s, w.u_near, cnt);
    if (st) {
        switch (lv) {
        case 0: launch_p2p_sym<double, 0, true>(w, n, s, g, a, sgrid, kSplit); break;
        case 1: launch_p2p_sym<double, 1, true>(w, n, s, g, a, sgrid, kSplit); break;
        case 2: launch_p2p_sym<double, 2, true>(w, n, s, g, a, sgrid, kSplit); break;
        default: launch_p2p_sym<float, 0, true>(w, n, s, g, a, sgrid, kSplit); break;
        }
        return hipGetLastError();
    }
    switch (lv) {
    case 0: launch_p2p_sym<double, 0, false>(w, n, s, g, a, sgrid, kSplit); break;
    case 1: launch_p2p_sym<double, 1, false>(w, n, s, g, a, sgrid, kSplit); break;
    case 2: launch_p2p_sym<double, 2, false>(w, n, s, g, a, sgrid, kSplit); break;
    default: launch_p2p_sym<float, 0, false>(w, n, s, g, a, sgrid, kSplit); break;
    }
    return hipGetLastError();
}

}  // namespace ewald
