// C ABI of the spectral Ewald library: plan (parameter selection, tables), workspace
// layout, and the stage sequence of Algorithm "se".
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "internal.h"
#include "screening.h"
#include "window.h"

namespace ewald {
int p2g_max_runs();
}

using namespace ewald;

namespace {

thread_local std::string g_err;
thread_local int g_fail_next = 0;  // evaluations left to fail (ewald_debug_fail_next)

int fail(int code, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
int fail(int code, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

int hip_fail(hipError_t e, const char* what)
{
    return fail(EWALD_EHIP, "%s: %s", what, hipGetErrorString(e));
}

bool is_pow2(int v) { return v > 0 && (v & (v - 1)) == 0; }
int ilog2(int v)
{
    int l = 0;
    while ((1 << l) < v) ++l;
    return l;
}
int next_pow2(double v)
{
    int p = 1;
    while (p < v) p *= 2;
    return p;
}

// ---- error estimates, Sec. 2.4 eq. (ese) (unit box, unit force norm) ----

double err_near(double xi, double rc)
{
    return std::sqrt(112.0 / 9.0 * std::pow(xi, 4) * rc * rc * rc) * std::exp(-xi * xi * rc * rc);
}

double err_far(double xi, double h)
{
    return 4.0 / (3.0 * h) * std::sqrt(3.5) * std::exp(-M_PI * M_PI / std::pow(2.0 * h * xi, 2));
}

// xi with E^F(xi, h) = target: pi^2 / (2 h xi)^2 = ln(4 sqrt(7/2) / (3 h target))
double xi_from_grid(double h, double target)
{
    const double a = std::log(4.0 * std::sqrt(3.5) / (3.0 * h * target));
    if (a <= 0.1) return M_PI / (2.0 * h * std::sqrt(0.1));
    return M_PI / (2.0 * h * std::sqrt(a));
}

// h with E^F(xi, h) = target (E^F increases with h on the branch of interest): bisection
double h_from_xi(double xi, double target)
{
    double lo = 1e-6 / xi, hi = 10.0 / xi;
    for (int it = 0; it < 200; ++it) {
        const double mid = std::sqrt(lo * hi);
        if (err_far(xi, mid) > target) hi = mid; else lo = mid;
    }
    return lo;
}

// r_c with E^N(xi, r_c) = target, on the decreasing branch r_c > 1/xi
double rc_from_xi(double xi, double target)
{
    double lo = 1.0 / xi, hi = 40.0 / xi;
    if (err_near(xi, lo) <= target) return lo;
    for (int it = 0; it < 200; ++it) {
        const double mid = 0.5 * (lo + hi);
        if (err_near(xi, mid) > target) lo = mid; else hi = mid;
    }
    return hi;
}

// xi with E^N(xi, r_c) = target for a given r_c (E^N decreases with xi for xi r_c > 1)
double xi_from_rc(double rc, double target)
{
    double lo = 1.0 / rc, hi = 40.0 / rc;
    for (int it = 0; it < 200; ++it) {
        const double mid = 0.5 * (lo + hi);
        if (err_near(mid, rc) > target) lo = mid; else hi = mid;
    }
    return hi;
}

// Gaussian window error model (relative to the far field).  Truncating the Gaussian at
// |d| = P h / 2 leaves e^{-m^2/2}; sampling it on the grid aliases the band k ~ 2 pi/h - k
// onto k, attenuated by what(2 pi/h - k)/what(k) and weighted by Ghat^F(k) ~ e^{-k^2/(4 xi^2)};
// the worst k gives exp(-(pi^2 P^2 / (2 m^2)) (1 - eta/2)), eta = (P h xi / m)^2.
double err_window(int P, double m, double h, double xi)
{
    const double eta = std::pow(P * h * xi / m, 2);
    const double alias = std::exp(-(M_PI * M_PI * P * P / (2.0 * m * m)) * std::max(0.0, 1.0 - 0.5 * eta));
    return std::exp(-0.5 * m * m) + alias;
}

double best_shape(int P, double h, double xi)
{
    double best_m = std::sqrt(M_PI * P), best_e = 1e300;
    for (double c = 0.6; c <= 1.4; c += 0.002) {
        const double m = c * std::sqrt(M_PI * P);
        const double e = err_window(P, m, h, xi);
        if (e < best_e) {
            best_e = e;
            best_m = m;
        }
    }
    return best_m;
}

// Kaiser-Bessel window (Sec. 2.2), with beta tuned per support: relative far-field error
// (log10) and the best beta/P at P = 6..16, measured against the direct Fourier sum for
// uniform particles at four values of xi h (the window error depends on xi h through the
// band the deconvolution amplifies).  Rows whose error stops falling with P have reached
// that grid's own Fourier truncation.  Interpolated linearly in xi h (clamped).
const double kKbXh[4] = {0.22, 0.28, 0.33, 0.40};
const int kKbP[6] = {6, 8, 10, 12, 14, 16};
const double kKbLogErr[4][6] = {{-6.20, -8.37, -10.40, -12.27, -13.78, -14.31},
                                {-5.90, -7.84, -9.60, -11.16, -12.48, -13.41},
                                {-5.68, -7.38, -8.75, -9.74, -10.26, -10.31},
                                {-5.25, -6.51, -7.14, -7.22, -7.22, -7.22}};
const double kKbBetaOverP[4][6] = {{2.8, 2.7, 2.6, 2.6, 2.4, 2.4},
                                   {2.7, 2.5, 2.4, 2.3, 2.2, 2.1},
                                   {2.5, 2.4, 2.2, 2.1, 1.9, 1.8},
                                   {2.3, 2.1, 1.9, 1.7, 1.6, 1.6}};

double kb_interp(const double tab[4][6], int P, double xh)
{
    int pi = 0;
    while (pi < 5 && kKbP[pi] < P) ++pi;
    xh = std::min(std::max(xh, kKbXh[0]), kKbXh[3]);
    int r = 0;
    while (r < 2 && xh > kKbXh[r + 1]) ++r;
    const double f = (xh - kKbXh[r]) / (kKbXh[r + 1] - kKbXh[r]);
    return (1.0 - f) * tab[r][pi] + f * tab[r + 1][pi];
}

double err_window_kb(int P, double h, double xi) { return std::pow(10.0, kb_interp(kKbLogErr, P, h * xi)); }
double kb_beta_over_p(int P, double h, double xi) { return kb_interp(kKbBetaOverP, P, h * xi); }

// 1D Kaiser-Bessel window at distance u (in grid spacings), support |u| < P/2, and its
// Fourier transform at k (a = P h / 2): 2a sinh(sqrt(beta^2 - (ka)^2)) / (sqrt(.) I0(beta)).
double kb_w(double u, int P, double beta)
{
    const double z = 1.0 - std::pow(2.0 * u / P, 2);
    return std::cyl_bessel_i(0.0, beta * std::sqrt(std::max(z, 0.0))) / std::cyl_bessel_i(0.0, beta);
}

double kb_hat(double k, double a, double beta)
{
    const double q = beta * beta - (k * a) * (k * a);
    const double sq = std::sqrt(std::fabs(q));
    double hyp = 1.0;
    if (sq > 0) hyp = (q > 0) ? std::sinh(sq) / sq : std::sin(sq) / sq;
    return 2.0 * a * hyp / std::cyl_bessel_i(0.0, beta);
}

// FP32 bulk: below this tolerance the grid and its transforms stay FP64
constexpr double kFourierFp32MinTol = 1e-6;

// ---- plan cost model (MI355X) ----
// Device time of one evaluation, per stage, fitted to stage timings measured on one
// MI355X (uniform particles in the unit cube, N = 3e3..3e6, grids 16^3..256^3, both
// modes; median error 4-17% per stage).  Used to choose the grid when nothing but the
// tolerance is given: every power-of-two grid is resolved by the error split and the
// cheapest one is taken.
struct CostModel {
    double pair, p2p0;          // ms per 1e9 evaluated pairs (each unordered pair once), fixed
    double p2g, p2g_cell, p2g0; // ms per 1e9 N P^3 at full occupancy, per 1e6 cells, fixed
    double g2p, g2p_group, g2p_cell, g2p0;  // ms per 1e9 matrix steps, per 1e6 groups, per 1e6 cells, fixed
    double fft_cell, fft0;
    double sort, sort_cell, sort0;
};
constexpr CostModel kCost64 = {5.217, 0.053, 0.108, 0.169, 0.072, 46.477, 2.738, 0.0037, 0.0, 0.066, 0.017,
                               0.177, 0.010, 0.052};
constexpr CostModel kCost32 = {4.423, 0.045, 0.146, 0.171, 0.059, 37.097, 2.584, 0.0002, 0.0016, 0.041, 0.021,
                               0.174, 0.010, 0.056};
constexpr double kWaveSlots = 2048.0;  // concurrent P2P waves at which the chip is full

int p2g_blocks(const int M[3], int P)
{
    const int npy = std::max(1, M[1] / 8), npz = std::max(1, M[2] / 8);
    return (M[0] / p2g_segment_length(M, P)) * npy * npz;
}

// predicted ms per stage (sort, P2P, P2G, FFT+CNV+IFFT, G2P) for n particles
double model_ms(int mode, bool grid64, double n, const double box[3], const int M[3], int P, double rc, int B,
                double* stage)
{
    const CostModel& c = (mode == EWALD_FP64) ? kCost64 : kCost32;
    const CostModel& cf = grid64 ? kCost64 : kCost32;
    const double V = box[0] * box[1] * box[2];
    const double cells = (double)M[0] * M[1] * M[2];
    const double pairs = 0.5 * n * n / V * (4.0 / 3.0) * M_PI * rc * rc * rc;
    // P2P waves: three per 64-target chunk (about n/64 + tiles/2 chunks), six when the launch
    // has very few (the rule of launch_p2p in p2p.hip, on its grid of tiles + n/64 chunks: fewer
    // than 2048)
    const double tiles = cells / ((double)B * B * B);
    const double grid_waves = tiles + std::ceil(n / 64.0);
    const double split = grid_waves < 2048.0 ? 6.0 : 3.0;
    const double waves = (n / 64.0 + 0.5 * tiles) * split;
    const double np3 = n * P * P * P;
    // G2P: groups of 16 targets of one tile; each runs ceil(U^2 / 4) x NB matrix steps, U = P - 1 +
    // the x (and y) spread of its targets (a 16-target run of a tile's Morton columns: about
    // 4 B / sqrt(particles per tile) cells, at most B), NB = ceil(3 (B + P - 1) / 16); four waves
    // per 64-target chunk fill the chip from 4096 waves on
    const double per_tile = std::max(n / tiles, 1e-9);
    const double spread = std::min((double)B, std::max(1.0, 4.0 * B / std::sqrt(per_tile)));
    const double U = P - 1 + spread;
    const double NB = std::ceil(3.0 * (B + P - 1) / 16.0);
    const double groups = tiles * std::ceil(per_tile / 16.0);
    const double g2p_occ = std::min(1.0, 4.0 * (n / 64.0 + tiles) / 4096.0);
    double st[5];
    st[0] = c.sort * n * 1e-6 + c.sort_cell * cells * 1e-6 + c.sort0;
    st[1] = c.pair * pairs * 1e-9 / std::min(1.0, waves / kWaveSlots) + c.p2p0;
    st[2] = c.p2g * np3 * 1e-9 / std::min(1.0, p2g_blocks(M, P) / 1024.0) + c.p2g_cell * cells * 1e-6 + c.p2g0;
    st[3] = cf.fft_cell * cells * 1e-6 + cf.fft0;
    // G2P's matrix instruction follows the grid's precision (FP32 only for an FP32 grid)
    st[4] = (cf.g2p * groups * std::ceil(U * U / 4.0) * NB * 1e-9 + cf.g2p_group * groups * 1e-6) / g2p_occ +
            cf.g2p_cell * cells * 1e-6 + cf.g2p0;
    double t = 0;
    for (int k = 0; k < 5; ++k) {
        if (stage) stage[k] = st[k];
        t += st[k];
    }
    return t;
}

// P2P tile: the smallest power of two in [2, 16] whose tiles hold about 128 particles at
// n particles, so that the 64-target chunks of a tile are mostly full; not above any M
int choose_tile(const double box[3], const int M[3], double n)
{
    const double per_cell = std::max(n, 1.0) / ((double)M[0] * M[1] * M[2]);
    int B = 2;
    while (B < 16 && per_cell * B * B * B < 128.0) B *= 2;
    for (int d = 0; d < 3; ++d) B = std::min(B, M[d]);
    (void)box;
    return B;
}

// The window error models give an error relative to the far field u^F.  At a particle u^F
// holds its own screened self-interaction, about (4 xi / sqrt(pi)) f, which the self term
// cancels; where that exceeds the typical |u| / |f| (few particles, fine grids, large xi),
// the window error relative to |u| grows by the ratio.  For n random sources in volume V,
// |u| / |f| ~ sqrt(8 pi n Lmin / V) (the periodic sum of 1/r kernels over random forces);
// half of it is taken as a conservative scale.
double window_budget_factor(double xi, double n, const double box[3])
{
    const double V = box[0] * box[1] * box[2];
    const double Lmin = std::min(box[0], std::min(box[1], box[2]));
    const double u_over_f = std::max(1.0, 2.5 * std::sqrt(std::max(n, 1.0) * Lmin / V));
    return std::max(1.0, 4.0 * xi / std::sqrt(M_PI) / u_over_f);
}

// smallest window support meeting the window error budget (16 if none does)
int choose_P(bool kb, double h, double xi, double budget)
{
    for (int P = kb ? 6 : 4; P <= 16; P += 2) {
        const double e = kb ? err_window_kb(P, h, xi) : err_window(P, best_shape(P, h, xi), h, xi);
        if (e <= budget) return P;
    }
    return 16;
}

int64_t align256(int64_t v) { return (v + 255) & ~(int64_t)255; }

}  // namespace

namespace ewald {

int64_t layout_work(const Plan& pl, int64_t n, char* base, Work* w, int nsys)
{
    const Geometry& g = pl.g;
    const int64_t ncells = (int64_t)g.ncells * nsys, ntiles = (int64_t)g.ntiles * nsys;  // all systems
    int64_t off = 0;
    auto take = [&](int64_t bytes) -> char* {
        char* p = base ? base + off : nullptr;
        off += align256(bytes);
        return p;
    };
    const int64_t nn = std::max<int64_t>(n, 1);
    const size_t real = pl.grid64 ? 8 : 4;
    const size_t recsz = sizeof(Rec64);
    Work tmp;
    Work* o = w ? w : &tmp;
    o->key = (int*)take(4 * nn);
    o->perm = (int*)take(4 * nn);
    o->count = (int*)take(4 * ncells);
    o->start = (int*)take(4 * (ncells + 1));
    o->chunk_off = (int*)take(4 * (ntiles + 1));
    o->part = (int*)take(4 * (int64_t)scan_part_elems((int)std::max(ncells, ntiles)));
    o->cell_lists = (int*)take(4 * cell_list_elems(nn));
    o->rec = (void*)take((int64_t)recsz * nn);
    o->u_near = (double*)take(8 * 3 * nn);
    o->srec = pl.stresslet ? (double*)take(8 * 6 * nn) : nullptr;
    o->grid = (void*)take((int64_t)real * (pl.stresslet ? 9 : 3) * ncells);
    const int64_t nh = p2g_halo_elems(pl) * nsys;
    o->p2g_halo = nh > 0 ? (double*)take(8 * nh) : nullptr;
    o->bytes = off;
    return off;
}

}  // namespace ewald

namespace {

// Workspace of ewald_eval_noalloc: one array per device, in the library's code object, so
// that evaluating needs no allocation.  In host code `scratch` names a host-side stand-in,
// never the device memory: kernels and copies get the device address that
// hipGetSymbolAddress returns for the current device (g_scratch, looked up once per device
// by the first plan created on it).
constexpr int64_t kScratchBytes = EWALD_NOALLOC_MAX_WORKSPACE;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mutex;
void* g_scratch[kMaxDevices] = {};

// Device address of `scratch` on `device` (the current device), looked up on first use.
int scratch_setup(int device)
{
    if (device < 0 || device >= kMaxDevices) return fail(EWALD_EUNSUPPORTED, "device %d above %d", device, kMaxDevices);
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (g_scratch[device]) return EWALD_OK;
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
    if (!p || ((uintptr_t)p & 255) != 0) return fail(EWALD_EHIP, "scratch array address %p not 256-byte aligned", p);
    g_scratch[device] = p;
    return EWALD_OK;
}

void* scratch_ptr(int device)
{
    if (device < 0 || device >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    return g_scratch[device];
}

int validate_and_resolve(const ewald_params* in, Plan* pl)
{
    ewald_params p = *in;
    for (int d = 0; d < 3; ++d)
        if (!(p.box[d] > 0.0) || !std::isfinite(p.box[d]))
            return fail(EWALD_EINVAL, "box[%d] = %g must be positive and finite", d, p.box[d]);
    if (!(p.tol >= 1e-12 && p.tol <= 1e-2))
        return fail(EWALD_EINVAL, "tol = %g outside [1e-12, 1e-2]", p.tol);
    if (p.reserved != 0) return fail(EWALD_EINVAL, "reserved field must be 0");
    if (p.n_max < 0) return fail(EWALD_EINVAL, "n_max = %lld < 0", (long long)p.n_max);
    if (p.n_max > (int64_t)1 << 30) return fail(EWALD_EUNSUPPORTED, "n_max above 2^30");
    const int mode = p.precision & 0xff;
    if (mode != EWALD_FP64 && mode != EWALD_FP32_BULK)
        return fail(EWALD_EINVAL, "unknown precision mode %d", mode);
    if (p.precision &
        ~(0xff | EWALD_FLAG_P2P_FP64_ACC | EWALD_FLAG_STAGE_TIMERS | EWALD_FLAG_WINDOW_KB | EWALD_FLAG_DETERMINISTIC |
          EWALD_FLAG_STRESSLET | EWALD_FLAG_CHECK_INPUTS))
        return fail(EWALD_EINVAL, "unknown precision flags 0x%x", p.precision);
    if ((p.precision & EWALD_FLAG_STRESSLET) && (p.precision & EWALD_FLAG_DETERMINISTIC))
        return fail(EWALD_EUNSUPPORTED, "stresslet sources are evaluated by the symmetric P2P only "
                                        "(EWALD_FLAG_DETERMINISTIC not available with EWALD_FLAG_STRESSLET)");
    if (mode == EWALD_FP32_BULK && p.tol < 1e-7)
        return fail(EWALD_EUNSUPPORTED, "tol = %g below 1e-7 needs the FP64 mode", p.tol);
    const bool grid_given = p.grid[0] > 0 && p.grid[1] > 0 && p.grid[2] > 0;
    if (grid_given)
        for (int d = 0; d < 3; ++d)
            if (!is_pow2(p.grid[d]) || p.grid[d] < 8 || p.grid[d] > 512)
                return fail(EWALD_EINVAL, "grid[%d] = %d must be a power of two in [8, 512]", d, p.grid[d]);
    if (p.P > 0 && (p.P % 2 != 0 || p.P < 4 || p.P > 16))
        return fail(EWALD_EINVAL, "P = %d must be even, in 4..16", p.P);
    const double third = p.tol / 3.0;
    const double Lmin = std::min(p.box[0], std::min(p.box[1], p.box[2]));

    // grid and split parameter (E^F = tol/3), cutoff (E^N = tol/3)
    double h = 0.0;
    if (grid_given) {
        for (int d = 0; d < 3; ++d) h = std::max(h, p.box[d] / p.grid[d]);
        if (!(p.xi > 0)) p.xi = xi_from_grid(h, third);
    } else if (!(p.xi > 0) && !(p.r_c > 0)) {
        // only the tolerance: the cheapest power-of-two grid by the cost model
        const bool kb = (p.precision & EWALD_FLAG_WINDOW_KB) != 0;
        const bool g64 = mode == EWALD_FP64 || p.tol < kFourierFp32MinTol;
        const double n = (double)std::max<int64_t>(p.n_max, 1000);
        double best = 1e300;
        int bestM[3] = {0, 0, 0};
        for (int m0 = 8; m0 <= 512; m0 *= 2) {
            int M[3];
            bool ok = true;
            for (int d = 0; d < 3; ++d) {
                M[d] = std::max(8, next_pow2(p.box[d] / Lmin * m0 * (1.0 - 1e-12)));
                ok = ok && M[d] <= 512;
            }
            if (!ok) break;
            double hh = 0.0, hl = 1e300;
            for (int d = 0; d < 3; ++d) {
                hh = std::max(hh, p.box[d] / M[d]);
                hl = std::min(hl, p.box[d] / M[d]);
            }
            const double xi = xi_from_grid(hh, third);
            const double rc = rc_from_xi(xi, third);
            if (rc > Lmin || rc < hl || xi * rc > kScreenXmax) continue;
            const int P = p.P > 0 ? p.P : choose_P(kb, hh, xi, third / window_budget_factor(xi, n, p.box));
            const double t = model_ms(mode, g64, n, p.box, M, P, rc, choose_tile(p.box, M, n), nullptr);
            if (t < best) {
                best = t;
                for (int d = 0; d < 3; ++d) bestM[d] = M[d];
            }
        }
        if (!(best < 1e300)) return fail(EWALD_EUNSUPPORTED, "no grid up to 512 meets tol = %g", p.tol);
        for (int d = 0; d < 3; ++d) p.grid[d] = bestM[d];
        for (int d = 0; d < 3; ++d) h = std::max(h, p.box[d] / p.grid[d]);
        p.xi = xi_from_grid(h, third);
    } else {
        // xi or r_c given: the grid that resolves xi (E^F = tol/3)
        const bool xi_given = p.xi > 0;
        if (!xi_given) p.xi = xi_from_rc(p.r_c, third);
        h = h_from_xi(p.xi, third);
        for (int d = 0; d < 3; ++d) {
            int M = next_pow2(p.box[d] / h);
            M = std::max(8, std::min(512, M));
            p.grid[d] = M;
        }
        h = 0.0;
        for (int d = 0; d < 3; ++d) h = std::max(h, p.box[d] / p.grid[d]);
        // the power-of-two grid is at least as fine as needed: unless xi was given, raise
        // xi to what the grid resolves (E^F = tol/3), which shrinks r_c and the P2P work;
        // a grid capped at 512 lowers xi instead
        if (!xi_given) p.xi = xi_from_grid(h, third);
        else p.xi = std::min(p.xi, xi_from_grid(h, third));
    }
    if (!(p.r_c > 0)) p.r_c = rc_from_xi(p.xi, third);
    if (!(p.xi > 0) || !std::isfinite(p.xi)) return fail(EWALD_EINVAL, "xi = %g invalid", p.xi);
    if (p.r_c > Lmin) return fail(EWALD_EINVAL, "r_c = %g exceeds the smallest box side %g", p.r_c, Lmin);
    if (p.xi * p.r_c > kScreenXmax)
        return fail(EWALD_EUNSUPPORTED, "xi r_c = %g above %g, the range of the near-field screening polynomial",
                    p.xi * p.r_c, kScreenXmax);
    double hmin = 1e300;
    for (int d = 0; d < 3; ++d) hmin = std::min(hmin, p.box[d] / p.grid[d]);
    if (p.r_c < hmin) return fail(EWALD_EINVAL, "r_c = %g below the grid spacing %g", p.r_c, hmin);

    // window support and shape
    const bool kb = (p.precision & EWALD_FLAG_WINDOW_KB) != 0;
    if (kb && p.P > 0 && p.P < 6) return fail(EWALD_EINVAL, "P = %d: the Kaiser-Bessel window needs P >= 6", p.P);
    if (!(p.P > 0)) p.P = choose_P(kb, h, p.xi, third / window_budget_factor(p.xi, (double)p.n_max, p.box));
    if (!(p.window_shape > 0)) p.window_shape = kb ? kb_beta_over_p(p.P, h, p.xi) : best_shape(p.P, h, p.xi);

    pl->p = p;
    pl->mode = mode;
    pl->grid64 = mode == EWALD_FP64 || p.tol < kFourierFp32MinTol;
    pl->fp64acc = true;  // FP64 near-field accumulation in both modes (EWALD_FLAG_P2P_FP64_ACC is implied)
    pl->deterministic = (p.precision & EWALD_FLAG_DETERMINISTIC) != 0;
    pl->stresslet = (p.precision & EWALD_FLAG_STRESSLET) != 0;
    pl->timers = (p.precision & EWALD_FLAG_STAGE_TIMERS) != 0;
    pl->check_inputs = (p.precision & EWALD_FLAG_CHECK_INPUTS) != 0;
    pl->P = p.P;
    pl->window_kb = kb;
    pl->m = p.window_shape;
    pl->beta = kb ? p.window_shape * p.P : 2.0 * p.window_shape * p.window_shape / ((double)p.P * p.P);
    pl->xi = p.xi;
    pl->rc = p.r_c;

    Geometry& g = pl->g;
    for (int d = 0; d < 3; ++d) {
        g.L[d] = p.box[d];
        g.M[d] = p.grid[d];
        g.h[d] = p.box[d] / p.grid[d];
    }
    const int B = choose_tile(p.box, p.grid, (double)p.n_max);
    g.B = B;
    g.log2B = ilog2(B);
    g.ncells = g.M[0] * g.M[1] * g.M[2];
    g.nsys = 1;
    g.ntiles = 1;
    for (int d = 0; d < 3; ++d) {
        g.NT[d] = g.M[d] / B;
        g.S[d] = (int)std::ceil(p.r_c / (B * g.h[d]) - 1e-12);
        g.ntiles *= g.NT[d];
    }
    // P2G run table bound: (8 + P - 1) window rows x z-tile segments
    const int W = 8 + p.P - 1;
    const int nzs = (W - 1) / B + 2;
    if (W * nzs > p2g_max_runs())
        return fail(EWALD_EUNSUPPORTED, "window P = %d with tile %d exceeds the P2G run table", p.P, B);

    ewald_plan_info& info = pl->info;
    std::memset(&info, 0, sizeof info);
    info.params = p;
    for (int d = 0; d < 3; ++d) {
        info.h[d] = g.h[d];
        info.n_tiles[d] = g.NT[d];
        info.stencil[d] = g.S[d];
    }
    info.fourier_fp64 = pl->grid64 ? 1 : 0;
    info.self_coef = 4.0 * p.xi / std::sqrt(M_PI);
    info.grid_bytes = (int64_t)3 * g.ncells * (pl->grid64 ? 8 : 4);
    info.err_near = err_near(p.xi, p.r_c);
    info.err_far = err_far(p.xi, h);
    info.err_window = kb ? err_window_kb(p.P, h, p.xi) : err_window(p.P, p.window_shape, h, p.xi);
    info.tile = B;
    info.workspace_bytes = layout_work(*pl, p.n_max, nullptr, nullptr);
    info.predicted_ms = model_ms(pl->mode, pl->grid64, (double)std::max<int64_t>(p.n_max, 1), p.box, p.grid, p.P,
                                 p.r_c, pl->g.B, nullptr);
    return EWALD_OK;
}

int build_tables(Plan* pl)
{
    const Geometry& g = pl->g;
    const int M1 = g.M[0], M2 = g.M[1], M3 = g.M[2], H = M3 / 2;
    // CNV factors E_d[k] = (alpha_d/pi) exp(k_d^2 (1/(2 alpha_d) - 1/(4 xi^2))), Nyquist -> 0,
    // with the scale h1 h2 h3 / (M1 M2 M3) folded into E_0
    const int lens[3] = {M1, M2, H};
    const double scale = (g.h[0] * g.h[1] * g.h[2]) / ((double)M1 * M2 * M3);
    std::vector<double> cnv;
    size_t cnv_off[3];
    for (int d = 0; d < 3; ++d) {
        cnv_off[d] = cnv.size();
        const double alpha = 2.0 * pl->m * pl->m / std::pow(pl->P * g.h[d], 2);
        const double a = pl->P * g.h[d] / 2.0;
        for (int k = 0; k < lens[d]; ++k) {
            int ks = k;
            if (d < 2) ks = (k < g.M[d] / 2) ? k : k - g.M[d];
            const bool nyq = (d < 2) && (k == g.M[d] / 2);
            const double kd = 2.0 * M_PI * ks / g.L[d];
            const double kk = kd * kd;
            double v = 0.0;
            if (!nyq) {
                if (pl->window_kb) {
                    const double wh = kb_hat(kd, a, pl->beta);
                    v = std::exp(-kk / (4.0 * pl->xi * pl->xi)) / (wh * wh);
                } else {
                    v = (alpha / M_PI) * std::exp(kk * (1.0 / (2.0 * alpha) - 1.0 / (4.0 * pl->xi * pl->xi)));
                }
            }
            if (d == 0) v *= scale;
            cnv.push_back(v);
        }
    }
    // Kaiser-Bessel weights: per stencil offset j, the weight as a polynomial of degree kKbDeg in
    // s = 2t - 1 (t the particle's fraction in its cell): Chebyshev interpolation at 32 points
    // (the weight is analytic in t), truncated, converted to monomials.
    std::vector<double> kb64;
    if (pl->window_kb) {
        const int P = pl->P, NC = 32, D = kKbDeg;
        for (int j = 0; j < P; ++j) {
            std::vector<double> val(NC), cheb(NC, 0.0);
            for (int q = 0; q < NC; ++q) {
                const double sq = std::cos(M_PI * (q + 0.5) / NC);
                const double t = 0.5 * (sq + 1.0);
                val[q] = kb_w(j - (P / 2 - 1) - t, P, pl->beta);
            }
            for (int c = 0; c < NC; ++c) {
                double acc = 0.0;
                for (int q = 0; q < NC; ++q) acc += val[q] * std::cos(M_PI * c * (q + 0.5) / NC);
                cheb[c] = (c ? 2.0 : 1.0) * acc / NC;
            }
            // Chebyshev -> monomial: T_0 = 1, T_1 = s, T_{c+1} = 2 s T_c - T_{c-1}
            std::vector<double> mono(D + 1, 0.0), tm1(D + 1, 0.0), t0(D + 1, 0.0), t1(D + 1, 0.0);
            t0[0] = 1.0;
            for (int c = 0; c <= D; ++c) {
                const std::vector<double>& tc = (c == 0) ? t0 : t1;
                for (int e = 0; e <= D; ++e) mono[e] += cheb[c] * tc[e];
                if (c == 0) {
                    t1.assign(D + 1, 0.0);
                    t1[1] = 1.0;
                    tm1 = t0;
                } else {
                    std::vector<double> nx(D + 1, 0.0);
                    for (int e = 0; e < D; ++e) nx[e + 1] += 2.0 * t1[e];
                    for (int e = 0; e <= D; ++e) nx[e] -= tm1[e];
                    tm1 = t1;
                    t1 = nx;
                }
            }
            kb64.insert(kb64.end(), mono.begin(), mono.end());
        }
    }
    // twiddles e^{-2 pi i j / n} for n = M1, M2, M3/2, M3
    const int tl[4] = {M1, M2, H, M3};
    std::vector<double> tw64;
    std::vector<float> tw32;
    for (int a = 0; a < 4; ++a) {
        pl->tw_off[a] = (int)(tw64.size() / 2);
        for (int j = 0; j < tl[a]; ++j) {
            const double ang = -2.0 * M_PI * (double)j / tl[a];
            const double c = std::cos(ang), s = std::sin(ang);
            tw64.push_back(c);
            tw64.push_back(s);
            tw32.push_back((float)c);
            tw32.push_back((float)s);
        }
    }
    const size_t b_cnv = align256(cnv.size() * 8);
    const size_t b_tw64 = align256(tw64.size() * 8);
    const size_t b_tw32 = align256(tw32.size() * 4);
    std::vector<float> kb32(kb64.begin(), kb64.end());
    const size_t b_kb64 = align256(kb64.size() * 8 + 8);
    const size_t b_kb32 = align256(kb32.size() * 4 + 4);
    char* d = nullptr;
    hipError_t e = hipMalloc((void**)&d, b_cnv + b_tw64 + b_tw32 + b_kb64 + b_kb32);
    if (e != hipSuccess) return fail(EWALD_ENOMEM, "plan tables: %s", hipGetErrorString(e));
    pl->d_tables = d;
    e = hipMemcpy(d, cnv.data(), cnv.size() * 8, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(d + b_cnv, tw64.data(), tw64.size() * 8, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(d + b_cnv + b_tw64, tw32.data(), tw32.size() * 4, hipMemcpyHostToDevice);
    char* dkb = d + b_cnv + b_tw64 + b_tw32;
    if (e == hipSuccess && !kb64.empty()) e = hipMemcpy(dkb, kb64.data(), kb64.size() * 8, hipMemcpyHostToDevice);
    if (e == hipSuccess && !kb32.empty()) e = hipMemcpy(dkb + b_kb64, kb32.data(), kb32.size() * 4, hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(e, "plan table upload");
    for (int k = 0; k < 3; ++k) pl->d_cnv[k] = (double*)d + cnv_off[k];
    pl->d_tw64 = d + b_cnv;
    pl->d_tw32 = d + b_cnv + b_tw64;
    pl->d_kb64 = pl->window_kb ? (double*)dkb : nullptr;
    pl->d_kb32 = pl->window_kb ? (float*)(dkb + b_kb64) : nullptr;
    return EWALD_OK;
}

int check_eval_args(ewald_plan_t plan, int64_t n, const void* x, const void* f, const void* o1,
                    const void* o2, void* ws, int64_t wsb, Work* w, int nsys = 1)
{
    if (!plan) return fail(EWALD_EINVAL, "null plan");
    const Plan* pl = reinterpret_cast<const Plan*>(plan);
    if (n < 0) return fail(EWALD_EINVAL, "n = %lld < 0", (long long)n);
    if (nsys == 1 && n > pl->p.n_max)
        return fail(EWALD_EINVAL, "n = %lld exceeds the plan's n_max = %lld", (long long)n, (long long)pl->p.n_max);
    if (n == 0) return EWALD_OK;
    if (!x || !f || !o1 || !o2) return fail(EWALD_EINVAL, "null array pointer");
    if (!ws) return fail(EWALD_EINVAL, "null workspace");
    if (((uintptr_t)ws & 255) != 0) return fail(EWALD_EINVAL, "workspace not 256-byte aligned");
    const int64_t need = layout_work(*pl, n, (char*)ws, w, nsys);
    if (wsb < need) return fail(EWALD_ENOMEM, "workspace of %lld bytes below the %lld needed", (long long)wsb, (long long)need);
    return EWALD_OK;
}

// Validate a batch description (host offsets, count + 1 entries) and fill *b.
int make_batch(const Plan* pl, int32_t count, const int64_t* offsets, Batch* b)
{
    if (count < 1 || count > kMaxBatch) return fail(EWALD_EINVAL, "count = %d outside [1, %d]", count, kMaxBatch);
    if (!offsets) return fail(EWALD_EINVAL, "null offsets");
    if (offsets[0] != 0) return fail(EWALD_EINVAL, "offsets[0] = %lld must be 0", (long long)offsets[0]);
    if (pl->stresslet) return fail(EWALD_EUNSUPPORTED, "batches of stresslet plans are not supported");
    if ((int64_t)pl->g.ncells * count + 1 > INT32_MAX)
        return fail(EWALD_EUNSUPPORTED, "%d systems of %d grid cells exceed the cell list's 32-bit range", count,
                    pl->g.ncells);
    b->count = count;
    for (int r = 0; r < count; ++r) {
        const int64_t nr = offsets[r + 1] - offsets[r];
        if (nr < 0) return fail(EWALD_EINVAL, "offsets decrease at %d", r);
        if (nr > pl->p.n_max)
            return fail(EWALD_EINVAL, "system %d has %lld particles, above the plan's n_max = %lld", r, (long long)nr,
                        (long long)pl->p.n_max);
        b->off[r] = (int)offsets[r];
    }
    if (offsets[count] > ((int64_t)1 << 30)) return fail(EWALD_EUNSUPPORTED, "batch of more than 2^30 particles");
    b->off[count] = (int)offsets[count];
    for (int r = count + 1; r <= kMaxBatch; ++r) b->off[r] = b->off[count];
    return EWALD_OK;
}

enum class Out { Full, Parts, Spread, FarGrid, CountPairs };

// near != nullptr: P2P runs on the stream `near`, forked from `stream` after the sort through the
// event `fork` and joined back through `join` before G2P (P2P is independent of P2G and the FFTs)
// batch != nullptr: the n64 particles are batch->count independent systems of the plan
int run(ewald_plan_t plan, int64_t n64, const double* x, const double* f, void* o1, void* o2, void* ws,
        int64_t wsb, void* stream, Out what, bool st = false, const double* q = nullptr, const double* nrm = nullptr,
        int64_t out_bytes = 0, hipStream_t near = nullptr, hipEvent_t fork = nullptr, hipEvent_t join = nullptr,
        const Batch* batch = nullptr)
{
    Work w;
    Batch one;
    if (!batch) {
        one.count = 1;
        for (int r = 0; r <= kMaxBatch; ++r) one.off[r] = (r == 0) ? 0 : (int)std::min<int64_t>(n64, INT32_MAX);
        batch = &one;
    }
    const int nsys = batch->count;
    if ((what == Out::Spread || what == Out::FarGrid) && plan) {
        const int64_t need = reinterpret_cast<const Plan*>(plan)->info.grid_bytes;
        if (n64 > 0 && out_bytes < need)
            return fail(EWALD_ENOMEM, "grid buffer of %lld bytes below the %lld the plan's grid needs",
                        (long long)out_bytes, (long long)need);
    }
    if (st) {
        if (!plan) return fail(EWALD_EINVAL, "null plan");
        if (!reinterpret_cast<const Plan*>(plan)->stresslet)
            return fail(EWALD_EINVAL, "stresslet sources need a plan created with EWALD_FLAG_STRESSLET");
        if (n64 > 0 && (!q || !nrm)) return fail(EWALD_EINVAL, "null stresslet vector pointer");
    }
    int rc = check_eval_args(plan, n64, x, f, o1, what == Out::Parts ? o2 : o1, ws, wsb, &w, nsys);
    if (rc != EWALD_OK || n64 == 0) return rc;
    if (g_fail_next > 0) {
        --g_fail_next;
        return fail(EWALD_EHIP, "injected failure (ewald_debug_fail_next)");
    }
    Plan* pl = reinterpret_cast<Plan*>(plan);
    hipStream_t s = (hipStream_t)stream;
    const int n = (int)n64;
    if (pl->check_inputs) {
        // debug mode: count the non-finite inputs into the workspace's scan partials, wait, refuse
        hipError_t e = launch_count_nonfinite(x, 3 * n64, w.part, s);
        if (e == hipSuccess) e = launch_count_nonfinite(f, 3 * n64, w.part + 1, s);
        if (st && e == hipSuccess) e = launch_count_nonfinite(q, 3 * n64, w.part + 1, s, false);
        if (st && e == hipSuccess) e = launch_count_nonfinite(nrm, 3 * n64, w.part + 1, s, false);
        int h[2] = {0, 0};
        if (e == hipSuccess) e = hipMemcpyAsync(h, w.part, sizeof h, hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) return hip_fail(e, "input check");
        if (h[0] + h[1] > 0)
            return fail(EWALD_EINVAL, "inputs hold %d non-finite values (%d in x)", h[0] + h[1], h[0]);
    }
    const bool t = pl->timers && what != Out::Spread && what != Out::FarGrid;
    hipError_t e;
    auto mark = [&](int k) {
        if (t) (void)hipEventRecord(pl->ev[k], s);
    };
    mark(0);
    if ((e = launch_sort(*pl, w, n, x, f, *batch, s)) != hipSuccess) return hip_fail(e, "sort");
    if (what == Out::CountPairs) {
        e = launch_count_pairs(*pl, w, n, (unsigned long long*)o1, s, nsys);
        return e == hipSuccess ? EWALD_OK : hip_fail(e, "pair count");
    }
    if (st && (e = launch_gather_st(*pl, w, n, q, nrm, s)) != hipSuccess) return hip_fail(e, "stresslet gather");
    mark(1);
    if (near) {
        // the near field on its own stream, beside P2G and the FFTs
        if ((e = hipEventRecord(fork, s)) != hipSuccess) return hip_fail(e, "fork event");
        if ((e = hipStreamWaitEvent(near, fork, 0)) != hipSuccess) return hip_fail(e, "fork wait");
        if ((e = launch_p2p(*pl, w, n, near, st, nsys)) != hipSuccess) return hip_fail(e, "P2P");
        if (t) (void)hipEventRecord(pl->ev[2], near);
        if ((e = hipEventRecord(join, near)) != hipSuccess) return hip_fail(e, "join event");
    } else {
        if (what == Out::Full || what == Out::Parts) {
            if ((e = launch_p2p(*pl, w, n, s, st, nsys)) != hipSuccess) return hip_fail(e, "P2P");
        }
        mark(2);
    }
    if ((e = launch_p2g(*pl, w, n, s, st, nsys)) != hipSuccess) return hip_fail(e, "P2G");
    mark(3);
    const size_t gbytes = (size_t)pl->info.grid_bytes;
    if (what == Out::Spread) {
        e = hipMemcpyAsync(o1, w.grid, gbytes, hipMemcpyDeviceToDevice, s);
        return e == hipSuccess ? EWALD_OK : hip_fail(e, "grid copy");
    }
    if ((e = launch_fgc(*pl, w, s, true, true, st, nsys)) != hipSuccess) return hip_fail(e, "FFT/CNV/IFFT");
    mark(4);
    if (what == Out::FarGrid) {
        e = hipMemcpyAsync(o1, w.grid, gbytes, hipMemcpyDeviceToDevice, s);
        return e == hipSuccess ? EWALD_OK : hip_fail(e, "grid copy");
    }
    if (near && (e = hipStreamWaitEvent(s, join, 0)) != hipSuccess) return hip_fail(e, "join wait");
    if (what == Out::Full)
        e = launch_g2p(*pl, w, n, f, (double*)o1, nullptr, nullptr, *batch, s);
    else
        e = launch_g2p(*pl, w, n, f, nullptr, (double*)o1, (double*)o2, *batch, s);
    if (e != hipSuccess) return hip_fail(e, "G2P");
    mark(5);
    if (t) {
        pl->ev_valid = true;
        pl->ev_overlapped = near != nullptr;
    }
    return EWALD_OK;
}

}  // namespace

extern "C" {

int ewald_plan_create(const ewald_params* params, ewald_plan_t* plan_out)
{
    if (!params || !plan_out) return fail(EWALD_EINVAL, "null argument");
    *plan_out = nullptr;
    Plan* pl = new (std::nothrow) Plan();
    if (!pl) return fail(EWALD_ENOMEM, "plan allocation");
    std::memset(pl, 0, sizeof *pl);
    int rc = validate_and_resolve(params, pl);
    if (rc == EWALD_OK) {
        hipError_t e = hipGetDevice(&pl->device);
        if (e != hipSuccess) rc = hip_fail(e, "hipGetDevice");
    }
    if (rc == EWALD_OK) rc = scratch_setup(pl->device);
    if (rc == EWALD_OK) rc = build_tables(pl);
    if (rc == EWALD_OK && pl->timers) {
        for (int k = 0; k <= kNumStages && rc == EWALD_OK; ++k) {
            hipError_t e = hipEventCreate(&pl->ev[k]);
            if (e != hipSuccess) rc = hip_fail(e, "hipEventCreate");
        }
    }
    if (rc != EWALD_OK) {
        ewald_plan_destroy(reinterpret_cast<ewald_plan_t>(pl));
        return rc;
    }
    *plan_out = reinterpret_cast<ewald_plan_t>(pl);
    return EWALD_OK;
}

int ewald_resolve(const ewald_params* params, ewald_plan_info* info)
{
    if (!params || !info) return fail(EWALD_EINVAL, "null argument");
    Plan* pl = new (std::nothrow) Plan();
    if (!pl) return fail(EWALD_ENOMEM, "plan allocation");
    std::memset(pl, 0, sizeof *pl);
    const int rc = validate_and_resolve(params, pl);
    if (rc == EWALD_OK) *info = pl->info;
    delete pl;
    return rc;
}

int ewald_plan_get_info(ewald_plan_t plan, ewald_plan_info* info)
{
    if (!plan || !info) return fail(EWALD_EINVAL, "null argument");
    *info = reinterpret_cast<Plan*>(plan)->info;
    return EWALD_OK;
}

int ewald_plan_destroy(ewald_plan_t plan)
{
    if (!plan) return EWALD_OK;
    Plan* pl = reinterpret_cast<Plan*>(plan);
    if (pl->d_tables) (void)hipFree(pl->d_tables);
    for (int k = 0; k <= kNumStages; ++k)
        if (pl->ev[k]) (void)hipEventDestroy(pl->ev[k]);
    delete pl;
    return EWALD_OK;
}

int64_t ewald_workspace_bytes(ewald_plan_t plan, int64_t n)
{
    if (!plan) return fail(EWALD_EINVAL, "null plan");
    if (n < 0) return fail(EWALD_EINVAL, "n = %lld < 0", (long long)n);
    return layout_work(*reinterpret_cast<Plan*>(plan), n, nullptr, nullptr);
}

int ewald_eval(ewald_plan_t plan, int64_t n, const double* x, const double* f, double* u, void* workspace,
               int64_t workspace_bytes, void* stream)
{
    return run(plan, n, x, f, u, u, workspace, workspace_bytes, stream, Out::Full);
}

int ewald_eval_noalloc(ewald_plan_t plan, int64_t n, const double* x, const double* f, double* u, void* stream)
{
    if (!plan) return fail(EWALD_EINVAL, "null plan");
    const Plan* pl = reinterpret_cast<const Plan*>(plan);
    if (n < 0 || n > pl->p.n_max) return run(plan, n, x, f, u, u, nullptr, 0, stream, Out::Full);
    const int64_t need = layout_work(*pl, n, nullptr, nullptr);
    if (need > kScratchBytes)
        return fail(EWALD_ENOMEM, "n = %lld needs a workspace of %lld bytes, above the %lld of the built-in scratch "
                    "array (use ewald_eval with a caller workspace)", (long long)n, (long long)need,
                    (long long)kScratchBytes);
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (dev != pl->device) return fail(EWALD_EINVAL, "current device %d is not the plan's device %d", dev, pl->device);
    void* ws = scratch_ptr(dev);
    if (!ws) return fail(EWALD_EHIP, "scratch array of device %d not set up", dev);
    return run(plan, n, x, f, u, u, ws, kScratchBytes, stream, Out::Full);
}

int ewald_eval_overlap(ewald_plan_t plan, int64_t n, const double* x, const double* f, double* u, void* workspace,
                       int64_t workspace_bytes, void* stream, void* near_stream, void* fork_event, void* join_event)
{
    if (n > 0 && (!near_stream || !fork_event || !join_event))
        return fail(EWALD_EINVAL, "null near-field stream or event");
    if (n > 0 && near_stream == stream) return fail(EWALD_EINVAL, "the near-field stream must differ from the stream");
    return run(plan, n, x, f, u, u, workspace, workspace_bytes, stream, Out::Full, false, nullptr, nullptr, 0,
               (hipStream_t)near_stream, (hipEvent_t)fork_event, (hipEvent_t)join_event);
}

int64_t ewald_workspace_bytes_batch(ewald_plan_t plan, int32_t count, const int64_t* offsets)
{
    if (!plan) return fail(EWALD_EINVAL, "null plan");
    Batch b;
    const int rc = make_batch(reinterpret_cast<Plan*>(plan), count, offsets, &b);
    if (rc != EWALD_OK) return rc;
    return layout_work(*reinterpret_cast<Plan*>(plan), offsets[count], nullptr, nullptr, count);
}

int ewald_eval_batch(ewald_plan_t plan, int32_t count, const int64_t* offsets, const double* x, const double* f,
                     double* u, void* workspace, int64_t workspace_bytes, void* stream)
{
    if (!plan) return fail(EWALD_EINVAL, "null plan");
    Batch b;
    const int rc = make_batch(reinterpret_cast<Plan*>(plan), count, offsets, &b);
    if (rc != EWALD_OK) return rc;
    return run(plan, offsets[count], x, f, u, u, workspace, workspace_bytes, stream, Out::Full, false, nullptr,
               nullptr, 0, nullptr, nullptr, nullptr, &b);
}

int ewald_eval_parts(ewald_plan_t plan, int64_t n, const double* x, const double* f, double* u_near,
                     double* u_far, void* workspace, int64_t workspace_bytes, void* stream)
{
    return run(plan, n, x, f, u_near, u_far, workspace, workspace_bytes, stream, Out::Parts);
}

int ewald_eval_combined(ewald_plan_t plan, int64_t n, const double* x, const double* f, const double* q,
                        const double* nrm, double* u, void* workspace, int64_t workspace_bytes, void* stream)
{
    return run(plan, n, x, f, u, u, workspace, workspace_bytes, stream, Out::Full, true, q, nrm);
}

int ewald_eval_combined_parts(ewald_plan_t plan, int64_t n, const double* x, const double* f, const double* q,
                              const double* nrm, double* u_near, double* u_far, void* workspace,
                              int64_t workspace_bytes, void* stream)
{
    return run(plan, n, x, f, u_near, u_far, workspace, workspace_bytes, stream, Out::Parts, true, q, nrm);
}

int ewald_spread(ewald_plan_t plan, int64_t n, const double* x, const double* f, void* grid, int64_t grid_bytes,
                 void* workspace, int64_t workspace_bytes, void* stream)
{
    return run(plan, n, x, f, grid, grid, workspace, workspace_bytes, stream, Out::Spread, false, nullptr, nullptr,
               grid_bytes);
}

int ewald_far_grid(ewald_plan_t plan, int64_t n, const double* x, const double* f, void* grid,
                   int64_t grid_bytes, void* workspace, int64_t workspace_bytes, void* stream)
{
    return run(plan, n, x, f, grid, grid, workspace, workspace_bytes, stream, Out::FarGrid, false, nullptr, nullptr,
               grid_bytes);
}

int ewald_count_pairs(ewald_plan_t plan, int64_t n, const double* x, const double* f, uint64_t* count,
                      void* workspace, int64_t workspace_bytes, void* stream)
{
    if (n == 0 && count && plan) {
        Work w{};
        const hipError_t e = launch_count_pairs(*reinterpret_cast<Plan*>(plan), w, 0, (unsigned long long*)count,
                                                (hipStream_t)stream);
        return e == hipSuccess ? EWALD_OK : hip_fail(e, "count reset");
    }
    return run(plan, n, x, f, count, count, workspace, workspace_bytes, stream, Out::CountPairs);
}

int ewald_stage_ms(ewald_plan_t plan, float* ms, int32_t count)
{
    if (!plan || !ms || count < 0) return fail(EWALD_EINVAL, "bad argument");
    Plan* pl = reinterpret_cast<Plan*>(plan);
    if (!pl->timers) return fail(EWALD_EINVAL, "plan was created without EWALD_FLAG_STAGE_TIMERS");
    if (!pl->ev_valid) return fail(EWALD_EINVAL, "no timed evaluation recorded yet");
    float v[kNumStages];
    if (pl->ev_overlapped) {
        // P2P ran beside P2G and the FFTs: each stage from its own start (the fork for P2P and
        // P2G), G2P from the later of the far field and the join
        float tk[kNumStages];
        for (int k = 1; k < kNumStages; ++k) {
            hipError_t e = hipEventElapsedTime(&tk[k], pl->ev[0], pl->ev[k]);
            if (e != hipSuccess) return hip_fail(e, "hipEventElapsedTime");
        }
        v[0] = tk[1];
        v[1] = tk[2] - tk[1];
        v[2] = tk[3] - tk[1];
        v[3] = tk[4] - tk[3];
        v[4] = tk[5] - std::max(tk[4], tk[2]);
        v[5] = tk[5];
    } else {
        for (int k = 0; k < kNumStages - 1; ++k) {
            hipError_t e = hipEventElapsedTime(&v[k], pl->ev[k], pl->ev[k + 1]);
            if (e != hipSuccess) return hip_fail(e, "hipEventElapsedTime");
        }
        hipError_t e = hipEventElapsedTime(&v[kNumStages - 1], pl->ev[0], pl->ev[kNumStages - 1]);
        if (e != hipSuccess) return hip_fail(e, "hipEventElapsedTime");
    }
    const int k = std::min<int>(count, kNumStages);
    for (int i = 0; i < k; ++i) ms[i] = v[i];
    return k;
}

int ewald_debug_fail_next(int32_t count)
{
    if (count < 0) return fail(EWALD_EINVAL, "count = %d < 0", count);
    g_fail_next = count;
    return EWALD_OK;
}

const char* ewald_last_error(void) { return g_err.c_str(); }

const char* ewald_version(void) { return "paper_2606_19059_amd 0.1 (gfx950)"; }

}  // extern "C"
