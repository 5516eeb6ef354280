/*
 * ewald_oracle.c -- TEST INFRASTRUCTURE, not part of the product.
 *
 * A slow, plain FP64 classical Ewald evaluation of the triply periodic
 * Stokeslet sum
 *
 *     u(x_i) = sum_j sum_p' G(x_i - x_j + p) f_j,   G(r) = I/|r| + r r^T/|r|^3
 *
 * (the periodised N-body sum of Sec. 2, eq. (potentials), with the Stokeslet
 * defined just below it).  The conditionally convergent image sum is given its
 * Hasimoto meaning: the k = 0 Fourier mode is dropped.
 *
 * Method (classical Ewald, no grid, no window, no FFT, no cell list):
 *   real space    u^N_i = sum_{j,p : 0 < |r| < r_cut} G^N(r) f_j,  r = x_i - x_j + p,
 *                 with the screened Stokeslet G^N of Sec. 2.1, eq. (g-near);
 *   Fourier space u^F_i = (1/V) sum_{k != 0, |k| <= k_max} Ghat^F(k) S(k) e^{i k.x_i},
 *                 S(k) = sum_j f_j e^{-i k.x_j}, Ghat^F of Sec. 2.2, eq. (GFk),
 *                 evaluated as a direct sum over the 3-periodic reciprocal lattice
 *                 k = 2 pi (n1/L1, n2/L2, n3/L3);
 *   self term     -G^F(0) f_i = -(4 xi / sqrt(pi)) f_i   (added by the Python side).
 *
 * Only the tests, the smoke check and the benchmark's CPU-baseline leg may
 * load this library.  It shares no code, header or table with the HIP
 * library; the two meet only through the seeded input arrays.
 *
 * Layout: positions, forces and outputs are structure-of-arrays (3, n) in
 * FP64: component d of particle i is at [d*n + i].  Targets are given as
 * indices into the particle set (NULL = all particles), so that a target and
 * the particle it coincides with give exactly r = 0, which is skipped (the
 * paper skips coincident points, Sec. 2).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define EWO_PI 3.14159265358979323846

/* Wrap one coordinate into [0, L). */
static double wrap1(double x, double L)
{
    double y = x - L * floor(x / L);
    if (y >= L) y -= L;
    if (y < 0.0) y = 0.0;
    return y;
}

void ewo_wrap(int64_t n, const double* x, const double L[3], double* xw)
{
    for (int d = 0; d < 3; ++d)
        for (int64_t i = 0; i < n; ++i) xw[d * n + i] = wrap1(x[d * n + i], L[d]);
}

int ewo_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Threads of the following calls (timing the oracle on fewer cores; arithmetic unchanged). */
void ewo_set_num_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/*
 * Real-space (near-field) sum at split parameter xi and cutoff r_cut.
 * Every image p in Z^3 L with 0 < |x_i - x_j + p| < r_cut contributes
 * G^N(r) f_j, eq. (g-near):
 *   G^N(r) = G(r) (erfc(xi r) + 2 xi r e^{-xi^2 r^2} / sqrt(pi)) - I 4 xi e^{-xi^2 r^2} / sqrt(pi).
 */
void ewo_real_space(int64_t n, const double* x, const double* f, int64_t nt, const int64_t* tidx,
                    const double L[3], double xi, double r_cut, double* u)
{
    double* xw = (double*)malloc(sizeof(double) * 3 * (size_t)(n > 0 ? n : 1));
    ewo_wrap(n, x, L, xw);
    const double rc2 = r_cut * r_cut;
    const double two_over_sqrtpi = 2.0 / sqrt(EWO_PI);
    const int64_t ntt = tidx ? nt : n;

#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t a = 0; a < ntt; ++a) {
        const int64_t i = tidx ? tidx[a] : a;
        const double xi0 = xw[i], xi1 = xw[n + i], xi2 = xw[2 * n + i];
        double s0 = 0.0, s1 = 0.0, s2 = 0.0;
        for (int64_t j = 0; j < n; ++j) {
            const double d0 = xi0 - xw[j], d1 = xi1 - xw[n + j], d2 = xi2 - xw[2 * n + j];
            /* image ranges: |d + m L| < r_cut */
            const int lo0 = (int)ceil((-r_cut - d0) / L[0]), hi0 = (int)floor((r_cut - d0) / L[0]);
            const int lo1 = (int)ceil((-r_cut - d1) / L[1]), hi1 = (int)floor((r_cut - d1) / L[1]);
            const int lo2 = (int)ceil((-r_cut - d2) / L[2]), hi2 = (int)floor((r_cut - d2) / L[2]);
            const double f0 = f[j], f1 = f[n + j], f2 = f[2 * n + j];
            for (int m0 = lo0; m0 <= hi0; ++m0) {
                const double r0 = d0 + m0 * L[0];
                for (int m1 = lo1; m1 <= hi1; ++m1) {
                    const double r1 = d1 + m1 * L[1];
                    for (int m2 = lo2; m2 <= hi2; ++m2) {
                        const double r2v = d2 + m2 * L[2];
                        const double rr = r0 * r0 + r1 * r1 + r2v * r2v;
                        if (!(rr < rc2) || rr == 0.0) continue;
                        const double r = sqrt(rr);
                        const double xr = xi * r;
                        const double e = exp(-xr * xr);
                        const double c = erfc(xr) + two_over_sqrtpi * xr * e; /* screening of G */
                        const double dterm = 2.0 * two_over_sqrtpi * xi * e;  /* 4 xi e / sqrt(pi) */
                        const double rf = r0 * f0 + r1 * f1 + r2v * f2;
                        const double a1 = c / r - dterm; /* coefficient of f */
                        const double a2 = c * rf / (rr * r); /* coefficient of r */
                        s0 += a1 * f0 + a2 * r0;
                        s1 += a1 * f1 + a2 * r1;
                        s2 += a1 * f2 + a2 * r2v;
                    }
                }
            }
        }
        u[a] = s0;
        u[ntt + a] = s1;
        u[2 * ntt + a] = s2;
    }
    free(xw);
}

/*
 * Fourier-space (far-field) sum, eq. (GFk) on the 3-periodic lattice:
 *   u_i = (1/V) sum_{k != 0, |k| <= k_max} A(k) Re{ e^{i k.x_i} (|k|^2 S(k) - k (k.S(k))) },
 *   A(k) = 8 pi / |k|^4 (1 + |k|^2 / (4 xi^2)) e^{-|k|^2 / (4 xi^2)}.
 * Implemented over the half space {n1 > 0} U {n1 = 0, n2 > 0} U {n1 = n2 = 0, n3 > 0}
 * with a factor 2 (the terms for k and -k are complex conjugates).
 */
void ewo_recip(int64_t n, const double* x, const double* f, int64_t nt, const int64_t* tidx,
               const double L[3], double xi, double k_max, double* u)
{
    const int64_t ntt = tidx ? nt : n;
    const double V = L[0] * L[1] * L[2];
    const int nk0 = (int)floor(k_max * L[0] / (2.0 * EWO_PI));
    const int nk1 = (int)floor(k_max * L[1] / (2.0 * EWO_PI));
    const int nk2 = (int)floor(k_max * L[2] / (2.0 * EWO_PI));
    const double km2 = k_max * k_max;
    const double inv4xi2 = 1.0 / (4.0 * xi * xi);

    /* enumerate the half-space wave vectors */
    int64_t cap = (int64_t)(nk0 + 1) * (2 * nk1 + 1) * (2 * nk2 + 1);
    int* kn = (int*)malloc(sizeof(int) * 3 * (size_t)cap);
    double* kv = (double*)malloc(sizeof(double) * 4 * (size_t)cap); /* k0,k1,k2,A */
    int64_t K = 0;
    for (int a = 0; a <= nk0; ++a)
        for (int b = -nk1; b <= nk1; ++b)
            for (int c = -nk2; c <= nk2; ++c) {
                if (a == 0 && (b < 0 || (b == 0 && c <= 0))) continue;
                const double k0 = 2.0 * EWO_PI * a / L[0];
                const double k1 = 2.0 * EWO_PI * b / L[1];
                const double k2 = 2.0 * EWO_PI * c / L[2];
                const double kk = k0 * k0 + k1 * k1 + k2 * k2;
                if (kk > km2) continue;
                kn[3 * K] = a;
                kn[3 * K + 1] = b;
                kn[3 * K + 2] = c;
                kv[4 * K] = k0;
                kv[4 * K + 1] = k1;
                kv[4 * K + 2] = k2;
                kv[4 * K + 3] = 8.0 * EWO_PI / (kk * kk) * (1.0 + kk * inv4xi2) * exp(-kk * inv4xi2);
                ++K;
            }

    /* structure factor S(k) = sum_j f_j e^{-i k.x_j}: 3 complex numbers per k */
    int nth = ewo_num_threads();
    double* Sloc = (double*)calloc((size_t)nth * (size_t)K * 6, sizeof(double));
    const int w0 = nk0 + 1, w1 = 2 * nk1 + 1, w2 = 2 * nk2 + 1;
#pragma omp parallel
    {
        int tid = 0;
#ifdef _OPENMP
        tid = omp_get_thread_num();
#endif
        double* S = Sloc + (size_t)tid * (size_t)K * 6;
        double* e0 = (double*)malloc(sizeof(double) * 2 * (size_t)w0);
        double* e1 = (double*)malloc(sizeof(double) * 2 * (size_t)w1);
        double* e2 = (double*)malloc(sizeof(double) * 2 * (size_t)w2);
#pragma omp for schedule(static)
        for (int64_t j = 0; j < n; ++j) {
            const double y0 = x[j], y1 = x[n + j], y2 = x[2 * n + j];
            /* e^{-i k_d y_d} per dimension, by direct cos/sin of each multiple */
            for (int a = 0; a < w0; ++a) {
                const double ph = 2.0 * EWO_PI * a * y0 / L[0];
                e0[2 * a] = cos(ph);
                e0[2 * a + 1] = -sin(ph);
            }
            for (int b = 0; b < w1; ++b) {
                const double ph = 2.0 * EWO_PI * (b - nk1) * y1 / L[1];
                e1[2 * b] = cos(ph);
                e1[2 * b + 1] = -sin(ph);
            }
            for (int c = 0; c < w2; ++c) {
                const double ph = 2.0 * EWO_PI * (c - nk2) * y2 / L[2];
                e2[2 * c] = cos(ph);
                e2[2 * c + 1] = -sin(ph);
            }
            const double fj0 = f[j], fj1 = f[n + j], fj2 = f[2 * n + j];
            for (int64_t q = 0; q < K; ++q) {
                const int a = kn[3 * q], b = kn[3 * q + 1] + nk1, c = kn[3 * q + 2] + nk2;
                const double pr = e0[2 * a] * e1[2 * b] - e0[2 * a + 1] * e1[2 * b + 1];
                const double pi = e0[2 * a] * e1[2 * b + 1] + e0[2 * a + 1] * e1[2 * b];
                const double re = pr * e2[2 * c] - pi * e2[2 * c + 1];
                const double im = pr * e2[2 * c + 1] + pi * e2[2 * c];
                double* s = S + 6 * q;
                s[0] += fj0 * re;
                s[1] += fj0 * im;
                s[2] += fj1 * re;
                s[3] += fj1 * im;
                s[4] += fj2 * re;
                s[5] += fj2 * im;
            }
        }
        free(e0);
        free(e1);
        free(e2);
    }
    /* reduce the per-thread partial structure factors in thread order */
    for (int t = 1; t < nth; ++t) {
        const double* src = Sloc + (size_t)t * (size_t)K * 6;
        for (int64_t q = 0; q < 6 * K; ++q) Sloc[q] += src[q];
    }
    const double* S = Sloc;

    /* per target: u_i = (2/V) sum_k A Re{ e^{i k.x_i} (|k|^2 S - k (k.S)) } */
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t t = 0; t < ntt; ++t) {
        const int64_t i = tidx ? tidx[t] : t;
        const double y0 = x[i], y1 = x[n + i], y2 = x[2 * n + i];
        double u0 = 0.0, u1 = 0.0, u2 = 0.0;
        for (int64_t q = 0; q < K; ++q) {
            const double k0 = kv[4 * q], k1 = kv[4 * q + 1], k2 = kv[4 * q + 2], A = kv[4 * q + 3];
            const double kk = k0 * k0 + k1 * k1 + k2 * k2;
            const double* s = S + 6 * q;
            /* v = |k|^2 S - k (k.S), complex 3-vector */
            const double dr = k0 * s[0] + k1 * s[2] + k2 * s[4];
            const double di = k0 * s[1] + k1 * s[3] + k2 * s[5];
            const double v0r = kk * s[0] - k0 * dr, v0i = kk * s[1] - k0 * di;
            const double v1r = kk * s[2] - k1 * dr, v1i = kk * s[3] - k1 * di;
            const double v2r = kk * s[4] - k2 * dr, v2i = kk * s[5] - k2 * di;
            const double ph = k0 * y0 + k1 * y1 + k2 * y2;
            const double c = cos(ph), sn = sin(ph);
            /* Re{(c + i sn)(vr + i vi)} = c vr - sn vi */
            u0 += A * (c * v0r - sn * v0i);
            u1 += A * (c * v1r - sn * v1i);
            u2 += A * (c * v2r - sn * v2i);
        }
        u[t] = 2.0 * u0 / V;
        u[ntt + t] = 2.0 * u1 / V;
        u[2 * ntt + t] = 2.0 * u2 / V;
    }
    free(Sloc);
    free(kn);
    free(kv);
}

/*
 * Plain truncated direct image sum (no Ewald splitting): for each target,
 * sum over whole image cells p in Z^3 L with |p| <= R of G(x_i - x_j + p) f_j,
 * skipping r = 0.  Used only to pin the Ewald value by brute force
 * (spherical summation converges, for zero net force, to the Ewald value plus
 * a shape-dependent affine field).
 */
void ewo_direct_sphere(int64_t n, const double* x, const double* f, const double L[3], double R,
                       double* u)
{
    const int m0 = (int)ceil(R / L[0]), m1 = (int)ceil(R / L[1]), m2 = (int)ceil(R / L[2]);
    const double R2 = R * R;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t i = 0; i < n; ++i) {
        double s0 = 0.0, s1 = 0.0, s2 = 0.0;
        for (int a = -m0; a <= m0; ++a)
            for (int b = -m1; b <= m1; ++b)
                for (int c = -m2; c <= m2; ++c) {
                    const double p0 = a * L[0], p1 = b * L[1], p2 = c * L[2];
                    if (p0 * p0 + p1 * p1 + p2 * p2 > R2) continue;
                    for (int64_t j = 0; j < n; ++j) {
                        const double r0 = x[i] - x[j] + p0;
                        const double r1 = x[n + i] - x[n + j] + p1;
                        const double r2v = x[2 * n + i] - x[2 * n + j] + p2;
                        const double rr = r0 * r0 + r1 * r1 + r2v * r2v;
                        if (rr == 0.0) continue;
                        const double r = sqrt(rr);
                        const double f0 = f[j], f1 = f[n + j], f2 = f[2 * n + j];
                        const double rf = (r0 * f0 + r1 * f1 + r2v * f2) / (rr * r);
                        s0 += f0 / r + rf * r0;
                        s1 += f1 / r + rf * r1;
                        s2 += f2 / r + rf * r2v;
                    }
                }
        u[i] = s0;
        u[n + i] = s1;
        u[2 * n + i] = s2;
    }
}

/* ---------------------------------------------------------------------------
 * Stresslet (double-layer) sources, Sec. 2.2 "Combined single and double layers":
 * each source j also carries vectors q_j, n_j, and
 *
 *     u_a(x_i) += sum_j sum_p' T_abc(x_i - x_j + p) q_jb n_jc,
 *     T_abc(r) = -6 r_a r_b r_c / |r|^5,
 *
 * written here with the source tensor S_j = q_j n_j^T given as 9 rows
 * S[(3 b + c) n + j].  The split uses the same screening as the Stokeslet's:
 * T^F has the Fourier transform That(k) (1 + k^2/(4 xi^2)) e^{-k^2/(4 xi^2)} with
 *     That_abc(k) = (8 pi i / k^4) (k^2 (delta_bc k_a + delta_ab k_c + delta_ac k_b) - 2 k_a k_b k_c),
 * and the real-space remainder (derived in the design notes from T = -2 d_a d_b d_c |r|
 * + 2 (delta_bc d_a + delta_ab d_c + delta_ac d_b) |r|^{-1}, with the Hasimoto split of
 * |r| and of 1/|r|) is
 *     T^N_abc(r) = A(r) rh_a rh_b rh_c + B(r) (delta_ab rh_c + delta_ac rh_b + delta_bc rh_a),
 *     A = -2 (3 erfc(xi r) / r^2 + (6 xi / (sqrt(pi) r) + 4 xi^3 r / sqrt(pi)) e^{-xi^2 r^2}),
 *     B = 4 xi^3 r e^{-xi^2 r^2} / sqrt(pi),      rh = r / |r|.
 * T^F is odd, so the far field needs no self correction.
 */
void ewo_real_space_st(int64_t n, const double* x, const double* S, int64_t nt, const int64_t* tidx,
                       const double L[3], double xi, double r_cut, double* u)
{
    double* xw = (double*)malloc(sizeof(double) * 3 * (size_t)(n > 0 ? n : 1));
    ewo_wrap(n, x, L, xw);
    const double rc2 = r_cut * r_cut;
    const double sqrtpi = sqrt(EWO_PI);
    const int64_t ntt = tidx ? nt : n;

#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t t = 0; t < ntt; ++t) {
        const int64_t i = tidx ? tidx[t] : t;
        double acc[3] = {0.0, 0.0, 0.0};
        for (int64_t j = 0; j < n; ++j) {
            const double d[3] = {xw[i] - xw[j], xw[n + i] - xw[n + j], xw[2 * n + i] - xw[2 * n + j]};
            int lo[3], hi[3];
            for (int a = 0; a < 3; ++a) {
                lo[a] = (int)ceil((-r_cut - d[a]) / L[a]);
                hi[a] = (int)floor((r_cut - d[a]) / L[a]);
            }
            double Sj[3][3];
            for (int b = 0; b < 3; ++b)
                for (int c = 0; c < 3; ++c) Sj[b][c] = S[(3 * b + c) * n + j];
            for (int m0 = lo[0]; m0 <= hi[0]; ++m0)
                for (int m1 = lo[1]; m1 <= hi[1]; ++m1)
                    for (int m2 = lo[2]; m2 <= hi[2]; ++m2) {
                        const double rv[3] = {d[0] + m0 * L[0], d[1] + m1 * L[1], d[2] + m2 * L[2]};
                        const double rr = rv[0] * rv[0] + rv[1] * rv[1] + rv[2] * rv[2];
                        if (!(rr < rc2) || rr == 0.0) continue;
                        const double r = sqrt(rr);
                        const double e = exp(-xi * xi * rr);
                        const double A = -2.0 * (3.0 * erfc(xi * r) / rr + (6.0 * xi / (sqrtpi * r) +
                                                                           4.0 * xi * xi * xi * r / sqrtpi) * e);
                        const double B = 4.0 * xi * xi * xi * r * e / sqrtpi;
                        const double rh[3] = {rv[0] / r, rv[1] / r, rv[2] / r};
                        for (int a = 0; a < 3; ++a)
                            for (int b = 0; b < 3; ++b)
                                for (int c = 0; c < 3; ++c) {
                                    const double T = A * rh[a] * rh[b] * rh[c] +
                                                     B * ((a == b) * rh[c] + (a == c) * rh[b] + (b == c) * rh[a]);
                                    acc[a] += T * Sj[b][c];
                                }
                    }
        }
        for (int a = 0; a < 3; ++a) u[a * ntt + t] = acc[a];
    }
    free(xw);
}

/*
 * Fourier-space stresslet sum on the 3-periodic lattice (k != 0, |k| <= k_max):
 *   u_a(x_i) = (1/V) sum_k Re{ e^{i k.x_i} That^F_abc(k) Shat_bc(k) },  Shat(k) = sum_j S_j e^{-i k.x_j},
 * with That^F = i A(k) P_abc(k), A = 8 pi / k^4 (1 + k^2/(4 xi^2)) e^{-k^2/(4 xi^2)},
 * P_abc = k^2 (delta_bc k_a + delta_ab k_c + delta_ac k_b) - 2 k_a k_b k_c (real); over the
 * half space with a factor 2 (the k and -k terms are complex conjugates).
 */
void ewo_recip_st(int64_t n, const double* x, const double* S, int64_t nt, const int64_t* tidx,
                  const double L[3], double xi, double k_max, double* u)
{
    const int64_t ntt = tidx ? nt : n;
    const double V = L[0] * L[1] * L[2];
    const int nk[3] = {(int)floor(k_max * L[0] / (2.0 * EWO_PI)), (int)floor(k_max * L[1] / (2.0 * EWO_PI)),
                       (int)floor(k_max * L[2] / (2.0 * EWO_PI))};
    const double km2 = k_max * k_max;
    const double inv4xi2 = 1.0 / (4.0 * xi * xi);
    int64_t cap = (int64_t)(nk[0] + 1) * (2 * nk[1] + 1) * (2 * nk[2] + 1);
    double* kv = (double*)malloc(sizeof(double) * 4 * (size_t)cap);
    int64_t K = 0;
    for (int a = 0; a <= nk[0]; ++a)
        for (int b = -nk[1]; b <= nk[1]; ++b)
            for (int c = -nk[2]; c <= nk[2]; ++c) {
                if (a == 0 && (b < 0 || (b == 0 && c <= 0))) continue;
                const double k0 = 2.0 * EWO_PI * a / L[0], k1 = 2.0 * EWO_PI * b / L[1], k2 = 2.0 * EWO_PI * c / L[2];
                const double kk = k0 * k0 + k1 * k1 + k2 * k2;
                if (kk > km2) continue;
                kv[4 * K] = k0;
                kv[4 * K + 1] = k1;
                kv[4 * K + 2] = k2;
                kv[4 * K + 3] = 8.0 * EWO_PI / (kk * kk) * (1.0 + kk * inv4xi2) * exp(-kk * inv4xi2);
                ++K;
            }
    /* structure factors Shat_bc(k): 9 complex numbers per k, summed per thread */
    int nth = ewo_num_threads();
    double* Sloc = (double*)calloc((size_t)nth * (size_t)K * 18, sizeof(double));
#pragma omp parallel
    {
        int tid = 0;
#ifdef _OPENMP
        tid = omp_get_thread_num();
#endif
        double* Sh = Sloc + (size_t)tid * (size_t)K * 18;
#pragma omp for schedule(static)
        for (int64_t j = 0; j < n; ++j) {
            for (int64_t q = 0; q < K; ++q) {
                const double ph = kv[4 * q] * x[j] + kv[4 * q + 1] * x[n + j] + kv[4 * q + 2] * x[2 * n + j];
                const double re = cos(ph), im = -sin(ph);
                for (int bc = 0; bc < 9; ++bc) {
                    const double s = S[bc * n + j];
                    Sh[18 * q + 2 * bc] += s * re;
                    Sh[18 * q + 2 * bc + 1] += s * im;
                }
            }
        }
    }
    for (int t = 1; t < nth; ++t) {
        const double* src = Sloc + (size_t)t * (size_t)K * 18;
        for (int64_t q = 0; q < 18 * K; ++q) Sloc[q] += src[q];
    }
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t t = 0; t < ntt; ++t) {
        const int64_t i = tidx ? tidx[t] : t;
        double acc[3] = {0.0, 0.0, 0.0};
        for (int64_t q = 0; q < K; ++q) {
            const double k[3] = {kv[4 * q], kv[4 * q + 1], kv[4 * q + 2]};
            const double Ak = kv[4 * q + 3];
            const double kk = k[0] * k[0] + k[1] * k[1] + k[2] * k[2];
            const double* sh = Sloc + 18 * q;
            const double ph = k[0] * x[i] + k[1] * x[n + i] + k[2] * x[2 * n + i];
            const double cph = cos(ph), sph = sin(ph);
            for (int a = 0; a < 3; ++a) {
                double wr = 0.0, wi = 0.0; /* w_a = P_abc Shat_bc */
                for (int b = 0; b < 3; ++b)
                    for (int c = 0; c < 3; ++c) {
                        const double P = kk * ((b == c) * k[a] + (a == b) * k[c] + (a == c) * k[b]) -
                                         2.0 * k[a] * k[b] * k[c];
                        wr += P * sh[2 * (3 * b + c)];
                        wi += P * sh[2 * (3 * b + c) + 1];
                    }
                /* Re{ e^{i ph} i A w } = -A (cos(ph) wi + sin(ph) wr) */
                acc[a] += -Ak * (cph * wi + sph * wr);
            }
        }
        for (int a = 0; a < 3; ++a) u[a * ntt + t] = 2.0 * acc[a] / V;
    }
    free(Sloc);
    free(kv);
}
