// Fourier grid convolution (FGC): FFT, CNV, IFFT of Sec. 2.2 steps (2)-(4), hand-written
// for gfx950.
//
// The three real grid components phi_d (M1 x M2 x M3, z fastest) are transformed in
// place into the half spectrum kz = 0..M3/2-1 (the kz = M3/2 Nyquist plane is zero after
// CNV and is never stored, so the spectrum occupies exactly the real grid's bytes):
//   pass 1  z, real-to-complex: each z-line is read as M3/2 complex numbers, transformed
//           with a length-M3/2 complex FFT and unpacked into the half spectrum;
//   pass 2  y, complex, strided;
//   pass 3  x, complex, strided, for the three components together: forward FFT, then
//           the diagonal CNV scaling of eq. (sca) with Ghat^F of eq. (GFk) evaluated in
//           FP64, then the inverse FFT, without leaving LDS;
//   pass 4  y inverse;
//   pass 5  z, complex-to-real (the inverse of pass 1).
// Where a (y, z) plane of one component fits in a workgroup's LDS, passes 1+2 and 4+5 are
// each one kernel (k_fft_zy, in-place transforms).
// Each 1D transform is a Stockham radix-4 (plus one radix-2 stage for odd log2 n)
// autosort FFT held in LDS, one workgroup per batch of adjacent columns (adjacent in
// memory, so every row of a batch is one contiguous read).  Twiddles come from FP64 host
// tables.  The k = 0 mode and the Nyquist planes are set to zero; the half-spectrum
// convolution is enough because every field involved is real (Sec. 3.4).  The global
// scale h1 h2 h3 / (M1 M2 M3) of the DFT round trip and of eq. (g2p) is folded into the
// CNV tables, so the inverse transforms are unnormalised.
#include "internal.h"

namespace ewald {

namespace {

// aligned to its size, so that one complex value is one 16-byte (FP64) or 8-byte (FP32) access:
// a pair of 8-byte LDS loads (ds_read2_b64) occupies the LDS pipeline twice as long as one
// ds_read_b128 on gfx950
template <typename T>
struct alignas(2 * sizeof(T)) C2 {
    T x, y;
};

template <typename T>
__device__ inline C2<T> cmul(C2<T> a, C2<T> b)
{
    return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}

template <typename T>
__device__ inline C2<T> cadd(C2<T> a, C2<T> b) { return {a.x + b.x, a.y + b.y}; }
template <typename T>
__device__ inline C2<T> csub(C2<T> a, C2<T> b) { return {a.x - b.x, a.y - b.y}; }

// Batched Stockham FFT of ncomp x ncols columns of length n stored as
// a[(comp * n + e) * ld + c] (n and ncols powers of two, ld >= ncols the row stride).  sign = -1 forward, +1
// inverse (unnormalised).  `b` is scratch of the same size.  Returns the buffer holding
// the result (a or b).  All threads of the block take part; ends with a barrier.
template <typename T>
__device__ C2<T>* lds_fft(C2<T>* a, C2<T>* b, int n, int ncols, int ld, int ncomp, int sign,
                          const C2<T>* __restrict__ tw)
{
    C2<T>* src = a;
    C2<T>* dst = b;
    const int cmask = ncols - 1;
    int lc = 0;
    while ((1 << lc) < ncols) ++lc;
    for (int p = 1; p < n;) {
        const int R = (n / p >= 4) ? 4 : 2;
        const int Tn = n / R;
        const int per = Tn * ncols;  // butterflies per component (power of two)
        int lp = 0;
        while ((1 << lp) < per) ++lp;
        const int total = per * ncomp;
        const int tws = n / (p * R);
        for (int bi = threadIdx.x; bi < total; bi += blockDim.x) {
            const int comp = bi >> lp;
            const int rem = bi & (per - 1);
            const int c = rem & cmask;
            const int i = rem >> lc;
            const int k = i & (p - 1);
            const int j = (i - k) * R + k;
            C2<T>* sp = src + (size_t)comp * n * ld;
            C2<T>* dp = dst + (size_t)comp * n * ld;
            if (R == 4) {
                C2<T> u0 = sp[(i)*ld + c];
                C2<T> u1 = sp[(i + Tn) * ld + c];
                C2<T> u2 = sp[(i + 2 * Tn) * ld + c];
                C2<T> u3 = sp[(i + 3 * Tn) * ld + c];
                if (k) {
                    C2<T> w1 = tw[(k * tws) & (n - 1)];
                    C2<T> w2 = tw[(2 * k * tws) & (n - 1)];
                    C2<T> w3 = tw[(3 * k * tws) & (n - 1)];
                    if (sign > 0) {
                        w1.y = -w1.y;
                        w2.y = -w2.y;
                        w3.y = -w3.y;
                    }
                    u1 = cmul(u1, w1);
                    u2 = cmul(u2, w2);
                    u3 = cmul(u3, w3);
                }
                const C2<T> t0 = cadd(u0, u2), t1 = csub(u0, u2), t2 = cadd(u1, u3), d = csub(u1, u3);
                // forward: -i d ; inverse: +i d
                const C2<T> rot = (sign < 0) ? C2<T>{d.y, -d.x} : C2<T>{-d.y, d.x};
                dp[(j)*ld + c] = cadd(t0, t2);
                dp[(j + p) * ld + c] = cadd(t1, rot);
                dp[(j + 2 * p) * ld + c] = csub(t0, t2);
                dp[(j + 3 * p) * ld + c] = csub(t1, rot);
            } else {
                C2<T> u0 = sp[(i)*ld + c];
                C2<T> u1 = sp[(i + Tn) * ld + c];
                if (k) {
                    C2<T> w1 = tw[(k * tws) & (n - 1)];
                    if (sign > 0) w1.y = -w1.y;
                    u1 = cmul(u1, w1);
                }
                dp[(j)*ld + c] = cadd(u0, u1);
                dp[(j + p) * ld + c] = csub(u0, u1);
            }
        }
        __syncthreads();
        C2<T>* tmp = src;
        src = dst;
        dst = tmp;
        p *= R;
    }
    return src;
}

// ---- pass 1 / 5: z-lines, real <-> half spectrum ----

template <typename T>
__global__ __launch_bounds__(256) void k_fft_z(T* __restrict__ grid, int64_t ncells, int nlines, int H,
                                               int ncols, int sign, const C2<T>* __restrict__ tw_half,
                                               const C2<T>* __restrict__ tw_full)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    // rows padded to ncols + 1 elements: a line's consecutive elements, which consecutive
    // threads load and store, then fall in different LDS banks (with a power-of-two row
    // stride they would all hit a few banks)
    const int ld = ncols + 1;
    C2<T>* a = reinterpret_cast<C2<T>*>(smem_raw);
    C2<T>* b = a + (size_t)H * ld;
    C2<T>* data = reinterpret_cast<C2<T>*>(grid + blockIdx.y * ncells);
    const int line0 = blockIdx.x * ncols;
    const int tot = H * ncols;

    if (sign < 0) {
        for (int idx = threadIdx.x; idx < tot; idx += blockDim.x) {
            const int c = idx / H, e = idx - c * H;
            if (line0 + c < nlines) a[e * ld + c] = data[(int64_t)(line0 + c) * H + e];
            else a[e * ld + c] = C2<T>{0, 0};
        }
        __syncthreads();
        C2<T>* C = lds_fft<T>(a, b, H, ncols, ld, 1, -1, tw_half);
        for (int idx = threadIdx.x; idx < tot; idx += blockDim.x) {
            const int c = idx / H, k = idx - c * H;
            if (line0 + c >= nlines) continue;
            const C2<T> ck = C[k * ld + c];
            const C2<T> cm0 = C[((H - k) & (H - 1)) * ld + c];
            const C2<T> cm = {cm0.x, -cm0.y};
            const C2<T> E = {(T)0.5 * (ck.x + cm.x), (T)0.5 * (ck.y + cm.y)};
            const C2<T> dd = csub(ck, cm);
            const C2<T> O = {(T)0.5 * dd.y, (T)-0.5 * dd.x};  // -i/2 (ck - cm)
            data[(int64_t)(line0 + c) * H + k] = cadd(E, cmul(tw_full[k], O));
        }
    } else {
        for (int idx = threadIdx.x; idx < tot; idx += blockDim.x) {
            const int c = idx / H, e = idx - c * H;
            if (line0 + c < nlines) b[e * ld + c] = data[(int64_t)(line0 + c) * H + e];
            else b[e * ld + c] = C2<T>{0, 0};
        }
        __syncthreads();
        for (int idx = threadIdx.x; idx < tot; idx += blockDim.x) {
            const int c = idx / H, k = idx - c * H;
            C2<T> xk = b[k * ld + c];
            C2<T> xm;
            if (k == 0) {
                xk.y = 0;             // DC of a real line
                xm = C2<T>{0, 0};     // Nyquist (zeroed by CNV)
            } else {
                const C2<T> v = b[(H - k) * ld + c];
                xm = C2<T>{v.x, -v.y};
            }
            const C2<T> E = cadd(xk, xm);
            C2<T> w = tw_full[k];
            w.y = -w.y;  // e^{+2 pi i k / M3}
            const C2<T> O = cmul(csub(xk, xm), w);
            a[k * ld + c] = C2<T>{E.x - O.y, E.y + O.x};  // E + i O
        }
        __syncthreads();
        C2<T>* z = lds_fft<T>(a, b, H, ncols, ld, 1, +1, tw_half);
        for (int idx = threadIdx.x; idx < tot; idx += blockDim.x) {
            const int c = idx / H, e = idx - c * H;
            if (line0 + c < nlines) data[(int64_t)(line0 + c) * H + e] = z[e * ld + c];
        }
    }
}

// ---- passes 1+2 / 4+5 fused: one (y, z) plane in LDS ----
//
// When a whole plane x = const of one component (M2 x M3/2 complex values) fits in the LDS of
// a workgroup, its z transforms and y transforms are done in one kernel: the plane is read
// from HBM once and written once per direction (five grid passes become three).  Out-of-place
// Stockham would need a second plane of LDS, so the transforms here are in place: radix-2
// Cooley-Tukey stages taken two at a time (each thread holds the four values of two
// consecutive stages' butterflies), decimation in time from bit-reversed input, or decimation
// in frequency to bit-reversed output.  The bit reversals cost nothing: they are folded into
// the global reads and writes, which stay within one plane row (one contiguous run per wave).

__device__ inline int brev_bits(int v, int bits)
{
    return (int)(__builtin_bitreverse32((unsigned)v) >> (32 - bits));
}

// w^s (s = -1: as tabulated, e^{-2 pi i k / n}; s = +1: conjugate)
template <typename T>
__device__ inline C2<T> twid(const C2<T>* __restrict__ tw, int k, int sign)
{
    C2<T> w = tw[k];
    if (sign > 0) w.y = -w.y;
    return w;
}

// In place, `nt` transforms of length n = 2^m for each of `ncomp` components: element e of
// transform t of component k at a[k * cs + t * ts + e * es] (nt a power of two; consecutive
// threads take consecutive transforms, so ts should be the bank-friendly stride).  DIT:
// bit-reversed input, natural output; DIF: the reverse.  tw: the length-n table
// e^{-2 pi i k / n}.  Ends with a barrier.
template <typename T, bool DIT>
__device__ void lds_fft_inplace(C2<T>* a, int n, int m, int nt, int lgnt, int ts, int es, int sign,
                                const C2<T>* __restrict__ tw, int ncomp = 1, int cs = 0)
{
    // one radix-2 stage of span q (twiddles W_{2q}^j = tw[j n / (2q)])
    auto single = [&](int q) {
        const int nb = n >> 1, lgnb = m - 1;
        for (int idx = threadIdx.x; idx < nt * nb * ncomp; idx += blockDim.x) {
            const int t = idx & (nt - 1), rest = idx >> lgnt;
            const int bi = rest & (nb - 1), k = rest >> lgnb;
            const int j = bi & (q - 1), e0 = 2 * (bi - j) + j;
            C2<T>* p0 = a + k * cs + t * ts + e0 * es;
            C2<T>* p1 = p0 + q * es;
            const C2<T> u = *p0, v = *p1;
            const C2<T> w = twid(tw, j * (n / (2 * q)), sign);
            if (DIT) {
                const C2<T> vw = cmul(v, w);
                *p0 = cadd(u, vw);
                *p1 = csub(u, vw);
            } else {
                *p0 = cadd(u, v);
                *p1 = cmul(csub(u, v), w);
            }
        }
        __syncthreads();
    };
    // the stages of spans q and 2q (DIT: q first; DIF: 2q first) on the four values at
    // e0 + {0, q, 2q, 3q}
    auto pair = [&](int q) {
        const int nb = n >> 2, lgnb = m - 2;
        for (int idx = threadIdx.x; idx < nt * nb * ncomp; idx += blockDim.x) {
            const int t = idx & (nt - 1), rest = idx >> lgnt;
            const int bi = rest & (nb - 1), k = rest >> lgnb;
            const int j = bi & (q - 1), e0 = 4 * (bi - j) + j;
            C2<T>* p0 = a + k * cs + t * ts + e0 * es;
            const int sq = q * es;
            const C2<T> x0 = p0[0], x1 = p0[sq], x2 = p0[2 * sq], x3 = p0[3 * sq];
            const C2<T> wa = twid(tw, j * (n / (2 * q)), sign);  // W_{2q}^j
            const C2<T> wb = twid(tw, j * (n / (4 * q)), sign);  // W_{4q}^j
            // W_{4q}^{j+q} = W_{4q}^j W_4^1, W_4^1 = -i (forward) or +i (inverse)
            const C2<T> wc = (sign < 0) ? C2<T>{wb.y, -wb.x} : C2<T>{-wb.y, wb.x};
            if (DIT) {
                const C2<T> v1 = cmul(x1, wa), v3 = cmul(x3, wa);
                const C2<T> t0 = cadd(x0, v1), t1 = csub(x0, v1), t2 = cadd(x2, v3), t3 = csub(x2, v3);
                const C2<T> u2 = cmul(t2, wb), u3 = cmul(t3, wc);
                p0[0] = cadd(t0, u2);
                p0[2 * sq] = csub(t0, u2);
                p0[sq] = cadd(t1, u3);
                p0[3 * sq] = csub(t1, u3);
            } else {
                const C2<T> t0 = cadd(x0, x2), t2 = cmul(csub(x0, x2), wb);
                const C2<T> t1 = cadd(x1, x3), t3 = cmul(csub(x1, x3), wc);
                p0[0] = cadd(t0, t1);
                p0[sq] = cmul(csub(t0, t1), wa);
                p0[2 * sq] = cadd(t2, t3);
                p0[3 * sq] = cmul(csub(t2, t3), wa);
            }
        }
        __syncthreads();
    };
    if (DIT) {
        int q = 1;
        if (m & 1) {
            single(1);
            q = 2;
        }
        for (; q < n; q *= 4) pair(q);
    } else {
        for (int q = n >> 2; q >= 1; q >>= 2) pair(q);
        if (m & 1) single(1);
    }
}

// sign -1: z (real to half spectrum) then y, forward; sign +1: y then z (half spectrum to real),
// inverse.  Grid: (M1 planes, components); the plane's LDS rows are padded by one element.
template <typename T>
__global__ __launch_bounds__(1024) void k_fft_zy(T* __restrict__ grid, int64_t ncells, int M2, int lgM2, int H,
                                                 int lgH, int sign, const C2<T>* __restrict__ tw_half,
                                                 const C2<T>* __restrict__ tw_full, const C2<T>* __restrict__ tw_y)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    C2<T>* a = reinterpret_cast<C2<T>*>(smem_raw);
    const int ld = H + 1;
    C2<T>* data = reinterpret_cast<C2<T>*>(grid + blockIdx.y * ncells) + (int64_t)blockIdx.x * M2 * H;
    const int tot = M2 * H;
    const int half = H >> 1;
    if (sign < 0) {
        for (int idx = threadIdx.x; idx < tot; idx += blockDim.x) {
            const int y = idx >> lgH, p = idx & (H - 1);
            a[y * ld + p] = data[y * H + brev_bits(p, lgH)];
        }
        __syncthreads();
        lds_fft_inplace<T, true>(a, H, lgH, M2, lgM2, ld, 1, -1, tw_half);
        // half spectrum of the real line from the length-H transform C of its even/odd pairs:
        // X_k = E_k + e^{-2 pi i k / M3} O_k, E_k = (C_k + conj C_{H-k}) / 2,
        // O_k = -i (C_k - conj C_{H-k}) / 2; k and H - k are done together (in place)
        for (int idx = threadIdx.x; idx < M2 * (half + 1); idx += blockDim.x) {
            const int y = idx & (M2 - 1), k = idx >> lgM2;
            C2<T>* row = a + y * ld;
            const int kh = (H - k) & (H - 1);
            const C2<T> ck = row[k], ch = row[kh];
            auto unpack = [&](C2<T> c, C2<T> d, int kk) {
                const C2<T> cm = {d.x, -d.y};
                const C2<T> E = {(T)0.5 * (c.x + cm.x), (T)0.5 * (c.y + cm.y)};
                const C2<T> dd = csub(c, cm);
                const C2<T> O = {(T)0.5 * dd.y, (T)-0.5 * dd.x};
                return cadd(E, cmul(tw_full[kk], O));
            };
            const C2<T> xk = unpack(ck, ch, k);
            if (kh != k) row[kh] = unpack(ch, ck, kh);
            row[k] = xk;
        }
        __syncthreads();
        lds_fft_inplace<T, false>(a, M2, lgM2, H, lgH, 1, ld, -1, tw_y);
        for (int idx = threadIdx.x; idx < tot; idx += blockDim.x) {
            const int p = idx >> lgH, kz = idx & (H - 1);
            data[brev_bits(p, lgM2) * H + kz] = a[p * ld + kz];
        }
    } else {
        for (int idx = threadIdx.x; idx < tot; idx += blockDim.x) {
            const int p = idx >> lgH, kz = idx & (H - 1);
            a[p * ld + kz] = data[brev_bits(p, lgM2) * H + kz];
        }
        __syncthreads();
        lds_fft_inplace<T, true>(a, M2, lgM2, H, lgH, 1, ld, +1, tw_y);
        // the inverse of the unpacking: C_k = E_k + i O_k with E_k = X_k + conj X_{H-k},
        // O_k = (X_k - conj X_{H-k}) e^{+2 pi i k / M3}; X_0 is real (its imaginary part holds
        // nothing) and the Nyquist value X_{M3/2} is zero (CNV)
        for (int idx = threadIdx.x; idx < M2 * (half + 1); idx += blockDim.x) {
            const int y = idx & (M2 - 1), k = idx >> lgM2;
            C2<T>* row = a + y * ld;
            const int kh = (H - k) & (H - 1);
            const C2<T> xk = row[k], xh = row[kh];
            auto pack = [&](C2<T> c, C2<T> d, int kk) {
                C2<T> xm;
                if (kk == 0) {
                    c.y = 0;
                    xm = C2<T>{0, 0};
                } else {
                    xm = C2<T>{d.x, -d.y};
                }
                const C2<T> E = cadd(c, xm);
                C2<T> w = tw_full[kk];
                w.y = -w.y;
                const C2<T> O = cmul(csub(c, xm), w);
                return C2<T>{E.x - O.y, E.y + O.x};
            };
            const C2<T> ck = pack(xk, xh, k);
            if (kh != k) row[kh] = pack(xh, xk, kh);
            row[k] = ck;
        }
        __syncthreads();
        lds_fft_inplace<T, false>(a, H, lgH, M2, lgM2, ld, 1, +1, tw_half);
        for (int idx = threadIdx.x; idx < tot; idx += blockDim.x) {
            const int y = idx >> lgH, p = idx & (H - 1);
            data[y * H + brev_bits(p, lgH)] = a[y * ld + p];
        }
    }
}

// ---- pass 2 / 4: y-columns ----

template <typename T>
__global__ __launch_bounds__(256) void k_fft_y(T* __restrict__ grid, int64_t ncells, int M2, int H,
                                               int ncols, int sign, const C2<T>* __restrict__ tw)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    C2<T>* a = reinterpret_cast<C2<T>*>(smem_raw);
    C2<T>* b = a + (size_t)M2 * ncols;
    C2<T>* data = reinterpret_cast<C2<T>*>(grid + blockIdx.y * ncells);
    const int tiles_per_x = H / ncols;
    // blocks of consecutive z-runs share cache lines: each XCD takes a contiguous range of blocks
    // (blocks are dealt to the 8 XCDs round robin), so that a line is fetched into one L2
    const int bx = xcd_remap((int)blockIdx.x, (int)gridDim.x);
    const int x = bx / tiles_per_x;
    const int kz0 = (bx - x * tiles_per_x) * ncols;
    const int64_t base = (int64_t)x * M2 * H + kz0;
    const int tot = M2 * ncols;
    for (int idx = threadIdx.x; idx < tot; idx += blockDim.x) {
        const int e = idx / ncols, c = idx - e * ncols;
        a[idx] = data[base + (int64_t)e * H + c];
    }
    __syncthreads();
    C2<T>* r = lds_fft<T>(a, b, M2, ncols, ncols, 1, sign, tw);
    for (int idx = threadIdx.x; idx < tot; idx += blockDim.x) {
        const int e = idx / ncols, c = idx - e * ncols;
        data[base + (int64_t)e * H + c] = r[idx];
    }
}

// ---- pass 3: x-columns, forward FFT + CNV + inverse FFT, 3 components together ----

struct CnvArgs {
    double twopi_over_L[3];
    double inv4xi2;
    double eightpi;
    const double* E0;  // per-axis factors (alpha/pi) exp(k^2 (1/(2 alpha) - 1/(4 xi^2))), scale folded in E0
    const double* E1;
    const double* E2;
};

// CNV at one wavenumber k = (k0, k1, k2) (index kx, kz; e1 = E1[ky]) of the three components
// r[idx], r[per + idx], r[2 per + idx]: the scaling of eq. (sca) with Ghat^F of eq. (GFk), FP64
template <typename T>
__device__ inline void cnv_point(C2<T>* r, int per, int idx, int kx, int kz, double k0, double k1, double k2,
                                 double e1, const CnvArgs& ca)
{
    const double K2 = k0 * k0 + k1 * k1 + k2 * k2;
    double A = 0.0;
    if (K2 > 0.0) A = ca.E0[kx] * e1 * ca.E2[kz] * ca.eightpi * (1.0 + K2 * ca.inv4xi2) / (K2 * K2);
    C2<T>* p0 = &r[idx];
    C2<T>* p1 = &r[per + idx];
    C2<T>* p2 = &r[2 * per + idx];
    const double q0r = p0->x, q0i = p0->y, q1r = p1->x, q1i = p1->y, q2r = p2->x, q2i = p2->y;
    const double dr = k0 * q0r + k1 * q1r + k2 * q2r;
    const double di = k0 * q0i + k1 * q1i + k2 * q2i;
    *p0 = C2<T>{(T)(A * (K2 * q0r - k0 * dr)), (T)(A * (K2 * q0i - k0 * di))};
    *p1 = C2<T>{(T)(A * (K2 * q1r - k1 * dr)), (T)(A * (K2 * q1i - k1 * di))};
    *p2 = C2<T>{(T)(A * (K2 * q2r - k2 * dr)), (T)(A * (K2 * q2i - k2 * di))};
}

template <typename T>
__global__ __launch_bounds__(256) void k_fft_x_cnv(T* __restrict__ grid, int64_t ncells, int M1, int M2,
                                                   int H, int ncols, int do_cnv, int do_inv,
                                                   const C2<T>* __restrict__ tw, CnvArgs ca)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int per = M1 * ncols;  // elements per component (power of two)
    C2<T>* a = reinterpret_cast<C2<T>*>(smem_raw);
    C2<T>* b = a + (size_t)3 * per;
    grid += (int64_t)blockIdx.y * 3 * ncells;  // system blockIdx.y of a batch
    const int tiles_per_y = H / ncols;
    // runs of ncols z-elements (2 complex at 128^3 FP64): the blocks of one cache line go to one
    // XCD (see k_fft_y)
    const int bx = xcd_remap((int)blockIdx.x, (int)gridDim.x);
    const int ky = bx / tiles_per_y;
    const int kz0 = (bx - ky * tiles_per_y) * ncols;
    const int64_t rowstride = (int64_t)M2 * H;  // complex elements between consecutive x
    const int tot = 3 * per;
    for (int idx = threadIdx.x; idx < tot; idx += blockDim.x) {
        const int comp = idx / per, rem = idx - comp * per;
        const int e = rem / ncols, c = rem - e * ncols;
        const C2<T>* data = reinterpret_cast<const C2<T>*>(grid + comp * ncells);
        a[idx] = data[(int64_t)e * rowstride + (int64_t)ky * H + kz0 + c];
    }
    __syncthreads();
    C2<T>* r = lds_fft<T>(a, b, M1, ncols, ncols, 3, -1, tw);
    if (do_cnv) {
        const int kys = (ky < M2 / 2) ? ky : ky - M2;
        const double k1 = ca.twopi_over_L[1] * kys;
        const double e1 = ca.E1[ky];
        for (int idx = threadIdx.x; idx < per; idx += blockDim.x) {
            const int kx = idx / ncols, c = idx - kx * ncols;
            const int kz = kz0 + c;
            const int kxs = (kx < M1 / 2) ? kx : kx - M1;
            const double k0 = ca.twopi_over_L[0] * kxs;
            cnv_point(r, per, idx, kx, kz, k0, k1, ca.twopi_over_L[2] * kz, e1, ca);
        }
        __syncthreads();
    }
    if (do_inv) r = lds_fft<T>(r, (r == a) ? b : a, M1, ncols, ncols, 3, +1, tw);
    for (int idx = threadIdx.x; idx < tot; idx += blockDim.x) {
        const int comp = idx / per, rem = idx - comp * per;
        const int e = rem / ncols, c = rem - e * ncols;
        C2<T>* data = reinterpret_cast<C2<T>*>(grid + comp * ncells);
        data[(int64_t)e * rowstride + (int64_t)ky * H + kz0 + c] = r[idx];
    }
}

// ---- pass 3 for combined single and double layer sources ----
// The 9 components (force 0-2, symmetric stresslet tensor 3-8: xx, yy, zz, xy, xz, yz) have
// been transformed along x (k_fft_x_cnv without CNV).  Per x-column batch: CNV 9 -> 3 in
// FP64 (Sec. 2.3, combined layers),
//   vhat_a = A(k) [ (k^2 phi_a - k_a (k.phi)) + i (k^2 (k_a tr S + 2 (S k)_a) - 2 k_a (k.S k)) ],
// the first term Ghat^F, the second That^F of the stresslet (That_abc = (8 pi i / k^4)
// (k^2 (delta_bc k_a + delta_ab k_c + delta_ac k_b) - 2 k_a k_b k_c), contracted with the
// symmetric S), A = 8 pi / k^4 (1 + k^2/(4 xi^2)) e^{-k^2/(4 xi^2)} / what^2 with the DFT and
// h^3 scales folded in; then the inverse x transform of the 3 results.
// The same pass (forward x FFT, CNV, inverse x FFT of the three components) with one LDS buffer:
// in-place stages (see lds_fft_inplace), forward by decimation in frequency, which leaves LDS row p
// holding kx = the bit reversal of p, CNV on that order, inverse by decimation in time, which
// takes it back to natural order.  Twice the columns per block of the two-buffer kernel in the
// same LDS.  lgM1, lgnc: log2 of M1 and of ncols.
template <typename T>
__global__ __launch_bounds__(256) void k_fft_x_cnv_ip(T* __restrict__ grid, int64_t ncells, int M1, int lgM1,
                                                      int M2, int H, int ncols, int lgnc,
                                                      const C2<T>* __restrict__ tw, CnvArgs ca)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int per = M1 * ncols;  // elements per component (power of two)
    C2<T>* a = reinterpret_cast<C2<T>*>(smem_raw);
    grid += (int64_t)blockIdx.y * 3 * ncells;  // system blockIdx.y of a batch
    const int tiles_per_y = H / ncols;
    const int bx = xcd_remap((int)blockIdx.x, (int)gridDim.x);
    const int ky = bx / tiles_per_y;
    const int kz0 = (bx - ky * tiles_per_y) * ncols;
    const int64_t rowstride = (int64_t)M2 * H;  // complex elements between consecutive x
    const int tot = 3 * per;
    for (int idx = threadIdx.x; idx < tot; idx += blockDim.x) {
        const int comp = idx / per, rem = idx - comp * per;
        const int e = rem >> lgnc, c = rem & (ncols - 1);
        const C2<T>* data = reinterpret_cast<const C2<T>*>(grid + comp * ncells);
        a[idx] = data[(int64_t)e * rowstride + (int64_t)ky * H + kz0 + c];
    }
    __syncthreads();
    lds_fft_inplace<T, false>(a, M1, lgM1, ncols, lgnc, 1, ncols, -1, tw, 3, per);
    const int kys = (ky < M2 / 2) ? ky : ky - M2;
    const double k1 = ca.twopi_over_L[1] * kys;
    const double e1 = ca.E1[ky];
    for (int idx = threadIdx.x; idx < per; idx += blockDim.x) {
        const int kx = brev_bits(idx >> lgnc, lgM1), c = idx & (ncols - 1);
        const int kz = kz0 + c;
        const int kxs = (kx < M1 / 2) ? kx : kx - M1;
        cnv_point(a, per, idx, kx, kz, ca.twopi_over_L[0] * kxs, k1, ca.twopi_over_L[2] * kz, e1, ca);
    }
    __syncthreads();
    lds_fft_inplace<T, true>(a, M1, lgM1, ncols, lgnc, 1, ncols, +1, tw, 3, per);
    for (int idx = threadIdx.x; idx < tot; idx += blockDim.x) {
        const int comp = idx / per, rem = idx - comp * per;
        const int e = rem >> lgnc, c = rem & (ncols - 1);
        C2<T>* data = reinterpret_cast<C2<T>*>(grid + comp * ncells);
        data[(int64_t)e * rowstride + (int64_t)ky * H + kz0 + c] = a[idx];
    }
}

template <typename T>
__global__ __launch_bounds__(256) void k_cnv_st_x(T* __restrict__ grid, int64_t ncells, int M1, int M2, int H,
                                                  int ncols, const C2<T>* __restrict__ tw, CnvArgs ca)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int per = M1 * ncols;
    C2<T>* a = reinterpret_cast<C2<T>*>(smem_raw);
    C2<T>* b = a + (size_t)3 * per;
    const int tiles_per_y = H / ncols;
    // runs of ncols z-elements (2 complex at 128^3 FP64): the blocks of one cache line go to one
    // XCD (see k_fft_y)
    const int bx = xcd_remap((int)blockIdx.x, (int)gridDim.x);
    const int ky = bx / tiles_per_y;
    const int kz0 = (bx - ky * tiles_per_y) * ncols;
    const int64_t rowstride = (int64_t)M2 * H;
    const int kys = (ky < M2 / 2) ? ky : ky - M2;
    const double k1 = ca.twopi_over_L[1] * kys;
    const double e1 = ca.E1[ky];
    for (int idx = threadIdx.x; idx < per; idx += blockDim.x) {
        const int kx = idx / ncols, c = idx - kx * ncols;
        const int kz = kz0 + c;
        const int kxs = (kx < M1 / 2) ? kx : kx - M1;
        const double k0 = ca.twopi_over_L[0] * kxs;
        const double k2 = ca.twopi_over_L[2] * kz;
        const double K2 = k0 * k0 + k1 * k1 + k2 * k2;
        double A = 0.0;
        if (K2 > 0.0) A = ca.E0[kx] * e1 * ca.E2[kz] * ca.eightpi * (1.0 + K2 * ca.inv4xi2) / (K2 * K2);
        const int64_t off = (int64_t)kx * rowstride + (int64_t)ky * H + kz;
        double vr[9], vi[9];
#pragma unroll
        for (int q = 0; q < 9; ++q) {
            const C2<T> v = reinterpret_cast<const C2<T>*>(grid + q * ncells)[off];
            vr[q] = v.x;
            vi[q] = v.y;
        }
        // Stokeslet part
        const double dr = k0 * vr[0] + k1 * vr[1] + k2 * vr[2];
        const double di = k0 * vi[0] + k1 * vi[1] + k2 * vi[2];
        // stresslet part: S k, k.S k, tr S (complex)
        const double skr0 = vr[3] * k0 + vr[6] * k1 + vr[7] * k2, ski0 = vi[3] * k0 + vi[6] * k1 + vi[7] * k2;
        const double skr1 = vr[6] * k0 + vr[4] * k1 + vr[8] * k2, ski1 = vi[6] * k0 + vi[4] * k1 + vi[8] * k2;
        const double skr2 = vr[7] * k0 + vr[8] * k1 + vr[5] * k2, ski2 = vi[7] * k0 + vi[8] * k1 + vi[5] * k2;
        const double ksk_r = k0 * skr0 + k1 * skr1 + k2 * skr2, ksk_i = k0 * ski0 + k1 * ski1 + k2 * ski2;
        const double tr_r = vr[3] + vr[4] + vr[5], tr_i = vi[3] + vi[4] + vi[5];
        const double kk[3] = {k0, k1, k2};
        const double skr[3] = {skr0, skr1, skr2}, ski[3] = {ski0, ski1, ski2};
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            const double wr = K2 * (kk[d] * tr_r + 2.0 * skr[d]) - 2.0 * kk[d] * ksk_r;
            const double wi = K2 * (kk[d] * tr_i + 2.0 * ski[d]) - 2.0 * kk[d] * ksk_i;
            // (K2 phi_d - k_d (k.phi)) + i w
            const double re = K2 * vr[d] - kk[d] * dr - wi;
            const double im = K2 * vi[d] - kk[d] * di + wr;
            a[(size_t)d * per + idx] = C2<T>{(T)(A * re), (T)(A * im)};
        }
    }
    __syncthreads();
    C2<T>* r = lds_fft<T>(a, b, M1, ncols, ncols, 3, +1, tw);
    const int tot = 3 * per;
    for (int idx = threadIdx.x; idx < tot; idx += blockDim.x) {
        const int comp = idx / per, rem = idx - comp * per;
        const int e = rem / ncols, c = rem - e * ncols;
        C2<T>* data = reinterpret_cast<C2<T>*>(grid + comp * ncells);
        data[(int64_t)e * rowstride + (int64_t)ky * H + kz0 + c] = r[idx];
    }
}

inline int pow2_floor(int v)
{
    int p = 1;
    while (p * 2 <= v) p *= 2;
    return p;
}

// the largest dynamic LDS one workgroup may take on the current device
int lds_per_block()
{
    int dev = 0, v = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 65536;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess) return 65536;
    return v;
}

template <typename T>
hipError_t launch_fgc_t(const Plan& pl, const Work& w, hipStream_t s, bool inverse_too, bool cnv, bool st, int nsys)
{
    const Geometry& g = pl.g;
    const int M1 = g.M[0], M2 = g.M[1], M3 = g.M[2], H = M3 / 2;
    const int64_t nc = g.ncells;
    T* grid = (T*)w.grid;
    const C2<T>* tw = (const C2<T>*)(sizeof(T) == 8 ? pl.d_tw64 : pl.d_tw32);
    const C2<T>* tw0 = tw + pl.tw_off[0];
    const C2<T>* tw1 = tw + pl.tw_off[1];
    const C2<T>* twh = tw + pl.tw_off[2];
    const C2<T>* twf = tw + pl.tw_off[3];
    const int budget = (sizeof(T) == 8) ? 1024 : 2048;  // complex elements per buffer

    // passes 1+2 fused when a plane fits in one workgroup's LDS
    int lgH = 0, lgM2 = 0;
    while ((1 << lgH) < H) ++lgH;
    while ((1 << lgM2) < M2) ++lgM2;
    const size_t shzy = (size_t)M2 * (H + 1) * sizeof(C2<T>);
    const bool fused = H >= 4 && M2 >= 4 && shzy <= (size_t)lds_per_block();
    if (fused && shzy > 65536) {
        const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_fft_zy<T>),
                                                 hipFuncAttributeMaxDynamicSharedMemorySize, (int)shzy);
        if (e != hipSuccess) return e;
    }
    // pass 1: z forward (R2C)
    const int nlines = M1 * M2;
    int ncz = pow2_floor(max(1, budget / H));
    if (ncz > nlines) ncz = pow2_floor(nlines);
    size_t shz = 2 * (size_t)H * (ncz + 1) * sizeof(C2<T>);  // rows padded by one element
    // forward transforms: force (+ stresslet tensor); the systems of a batch hold consecutive
    // groups of 3 grid components
    const int ncomp_in = st ? 9 : 3 * nsys;
    dim3 gz((nlines + ncz - 1) / ncz, ncomp_in);
    // pass 2: y forward
    int ncy = pow2_floor(max(1, budget / M2));
    if (ncy > H) ncy = H;
    size_t shy = 2 * (size_t)M2 * ncy * sizeof(C2<T>);
    dim3 gy(M1 * (H / ncy), ncomp_in);
    dim3 gzy(M1, ncomp_in);
    if (fused) {
        hipLaunchKernelGGL((k_fft_zy<T>), gzy, dim3(1024), shzy, s, grid, nc, M2, lgM2, H, lgH, -1, twh, twf, tw1);
    } else {
        hipLaunchKernelGGL((k_fft_z<T>), gz, dim3(256), shz, s, grid, nc, nlines, H, ncz, -1, twh, twf);
        hipLaunchKernelGGL((k_fft_y<T>), gy, dim3(256), shy, s, grid, nc, M2, H, ncy, -1, tw1);
    }
    gy.y = 3 * nsys;  // the inverse transforms carry the 3 velocity components
    gz.y = 3 * nsys;
    gzy.y = 3 * nsys;
    // pass 3: x forward + CNV (+ inverse)
    int ncx = pow2_floor(max(1, budget / (3 * M1)));
    if (ncx > H) ncx = H;
    size_t shx = 2 * (size_t)3 * M1 * ncx * sizeof(C2<T>);
    CnvArgs ca;
    for (int d = 0; d < 3; ++d) ca.twopi_over_L[d] = 2.0 * M_PI / g.L[d];
    ca.inv4xi2 = 1.0 / (4.0 * pl.xi * pl.xi);
    ca.eightpi = 8.0 * M_PI;
    ca.E0 = pl.d_cnv[0];
    ca.E1 = pl.d_cnv[1];
    ca.E2 = pl.d_cnv[2];
    if (st) {
        // forward x transforms of the 9 components, three at a time; then CNV 9 -> 3 and the
        // inverse x transform
        for (int grp = 0; grp < 3; ++grp)
            hipLaunchKernelGGL((k_fft_x_cnv<T>), dim3(M2 * (H / ncx)), dim3(256), shx, s,
                               grid + (int64_t)3 * grp * nc, nc, M1, M2, H, ncx, 0, 0, tw0, ca);
        if (cnv && inverse_too)
            hipLaunchKernelGGL((k_cnv_st_x<T>), dim3(M2 * (H / ncx)), dim3(256), shx, s, grid, nc, M1, M2, H, ncx,
                               tw0, ca);
    } else if (cnv && inverse_too && M1 >= 4) {
        // one LDS buffer: twice the columns per block
        int lgM1 = 0, lgnc = 0;
        while ((1 << lgM1) < M1) ++lgM1;
        int nci = pow2_floor(max(1, 2 * budget / (3 * M1)));
        if (nci > H) nci = H;
        while ((1 << lgnc) < nci) ++lgnc;
        const size_t shi = (size_t)3 * M1 * nci * sizeof(C2<T>);
        hipLaunchKernelGGL((k_fft_x_cnv_ip<T>), dim3(M2 * (H / nci), nsys), dim3(256), shi, s, grid, nc, M1, lgM1,
                           M2, H, nci, lgnc, tw0, ca);
    } else {
        hipLaunchKernelGGL((k_fft_x_cnv<T>), dim3(M2 * (H / ncx), nsys), dim3(256), shx, s, grid, nc, M1, M2, H,
                           ncx, cnv ? 1 : 0, inverse_too ? 1 : 0, tw0, ca);
    }
    if (inverse_too && fused) {
        hipLaunchKernelGGL((k_fft_zy<T>), gzy, dim3(1024), shzy, s, grid, nc, M2, lgM2, H, lgH, +1, twh, twf, tw1);
    } else if (inverse_too) {
        hipLaunchKernelGGL((k_fft_y<T>), gy, dim3(256), shy, s, grid, nc, M2, H, ncy, +1, tw1);
        hipLaunchKernelGGL((k_fft_z<T>), gz, dim3(256), shz, s, grid, nc, nlines, H, ncz, +1, twh, twf);
    }
    return hipGetLastError();
}

}  // namespace

hipError_t launch_fgc(const Plan& pl, const Work& w, hipStream_t s, bool inverse_too, bool cnv, bool st, int nsys)
{
    if (pl.grid64) return launch_fgc_t<double>(pl, w, s, inverse_too, cnv, st, nsys);
    return launch_fgc_t<float>(pl, w, s, inverse_too, cnv, st, nsys);
}

}  // namespace ewald
