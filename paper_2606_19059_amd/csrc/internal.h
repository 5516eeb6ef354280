// Internal declarations of the MI355X spectral Ewald library (not installed).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ewald.h"  // include/ (on the compiler include path)

namespace ewald {

constexpr int kNumStages = 6;  // bin/sort, P2P, P2G, FFT+CNV+IFFT, G2P+sum, total
constexpr int kWave = 64;      // CDNA wavefront width

// Grid / cell geometry, passed by value to kernels.
struct Geometry {
    double L[3];      // box sides
    double h[3];      // grid spacing L/M
    int M[3];         // grid points per dimension (powers of two)
    int B;            // P2P tile edge in grid cells (power of two)
    int log2B;
    int NT[3];        // tiles per dimension (M / B)
    int S[3];         // P2P stencil half-width in tiles
    int ncells;       // M1 M2 M3 (sort bins = grid cells) of one system
    int ntiles;       // NT1 NT2 NT3 of one system
    int nsys;         // independent systems evaluated together (1, or a batch's count): system r
                      // owns cells [r ncells, (r + 1) ncells) of the cell list, tiles
                      // [r ntiles, (r + 1) ntiles) and grid components [3 r, 3 r + 3)
};

// Particle ranges of the systems of one evaluation: system r owns particles [off[r], off[r + 1])
// of the input arrays (and, after the sort, of the sorted order).  Passed by value to kernels.
constexpr int kMaxBatch = EWALD_MAX_BATCH;
struct Batch {
    int count;
    int off[kMaxBatch + 1];
};

// system of particle (or sorted slot) i: the last r with off[r] <= i
__host__ __device__ inline int batch_system(const Batch& b, int i)
{
    int lo = 0, hi = b.count;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (b.off[mid] <= i) lo = mid; else hi = mid;
    }
    return lo;
}

// Interleave the bits of x (odd positions) and y (even positions), 4 bits each.
__host__ __device__ inline int morton2(int x, int y)
{
    int k = 0;
#pragma unroll
    for (int i = 0; i < 4; ++i) k |= (((x >> i) & 1) << (2 * i + 1)) | (((y >> i) & 1) << (2 * i));
    return k;
}

// Sort key of grid cell (cx, cy, cz): tile-major, so that each P2P tile is one contiguous
// range of sorted particles; inside a tile the (x, y) columns follow a Morton curve (so a
// run of consecutive particles, a P2P target chunk, fills a compact sub-block) and z is
// fastest (so the cells of one column segment are consecutive keys, which P2G uses).
__host__ __device__ inline int cell_key(int cx, int cy, int cz, const Geometry& g)
{
    const int b = g.log2B, m = g.B - 1;
    const int tile = ((cx >> b) * g.NT[1] + (cy >> b)) * g.NT[2] + (cz >> b);
    return (tile << (3 * b)) | (morton2(cx & m, cy & m) << b) | (cz & m);
}

// LDS hand-off between the lanes of one wavefront (for data private to one wave of a block,
// which the other waves need not wait for): orders the wave's LDS accesses before and after it
__device__ inline void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// One LDS value per instruction: the compiler pairs two loads of one base address into a
// ds_read2_b64 / ds_read2st64_b64, which occupies the LDS pipeline for 8 cycles per wave on
// gfx950, twice as long as two ds_read_b64 (2 cycles each).  A volatile access is never
// paired; the address-space cast keeps it a plain LDS load (r must be an element of a
// __shared__ array).
template <typename T>
__device__ inline T ld1(const T& r)
{
    typedef __attribute__((address_space(3))) T LdsT;
    return *(const volatile LdsT*)(const LdsT*)&r;
}

// Block index -> work item such that each XCD (blocks are dealt to the 8 XCDs round
// robin) processes one contiguous range of items: neighbouring (cell-sorted) items then
// share that XCD's L2.  A bijection on [0, nb).
__device__ inline int xcd_remap(int b, int nb)
{
    const int x = b & 7, l = b >> 3, q = nb >> 3, r = nb & 7;
    return (x < r ? x * (q + 1) : r * (q + 1) + (x - r) * q) + l;
}

// Sorted particle record, FP64 mode: wrapped position (in [0, L)) and its grid cell, so
// that every kernel uses the cell assignment of the sort (the fraction is x/h - c); 64 bytes.
struct alignas(64) Rec64 {
    double x[3];
    int c[3];
    int orig;  // original particle index
    double f[3];
};
static_assert(sizeof(Rec64) == 64, "Rec64 layout");

struct Plan {
    ewald_params p;        // resolved parameters
    ewald_plan_info info;  // what get_info returns
    Geometry g;
    int P;                 // window support
    bool window_kb;        // Kaiser-Bessel window (else Gaussian)
    double m;              // Gaussian shape m, or Kaiser-Bessel beta / P
    double beta;           // Gaussian: 2 m^2 / P^2 (w0 = exp(-beta u^2), u = distance / h); KB: beta
    double xi, rc;
    int mode;              // EWALD_FP64 or EWALD_FP32_BULK
    bool grid64;           // grid, FFT, CNV, IFFT in FP64 (always in FP64 mode)
    bool fp64acc;          // FP32 bulk: FP64 near-field accumulation
    bool deterministic;    // bitwise reproducible P2P (one-sided pair evaluation)
    bool stresslet;        // workspace sized for combined Stokeslet + stresslet sources
    bool timers;
    bool check_inputs;     // count non-finite inputs before evaluating (debug mode)
    int device;
    // device tables owned by the plan
    void* d_tables;        // one allocation holding everything below
    double* d_cnv[3];      // per-axis CNV factors E_d[k] (FP64), lengths M1, M2, M3/2
    void* d_tw64;          // twiddles e^{-2 pi i j / n} (double2), per FFT length
    void* d_tw32;          // same in float2
    double* d_kb64;        // Kaiser-Bessel weight polynomials, P x (kKbDeg + 1) (KB plans only)
    float* d_kb32;
    int tw_off[4];         // element offsets: axis0 (M1), axis1 (M2), half z (M3/2), full z (M3)
    hipEvent_t ev[kNumStages + 1];
    float stage_ms[kNumStages];
    bool ev_valid;
    bool ev_overlapped;    // the timed evaluation ran P2P on a second stream
};

// Device pointers carved out of the caller's workspace.
struct Work {
    int* key;        // [n]   sort key of each input particle; after the sort, its sorted position
    int* perm;       // [n]   sorted slot -> original index (also carried in records)
    int* count;      // [ncells]   histogram, then scatter cursor
    int* start;      // [ncells+1] exclusive scan of count
    int* chunk_off;  // [ntiles+1] P2P wave work-list offsets
    int* part;       // scan partials
    int* cell_lists; // [cell_list_elems(n)] cells too large for a one-thread sort of their order
    void* rec;       // [n] Rec64, sorted order
    double* u_near;  // [3][n] near field, sorted order
    double* srec;    // [n][6] symmetric stresslet tensors (xx, yy, zz, xy, xz, yz), sorted order
                     // (stresslet plans only)
    void* grid;      // 3 (9 for stresslet plans) x ncells reals (double or float), then the
                     // in-place half spectrum
    double* p2g_halo;  // P2G's partial sums next to its x-segment boundaries (p2g_halo_elems)
    int64_t bytes;
};

// workspace layout for n particles in `nsys` systems (a batch) of this plan
int64_t layout_work(const Plan& pl, int64_t n, char* base, Work* w, int nsys = 1);
// doubles of P2G's segment-boundary buffer for this plan (0: the sweep uses no halo)
int64_t p2g_halo_elems(const Plan& pl);
// length of the x-segments of P2G's sweep (a power of two dividing M[0])
int p2g_segment_length(const int M[3], int P);

// Launchers (all enqueue on `s`, return hipSuccess or the launch error).
hipError_t launch_sort(const Plan& pl, const Work& w, int n, const double* x, const double* f,
                       const Batch& b, hipStream_t s);
// `st`: this evaluation has stresslet sources (w.srec filled, 9 grid components)
hipError_t launch_gather_st(const Plan& pl, const Work& w, int n, const double* q, const double* nrm,
                            hipStream_t s);
hipError_t launch_p2p(const Plan& pl, const Work& w, int n, hipStream_t s, bool st, int nsys = 1);
// exact number of ordered pairs (i != j, all images) with 0 < |r| < r_c, written to *count
hipError_t launch_count_pairs(const Plan& pl, const Work& w, int n, unsigned long long* count, hipStream_t s,
                              int nsys = 1);
hipError_t launch_p2g(const Plan& pl, const Work& w, int n, hipStream_t s, bool st, int nsys = 1);
hipError_t launch_fgc(const Plan& pl, const Work& w, hipStream_t s, bool inverse_too, bool cnv, bool st,
                      int nsys = 1);
hipError_t launch_g2p(const Plan& pl, const Work& w, int n, const double* f, double* u,
                      double* u_near_out, double* u_far_out, const Batch& b, hipStream_t s);
hipError_t launch_fill_i32(int* p, int64_t count, int value, hipStream_t s);
// *out (= 0 first when `reset`) += number of non-finite values among a[0..count)
hipError_t launch_count_nonfinite(const double* a, int64_t count, int* out, hipStream_t s, bool reset = true);

// Exclusive scan of in[0..count) into out[0..count] (out[count] = total); `part`
// needs scan_part_elems(count) ints.
hipError_t launch_exclusive_scan(const int* in, int* out, int count, int* part, hipStream_t s);
int scan_part_elems(int count);
// ints of the sort's lists of large cells for n particles
int64_t cell_list_elems(int64_t n);

}  // namespace ewald
