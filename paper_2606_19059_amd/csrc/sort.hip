// Bin / sort stage: counting sort of the particles by grid cell (tile-major key), the
// cell list every other kernel reads (Sec. 3: cell lists of the near and far field; here
// one compact CSR list keyed by grid cell serves both, since P2P cells are unions of grid
// cells).  Integer atomics touch only the per-cell counters; the order inside a cell is
// made deterministic by sorting it by original index.
#include <algorithm>
#include <climits>

#include "internal.h"

namespace ewald {

namespace {

constexpr int kScanThreads = 256;
constexpr int kScanItems = 16;
constexpr int kScanChunk = kScanThreads * kScanItems;  // elements per block

__global__ void k_fill_i32(int* __restrict__ p, int64_t count, int value)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t k = i; k < count; k += stride) p[k] = value;
}

// Periodic wrap into [0, L) and grid cell / fraction along one axis: c = floor(y/h),
// t = y/h - c.  The same function is used wherever a particle's cell is needed.
__device__ inline void cell_of(double x, double L, double h, int M, int& c, double& t, double& w)
{
    w = x - L * floor(x / L);
    if (w >= L) w -= L;
    if (w < 0.0) w = 0.0;
    const double s = w / h;
    int ci = (int)floor(s);
    if (ci >= M) ci = M - 1;
    if (ci < 0) ci = 0;
    c = ci;
    t = s - (double)ci;
}

// key = system * ncells + cell key: the systems of a batch occupy consecutive key ranges
__global__ void k_bin(int n, const double* __restrict__ x, Geometry g, int* __restrict__ key,
                      int* __restrict__ count, Batch b)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int c[3];
    double t, wx;
#pragma unroll
    for (int d = 0; d < 3; ++d) cell_of(x[(int64_t)d * n + i], g.L[d], g.h[d], g.M[d], c[d], t, wx);
    const int k = batch_system(b, i) * g.ncells + cell_key(c[0], c[1], c[2], g);
    key[i] = k;
    atomicAdd(&count[k], 1);
}

__global__ void k_copy_i32(const int* __restrict__ a, int* __restrict__ b, int count)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) b[i] = a[i];
}

__global__ void k_scatter(int n, const int* __restrict__ key, int* __restrict__ cursor,
                          int* __restrict__ perm)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int slot = atomicAdd(&cursor[key[i]], 1);
    perm[slot] = i;
}

// Order each cell's particles by original index, so that the sorted order (and every sum
// taken in it) does not depend on the order of the scatter's atomics.  Cells of up to
// kCellSerial particles are sorted here by one thread (insertion sort); larger ones are
// appended to one of two lists (`lists[0]`, `lists[1]` hold their lengths) and sorted by
// k_sort_mid_cells (one wavefront per cell, up to kCellMid particles) or k_sort_big_cells
// (one block per cell, any size).  The lists' order varies, but each cell's result does not.
constexpr int kCellSerial = 16;
constexpr int kCellMid = 256;
constexpr int kBigThreads = 256;
constexpr int kBigRun = 8192;  // ints sorted in LDS at once (32 KB)

__host__ __device__ inline int64_t mid_list_cap(int64_t n) { return n / (kCellSerial + 1) + 1; }
__host__ __device__ inline int64_t big_list_cap(int64_t n) { return n / (kCellMid + 1) + 1; }

__global__ void k_cell_order(int ncells, const int* __restrict__ start, int* __restrict__ perm,
                             int* __restrict__ lists, int64_t mid_cap)
{
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= ncells) return;
    const int a = start[c], b = start[c + 1];
    if (b - a < 2) return;
    if (b - a > kCellMid) {
        const int k = atomicAdd(&lists[1], 1);
        lists[2 + mid_cap + k] = c;
        return;
    }
    if (b - a > kCellSerial) {
        const int k = atomicAdd(&lists[0], 1);
        lists[2 + k] = c;
        return;
    }
    for (int i = a + 1; i < b; ++i) {
        const int v = perm[i];
        int j = i - 1;
        while (j >= a && perm[j] > v) {
            perm[j + 1] = perm[j];
            --j;
        }
        perm[j + 1] = v;
    }
}

// One wavefront per listed cell (kCellSerial < size <= kCellMid): every lane holds up to
// four of the cell's (distinct) indices, counts how many of the cell's indices are smaller
// (a broadcast read of each from LDS) and writes its index at that rank.
__global__ void __launch_bounds__(256) k_sort_mid_cells(const int* __restrict__ start, int* __restrict__ perm,
                                                        const int* __restrict__ lists)
{
    constexpr int kPer = kCellMid / kWave;
    __shared__ int sh[256 / kWave][kCellMid];
    const int lane = threadIdx.x & (kWave - 1), wv = threadIdx.x / kWave;
    int* s = sh[wv];
    const int nmid = lists[0];
    const int waves = gridDim.x * (blockDim.x / kWave);
    for (int q = blockIdx.x * (blockDim.x / kWave) + wv; q < nmid; q += waves) {
        const int c = lists[2 + q];
        const int a = start[c], m = start[c + 1] - a;
        int v[kPer];
#pragma unroll
        for (int k = 0; k < kPer; ++k) {
            const int i = lane + k * kWave;
            v[k] = i < m ? perm[a + i] : 0;
            if (i < m) s[i] = v[k];
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        int rank[kPer];
#pragma unroll
        for (int k = 0; k < kPer; ++k) rank[k] = 0;
        for (int t = 0; t < m; ++t) {
            const int o = s[t];
#pragma unroll
            for (int k = 0; k < kPer; ++k) rank[k] += (o < v[k]) ? 1 : 0;
        }
#pragma unroll
        for (int k = 0; k < kPer; ++k)
            if (lane + k * kWave < m) perm[a + rank[k]] = v[k];
        // the next cell overwrites this wave's LDS row
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
}

// number of entries of the ascending, distinct a[0..len) below v
__device__ inline int count_below(const int* __restrict__ a, int len, int v)
{
    int lo = 0, hi = len;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (a[mid] < v) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

// One block per listed cell (size > kCellMid): runs of kBigRun indices are sorted in LDS
// (bitonic network, padded to a power of two), then merged pairwise, each index placed at
// its rank in the merged run (its offset in its own run plus the count of smaller indices
// in the other, by binary search), ping-ponging between the cell's range of `perm` and
// the same range of `scratch`.
__global__ void __launch_bounds__(kBigThreads) k_sort_big_cells(const int* __restrict__ start, int* __restrict__ perm,
                                                                int* __restrict__ scratch, const int* __restrict__ lists,
                                                                int64_t mid_cap)
{
    __shared__ int s[kBigRun];
    const int nbig = lists[1];
    const int tid = threadIdx.x;
    for (int q = blockIdx.x; q < nbig; q += gridDim.x) {
        const int c = lists[2 + mid_cap + q];
        const int a = start[c], m = start[c + 1] - a;
        int* v = perm + a;
        for (int r0 = 0; r0 < m; r0 += kBigRun) {
            const int len = min(kBigRun, m - r0);
            int p2 = 1;
            while (p2 < len) p2 <<= 1;
            for (int i = tid; i < p2; i += kBigThreads) s[i] = i < len ? v[r0 + i] : INT_MAX;
            __syncthreads();
            for (int k = 2; k <= p2; k <<= 1)
                for (int j = k >> 1; j > 0; j >>= 1) {
                    for (int i = tid; i < p2; i += kBigThreads) {
                        const int l = i ^ j;
                        if (l > i) {
                            const int x = s[i], y = s[l];
                            if ((x > y) == ((i & k) == 0)) {
                                s[i] = y;
                                s[l] = x;
                            }
                        }
                    }
                    __syncthreads();
                }
            for (int i = tid; i < len; i += kBigThreads) v[r0 + i] = s[i];
            __syncthreads();
        }
        int* src = v;
        int* dst = scratch + a;
        for (int w = kBigRun; w < m; w *= 2) {
            for (int i = tid; i < m; i += kBigThreads) {
                const int lo = (i / (2 * w)) * (2 * w);
                const int mid = min(lo + w, m), hi = min(lo + 2 * w, m);
                const int val = src[i];
                const int pos = (i < mid) ? (i - lo) + count_below(src + mid, hi - mid, val)
                                          : (i - mid) + count_below(src + lo, mid - lo, val);
                dst[lo + pos] = val;
            }
            __syncthreads();
            int* t = src;
            src = dst;
            dst = t;
        }
        if (src != v) {
            for (int i = tid; i < m; i += kBigThreads) v[i] = src[i];
        }
        __syncthreads();
    }
}

// inv[perm[s]] = s: the sorted position of each input particle.  The gathers below then read the
// caller's (3, N) arrays in their own order (coalesced) and write each whole record to its sorted
// position; gathering through perm instead reads six arrays at random positions, which costs a full
// memory segment per 8-byte value (15 times the bytes used at 1e6 uniform particles).
__global__ void k_invert(int n, const int* __restrict__ perm, int* __restrict__ inv)
{
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s < n) inv[perm[s]] = s;
}

__global__ void k_gather64(int n, const double* __restrict__ x, const double* __restrict__ f,
                           const int* __restrict__ inv, Geometry g, Rec64* __restrict__ rec)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    Rec64 r;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        double t;
        cell_of(x[(int64_t)d * n + i], g.L[d], g.h[d], g.M[d], r.c[d], t, r.x[d]);
        r.f[d] = f[(int64_t)d * n + i];
    }
    r.orig = i;
    rec[inv[i]] = r;
}

// Symmetric part of each stresslet source tensor q n^T, in sorted order: the stresslet
// kernel is symmetric in all three indices, so only (q n^T + n q^T)/2 contributes.
__global__ void k_gather_st(int n, const double* __restrict__ q, const double* __restrict__ nrm,
                            const int* __restrict__ inv, double* __restrict__ srec)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double q0 = q[i], q1 = q[(int64_t)n + i], q2 = q[2 * (int64_t)n + i];
    const double n0 = nrm[i], n1 = nrm[(int64_t)n + i], n2 = nrm[2 * (int64_t)n + i];
    double* o = srec + 6 * (int64_t)inv[i];
    o[0] = q0 * n0;
    o[1] = q1 * n1;
    o[2] = q2 * n2;
    o[3] = 0.5 * (q0 * n1 + q1 * n0);
    o[4] = 0.5 * (q0 * n2 + q2 * n0);
    o[5] = 0.5 * (q1 * n2 + q2 * n1);
}

// Number of 64-target waves per P2P tile (the tiles of all systems).
__global__ void k_tile_chunks(Geometry g, const int* __restrict__ start, int* __restrict__ chunks)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= g.ntiles * g.nsys) return;
    const int per = 1 << (3 * g.log2B);
    const int cnt = start[(t + 1) * per] - start[t * per];
    chunks[t] = (cnt + kWave - 1) / kWave;
}

// ---- exclusive scan (three phases: block sums, scan of sums, block scans) ----

__device__ inline int block_exclusive_scan(int v, int* sh, int& total)
{
    // inclusive scan within each wave
    const int lane = threadIdx.x & (kWave - 1);
    const int wid = threadIdx.x / kWave;
    int inc = v;
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
        const int y = __shfl_up(inc, o, kWave);
        if (lane >= o) inc += y;
    }
    if (lane == kWave - 1) sh[wid] = inc;
    __syncthreads();
    const int nw = blockDim.x / kWave;
    int off = 0, tot = 0;
    for (int k = 0; k < nw; ++k) {
        const int s = sh[k];
        if (k < wid) off += s;
        tot += s;
    }
    __syncthreads();
    total = tot;
    return off + inc - v;
}

__global__ void k_scan_reduce(const int* __restrict__ in, int count, int* __restrict__ part)
{
    __shared__ int sh[kScanThreads / kWave];
    const int base = blockIdx.x * kScanChunk;
    int s = 0;
    for (int k = 0; k < kScanItems; ++k) {
        const int i = base + k * kScanThreads + threadIdx.x;
        if (i < count) s += in[i];
    }
    int total;
    block_exclusive_scan(s, sh, total);
    if (threadIdx.x == 0) part[blockIdx.x] = total;
}

// Single block: exclusive scan of part[0..nb) in place; part[nb] = grand total.
__global__ void k_scan_parts(int* __restrict__ part, int nb)
{
    __shared__ int sh[1024 / kWave];
    const int per = (nb + blockDim.x - 1) / blockDim.x;
    const int a = threadIdx.x * per;
    int s = 0;
    for (int k = 0; k < per; ++k)
        if (a + k < nb) s += part[a + k];
    int total;
    int off = block_exclusive_scan(s, sh, total);
    for (int k = 0; k < per; ++k)
        if (a + k < nb) {
            const int v = part[a + k];
            part[a + k] = off;
            off += v;
        }
    if (threadIdx.x == 0) part[nb] = total;
}

__global__ void k_scan_final(const int* __restrict__ in, int count, const int* __restrict__ part,
                             int* __restrict__ out, int nb)
{
    __shared__ int sh[kScanThreads / kWave];
    const int base = blockIdx.x * kScanChunk + threadIdx.x * kScanItems;
    int v[kScanItems];
    int s = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        const int i = base + k;
        v[k] = (i < count) ? in[i] : 0;
        s += v[k];
    }
    int total;
    int off = block_exclusive_scan(s, sh, total) + part[blockIdx.x];
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        const int i = base + k;
        if (i < count) out[i] = off;
        off += v[k];
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) out[count] = part[nb];
}

inline int blocks_for(int64_t n, int t) { return (int)((n + t - 1) / t); }

}  // namespace

int scan_part_elems(int count) { return (count + kScanChunk - 1) / kScanChunk + 1; }

int64_t cell_list_elems(int64_t n) { return 2 + mid_list_cap(n) + big_list_cap(n); }

hipError_t launch_fill_i32(int* p, int64_t count, int value, hipStream_t s)
{
    if (count <= 0) return hipSuccess;
    int blocks = (int)((count + 255) / 256);
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(k_fill_i32, dim3(blocks), dim3(256), 0, s, p, count, value);
    return hipGetLastError();
}

namespace {

__global__ void k_count_nonfinite(const double* __restrict__ a, int64_t count, int* __restrict__ out)
{
    int bad = 0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += stride)
        bad += isfinite(a[i]) ? 0 : 1;
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) bad += __shfl_xor(bad, o, kWave);
    if ((threadIdx.x & (kWave - 1)) == 0 && bad) atomicAdd(out, bad);
}

}  // namespace

hipError_t launch_count_nonfinite(const double* a, int64_t count, int* out, hipStream_t s, bool reset)
{
    if (reset) {
        hipError_t e = launch_fill_i32(out, 1, 0, s);
        if (e != hipSuccess) return e;
    }
    const int blocks = (int)std::min<int64_t>(1024, std::max<int64_t>(1, (count + 255) / 256));
    hipLaunchKernelGGL(k_count_nonfinite, dim3(blocks), dim3(256), 0, s, a, count, out);
    return hipGetLastError();
}

hipError_t launch_exclusive_scan(const int* in, int* out, int count, int* part, hipStream_t s)
{
    const int nb = (count + kScanChunk - 1) / kScanChunk;
    hipLaunchKernelGGL(k_scan_reduce, dim3(nb), dim3(kScanThreads), 0, s, in, count, part);
    hipLaunchKernelGGL(k_scan_parts, dim3(1), dim3(1024), 0, s, part, nb);
    hipLaunchKernelGGL(k_scan_final, dim3(nb), dim3(kScanThreads), 0, s, in, count, part, out, nb);
    return hipGetLastError();
}

hipError_t launch_sort(const Plan& pl, const Work& w, int n, const double* x, const double* f,
                       const Batch& b, hipStream_t s)
{
    Geometry g = pl.g;
    g.nsys = b.count;
    const int ncells = g.ncells * g.nsys, ntiles = g.ntiles * g.nsys;  // over all systems
    hipError_t e = launch_fill_i32(w.count, ncells, 0, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_bin, dim3(blocks_for(n, 256)), dim3(256), 0, s, n, x, g, w.key, w.count, b);
    e = launch_exclusive_scan(w.count, w.start, ncells, w.part, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_copy_i32, dim3(blocks_for(ncells, 256)), dim3(256), 0, s, w.start, w.count, ncells);
    hipLaunchKernelGGL(k_scatter, dim3(blocks_for(n, 256)), dim3(256), 0, s, n, w.key, w.count, w.perm);
    // per-cell order by original index; the key array is free after the scatter and serves as
    // the merge buffer of the largest cells
    if ((e = launch_fill_i32(w.cell_lists, 2, 0, s)) != hipSuccess) return e;
    const int64_t mid_cap = mid_list_cap(n);
    hipLaunchKernelGGL(k_cell_order, dim3(blocks_for(ncells, 256)), dim3(256), 0, s, ncells, w.start,
                       w.perm, w.cell_lists, mid_cap);
    const int mid_blocks = (int)std::min<int64_t>(2048, std::max<int64_t>(1, mid_list_cap(n) / 4));
    hipLaunchKernelGGL(k_sort_mid_cells, dim3(mid_blocks), dim3(256), 0, s, w.start, w.perm, w.cell_lists);
    const int big_blocks = (int)std::min<int64_t>(512, big_list_cap(n));
    hipLaunchKernelGGL(k_sort_big_cells, dim3(big_blocks), dim3(kBigThreads), 0, s, w.start, w.perm, w.key,
                       w.cell_lists, mid_cap);
    // the key array is free again: it takes the inverse permutation (read by both gathers)
    hipLaunchKernelGGL(k_invert, dim3(blocks_for(n, 256)), dim3(256), 0, s, n, w.perm, w.key);
    hipLaunchKernelGGL(k_gather64, dim3(blocks_for(n, 256)), dim3(256), 0, s, n, x, f, w.key, g,
                       (Rec64*)w.rec);
    // P2P work list: waves per tile, then their offsets
    hipLaunchKernelGGL(k_tile_chunks, dim3(blocks_for(ntiles, 256)), dim3(256), 0, s, g, w.start,
                       w.count);
    return launch_exclusive_scan(w.count, w.chunk_off, ntiles, w.part, s);
}

hipError_t launch_gather_st(const Plan& pl, const Work& w, int n, const double* q, const double* nrm,
                            hipStream_t s)
{
    (void)pl;
    hipLaunchKernelGGL(k_gather_st, dim3(blocks_for(n, 256)), dim3(256), 0, s, n, q, nrm, w.key, w.srec);
    return hipGetLastError();
}

}  // namespace ewald
