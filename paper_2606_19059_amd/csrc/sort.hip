// Bin / sort stage: counting sort of the particles by grid cell (tile-major key), the
// cell list every other kernel reads (Sec. 3: cell lists of the near and far field; here
// one compact CSR list keyed by grid cell serves both, since P2P cells are unions of grid
// cells).  Integer atomics touch only the per-cell counters; the order inside a cell is
// made deterministic by sorting it by original index.
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

__global__ void k_bin(int n, const double* __restrict__ x, Geometry g, int* __restrict__ key,
                      int* __restrict__ count)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int c[3];
    double t, wx;
#pragma unroll
    for (int d = 0; d < 3; ++d) cell_of(x[(int64_t)d * n + i], g.L[d], g.h[d], g.M[d], c[d], t, wx);
    const int k = cell_key(c[0], c[1], c[2], g);
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

// Order each cell's particles by original index (insertion sort; cells of the sizes
// seen here hold a few to a few hundred particles).  Cells above `cap` keep the
// scatter order: still correct, only not bitwise reproducible.
__global__ void k_cell_order(int ncells, const int* __restrict__ start, int* __restrict__ perm, int cap)
{
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= ncells) return;
    const int a = start[c], b = start[c + 1];
    if (b - a < 2 || b - a > cap) return;
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

__global__ void k_gather64(int n, const double* __restrict__ x, const double* __restrict__ f,
                           const int* __restrict__ perm, Geometry g, Rec64* __restrict__ rec)
{
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    const int i = perm[s];
    Rec64 r;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        double t;
        cell_of(x[(int64_t)d * n + i], g.L[d], g.h[d], g.M[d], r.c[d], t, r.x[d]);
        r.f[d] = f[(int64_t)d * n + i];
    }
    r.orig = i;
    rec[s] = r;
}

// Symmetric part of each stresslet source tensor q n^T, in sorted order: the stresslet
// kernel is symmetric in all three indices, so only (q n^T + n q^T)/2 contributes.
__global__ void k_gather_st(int n, const double* __restrict__ q, const double* __restrict__ nrm,
                            const int* __restrict__ perm, double* __restrict__ srec)
{
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    const int i = perm[s];
    const double q0 = q[i], q1 = q[(int64_t)n + i], q2 = q[2 * (int64_t)n + i];
    const double n0 = nrm[i], n1 = nrm[(int64_t)n + i], n2 = nrm[2 * (int64_t)n + i];
    double* o = srec + 6 * (int64_t)s;
    o[0] = q0 * n0;
    o[1] = q1 * n1;
    o[2] = q2 * n2;
    o[3] = 0.5 * (q0 * n1 + q1 * n0);
    o[4] = 0.5 * (q0 * n2 + q2 * n0);
    o[5] = 0.5 * (q1 * n2 + q2 * n1);
}

// Number of 64-target waves per P2P tile.
__global__ void k_tile_chunks(Geometry g, const int* __restrict__ start, int* __restrict__ chunks)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= g.ntiles) return;
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

hipError_t launch_fill_i32(int* p, int64_t count, int value, hipStream_t s)
{
    if (count <= 0) return hipSuccess;
    int blocks = (int)((count + 255) / 256);
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(k_fill_i32, dim3(blocks), dim3(256), 0, s, p, count, value);
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
                       hipStream_t s)
{
    const Geometry& g = pl.g;
    hipError_t e = launch_fill_i32(w.count, g.ncells, 0, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_bin, dim3(blocks_for(n, 256)), dim3(256), 0, s, n, x, g, w.key, w.count);
    e = launch_exclusive_scan(w.count, w.start, g.ncells, w.part, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_copy_i32, dim3(blocks_for(g.ncells, 256)), dim3(256), 0, s, w.start, w.count,
                       g.ncells);
    hipLaunchKernelGGL(k_scatter, dim3(blocks_for(n, 256)), dim3(256), 0, s, n, w.key, w.count, w.perm);
    hipLaunchKernelGGL(k_cell_order, dim3(blocks_for(g.ncells, 256)), dim3(256), 0, s, g.ncells, w.start,
                       w.perm, 512);
    hipLaunchKernelGGL(k_gather64, dim3(blocks_for(n, 256)), dim3(256), 0, s, n, x, f, w.perm, g,
                       (Rec64*)w.rec);
    // P2P work list: waves per tile, then their offsets
    hipLaunchKernelGGL(k_tile_chunks, dim3(blocks_for(g.ntiles, 256)), dim3(256), 0, s, g, w.start,
                       w.count);
    return launch_exclusive_scan(w.count, w.chunk_off, g.ntiles, w.part, s);
}

hipError_t launch_gather_st(const Plan& pl, const Work& w, int n, const double* q, const double* nrm,
                            hipStream_t s)
{
    (void)pl;
    hipLaunchKernelGGL(k_gather_st, dim3(blocks_for(n, 256)), dim3(256), 0, s, n, q, nrm, w.perm, w.srec);
    return hipGetLastError();
}

}  // namespace ewald
