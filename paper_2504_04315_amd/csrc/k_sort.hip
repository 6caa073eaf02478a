// Spatial ordering of a training batch: a counting sort of the vertices by
// the Morton code of their cell in a 64^3 grid over the unit cube.  The
// gradient is a sum over vertices, so the order changes nothing but the
// rounding order of its FP32 sums; it makes neighbouring lanes of the grid
// scatter hit the same cache lines (whose number sets the atomic throughput)
// and the grid gathers hit the same L2 lines.
#include "device_math.h"

namespace npm {

constexpr int kSortBits = 6;                       // per axis
constexpr int kSortCells = 1 << (3 * kSortBits);  // 262,144

__device__ __forceinline__ uint32_t spread3(uint32_t x)
{
    // bit i of x moves to bit 3i (x < 2^10)
    x &= 0x3ffu;
    x = (x | (x << 16)) & 0x030000ffu;
    x = (x | (x << 8)) & 0x0300f00fu;
    x = (x | (x << 4)) & 0x030c30c3u;
    x = (x | (x << 2)) & 0x09249249u;
    return x;
}

__device__ __forceinline__ uint32_t sort_cell(const float *__restrict__ pos, int64_t n, int64_t v)
{
    const float s = (float)(1 << kSortBits);
    uint32_t c[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const float x = fminf(fmaxf(pos[d * n + v], 0.0f), 1.0f) * s;
        c[d] = (uint32_t)min((int)x, (1 << kSortBits) - 1);
    }
    return spread3(c[0]) | (spread3(c[1]) << 1) | (spread3(c[2]) << 2);
}

__global__ void k_sort_zero(uint32_t *__restrict__ cnt)
{
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < kSortCells; i += gridDim.x * blockDim.x)
        cnt[i] = 0u;
}

// Counts the vertices of each cell; the count a vertex's increment returns
// is its rank within the cell, kept in rank[v] so that placement needs no
// second atomic.
__global__ void k_sort_count(const float *__restrict__ pos, int64_t n, uint32_t *__restrict__ cnt,
                             uint32_t *__restrict__ rank)
{
    const int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (v < n) rank[v] = atomicAdd(cnt + sort_cell(pos, n, v), 1u);
}

// Exclusive prefix sum of the 2^18 counts in two coalesced passes: each block
// of 1024 threads scans its 1024 counts in LDS and records their total; then
// each block adds the totals of the blocks before it.
constexpr int kScanBlocks = kSortCells / 1024;     // 256
static_assert(kSortCells + kScanBlocks == (int)kSortCellWords, "cell scratch layout");

__device__ __forceinline__ uint32_t block_inclusive_scan(uint32_t v, uint32_t *part)
{
    const int t = threadIdx.x;
    part[t] = v;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        const uint32_t add = t >= off ? part[t - off] : 0u;
        __syncthreads();
        part[t] += add;
        __syncthreads();
    }
    return part[t];
}

__global__ __launch_bounds__(1024) void k_sort_scan_local(uint32_t *__restrict__ cnt,
                                                          uint32_t *__restrict__ sums)
{
    __shared__ uint32_t part[1024];
    const int i = blockIdx.x * 1024 + threadIdx.x;
    const uint32_t v = cnt[i];
    const uint32_t incl = block_inclusive_scan(v, part);
    cnt[i] = incl - v;
    if (threadIdx.x == 1023) sums[blockIdx.x] = incl;
}

__global__ __launch_bounds__(1024) void k_sort_scan_add(uint32_t *__restrict__ cnt,
                                                        const uint32_t *__restrict__ sums)
{
    __shared__ uint32_t part[kScanBlocks];
    const int t = threadIdx.x;
    if (t < kScanBlocks) part[t] = t < (int)blockIdx.x ? sums[t] : 0u;
    __syncthreads();
    for (int w = kScanBlocks / 2; w > 0; w >>= 1) {
        if (t < w) part[t] += part[t + w];
        __syncthreads();
    }
    cnt[blockIdx.x * 1024 + t] += part[0];
}

// Places vertex v at its slot, the cell's offset plus its rank (read from
// inv[v], then replaced by the slot): perm[slot] = v, inv[v] = slot, and
// its inputs as one record rec[slot] = (pos, dir, radiance, pdf), with zeros
// for the arrays the call does not have; with the NPM-product inputs aux
// [7][n] the record is 16 floats, followed by (omega_o, normal, roughness, 0).
__global__ void k_sort_place(const float *__restrict__ pos, const float *__restrict__ aux,
                             const float *__restrict__ dir, const float *__restrict__ rad,
                             const float *__restrict__ spdf, int64_t n, uint32_t *__restrict__ off,
                             uint32_t *__restrict__ perm, uint32_t *__restrict__ inv,
                             float *__restrict__ rec)
{
    const int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (v >= n) return;
    const uint32_t slot = off[sort_cell(pos, n, v)] + inv[v];
    perm[slot] = (uint32_t)v;
    inv[v] = slot;
    if (rec) {
        f32x4 a, b;
        a[0] = pos[v]; a[1] = pos[n + v]; a[2] = pos[2 * n + v];
        a[3] = dir ? dir[v] : 0.0f;
        b[0] = dir ? dir[n + v] : 0.0f; b[1] = dir ? dir[2 * n + v] : 0.0f;
        b[2] = rad ? rad[v] : 0.0f; b[3] = spdf ? spdf[v] : 0.0f;
        f32x4 *r = reinterpret_cast<f32x4 *>(rec + (size_t)slot * (aux ? 16 : 8));
        r[0] = a;
        r[1] = b;
        if (aux) {
            f32x4 c, d;
            c[0] = aux[v]; c[1] = aux[n + v]; c[2] = aux[2 * n + v]; c[3] = aux[3 * n + v];
            d[0] = aux[4 * n + v]; d[1] = aux[5 * n + v]; d[2] = aux[6 * n + v]; d[3] = 0.0f;
            r[2] = c;
            r[3] = d;
        }
    }
}

// cells: kSortCells counters followed by kScanBlocks block totals; inv
// receives the inverse of perm, rec (optional) the inputs in visiting order,
// 8 floats per slot (16 with aux)
hipError_t spatial_order(npm_ctx *ctx, int64_t n, const float *pos, const float *aux,
                         const float *dir, const float *rad, const float *spdf, uint32_t *perm,
                         uint32_t *inv, float *rec, uint32_t *cells, hipStream_t s)
{
    int tok;
    timed_begin(ctx, "spatial_sort", s, &tok);
    const unsigned blocks = (unsigned)((n + 255) / 256);
    hipLaunchKernelGGL(k_sort_zero, dim3(256), dim3(256), 0, s, cells);
    hipLaunchKernelGGL(k_sort_count, dim3(blocks), dim3(256), 0, s, pos, n, cells, inv);
    hipLaunchKernelGGL(k_sort_scan_local, dim3(kScanBlocks), dim3(1024), 0, s, cells,
                       cells + kSortCells);
    hipLaunchKernelGGL(k_sort_scan_add, dim3(kScanBlocks), dim3(1024), 0, s, cells,
                       cells + kSortCells);
    hipLaunchKernelGGL(k_sort_place, dim3(blocks), dim3(256), 0, s, pos, aux, dir, rad, spdf, n,
                       cells, perm, inv, rec);
    timed_end(ctx, tok, s);
    return hipGetLastError();
}

}  // namespace npm
