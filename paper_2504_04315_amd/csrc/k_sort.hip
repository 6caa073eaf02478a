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

__global__ void k_sort_count(const float *__restrict__ pos, int64_t n, uint32_t *__restrict__ cnt)
{
    const int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (v < n) atomicAdd(cnt + sort_cell(pos, n, v), 1u);
}

// Exclusive prefix sum of the 2^18 counts in one block of 1024 threads.
__global__ __launch_bounds__(1024) void k_sort_scan(uint32_t *__restrict__ cnt)
{
    constexpr int PER = kSortCells / 1024;
    __shared__ uint32_t part[1024];
    const int t = threadIdx.x;
    uint32_t s = 0;
    for (int i = 0; i < PER; ++i) s += cnt[t * PER + i];
    part[t] = s;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        const uint32_t add = t >= off ? part[t - off] : 0u;
        __syncthreads();
        part[t] += add;
        __syncthreads();
    }
    uint32_t run = part[t] - s;                     // exclusive prefix of this chunk
    for (int i = 0; i < PER; ++i) {
        const uint32_t c = cnt[t * PER + i];
        cnt[t * PER + i] = run;
        run += c;
    }
}

__global__ void k_sort_place(const float *__restrict__ pos, int64_t n, uint32_t *__restrict__ off,
                             uint32_t *__restrict__ perm)
{
    const int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (v < n) perm[atomicAdd(off + sort_cell(pos, n, v), 1u)] = (uint32_t)v;
}

hipError_t spatial_order(npm_ctx *ctx, int64_t n, const float *pos, uint32_t *perm,
                         uint32_t *cells, hipStream_t s)
{
    int tok;
    timed_begin(ctx, "spatial_sort", s, &tok);
    const unsigned blocks = (unsigned)((n + 255) / 256);
    hipLaunchKernelGGL(k_sort_zero, dim3(256), dim3(256), 0, s, cells);
    hipLaunchKernelGGL(k_sort_count, dim3(blocks), dim3(256), 0, s, pos, n, cells);
    hipLaunchKernelGGL(k_sort_scan, dim3(1), dim3(1024), 0, s, cells);
    hipLaunchKernelGGL(k_sort_place, dim3(blocks), dim3(256), 0, s, pos, n, cells, perm);
    timed_end(ctx, tok, s);
    return hipGetLastError();
}

}  // namespace npm
