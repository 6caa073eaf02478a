// Achievable rates of the device (include/npm_probe.h): plain kernels that
// do one thing each -- matrix instructions with no memory traffic, a read
// stream, a copy -- timed with HIP events, so that the hot-path kernels can
// be put against what this device reaches as well as against its published
// peaks.
#include <string>

#include "device_math.h"
#include "npm_probe.h"

namespace npm {

namespace {

constexpr int kPeakThreads = 256;          // four waves per block
constexpr int kPeakBlocks = 1024;          // four blocks per CU: four waves per SIMD
constexpr int kChains = 4;                 // independent accumulators per wave
constexpr int kReadBlocks = 4 * kPeakBlocks;   // the read stream's grid (the sink holds one word per block)
constexpr int kCopyBlocks = kPeakBlocks;       // the copy's grid (timed best of 1,024 / 4,096 / 16,384)

// A wave keeps kChains accumulators in flight, so that each matrix
// instruction waits on none issued just before it.  The inputs stay small
// (the sums cannot overflow in the iterations run) and the accumulators are
// kept alive by a store the value never triggers.
__global__ __launch_bounds__(kPeakThreads) void k_peak_mfma_f32(int iters, float *sink)
{
    f32x16 c[kChains];
#pragma unroll
    for (int k = 0; k < kChains; ++k)
#pragma unroll
        for (int v = 0; v < 16; ++v) c[k][v] = 0.0f;
    const float a = 1e-6f * (float)(threadIdx.x & 7), b = 1e-6f;
    for (int i = 0; i < iters; ++i)
#pragma unroll
        for (int k = 0; k < kChains; ++k) c[k] = __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, c[k], 0, 0, 0);
    float s = 0.0f;
#pragma unroll
    for (int k = 0; k < kChains; ++k) s += c[k][0] + c[k][15];
    if (s == -1.0f) sink[blockIdx.x] = s;
}

__global__ __launch_bounds__(kPeakThreads) void k_peak_mfma_bf16(int iters, float *sink)
{
    f32x16 c[kChains];
#pragma unroll
    for (int k = 0; k < kChains; ++k)
#pragma unroll
        for (int v = 0; v < 16; ++v) c[k][v] = 0.0f;
    bf16x8 a, b;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        a[e] = (__bf16)(1e-6f * (float)((threadIdx.x + e) & 7));
        b[e] = (__bf16)1e-6f;
    }
    for (int i = 0; i < iters; ++i)
#pragma unroll
        for (int k = 0; k < kChains; ++k) c[k] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c[k], 0, 0, 0);
    float s = 0.0f;
#pragma unroll
    for (int k = 0; k < kChains; ++k) s += c[k][0] + c[k][15];
    if (s == -1.0f) sink[blockIdx.x] = s;
}

// One pass over n4 16-byte words, four loads in flight per thread.
__global__ __launch_bounds__(kPeakThreads) void k_peak_read(const f32x4 *__restrict__ src, int64_t n4,
                                                            float *sink)
{
    const int64_t stride = (int64_t)gridDim.x * kPeakThreads;
    f32x4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
    int64_t i = blockIdx.x * (int64_t)kPeakThreads + threadIdx.x;
    for (; i + 3 * stride < n4; i += 4 * stride) {
        const f32x4 x0 = src[i], x1 = src[i + stride], x2 = src[i + 2 * stride], x3 = src[i + 3 * stride];
        acc += x0 + x1 + x2 + x3;
    }
    for (; i < n4; i += stride) acc += src[i];
    const float s = acc[0] + acc[1] + acc[2] + acc[3];
    if (s == -1.0f) sink[blockIdx.x] = s;
}

__global__ __launch_bounds__(kPeakThreads) void k_peak_copy(const f32x4 *__restrict__ src,
                                                            f32x4 *__restrict__ dst, int64_t n4)
{
    const int64_t stride = (int64_t)gridDim.x * kPeakThreads;
    for (int64_t i = blockIdx.x * (int64_t)kPeakThreads + threadIdx.x; i < n4; i += stride)
        dst[i] = src[i];
}

}  // namespace

}  // namespace npm

using namespace npm;

extern "C" npm_status npm_measure_peaks(double out[4], int32_t reps)
{
    auto fail = [](npm_status st, const std::string &m) {
        set_error(m.c_str());
        return st;
    };
    if (!out || reps < 1) return fail(NPM_ERR_INVALID_ARG, "npm_measure_peaks: null out or reps < 1");
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0)
        return fail(NPM_ERR_NO_DEVICE, "no HIP device");
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess ||
        std::string(prop.gcnArchName).compare(0, 6, "gfx950") != 0)
        return fail(NPM_ERR_NO_DEVICE, "no gfx950 device");

    const int64_t read_bytes = (int64_t)2 << 30, copy_bytes = (int64_t)1 << 30;
    char *buf = nullptr, *dst = nullptr;
    float *sink = nullptr;
    hipStream_t s = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = hipMalloc((void **)&buf, (size_t)read_bytes);
    if (e == hipSuccess) e = hipMalloc((void **)&dst, (size_t)copy_bytes);
    if (e == hipSuccess) e = hipMalloc((void **)&sink, kReadBlocks * sizeof(float));
    if (e == hipSuccess) e = hipMemset(buf, 0, (size_t)read_bytes);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);

    // best (shortest) of reps timed launches after one untimed launch, in ms
    auto best_ms = [&](auto launch) {
        double best = 1e30;
        for (int r = 0; r <= reps && e == hipSuccess; ++r) {
            e = hipEventRecord(e0, s);
            if (e == hipSuccess) launch();
            if (e == hipSuccess) e = hipGetLastError();
            if (e == hipSuccess) e = hipEventRecord(e1, s);
            if (e == hipSuccess) e = hipEventSynchronize(e1);
            float ms = 0.0f;
            if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
            if (e == hipSuccess && r > 0 && ms < best) best = ms;
        }
        return best;
    };
    const int iters_f32 = 4096, iters_bf16 = 8192;
    const double waves = (double)kPeakBlocks * kPeakThreads / 64;
    double res[4] = {0.0, 0.0, 0.0, 0.0};
    if (e == hipSuccess) {
        const double ms = best_ms([&] {
            hipLaunchKernelGGL(k_peak_mfma_f32, dim3(kPeakBlocks), dim3(kPeakThreads), 0, s, iters_f32, sink);
        });
        res[0] = waves * iters_f32 * kChains * (2.0 * 32 * 32 * 2) / (ms * 1e-3) / 1e12;
    }
    if (e == hipSuccess) {
        const double ms = best_ms([&] {
            hipLaunchKernelGGL(k_peak_mfma_bf16, dim3(kPeakBlocks), dim3(kPeakThreads), 0, s, iters_bf16, sink);
        });
        res[1] = waves * iters_bf16 * kChains * (2.0 * 32 * 32 * 16) / (ms * 1e-3) / 1e12;
    }
    if (e == hipSuccess) {
        const double ms = best_ms([&] {
            hipLaunchKernelGGL(k_peak_read, dim3(kReadBlocks), dim3(kPeakThreads), 0, s,
                               reinterpret_cast<const f32x4 *>(buf), read_bytes / 16, sink);
        });
        res[2] = (double)read_bytes / (ms * 1e-3) / 1e9;
    }
    if (e == hipSuccess) {
        const double ms = best_ms([&] {
            hipLaunchKernelGGL(k_peak_copy, dim3(kCopyBlocks), dim3(kPeakThreads), 0, s,
                               reinterpret_cast<const f32x4 *>(buf), reinterpret_cast<f32x4 *>(dst),
                               copy_bytes / 16);
        });
        res[3] = 2.0 * (double)copy_bytes / (ms * 1e-3) / 1e9;
    }
    const hipError_t e_run = e;
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (s) (void)hipStreamDestroy(s);
    if (sink) (void)hipFree(sink);
    if (dst) (void)hipFree(dst);
    if (buf) (void)hipFree(buf);
    if (e_run != hipSuccess)
        return fail(e_run == hipErrorOutOfMemory ? NPM_ERR_OOM : NPM_ERR_HIP,
                    std::string("npm_measure_peaks: ") + hipGetErrorString(e_run));
    for (int i = 0; i < 4; ++i) out[i] = res[i];
    return NPM_OK;
}
