// Persistent multi-session kernels of the serving form.  One launch covers
// every query (or every training batch) of a round, whatever the session:
// blocks pull chunks of tiles from a device counter, find the request a
// chunk belongs to, and restage that session's weight images and level table
// into LDS only when the session changes.  The per-tile work is exactly the
// fused path's (fused_tiles.h), so a request gives the same result alone or
// in a mix (queries bit for bit; training up to the order of atomic adds).
#include <cstring>

#include "fused_tiles.h"
#include "serve_internal.h"

namespace npm {

// Device descriptor of one request of a round.
struct DevReq {
    GridDesc g;
    const __half *grid16;
    const void *img;             // BF16 images of the session: forward then backward
    float *grad;                 // the session's gradient buffer (train)
    const float *pos, *dir, *rad, *spdf;
    float *lobes, *pdf, *sdir, *spdf_out;
    double *loss;                // loss slot of the round buffer (train)
    int64_t n;
    int64_t mlp_off;             // first MLP weight in the flat parameters
    uint64_t seed;
    uint32_t sid;
    int32_t skey;                // session identity (restaging test)
    int32_t chunk_begin;         // first chunk of the request in its launch
    int32_t fwd_elems, bwd_elems, n_in, width;
    float invN;
};

// A round launches one kernel per (network shape, request kind) group: at
// most two kinds for each of the kServeShapes shapes serve_supports admits.
constexpr int kServeShapes = 4;
constexpr int kMaxRoundGroups = 2 * kServeShapes;

struct RoundHdr {
    uint32_t counter[kMaxRoundGroups];   // chunk counters, one per launch (zero at upload)
    int32_t n_req;
    int32_t pad[3];
};
static_assert(sizeof(RoundHdr) <= 64, "the round header sits in the first 64 bytes");

constexpr int kQueryChunkTiles = 4;    // one tile per wave
constexpr int kTrainChunkTiles = 16;   // four rounds of one tile per wave

// Bytes of a training block's LDS exchange buffer (BF16, after the images).
template <int IN_P, int HID_P, int NH>
constexpr size_t serve_xch_bytes()
{
    using Plan = BlockPlan<IN_P, HID_P, NH, 4>;
    return ((size_t)Plan::max_rows() * Plan::xs(true) * 2 + 15) / 16 * 16;
}

// Request of chunk c among [r0, r1): the last one whose chunk_begin <= c.
__device__ __forceinline__ int find_request(const int *s_begin, int r0, int r1, int c)
{
    int lo = r0, hi = r1 - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (s_begin[mid] <= c) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

__device__ __forceinline__ void stage_bytes(char *dst, const void *src, int bytes)
{
    for (int i = threadIdx.x; i < bytes / 16; i += blockDim.x)
        reinterpret_cast<f32x4 *>(dst)[i] = reinterpret_cast<const f32x4 *>(src)[i];
}

// Queries of requests [r0, r1) of the round; `which` selects the counter.
template <int IN_P, int HID_P, int NH, int F>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2, 2))) void k_serve_query(RoundHdr *hdr, const DevReq *__restrict__ reqs,
                                                     int r0, int r1, int n_chunks, int which)
{
    extern __shared__ __attribute__((aligned(16))) char smem[];
    __shared__ uint32_t s_off[NPM_MAX_LEVELS];
    __shared__ int s_res[NPM_MAX_LEVELS];
    __shared__ int s_begin[kMaxRoundRequests];
    __shared__ int s_chunk;
    for (int i = r0 + threadIdx.x; i < r1; i += blockDim.x) s_begin[i] = reqs[i].chunk_begin;
    int staged = -1;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    for (;;) {
        __syncthreads();
        if (threadIdx.x == 0) s_chunk = (int)atomicAdd(&hdr->counter[which], 1u);
        __syncthreads();
        const int chunk = s_chunk;
        if (chunk >= n_chunks) break;
        const int r = find_request(s_begin, r0, r1, chunk);
        const DevReq &q = reqs[r];
        if (q.skey != staged) {
            stage_bytes(smem, q.img, q.fwd_elems * 2);
            stage_levels(q.g, s_off, s_res);
            staged = q.skey;
            __syncthreads();
        }
        const int64_t t = (int64_t)(chunk - q.chunk_begin) * kQueryChunkTiles + wave;
        if (t * 32 < q.n) {
            const GridView gv = grid_view(q.g, s_off, s_res, nullptr, q.grid16);
            const QueryIO io{q.n, q.pos, q.dir, q.lobes, q.pdf, q.sdir, q.spdf_out, q.seed, q.sid};
            query_tile<IN_P, HID_P, NH, F, true>(gv, smem, io, t, lane);
        }
    }
}

// Training batches of requests [r0, r1), the fused path's block-cooperative
// scheme (fused_tiles.h): a chunk is kTrainChunkTiles tiles of one request,
// run as rounds of one tile per wave; per layer the waves exchange deltas and
// inputs in LDS and each wave accumulates its share of the weight-gradient
// blocks over the round's 128 vertices.  The shares stay in registers while
// the block's chunks belong to one request (its chunks are handed out in
// order, so a block usually takes several in a row) and are added into that
// session's gradient with FP32 atomics when the request changes and at the
// end: per block and request, one add per weight.  Each tile's grid gradient
// is scattered from the wave's LDS buffer, its coarse levels through a 32-bit
// fixed-point window (no FP64 accumulator), the rest by FP32 atomics.
template <int IN_P, int HID_P, int NH, int F>
__global__ __launch_bounds__(256) void k_serve_train(RoundHdr *hdr, const DevReq *__restrict__ reqs,
                                                     int r0, int r1, int n_chunks, int which,
                                                     int img_bytes_max)
{
    constexpr int WV = 4;
    using Plan = BlockPlan<IN_P, HID_P, NH, WV>;
    constexpr int IN0 = Plan::IN0;
    constexpr int XS = Plan::xs(true);
    constexpr int NS = Plan::slots();
    constexpr int WIN_PTS = (HID_P - IN0) * kStride / (2 * F);
    static_assert(Plan::scratch_fits(true), "split blocks' sums fit in the exchange buffer");
    extern __shared__ __attribute__((aligned(16))) char smem[];
    __shared__ uint32_t s_off[NPM_MAX_LEVELS];
    __shared__ int s_res[NPM_MAX_LEVELS];
    __shared__ int s_begin[kMaxRoundRequests];
    __shared__ int s_chunk;
    for (int i = r0 + threadIdx.x; i < r1; i += blockDim.x) s_begin[i] = reqs[i].chunk_begin;
    int staged = -1, cur = -1;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, h = lane >> 5;
    const size_t img_al = ((size_t)img_bytes_max + 15) / 16 * 16;
    __bf16 *xb = reinterpret_cast<__bf16 *>(smem + img_al);
    float *tbuf = reinterpret_cast<float *>(smem + img_al + serve_xch_bytes<IN_P, HID_P, NH>()) +
                  wave * HID_P * kStride;
    f32x16 acc[NS];
#pragma unroll
    for (int k = 0; k < NS; ++k)
#pragma unroll
        for (int v = 0; v < 16; ++v) acc[k][v] = 0.0f;
    for (;;) {
        __syncthreads();
        if (threadIdx.x == 0) s_chunk = (int)atomicAdd(&hdr->counter[which], 1u);
        __syncthreads();
        const int chunk = s_chunk;
        const int r = chunk < n_chunks ? find_request(s_begin, r0, r1, chunk) : -1;
        if (r != cur) {
            if (cur >= 0) {
                const DevReq &c = reqs[cur];
                dw_write<Plan, NH, WV, true>(c.grad + c.mlp_off, c.n_in, c.width, wave, acc, lane,
                                             reinterpret_cast<float *>(xb));
#pragma unroll
                for (int k = 0; k < NS; ++k)
#pragma unroll
                    for (int v = 0; v < 16; ++v) acc[k][v] = 0.0f;
            }
            cur = r;
        }
        if (chunk >= n_chunks) break;
        const DevReq &q = reqs[r];
        if (q.skey != staged) {
            stage_bytes(smem, q.img, (q.fwd_elems + q.bwd_elems) * 2);
            stage_levels(q.g, s_off, s_res);
            staged = q.skey;
            __syncthreads();
        }
        const GridView gv = grid_view(q.g, s_off, s_res, nullptr, q.grid16);
        const TrainIO io{q.n, q.pos, q.dir, q.rad, q.spdf, q.grad, q.invN, nullptr};
        const char *fwd = smem;
        const char *bwd = smem + (size_t)q.fwd_elems * 2;
        const int64_t ntiles = (q.n + 31) / 32;
        const int64_t c0 = (int64_t)(chunk - q.chunk_begin) * kTrainChunkTiles;
        double lacc = 0.0;
        for (int rr = 0; rr < kTrainChunkTiles / WV; ++rr) {
            // every wave runs every round of the chunk (the phases
            // synchronise); a wave past the batch takes a tile with no valid
            // vertex
            const int64_t t0 = c0 + (int64_t)rr * WV;
            if (t0 >= ntiles) break;                    // uniform over the block
            const int64_t t = t0 + wave;
            const int64_t v = t * 32 + (lane & 31);
            const bool valid = v < q.n;
            const int64_t vs = valid ? v : q.n - 1;
            const TrainInputs in = train_inputs(io, vs, vs);
            float x[IN0 / 2];
            tile_input<IN_P, F, true, 0>(gv, io, in, vs, vs, h, x);
            float acts[NH][HID_P / 2], o[16], d[16];
            mlp_forward<IN_P, HID_P, NH, true, true>(fwd, x, acts, o, lane);
            kl_head(o, in, valid, io.invN, h, d, lacc);
            // ---- output layer's dW, then the delta chain
            float dh[HID_P / 2];
            dw_phase<Plan, NH, WV, XS>(xb, d, acts[NH - 1], wave, acc, lane);
            layer<true, 32, HID_P>(bwd, d, dh, lane);
            __syncthreads();
            const char *im = bwd + (size_t)HID_P * 32 * 2;
            static_for_down<NH - 1, 1>([&](auto LC) {
                constexpr int li = decltype(LC)::value;
#pragma unroll
                for (int i = 0; i < HID_P / 2; ++i) dh[i] = acts[li][i] > 0.0f ? dh[i] : 0.0f;
                dw_phase<Plan, li, WV, XS>(xb, dh, acts[li - 1], wave, acc, lane);
                float nd[HID_P / 2];
                layer<true, HID_P, HID_P>(im, dh, nd, lane);
                im += (size_t)HID_P * HID_P * 2;
#pragma unroll
                for (int i = 0; i < HID_P / 2; ++i) dh[i] = nd[i];
                __syncthreads();
            });
#pragma unroll
            for (int i = 0; i < HID_P / 2; ++i) dh[i] = acts[0][i] > 0.0f ? dh[i] : 0.0f;
            dw_phase<Plan, 0, WV, XS>(xb, dh, x, wave, acc, lane);
            float dG[IN0 / 2];
            layer<true, HID_P, IN0>(im, dh, dG, lane);
            __syncthreads();
            // ---- the tile's grid scatter from the wave's own buffer
            if (t < ntiles) {
                float lo[3], hi[3];
                if constexpr (WIN_PTS > 0) tile_bbox(in.px, in.py, in.pz, lo, hi);
                wave_lds_fence();
                t32_to_lds<IN0 / 2>(tbuf, dG, lane);
                wave_lds_fence();
                scatter_tile<F, WIN_PTS, int>(gv, tbuf, io.pos, nullptr, q.n, t, lane, io.grad, lo,
                                              hi, reinterpret_cast<int *>(tbuf + IN0 * kStride));
            }
        }
        // FP64 loss of the wave (half 0 holds it), one atomic per wave
        double l = lacc;
        for (int off = 16; off > 0; off >>= 1) l += __shfl_xor(l, off, 64);
        if (lane == 0 && l != 0.0) atomicAdd(q.loss, l);
    }
}

// stats[0] = loss / n for each training request of the round.
__global__ void k_serve_finish(const DevReq *__restrict__ reqs, const double *const *stats_out,
                               int r0, int r1)
{
    const int i = r0 + blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= r1) return;
    double *st = const_cast<double *>(stats_out[i]);
    if (st) st[0] = *reqs[i].loss * (1.0 / (double)reqs[i].n);
}

// ------------------------------------------------------------------ host side
struct RoundLayout {
    size_t hdr = 0, reqs = 0, loss = 0, stats = 0, total = 0;
};

static RoundLayout round_layout()
{
    RoundLayout L;
    L.hdr = 0;
    L.reqs = 64;
    L.loss = L.reqs + sizeof(DevReq) * kMaxRoundRequests;
    L.stats = L.loss + sizeof(double) * kMaxRoundRequests;
    L.total = L.stats + sizeof(double *) * kMaxRoundRequests;
    return L;
}

hipError_t round_buffers_init(RoundBuffers *b)
{
    const RoundLayout L = round_layout();
    b->bytes = L.total;
    hipError_t e = hipHostMalloc(&b->host, L.total, hipHostMallocDefault);
    if (e == hipSuccess) e = hipMalloc(&b->dev, L.total);
    return e;
}

void round_buffers_free(RoundBuffers *b)
{
    if (b->host) (void)hipHostFree(b->host);
    if (b->dev) (void)hipFree(b->dev);
    b->host = b->dev = nullptr;
}

static int shape_key(const Net &net)
{
    const MlpDesc &m = net.mlp;
    return net.grid.feat * 1000 + (m.in_p == 32) * 100 + (m.hid_p == 64) * 10 + m.n_hidden;
}

bool serve_supports(const npm_config *cfg)
{
    Net net;
    std::string err;
    if (describe(cfg, &net, &err) != NPM_OK) return false;
    if (cfg->sh_degree != 0) return false;
    const int k = shape_key(net);
    static_assert(kServeShapes == 4, "the shapes listed here and in launch_shape");
    return k == 2113 || k == 4012 || k == 2002 || k == 2112;
}

template <int IN_P, int HID_P, int NH, int F>
static hipError_t launch_group(RoundHdr *hdr, const DevReq *reqs, int r0, int r1, int chunks,
                               int which, bool train, int img_bytes_max, hipStream_t s)
{
    if (chunks <= 0) return hipSuccess;
    const int blocks = std::max(1, std::min(chunks, 1024));
    if (!train) {
        auto k = k_serve_query<IN_P, HID_P, NH, F>;
        const int lds = img_bytes_max;
        const hipError_t e = hipFuncSetAttribute((const void *)k,
                                                 hipFuncAttributeMaxDynamicSharedMemorySize, lds);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k, dim3(blocks), dim3(256), lds, s, hdr, reqs, r0, r1, chunks, which);
    } else {
        auto k = k_serve_train<IN_P, HID_P, NH, F>;
        // images, the exchange buffer, four waves' scatter buffers
        const int lds = (img_bytes_max + 15) / 16 * 16 + (int)serve_xch_bytes<IN_P, HID_P, NH>() +
                        4 * HID_P * kStride * (int)sizeof(float);
        const hipError_t e = hipFuncSetAttribute((const void *)k,
                                                 hipFuncAttributeMaxDynamicSharedMemorySize, lds);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k, dim3(std::min(blocks, 256)), dim3(256), lds, s, hdr, reqs, r0, r1,
                           chunks, which, img_bytes_max);
    }
    return hipGetLastError();
}

static hipError_t launch_shape(int key, RoundHdr *hdr, const DevReq *reqs, int r0, int r1,
                               int chunks, int which, bool train, int img_bytes_max, hipStream_t s)
{
    switch (key) {
    case 2113: return launch_group<32, 64, 3, 2>(hdr, reqs, r0, r1, chunks, which, train, img_bytes_max, s);
    case 2112: return launch_group<32, 64, 2, 2>(hdr, reqs, r0, r1, chunks, which, train, img_bytes_max, s);
    case 4012: return launch_group<16, 64, 2, 4>(hdr, reqs, r0, r1, chunks, which, train, img_bytes_max, s);
    case 2002: return launch_group<16, 32, 2, 2>(hdr, reqs, r0, r1, chunks, which, train, img_bytes_max, s);
    default: return hipErrorNotSupported;
    }
}

// Round buffer: [header][DevReq x n][loss x n][stats pointer x n].  Requests
// are ordered by (shape, kind) so that each launch covers a contiguous range.
hipError_t serve_launch_round(RoundBuffers *b, const std::vector<ServeRequest> &in,
                              hipStream_t s)
{
    const RoundLayout L = round_layout();
    const int nreq = (int)in.size();
    if (nreq == 0) return hipSuccess;
    if (nreq > kMaxRoundRequests) return hipErrorInvalidValue;
    std::vector<int> order(nreq);
    for (int i = 0; i < nreq; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](int a, int c) {
        const int ka = shape_key(in[a].ctx->net) * 2 + in[a].kind;
        const int kc = shape_key(in[c].ctx->net) * 2 + in[c].kind;
        return ka < kc;
    });
    char *host = (char *)b->host;
    char *dev = (char *)b->dev;
    std::memset(host, 0, L.reqs);
    RoundHdr *hh = (RoundHdr *)host;
    hh->n_req = nreq;
    DevReq *hr = (DevReq *)(host + L.reqs);
    double *hloss = (double *)(host + L.loss);
    double **hstats = (double **)(host + L.stats);
    DevReq *dr = (DevReq *)(dev + L.reqs);
    double *dloss = (double *)(dev + L.loss);
    struct Group { int key, kind, r0, r1, chunks, img; };
    std::vector<Group> groups;
    for (int j = 0; j < nreq; ++j) {
        const ServeRequest &q = in[order[j]];
        npm_ctx *ctx = q.ctx;
        const Net &net = ctx->net;
        const int key = shape_key(net);
        if (groups.empty() || groups.back().key != key || groups.back().kind != q.kind)
            groups.push_back({key, q.kind, j, j, 0, 0});
        Group &g = groups.back();
        DevReq &d = hr[j];
        std::memset(&d, 0, sizeof(d));
        d.g = net.grid;
        const Weights w = q.kind == 0 ? query_weights(ctx) : trained_weights(ctx);
        d.grid16 = (const __half *)w.grid16;
        d.img = w.img16;
        d.grad = ctx->grads;
        d.pos = q.pos; d.dir = q.dir; d.rad = q.rad; d.spdf = q.spdf;
        d.lobes = q.lobes; d.pdf = q.pdf; d.sdir = q.sdir; d.spdf_out = q.spdf_out;
        d.loss = dloss + j;
        d.n = q.n;
        d.mlp_off = net.lay.grid_params;
        d.seed = q.seed;
        d.sid = q.stream_id;
        d.skey = q.session;
        d.fwd_elems = (int)net.mlp.fwd_elems;
        d.bwd_elems = (int)net.mlp.bwd_elems;
        d.n_in = net.mlp.n_in;
        d.width = net.mlp.width;
        d.invN = q.n > 0 ? 1.0f / (float)q.n : 0.0f;
        const int64_t tiles = (q.n + 31) / 32;
        const int per = q.kind == 0 ? kQueryChunkTiles : kTrainChunkTiles;
        d.chunk_begin = g.chunks;
        g.chunks += (int)((tiles + per - 1) / per);
        g.r1 = j + 1;
        const int img = (int)((q.kind == 0 ? net.mlp.fwd_elems : net.mlp.fwd_elems + net.mlp.bwd_elems) * 2);
        g.img = std::max(g.img, img);
        hloss[j] = 0.0;
        hstats[j] = q.stats;
    }
    // one counter per launch; serve_supports admits kServeShapes shapes
    if ((int)groups.size() > kMaxRoundGroups) return hipErrorNotSupported;
    hipError_t e = hipMemcpyAsync(dev, host, L.total, hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return e;
    RoundHdr *dh = (RoundHdr *)dev;
    for (int gi = 0; gi < (int)groups.size(); ++gi) {
        const Group &g = groups[gi];
        e = launch_shape(g.key, dh, dr, g.r0, g.r1, g.chunks, gi, g.kind == 1, g.img, s);
        if (e != hipSuccess) return e;
        if (g.kind == 1) {
            hipLaunchKernelGGL(k_serve_finish, dim3((g.r1 - g.r0 + 63) / 64), dim3(64), 0, s, dr,
                               (const double *const *)(dev + L.stats), g.r0, g.r1);
            e = hipGetLastError();
            if (e != hipSuccess) return e;
            for (int j = g.r0; j < g.r1; ++j) {
                const ServeRequest &q = in[order[j]];
                q.ctx->step += 1;
                e = launch_adam(q.ctx, q.ctx->grads, q.stats ? q.stats + 1 : nullptr, s);
                if (e != hipSuccess) return e;
            }
        }
    }
    return hipSuccess;
}

}  // namespace npm
