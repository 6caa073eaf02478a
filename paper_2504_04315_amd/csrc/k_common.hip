// Kernels shared by every execution mode: parameter initialisation, packing of
// the MLP weights into MFMA-ready LDS images (and their BF16 copies), the FP16
// grid copy, fused Adam (Sec. 5.3, Kingma and Ba), and FP64 reductions.
#include "device_math.h"

namespace npm {

// ---------------------------------------------------------------- timing
void timed_begin(npm_ctx *ctx, const char *name, hipStream_t s, int *token)
{
    *token = -1;
    Timing &t = ctx->timing;
    if (!t.enabled) return;
    int id = -1;
    for (size_t i = 0; i < t.names.size(); ++i)
        if (t.names[i] == name) { id = (int)i; break; }
    if (id < 0) {
        id = (int)t.names.size();
        t.names.emplace_back(name);
        t.launches.push_back(0);
        t.total_ms.push_back(0.0);
    }
    hipEvent_t a, b;
    for (hipEvent_t *e : {&a, &b}) {
        if (!t.free_events.empty()) { *e = t.free_events.back(); t.free_events.pop_back(); }
        else if (hipEventCreate(e) != hipSuccess) return;
    }
    (void)hipEventRecord(a, s);      // a failed record only loses the timing
    t.pending.push_back({id, a, b});
    *token = (int)t.pending.size() - 1;
}

void timed_end(npm_ctx *ctx, int token, hipStream_t s)
{
    if (token < 0) return;
    (void)hipEventRecord(ctx->timing.pending[token].b, s);
}

// ---------------------------------------------------------------- init
// Parameters from Philox4x32-10 keyed by the seed, one counter per parameter:
// grid N(0, scale^2) or U(-scale, scale); MLP layer i Xavier-uniform.
struct InitDesc {
    int64_t grid_params;
    int64_t layer_off[NPM_MAX_LAYERS + 1];
    float layer_bound[NPM_MAX_LAYERS];
    int n_layers;
    int grid_init;
    float grid_scale;
    uint64_t seed;
};

__global__ void k_init(InitDesc d, float *__restrict__ p, int64_t np)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < np;
         i += (int64_t)gridDim.x * blockDim.x) {
        float u[3];
        philox_uniforms((uint64_t)i, d.seed, 0x1417u, 0u, u);
        float v;
        if (i < d.grid_params) {
            if (d.grid_init == NPM_INIT_NORMAL) {
                const float r = sqrtf(-2.0f * logf(1.0f - u[0]));    // 1 - u0 in (0, 1]
                v = d.grid_scale * r * cospif(2.0f * u[1]);
            } else {
                v = d.grid_scale * (2.0f * u[0] - 1.0f);
            }
        } else {
            int li = 0;
            while (li + 1 < d.n_layers && i >= d.layer_off[li + 1]) ++li;
            v = d.layer_bound[li] * (2.0f * u[0] - 1.0f);
        }
        p[i] = v;
    }
}

hipError_t launch_init_params(npm_ctx *ctx, hipStream_t s)
{
    const Net &net = ctx->net;
    InitDesc d{};
    d.grid_params = net.lay.grid_params;
    d.n_layers = net.lay.n_layers;
    for (int i = 0; i < d.n_layers; ++i) {
        d.layer_off[i] = net.lay.layer_offset[i];
        d.layer_bound[i] = sqrtf(6.0f / (float)(net.lay.layer_in[i] + net.lay.layer_out[i]));
    }
    d.layer_off[d.n_layers] = net.lay.n_params;
    d.grid_init = net.cfg.grid_init;
    d.grid_scale = net.cfg.grid_init_scale;
    d.seed = net.cfg.seed;
    const int64_t np = net.lay.n_params;
    const int blocks = (int)std::min<int64_t>((np + 255) / 256, 8192);
    hipLaunchKernelGGL(k_init, dim3(blocks), dim3(256), 0, s, d, ctx->params, np);
    return hipGetLastError();
}

// ---------------------------------------------------------------- packing
// One segment per (layer, direction) of the packed images.  Element idx of a
// segment maps to (block b, step, lane, e) and reads W[row][col] of the layer
// (forward) or of its transpose (backward), zero outside the real shape.
struct PackSeg {
    int64_t dst;        // first element in the image
    int64_t src;        // first weight of the layer in the flat parameters
    int32_t out_p, in_p; // padded shape of the image matrix
    int32_t out_r, in_r; // real shape of the image matrix
    int32_t ld;          // row length of the stored (untransposed) matrix
    int32_t transpose;
};

struct PackDesc {
    PackSeg seg[2 * NPM_MAX_LAYERS];
    int n_seg;
    int64_t total;
};

template <bool BF16>
__global__ void k_pack(PackDesc d, const float *__restrict__ params, float *__restrict__ img32,
                       __bf16 *__restrict__ img16)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < d.total;
         i += (int64_t)gridDim.x * blockDim.x) {
        int si = 0;
        while (si + 1 < d.n_seg && i >= d.seg[si + 1].dst) ++si;
        const PackSeg &g = d.seg[si];
        const int64_t k = i - g.dst;
        int lane, b, step;
        if (!BF16) {
            const int e = (int)(k & 3);
            lane = (int)((k >> 2) & 63);
            const int64_t rest = k >> 8;
            const int ns4 = g.in_p / 8;
            b = (int)(rest / ns4);
            step = (int)(rest % ns4) * 4 + e;
        } else {
            const int e = (int)(k & 7);
            lane = (int)((k >> 3) & 63);
            const int64_t rest = k >> 9;
            const int ns = g.in_p / 16;
            b = (int)(rest / ns);
            step = (int)(rest % ns) * 8 + e;
        }
        const int row = 32 * b + (lane & 31);
        const int col = nf(lane >> 5, step);
        float v = 0.0f;
        if (row < g.out_r && col < g.in_r)
            v = g.transpose ? params[g.src + (int64_t)col * g.ld + row]
                            : params[g.src + (int64_t)row * g.ld + col];
        if (BF16) img16[i] = (__bf16)v;
        else img32[i] = v;
    }
}

static PackDesc pack_desc(const Net &net)
{
    const MlpDesc &m = net.mlp;
    const npm_layout &L = net.lay;
    PackDesc d{};
    int n = 0;
    for (int i = 0; i < L.n_layers; ++i) {
        PackSeg &g = d.seg[n++];
        g.dst = m.fwd_off[i];
        g.src = L.layer_offset[i];
        g.in_p = (i == 0) ? m.in_p : m.hid_p;
        g.out_p = (i == L.n_layers - 1) ? 32 : m.hid_p;
        g.out_r = L.layer_out[i];
        g.in_r = L.layer_in[i];
        g.ld = L.layer_in[i];
        g.transpose = 0;
    }
    // backward images are stored from the last layer to the first; segments
    // must be in increasing dst order for the lookup in k_pack
    for (int i = L.n_layers - 1; i >= 0; --i) {
        PackSeg &g = d.seg[n++];
        g.dst = m.fwd_elems + m.bwd_off[i];
        g.src = L.layer_offset[i];
        const int fin = (i == 0) ? m.in_p : m.hid_p;
        const int fout = (i == L.n_layers - 1) ? 32 : m.hid_p;
        g.in_p = fout;
        g.out_p = fin < 32 ? 32 : fin;
        g.out_r = L.layer_in[i];
        g.in_r = L.layer_out[i];
        g.ld = L.layer_in[i];
        g.transpose = 1;
    }
    d.n_seg = n;
    d.total = m.fwd_elems + m.bwd_elems;
    return d;
}

static void pack_images(const PackDesc &d, const float *src, float *img, void *img16,
                        hipStream_t s)
{
    const int blocks = (int)std::min<int64_t>((d.total + 255) / 256, 1024);
    hipLaunchKernelGGL(k_pack<false>, dim3(blocks), dim3(256), 0, s, d, src, img,
                       (__bf16 *)nullptr);
    if (img16)
        hipLaunchKernelGGL(k_pack<true>, dim3(blocks), dim3(256), 0, s, d, src, (float *)nullptr,
                           (__bf16 *)img16);
}

// The row-major image of the training kernel (MlpDesc::rm_off): layer L as
// its padded rows x cols matrix, rows cols + 1 floats apart, zero outside
// the real weights.
struct RmDesc {
    int64_t off[NPM_MAX_LAYERS + 1];
    int64_t src[NPM_MAX_LAYERS];
    int32_t cols[NPM_MAX_LAYERS], out_r[NPM_MAX_LAYERS], in_r[NPM_MAX_LAYERS];
    int32_t n_layers;
};

__global__ void k_pack_rm(RmDesc d, const float *__restrict__ params, float *__restrict__ dst)
{
    const int64_t total = d.off[d.n_layers];
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total;
         i += (int64_t)gridDim.x * blockDim.x) {
        int L = 0;
        while (L + 1 < d.n_layers && i >= d.off[L + 1]) ++L;
        const int64_t k = i - d.off[L];
        const int S = d.cols[L] + 1;
        const int o = (int)(k / S), c = (int)(k % S);
        dst[i] = (o < d.out_r[L] && c < d.in_r[L]) ? params[d.src[L] + (int64_t)o * d.in_r[L] + c]
                                                   : 0.0f;
    }
}

hipError_t launch_pack_mlp(npm_ctx *ctx, hipStream_t s)
{
    const PackDesc d = pack_desc(ctx->net);
    pack_images(d, ctx->params, ctx->mlp_img, ctx->mlp_img16, s);
    {
        const Net &net = ctx->net;
        RmDesc r{};
        r.n_layers = net.lay.n_layers;
        for (int i = 0; i < r.n_layers; ++i) {
            r.off[i] = net.mlp.rm_off[i];
            r.src[i] = net.lay.layer_offset[i];
            r.cols[i] = i == 0 ? std::max(net.mlp.in_p, 32) : net.mlp.hid_p;
            r.out_r[i] = net.lay.layer_out[i];
            r.in_r[i] = net.lay.layer_in[i];
        }
        r.off[r.n_layers] = net.mlp.rm_elems;
        const int blocks = (int)std::min<int64_t>((net.mlp.rm_elems + 255) / 256, 256);
        hipLaunchKernelGGL(k_pack_rm, dim3(blocks), dim3(256), 0, s, r, ctx->params,
                           ctx->mlp_img + net.mlp.fwd_elems + net.mlp.bwd_elems);
    }
    if (ctx->ema) pack_images(d, ctx->ema, ctx->ema_img, ctx->ema_img16, s);
    return hipGetLastError();
}

__global__ void k_grid_to_half(const float *__restrict__ p, __half *__restrict__ h, int64_t n)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        h[i] = __float2half_rn(p[i]);
}

hipError_t launch_refresh_lowp(npm_ctx *ctx, hipStream_t s)
{
    hipError_t e = launch_pack_mlp(ctx, s);
    if (e != hipSuccess) return e;
    const int64_t n = ctx->net.lay.grid_params;
    if (ctx->grid16)
        hipLaunchKernelGGL(k_grid_to_half, dim3(2048), dim3(256), 0, s, ctx->params,
                           (__half *)ctx->grid16, n);
    if (ctx->ema_grid16)
        hipLaunchKernelGGL(k_grid_to_half, dim3(2048), dim3(256), 0, s, ctx->ema,
                           (__half *)ctx->ema_grid16, n);
    return hipGetLastError();
}

// ---------------------------------------------------------------- Adam
// m <- b1 m + (1-b1) g; v <- b2 v + (1-b2) g^2; p <- p - lr m^/(sqrt(v^) + eps)
// with m^ = m / (1 - b1^t), v^ = v / (1 - b2^t); g is zeroed; the FP16 copy of
// the grid is written in the same pass; sum g^2 is reduced in FP64.  With a
// moving average kept (ema non-null), ema <- d ema + (1 - d) p after the step,
// and its FP16 grid copy too.
__global__ __launch_bounds__(256) void k_adam(float *__restrict__ p, float *__restrict__ g,
                                              float *__restrict__ m, float *__restrict__ v,
                                              int64_t np, float lr, float b1, float b2, float eps,
                                              float c1inv, float c2inv, __half *__restrict__ grid16,
                                              int64_t grid_params, double *__restrict__ partials,
                                              float *__restrict__ ema, __half *__restrict__ ema16,
                                              float decay)
{
    double acc = 0.0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < np;
         i += (int64_t)gridDim.x * blockDim.x) {
        const float gi = g[i];
        const float mi = b1 * m[i] + (1.0f - b1) * gi;
        const float vi = b2 * v[i] + (1.0f - b2) * (gi * gi);
        const float pi = p[i] - lr * (mi * c1inv) / (sqrtf(vi * c2inv) + eps);
        m[i] = mi;
        v[i] = vi;
        p[i] = pi;
        g[i] = 0.0f;
        if (grid16 && i < grid_params) grid16[i] = __float2half_rn(pi);
        if (ema) {
            const float ei = decay * ema[i] + (1.0f - decay) * pi;
            ema[i] = ei;
            if (ema16 && i < grid_params) ema16[i] = __float2half_rn(ei);
        }
        acc += (double)gi * (double)gi;
    }
    __shared__ double red[256];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) partials[blockIdx.x] = red[0];
}

hipError_t launch_adam(npm_ctx *ctx, float *grad, double *gradnorm_out, hipStream_t s)
{
    const npm_config &c = ctx->net.cfg;
    const double t = (double)ctx->step;
    const float c1inv = (float)(1.0 / (1.0 - pow((double)c.beta1, t)));
    const float c2inv = (float)(1.0 / (1.0 - pow((double)c.beta2, t)));
    const int64_t np = ctx->net.lay.n_params;
    const int blocks = (int)std::min<int64_t>((np + 255) / 256, 2048);
    int tok;
    timed_begin(ctx, "adam", s, &tok);
    hipLaunchKernelGGL(k_adam, dim3(blocks), dim3(256), 0, s, ctx->params, grad, ctx->adam_m,
                       ctx->adam_v, np, c.lr, c.beta1, c.beta2, c.eps, c1inv, c2inv,
                       (__half *)ctx->grid16, ctx->net.lay.grid_params, ctx->partials, ctx->ema,
                       (__half *)ctx->ema_grid16, c.ema_decay);
    timed_end(ctx, tok, s);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    // the packed MLP images (and their BF16 copy) follow the new weights
    e = launch_pack_mlp(ctx, s);
    if (e != hipSuccess) return e;
    if (gradnorm_out) return launch_reduce_partials(ctx, blocks, gradnorm_out, s);
    return hipSuccess;
}

// ---------------------------------------------------------------- reductions
// Sums nparts FP64 partials in a fixed order into *out (times scale).
__global__ void k_reduce(const double *__restrict__ part, int nparts, double scale,
                         double *__restrict__ out)
{
    __shared__ double red[256];
    double a = 0.0;
    for (int i = threadIdx.x; i < nparts; i += 256) a += part[i];
    red[threadIdx.x] = a;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = red[0] * scale;
}

hipError_t launch_reduce_partials(npm_ctx *ctx, int nparts, double *out, hipStream_t s)
{
    hipLaunchKernelGGL(k_reduce, dim3(1), dim3(256), 0, s, ctx->partials, nparts, 1.0, out);
    return hipGetLastError();
}

hipError_t launch_reduce_scaled(const double *part, int nparts, double scale, double *out,
                                hipStream_t s)
{
    hipLaunchKernelGGL(k_reduce, dim3(1), dim3(256), 0, s, part, nparts, scale, out);
    return hipGetLastError();
}

__global__ void k_fill(float *__restrict__ p, int64_t n, float v)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

hipError_t launch_fill_f32(float *p, int64_t n, float v, hipStream_t s)
{
    const int blocks = (int)std::min<int64_t>((n + 255) / 256, 4096);
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill, dim3(blocks), dim3(256), 0, s, p, n, v);
    return hipGetLastError();
}

}  // namespace npm
