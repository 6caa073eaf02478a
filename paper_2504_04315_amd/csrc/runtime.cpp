// libnpm C ABI: configuration and layout, context lifetime, argument
// validation, dispatch to the staged or fused kernels, state export/import
// and kernel timing.  No C++ exception crosses the ABI.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>

#include "npm_internal.h"

using namespace npm;

namespace {

thread_local std::string g_err;

npm_status fail(npm_status st, const std::string &msg)
{
    g_err = msg;
    return st;
}

npm_status hip_fail(hipError_t e, const char *what)
{
    return fail(e == hipErrorOutOfMemory ? NPM_ERR_OOM : NPM_ERR_HIP,
                std::string(what) + ": " + hipGetErrorString(e));
}

#define NPM_HIP(call, what)                                \
    do {                                                   \
        hipError_t e_ = (call);                            \
        if (e_ != hipSuccess) return hip_fail(e_, what);   \
    } while (0)

bool aligned4(const void *p) { return ((uintptr_t)p & 3u) == 0; }

}  // namespace

void npm::set_error(const char *msg) { g_err = msg ? msg : ""; }

// --------------------------------------------------------------------------
// Configuration and layout (Sec. 5.1 grid levels, Sec. 5.3 MLP)
// --------------------------------------------------------------------------
static_assert(sizeof(((npm_config *)nullptr)->resolution) / sizeof(int32_t) == NPM_MAX_LEVELS,
              "one resolution per level");

npm_status npm::describe(const npm_config *cfg, Net *net, std::string *err)
{
    auto bad = [&](const char *m) { *err = m; return NPM_ERR_INVALID_ARG; };
    if (!cfg || !net) return bad("null argument");
    const npm_config &c = *cfg;
    if (c.grid_kind != NPM_GRID_DENSE && c.grid_kind != NPM_GRID_HASH) return bad("grid_kind");
    if (c.n_levels < 1 || c.n_levels > NPM_MAX_LEVELS) return bad("n_levels must be 1..32");
    if (c.feat_per_level != 1 && c.feat_per_level != 2 && c.feat_per_level != 4)
        return bad("feat_per_level must be 1, 2 or 4");
    if (c.n_levels * c.feat_per_level > 32) return bad("n_levels * feat_per_level must be <= 32");
    if (c.grid_kind == NPM_GRID_HASH && (c.log2_table_size < 4 || c.log2_table_size > 26))
        return bad("log2_table_size must be 4..26");
    const bool table = c.resolution[0] != 0;
    if (table) {
        for (int l = 0; l < NPM_MAX_LEVELS; ++l) {
            const int D = c.resolution[l];
            if (l >= c.n_levels) {
                if (D != 0) return bad("resolution[] entries from n_levels on must be 0");
            } else if (D < 1 || D > 65535 || (l > 0 && D < c.resolution[l - 1])) {
                return bad("resolution[] must hold n_levels values in 1..65535, non-decreasing");
            }
        }
    } else {
        for (int l = 1; l < NPM_MAX_LEVELS; ++l)
            if (c.resolution[l] != 0)
                return bad("resolution[]: a table starts at resolution[0]; all 0 derives it");
        if (c.base_resolution < 1 || c.max_resolution < c.base_resolution ||
            c.max_resolution > 65535)
            return bad("resolutions must satisfy 1 <= base <= max <= 65535");
    }
    if (c.mlp_width < 1 || c.mlp_width > 64) return bad("mlp_width must be 1..64");
    if (c.mlp_hidden_layers < 1 || c.mlp_hidden_layers > 4) return bad("mlp_hidden_layers must be 1..4");
    if (c.n_lobes != kLobes) return bad("n_lobes must be 8");
    if (c.precision != NPM_PREC_FP32 && c.precision != NPM_PREC_BF16) return bad("precision");
    if (c.exec_mode != NPM_EXEC_STAGED && c.exec_mode != NPM_EXEC_FUSED) return bad("exec_mode");
    if (c.precision == NPM_PREC_BF16 && c.exec_mode != NPM_EXEC_FUSED)
        return bad("the BF16 precision form runs fused only");
    if (c.grid_init != NPM_INIT_NORMAL && c.grid_init != NPM_INIT_UNIFORM) return bad("grid_init");
    if (c.batch_order < NPM_ORDER_AUTO || c.batch_order > NPM_ORDER_SPATIAL) return bad("batch_order");
    if (c.scatter_mode < NPM_SCATTER_AUTO || c.scatter_mode > NPM_SCATTER_BINNED)
        return bad("scatter_mode");
    if (!(std::isfinite(c.grid_init_scale) && c.grid_init_scale >= 0.0f)) return bad("grid_init_scale");
    if (!(std::isfinite(c.lr) && c.lr > 0.0f)) return bad("lr must be > 0");
    if (!(c.beta1 >= 0.0f && c.beta1 < 1.0f && c.beta2 >= 0.0f && c.beta2 < 1.0f))
        return bad("betas must be in [0, 1)");
    if (!(std::isfinite(c.eps) && c.eps > 0.0f)) return bad("eps must be > 0");
    if (!(c.ema_decay >= 0.0f && c.ema_decay < 1.0f)) return bad("ema_decay must be in [0, 1)");
    if (c.sh_degree < 0 || c.sh_degree > 4) return bad("sh_degree must be 0..4");
    if (c.learn_selection != 0 && c.learn_selection != 1) return bad("learn_selection must be 0 or 1");
    if (c.sh_degree > 0 && c.exec_mode == NPM_EXEC_FUSED &&
        !((c.sh_degree == 4 && c.n_levels * c.feat_per_level == 32) ||
          (c.sh_degree == 2 && c.n_levels * c.feat_per_level == 4)))
        return bad("fused NPM-product: sh_degree 4 with 32 grid features or 2 with 4; "
                   "the staged path takes other shapes");

    Net n{};
    n.cfg = c;
    npm_layout &L = n.lay;
    const int nl = c.n_levels;
    int64_t entries = 0;
    const double ratio = (double)c.max_resolution / (double)c.base_resolution;
    for (int l = 0; l < nl; ++l) {
        int D;
        if (table) D = c.resolution[l];
        else if (l == nl - 1) D = c.max_resolution;
        else if (l == 0) D = c.base_resolution;
        else {
            const double b = std::exp(std::log(ratio) / (double)(nl - 1));
            D = (int)std::floor((double)c.base_resolution * std::pow(b, (double)l) + 1e-6);
        }
        const int64_t pts = (int64_t)(D + 1) * (D + 1) * (D + 1);
        const bool hashed = c.grid_kind == NPM_GRID_HASH && pts > ((int64_t)1 << c.log2_table_size);
        L.resolution[l] = D;
        L.hashed[l] = hashed ? 1 : 0;
        L.level_size[l] = hashed ? ((int64_t)1 << c.log2_table_size) : pts;
        L.level_offset[l] = entries;
        entries += L.level_size[l];
        if (entries > ((int64_t)1 << 31) - 1) return bad("grid too large (more than 2^31 entries)");
    }
    L.grid_entries = entries;
    L.grid_params = entries * c.feat_per_level;
    const int n_aux = c.sh_degree ? 2 * c.sh_degree * c.sh_degree + 1 : 0;
    L.n_in = nl * c.feat_per_level + n_aux;
    L.n_out = 4 * kLobes + (c.learn_selection ? 1 : 0);
    L.n_layers = c.mlp_hidden_layers + 1;
    int64_t off = L.grid_params;
    for (int i = 0; i < L.n_layers; ++i) {
        L.layer_in[i] = (i == 0) ? L.n_in : c.mlp_width;
        L.layer_out[i] = (i == L.n_layers - 1) ? L.n_out : c.mlp_width;
        L.layer_offset[i] = off;
        off += (int64_t)L.layer_in[i] * L.layer_out[i];
    }
    L.n_params = off;

    GridDesc &g = n.grid;
    for (int l = 0; l < nl; ++l) {
        g.offset[l] = (uint32_t)L.level_offset[l];
        g.res[l] = L.resolution[l];
        if (L.hashed[l]) g.hashed_mask |= 1u << l;
    }
    g.table_mask = c.grid_kind == NPM_GRID_HASH ? (uint32_t)((1u << c.log2_table_size) - 1u) : 0u;
    g.n_levels = nl;
    g.feat = c.feat_per_level;

    MlpDesc &m = n.mlp;
    m.n_in = L.n_in;
    m.width = c.mlp_width;
    m.n_hidden = c.mlp_hidden_layers;
    m.in_p = L.n_in <= 16 ? 16 : L.n_in <= 32 ? 32 : L.n_in <= 64 ? 64 : 96;
    m.gf = nl * c.feat_per_level;
    m.sh_degree = c.sh_degree;
    m.hid_p = c.mlp_width <= 32 ? 32 : 64;
    int64_t fo = 0;
    for (int i = 0; i < L.n_layers; ++i) {
        const int in_p = i == 0 ? m.in_p : m.hid_p;
        const int out_p = i == L.n_layers - 1 ? 32 : m.hid_p;
        m.fwd_off[i] = fo;
        fo += (int64_t)in_p * out_p;
    }
    m.fwd_elems = fo;
    int64_t bo = 0;   // backward images from the last layer to the first
    for (int i = L.n_layers - 1; i >= 0; --i) {
        const int in_p = i == 0 ? m.in_p : m.hid_p;
        const int out_p = i == L.n_layers - 1 ? 32 : m.hid_p;
        m.bwd_off[i] = bo;
        bo += (int64_t)std::max(in_p, 32) * out_p;
    }
    m.bwd_elems = bo;
    int64_t ro = 0;   // row-major image, layers in order
    for (int i = 0; i < L.n_layers; ++i) {
        const int cols = i == 0 ? std::max(m.in_p, 32) : m.hid_p;
        const int rows = i == L.n_layers - 1 ? 32 : m.hid_p;
        m.rm_off[i] = ro;
        ro += (int64_t)rows * (cols + 1);
    }
    m.rm_elems = ro;
    const int64_t img = m.fwd_elems + m.bwd_elems;
    const int64_t lowp_grid = c.precision == NPM_PREC_BF16 ? 2 * L.grid_params : 0;
    L.device_bytes = 16 * L.n_params + 6 * img + 4 * m.rm_elems + (int64_t)kPartials * 8 + 64 + lowp_grid +
                     (c.ema_decay > 0.0f ? 4 * L.n_params + 6 * img + lowp_grid : 0);
    if (c.exec_mode == NPM_EXEC_FUSED && c.learn_selection && !fused_shape_supported(n))
        return bad("no fused kernels with the selection output for this network shape (fused: "
                   "radiance-based, as (F, inputs, hidden width x layers): (2, <= 16, <= 32 x 2), "
                   "(4, <= 16, 33..64 x 2), (4, 17..32, 33..64 x 2), (2, 17..32, 33..64 x 3)); "
                   "the staged path takes any shape");
    if (c.exec_mode == NPM_EXEC_FUSED && !fused_shape_supported(n))
        return bad("no fused kernels for this network shape (fused: F 1, 2 or 4; 16 or 32 grid "
                   "features; hidden width 32 (16 inputs, 2 hidden layers) or 64 (2 or 3 hidden "
                   "layers)); the staged path takes any shape");
    *net = n;
    return NPM_OK;
}

// --------------------------------------------------------------------------
// Scratch of npm_backward_static, the entry point for callers that cannot
// allocate: one fixed array per device (each device holds its own copy of a
// __device__ array, at its own address, until the process ends).  In host
// code `scratch` names a host-side stand-in, never device memory: kernels and
// copies get the device address that hipGetSymbolAddress returns, resolved
// once per device by the first npm_create on it (with that device current).
static __device__ __align__(256) unsigned char scratch[NPM_STATIC_SCRATCH_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};
hipError_t g_scratch_err[kMaxDevices] = {};
bool g_scratch_done[kMaxDevices] = {};

// Byte offsets of the parts of the array for a batch of at most
// NPM_STATIC_MAX_N vertices: the sort's cell counters, the visiting order
// and its inverse, the input records (64 bytes with NPM-product inputs), the
// per-tile dG (at most 96 rows of 32 floats per 32-vertex tile).
constexpr size_t kScrCells = 0;
constexpr size_t kScrPerm = kScrCells + ((kSortCellWords * 4 + 255) / 256) * 256;
constexpr size_t kScrInv = kScrPerm + (size_t)NPM_STATIC_MAX_N * 4;
constexpr size_t kScrRec = kScrInv + (size_t)NPM_STATIC_MAX_N * 4;
constexpr size_t kScrDgt = kScrRec + (size_t)NPM_STATIC_MAX_N * 64;
constexpr size_t kScrEnd = kScrDgt + (size_t)(NPM_STATIC_MAX_N / 32) * 96 * 32 * 4;
static_assert(kScrEnd <= NPM_STATIC_SCRATCH_BYTES, "static scratch layout exceeds the array");
}  // namespace

// Resolves the array's address on device `dev` (the current device) once.
static void static_scratch_setup(int dev)
{
    if (dev < 0 || dev >= kMaxDevices) return;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch_done[dev]) return;
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    g_scratch_err[dev] = e;
    g_scratch_ptr[dev] = e == hipSuccess ? p : nullptr;
    g_scratch_done[dev] = true;
}

// The array's device address on `dev`, or null with the reason in *err.
static void *static_scratch(int dev, std::string *err)
{
    if (dev < 0 || dev >= kMaxDevices) {
        *err = "device index beyond the static scratch table";
        return nullptr;
    }
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev])
        *err = std::string("static scratch address not resolved: ") +
               (g_scratch_done[dev] ? hipGetErrorString(g_scratch_err[dev]) : "no context created");
    return g_scratch_ptr[dev];
}

// --------------------------------------------------------------------------
extern "C" {

const char *npm_last_error(void) { return g_err.c_str(); }

const char *npm_version(void) { return "npm-mi355x 0.1 (gfx950)"; }

npm_status npm_config_default(npm_config *cfg)
{
    if (!cfg) return fail(NPM_ERR_INVALID_ARG, "null cfg");
    std::memset(cfg, 0, sizeof(*cfg));
    cfg->grid_kind = NPM_GRID_HASH;
    cfg->n_levels = 16;
    cfg->feat_per_level = 2;
    cfg->log2_table_size = 19;
    cfg->base_resolution = 16;
    cfg->max_resolution = 2048;
    cfg->mlp_width = 64;
    cfg->mlp_hidden_layers = 2;
    cfg->n_lobes = kLobes;
    cfg->precision = NPM_PREC_FP32;
    cfg->exec_mode = NPM_EXEC_STAGED;
    cfg->grid_init = NPM_INIT_UNIFORM;
    cfg->grid_init_scale = 1e-4f;
    cfg->lr = 5e-3f;
    cfg->beta1 = 0.9f;
    cfg->beta2 = 0.999f;
    cfg->eps = 1e-8f;
    cfg->seed = 1;
    return NPM_OK;
}

npm_status npm_get_layout(const npm_config *cfg, npm_layout *out)
{
    if (!cfg || !out) return fail(NPM_ERR_INVALID_ARG, "null argument");
    Net net;
    std::string err;
    npm_status st = describe(cfg, &net, &err);
    if (st != NPM_OK) return fail(st, "invalid config: " + err);
    *out = net.lay;
    return NPM_OK;
}

static void free_scratch(npm_ctx *ctx)
{
    for (float **p : {&ctx->s_G, &ctx->s_raw, &ctx->s_acts, &ctx->s_delta, &ctx->s_draw, &ctx->s_dG}) {
        if (*p) (void)hipFree(*p);
        *p = nullptr;
    }
    ctx->scratch_n = 0;
}

static void free_ctx(npm_ctx *ctx)
{
    free_scratch(ctx);
    for (void *p : {(void *)ctx->params, (void *)ctx->grads, (void *)ctx->adam_m,
                    (void *)ctx->adam_v, ctx->grid16, (void *)ctx->mlp_img, ctx->mlp_img16,
                    (void *)ctx->partials, (void *)ctx->stats, (void *)ctx->s_dw_part,
                    (void *)ctx->s_perm, (void *)ctx->s_inv, (void *)ctx->s_rec,
                    (void *)ctx->s_qstage,
                    (void *)ctx->s_cells, (void *)ctx->s_dgt, (void *)ctx->s_bin_cnt,
                    (void *)ctx->s_bin_items,
                    (void *)ctx->ema, (void *)ctx->ema_img, ctx->ema_img16, ctx->ema_grid16})
        if (p) (void)hipFree(p);
    for (auto &p : ctx->timing.pending) { (void)hipEventDestroy(p.a); (void)hipEventDestroy(p.b); }
    for (auto e : ctx->timing.free_events) (void)hipEventDestroy(e);
    if (ctx->ev_fork) (void)hipEventDestroy(ctx->ev_fork);
    if (ctx->ev_join) (void)hipEventDestroy(ctx->ev_join);
    if (ctx->side) (void)hipStreamDestroy(ctx->side);
    delete ctx;
}

npm_status npm_create(const npm_config *cfg, npm_ctx **out)
{
    if (!cfg || !out) return fail(NPM_ERR_INVALID_ARG, "null argument");
    *out = nullptr;
    Net net;
    std::string err;
    npm_status st = describe(cfg, &net, &err);
    if (st != NPM_OK) return fail(st, "invalid config: " + err);
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0)
        return fail(NPM_ERR_NO_DEVICE, "no HIP device");
    int dev = 0;
    NPM_HIP(hipGetDevice(&dev), "hipGetDevice");
    hipDeviceProp_t prop;
    NPM_HIP(hipGetDeviceProperties(&prop, dev), "hipGetDeviceProperties");
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
        return fail(NPM_ERR_NO_DEVICE, std::string("device is ") + prop.gcnArchName +
                                           ", the library is built for gfx950");
    static_scratch_setup(dev);
    npm_ctx *ctx = new (std::nothrow) npm_ctx();
    if (!ctx) return fail(NPM_ERR_OOM, "host allocation");
    ctx->net = net;
    ctx->device = dev;
    const int64_t np = net.lay.n_params;
    const int64_t img = net.mlp.fwd_elems + net.mlp.bwd_elems;
    int64_t max_layer = 0;
    for (int i = 0; i < net.lay.n_layers; ++i)
        max_layer = std::max<int64_t>(max_layer, (int64_t)net.lay.layer_in[i] * net.lay.layer_out[i]);
    hipError_t e = hipSuccess;
    auto alloc = [&](void **p, size_t bytes) {
        if (e == hipSuccess) e = hipMalloc(p, bytes);
    };
    alloc((void **)&ctx->params, np * 4);
    alloc((void **)&ctx->grads, np * 4);
    alloc((void **)&ctx->adam_m, np * 4);
    alloc((void **)&ctx->adam_v, np * 4);
    alloc((void **)&ctx->mlp_img, (img + net.mlp.rm_elems) * 4);
    alloc((void **)&ctx->mlp_img16, img * 2);
    alloc((void **)&ctx->partials, kPartials * 8);
    alloc((void **)&ctx->stats, 64);
    // weight-gradient partials: 256 blocks x one layer (staged) or 1024 waves x
    // all MLP weights (fused)
    const int64_t mlp_w = np - net.lay.grid_params;
    alloc((void **)&ctx->s_dw_part, std::max<int64_t>(256 * max_layer, 1024 * mlp_w) * 4);
    if (net.cfg.precision == NPM_PREC_BF16) alloc(&ctx->grid16, net.lay.grid_params * 2);
    if (net.cfg.ema_decay > 0.0f) {
        alloc((void **)&ctx->ema, np * 4);
        alloc((void **)&ctx->ema_img, img * 4);
        alloc(&ctx->ema_img16, img * 2);
        if (net.cfg.precision == NPM_PREC_BF16) alloc(&ctx->ema_grid16, net.lay.grid_params * 2);
    }
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&ctx->side, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&ctx->ev_fork, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&ctx->ev_join, hipEventDisableTiming);
    if (e == hipSuccess) e = hipMemset(ctx->grads, 0, np * 4);
    if (e == hipSuccess) e = hipMemset(ctx->adam_m, 0, np * 4);
    if (e == hipSuccess) e = hipMemset(ctx->adam_v, 0, np * 4);
    if (e == hipSuccess) e = launch_init_params(ctx, nullptr);
    if (e == hipSuccess && ctx->ema)
        e = hipMemcpy(ctx->ema, ctx->params, np * 4, hipMemcpyDeviceToDevice);
    if (e == hipSuccess) e = launch_refresh_lowp(ctx, nullptr);
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e != hipSuccess) {
        free_ctx(ctx);
        return hip_fail(e, "npm_create");
    }
    *out = ctx;
    return NPM_OK;
}

npm_status npm_destroy(npm_ctx *ctx)
{
    if (!ctx) return NPM_OK;
    (void)hipDeviceSynchronize();   // the frees that follow synchronise too
    free_ctx(ctx);
    return NPM_OK;
}

static hipError_t ensure_scratch(npm_ctx *ctx, int64_t n)
{
    if (n <= ctx->scratch_n) return hipSuccess;
    // buffers may still be in use by queued work
    hipError_t e = hipDeviceSynchronize();
    if (e != hipSuccess) return e;
    free_scratch(ctx);
    const MlpDesc &m = ctx->net.mlp;
    const size_t f = sizeof(float);
    auto alloc = [&](float **p, int64_t elems) {
        if (e == hipSuccess) e = hipMalloc((void **)p, (size_t)elems * f);
    };
    alloc(&ctx->s_G, (int64_t)m.n_in * n);
    alloc(&ctx->s_raw, (int64_t)ctx->net.lay.n_out * n);
    alloc(&ctx->s_acts, (int64_t)m.n_hidden * m.width * n);
    alloc(&ctx->s_delta, (int64_t)m.n_hidden * m.width * n);
    alloc(&ctx->s_draw, (int64_t)ctx->net.lay.n_out * n);
    alloc(&ctx->s_dG, (int64_t)m.n_in * n);
    if (e != hipSuccess) { free_scratch(ctx); return e; }
    ctx->scratch_n = n;
    return hipSuccess;
}

static npm_status check_batch(npm_ctx *ctx, int64_t n, const float *pos)
{
    if (!ctx) return fail(NPM_ERR_INVALID_ARG, "null context");
    if (n < 0 || n > ((int64_t)1 << 31) - 1) return fail(NPM_ERR_INVALID_ARG, "n out of range");
    if (n > 0 && (!pos || !aligned4(pos))) return fail(NPM_ERR_INVALID_ARG, "pos must be a 4-byte aligned device pointer");
    return NPM_OK;
}

// The NPM-product inputs: required exactly when the network takes them.
static npm_status check_aux(npm_ctx *ctx, int64_t n, const float *aux)
{
    if (ctx->net.cfg.sh_degree > 0) {
        if (n > 0 && (!aux || !aligned4(aux)))
            return fail(NPM_ERR_INVALID_ARG, "this network takes omega_o, normal and roughness: "
                                             "use the *_aux calls with aux [7][n]");
    } else if (aux) {
        return fail(NPM_ERR_INVALID_ARG, "aux inputs given to a radiance-based network");
    }
    return NPM_OK;
}

static bool use_order(const npm_ctx *ctx, int64_t n, bool query = false);
static hipError_t ensure_sort(npm_ctx *ctx, int64_t n);
static hipError_t ensure_qstage(npm_ctx *ctx, int64_t n);

npm_status npm_query(npm_ctx *ctx, int64_t n, const float *pos, const float *dir,
                     uint64_t rng_seed, uint32_t rng_stream, float *lobes, float *pdf,
                     float *sample_dir, float *sample_pdf, void *stream)
{
    return npm_query_aux(ctx, n, pos, nullptr, dir, rng_seed, rng_stream, lobes, pdf, sample_dir,
                         sample_pdf, stream);
}

// The query of npm_query_aux and npm_query_select (sel: the selection
// probability, selection networks only).
static npm_status query_impl(npm_ctx *ctx, int64_t n, const float *pos, const float *aux,
                             const float *dir, uint64_t rng_seed, uint32_t rng_stream,
                             float *lobes, float *pdf, float *sample_dir, float *sample_pdf,
                             float *sel, hipStream_t s)
{
    const bool any = lobes || pdf || sample_dir || sample_pdf || sel;
    try {
        if (ctx->net.cfg.exec_mode == NPM_EXEC_FUSED) {
            const uint32_t *perm = nullptr;
            if (use_order(ctx, n, true) && any) {
                NPM_HIP(ensure_sort(ctx, n), "order scratch allocation");
                NPM_HIP(ensure_qstage(ctx, n), "query staging allocation");
                NPM_HIP(spatial_order(ctx, n, pos, aux, dir, nullptr, nullptr, ctx->s_perm,
                                      ctx->s_inv, ctx->s_rec, ctx->s_cells, s), "spatial order");
                perm = ctx->s_perm;
            }
            NPM_HIP(fused_query(ctx, n, pos, aux, dir, rng_seed, rng_stream, lobes, pdf,
                                sample_dir, sample_pdf, perm, ctx->s_inv, ctx->s_rec,
                                ctx->s_qstage, s, sel), "fused query");
            return NPM_OK;
        }
        NPM_HIP(ensure_scratch(ctx, n), "scratch allocation");
        const Weights w = query_weights(ctx);
        NPM_HIP(staged_encode(ctx, n, pos, ctx->s_G, s, &w, aux), "encode");
        NPM_HIP(staged_mlp_fwd(ctx, n, ctx->s_G, nullptr, ctx->s_raw, s, &w), "mlp forward");
        if (any)
            NPM_HIP(staged_head(ctx, n, ctx->s_raw, dir, rng_seed, rng_stream, lobes, pdf,
                                sample_dir, sample_pdf, s, sel), "head");
    } catch (...) {
        return fail(NPM_ERR_HIP, "unexpected exception");
    }
    return NPM_OK;
}

npm_status npm_query_aux(npm_ctx *ctx, int64_t n, const float *pos, const float *aux,
                         const float *dir, uint64_t rng_seed, uint32_t rng_stream, float *lobes,
                         float *pdf, float *sample_dir, float *sample_pdf, void *stream)
{
    npm_status st = check_batch(ctx, n, pos);
    if (st != NPM_OK) return st;
    if ((st = check_aux(ctx, n, aux)) != NPM_OK) return st;
    if (pdf && !dir) return fail(NPM_ERR_INVALID_ARG, "pdf needs dir");
    for (const void *p : {(const void *)dir, (const void *)lobes, (const void *)pdf,
                          (const void *)sample_dir, (const void *)sample_pdf})
        if (p && !aligned4(p)) return fail(NPM_ERR_INVALID_ARG, "misaligned buffer");
    if (n == 0) return NPM_OK;
    return query_impl(ctx, n, pos, aux, dir, rng_seed, rng_stream, lobes, pdf, sample_dir,
                      sample_pdf, nullptr, (hipStream_t)stream);
}

static npm_status check_train(npm_ctx *ctx, int64_t n, const float *pos, const float *dir,
                              const float *rad, const float *spdf)
{
    npm_status st = check_batch(ctx, n, pos);
    if (st != NPM_OK) return st;
    if (n > 0) {
        for (const void *p : {(const void *)dir, (const void *)rad, (const void *)spdf})
            if (!p || !aligned4(p))
                return fail(NPM_ERR_INVALID_ARG, "dir, radiance and sampling_pdf are required device pointers");
    }
    return NPM_OK;
}

// Whether a fused call visits a batch of n vertices in spatial order.  Auto
// sorts training batches of kSortMinBatch or more, and queries of that size
// on grids with hashed levels: on the paper's dense 8-level grid (16.5 MB)
// an unordered 921,600-vertex query takes 0.32 ms and an ordered one 0.44 ms
// with the sort and the un-permute, while on the 16-level hash grid ordering
// saves a fifth of the query.
static bool use_order(const npm_ctx *ctx, int64_t n, bool query)
{
    const int order = ctx->net.cfg.batch_order;
    const bool auto_sorts = n >= kSortMinBatch && (!query || ctx->net.grid.hashed_mask != 0);
    return ctx->net.cfg.exec_mode == NPM_EXEC_FUSED && n > 1 &&
           (order == NPM_ORDER_SPATIAL || (order == NPM_ORDER_AUTO && auto_sorts));
}

// The binned pass of a fused training batch: the plan, or false for the
// atomic scatter alone.
static bool use_bins(const npm_ctx *ctx, int64_t n, bool ordered, BinDesc *b)
{
    const int mode = ctx->net.cfg.scatter_mode;
    if (ctx->net.cfg.exec_mode != NPM_EXEC_FUSED || mode == NPM_SCATTER_ATOMIC) return false;
    if (mode == NPM_SCATTER_AUTO && n < kBinMinBatch) return false;
    if (!bin_plan(ctx, n, ordered, b)) return false;
    // a reduce of fewer blocks than compute units leaves most of the chip idle
    return mode == NPM_SCATTER_BINNED || b->nbins >= kBinMinBins;
}

static hipError_t ensure_bins(npm_ctx *ctx, const BinDesc &b)
{
    const size_t cw = bin_count_words(b), iw = bin_item_words(b, ctx->net.grid.feat);
    if (cw <= ctx->bin_cnt_words && iw <= ctx->bin_item_words) return hipSuccess;
    hipError_t e = hipDeviceSynchronize();
    if (e != hipSuccess) return e;
    if (cw > ctx->bin_cnt_words) {
        if (ctx->s_bin_cnt) (void)hipFree(ctx->s_bin_cnt);
        ctx->s_bin_cnt = nullptr;
        ctx->bin_cnt_words = 0;
        if ((e = hipMalloc((void **)&ctx->s_bin_cnt, cw * 4)) != hipSuccess) return e;
        ctx->bin_cnt_words = cw;
    }
    if (iw > ctx->bin_item_words) {
        if (ctx->s_bin_items) (void)hipFree(ctx->s_bin_items);
        ctx->s_bin_items = nullptr;
        ctx->bin_item_words = 0;
        if ((e = hipMalloc((void **)&ctx->s_bin_items, iw * 4)) != hipSuccess) return e;
        ctx->bin_item_words = iw;
    }
    return hipSuccess;
}

static hipError_t ensure_qstage(npm_ctx *ctx, int64_t n)
{
    if (n <= ctx->qstage_n) return hipSuccess;
    hipError_t e = hipDeviceSynchronize();
    if (e != hipSuccess) return e;
    if (ctx->s_qstage) (void)hipFree(ctx->s_qstage);
    ctx->s_qstage = nullptr;
    ctx->qstage_n = 0;
    e = hipMalloc((void **)&ctx->s_qstage, (size_t)n * 40 * sizeof(float));
    if (e != hipSuccess) return e;
    ctx->qstage_n = n;
    return hipSuccess;
}

static hipError_t ensure_sort(npm_ctx *ctx, int64_t n)
{
    if (n <= ctx->sort_n) return hipSuccess;
    hipError_t e = hipDeviceSynchronize();
    if (e != hipSuccess) return e;
    if (ctx->s_perm) (void)hipFree(ctx->s_perm);
    if (ctx->s_inv) (void)hipFree(ctx->s_inv);
    if (ctx->s_rec) (void)hipFree(ctx->s_rec);
    ctx->s_perm = ctx->s_inv = nullptr;
    ctx->s_rec = nullptr;
    ctx->sort_n = 0;
    e = hipMalloc((void **)&ctx->s_perm, (size_t)n * 4);
    if (e == hipSuccess) e = hipMalloc((void **)&ctx->s_inv, (size_t)n * 4);
    if (e == hipSuccess)
        e = hipMalloc((void **)&ctx->s_rec, (size_t)n * (ctx->net.cfg.sh_degree ? 64 : 32));
    if (e == hipSuccess && !ctx->s_cells)
        e = hipMalloc((void **)&ctx->s_cells, kSortCellWords * 4);  // counts, block totals
    if (e != hipSuccess) return e;
    ctx->sort_n = n;
    return hipSuccess;
}

static hipError_t ensure_dgt(npm_ctx *ctx, int64_t n)
{
    const int64_t tiles = (n + 31) / 32;
    if (tiles <= ctx->dgt_tiles) return hipSuccess;
    hipError_t e = hipDeviceSynchronize();
    if (e != hipSuccess) return e;
    if (ctx->s_dgt) (void)hipFree(ctx->s_dgt);
    ctx->s_dgt = nullptr;
    ctx->dgt_tiles = 0;
    const int64_t rows = std::max(ctx->net.mlp.in_p, 32);
    e = hipMalloc((void **)&ctx->s_dgt, (size_t)tiles * rows * 32 * sizeof(float));
    if (e != hipSuccess) return e;
    ctx->dgt_tiles = tiles;
    return hipSuccess;
}

// bsdf: the selection term's BSDF densities (selection networks), or null
static npm_status backward_impl(npm_ctx *ctx, int64_t n, const float *pos, const float *aux,
                                const float *dir, const float *rad, const float *spdf, float *grad,
                                double *loss_out, hipStream_t s, const float *bsdf = nullptr)
{
    if (ctx->net.cfg.exec_mode == NPM_EXEC_FUSED) {
        const uint32_t *perm = nullptr;
        if (grad && use_order(ctx, n)) {
            NPM_HIP(ensure_sort(ctx, n), "order scratch allocation");
            NPM_HIP(spatial_order(ctx, n, pos, aux, dir, rad, spdf, ctx->s_perm, ctx->s_inv,
                                  ctx->s_rec, ctx->s_cells, s), "spatial order");
            perm = ctx->s_perm;
        }
        if (grad) NPM_HIP(ensure_dgt(ctx, n), "dG scratch allocation");
        BinDesc bins;
        const bool binned = grad && use_bins(ctx, n, perm != nullptr, &bins);
        if (binned) NPM_HIP(ensure_bins(ctx, bins), "bin scratch allocation");
        NPM_HIP(fused_backward(ctx, n, pos, aux, dir, rad, spdf, grad, loss_out, perm,
                               perm ? ctx->s_rec : nullptr, grad ? ctx->s_dgt : nullptr,
                               binned ? &bins : nullptr, s, bsdf),
                "fused backward");
        return NPM_OK;
    }
    NPM_HIP(ensure_scratch(ctx, n), "scratch allocation");
    NPM_HIP(staged_encode(ctx, n, pos, ctx->s_G, s, nullptr, aux), "encode");
    NPM_HIP(staged_mlp_fwd(ctx, n, ctx->s_G, ctx->s_acts, ctx->s_raw, s), "mlp forward");
    NPM_HIP(staged_loss_grad(ctx, n, ctx->s_raw, dir, rad, spdf, ctx->s_draw, loss_out, s, bsdf),
            "loss gradient");
    NPM_HIP(staged_mlp_bwd(ctx, n, ctx->s_draw, ctx->s_acts, ctx->s_delta, ctx->s_dG, s),
            "mlp backward");
    NPM_HIP(staged_mlp_dw(ctx, n, ctx->s_G, ctx->s_acts, ctx->s_delta, ctx->s_draw, grad, s),
            "weight gradient");
    NPM_HIP(staged_scatter(ctx, n, pos, ctx->s_dG, grad, s), "grid scatter");
    return NPM_OK;
}

npm_status npm_backward(npm_ctx *ctx, int64_t n, const float *pos, const float *dir,
                        const float *radiance, const float *sampling_pdf, float *grad_out,
                        double *loss_out, void *stream)
{
    return npm_backward_aux(ctx, n, pos, nullptr, dir, radiance, sampling_pdf, grad_out, loss_out,
                            stream);
}

npm_status npm_backward_aux(npm_ctx *ctx, int64_t n, const float *pos, const float *aux,
                            const float *dir, const float *radiance, const float *sampling_pdf,
                            float *grad_out, double *loss_out, void *stream)
{
    npm_status st = check_train(ctx, n, pos, dir, radiance, sampling_pdf);
    if (st != NPM_OK) return st;
    if ((st = check_aux(ctx, n, aux)) != NPM_OK) return st;
    if (grad_out && !aligned4(grad_out)) return fail(NPM_ERR_INVALID_ARG, "misaligned grad_out");
    if (n == 0) return NPM_OK;
    try {
        return backward_impl(ctx, n, pos, aux, dir, radiance, sampling_pdf,
                             grad_out ? grad_out : ctx->grads, loss_out, (hipStream_t)stream);
    } catch (...) {
        return fail(NPM_ERR_HIP, "unexpected exception");
    }
}

npm_status npm_backward_static(npm_ctx *ctx, int64_t n, const float *pos, const float *aux,
                               const float *dir, const float *radiance, const float *sampling_pdf,
                               float *grad_out, double *loss_out, void *stream)
{
    npm_status st = check_train(ctx, n, pos, dir, radiance, sampling_pdf);
    if (st != NPM_OK) return st;
    if ((st = check_aux(ctx, n, aux)) != NPM_OK) return st;
    if (grad_out && !aligned4(grad_out)) return fail(NPM_ERR_INVALID_ARG, "misaligned grad_out");
    if (n > NPM_STATIC_MAX_N)
        return fail(NPM_ERR_INVALID_ARG, "npm_backward_static takes at most NPM_STATIC_MAX_N = " +
                                             std::to_string(NPM_STATIC_MAX_N) +
                                             " vertices (its scratch is a fixed array); got " +
                                             std::to_string(n));
    if (ctx->net.cfg.exec_mode != NPM_EXEC_FUSED)
        return fail(NPM_ERR_STATE, "npm_backward_static runs the fused path: the context must be "
                                   "NPM_EXEC_FUSED");
    if (ctx->net.mlp.in_p > 96) return fail(NPM_ERR_STATE, "network input too wide for the static scratch");
    if (n == 0) return NPM_OK;
    std::string why;
    unsigned char *base = (unsigned char *)static_scratch(ctx->device, &why);
    if (!base) return fail(NPM_ERR_HIP, why);
    uint32_t *cells = (uint32_t *)(base + kScrCells);
    uint32_t *perm = (uint32_t *)(base + kScrPerm);
    uint32_t *inv = (uint32_t *)(base + kScrInv);
    float *rec = (float *)(base + kScrRec);
    float *dgt = (float *)(base + kScrDgt);
    float *grad = grad_out ? grad_out : ctx->grads;
    hipStream_t s = (hipStream_t)stream;
    // no event pairs: timing would create events, which allocates
    const bool timing = ctx->timing.enabled;
    ctx->timing.enabled = false;
    hipError_t e = hipSuccess;
    const bool ordered = use_order(ctx, n);
    try {
        // every part of the array a kernel reads below is written earlier in
        // this call: the sort zeroes its counters with a kernel and writes the
        // order, its inverse and the records of the n slots; the tile kernel
        // writes every dG row the scatter reads, for every tile of the batch
        if (ordered)
            e = spatial_order(ctx, n, pos, aux, dir, radiance, sampling_pdf, perm, inv, rec, cells,
                              s);
        if (e == hipSuccess)
            e = fused_backward(ctx, n, pos, aux, dir, radiance, sampling_pdf, grad, loss_out,
                               ordered ? perm : nullptr, ordered ? rec : nullptr, dgt, nullptr, s);
    } catch (...) {
        ctx->timing.enabled = timing;
        return fail(NPM_ERR_HIP, "unexpected exception");
    }
    ctx->timing.enabled = timing;
    if (e != hipSuccess) return hip_fail(e, "static backward");
    return NPM_OK;
}

npm_status npm_loss(npm_ctx *ctx, int64_t n, const float *pos, const float *dir,
                    const float *radiance, const float *sampling_pdf, double *loss_out,
                    void *stream)
{
    return npm_loss_aux(ctx, n, pos, nullptr, dir, radiance, sampling_pdf, loss_out, stream);
}

npm_status npm_loss_aux(npm_ctx *ctx, int64_t n, const float *pos, const float *aux,
                        const float *dir, const float *radiance, const float *sampling_pdf,
                        double *loss_out, void *stream)
{
    npm_status st = check_train(ctx, n, pos, dir, radiance, sampling_pdf);
    if (st != NPM_OK) return st;
    if ((st = check_aux(ctx, n, aux)) != NPM_OK) return st;
    if (n == 0) return NPM_OK;
    hipStream_t s = (hipStream_t)stream;
    try {
        NPM_HIP(ensure_scratch(ctx, n), "scratch allocation");
        if (ctx->net.cfg.exec_mode == NPM_EXEC_FUSED && ctx->net.cfg.precision == NPM_PREC_BF16) {
            // the loss of the precision form: the fused kernel with no gradient output
            NPM_HIP(fused_backward(ctx, n, pos, aux, dir, radiance, sampling_pdf, nullptr,
                                   loss_out, nullptr, nullptr, nullptr, nullptr, s), "fused loss");
            return NPM_OK;
        }
        NPM_HIP(staged_encode(ctx, n, pos, ctx->s_G, s, nullptr, aux), "encode");
        NPM_HIP(staged_mlp_fwd(ctx, n, ctx->s_G, nullptr, ctx->s_raw, s), "mlp forward");
        NPM_HIP(staged_loss_grad(ctx, n, ctx->s_raw, dir, radiance, sampling_pdf, ctx->s_draw,
                                 loss_out, s), "loss");
    } catch (...) {
        return fail(NPM_ERR_HIP, "unexpected exception");
    }
    return NPM_OK;
}

npm_status npm_optimizer_step(npm_ctx *ctx, float *grad, double *gradnorm_out, void *stream)
{
    if (!ctx) return fail(NPM_ERR_INVALID_ARG, "null context");
    if (grad && !aligned4(grad)) return fail(NPM_ERR_INVALID_ARG, "misaligned grad");
    ctx->step += 1;
    hipError_t e = launch_adam(ctx, grad ? grad : ctx->grads, gradnorm_out, (hipStream_t)stream);
    if (e != hipSuccess) {
        ctx->step -= 1;
        return hip_fail(e, "adam");
    }
    return NPM_OK;
}

npm_status npm_train_step(npm_ctx *ctx, int64_t n, const float *pos, const float *dir,
                          const float *radiance, const float *sampling_pdf, double *stats_out,
                          void *stream)
{
    return npm_train_step_aux(ctx, n, pos, nullptr, dir, radiance, sampling_pdf, stats_out,
                              stream);
}

npm_status npm_train_step_aux(npm_ctx *ctx, int64_t n, const float *pos, const float *aux,
                              const float *dir, const float *radiance, const float *sampling_pdf,
                              double *stats_out, void *stream)
{
    npm_status st = check_train(ctx, n, pos, dir, radiance, sampling_pdf);
    if (st != NPM_OK) return st;
    if ((st = check_aux(ctx, n, aux)) != NPM_OK) return st;
    if (n > 0) {
        try {
            st = backward_impl(ctx, n, pos, aux, dir, radiance, sampling_pdf, ctx->grads,
                               stats_out, (hipStream_t)stream);
        } catch (...) {
            return fail(NPM_ERR_HIP, "unexpected exception");
        }
        if (st != NPM_OK) return st;
    }
    return npm_optimizer_step(ctx, nullptr, stats_out ? stats_out + 1 : nullptr, stream);
}

// ---------------------------------------------------------------------------
// Learned BSDF-selection probability
static npm_status check_select(npm_ctx *ctx)
{
    if (!ctx) return fail(NPM_ERR_INVALID_ARG, "null context");
    if (!ctx->net.cfg.learn_selection)
        return fail(NPM_ERR_STATE, "the network has no selection output (learn_selection = 0)");
    return NPM_OK;
}

npm_status npm_query_select(npm_ctx *ctx, int64_t n, const float *pos, const float *aux,
                            const float *dir, uint64_t rng_seed, uint32_t rng_stream,
                            float *lobes, float *pdf, float *sample_dir, float *sample_pdf,
                            float *select_prob, void *stream)
{
    npm_status st = check_select(ctx);
    if (st != NPM_OK) return st;
    if ((st = check_batch(ctx, n, pos)) != NPM_OK) return st;
    if ((st = check_aux(ctx, n, aux)) != NPM_OK) return st;
    if (pdf && !dir) return fail(NPM_ERR_INVALID_ARG, "pdf needs dir");
    for (const void *p : {(const void *)dir, (const void *)lobes, (const void *)pdf,
                          (const void *)sample_dir, (const void *)sample_pdf,
                          (const void *)select_prob})
        if (p && !aligned4(p)) return fail(NPM_ERR_INVALID_ARG, "misaligned buffer");
    if (n == 0) return NPM_OK;
    return query_impl(ctx, n, pos, aux, dir, rng_seed, rng_stream, lobes, pdf, sample_dir,
                      sample_pdf, select_prob, (hipStream_t)stream);
}

static npm_status check_train_select(npm_ctx *ctx, int64_t n, const float *pos, const float *aux,
                                     const float *dir, const float *rad, const float *spdf,
                                     const float *bsdf)
{
    npm_status st = check_select(ctx);
    if (st != NPM_OK) return st;
    if ((st = check_train(ctx, n, pos, dir, rad, spdf)) != NPM_OK) return st;
    if ((st = check_aux(ctx, n, aux)) != NPM_OK) return st;
    if (n > 0 && (!bsdf || !aligned4(bsdf)))
        return fail(NPM_ERR_INVALID_ARG, "bsdf_pdf is a required device pointer");
    return NPM_OK;
}

npm_status npm_backward_select(npm_ctx *ctx, int64_t n, const float *pos, const float *aux,
                               const float *dir, const float *radiance,
                               const float *sampling_pdf, const float *bsdf_pdf,
                               float *grad_out, double *loss_out, void *stream)
{
    npm_status st = check_train_select(ctx, n, pos, aux, dir, radiance, sampling_pdf, bsdf_pdf);
    if (st != NPM_OK) return st;
    if (grad_out && !aligned4(grad_out)) return fail(NPM_ERR_INVALID_ARG, "misaligned grad_out");
    if (n == 0) return NPM_OK;
    try {
        return backward_impl(ctx, n, pos, aux, dir, radiance, sampling_pdf,
                             grad_out ? grad_out : ctx->grads, loss_out, (hipStream_t)stream,
                             bsdf_pdf);
    } catch (...) {
        return fail(NPM_ERR_HIP, "unexpected exception");
    }
}

npm_status npm_train_step_select(npm_ctx *ctx, int64_t n, const float *pos, const float *aux,
                                 const float *dir, const float *radiance,
                                 const float *sampling_pdf, const float *bsdf_pdf,
                                 double *stats_out, void *stream)
{
    npm_status st = check_train_select(ctx, n, pos, aux, dir, radiance, sampling_pdf, bsdf_pdf);
    if (st != NPM_OK) return st;
    if (n > 0) {
        try {
            st = backward_impl(ctx, n, pos, aux, dir, radiance, sampling_pdf, ctx->grads,
                               stats_out, (hipStream_t)stream, bsdf_pdf);
        } catch (...) {
            return fail(NPM_ERR_HIP, "unexpected exception");
        }
        if (st != NPM_OK) return st;
    }
    return npm_optimizer_step(ctx, nullptr, stats_out ? stats_out + 2 : nullptr, stream);
}

npm_status npm_corner_index(npm_ctx *ctx, int64_t n, const float *pos, uint32_t *idx, void *stream)
{
    npm_status st = check_batch(ctx, n, pos);
    if (st != NPM_OK) return st;
    if (n > 0 && (!idx || !aligned4(idx))) return fail(NPM_ERR_INVALID_ARG, "idx required");
    if (n == 0) return NPM_OK;
    NPM_HIP(staged_corner_index(ctx, n, pos, idx, (hipStream_t)stream), "corner index");
    return NPM_OK;
}

npm_status npm_encode(npm_ctx *ctx, int64_t n, const float *pos, float *G, void *stream)
{
    return npm_encode_aux(ctx, n, pos, nullptr, G, stream);
}

npm_status npm_encode_aux(npm_ctx *ctx, int64_t n, const float *pos, const float *aux, float *G,
                          void *stream)
{
    npm_status st = check_batch(ctx, n, pos);
    if (st != NPM_OK) return st;
    if ((st = check_aux(ctx, n, aux)) != NPM_OK) return st;
    if (n > 0 && (!G || !aligned4(G))) return fail(NPM_ERR_INVALID_ARG, "G required");
    if (n == 0) return NPM_OK;
    const Weights w = query_weights(ctx);
    NPM_HIP(staged_encode(ctx, n, pos, G, (hipStream_t)stream, &w, aux), "encode");
    return NPM_OK;
}

npm_status npm_forward_raw(npm_ctx *ctx, int64_t n, const float *pos, float *raw, void *stream)
{
    return npm_forward_raw_aux(ctx, n, pos, nullptr, raw, stream);
}

npm_status npm_forward_raw_aux(npm_ctx *ctx, int64_t n, const float *pos, const float *aux,
                               float *raw, void *stream)
{
    npm_status st = check_batch(ctx, n, pos);
    if (st != NPM_OK) return st;
    if ((st = check_aux(ctx, n, aux)) != NPM_OK) return st;
    if (n > 0 && (!raw || !aligned4(raw))) return fail(NPM_ERR_INVALID_ARG, "raw required");
    if (n == 0) return NPM_OK;
    hipStream_t s = (hipStream_t)stream;
    NPM_HIP(ensure_scratch(ctx, n), "scratch allocation");
    const Weights w = query_weights(ctx);
    NPM_HIP(staged_encode(ctx, n, pos, ctx->s_G, s, &w, aux), "encode");
    NPM_HIP(staged_mlp_fwd(ctx, n, ctx->s_G, nullptr, raw, s, &w), "mlp forward");
    return NPM_OK;
}

static float *state_buf(npm_ctx *ctx, int which)
{
    switch (which) {
    case NPM_STATE_PARAMS: return ctx->params;
    case NPM_STATE_GRADS: return ctx->grads;
    case NPM_STATE_ADAM_M: return ctx->adam_m;
    case NPM_STATE_ADAM_V: return ctx->adam_v;
    case NPM_STATE_EMA: return ctx->ema;
    default: return nullptr;
    }
}

npm_status npm_get_state(npm_ctx *ctx, int which, float *host, int64_t count)
{
    if (!ctx || !host) return fail(NPM_ERR_INVALID_ARG, "null argument");
    float *src = state_buf(ctx, which);
    if (which == NPM_STATE_EMA && !src) return fail(NPM_ERR_STATE, "no moving average is kept");
    if (!src) return fail(NPM_ERR_INVALID_ARG, "unknown state buffer");
    if (count != ctx->net.lay.n_params) return fail(NPM_ERR_INVALID_ARG, "count must equal n_params");
    NPM_HIP(hipDeviceSynchronize(), "synchronize");
    NPM_HIP(hipMemcpy(host, src, count * 4, hipMemcpyDeviceToHost), "copy state");
    return NPM_OK;
}

npm_status npm_set_state(npm_ctx *ctx, int which, const float *host, int64_t count)
{
    if (!ctx || !host) return fail(NPM_ERR_INVALID_ARG, "null argument");
    float *dst = state_buf(ctx, which);
    if (which == NPM_STATE_EMA && !dst) return fail(NPM_ERR_STATE, "no moving average is kept");
    if (!dst) return fail(NPM_ERR_INVALID_ARG, "unknown state buffer");
    if (count != ctx->net.lay.n_params) return fail(NPM_ERR_INVALID_ARG, "count must equal n_params");
    NPM_HIP(hipDeviceSynchronize(), "synchronize");
    NPM_HIP(hipMemcpy(dst, host, count * 4, hipMemcpyHostToDevice), "copy state");
    if (which == NPM_STATE_PARAMS && ctx->ema)      // the average restarts here
        NPM_HIP(hipMemcpy(ctx->ema, ctx->params, count * 4, hipMemcpyDeviceToDevice), "copy state");
    if (which == NPM_STATE_PARAMS || which == NPM_STATE_EMA) {
        NPM_HIP(launch_refresh_lowp(ctx, nullptr), "refresh packed weights");
        NPM_HIP(hipDeviceSynchronize(), "synchronize");
    }
    return NPM_OK;
}

npm_status npm_get_step(npm_ctx *ctx, int64_t *step)
{
    if (!ctx || !step) return fail(NPM_ERR_INVALID_ARG, "null argument");
    *step = ctx->step;
    return NPM_OK;
}

npm_status npm_set_step(npm_ctx *ctx, int64_t step)
{
    if (!ctx || step < 0) return fail(NPM_ERR_INVALID_ARG, "bad argument");
    ctx->step = step;
    return NPM_OK;
}

npm_status npm_state_device_ptr(npm_ctx *ctx, int which, void **ptr)
{
    if (!ctx || !ptr) return fail(NPM_ERR_INVALID_ARG, "null argument");
    float *p = state_buf(ctx, which);
    if (which == NPM_STATE_EMA && !p) return fail(NPM_ERR_STATE, "no moving average is kept");
    if (!p) return fail(NPM_ERR_INVALID_ARG, "unknown state buffer");
    *ptr = p;
    return NPM_OK;
}

npm_status npm_set_timing(npm_ctx *ctx, int enabled)
{
    if (!ctx) return fail(NPM_ERR_INVALID_ARG, "null context");
    ctx->timing.enabled = enabled != 0;
    return NPM_OK;
}

static hipError_t collect_timing(npm_ctx *ctx)
{
    Timing &t = ctx->timing;
    if (t.pending.empty()) return hipSuccess;
    hipError_t e = hipDeviceSynchronize();
    if (e != hipSuccess) return e;
    for (auto &p : t.pending) {
        float ms = 0.0f;
        if (hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
            t.total_ms[p.id] += ms;
            t.launches[p.id] += 1;
        }
        t.free_events.push_back(p.a);
        t.free_events.push_back(p.b);
    }
    t.pending.clear();
    return hipSuccess;
}

npm_status npm_kernel_times(npm_ctx *ctx, npm_kernel_time *out, int32_t cap, int32_t *count)
{
    if (!ctx || !count || (cap > 0 && !out)) return fail(NPM_ERR_INVALID_ARG, "null argument");
    NPM_HIP(collect_timing(ctx), "collect timing");
    const Timing &t = ctx->timing;
    const int nk = (int)t.names.size();
    for (int i = 0; i < nk && i < cap; ++i) {
        std::memset(out[i].name, 0, sizeof(out[i].name));
        std::strncpy(out[i].name, t.names[i].c_str(), sizeof(out[i].name) - 1);
        out[i].launches = t.launches[i];
        out[i].total_ms = t.total_ms[i];
    }
    *count = nk;
    return NPM_OK;
}

npm_status npm_reset_timing(npm_ctx *ctx)
{
    if (!ctx) return fail(NPM_ERR_INVALID_ARG, "null context");
    NPM_HIP(collect_timing(ctx), "collect timing");
    Timing &t = ctx->timing;
    std::fill(t.launches.begin(), t.launches.end(), 0);
    std::fill(t.total_ms.begin(), t.total_ms.end(), 0.0);
    return NPM_OK;
}

}  // extern "C"
