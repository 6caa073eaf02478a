// Internal host-side declarations of libnpm: the context, the derived network
// description, and the launchers each kernel file provides.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "npm.h"

namespace npm {

constexpr int kLobes = 8;             // K (Sec. 5.3)
constexpr int kOut = 4 * kLobes;      // lobe raw outputs per vertex (a selection
                                      // network has one more, the logit, at kOut)
constexpr int kWave = 64;             // CDNA wavefront
constexpr int kTile = 32;             // vertices per wave tile (32x32 MFMA)

// Grid description passed to kernels by value.
struct GridDesc {
    uint32_t offset[NPM_MAX_LEVELS];  // first entry of each level
    int32_t res[NPM_MAX_LEVELS];      // D_l
    uint32_t hashed_mask;             // bit l set: level l is hashed
    uint32_t table_mask;              // 2^log2T - 1
    int32_t n_levels;
    int32_t feat;
};

// MLP shape as the kernels see it: widths padded to MFMA tiles.
struct MlpDesc {
    int n_in, width, n_hidden;        // real sizes
    int in_p, hid_p;                  // padded: in_p in {16, 32, 64, 96}, hid_p in {32, 64}
    int gf;                           // grid features (n_levels * feat), the first inputs
    int sh_degree;                    // NPM-product: SH bands of omega_o and the normal
    int64_t fwd_off[NPM_MAX_LAYERS];  // offset of each layer's image in the packed
    int64_t bwd_off[NPM_MAX_LAYERS];  //   forward / backward weight images (elements)
    int64_t fwd_elems, bwd_elems;
    // Row-major FP32 image of the training kernel: layer L as its padded
    // out_p x c_L matrix (c_0 = max(in_p, 32), c_L = hid_p otherwise) with
    // rows c_L + 1 floats apart, read as W (forward) and as W^T (backward)
    int64_t rm_off[NPM_MAX_LAYERS];
    int64_t rm_elems;
};

struct Net {
    npm_config cfg;
    npm_layout lay;
    GridDesc grid;
    MlpDesc mlp;
};

// Fills *net from *cfg; returns NPM_OK or NPM_ERR_INVALID_ARG with a message.
npm_status describe(const npm_config *cfg, Net *net, std::string *err);

// Sets the calling thread's npm_last_error() message.
void set_error(const char *msg);

// Per-kernel event timing.
struct Timing {
    bool enabled = false;
    std::vector<std::string> names;
    std::vector<int64_t> launches;
    std::vector<double> total_ms;
    struct Pending { int id; hipEvent_t a, b; };
    std::vector<Pending> pending;
    std::vector<hipEvent_t> free_events;
};

}  // namespace npm

struct npm_ctx {
    npm::Net net;
    int device = 0;
    int64_t step = 0;
    // FP32 master state, n_params each
    float *params = nullptr, *grads = nullptr, *adam_m = nullptr, *adam_v = nullptr;
    // Low-precision copies (NPM_PREC_BF16): FP16 grid, BF16 packed MLP images
    void *grid16 = nullptr;
    // Packed MLP weight images (forward and backward), FP32 and BF16
    float *mlp_img = nullptr;          // [fwd_elems + bwd_elems + rm_elems] FP32
    void *mlp_img16 = nullptr;         // [fwd_elems + bwd_elems] BF16
    // Exponential moving average of the parameters (ema_decay > 0): FP32
    // master, its packed images and (NPM_PREC_BF16) its FP16 grid
    float *ema = nullptr, *ema_img = nullptr;
    void *ema_img16 = nullptr, *ema_grid16 = nullptr;
    // FP64 reduction scratch
    double *partials = nullptr;        // kPartials doubles
    double *stats = nullptr;           // 4 doubles: loss, gradnorm, spare
    // Staged-path scratch, grown on demand
    int64_t scratch_n = 0;
    float *s_G = nullptr, *s_raw = nullptr, *s_acts = nullptr, *s_delta = nullptr,
          *s_draw = nullptr, *s_dG = nullptr;
    float *s_dw_part = nullptr;        // dW partials
    int64_t dw_part_elems = 0;
    // spatial order of a training batch (fused path)
    uint32_t *s_perm = nullptr;        // [sort_n] visiting slot -> vertex
    uint32_t *s_inv = nullptr;         // [sort_n] vertex -> visiting slot
    float *s_rec = nullptr;            // [sort_n][8] inputs in visiting order
    float *s_qstage = nullptr;         // [qstage_n][40] staged query outputs
    int64_t qstage_n = 0;
    uint32_t *s_cells = nullptr;       // 2^18 cell counts / offsets, 256 block totals
    int64_t sort_n = 0;
    // per-tile dG of a fused training batch, for the aggregated scatter
    float *s_dgt = nullptr;            // [dgt_tiles][max(in_p, 32)][32]
    int64_t dgt_tiles = 0;
    // binned scatter of the hashed levels: per-chunk bin counts / offsets
    // (and the scan's block totals), and the binned items
    uint32_t *s_bin_cnt = nullptr, *s_bin_items = nullptr;
    size_t bin_cnt_words = 0, bin_item_words = 0;
    // a second stream (default priority) on which the windowed scatter and
    // the weight-gradient sum run beside the binned scatter, forked from and
    // joined back to the caller's stream by the two events
    hipStream_t side = nullptr;
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    npm::Timing timing;
};

namespace npm {

constexpr int kPartials = 4096;        // FP64 partial slots per reduction

// The weights a kernel reads: the trained ones, or, for the network npm_query
// evaluates, their moving average when it is kept.
struct Weights {
    const float *grid32;      // FP32 grid (the head of the flat parameters)
    const void *grid16;       // FP16 grid (precision form) or null
    const float *img;         // packed FP32 images
    const void *img16;        // packed BF16 images
};
inline Weights trained_weights(const npm_ctx *c)
{
    return Weights{c->params, c->grid16, c->mlp_img, c->mlp_img16};
}
inline Weights query_weights(const npm_ctx *c)
{
    return c->ema ? Weights{c->ema, c->ema_grid16, c->ema_img, c->ema_img16} : trained_weights(c);
}

// The selection row of the last layer within the flat parameters `flat`
// (width FP32 weights after the output layer's 4K rows), or null when the
// network has no selection output.
inline const float *selection_row(const npm_ctx *c, const float *flat)
{
    const npm_layout &L = c->net.lay;
    if (!c->net.cfg.learn_selection) return nullptr;
    return flat + L.layer_offset[L.n_layers - 1] + (int64_t)kOut * c->net.mlp.width;
}

// ---------------------------------------------------------------- launchers
// All return hipSuccess or the first launch error.  `s` is the stream.
struct Launch {
    npm_ctx *ctx;
    hipStream_t s;
};

// Timing bracket (no-op unless enabled).
void timed_begin(npm_ctx *ctx, const char *name, hipStream_t s, int *token);
void timed_end(npm_ctx *ctx, int token, hipStream_t s);

// common kernels (k_common.hip)
hipError_t launch_init_params(npm_ctx *ctx, hipStream_t s);
// packs the MLP images of the parameters (and of their average when kept)
hipError_t launch_pack_mlp(npm_ctx *ctx, hipStream_t s);
// repacks the images and rewrites the FP16 grids from the FP32 masters
hipError_t launch_refresh_lowp(npm_ctx *ctx, hipStream_t s);
hipError_t launch_adam(npm_ctx *ctx, float *grad, double *gradnorm_out, hipStream_t s);
hipError_t launch_reduce_partials(npm_ctx *ctx, int nparts, double *out, hipStream_t s);
hipError_t launch_reduce_scaled(const double *part, int nparts, double scale, double *out,
                                hipStream_t s);
hipError_t launch_fill_f32(float *p, int64_t n, float v, hipStream_t s);

// staged path (k_staged.hip)
hipError_t staged_corner_index(npm_ctx *ctx, int64_t n, const float *pos, uint32_t *idx,
                               hipStream_t s);
// w: the weights to evaluate (the trained ones by default)
// aux: the NPM-product inputs [7][n] (required when the network takes them)
hipError_t staged_encode(npm_ctx *ctx, int64_t n, const float *pos, float *G, hipStream_t s,
                         const Weights *w = nullptr, const float *aux = nullptr);
hipError_t staged_mlp_fwd(npm_ctx *ctx, int64_t n, const float *G, float *acts, float *raw,
                          hipStream_t s, const Weights *w = nullptr);
// sel (or null): the selection probability of each vertex (selection networks)
hipError_t staged_head(npm_ctx *ctx, int64_t n, const float *raw, const float *dir,
                       uint64_t seed, uint32_t stream_id, float *lobes, float *pdf,
                       float *sdir, float *spdf, hipStream_t s, float *sel = nullptr);
// bsdf (or null): the BSDF density of each sample, for the selection term of a
// network with the selection output; its loss then goes to loss_out[1]
hipError_t staged_loss_grad(npm_ctx *ctx, int64_t n, const float *raw, const float *dir,
                            const float *rad, const float *spdf, float *draw, double *loss_out,
                            hipStream_t s, const float *bsdf = nullptr);
hipError_t staged_mlp_bwd(npm_ctx *ctx, int64_t n, const float *draw, const float *acts,
                          float *delta, float *dG, hipStream_t s);
hipError_t staged_mlp_dw(npm_ctx *ctx, int64_t n, const float *G, const float *acts,
                         const float *delta, const float *draw, float *grad, hipStream_t s);
hipError_t staged_scatter(npm_ctx *ctx, int64_t n, const float *pos, const float *dG,
                          float *grad, hipStream_t s);

// spatial order of a batch (k_sort.hip): perm lists the vertices by cell,
// inv (required, n entries) receives its inverse
hipError_t spatial_order(npm_ctx *ctx, int64_t n, const float *pos, const float *aux,
                         const float *dir, const float *rad, const float *spdf, uint32_t *perm,
                         uint32_t *inv, float *rec, uint32_t *cells, hipStream_t s);
// Smallest batch NPM_ORDER_AUTO sorts.  On the 16-level hash grid at 2^20
// vertices the sort (0.22 ms) halves the scatter's line requests through the
// LDS window (4.43 -> 2.42 ms) and speeds the tile kernel's gathers (1.61 ->
// 1.28 ms); a batch of 2^15 vertices is still dense enough for the window to
// cover the coarse levels.
constexpr int64_t kSortMinBatch = 1 << 15;
// 32-bit words of the sort's cell scratch: 2^18 cell counters, then 256
// block totals of its scan.
constexpr size_t kSortCellWords = ((size_t)1 << 18) + 256;

// Binned scatter of the hashed levels (k_bin.hip).  The corner contributions
// of a training batch are binned by (level, table slice) in chunks of
// kBinChunk visiting slots, as pairs of x-neighbour corners (which the hash
// keeps in one slice), and each bin (a slice of kBinSliceFloats table floats)
// is summed by one block in LDS, replacing one memory-side FP32 atomic per
// corner.
constexpr int kBinChunk = 1024;           // 512 with one item per corner (its LDS then capped it)
constexpr int kBinSliceFloats = 16384;      // table floats per bin (8,192 entries at F = 2)
constexpr int kBinReduceThreads = 1024;
constexpr int kBinReduceBatch = 4;         // items in flight per thread
constexpr int kBinMaxBins = 2048;
constexpr int kBinMaxSlices = 1024;
// Smallest batch NPM_SCATTER_AUTO bins (the count, scan, place and reduce
// launches cost a few microseconds each).
constexpr int64_t kBinMinBatch = 1 << 15;
// ... and only grids whose binned levels split into this many slices (small
// tables leave the reduce too few blocks).
constexpr int kBinMinBins = 256;
// In a spatially ordered batch the hashed levels with D_l below this mostly
// fit the tile's LDS window and stay with the windowed scatter (on the
// 16-level production grid binning from D_l >= 100 on beats binning every
// hashed level: 1.01 against 1.05 ms per 2^20-vertex batch).
constexpr int kBinMinResOrdered = 100;
struct BinDesc {
    int32_t nb;                        // binned levels
    int32_t lv[NPM_MAX_LEVELS];        // their indices
    int32_t log2s;                     // log2 of the table entries per slice
    int32_t ns;                        // slices per level
    int32_t nbins;                     // nb * ns
    int64_t n_chunks;                  // ceil(n / kBinChunk)
    int64_t cap;                       // item (corner pair) capacity: n * 4 * nb
};
// false when the batch has no level to bin or exceeds the pass's limits
bool bin_plan(const npm_ctx *ctx, int64_t n, bool ordered, BinDesc *out);
size_t bin_count_words(const BinDesc &b);
size_t bin_item_words(const BinDesc &b, int feat);
// dgt/rows: the per-tile dG of the batch in visiting order (perm / rec as
// for the fused backward); cnt and items: bin_count_words and
// bin_item_words 32-bit words
hipError_t binned_scatter(npm_ctx *ctx, const BinDesc &b, int64_t n, const float *pos,
                          const uint32_t *perm, const float *rec, int rec_stride,
                          const float *dgt, int rows, float *grad, uint32_t *cnt,
                          uint32_t *items, hipStream_t s);

// fused path (k_fused.hip)
// whether the fused kernels are instantiated for the network's shape (the
// dispatch tables of k_fused.hip)
bool fused_shape_supported(const Net &net);
// perm/inv (optional): visiting order and its inverse; the outputs then go
// through `stage` (n slots of 40 floats) and an un-permuting pass
hipError_t fused_query(npm_ctx *ctx, int64_t n, const float *pos, const float *aux,
                       const float *dir, uint64_t seed, uint32_t stream_id, float *lobes,
                       float *pdf, float *sdir, float *spdf, const uint32_t *perm,
                       const uint32_t *inv, const float *rec, float *stage, hipStream_t s,
                       float *sel = nullptr);
// perm (optional): the order in which to visit the vertices; dg_tiles: the
// per-tile dG buffer (required when grad is set); bins (optional): the levels
// to scatter through the binned pass, with the context's bin buffers
hipError_t fused_backward(npm_ctx *ctx, int64_t n, const float *pos, const float *aux,
                          const float *dir, const float *rad, const float *spdf, float *grad,
                          double *loss_out, const uint32_t *perm, const float *rec,
                          float *dg_tiles, const BinDesc *bins, hipStream_t s,
                          const float *bsdf = nullptr);

}  // namespace npm
