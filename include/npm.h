/*
 * npm.h -- C ABI of libnpm.so, the MI355X (gfx950) hot path of Neural
 * Parametric Mixtures (Dong, Wang, Li, "Neural Parametric Mixtures for Path
 * Guiding", SIGGRAPH 2023).
 *
 * A guiding network maps a shading position x to a K-lobe von Mises-Fisher
 * mixture (Sec. 4.1, eq. npmradiance): a multiresolution grid embedding G(x)
 * (Sec. 5.1) is decoded by a small ReLU MLP (Sec. 5.3) into raw outputs that
 * the Table 1 mappings turn into lobe parameters.  The library evaluates the
 * mixture, samples it (Sec. 5.3, Jakob 2012), and trains it by the Monte
 * Carlo KL gradient (Sec. 4.2, eq. mcgradients) with Adam.
 *
 * Conventions shared by every entry point:
 *   - Every call returns an npm_status; NPM_OK is 0, failures are negative
 *     and set a thread-local message readable with npm_last_error().  No C++
 *     exception crosses the ABI.  A call that fails validation changes
 *     nothing.
 *   - Batch buffers are DEVICE pointers owned by the caller, in
 *     structure-of-arrays layout: a [3][n] array holds all x, then all y,
 *     then all z.  Each pointer must be 4-byte aligned and stay valid until
 *     the work enqueued on `stream` completes.
 *   - Work is enqueued on the caller's HIP stream (`stream` is a hipStream_t;
 *     NULL is the null stream) and the call returns without waiting.
 *     Outputs are valid once the stream has reached the call.  Calls on one
 *     context must not run concurrently on different streams.  A fused
 *     training step may fork part of its grid scatter onto a stream of the
 *     context (default priority) and joins it back to `stream` with events
 *     before returning, so the caller's ordering on `stream` still holds.
 *   - n == 0 is a no-op that returns NPM_OK.  Optional outputs may be NULL,
 *     and the work that only feeds them is skipped.
 *   - The library owns parameters, gradients, Adam state and scratch; they
 *     live in device memory allocated by npm_create and released by
 *     npm_destroy.
 *
 * Flat parameter layout (used by npm_get_state / npm_set_state): the grid
 * tables first, level after level, entry-major with F features per entry
 * (feature f of entry e of level l at (offset_l + e) * F + f); then the MLP
 * weight matrices W_0 .. W_{hidden}, each row-major [out][in].  The MLP has
 * no biases.  With learn_selection the last matrix has 4K + 1 rows, the
 * selection logit's last.
 */
#ifndef NPM_H
#define NPM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    NPM_OK = 0,
    NPM_ERR_INVALID_ARG = -1, /* bad pointer, size or configuration          */
    NPM_ERR_NO_DEVICE = -2,   /* no usable gfx950 device                     */
    NPM_ERR_OOM = -3,         /* device allocation failed                    */
    NPM_ERR_BUDGET = -4,      /* serving: session does not fit the budget    */
    NPM_ERR_HIP = -5,         /* a HIP runtime call failed                   */
    NPM_ERR_STATE = -6,       /* call not valid in the object's state        */
    NPM_ERR_TIMEOUT = -7      /* serving: wait timed out                     */
} npm_status;

enum { NPM_GRID_DENSE = 0, NPM_GRID_HASH = 1 };
/* NPM_PREC_BF16: MLP weights and activations in bfloat16 on MFMA with FP32
 * accumulation, grid features stored in FP16; the output mappings, softmax,
 * log-density and sampling stay in FP32; Adam keeps FP32 master copies.     */
enum { NPM_PREC_FP32 = 0, NPM_PREC_BF16 = 1 };
/* NPM_EXEC_STAGED runs one kernel per step of the path with intermediate
 * buffers in HBM; NPM_EXEC_FUSED keeps a tile of vertices on chip from the
 * grid lookup to the sampled direction (and, in training, to the scatter).  */
enum { NPM_EXEC_STAGED = 0, NPM_EXEC_FUSED = 1 };
enum { NPM_INIT_NORMAL = 0, NPM_INIT_UNIFORM = 1 };
/* Order in which the fused path visits a batch.
 * NPM_ORDER_SPATIAL sorts the batch by the Morton code of each vertex's 64^3
 * cell (a counting sort on the device, kept in context scratch) so that a
 * wave's consecutive tiles touch nearby grid entries; NPM_ORDER_NONE keeps
 * the caller's order; NPM_ORDER_AUTO sorts training batches of 2^15
 * vertices or more, and queries of that size on grids with hashed levels
 * (on a small dense grid the gathers already hit the cache).
 * A query's outputs do not depend on the order (each vertex keeps its own
 * uniforms; the outputs are staged and un-permuted); a gradient changes only
 * in the order of its floating-point sums.                                  */
enum { NPM_ORDER_AUTO = 0, NPM_ORDER_NONE = 1, NPM_ORDER_SPATIAL = 2 };
/* How the fused training path adds the gradient into the grid's hashed
 * levels (Sec. 4.2 gradient through the interpolation of Sec. 5.1).
 * NPM_SCATTER_ATOMIC adds each corner's contribution with an FP32 atomic
 * (through a tile's LDS window where its corners fall together);
 * NPM_SCATTER_BINNED first bins the contributions of the hashed levels by
 * table slice and sums each slice in one block (in FP64, or in 64-bit fixed
 * point in the precision form; rounded once to FP32), then adds it to the
 * gradient.  Device scratch: 16 (1 + 2 F) n bytes
 * per binned level (80 n at F = 2), kept in the context.  In a spatially
 * ordered batch only the hashed levels with D_l >= 100 are binned; the others
 * keep the atomic path.  NPM_SCATTER_AUTO bins training batches of 2^15
 * vertices or more whose binned levels split into at least 256 slices
 * (16384 / F table entries each).  Both fall back to the atomic path when
 * the pass does not apply: no hashed level to bin, more than 2048 bins or
 * 1024 slices per level, or 2^32 items or more (n * 8 * binned levels).
 * Either way the gradient changes only in the order and width of its
 * floating-point sums.                                                     */
enum { NPM_SCATTER_AUTO = 0, NPM_SCATTER_ATOMIC = 1, NPM_SCATTER_BINNED = 2 };

/* Network configuration (copied at create).
 * Grid (Sec. 5.1): n_levels uniform grids over the unit cube whose
 *   resolution grows exponentially from base_resolution to max_resolution:
 *   D_l = floor(base * b^l + 1e-6), b = (max/base)^(1/(L-1)), the last level
 *   exactly max_resolution -- or, when resolution[0] != 0, the explicit
 *   integer table resolution[0 .. n_levels-1] (each 1..65535,
 *   non-decreasing; entries from n_levels on must be 0; base and max are
 *   then not used), e.g. a table quoted with the network.  Level l has
 *   (D_l+1)^3 lattice points with feat_per_level features each.  With NPM_GRID_HASH a level
 *   with more than 2^log2_table_size points stores a 2^log2_table_size
 *   table addressed by the spatial hash (x * 1) ^ (y * 2654435761) ^
 *   (z * 805459861) mod 2^log2_table_size; other levels are dense.
 *   Limits: 1 <= n_levels <= 32, feat_per_level in {1, 2, 4},
 *   n_levels * feat_per_level <= 32, 1 <= base <= max <= 65535.
 * MLP (Sec. 5.3): n_levels*feat inputs, mlp_hidden_layers (1..4) ReLU layers
 *   of mlp_width (1..64) units, then a linear layer with 4 * n_lobes outputs,
 *   lobe-major (theta', phi', kappa', lambda').  n_lobes must be 8.
 * Init: grid N(0, scale^2) (NPM_INIT_NORMAL) or U(-scale, scale)
 *   (NPM_INIT_UNIFORM); MLP Xavier-uniform; all from `seed`.
 * Adam (Sec. 5.3): lr, beta1, beta2, eps, bias-corrected, eps outside the
 *   square root.
 * batch_order: one of NPM_ORDER_* (fused path: training and queries).
 * scatter_mode: one of NPM_SCATTER_* (fused path: training).
 * sh_degree: 0 for the radiance-based network (Sec. 4.1), or 1..4 for
 *   NPM-product (Sec. 4.3, Full Integrand Learning): the MLP input is G(x)
 *   followed by the real orthonormal spherical harmonics of sh_degree bands
 *   (sh_degree^2 values, index l*l + l + m, no Condon-Shortley phase) of the
 *   outgoing direction omega_o, the same of the surface normal, and the
 *   roughness; such a context takes these per vertex through the *_aux
 *   entry points.  The fused path is built for sh_degree 4 with
 *   n_levels * feat_per_level = 32 (65 inputs) and sh_degree 2 with
 *   n_levels * feat_per_level = 4; the staged path takes any.
 * ema_decay: 0 (off) or d in (0, 1).  When on, every optimizer step also
 *   updates an exponential moving average of the parameters,
 *   ema <- d * ema + (1 - d) * p (after the step, initialised to the
 *   initial parameters), and npm_query, npm_encode and npm_forward_raw
 *   evaluate the network with the averaged weights, as the paper does for
 *   inference (Sec. 5.3); training always uses the current weights.
 * learn_selection: 0, or 1 for the learned BSDF-selection probability
 *   (Sec. 6.3, Discussion: an extension the paper proposes without a
 *   formula).  The last layer gets one more output c' (n_out = 4K + 1), and
 *   c = 1 / (1 + e^{-c'}) is the probability with which the renderer
 *   samples the BSDF rather than the mixture; it is returned by
 *   npm_query_select and trained by npm_backward_select /
 *   npm_train_step_select.  The staged path takes any radiance-based or
 *   NPM-product shape; the fused path (FP32 or the precision form) the
 *   radiance-based shapes (F, inputs, hidden width x layers) (2, <= 16,
 *   <= 32 x 2), (4, <= 16, 33..64 x 2), (4, 17..32, 33..64 x 2) and (2,
 *   17..32, 33..64 x 3) -- the tiny, cfg1, paper and production networks.
 *   The plain calls work on such a network and leave the selection row's
 *   gradient 0.                                                            */
typedef struct {
    int32_t grid_kind;
    int32_t n_levels;
    int32_t feat_per_level;
    int32_t log2_table_size;
    int32_t base_resolution;
    int32_t max_resolution;
    int32_t mlp_width;
    int32_t mlp_hidden_layers;
    int32_t n_lobes;
    int32_t precision;
    int32_t exec_mode;
    int32_t grid_init;
    float grid_init_scale;
    float lr;
    float beta1;
    float beta2;
    float eps;
    int32_t batch_order;
    float ema_decay;
    int32_t sh_degree;
    int32_t scatter_mode;
    int32_t resolution[32];       /* explicit D_l table, or all 0: derive    */
    int32_t learn_selection;      /* 0 or 1                                  */
    uint64_t seed;
} npm_config;

/* Derived sizes of a configuration (host-only, no device needed).          */
#define NPM_MAX_LEVELS 32
#define NPM_MAX_LAYERS 5
typedef struct {
    int64_t n_params;                      /* grid_params + MLP weights     */
    int64_t grid_entries;
    int64_t grid_params;                   /* grid_entries * feat           */
    int64_t level_offset[NPM_MAX_LEVELS];  /* first entry of each level     */
    int64_t level_size[NPM_MAX_LEVELS];    /* entries of each level         */
    int64_t layer_offset[NPM_MAX_LAYERS];  /* first weight of each matrix   */
    int32_t resolution[NPM_MAX_LEVELS];
    int32_t hashed[NPM_MAX_LEVELS];
    int32_t layer_in[NPM_MAX_LAYERS];
    int32_t layer_out[NPM_MAX_LAYERS];
    int32_t n_layers;
    int32_t n_in;
    int32_t n_out;
    int32_t reserved;
    int64_t device_bytes;                  /* persistent device memory of a
                                              context, scratch excluded     */
} npm_layout;

typedef struct npm_ctx npm_ctx;

/* Fills *cfg with the paper's network (Sec. 5.3: three linear layers of
 * width 64, K = 8) on the hashed 16-level grid, FP32, staged, lr 5e-3.      */
npm_status npm_config_default(npm_config *cfg);

/* Validates *cfg and fills *out; needs no device.                          */
npm_status npm_get_layout(const npm_config *cfg, npm_layout *out);

/* Creates a guiding network on the current HIP device: the multiresolution
 * grid of Sec. 5.1 and the decoder MLP of Sec. 5.3 (with NPM-product inputs,
 * Sec. 4.3), laid out as npm_get_layout reports.  Allocates parameters,
 * gradients, Adam moments (zero) and initialises the parameters from
 * cfg->seed (grid as grid_init, weights Xavier-uniform).  *out receives the
 * context, owned by the caller until npm_destroy.  Returns
 * NPM_ERR_INVALID_ARG for an invalid configuration (nothing allocated),
 * NPM_ERR_NO_DEVICE without a gfx950 device, NPM_ERR_OOM when device memory
 * runs out (everything allocated so far is freed).                          */
npm_status npm_create(const npm_config *cfg, npm_ctx **out);

/* Waits for the context's outstanding work and frees it.  NULL is a no-op. */
npm_status npm_destroy(npm_ctx *ctx);

/* Query (Sec. 4.1 eq. npmradiance; Preliminary vMF mixture; Sec. 5.3
 * sampling).  For each vertex i:
 *   pos        [3][n] positions in the unit cube (clamped into it).
 *   dir        [3][n] unit directions at which to evaluate the mixture, or
 *              NULL.  Directions are used as given (not renormalised).
 *   rng_seed, rng_stream: the sample of vertex i uses the Philox4x32-10
 *              block with key (seed lo, seed hi) and counter (i lo, i hi,
 *              rng_stream, 0); uniforms are (word >> 8) * 2^-24.
 *   lobes      [4][K][n] out: theta, phi, kappa, lambda of each lobe, or NULL
 *              (theta, phi in (0,1) are the normalised spherical
 *              coordinates of the lobe axis: polar angle pi*theta, azimuth
 *              2*pi*phi).
 *   pdf        [n] out: mixture density at dir (needs dir), or NULL.
 *   sample_dir [3][n] out: one direction drawn from the mixture, or NULL.
 *   sample_pdf [n] out: mixture density at sample_dir, or NULL.
 * With ema_decay > 0 the network is evaluated with the averaged weights.   */
npm_status npm_query(npm_ctx *ctx, int64_t n, const float *pos, const float *dir,
                     uint64_t rng_seed, uint32_t rng_stream, float *lobes, float *pdf,
                     float *sample_dir, float *sample_pdf, void *stream);

/* Training gradient (Sec. 4.2, eq. mcgradients) of the surrogate loss
 *   loss = -(1/n) sum_i w_i log V(dir_i | Theta(pos_i)),
 *   w_i = radiance_i / sampling_pdf_i (0 unless both are finite and > 0),
 * back-propagated through the MLP and scattered into the eight corners of
 * every grid level; the encoding is recomputed, not stored.
 *   radiance     [n] Monte Carlo estimate of the incident radiance.
 *   sampling_pdf [n] density the direction was drawn with.
 *   grad_out     device FP32 buffer of n_params entries to ACCUMULATE
 *                into, or NULL for the context's own gradient buffer.
 *   loss_out     device pointer to one double (the loss, reduced in FP64),
 *                or NULL.                                                 */
npm_status npm_backward(npm_ctx *ctx, int64_t n, const float *pos, const float *dir,
                        const float *radiance, const float *sampling_pdf, float *grad_out,
                        double *loss_out, void *stream);

/* Surrogate loss only (no gradient); loss_out as in npm_backward.          */
npm_status npm_loss(npm_ctx *ctx, int64_t n, const float *pos, const float *dir,
                    const float *radiance, const float *sampling_pdf, double *loss_out,
                    void *stream);

/* One Adam step (Sec. 5.3) over every parameter, with the step counter
 * advanced first (t = 1 on the first call).  grad is a device FP32 buffer of
 * n_params entries, or NULL for the context's own buffer; it is consumed and
 * zeroed.  gradnorm_out: device pointer to one double receiving the squared
 * L2 norm of the gradient (FP64 reduction), or NULL.                      */
npm_status npm_optimizer_step(npm_ctx *ctx, float *grad, double *gradnorm_out, void *stream);

/* npm_backward into the context's buffer followed by npm_optimizer_step.
 * stats_out: device pointer to two doubles (loss, squared gradient norm), or
 * NULL.                                                                    */
npm_status npm_train_step(npm_ctx *ctx, int64_t n, const float *pos, const float *dir,
                          const float *radiance, const float *sampling_pdf, double *stats_out,
                          void *stream);

/* NPM-product (sh_degree > 0): the same calls with the extra per-vertex
 * inputs aux [7][n] float32 SoA on the device: omega_o (3 rows, unit
 * outgoing direction), the surface normal (3 rows, unit), the roughness
 * (1 row); used as given.  The calls without aux fail with
 * NPM_ERR_INVALID_ARG on such a context, and these calls with aux == NULL
 * are the plain ones on a radiance-based context.                          */
npm_status npm_query_aux(npm_ctx *ctx, int64_t n, const float *pos, const float *aux,
                         const float *dir, uint64_t rng_seed, uint32_t rng_stream, float *lobes,
                         float *pdf, float *sample_dir, float *sample_pdf, void *stream);
npm_status npm_backward_aux(npm_ctx *ctx, int64_t n, const float *pos, const float *aux,
                            const float *dir, const float *radiance, const float *sampling_pdf,
                            float *grad_out, double *loss_out, void *stream);
npm_status npm_loss_aux(npm_ctx *ctx, int64_t n, const float *pos, const float *aux,
                        const float *dir, const float *radiance, const float *sampling_pdf,
                        double *loss_out, void *stream);
npm_status npm_train_step_aux(npm_ctx *ctx, int64_t n, const float *pos, const float *aux,
                              const float *dir, const float *radiance, const float *sampling_pdf,
                              double *stats_out, void *stream);
npm_status npm_encode_aux(npm_ctx *ctx, int64_t n, const float *pos, const float *aux, float *G,
                          void *stream);
npm_status npm_forward_raw_aux(npm_ctx *ctx, int64_t n, const float *pos, const float *aux,
                               float *raw, void *stream);

/* npm_backward for callers that cannot allocate device memory: code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc.
 * Same arguments and result as npm_backward_aux (aux NULL on a
 * radiance-based network), but the call allocates nothing: its scratch (the
 * spatial order of the batch and the per-tile input gradients) lives in one
 * fixed array of NPM_STATIC_SCRATCH_BYTES per device, held from the first
 * npm_create on that device until the process ends, instead of the
 * context's grow-on-demand buffers.
 *   - n must be at most NPM_STATIC_MAX_N (NPM_ERR_INVALID_ARG otherwise).
 *   - The context must be NPM_EXEC_FUSED (NPM_ERR_STATE otherwise).
 *   - The grid gradient is always added with the atomic scatter (never the
 *     binned pass, whose scratch grows with n); the result differs from
 *     npm_backward's only in the order of its floating-point sums.
 *   - Kernel timing (npm_set_timing) does not cover these calls.
 *   - Every call on a device shares that device's array, which keeps the
 *     last call's contents: calls that overlap on one device (two streams,
 *     two contexts, two threads) race and give wrong gradients; serialise
 *     them on one stream.                                                  */
#define NPM_STATIC_MAX_N 32768
#define NPM_STATIC_SCRATCH_BYTES (16u << 20)
npm_status npm_backward_static(npm_ctx *ctx, int64_t n, const float *pos, const float *aux,
                               const float *dir, const float *radiance, const float *sampling_pdf,
                               float *grad_out, double *loss_out, void *stream);

/* Learned BSDF-selection probability (learn_selection = 1; Sec. 6.3
 * extension).  The renderer samples the BSDF with probability c and the
 * mixture V otherwise, so its one-sample MIS density is
 *   p_c(w) = c p_bsdf(w) + (1 - c) V(w).
 * npm_query_select: npm_query_aux plus
 *   select_prob [n] out: c at each vertex, or NULL.
 * npm_backward_select: the gradient of the mixture's loss (npm_backward)
 *   plus that of the selection term, the Sec. 4.2 KL estimator applied to
 *   p_c with V held fixed (it moves c only):
 *     loss_sel = -(1/n) sum_i w_i log p_c(dir_i),
 *     d loss_sel / d c'_i = -(w_i/n) c (1 - c) (p_bsdf - V) / p_c,
 *   with the same weights w_i = radiance_i / sampling_pdf_i.
 *   bsdf_pdf [n] (required): the BSDF's sampling density of dir_i; a sample
 *   whose density is not finite and >= 0 (a delta lobe) has no selection
 *   term.  loss_out: device pointer to two doubles (the mixture's loss,
 *   loss_sel), or NULL.
 * npm_train_step_select: npm_backward_select into the context's buffer,
 *   then npm_optimizer_step; stats_out: three doubles (loss, loss_sel,
 *   squared gradient norm), or NULL.
 * All three fail with NPM_ERR_STATE on a network without the selection
 * output; aux as in the *_aux calls.                                        */
npm_status npm_query_select(npm_ctx *ctx, int64_t n, const float *pos, const float *aux,
                            const float *dir, uint64_t rng_seed, uint32_t rng_stream,
                            float *lobes, float *pdf, float *sample_dir, float *sample_pdf,
                            float *select_prob, void *stream);
npm_status npm_backward_select(npm_ctx *ctx, int64_t n, const float *pos, const float *aux,
                               const float *dir, const float *radiance,
                               const float *sampling_pdf, const float *bsdf_pdf,
                               float *grad_out, double *loss_out, void *stream);
npm_status npm_train_step_select(npm_ctx *ctx, int64_t n, const float *pos, const float *aux,
                                 const float *dir, const float *radiance,
                                 const float *sampling_pdf, const float *bsdf_pdf,
                                 double *stats_out, void *stream);

/* Stage outputs, for checking each step of the path on its own.
 *   npm_corner_index: idx [L][8][n] global table entry of corner b of level
 *     l (corner b has offsets (b&1, b>>1&1, b>>2&1) in x, y, z).
 *   npm_encode: G [n_in][n], the MLP input: the concatenated embedding
 *     (Sec. 5.1), then the NPM-product inputs when sh_degree > 0.
 *   npm_forward_raw: raw [n_out][n], the MLP output before the mappings
 *     (4K lobe outputs, then the selection logit on a selection network).  */
npm_status npm_corner_index(npm_ctx *ctx, int64_t n, const float *pos, uint32_t *idx,
                            void *stream);
npm_status npm_encode(npm_ctx *ctx, int64_t n, const float *pos, float *G, void *stream);
npm_status npm_forward_raw(npm_ctx *ctx, int64_t n, const float *pos, float *raw, void *stream);

/* Host copies of the state.  which: NPM_STATE_PARAMS (FP32 master
 * parameters), NPM_STATE_GRADS (the context's gradient buffer),
 * NPM_STATE_ADAM_M, NPM_STATE_ADAM_V, NPM_STATE_EMA (the averaged
 * parameters; NPM_ERR_STATE when ema_decay is 0).  count must equal
 * n_params.  These calls synchronise the device.  Setting PARAMS also
 * restarts the average at the new parameters; setting PARAMS or EMA
 * refreshes the low-precision copies used by NPM_PREC_BF16.                */
enum { NPM_STATE_PARAMS = 0, NPM_STATE_GRADS = 1, NPM_STATE_ADAM_M = 2, NPM_STATE_ADAM_V = 3,
       NPM_STATE_EMA = 4 };
npm_status npm_get_state(npm_ctx *ctx, int which, float *host, int64_t count);
npm_status npm_set_state(npm_ctx *ctx, int which, const float *host, int64_t count);
/* Adam step counter (number of optimizer steps taken).                     */
npm_status npm_get_step(npm_ctx *ctx, int64_t *step);
npm_status npm_set_step(npm_ctx *ctx, int64_t step);
/* Device address of a state buffer (n_params FP32 entries), owned by the
 * context; valid until npm_destroy.                                         */
npm_status npm_state_device_ptr(npm_ctx *ctx, int which, void **ptr);

/* Per-kernel timing: when enabled, every kernel the context launches is
 * bracketed by HIP events on the stream it runs on; npm_kernel_times
 * returns, for up to `cap` kernels, a name, the number of launches and the
 * summed event time in milliseconds since the last reset (it synchronises
 * the context's streams).                                                  */
npm_status npm_set_timing(npm_ctx *ctx, int enabled);
typedef struct {
    char name[48];
    int64_t launches;
    double total_ms;
} npm_kernel_time;
npm_status npm_kernel_times(npm_ctx *ctx, npm_kernel_time *out, int32_t cap, int32_t *count);
npm_status npm_reset_timing(npm_ctx *ctx);

/* Thread-local message of the last failure on this thread ("" if none).    */
const char *npm_last_error(void);
/* Library version string.                                                  */
const char *npm_version(void);

#ifdef __cplusplus
}
#endif
#endif /* NPM_H */
