// Fused execution of the NPM hot path.  A wave owns a tile of 32 vertices and
// keeps it on chip from the grid lookup to the outputs:
//
//   query:     encode (Sec. 5.1) -> MLP on MFMA (Sec. 5.3) -> Table 1 mappings
//              -> mixture pdf at dir -> lobe selection and vMF sample (Jakob
//              2012) -> pdf at the sample.
//   backward:  encode -> MLP forward (activations in registers) -> KL-gradient
//              head (Sec. 4.2, eq. mcgradients) -> delta chain -> weight
//              gradients (MFMA with the tile's vertices as the reduction
//              dimension, accumulated per wave) -> the tile's dG stored;
//              then the aggregated grid scatter (FP32 atomics) in a kernel of
//              its own.
// Batches of 2^15 vertices or more are visited in a spatial order (k_sort.hip)
// with their inputs read from one record per slot; a query's outputs are
// staged per slot and un-permuted.  NPM-product kernels (PG > 0) also take
// the outgoing direction, normal and roughness (Sec. 4.3).
//
// Tile layout (device_math.h): lane l holds vertex l % 32; of a feature vector
// the half-wave h = l / 32 holds the features nf(h, a).  After the output layer
// half h holds lobes k = 2r + h (r = 0..3), components in registers 4r..4r+3,
// so softmax, log-sum-exp and the lobe CDF need one exchange with lane l ^ 32.
//
// Precision form (BF16 = true): grid features read from an FP16 copy, MLP
// weights and activations in BF16 on v_mfma_f32_32x32x16_bf16 with FP32
// accumulation; mappings, softmax, log-density and sampling in FP32.
#include <type_traits>

#include "fused_tiles.h"

namespace npm {

struct FusedArgs {
    GridDesc g;
    int64_t n;
    const float *pos, *dir, *rad, *spdf;
    const float *grid32;     // FP32 grid (plain form)
    const __half *grid16;    // FP16 grid (precision form)
    const void *img;         // packed MLP images: forward then backward
    int fwd_elems, bwd_elems;
    int n_in, width;
    uint64_t seed;
    uint32_t sid;
    float *lobes, *pdf, *sdir, *spdf_out;
    float *grad;             // accumulated gradient (backward)
    float *dw_part;          // per-wave weight-gradient partials (backward)
    double *partials;        // per-block FP64 loss partials
    float invN;
    const uint32_t *perm;    // visiting order of the vertices (backward), or null
    float *dg_tiles;         // per-tile dG for the aggregated scatter (backward)
    float *qstage;           // staged query outputs in visiting order (with perm)
    const float *rec;        // inputs in visiting order (with perm), rec_stride floats each
    const float *aux;        // NPM-product inputs [7][n]
    int rec_stride;
    // learned selection probability (networks with the selection output)
    const float *wsel;       // the selection row of the last layer (FP32 weights)
    const float *bsdf;       // BSDF densities [n] of the selection term (backward), or null
    double *partials_sel;    // per-block FP64 partials of the selection loss
    float *sel;              // selection probability [n] (query), or null
};
// SEL: the network has the selection output (its logit is computed from the
// last hidden layer and the row staged in LDS; a.sel receives sigmoid of it).
template <int IN_P, int HID_P, int NH, int F, bool BF, int PG, bool SEL = false>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3, 3))) void k_query_fused(FusedArgs a)
{
    extern __shared__ __attribute__((aligned(16))) char smem[];
    __shared__ uint32_t s_off[NPM_MAX_LEVELS];
    __shared__ int s_res[NPM_MAX_LEVELS];
    __shared__ __attribute__((aligned(16))) float s_wsel[SEL ? HID_P : 4];
    {
        const int bytes = a.fwd_elems * (BF ? 2 : 4);
        for (int i = threadIdx.x; i < bytes / 16; i += blockDim.x)
            reinterpret_cast<f32x4 *>(smem)[i] = reinterpret_cast<const f32x4 *>(a.img)[i];
        stage_levels(a.g, s_off, s_res);
        if constexpr (SEL)
            for (int i = threadIdx.x; i < HID_P; i += blockDim.x)
                s_wsel[i] = i < a.width ? a.wsel[i] : 0.0f;
    }
    __syncthreads();
    const GridView gv = grid_view(a.g, s_off, s_res, a.grid32, a.grid16);
    const QueryIO io{a.n, a.pos, a.dir, a.lobes, a.pdf, a.sdir, a.spdf_out, a.seed, a.sid,
                     a.perm, a.qstage, a.rec, a.aux, a.rec_stride, a.sel, s_wsel};
    const int lane = threadIdx.x & 63;
    const int64_t ntiles = (a.n + 31) / 32;
    const int wpb = blockDim.x / 64, wave = threadIdx.x >> 6;
    if (gridDim.x % 8 == 0) {
        // Workgroups are dispatched to the eight XCDs in turn (block b on XCD
        // b mod 8), each XCD with its own L2: give each XCD a contiguous
        // eighth of the tiles, so that the tiles it runs at one time are
        // neighbours in the batch's order and share grid lines in its L2
        // (FP32 query 0.56 -> 0.53 ms at 2^20 vertices).  Any placement of
        // the blocks still covers every tile once.
        const int64_t xcd = blockIdx.x % 8, bl = blockIdx.x / 8;
        const int64_t wpx = (int64_t)(gridDim.x / 8) * wpb, span = (ntiles + 7) / 8;
        const int64_t t0 = xcd * span, t1 = t0 + span < ntiles ? t0 + span : ntiles;
        for (int64_t t = t0 + bl * wpb + wave; t < t1; t += wpx)
            query_tile<IN_P, HID_P, NH, F, BF, PG, SEL>(gv, smem, io, t, lane);
    } else {
        const int64_t nwaves = (int64_t)gridDim.x * wpb;
        for (int64_t t = blockIdx.x * (int64_t)wpb + wave; t < ntiles; t += nwaves)
            query_tile<IN_P, HID_P, NH, F, BF, PG, SEL>(gv, smem, io, t, lane);
    }
}

// ------------------------------------------------------------------ training
// The block-cooperative weight gradients (BlockPlan, dw_phase, dw_write) are
// in fused_tiles.h, shared with the serving kernel.

// Weight-image elements a BF16 training block stages in LDS: the forward and
// backward images, except that with NPM-product inputs only the grid
// features' input gradient is needed, so of W_0^T -- the last segment, its
// 32-row blocks in order -- only the first block is staged.
static int64_t staged_elems(const FusedArgs &a, int in_p, int hid_p, int pg)
{
    const int in0 = in_p < 32 ? 32 : in_p;
    const int dg_rows = pg > 0 ? 32 : in0;
    return (int64_t)a.fwd_elems + a.bwd_elems - (int64_t)(in0 - dg_rows) * hid_p;
}

// 32 exchange-buffer values of a and b (16-byte aligned) multiplied and summed.
__device__ __forceinline__ float dot32(const float *a, const float *b)
{
    float s = 0.0f;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        const f32x4 x = reinterpret_cast<const f32x4 *>(a)[q];
        const f32x4 y = reinterpret_cast<const f32x4 *>(b)[q];
#pragma unroll
        for (int e = 0; e < 4; ++e) s = fmaf(x[e], y[e], s);
    }
    return s;
}
__device__ __forceinline__ float dot32(const __bf16 *a, const __bf16 *b)
{
    float s = 0.0f;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const bf16x8 x = reinterpret_cast<const bf16x8 *>(a)[q];
        const bf16x8 y = reinterpret_cast<const bf16x8 *>(b)[q];
#pragma unroll
        for (int e = 0; e < 8; ++e) s = fmaf((float)x[e], (float)y[e], s);
    }
    return s;
}

// SEL: the network has the selection output (the learned BSDF-selection
// probability).  Its logit c' is the last hidden layer dotted with the
// selection row (staged in LDS); with BSDF densities the head adds the
// selection term's derivative d (eq. mcgradients applied to the one-sample
// density c p_bsdf + (1 - c) V, V fixed) and the chain adds d times the row to
// the last hidden layer's delta.  The row's weight gradient sums d times the
// last hidden layer over the round: d goes into the exchange buffer one row
// after the output layer's deltas and inputs, and lane f of wave q sums
// feature f over wave q's 32 vertices; the waves' sums add at the end.
template <int IN_P, int HID_P, int NH, int F, bool BF, int PG, int WV, bool SEL = false>
__global__ __launch_bounds__(64 * WV) void k_backward_fused(FusedArgs a, int mlp_weights,
                                                           int img_bytes)
{
    // the FP32 selection instantiation of the three-hidden-layer network
    // keeps whole blocks: there the split's extra accumulator would not fit
    // beside the selection sums (it would spill)
    using Plan = BlockPlan<IN_P, HID_P, NH, WV, !(SEL && !BF && NH >= 3)>;
    using XT = typename std::conditional<BF, __bf16, float>::type;
    constexpr int IN0 = Plan::IN0;
    constexpr int XS = Plan::xs(BF);
    constexpr int NS = Plan::slots();
    constexpr int ESZ = BF ? 2 : 4;
    constexpr int DGR = PG > 0 ? 32 : IN0;      // input-gradient rows (grid features only with PG)
    extern __shared__ __attribute__((aligned(16))) char smem[];
    __shared__ uint32_t s_off[NPM_MAX_LEVELS];
    __shared__ int s_res[NPM_MAX_LEVELS];
    __shared__ double red[64 * WV];
    __shared__ __attribute__((aligned(16))) float s_wsel[SEL ? HID_P : 4];
    // weights: BF16 the packed forward and backward images, FP32 the
    // row-major image (both directions)
    for (int i = threadIdx.x; i < img_bytes / 16; i += blockDim.x)
        reinterpret_cast<f32x4 *>(smem)[i] = reinterpret_cast<const f32x4 *>(a.img)[i];
    stage_levels(a.g, s_off, s_res);
    if constexpr (SEL)
        for (int i = threadIdx.x; i < HID_P; i += blockDim.x) s_wsel[i] = i < a.width ? a.wsel[i] : 0.0f;
    __syncthreads();
    XT *xb = reinterpret_cast<XT *>(smem + ((size_t)img_bytes + 15) / 16 * 16);
    const GridView gv = grid_view(a.g, s_off, s_res, a.grid32, a.grid16);
    const TrainIO io{a.n, a.pos, a.dir, a.rad, a.spdf, a.grad, a.invN, a.perm, a.rec, a.aux,
                     a.rec_stride, a.bsdf};
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, h = lane >> 5;
    float selacc = 0.0f;          // SEL: the row's gradient, feature `lane`, this wave's vertices
    double lsel = 0.0;            // SEL: -w log p_c of half 0's vertices
    const float *rm = reinterpret_cast<const float *>(smem);
    const char *fwd = smem;
    const char *bwd = smem + (size_t)a.fwd_elems * ESZ;
    f32x16 acc[NS];
#pragma unroll
    for (int k = 0; k < NS; ++k)
#pragma unroll
        for (int v = 0; v < 16; ++v) acc[k][v] = 0.0f;
    double lacc = 0.0;
    const int64_t n = a.n;
    const int64_t ntiles = (n + 31) / 32;
    // Rounds of WV consecutive tiles are dealt to the blocks in turn.
    // Workgroups are dispatched to the eight XCDs in turn (block b on XCD
    // b mod 8), each XCD with its own L2: with a multiple of eight blocks each
    // XCD takes a contiguous eighth of the tiles and its blocks take that
    // eighth's rounds in turn, so that the rounds an XCD runs at one time are
    // neighbours in the batch's order and share grid lines in its L2.  A
    // block with no round still writes its (zero) partials.
    int64_t t_lo = 0, t_end = ntiles, bl = blockIdx.x, nb = gridDim.x;
    if (gridDim.x % 8 == 0) {
        nb = gridDim.x / 8;
        bl = blockIdx.x / 8;
        const int64_t span = ((ntiles + 7) / 8 + WV - 1) / WV * WV;
        t_lo = (int64_t)(blockIdx.x % 8) * span;
        t_end = t_lo + span < ntiles ? t_lo + span : ntiles;
    }
    const int64_t stride = nb * WV;            // tiles from one of this block's rounds to the next
    const int64_t t_first = t_lo + bl * WV;
    // the visiting slot of this lane in tile tt (the last vertex for a tile
    // past the span or a lane past the batch)
    auto slot = [&](int64_t tt) {
        const int64_t v = tt * 32 + (lane & 31);
        return tt < t_end && v < n ? v : n - 1;
    };
    // Software pipeline over the rounds: a round's grid gathers are issued
    // during the round before (one wave per SIMD leaves the registers for
    // them: 8 levels x 8 corners x F = 2 per half-wave on the production
    // grid), and its inputs are loaded two rounds ahead.  Shapes whose
    // gathers would not fit beside the rest (F = 1, NPM-product's wide
    // first layer) gather in the round itself.
    constexpr bool PIPE = IN_P <= 32 && F >= 2 && PG == 0;
    constexpr int ING = PG > 0 ? ProductShape<PG>::GF : IN_P;   // grid features
    TileGather<ING, F, BF> gath;
    TrainInputs in_next = train_inputs(io, slot(t_first + wave), visit(io.perm, slot(t_first + wave)));
    TrainInputs in_after = train_inputs(io, slot(t_first + stride + wave),
                                        visit(io.perm, slot(t_first + stride + wave)));
    if (PIPE && t_first < t_end)
        encode_issue<ING, F, BF>(gv, h, in_next.px, in_next.py, in_next.pz, gath);
    for (int64_t t0 = t_first; t0 < t_end; t0 += stride) {
        // every wave of the block runs every round (the phases synchronise);
        // a wave past the run's end takes a tile with no valid vertex
        const int64_t t = t0 + wave;
        const int64_t v = t * 32 + (lane & 31);
        const bool valid = t < t_end && v < n;
        const int64_t vs = slot(t);
        const int64_t vv = visit(io.perm, vs);
        const TrainInputs in = in_next;
        in_next = in_after;
        const int64_t s2 = slot(t + 2 * stride);
        in_after = train_inputs(io, s2, visit(io.perm, s2));
        float x[IN0 / 2];
        if constexpr (PIPE) {
            encode_finish<IN_P, ING, F, BF>(gv, h, gath, x);
#pragma unroll
            for (int i = IN_P / 2; i < IN0 / 2; ++i) x[i] = 0.0f;
            // the next round's gathers, in flight while this round's MLP runs
            if (t0 + stride < t_end)
                encode_issue<ING, F, BF>(gv, h, in_next.px, in_next.py, in_next.pz, gath);
        } else {
            tile_input<IN_P, F, BF, PG>(gv, io, in, vs, vv, h, x);
        }
        float acts[NH][HID_P / 2];
        float o[16];
        if constexpr (BF) {
            mlp_forward<IN_P, HID_P, NH, true, true>(fwd, x, acts, o, lane);
        } else {
            mfma_layer_rm<IN_P, HID_P, Plan::rm_stride(0), false>(rm, x, acts[0], lane);
#pragma unroll
            for (int i = 0; i < HID_P / 2; ++i) acts[0][i] = fmaxf(acts[0][i], 0.0f);
#pragma unroll
            for (int li = 1; li < NH; ++li) {
                // the hidden layers' rows have one stride, HID_P + 1
                mfma_layer_rm<HID_P, HID_P, Plan::rm_stride(1), false>(
                    rm + Plan::rm_off(1) + (li - 1) * HID_P * Plan::rm_stride(1), acts[li - 1],
                    acts[li], lane);
#pragma unroll
                for (int i = 0; i < HID_P / 2; ++i) acts[li][i] = fmaxf(acts[li][i], 0.0f);
            }
            mfma_layer_rm<HID_P, 32, Plan::rm_stride(NH), false>(rm + Plan::rm_off(NH),
                                                                  acts[NH - 1], o, lane);
        }
        float d[16];
        const float lv = kl_head(o, in, valid, io.invN, h, d, lacc);
        float ds = 0.0f;            // SEL: d loss / d c'
        if constexpr (SEL) {
            const float cp = select_logit<HID_P>(s_wsel, acts[NH - 1], h);
            const float wgt = valid ? sample_weight(in.rad, in.spdf) : 0.0f;
            if (wgt != 0.0f && io.bsdf) {
                const float pb = io.bsdf[vv];
                if (bsdf_valid(pb)) {
                    const float lpc = select_term(cp, pb, lv, -wgt * io.invN, ds);
                    if (h == 0) lsel -= (double)wgt * (double)lpc;
                }
            }
        }
        if (!a.grad) continue;      // loss only (uniform over the grid)
        // ---- output layer: its dW, then the first delta of the chain
        float dh[HID_P / 2];
        if constexpr (SEL)
            if (h == 0) xb[Plan::sel_row() * XS + 32 * wave + (lane & 31)] = XT(ds);
        dw_phase<Plan, NH, WV, XS>(xb, d, acts[NH - 1], wave, acc, lane);
        if constexpr (SEL)
            if (lane < HID_P)
                selacc += dot32(xb + Plan::sel_row() * XS + 32 * wave,
                                xb + (Plan::out_p(NH) + lane) * XS + 32 * wave);
        if constexpr (BF) layer<true, 32, HID_P>(bwd, d, dh, lane);
        else mfma_layer_rm<32, HID_P, Plan::rm_stride(NH), true>(rm + Plan::rm_off(NH), d, dh, lane);
        if constexpr (SEL) {
#pragma unroll
            for (int q = 0; q < HID_P / 8; ++q) {
                const f32x4 w = *reinterpret_cast<const f32x4 *>(s_wsel + 8 * q + 4 * h);
#pragma unroll
                for (int e = 0; e < 4; ++e) dh[4 * q + e] = fmaf(ds, w[e], dh[4 * q + e]);
            }
        }
        __syncthreads();
        // ---- hidden layers NH-1 .. 1
        const char *im = bwd + (size_t)HID_P * 32 * ESZ;
        static_for_down<NH - 1, 1>([&](auto LC) {
            constexpr int li = decltype(LC)::value;
#pragma unroll
            for (int i = 0; i < HID_P / 2; ++i) dh[i] = acts[li][i] > 0.0f ? dh[i] : 0.0f;
            dw_phase<Plan, li, WV, XS>(xb, dh, acts[li - 1], wave, acc, lane);
            float nd[HID_P / 2];
            if constexpr (BF) {
                layer<true, HID_P, HID_P>(im, dh, nd, lane);
                im += (size_t)HID_P * HID_P * ESZ;
            } else {
                mfma_layer_rm<HID_P, HID_P, Plan::rm_stride(li), true>(rm + Plan::rm_off(li), dh, nd,
                                                                        lane);
            }
#pragma unroll
            for (int i = 0; i < HID_P / 2; ++i) dh[i] = nd[i];
            __syncthreads();
        });
        // ---- first layer: its dW and the input gradient dG (the grid
        // features' rows only with NPM-product inputs), stored per tile for
        // the scatter kernels
#pragma unroll
        for (int i = 0; i < HID_P / 2; ++i) dh[i] = acts[0][i] > 0.0f ? dh[i] : 0.0f;
        dw_phase<Plan, 0, WV, XS>(xb, dh, x, wave, acc, lane);
        float dG[DGR / 2];
        if constexpr (BF) layer<true, HID_P, DGR>(im, dh, dG, lane);
        else mfma_layer_rm<HID_P, DGR, Plan::rm_stride(0), true>(rm, dh, dG, lane);
        if (t < t_end) {
            float *dst = a.dg_tiles + (size_t)t * IN0 * 32 + (lane & 31);
#pragma unroll
            for (int q = 0; q < DGR / 2; ++q) dst[nf(h, q) * 32] = dG[q];
        }
        __syncthreads();
    }
    // ---- loss partial of the block (FP64)
    red[threadIdx.x] = lacc;
    __syncthreads();
    for (int w = (int)blockDim.x / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) a.partials[blockIdx.x] = red[0];
    if constexpr (SEL) {
        __syncthreads();
        red[threadIdx.x] = lsel;
        __syncthreads();
        for (int w = (int)blockDim.x / 2; w > 0; w >>= 1) {
            if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
            __syncthreads();
        }
        if (threadIdx.x == 0) a.partials_sel[blockIdx.x] = red[0];
    }
    if (!a.grad) return;
    static_assert(Plan::scratch_fits(BF), "split blocks' sums fit in the exchange buffer");
    dw_write<Plan, NH, WV>(a.dw_part + (int64_t)blockIdx.x * mlp_weights, a.n_in, a.width, wave,
                           acc, lane, reinterpret_cast<float *>(xb));
    if constexpr (SEL) {
        // the selection row (after the output layer's 32 rows): the waves' sums
        __syncthreads();
        red[threadIdx.x] = selacc;
        __syncthreads();
        if (wave == 0 && lane < a.width) {
            float sum = 0.0f;
            for (int w = 0; w < WV; ++w) sum += (float)red[64 * w + lane];
            const int64_t row = (int64_t)a.width * a.n_in + (int64_t)(NH - 1) * a.width * a.width +
                                32 * a.width;
            a.dw_part[(int64_t)blockIdx.x * mlp_weights + row + lane] = sum;
        }
    }
}

// Aggregated grid scatter of the per-tile dG (stride `rows` rows of 32 per
// tile) in the same visiting order.  A wave takes a contiguous run of tiles;
// per tile it stages the n_levels * F dG rows in LDS, takes the tile's
// bounding box and scatters with the LDS window (scatter_tile).  Kept apart
// from the MLP kernel: the atomics are bound by the rate of line requests
// the memory system accepts, and at the one wave per SIMD the MLP kernel's
// registers allow, a wave waiting on its atomics leaves its SIMD idle, while
// this kernel runs four waves per SIMD.
// per wave: 32 dG rows, then the window of kScatterWinRows rows holding the
// sums -- FP64 (LDS FP64 atomic adds run several times faster than FP32 ones
// on this chip), or 32-bit fixed point in the precision form (WT = int, no
// FP64): kScatterWinRows * kStride / (2 F) lattice points
constexpr int kScatterWinRows = 32;
constexpr int kScatterRows = 32 + kScatterWinRows;

template <int F, typename WT>
__global__ __launch_bounds__(256) void k_scatter_tiles(GridDesc g, int64_t n,
                                                       const float *__restrict__ pos,
                                                       const uint32_t *perm,
                                                       const float *__restrict__ rec,
                                                       int rec_stride,
                                                       const float *__restrict__ dgt, int rows,
                                                       float *__restrict__ grad, uint32_t skip_mask)
{
    __shared__ uint32_t s_off[NPM_MAX_LEVELS];
    __shared__ int s_res[NPM_MAX_LEVELS];
    __shared__ __attribute__((aligned(16))) float buf[4 * kScatterRows * kStride];
    stage_levels(g, s_off, s_res);
    __syncthreads();
    const GridView gv = grid_view(g, s_off, s_res, nullptr, nullptr);
    constexpr int WIN_PTS = kScatterWinRows * kStride / (2 * F);
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    float *tb = buf + wave * kScatterRows * kStride;
    const int lr = g.n_levels * g.feat;           // dG rows the scatter reads (<= 32)
    const int64_t ntiles = (n + 31) / 32;
    const int64_t nwaves = (int64_t)gridDim.x * 4;
    const int64_t gwave = blockIdx.x * (int64_t)4 + wave;
    const int64_t per = (ntiles + nwaves - 1) / nwaves;
    const int64_t t_end = (gwave + 1) * per < ntiles ? (gwave + 1) * per : ntiles;
    for (int64_t t = gwave * per; t < t_end; ++t) {
        const int64_t v = t * 32 + (lane & 31);
        float lo[3], hi[3];
        if (rec) {
            const f32x4 a = *reinterpret_cast<const f32x4 *>(rec + (size_t)(v < n ? v : n - 1) * rec_stride);
            tile_bbox(a[0], a[1], a[2], lo, hi);
        } else {
            const int64_t vv = visit(perm, v < n ? v : n - 1);
            tile_bbox(pos[vv], pos[n + vv], pos[2 * n + vv], lo, hi);
        }
        const float *src = dgt + (size_t)t * rows * 32;
        for (int i = lane; i < lr * 8; i += 64) {
            const f32x4 q = reinterpret_cast<const f32x4 *>(src)[i];
            *reinterpret_cast<f32x4 *>(tb + (i >> 3) * kStride + (i & 7) * 4) = q;
        }
        wave_lds_fence();
        scatter_tile<F, WIN_PTS, WT>(gv, tb, pos, perm, n, t, lane, grad, lo, hi,
                                     reinterpret_cast<WT *>(tb + 32 * kStride), rec, rec_stride,
                                     skip_mask);
        wave_lds_fence();
    }
}

// Moves the staged outputs of a spatially ordered query to the caller's SoA
// buffers: vertex i (coalesced writes) reads its 160-byte slot inv[i].
__global__ __launch_bounds__(256) void k_query_unstage(int64_t n, const uint32_t *__restrict__ inv,
                                                       const float *__restrict__ stage,
                                                       float *__restrict__ lobes,
                                                       float *__restrict__ pdf,
                                                       float *__restrict__ sdir,
                                                       float *__restrict__ spdf,
                                                       float *__restrict__ sel)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    const f32x4 *src = reinterpret_cast<const f32x4 *>(stage + (size_t)inv[i] * kStageFloats);
    f32x4 r[kStageFloats / 4];
#pragma unroll
    for (int q = 0; q < kStageFloats / 4; ++q) r[q] = src[q];
    const float *c = reinterpret_cast<const float *>(r);
    if (lobes)
#pragma unroll
        for (int k = 0; k < kLobes; ++k)
#pragma unroll
            for (int q = 0; q < 4; ++q)
                lobes[(int64_t)(q * kLobes + k) * n + i] = c[20 * (k & 1) + 4 * (k >> 1) + q];
    if (pdf) pdf[i] = c[kStagePdf];
    if (sdir)
#pragma unroll
        for (int d = 0; d < 3; ++d) sdir[(int64_t)d * n + i] = c[kStageSdir + d];
    if (spdf) spdf[i] = c[kStageSpdf];
    if (sel) sel[i] = c[kStageSel];
}

// Sum of the blocks' weight-gradient partials into the gradient: a block of
// 256 threads covers 16 weights, its 16 thread rows a sixteenth of the
// partials each (several loads in flight per thread, 768 blocks at the
// production size), then the rows add in LDS.
__global__ __launch_bounds__(256) void k_dw_sum(const float *__restrict__ part, int nparts,
                                                int count, float *__restrict__ grad)
{
    __shared__ float red[16][17];
    const int x = threadIdx.x & 15, y = threadIdx.x >> 4;
    const int i = blockIdx.x * 16 + x;
    float s0 = 0.0f, s1 = 0.0f;
    if (i < count) {
        int p = y;
        for (; p + 16 < nparts; p += 32) {
            s0 += part[(int64_t)p * count + i];
            s1 += part[(int64_t)(p + 16) * count + i];
        }
        if (p < nparts) s0 += part[(int64_t)p * count + i];
    }
    red[y][x] = s0 + s1;
    __syncthreads();
    if (y == 0 && i < count) {
        float t = 0.0f;
#pragma unroll
        for (int r = 0; r < 16; ++r) t += red[r][x];
        grad[i] += t;
    }
}

// ------------------------------------------------------------------ launch
static FusedArgs fused_args(npm_ctx *ctx, int64_t n, const float *pos)
{
    FusedArgs a{};
    const Net &net = ctx->net;
    a.g = net.grid;
    a.n = n;
    a.pos = pos;
    a.grid32 = ctx->params;
    a.grid16 = (const __half *)ctx->grid16;
    const bool bf = net.cfg.precision == NPM_PREC_BF16;
    a.img = bf ? ctx->mlp_img16 : (const void *)ctx->mlp_img;
    a.fwd_elems = (int)net.mlp.fwd_elems;
    a.bwd_elems = (int)net.mlp.bwd_elems;
    a.n_in = net.mlp.n_in;
    a.width = net.mlp.width;
    a.rec_stride = net.cfg.sh_degree ? 16 : 8;
    return a;
}

template <int IN_P, int HID_P, int NH, int F, bool BF, int PG = 0, bool SEL = false>
static hipError_t run_query(npm_ctx *ctx, FusedArgs a, hipStream_t s)
{
    const int64_t tiles = (a.n + 31) / 32;
    const int blocks = (int)std::max<int64_t>(1, std::min<int64_t>((tiles + 3) / 4, 2048));
    const size_t lds = (size_t)a.fwd_elems * (BF ? 2 : 4);
    auto k = k_query_fused<IN_P, HID_P, NH, F, BF, PG, SEL>;
    const hipError_t e = hipFuncSetAttribute((const void *)k,
                                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k, dim3(blocks), dim3(256), lds, s, a);
    return hipGetLastError();
}

// Blocks of the training kernel: one per compute unit at most (the weight
// image and the exchange buffer take most of its LDS), WV waves each.
constexpr int kTrainWaves = 4;
constexpr int kTrainMaxBlocks = 256;
static int backward_blocks(int64_t n)
{
    const int64_t tiles = (n + 31) / 32;
    return (int)std::max<int64_t>(1, std::min<int64_t>((tiles + kTrainWaves - 1) / kTrainWaves,
                                                       kTrainMaxBlocks));
}

// Dynamic LDS a training block may take: gfx950's 160 KB per workgroup less
// room for the kernel's static arrays (level table, FP64 loss partials).
constexpr size_t kLdsBytes = 160 * 1024 - 4096;

template <int IN_P, int HID_P, int NH, int F, bool BF, int PG = 0, bool SEL = false>
static hipError_t run_backward(npm_ctx *ctx, FusedArgs a, hipStream_t s)
{
    using Plan = BlockPlan<IN_P, HID_P, NH, kTrainWaves>;
    const int blocks = backward_blocks(a.n);
    const size_t img = BF ? (size_t)staged_elems(a, IN_P, HID_P, PG) * 2
                          : (size_t)Plan::rm_elems() * 4;
    if (!BF && (int64_t)Plan::rm_elems() != ctx->net.mlp.rm_elems) return hipErrorInvalidValue;
    const size_t lds = (img + 15) / 16 * 16 +
                       (size_t)Plan::max_rows() * Plan::xs(BF) * (BF ? 2 : 4);
    const int count = (int)(ctx->net.lay.n_params - ctx->net.lay.grid_params);
    if (lds > kLdsBytes) return hipErrorInvalidValue;
    if (!BF) a.img = ctx->mlp_img + ctx->net.mlp.fwd_elems + ctx->net.mlp.bwd_elems;
    auto k = k_backward_fused<IN_P, HID_P, NH, F, BF, PG, kTrainWaves, SEL>;
    const hipError_t e = hipFuncSetAttribute((const void *)k,
                                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k, dim3(blocks), dim3(64 * kTrainWaves), lds, s, a, count, (int)img);
    return hipGetLastError();
}

#define NPM_FUSED_DISPATCH(RUN, BFV)                                                              \
    do {                                                                                          \
        const MlpDesc &m_ = ctx->net.mlp;                                                         \
        const int F_ = ctx->net.grid.feat;                                                        \
        const int key_ = F_ * 1000 + (m_.in_p == 32) * 100 + (m_.hid_p == 64) * 10 + m_.n_hidden; \
        switch (key_) {                                                                           \
        case 1002: e = RUN<16, 32, 2, 1, BFV>(ctx, a, s); break;                                  \
        case 1112: e = RUN<32, 64, 2, 1, BFV>(ctx, a, s); break;                                  \
        case 1113: e = RUN<32, 64, 3, 1, BFV>(ctx, a, s); break;                                  \
        case 2002: e = RUN<16, 32, 2, 2, BFV>(ctx, a, s); break;                                  \
        case 2012: e = RUN<16, 64, 2, 2, BFV>(ctx, a, s); break;                                  \
        case 2112: e = RUN<32, 64, 2, 2, BFV>(ctx, a, s); break;                                  \
        case 2113: e = RUN<32, 64, 3, 2, BFV>(ctx, a, s); break;                                  \
        case 4012: e = RUN<16, 64, 2, 4, BFV>(ctx, a, s); break;                                  \
        case 4013: e = RUN<16, 64, 3, 4, BFV>(ctx, a, s); break;                                  \
        case 4112: e = RUN<32, 64, 2, 4, BFV>(ctx, a, s); break;                                  \
        case 4113: e = RUN<32, 64, 3, 4, BFV>(ctx, a, s); break;                                  \
        default: return hipErrorNotSupported;                                                     \
        }                                                                                         \
    } while (0)

// NPM-product shapes (sh_degree 4 on 32 grid features, 65 inputs in a 96-wide
// first layer; sh_degree 2 on 4 grid features, 13 inputs).
#define NPM_FUSED_PRODUCT_DISPATCH(RUN, BFV)                                                      \
    do {                                                                                          \
        const MlpDesc &m_ = ctx->net.mlp;                                                         \
        const int F_ = ctx->net.grid.feat;                                                        \
        const int key_ = m_.sh_degree * 100000 + F_ * 10000 + m_.in_p * 100 +                    \
                         (m_.hid_p == 64) * 10 + m_.n_hidden;                                     \
        switch (key_) {                                                                           \
        case 429612: e = RUN<96, 64, 2, 2, BFV, 1>(ctx, a, s); break;                             \
        case 429613: e = RUN<96, 64, 3, 2, BFV, 1>(ctx, a, s); break;                             \
        case 449612: e = RUN<96, 64, 2, 4, BFV, 1>(ctx, a, s); break;                             \
        case 449613: e = RUN<96, 64, 3, 4, BFV, 1>(ctx, a, s); break;                             \
        case 221602: e = RUN<16, 32, 2, 2, BFV, 2>(ctx, a, s); break;                             \
        default: return hipErrorNotSupported;                                                     \
        }                                                                                         \
    } while (0)

// Networks with the selection output: the tiny (4 inputs, width 8), cfg1
// (16 inputs, 64 x 2), the paper's (32 inputs, 64 x 2) and the production
// (32 inputs, 64 x 3) shapes.
#define NPM_FUSED_SEL_DISPATCH(RUN, BFV)                                                          \
    do {                                                                                          \
        const MlpDesc &m_ = ctx->net.mlp;                                                         \
        const int F_ = ctx->net.grid.feat;                                                        \
        const int key_ = F_ * 1000 + (m_.in_p == 32) * 100 + (m_.hid_p == 64) * 10 + m_.n_hidden; \
        switch (key_) {                                                                           \
        case 2002: e = RUN<16, 32, 2, 2, BFV, 0, true>(ctx, a, s); break;                         \
        case 4012: e = RUN<16, 64, 2, 4, BFV, 0, true>(ctx, a, s); break;                         \
        case 4112: e = RUN<32, 64, 2, 4, BFV, 0, true>(ctx, a, s); break;                         \
        case 2113: e = RUN<32, 64, 3, 2, BFV, 0, true>(ctx, a, s); break;                         \
        default: return hipErrorNotSupported;                                                     \
        }                                                                                         \
    } while (0)

#define NPM_FUSED_RUN(RUN)                                                                        \
    do {                                                                                          \
        const bool bf_ = ctx->net.cfg.precision == NPM_PREC_BF16;                                 \
        if (ctx->net.cfg.learn_selection) {                                                       \
            if (bf_) NPM_FUSED_SEL_DISPATCH(RUN, true);                                           \
            else NPM_FUSED_SEL_DISPATCH(RUN, false);                                              \
        } else if (ctx->net.mlp.sh_degree > 0) {                                                  \
            if (bf_) NPM_FUSED_PRODUCT_DISPATCH(RUN, true);                                       \
            else NPM_FUSED_PRODUCT_DISPATCH(RUN, false);                                          \
        } else {                                                                                  \
            if (bf_) NPM_FUSED_DISPATCH(RUN, true);                                               \
            else NPM_FUSED_DISPATCH(RUN, false);                                                  \
        }                                                                                         \
    } while (0)

bool fused_shape_supported(const Net &net)
{
    const MlpDesc &m = net.mlp;
    const int F = net.grid.feat;
    if (net.cfg.learn_selection) {
        if (m.sh_degree > 0) return false;
        switch (F * 1000 + (m.in_p == 32) * 100 + (m.hid_p == 64) * 10 + m.n_hidden) {
        case 2002: case 4012: case 4112: case 2113: return m.in_p <= 32;
        default: return false;
        }
    }
    if (m.sh_degree > 0) {
        switch (m.sh_degree * 100000 + F * 10000 + m.in_p * 100 + (m.hid_p == 64) * 10 + m.n_hidden) {
        case 429612: case 429613: case 449612: case 449613: case 221602: return true;
        default: return false;
        }
    }
    switch (F * 1000 + (m.in_p == 32) * 100 + (m.hid_p == 64) * 10 + m.n_hidden) {
    case 1002: case 1112: case 1113: case 2002: case 2012: case 2112: case 2113:
    case 4012: case 4013: case 4112: case 4113: return m.in_p <= 32;
    default: return false;
    }
}

hipError_t fused_query(npm_ctx *ctx, int64_t n, const float *pos, const float *aux,
                       const float *dir, uint64_t seed, uint32_t stream_id, float *lobes,
                       float *pdf, float *sdir, float *spdf, const uint32_t *perm,
                       const uint32_t *inv, const float *rec, float *stage, hipStream_t s,
                       float *sel)
{
    FusedArgs a = fused_args(ctx, n, pos);
    a.aux = aux;
    const Weights w = query_weights(ctx);
    a.grid32 = w.grid32;
    a.grid16 = (const __half *)w.grid16;
    a.img = ctx->net.cfg.precision == NPM_PREC_BF16 ? w.img16 : (const void *)w.img;
    a.dir = dir;
    a.seed = seed;
    a.sid = stream_id;
    a.lobes = lobes;
    a.pdf = pdf;
    a.sdir = sdir;
    a.spdf_out = spdf;
    a.perm = perm;
    a.qstage = perm ? stage : nullptr;
    a.rec = perm ? rec : nullptr;
    a.wsel = selection_row(ctx, w.grid32);
    a.sel = sel;
    hipError_t e = hipSuccess;
    int tok;
    timed_begin(ctx, "fused_query", s, &tok);
    NPM_FUSED_RUN(run_query);
    timed_end(ctx, tok, s);
    if (e != hipSuccess || !perm) return e;
    timed_begin(ctx, "query_unstage", s, &tok);
    hipLaunchKernelGGL(k_query_unstage, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, inv,
                       stage, lobes, pdf, sdir, spdf, sel);
    timed_end(ctx, tok, s);
    return hipGetLastError();
}

hipError_t fused_backward(npm_ctx *ctx, int64_t n, const float *pos, const float *aux,
                          const float *dir, const float *rad, const float *spdf, float *grad,
                          double *loss_out, const uint32_t *perm, const float *rec,
                          float *dg_tiles, const BinDesc *bins, hipStream_t s, const float *bsdf)
{
    FusedArgs a = fused_args(ctx, n, pos);
    a.aux = aux;
    a.perm = perm;
    a.rec = perm ? rec : nullptr;
    a.dir = dir;
    a.rad = rad;
    a.spdf = spdf;
    a.grad = grad;
    a.dw_part = ctx->s_dw_part;
    a.partials = ctx->partials;
    a.invN = 1.0f / (float)n;
    a.dg_tiles = grad ? dg_tiles : nullptr;
    a.wsel = selection_row(ctx, ctx->params);
    a.bsdf = bsdf;
    a.partials_sel = ctx->partials + kPartials / 2;
    hipError_t e = hipSuccess;
    int tok;
    timed_begin(ctx, "fused_backward", s, &tok);
    NPM_FUSED_RUN(run_backward);
    timed_end(ctx, tok, s);
    if (e != hipSuccess) return e;
    const int blocks = backward_blocks(n);
    if (grad) {
        const int64_t tiles = (n + 31) / 32;
        const int64_t waves = std::min<int64_t>(tiles, 4096);
        const int rows = std::max(ctx->net.mlp.in_p, 32);
        uint32_t skip = 0u;
        if (bins)
            for (int j = 0; j < bins->nb; ++j) skip |= 1u << bins->lv[j];
        const uint32_t all = ctx->net.grid.n_levels >= 32 ? ~0u : (1u << ctx->net.grid.n_levels) - 1u;
        // The windowed scatter and the weight-gradient sum write other parts
        // of the gradient than the binned scatter and read only the per-tile
        // dG: with bins they run on the side stream, beside the binned passes
        // (which leave CUs idle in their scan and in the reduce's last wave of
        // blocks), and the caller's stream waits for both.
        hipStream_t s2 = s;
        if (bins) {
            s2 = ctx->side;
            e = hipEventRecord(ctx->ev_fork, s);
            if (e == hipSuccess) e = hipStreamWaitEvent(s2, ctx->ev_fork, 0);
            if (e != hipSuccess) return e;
        }
        if (skip != all) {
            timed_begin(ctx, "fused_scatter", s2, &tok);
            const bool fixed = ctx->net.cfg.precision == NPM_PREC_BF16;
            const dim3 grid((unsigned)((waves + 3) / 4)), block(256);
#define NPM_SCATTER_LAUNCH(FV, WT)                                                                 \
    hipLaunchKernelGGL((k_scatter_tiles<FV, WT>), grid, block, 0, s2, ctx->net.grid, n, pos, perm, \
                       rec, a.rec_stride, dg_tiles, rows, grad, skip)
            switch (ctx->net.grid.feat) {
            case 1: if (fixed) NPM_SCATTER_LAUNCH(1, int); else NPM_SCATTER_LAUNCH(1, double); break;
            case 2: if (fixed) NPM_SCATTER_LAUNCH(2, int); else NPM_SCATTER_LAUNCH(2, double); break;
            default: if (fixed) NPM_SCATTER_LAUNCH(4, int); else NPM_SCATTER_LAUNCH(4, double); break;
            }
#undef NPM_SCATTER_LAUNCH
            timed_end(ctx, tok, s2);
            e = hipGetLastError();
            if (e != hipSuccess) return e;
        }
        const int count = (int)(ctx->net.lay.n_params - ctx->net.lay.grid_params);
        timed_begin(ctx, "fused_dw_sum", s2, &tok);
        hipLaunchKernelGGL(k_dw_sum, dim3((count + 15) / 16), dim3(256), 0, s2, ctx->s_dw_part,
                           blocks, count, grad + ctx->net.lay.grid_params);
        timed_end(ctx, tok, s2);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
        if (bins) {
            e = binned_scatter(ctx, *bins, n, pos, perm, rec, a.rec_stride, dg_tiles, rows, grad,
                               ctx->s_bin_cnt, ctx->s_bin_items, s);
            if (e == hipSuccess) e = hipEventRecord(ctx->ev_join, s2);
            if (e == hipSuccess) e = hipStreamWaitEvent(s, ctx->ev_join, 0);
            if (e != hipSuccess) return e;
        }
    }
    if (!loss_out) return hipSuccess;
    e = launch_reduce_scaled(ctx->partials, blocks, 1.0 / (double)n, loss_out, s);
    if (e != hipSuccess || !(bsdf && a.wsel)) return e;
    return launch_reduce_scaled(a.partials_sel, blocks, 1.0 / (double)n, loss_out + 1, s);
}

}  // namespace npm
