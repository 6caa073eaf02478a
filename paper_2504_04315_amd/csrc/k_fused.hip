// Fused execution of the NPM hot path.  A wave owns a tile of 32 vertices and
// keeps it on chip from the grid lookup to the outputs:
//
//   query:     encode (Sec. 5.1) -> MLP on MFMA (Sec. 5.3) -> Table 1 mappings
//              -> mixture pdf at dir -> lobe selection and vMF sample (Jakob
//              2012) -> pdf at the sample.
//   backward:  encode -> MLP forward (activations in registers) -> KL-gradient
//              head (Sec. 4.2, eq. mcgradients) -> delta chain -> grid scatter
//              (FP32 atomics) and weight gradients (MFMA with the tile's
//              vertices as the reduction dimension, accumulated per wave).
//
// Tile layout (device_math.h): lane l holds vertex l % 32; of a feature vector
// the half-wave h = l / 32 holds the features nf(h, a).  After the output layer
// half h holds lobes k = 2r + h (r = 0..3), components in registers 4r..4r+3,
// so softmax, log-sum-exp and the lobe CDF need one exchange with lane l ^ 32.
//
// Precision form (BF16 = true): grid features read from an FP16 copy, MLP
// weights and activations in BF16 on v_mfma_f32_32x32x16_bf16 with FP32
// accumulation; mappings, softmax, log-density and sampling in FP32.
#include "device_math.h"

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
};

// ------------------------------------------------------------------ encode
// Features of the tile vertex for this half-wave: register 4 g + j F + f holds
// feature f of level (8 g + 4 h) / F + j.
template <int IN_P, int F, bool BF>
__device__ __forceinline__ void encode_tile(const FusedArgs &a, const uint32_t *s_off,
                                            const int *s_res, int h, float px, float py, float pz,
                                            float *x)
{
    constexpr int PER = 4 / F;   // levels per group and half
#pragma unroll
    for (int g = 0; g < IN_P / 8; ++g) {
#pragma unroll
        for (int j = 0; j < PER; ++j) {
            const int l = (8 * g + 4 * h) / F + j;
            float acc[F];
#pragma unroll
            for (int f = 0; f < F; ++f) acc[f] = 0.0f;
            if (l < a.g.n_levels) {
                const int D = s_res[l];
                int cx, cy, cz;
                float fx, fy, fz;
                lattice_cell(px, D, cx, fx);
                lattice_cell(py, D, cy, fy);
                lattice_cell(pz, D, cz, fz);
                const uint32_t d1 = (uint32_t)D + 1u;
                const bool hashed = (a.g.hashed_mask >> l) & 1u;
                const uint32_t off = s_off[l];
                float val[8][F];
#pragma unroll
                for (int b = 0; b < 8; ++b) {
                    const uint32_t X = cx + (b & 1), Y = cy + ((b >> 1) & 1), Z = cz + ((b >> 2) & 1);
                    const uint32_t e = off + (hashed ? ((X ^ (Y * 2654435761u) ^ (Z * 805459861u)) & a.g.table_mask)
                                                     : X + d1 * (Y + d1 * Z));
                    if constexpr (BF) {
                        if constexpr (F == 2) {
                            const __half2 t = *reinterpret_cast<const __half2 *>(a.grid16 + 2 * (size_t)e);
                            val[b][0] = __low2float(t); val[b][1] = __high2float(t);
                        } else {
#pragma unroll
                            for (int f = 0; f < F; ++f) val[b][f] = __half2float(a.grid16[(size_t)e * F + f]);
                        }
                    } else {
                        if constexpr (F == 1) {
                            val[b][0] = a.grid32[e];
                        } else if constexpr (F == 2) {
                            const float2 t = *reinterpret_cast<const float2 *>(a.grid32 + 2 * (size_t)e);
                            val[b][0] = t.x; val[b][1] = t.y;
                        } else {
                            const float4 t = *reinterpret_cast<const float4 *>(a.grid32 + 4 * (size_t)e);
                            val[b][0] = t.x; val[b][1] = t.y; val[b][2] = t.z; val[b][3] = t.w;
                        }
                    }
                }
                const float wx[2] = {1.0f - fx, fx}, wy[2] = {1.0f - fy, fy}, wz[2] = {1.0f - fz, fz};
#pragma unroll
                for (int b = 0; b < 8; ++b) {
                    const float w = wx[b & 1] * wy[(b >> 1) & 1] * wz[(b >> 2) & 1];
#pragma unroll
                    for (int f = 0; f < F; ++f) acc[f] += w * val[b][f];
                }
            }
#pragma unroll
            for (int f = 0; f < F; ++f) x[4 * g + j * F + f] = acc[f];
        }
    }
}

// ------------------------------------------------------------------ MLP
template <bool BF, int IN_P, int OUT_P>
__device__ __forceinline__ void layer(const void *img, const float *x, float *y, int lane)
{
    if constexpr (BF) mfma_layer_bf16<IN_P, OUT_P>((const __bf16 *)img, x, y, lane);
    else mfma_layer_f32<IN_P, OUT_P>((const float *)img, x, y, lane);
}

template <bool BF>
__device__ __forceinline__ const void *img_at(const void *base, int elems)
{
    return BF ? (const void *)((const __bf16 *)base + elems) : (const void *)((const float *)base + elems);
}

// Forward of all layers; hidden activations into acts[NH][HID_P/2] when KEEP.
template <int IN_P, int HID_P, int NH, bool BF, bool KEEP>
__device__ __forceinline__ void mlp_forward(const void *img, const float *x, float (*acts)[HID_P / 2],
                                            float *o, int lane)
{
    float a[HID_P / 2], b[HID_P / 2];
    layer<BF, IN_P, HID_P>(img, x, a, lane);
#pragma unroll
    for (int i = 0; i < HID_P / 2; ++i) a[i] = fmaxf(a[i], 0.0f);
    if constexpr (KEEP) {
#pragma unroll
        for (int i = 0; i < HID_P / 2; ++i) acts[0][i] = a[i];
    }
#pragma unroll
    for (int li = 1; li < NH; ++li) {
        layer<BF, HID_P, HID_P>(img_at<BF>(img, HID_P * IN_P + (li - 1) * HID_P * HID_P), a, b, lane);
#pragma unroll
        for (int i = 0; i < HID_P / 2; ++i) a[i] = fmaxf(b[i], 0.0f);
        if constexpr (KEEP) {
#pragma unroll
            for (int i = 0; i < HID_P / 2; ++i) acts[li][i] = a[i];
        }
    }
    layer<BF, HID_P, 32>(img_at<BF>(img, HID_P * IN_P + (NH - 1) * HID_P * HID_P), a, o, lane);
}

// ------------------------------------------------------------------ head
// The four lobes of this half-wave mapped from the raw outputs o[16], with the
// log-sum-exp of lambda' over all eight lobes.
__device__ __forceinline__ void map_half(const float *o, Lobe *L)
{
    float mx = fmaxf(fmaxf(o[3], o[7]), fmaxf(o[11], o[15]));
    mx = fmaxf(mx, xor32(mx));
    float se = 0.0f;
#pragma unroll
    for (int r = 0; r < 4; ++r) se += expf(o[4 * r + 3] - mx);
    se += xor32(se);
    const float lse = mx + logf(se);
#pragma unroll
    for (int r = 0; r < 4; ++r) map_lobe(o[4 * r], o[4 * r + 1], o[4 * r + 2], o[4 * r + 3], lse, L[r]);
}

// log V(w) over all eight lobes; lt[r] receives this half's log terms.
__device__ __forceinline__ float logpdf_half(const Lobe *L, float wx, float wy, float wz, float *lt)
{
    float m = -INFINITY;
#pragma unroll
    for (int r = 0; r < 4; ++r) { lt[r] = lobe_logterm(L[r], wx, wy, wz); m = fmaxf(m, lt[r]); }
    float s = 0.0f;
#pragma unroll
    for (int r = 0; r < 4; ++r) s += expf(lt[r] - m);
    const float mo = xor32(m), so = xor32(s);
    const float M = fmaxf(m, mo);
    const float S = s * expf(m - M) + so * expf(mo - M);
    return M + logf(S);
}

// ------------------------------------------------------------------ query
template <int IN_P, int HID_P, int NH, int F, bool BF>
__global__ __launch_bounds__(256) void k_query_fused(FusedArgs a)
{
    extern __shared__ __attribute__((aligned(16))) char smem[];
    __shared__ uint32_t s_off[NPM_MAX_LEVELS];
    __shared__ int s_res[NPM_MAX_LEVELS];
    {
        const int bytes = a.fwd_elems * (BF ? 2 : 4);
        for (int i = threadIdx.x; i < bytes / 16; i += blockDim.x)
            reinterpret_cast<f32x4 *>(smem)[i] = reinterpret_cast<const f32x4 *>(a.img)[i];
        if (threadIdx.x < NPM_MAX_LEVELS) {
            s_off[threadIdx.x] = a.g.offset[threadIdx.x];
            s_res[threadIdx.x] = a.g.res[threadIdx.x];
        }
    }
    __syncthreads();
    const int lane = threadIdx.x & 63, h = lane >> 5;
    const int64_t n = a.n;
    const int64_t ntiles = (n + 31) / 32;
    const int64_t nwaves = (int64_t)gridDim.x * (blockDim.x / 64);
    for (int64_t t = blockIdx.x * (int64_t)(blockDim.x / 64) + (threadIdx.x >> 6); t < ntiles;
         t += nwaves) {
        const int64_t v = t * 32 + (lane & 31);
        const bool valid = v < n;
        const int64_t vv = valid ? v : n - 1;
        const float px = a.pos[vv], py = a.pos[n + vv], pz = a.pos[2 * n + vv];
        float x[IN_P / 2];
        encode_tile<IN_P, F, BF>(a, s_off, s_res, h, px, py, pz, x);
        float o[16];
        mlp_forward<IN_P, HID_P, NH, BF, false>(smem, x, nullptr, o, lane);
        Lobe L[4];
        map_half(o, L);
        if (a.lobes && valid) {
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int k = 2 * r + h;
                a.lobes[(int64_t)(0 * kLobes + k) * n + v] = L[r].theta;
                a.lobes[(int64_t)(1 * kLobes + k) * n + v] = L[r].phi;
                a.lobes[(int64_t)(2 * kLobes + k) * n + v] = L[r].kappa;
                a.lobes[(int64_t)(3 * kLobes + k) * n + v] = expf(L[r].loglam);
            }
        }
        if (a.pdf) {
            const float wx = a.dir[vv], wy = a.dir[n + vv], wz = a.dir[2 * n + vv];
            float lt[4];
            const float lv = logpdf_half(L, wx, wy, wz, lt);
            if (valid && h == 0) a.pdf[v] = expf(lv);
        }
        if (a.sdir || a.spdf_out) {
            float u[3];
            philox_uniforms((uint64_t)vv, a.seed, a.sid, 0u, u);
            // lambda in lobe order 0..7: this half has k = 2r + h, the partner the rest
            float lam_own[4], lam_oth[4];
#pragma unroll
            for (int r = 0; r < 4; ++r) { lam_own[r] = expf(L[r].loglam); lam_oth[r] = xor32(lam_own[r]); }
            float C[kLobes], acc = 0.0f;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                acc += h == 0 ? lam_own[r] : lam_oth[r];
                C[2 * r] = acc;
                acc += h == 0 ? lam_oth[r] : lam_own[r];
                C[2 * r + 1] = acc;
            }
            const float target = u[0] * C[kLobes - 1];
            int sel = kLobes - 1;
#pragma unroll
            for (int k = kLobes - 2; k >= 0; --k) sel = (target < C[k]) ? k : sel;
            const int rs = sel >> 1;
            Lobe S = L[0];
#pragma unroll
            for (int r = 1; r < 4; ++r) if (r == rs) S = L[r];
            float w[3];
            lobe_sample(S, u[1], u[2], w);
            const bool mine = (sel & 1) == h;
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                const float other = xor32(w[d]);
                w[d] = mine ? w[d] : other;
            }
            float lt[4];
            const float lv = logpdf_half(L, w[0], w[1], w[2], lt);
            if (valid && h == 0) {
                if (a.sdir) { a.sdir[v] = w[0]; a.sdir[n + v] = w[1]; a.sdir[2 * n + v] = w[2]; }
                if (a.spdf_out) a.spdf_out[v] = expf(lv);
            }
        }
    }
}

// ------------------------------------------------------------------ backward
// Per tile: forward with activations in registers, the KL-gradient head, the
// delta chain (backward images: W^T as the A operand), the grid scatter, and
// the weight gradients.  For the weight gradients the tile's deltas and layer
// inputs are transposed through a per-wave LDS buffer (rows = features,
// 36-float stride) so that the 32 vertices become the MFMA reduction
// dimension; each wave accumulates dW over all its tiles in registers and
// writes one partial at the end.
constexpr int kStride = 36;   // LDS row stride (floats) of the transpose buffer

// Writes a T32-layout vector of width 2*REGS into the wave's LDS buffer.
template <int REGS>
__device__ __forceinline__ void t32_to_lds(float *buf, const float *x, int lane)
{
    const int h = lane >> 5, j = lane & 31;
#pragma unroll
    for (int a = 0; a < REGS; ++a) buf[nf(h, a) * kStride + j] = x[a];
}

// Reads rows [32 b, 32 b + 32) of the buffer transposed: lane l gets row
// 32 b + l % 32 at vertices 16 (l / 32) + s, s = 0..15.
__device__ __forceinline__ void lds_rows(const float *buf, int b, int lane, float *r)
{
    const float *p = buf + (32 * b + (lane & 31)) * kStride + 16 * (lane >> 5);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const f32x4 t = *reinterpret_cast<const f32x4 *>(p + 4 * q);
        r[4 * q] = t[0]; r[4 * q + 1] = t[1]; r[4 * q + 2] = t[2]; r[4 * q + 3] = t[3];
    }
}

__device__ __forceinline__ void wave_lds_fence()
{
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

// dW (OUT_P x IN_P block grid) += dz^T-contraction over the tile's vertices.
template <int OUT_P, int IN_P>
__device__ __forceinline__ void dw_tile(float *buf, const float *dz, const float *xin,
                                        f32x16 (*acc)[IN_P / 32], int lane)
{
    constexpr int NBO = OUT_P / 32, NBI = IN_P / 32;
    float A[NBO][16], Bv[NBI][16];
    wave_lds_fence();
    t32_to_lds<OUT_P / 2>(buf, dz, lane);
    wave_lds_fence();
#pragma unroll
    for (int b = 0; b < NBO; ++b) lds_rows(buf, b, lane, A[b]);
    wave_lds_fence();
    t32_to_lds<IN_P / 2>(buf, xin, lane);
    wave_lds_fence();
#pragma unroll
    for (int b = 0; b < NBI; ++b) lds_rows(buf, b, lane, Bv[b]);
#pragma unroll
    for (int s = 0; s < 16; ++s)
#pragma unroll
        for (int bo = 0; bo < NBO; ++bo)
#pragma unroll
            for (int bi = 0; bi < NBI; ++bi)
                acc[bo][bi] = __builtin_amdgcn_mfma_f32_32x32x2f32(A[bo][s], Bv[bi][s], acc[bo][bi], 0, 0, 0);
}

template <int OUT_P, int IN_P>
__device__ __forceinline__ void dw_store(float *dst, int out_r, int in_r, f32x16 (*acc)[IN_P / 32],
                                         int lane)
{
    const int h = lane >> 5, j = lane & 31;
#pragma unroll
    for (int bo = 0; bo < OUT_P / 32; ++bo)
#pragma unroll
        for (int bi = 0; bi < IN_P / 32; ++bi)
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int row = 32 * bo + nf(h, r), col = 32 * bi + j;
                if (row < out_r && col < in_r) dst[row * in_r + col] = acc[bo][bi][r];
            }
}

template <int IN_P, int HID_P, int NH, int F, bool BF>
__global__ __launch_bounds__(256) void k_backward_fused(FusedArgs a, int out_layers_in0)
{
    extern __shared__ __attribute__((aligned(16))) char smem[];
    __shared__ uint32_t s_off[NPM_MAX_LEVELS];
    __shared__ int s_res[NPM_MAX_LEVELS];
    __shared__ double red[256];
    constexpr int ESZ = BF ? 2 : 4;
    const int img_bytes = (a.fwd_elems + a.bwd_elems) * ESZ;
    for (int i = threadIdx.x; i < img_bytes / 16; i += blockDim.x)
        reinterpret_cast<f32x4 *>(smem)[i] = reinterpret_cast<const f32x4 *>(a.img)[i];
    if (threadIdx.x < NPM_MAX_LEVELS) {
        s_off[threadIdx.x] = a.g.offset[threadIdx.x];
        s_res[threadIdx.x] = a.g.res[threadIdx.x];
    }
    __syncthreads();
    const char *fwd = smem;
    const char *bwd = smem + (size_t)a.fwd_elems * ESZ;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, h = lane >> 5;
    float *tbuf = reinterpret_cast<float *>(smem + (((size_t)img_bytes + 15) / 16) * 16) +
                  wave * HID_P * kStride;
    constexpr int IN0 = IN_P < 32 ? 32 : IN_P;       // layer-0 input rows padded to a 32 block
    constexpr int OUT0 = IN0;
    // weight-gradient accumulators: layer 0 (HID x IN0), hidden (HID x HID), last (32 x HID)
    f32x16 acc0[HID_P / 32][IN0 / 32];
    f32x16 accH[NH > 1 ? NH - 1 : 1][HID_P / 32][HID_P / 32];
    f32x16 accL[1][HID_P / 32];
#pragma unroll
    for (int i = 0; i < HID_P / 32; ++i) {
#pragma unroll
        for (int j = 0; j < IN0 / 32; ++j) acc0[i][j] = 0.0f;
#pragma unroll
        for (int li = 0; li < (NH > 1 ? NH - 1 : 1); ++li)
#pragma unroll
            for (int j = 0; j < HID_P / 32; ++j) accH[li][i][j] = 0.0f;
        accL[0][i] = 0.0f;
    }
    double lacc = 0.0;
    const int64_t n = a.n;
    const int64_t ntiles = (n + 31) / 32;
    const int64_t nwaves = (int64_t)gridDim.x * (blockDim.x / 64);
    const int64_t gwave = blockIdx.x * (int64_t)(blockDim.x / 64) + wave;
    for (int64_t t = gwave; t < ntiles; t += nwaves) {
        const int64_t v = t * 32 + (lane & 31);
        const bool valid = v < n;
        const int64_t vv = valid ? v : n - 1;
        const float px = a.pos[vv], py = a.pos[n + vv], pz = a.pos[2 * n + vv];
        float x[IN0 / 2];
        encode_tile<IN_P, F, BF>(a, s_off, s_res, h, px, py, pz, x);
#pragma unroll
        for (int i = IN_P / 2; i < IN0 / 2; ++i) x[i] = 0.0f;
        float acts[NH][HID_P / 2];
        float o[16];
        mlp_forward<IN_P, HID_P, NH, BF, true>(fwd, x, acts, o, lane);
        // ---- KL-gradient head
        const float wgt = valid ? sample_weight(a.rad[vv], a.spdf[vv]) : 0.0f;
        float d[16];
#pragma unroll
        for (int i = 0; i < 16; ++i) d[i] = 0.0f;
        {
            Lobe L[4];
            map_half(o, L);
            const float wx = a.dir[vv], wy = a.dir[n + vv], wz = a.dir[2 * n + vv];
            float lt[4];
            const float lv = logpdf_half(L, wx, wy, wz, lt);
            if (wgt != 0.0f) {
                const float g = -wgt * a.invN;
#pragma unroll
                for (int r = 0; r < 4; ++r)
                    lobe_grad(L[r], o[4 * r], o[4 * r + 1], o[4 * r + 2], expf(lt[r] - lv),
                              expf(L[r].loglam), g, wx, wy, wz, d + 4 * r);
                if (h == 0) lacc -= (double)wgt * (double)lv;
            }
        }
        if (!a.grad) continue;          // loss only
        // ---- weight gradient of the output layer, then the delta chain
        dw_tile<32, HID_P>(tbuf, d, acts[NH - 1], accL, lane);
        float dh[HID_P / 2];
        layer<BF, 32, HID_P>(bwd, d, dh, lane);
        const char *im = bwd + (size_t)HID_P * 32 * ESZ;
#pragma unroll
        for (int li = NH - 1; li >= 0; --li) {
#pragma unroll
            for (int i = 0; i < HID_P / 2; ++i) dh[i] = acts[li][i] > 0.0f ? dh[i] : 0.0f;
            if (li > 0) {
                dw_tile<HID_P, HID_P>(tbuf, dh, acts[li - 1], accH[li - 1], lane);
                float nd[HID_P / 2];
                layer<BF, HID_P, HID_P>(im, dh, nd, lane);
                im += (size_t)HID_P * HID_P * ESZ;
#pragma unroll
                for (int i = 0; i < HID_P / 2; ++i) dh[i] = nd[i];
            } else {
                dw_tile<HID_P, IN0>(tbuf, dh, x, acc0, lane);
            }
        }
        float dG[OUT0 / 2];
        layer<BF, HID_P, OUT0>(im, dh, dG, lane);
        // ---- grid scatter: recompute this half's corners, add w * dG
        if (valid) {
            constexpr int PER = 4 / F;
#pragma unroll
            for (int g = 0; g < IN_P / 8; ++g) {
#pragma unroll
                for (int j = 0; j < PER; ++j) {
                    const int l = (8 * g + 4 * h) / F + j;
                    if (l >= a.g.n_levels) continue;
                    float df[F];
                    bool any = false;
#pragma unroll
                    for (int f = 0; f < F; ++f) { df[f] = dG[4 * g + j * F + f]; any |= df[f] != 0.0f; }
                    if (!any) continue;
                    const int D = s_res[l];
                    int cx, cy, cz;
                    float fx, fy, fz;
                    lattice_cell(px, D, cx, fx);
                    lattice_cell(py, D, cy, fy);
                    lattice_cell(pz, D, cz, fz);
                    const uint32_t d1 = (uint32_t)D + 1u;
                    const bool hashed = (a.g.hashed_mask >> l) & 1u;
                    const float wxs[2] = {1.0f - fx, fx}, wys[2] = {1.0f - fy, fy}, wzs[2] = {1.0f - fz, fz};
#pragma unroll
                    for (int b = 0; b < 8; ++b) {
                        const uint32_t X = cx + (b & 1), Y = cy + ((b >> 1) & 1), Z = cz + ((b >> 2) & 1);
                        const uint32_t e = s_off[l] + (hashed ? ((X ^ (Y * 2654435761u) ^ (Z * 805459861u)) & a.g.table_mask)
                                                              : X + d1 * (Y + d1 * Z));
                        const float w = wxs[b & 1] * wys[(b >> 1) & 1] * wzs[(b >> 2) & 1];
#pragma unroll
                        for (int f = 0; f < F; ++f) unsafeAtomicAdd(a.grad + (size_t)e * F + f, w * df[f]);
                    }
                }
            }
        }
    }
    // ---- loss partial of the block (FP64)
    red[threadIdx.x] = lacc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) a.partials[blockIdx.x] = red[0];
    if (!a.grad) return;
    // ---- per-wave weight-gradient partials, in the flat layer layout
    const int nw = a.width;
    float *dst = a.dw_part + gwave * (int64_t)(out_layers_in0);
    dw_store<HID_P, IN0>(dst, nw, a.n_in, acc0, lane);
    dst += nw * a.n_in;
#pragma unroll
    for (int li = 0; li < NH - 1; ++li) {
        dw_store<HID_P, HID_P>(dst, nw, nw, accH[li], lane);
        dst += nw * nw;
    }
    dw_store<32, HID_P>(dst, 32, nw, accL, lane);
}

// Sums the per-wave partials of the MLP weight gradient into grad.
__global__ void k_dw_sum(const float *__restrict__ part, int nparts, int count,
                         float *__restrict__ grad)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    float s = 0.0f;
    for (int p = 0; p < nparts; ++p) s += part[(int64_t)p * count + i];
    grad[i] += s;
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
    return a;
}

template <int IN_P, int HID_P, int NH, int F, bool BF>
static hipError_t run_query(npm_ctx *ctx, FusedArgs a, hipStream_t s)
{
    const int64_t tiles = (a.n + 31) / 32;
    const int blocks = (int)std::max<int64_t>(1, std::min<int64_t>((tiles + 3) / 4, 2048));
    const size_t lds = (size_t)a.fwd_elems * (BF ? 2 : 4);
    auto k = k_query_fused<IN_P, HID_P, NH, F, BF>;
    hipFuncSetAttribute((const void *)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    hipLaunchKernelGGL(k, dim3(blocks), dim3(256), lds, s, a);
    return hipGetLastError();
}

// Number of waves the backward kernel runs (one partial each).
static int backward_waves(int64_t n)
{
    const int64_t tiles = (n + 31) / 32;
    return (int)std::max<int64_t>(4, std::min<int64_t>(((tiles + 3) / 4) * 4, 1024));
}

template <int IN_P, int HID_P, int NH, int F, bool BF>
static hipError_t run_backward(npm_ctx *ctx, FusedArgs a, hipStream_t s)
{
    const int waves = backward_waves(a.n);
    const int blocks = waves / 4;
    const size_t img = ((size_t)(a.fwd_elems + a.bwd_elems) * (BF ? 2 : 4) + 15) / 16 * 16;
    const size_t lds = img + (size_t)4 * HID_P * kStride * sizeof(float);
    const int count = (int)(ctx->net.lay.n_params - ctx->net.lay.grid_params);
    auto k = k_backward_fused<IN_P, HID_P, NH, F, BF>;
    hipFuncSetAttribute((const void *)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    hipLaunchKernelGGL(k, dim3(blocks), dim3(256), lds, s, a, count);
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

hipError_t fused_query(npm_ctx *ctx, int64_t n, const float *pos, const float *dir, uint64_t seed,
                       uint32_t stream_id, float *lobes, float *pdf, float *sdir, float *spdf,
                       hipStream_t s)
{
    FusedArgs a = fused_args(ctx, n, pos);
    a.dir = dir;
    a.seed = seed;
    a.sid = stream_id;
    a.lobes = lobes;
    a.pdf = pdf;
    a.sdir = sdir;
    a.spdf_out = spdf;
    hipError_t e = hipSuccess;
    int tok;
    timed_begin(ctx, "fused_query", s, &tok);
    if (ctx->net.cfg.precision == NPM_PREC_BF16) NPM_FUSED_DISPATCH(run_query, true);
    else NPM_FUSED_DISPATCH(run_query, false);
    timed_end(ctx, tok, s);
    return e;
}

hipError_t fused_backward(npm_ctx *ctx, int64_t n, const float *pos, const float *dir,
                          const float *rad, const float *spdf, float *grad, double *loss_out,
                          hipStream_t s)
{
    FusedArgs a = fused_args(ctx, n, pos);
    a.dir = dir;
    a.rad = rad;
    a.spdf = spdf;
    a.grad = grad;
    a.dw_part = ctx->s_dw_part;
    a.partials = ctx->partials;
    a.invN = 1.0f / (float)n;
    hipError_t e = hipSuccess;
    int tok;
    timed_begin(ctx, "fused_backward", s, &tok);
    if (ctx->net.cfg.precision == NPM_PREC_BF16) NPM_FUSED_DISPATCH(run_backward, true);
    else NPM_FUSED_DISPATCH(run_backward, false);
    timed_end(ctx, tok, s);
    if (e != hipSuccess) return e;
    const int waves = backward_waves(n);
    if (grad) {
        const int count = (int)(ctx->net.lay.n_params - ctx->net.lay.grid_params);
        timed_begin(ctx, "fused_dw_sum", s, &tok);
        hipLaunchKernelGGL(k_dw_sum, dim3((count + 255) / 256), dim3(256), 0, s, ctx->s_dw_part,
                           waves, count, grad + ctx->net.lay.grid_params);
        timed_end(ctx, tok, s);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    if (loss_out) return launch_reduce_scaled(ctx->partials, waves / 4, 1.0 / (double)n, loss_out, s);
    return hipSuccess;
}

}  // namespace npm
