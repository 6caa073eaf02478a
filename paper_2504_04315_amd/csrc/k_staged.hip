// The per-stage ("staged") execution of the NPM hot path: one kernel per step,
// intermediate per-vertex arrays in HBM in feature-major layout ([feature][n],
// coalesced over vertices).  It is the plain FP32 baseline the fused forms are
// measured against, and the path whose stages are checked one by one.
//
//   encode      Sec. 5.1   G(x): 8-corner trilinear gather per level, concat
//   mlp_fwd     Sec. 5.3   ReLU MLP on 32x32 FP32 MFMA tiles, weights in LDS
//   head        Table 1 + vMF mixture pdf + sampling (Sec. 5.3, Jakob 2012)
//   loss_grad   Sec. 4.2   eq. mcgradients through the Table 1 mappings
//   mlp_bwd     backprop of the MLP (delta chain and dG)
//   mlp_dw      weight gradients, batch as the MFMA reduction dimension
//   scatter     dG into the eight corners of every level (FP32 atomics)
//
// With the learned BSDF-selection probability (Sec. 6.3, Discussion) the last
// layer has one more row: its output c' is a dot product of the last hidden
// layer with that row, folded into mlp_fwd; its derivative is written by
// loss_grad and added back by mlp_bwd, and mlp_dw treats the 33 rows as one
// matrix.
#include "device_math.h"

namespace npm {

// ============================================================= corner index
__global__ __launch_bounds__(256) void k_corner_index(GridDesc g, int64_t n,
                                                      const float *__restrict__ pos,
                                                      uint32_t *__restrict__ idx)
{
    const int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const int l = blockIdx.y;
    if (v >= n) return;
    Corners c;
    level_corners(g, l, pos[v], pos[n + v], pos[2 * n + v], c);
#pragma unroll
    for (int b = 0; b < 8; ++b) idx[((int64_t)l * 8 + b) * n + v] = c.e[b];
}

hipError_t staged_corner_index(npm_ctx *ctx, int64_t n, const float *pos, uint32_t *idx,
                               hipStream_t s)
{
    const GridDesc &g = ctx->net.grid;
    dim3 grid((unsigned)((n + 255) / 256), (unsigned)g.n_levels);
    hipLaunchKernelGGL(k_corner_index, grid, dim3(256), 0, s, g, n, pos, idx);
    return hipGetLastError();
}

// ============================================================= encode
template <int F>
__device__ __forceinline__ void load_feat(const float *__restrict__ grid, uint32_t e, float *v)
{
    if constexpr (F == 1) {
        v[0] = grid[e];
    } else if constexpr (F == 2) {
        const float2 t = *reinterpret_cast<const float2 *>(grid + 2 * (size_t)e);
        v[0] = t.x; v[1] = t.y;
    } else {
        const float4 t = *reinterpret_cast<const float4 *>(grid + 4 * (size_t)e);
        v[0] = t.x; v[1] = t.y; v[2] = t.z; v[3] = t.w;
    }
}

// One thread per (vertex, level): the level is uniform across the block.
template <int F>
__global__ __launch_bounds__(256) void k_encode(GridDesc g, int64_t n, const float *__restrict__ pos,
                                                const float *__restrict__ grid,
                                                float *__restrict__ G)
{
    const int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const int l = blockIdx.y;
    if (v >= n) return;
    Corners c;
    level_corners(g, l, pos[v], pos[n + v], pos[2 * n + v], c);
    float acc[F];
#pragma unroll
    for (int f = 0; f < F; ++f) acc[f] = 0.0f;
#pragma unroll
    for (int b = 0; b < 8; ++b) {
        float val[F];
        load_feat<F>(grid, c.e[b], val);
#pragma unroll
        for (int f = 0; f < F; ++f) acc[f] += c.w[b] * val[f];
    }
#pragma unroll
    for (int f = 0; f < F; ++f) G[((int64_t)l * F + f) * n + v] = acc[f];
}

// NPM-product rows of the MLP input: G[gf + k][v] for the SH of omega_o
// (d^2 values), of the normal (d^2), and the roughness; aux is [7][n].
__global__ void k_aux_rows(int64_t n, int gf, int deg, const float *__restrict__ aux,
                           float *__restrict__ G)
{
    const int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (v >= n) return;
    const int nb = deg * deg;
    float y[16];
    sh_bands4(aux[v], aux[n + v], aux[2 * n + v], y);
    for (int k = 0; k < nb; ++k) G[(int64_t)(gf + k) * n + v] = y[k];
    sh_bands4(aux[3 * n + v], aux[4 * n + v], aux[5 * n + v], y);
    for (int k = 0; k < nb; ++k) G[(int64_t)(gf + nb + k) * n + v] = y[k];
    G[(int64_t)(gf + 2 * nb) * n + v] = aux[6 * n + v];
}

hipError_t staged_encode(npm_ctx *ctx, int64_t n, const float *pos, float *G, hipStream_t s,
                         const Weights *w, const float *aux)
{
    const GridDesc &g = ctx->net.grid;
    const float *table = w ? w->grid32 : ctx->params;
    dim3 grid((unsigned)((n + 255) / 256), (unsigned)g.n_levels);
    int tok;
    timed_begin(ctx, "staged_encode", s, &tok);
    switch (g.feat) {
    case 1: hipLaunchKernelGGL(k_encode<1>, grid, dim3(256), 0, s, g, n, pos, table, G); break;
    case 2: hipLaunchKernelGGL(k_encode<2>, grid, dim3(256), 0, s, g, n, pos, table, G); break;
    case 4: hipLaunchKernelGGL(k_encode<4>, grid, dim3(256), 0, s, g, n, pos, table, G); break;
    default: return hipErrorInvalidValue;
    }
    if (ctx->net.mlp.sh_degree > 0)
        hipLaunchKernelGGL(k_aux_rows, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n,
                           ctx->net.mlp.gf, ctx->net.mlp.sh_degree, aux, G);
    timed_end(ctx, tok, s);
    return hipGetLastError();
}

// ============================================================= MLP helpers
// Copies `count` floats (multiple of 4) of a packed image into LDS.
__device__ __forceinline__ void stage_image(float *lds, const float *__restrict__ img, int count)
{
    for (int i = threadIdx.x; i < count / 4; i += blockDim.x)
        reinterpret_cast<f32x4 *>(lds)[i] = reinterpret_cast<const f32x4 *>(img)[i];
}

// Loads W = 2*REGS features of tile vertex v from a feature-major array with
// `rows` real rows (zero beyond them or beyond n).
template <int REGS>
__device__ __forceinline__ void load_tile(const float *__restrict__ src, int rows, int64_t n,
                                          int64_t v, int h, float *x)
{
#pragma unroll
    for (int a = 0; a < REGS; ++a) {
        const int f = nf(h, a);
        x[a] = (v < n && f < rows) ? src[(int64_t)f * n + v] : 0.0f;
    }
}

template <int REGS>
__device__ __forceinline__ void store_tile(float *__restrict__ dst, int rows, int64_t n, int64_t v,
                                           int h, const float *x)
{
#pragma unroll
    for (int a = 0; a < REGS; ++a) {
        const int f = nf(h, a);
        if (v < n && f < rows) dst[(int64_t)f * n + v] = x[a];
    }
}

// ============================================================= MLP forward
// Wave tiles of 32 vertices in a grid-stride loop; all layer images in LDS.
// acts (optional) receives every hidden layer's output [n_hidden][width][n].
// wsel (or null): the selection row of the last layer, width weights; its
// output goes to raw row kOut.
template <int IN_P, int HID_P, int NH>
__global__ __launch_bounds__(256) void k_mlp_fwd(int64_t n, int n_in, int width,
                                                 const float *__restrict__ img, int img_elems,
                                                 const float *__restrict__ G,
                                                 float *__restrict__ acts, float *__restrict__ raw,
                                                 const float *__restrict__ wsel)
{
    extern __shared__ float lds[];
    stage_image(lds, img, img_elems);
    __syncthreads();
    const int lane = threadIdx.x & 63, h = lane >> 5;
    const int64_t ntiles = (n + 31) / 32;
    const int64_t wave = blockIdx.x * (int64_t)(blockDim.x / 64) + (threadIdx.x >> 6);
    const int64_t nwaves = (int64_t)gridDim.x * (blockDim.x / 64);
    constexpr int L0 = 0, L1 = HID_P * IN_P;           // image offsets of layer 0 and 1
    for (int64_t t = wave; t < ntiles; t += nwaves) {
        const int64_t v = t * 32 + (lane & 31);
        float x[IN_P / 2], a[HID_P / 2], b[HID_P / 2];
        load_tile<IN_P / 2>(G, n_in, n, v, h, x);
        mfma_layer_f32<IN_P, HID_P>(lds + L0, x, a, lane);
#pragma unroll
        for (int i = 0; i < HID_P / 2; ++i) a[i] = fmaxf(a[i], 0.0f);
        if (acts) store_tile<HID_P / 2>(acts, width, n, v, h, a);
#pragma unroll
        for (int layer = 1; layer < NH; ++layer) {
            mfma_layer_f32<HID_P, HID_P>(lds + L1 + (layer - 1) * HID_P * HID_P, a, b, lane);
#pragma unroll
            for (int i = 0; i < HID_P / 2; ++i) a[i] = fmaxf(b[i], 0.0f);
            if (acts) store_tile<HID_P / 2>(acts + (int64_t)layer * width * n, width, n, v, h, a);
        }
        float o[16];
        mfma_layer_f32<HID_P, 32>(lds + L1 + (NH - 1) * HID_P * HID_P, a, o, lane);
        store_tile<16>(raw, 32, n, v, h, o);
        if (wsel) {
            // the two half-waves hold the two halves of a vertex's features
            float part = 0.0f;
#pragma unroll
            for (int i = 0; i < HID_P / 2; ++i) {
                const int f = nf(h, i);
                if (f < width) part = fmaf(wsel[f], a[i], part);
            }
            part += __shfl_xor(part, 32);
            if (h == 0 && v < n) raw[(int64_t)kOut * n + v] = part;
        }
    }
}

// ============================================================= MLP backward
// delta chain: d = draw; for the output layer dh = W^T d, then for each hidden
// layer (from the last) dz = dh * [h > 0] (stored for the weight gradient) and
// dh = W^T dz; finally dG = W_0^T dz_0.  Transposed images come packed.
// wsel (or null): the selection row; its derivative (draw row kOut) adds
// d c' / d h = wsel to the last hidden layer's delta.
template <int IN_P, int HID_P, int NH>
__global__ __launch_bounds__(256) void k_mlp_bwd(int64_t n, int n_in, int width,
                                                 const float *__restrict__ img, int img_elems,
                                                 const float *__restrict__ draw,
                                                 const float *__restrict__ acts,
                                                 float *__restrict__ delta, float *__restrict__ dG,
                                                 const float *__restrict__ wsel)
{
    extern __shared__ float lds[];
    stage_image(lds, img, img_elems);
    __syncthreads();
    const int lane = threadIdx.x & 63, h = lane >> 5;
    const int64_t ntiles = (n + 31) / 32;
    const int64_t wave = blockIdx.x * (int64_t)(blockDim.x / 64) + (threadIdx.x >> 6);
    const int64_t nwaves = (int64_t)gridDim.x * (blockDim.x / 64);
    // backward image order: layer NH (HID_P x 32), NH-1 .. 1 (HID_P x HID_P), 0
    constexpr int OUT0 = IN_P < 32 ? 32 : IN_P;
    for (int64_t t = wave; t < ntiles; t += nwaves) {
        const int64_t v = t * 32 + (lane & 31);
        float d[16], dh[HID_P / 2], hv[HID_P / 2];
        load_tile<16>(draw, 32, n, v, h, d);
        const float *im = lds;
        mfma_layer_f32<32, HID_P>(im, d, dh, lane);
        im += HID_P * 32;
        if (wsel) {
            const float ds = v < n ? draw[(int64_t)kOut * n + v] : 0.0f;
#pragma unroll
            for (int i = 0; i < HID_P / 2; ++i) {
                const int f = nf(h, i);
                if (f < width) dh[i] = fmaf(ds, wsel[f], dh[i]);
            }
        }
#pragma unroll
        for (int layer = NH - 1; layer >= 0; --layer) {
            load_tile<HID_P / 2>(acts + (int64_t)layer * width * n, width, n, v, h, hv);
#pragma unroll
            for (int i = 0; i < HID_P / 2; ++i) dh[i] = hv[i] > 0.0f ? dh[i] : 0.0f;
            store_tile<HID_P / 2>(delta + (int64_t)layer * width * n, width, n, v, h, dh);
            if (layer > 0) {
                float nd[HID_P / 2];
                mfma_layer_f32<HID_P, HID_P>(im, dh, nd, lane);
                im += HID_P * HID_P;
#pragma unroll
                for (int i = 0; i < HID_P / 2; ++i) dh[i] = nd[i];
            }
        }
        float g[OUT0 / 2];
        mfma_layer_f32<HID_P, OUT0>(im, dh, g, lane);
        store_tile<OUT0 / 2>(dG, n_in, n, v, h, g);
    }
}

// ============================================================= weight gradient
// dW[o][i] = sum_v dz[o][v] x[i][v] for one layer, the batch as the MFMA K
// dimension: at step s lane l supplies dz[32 bo + l%32][v0 + 16 (l/32) + s] and
// x[32 bi + l%32][same vertex].  Each block reduces its four waves in LDS and
// writes one partial matrix; k_dw_reduce sums the partials in block order.
template <int OUT_P, int IN_P>
__global__ __launch_bounds__(256) void k_dw(int64_t n, int out_r, int in_r,
                                            const float *__restrict__ dz,
                                            const float *__restrict__ x,
                                            float *__restrict__ part)
{
    constexpr int NBO = OUT_P / 32, NBI = IN_P / 32;
    const int lane = threadIdx.x & 63, h = lane >> 5, j = lane & 31;
    const int w = threadIdx.x >> 6;
    f32x16 acc[NBO][NBI];
#pragma unroll
    for (int a = 0; a < NBO; ++a)
#pragma unroll
        for (int b = 0; b < NBI; ++b)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[a][b][r] = 0.0f;
    const int64_t ntiles = (n + 31) / 32;
    for (int64_t t = blockIdx.x * 4 + w; t < ntiles; t += (int64_t)gridDim.x * 4) {
        const int64_t v0 = t * 32 + 16 * h;
        float A[NBO][16], B[NBI][16];
#pragma unroll
        for (int a = 0; a < NBO; ++a) {
            const int row = 32 * a + j;
#pragma unroll
            for (int s = 0; s < 16; ++s)
                A[a][s] = (row < out_r && v0 + s < n) ? dz[(int64_t)row * n + v0 + s] : 0.0f;
        }
#pragma unroll
        for (int b = 0; b < NBI; ++b) {
            const int row = 32 * b + j;
#pragma unroll
            for (int s = 0; s < 16; ++s)
                B[b][s] = (row < in_r && v0 + s < n) ? x[(int64_t)row * n + v0 + s] : 0.0f;
        }
#pragma unroll
        for (int s = 0; s < 16; ++s)
#pragma unroll
            for (int a = 0; a < NBO; ++a)
#pragma unroll
                for (int b = 0; b < NBI; ++b)
                    acc[a][b] = __builtin_amdgcn_mfma_f32_32x32x2f32(A[a][s], B[b][s], acc[a][b],
                                                                     0, 0, 0);
    }
    // reduce the 4 waves of the block through LDS, one (a, b) block at a time
    __shared__ float red[4][1024];
    float *mine = part + (int64_t)blockIdx.x * out_r * in_r;
#pragma unroll
    for (int a = 0; a < NBO; ++a)
#pragma unroll
        for (int b = 0; b < NBI; ++b) {
#pragma unroll
            for (int r = 0; r < 16; ++r) red[w][r * 64 + lane] = acc[a][b][r];
            __syncthreads();
            for (int q = threadIdx.x; q < 1024; q += 256) {
                const float s = red[0][q] + red[1][q] + red[2][q] + red[3][q];
                const int r = q >> 6, ln = q & 63;
                const int row = 32 * a + 8 * (r >> 2) + 4 * (ln >> 5) + (r & 3);
                const int col = 32 * b + (ln & 31);
                if (row < out_r && col < in_r) mine[(int64_t)row * in_r + col] = s;
            }
            __syncthreads();
        }
}

// Sums the blocks' partial matrices into the gradient.  Eight independent
// running sums (partials b = k mod 8), added in a fixed order at the end, keep
// eight loads in flight per thread: with one sum a thread waited for every
// load in turn (61 us per layer for 256 partials of a 64 x 64 matrix).
__global__ void k_dw_reduce(const float *__restrict__ part, int nblocks, int count,
                            float *__restrict__ grad)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    float s[8] = {0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
    int b = 0;
    for (; b + 8 <= nblocks; b += 8)
#pragma unroll
        for (int k = 0; k < 8; ++k) s[k] += part[(int64_t)(b + k) * count + i];
    for (int k = 0; b + k < nblocks; ++k) s[k] += part[(int64_t)(b + k) * count + i];
    grad[i] += ((s[0] + s[1]) + (s[2] + s[3])) + ((s[4] + s[5]) + (s[6] + s[7]));
}

// ============================================================= head (query)
// One thread per vertex over the 32 raw outputs in [32][n]; sel (or null)
// receives the selection probability sigmoid(raw row kOut).
__global__ __launch_bounds__(256) void k_head(int64_t n, const float *__restrict__ raw,
                                              const float *__restrict__ dir, uint64_t seed,
                                              uint32_t sid, float *__restrict__ lobes,
                                              float *__restrict__ pdf, float *__restrict__ sdir,
                                              float *__restrict__ spdf, float *__restrict__ sel)
{
    const int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (v >= n) return;
    if (sel) sel[v] = 1.0f / (1.0f + expf(-raw[(int64_t)kOut * n + v]));
    if (!lobes && !pdf && !sdir && !spdf) return;
    float r[32];
#pragma unroll
    for (int j = 0; j < 32; ++j) r[j] = raw[(int64_t)j * n + v];
    float mx = r[3];
#pragma unroll
    for (int k = 1; k < kLobes; ++k) mx = fmaxf(mx, r[4 * k + 3]);
    float se = 0.0f;
#pragma unroll
    for (int k = 0; k < kLobes; ++k) se += expf(r[4 * k + 3] - mx);
    const float lse = mx + logf(se);
    Lobe L[kLobes];
#pragma unroll
    for (int k = 0; k < kLobes; ++k) map_lobe(r[4 * k], r[4 * k + 1], r[4 * k + 2], r[4 * k + 3], lse, L[k]);
    if (lobes) {
#pragma unroll
        for (int k = 0; k < kLobes; ++k) {
            lobes[(int64_t)(0 * kLobes + k) * n + v] = L[k].theta;
            lobes[(int64_t)(1 * kLobes + k) * n + v] = L[k].phi;
            lobes[(int64_t)(2 * kLobes + k) * n + v] = L[k].kappa;
            lobes[(int64_t)(3 * kLobes + k) * n + v] = expf(L[k].loglam);
        }
    }
    if (pdf && dir) {
        const float wx = dir[v], wy = dir[n + v], wz = dir[2 * n + v];
        float lt[kLobes], m = -INFINITY;
#pragma unroll
        for (int k = 0; k < kLobes; ++k) { lt[k] = lobe_logterm(L[k], wx, wy, wz); m = fmaxf(m, lt[k]); }
        float s = 0.0f;
#pragma unroll
        for (int k = 0; k < kLobes; ++k) s += expf(lt[k] - m);
        pdf[v] = expf(m + logf(s));
    }
    if (sdir || spdf) {
        float u[3];
        philox_uniforms((uint64_t)v, seed, sid, 0u, u);
        float C[kLobes], acc = 0.0f;
#pragma unroll
        for (int k = 0; k < kLobes; ++k) { acc += expf(L[k].loglam); C[k] = acc; }
        const float target = u[0] * C[kLobes - 1];
        int sel = kLobes - 1;
#pragma unroll
        for (int k = kLobes - 2; k >= 0; --k) sel = (target < C[k]) ? k : sel;
        Lobe S = L[0];
#pragma unroll
        for (int k = 1; k < kLobes; ++k) if (k == sel) S = L[k];
        float w[3];
        lobe_sample(S, u[1], u[2], w);
        if (sdir) { sdir[v] = w[0]; sdir[n + v] = w[1]; sdir[2 * n + v] = w[2]; }
        if (spdf) {
            float lt[kLobes], m = -INFINITY;
#pragma unroll
            for (int k = 0; k < kLobes; ++k) { lt[k] = lobe_logterm(L[k], w[0], w[1], w[2]); m = fmaxf(m, lt[k]); }
            float s = 0.0f;
#pragma unroll
            for (int k = 0; k < kLobes; ++k) s += expf(lt[k] - m);
            spdf[v] = expf(m + logf(s));
        }
    }
}

// ============================================================= loss gradient
// draw[kOut (+1)][n] = d loss / d raw, loss partial sums of -w log V in FP64.
// sel: the network has the selection output (draw row kOut is written: the
// selection term's derivative where bsdf is given and the sample's density
// is finite and >= 0, else 0); its loss partial sums go to partials_sel.
__global__ __launch_bounds__(256) void k_loss_grad(int64_t n, const float *__restrict__ raw,
                                                   const float *__restrict__ dir,
                                                   const float *__restrict__ rad,
                                                   const float *__restrict__ spdf, float invN,
                                                   float *__restrict__ draw,
                                                   double *__restrict__ partials, int sel,
                                                   const float *__restrict__ bsdf,
                                                   double *__restrict__ partials_sel)
{
    double lacc = 0.0, sacc = 0.0;
    for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n;
         v += (int64_t)gridDim.x * blockDim.x) {
        const float wgt = sample_weight(rad[v], spdf[v]);
        float out[32], ds = 0.0f;
#pragma unroll
        for (int j = 0; j < 32; ++j) out[j] = 0.0f;
        if (wgt != 0.0f) {
            float r[32];
#pragma unroll
            for (int j = 0; j < 32; ++j) r[j] = raw[(int64_t)j * n + v];
            float mx = r[3];
#pragma unroll
            for (int k = 1; k < kLobes; ++k) mx = fmaxf(mx, r[4 * k + 3]);
            float se = 0.0f;
#pragma unroll
            for (int k = 0; k < kLobes; ++k) se += expf(r[4 * k + 3] - mx);
            const float lse = mx + logf(se);
            const float wx = dir[v], wy = dir[n + v], wz = dir[2 * n + v];
            Lobe L[kLobes];
            float lt[kLobes], m = -INFINITY;
#pragma unroll
            for (int k = 0; k < kLobes; ++k) {
                map_lobe(r[4 * k], r[4 * k + 1], r[4 * k + 2], r[4 * k + 3], lse, L[k]);
                lt[k] = lobe_logterm(L[k], wx, wy, wz);
                m = fmaxf(m, lt[k]);
            }
            float s = 0.0f;
#pragma unroll
            for (int k = 0; k < kLobes; ++k) s += expf(lt[k] - m);
            const float lv = m + logf(s);
            const float g = -wgt * invN;
#pragma unroll
            for (int k = 0; k < kLobes; ++k)
                lobe_grad(L[k], r[4 * k], r[4 * k + 1], r[4 * k + 2], expf(lt[k] - lv),
                          expf(L[k].loglam), g, wx, wy, wz, out + 4 * k);
            lacc -= (double)wgt * (double)lv;
            if (sel && bsdf) {
                const float pb = bsdf[v];
                if (isfinite(pb) && pb >= 0.0f) {
                    const float lpc = select_term(raw[(int64_t)kOut * n + v], pb, lv, g, ds);
                    sacc -= (double)wgt * (double)lpc;
                }
            }
        }
#pragma unroll
        for (int j = 0; j < 32; ++j) draw[(int64_t)j * n + v] = out[j];
        if (sel) draw[(int64_t)kOut * n + v] = ds;
    }
    __shared__ double red[2][256];
    red[0][threadIdx.x] = lacc;
    red[1][threadIdx.x] = sacc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            red[0][threadIdx.x] += red[0][threadIdx.x + w];
            red[1][threadIdx.x] += red[1][threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        partials[blockIdx.x] = red[0][0];
        if (partials_sel) partials_sel[blockIdx.x] = red[1][0];
    }
}

// ============================================================= scatter
// dV_l[corner] += w_corner * dG[l F + f] with FP32 atomics.  Their throughput
// is set by the distinct 64-byte lines per wave instruction, so 8F
// consecutive threads take the corners x features of one vertex (the
// x-adjacent corners and the features of an entry are contiguous) and a wave
// covers 64 / (8F) consecutive vertices of one level.
template <int F>
__global__ __launch_bounds__(256) void k_scatter(GridDesc g, int64_t n, const float *__restrict__ pos,
                                                 const float *__restrict__ dG,
                                                 float *__restrict__ grad)
{
    constexpr int LPV = 8 * F;
    const int64_t gid = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const int64_t v = gid / LPV;
    const int sub = (int)(gid % LPV), b = sub / F, f = sub % F;
    const int l = blockIdx.y;
    if (v >= n) return;
    const float d = dG[((int64_t)l * F + f) * n + v];
    if (d == 0.0f) return;
    const int D = g.res[l];
    int cx, cy, cz;
    float fx, fy, fz;
    lattice_cell(pos[v], D, cx, fx);
    lattice_cell(pos[n + v], D, cy, fy);
    lattice_cell(pos[2 * n + v], D, cz, fz);
    const int bx = b & 1, by = (b >> 1) & 1, bz = (b >> 2) & 1;
    const uint32_t e = corner_entry(g, l, cx + bx, cy + by, cz + bz);
    const float w = (bx ? fx : 1.0f - fx) * (by ? fy : 1.0f - fy) * (bz ? fz : 1.0f - fz);
    unsafeAtomicAdd(grad + (size_t)e * F + f, w * d);
}

// ============================================================= launchers
#define NPM_MLP_DISPATCH(KERNEL, ...)                                                             \
    do {                                                                                          \
        const MlpDesc &m_ = ctx->net.mlp;                                                         \
        const int key_ = (m_.in_p / 16) * 100 + (m_.hid_p == 64) * 10 + m_.n_hidden;              \
        switch (key_) {                                                                           \
        case 101: KERNEL<16, 32, 1> __VA_ARGS__; break;                                               \
        case 102: KERNEL<16, 32, 2> __VA_ARGS__; break;                                               \
        case 103: KERNEL<16, 32, 3> __VA_ARGS__; break;                                               \
        case 104: KERNEL<16, 32, 4> __VA_ARGS__; break;                                               \
        case 111: KERNEL<16, 64, 1> __VA_ARGS__; break;                                               \
        case 112: KERNEL<16, 64, 2> __VA_ARGS__; break;                                               \
        case 113: KERNEL<16, 64, 3> __VA_ARGS__; break;                                               \
        case 114: KERNEL<16, 64, 4> __VA_ARGS__; break;                                               \
        case 201: KERNEL<32, 32, 1> __VA_ARGS__; break;                                               \
        case 202: KERNEL<32, 32, 2> __VA_ARGS__; break;                                               \
        case 203: KERNEL<32, 32, 3> __VA_ARGS__; break;                                               \
        case 204: KERNEL<32, 32, 4> __VA_ARGS__; break;                                               \
        case 211: KERNEL<32, 64, 1> __VA_ARGS__; break;                                               \
        case 212: KERNEL<32, 64, 2> __VA_ARGS__; break;                                               \
        case 213: KERNEL<32, 64, 3> __VA_ARGS__; break;                                               \
        case 214: KERNEL<32, 64, 4> __VA_ARGS__; break;                                               \
        case 401: KERNEL<64, 32, 1> __VA_ARGS__; break;                                               \
        case 402: KERNEL<64, 32, 2> __VA_ARGS__; break;                                               \
        case 403: KERNEL<64, 32, 3> __VA_ARGS__; break;                                               \
        case 404: KERNEL<64, 32, 4> __VA_ARGS__; break;                                               \
        case 411: KERNEL<64, 64, 1> __VA_ARGS__; break;                                               \
        case 412: KERNEL<64, 64, 2> __VA_ARGS__; break;                                               \
        case 413: KERNEL<64, 64, 3> __VA_ARGS__; break;                                               \
        case 414: KERNEL<64, 64, 4> __VA_ARGS__; break;                                               \
        case 601: KERNEL<96, 32, 1> __VA_ARGS__; break;                                               \
        case 602: KERNEL<96, 32, 2> __VA_ARGS__; break;                                               \
        case 603: KERNEL<96, 32, 3> __VA_ARGS__; break;                                               \
        case 604: KERNEL<96, 32, 4> __VA_ARGS__; break;                                               \
        case 611: KERNEL<96, 64, 1> __VA_ARGS__; break;                                               \
        case 612: KERNEL<96, 64, 2> __VA_ARGS__; break;                                               \
        case 613: KERNEL<96, 64, 3> __VA_ARGS__; break;                                               \
        case 614: KERNEL<96, 64, 4> __VA_ARGS__; break;                                               \
        default: return hipErrorInvalidValue;                                                     \
        }                                                                                         \
    } while (0)

template <int IN_P, int HID_P, int NH>
struct MlpFwd {
    static hipError_t run(npm_ctx *ctx, int blocks, int64_t n, const float *G, float *acts,
                          float *raw, hipStream_t s, const float *img, const float *wsel)
    {
        const MlpDesc &m = ctx->net.mlp;
        const int elems = (int)m.fwd_elems;
        const hipError_t e = hipFuncSetAttribute((const void *)k_mlp_fwd<IN_P, HID_P, NH>,
                                                 hipFuncAttributeMaxDynamicSharedMemorySize,
                                                 elems * sizeof(float));
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL((k_mlp_fwd<IN_P, HID_P, NH>), dim3(blocks), dim3(256),
                           elems * sizeof(float), s, n, m.n_in, m.width, img, elems, G,
                           acts, raw, wsel);
        return hipGetLastError();
    }
};

template <int IN_P, int HID_P, int NH>
struct MlpBwd {
    static hipError_t run(npm_ctx *ctx, int blocks, int64_t n, const float *draw,
                          const float *acts, float *delta, float *dG, hipStream_t s,
                          const float *wsel)
    {
        const MlpDesc &m = ctx->net.mlp;
        const int elems = (int)m.bwd_elems;
        const hipError_t e = hipFuncSetAttribute((const void *)k_mlp_bwd<IN_P, HID_P, NH>,
                                                 hipFuncAttributeMaxDynamicSharedMemorySize,
                                                 elems * sizeof(float));
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL((k_mlp_bwd<IN_P, HID_P, NH>), dim3(blocks), dim3(256),
                           elems * sizeof(float), s, n, m.n_in, m.width,
                           ctx->mlp_img + m.fwd_elems, elems, draw, acts, delta, dG, wsel);
        return hipGetLastError();
    }
};

static int tile_blocks(int64_t n)
{
    const int64_t tiles = (n + 31) / 32;
    const int64_t b = (tiles + 3) / 4;
    return (int)std::max<int64_t>(1, std::min<int64_t>(b, 1024));
}

hipError_t staged_mlp_fwd(npm_ctx *ctx, int64_t n, const float *G, float *acts, float *raw,
                          hipStream_t s, const Weights *w)
{
    const int blocks = tile_blocks(n);
    const float *img = w ? w->img : ctx->mlp_img;
    const float *wsel = selection_row(ctx, w ? w->grid32 : ctx->params);
    int tok;
    timed_begin(ctx, acts ? "staged_mlp_fwd_train" : "staged_mlp_fwd", s, &tok);
    hipError_t e = hipSuccess;
    NPM_MLP_DISPATCH(e = MlpFwd, ::run(ctx, blocks, n, G, acts, raw, s, img, wsel));
    timed_end(ctx, tok, s);
    return e;
}

hipError_t staged_mlp_bwd(npm_ctx *ctx, int64_t n, const float *draw, const float *acts,
                          float *delta, float *dG, hipStream_t s)
{
    const int blocks = tile_blocks(n);
    int tok;
    timed_begin(ctx, "staged_mlp_bwd", s, &tok);
    const float *wsel = selection_row(ctx, ctx->params);
    hipError_t e = hipSuccess;
    NPM_MLP_DISPATCH(e = MlpBwd, ::run(ctx, blocks, n, draw, acts, delta, dG, s, wsel));
    timed_end(ctx, tok, s);
    return e;
}

static constexpr int kDwBlocks = 256;

hipError_t staged_mlp_dw(npm_ctx *ctx, int64_t n, const float *G, const float *acts,
                         const float *delta, const float *draw, float *grad, hipStream_t s)
{
    const MlpDesc &m = ctx->net.mlp;
    const npm_layout &L = ctx->net.lay;
    const int blocks = (int)std::max<int64_t>(1, std::min<int64_t>(kDwBlocks, ((n + 31) / 32 + 3) / 4));
    int tok;
    timed_begin(ctx, "staged_mlp_dw", s, &tok);
    for (int i = 0; i < L.n_layers; ++i) {
        const int out_r = L.layer_out[i], in_r = L.layer_in[i];
        const float *dz = (i == L.n_layers - 1) ? draw : delta + (int64_t)i * m.width * n;
        const float *x = (i == 0) ? G : acts + (int64_t)(i - 1) * m.width * n;
        const int out_p = (i == L.n_layers - 1) ? (out_r > 32 ? 64 : 32) : m.hid_p;
        const int in_p = (i == 0) ? std::max(m.in_p, 32) : m.hid_p;   // at least one 32 block
        float *part = ctx->s_dw_part;
#define NPM_DW(OP, IP) hipLaunchKernelGGL((k_dw<OP, IP>), dim3(blocks), dim3(256), 0, s, n, out_r, in_r, dz, x, part)
        if (out_p == 32 && in_p == 32) NPM_DW(32, 32);
        else if (out_p == 32 && in_p == 64) NPM_DW(32, 64);
        else if (out_p == 32 && in_p == 96) NPM_DW(32, 96);
        else if (out_p == 64 && in_p == 32) NPM_DW(64, 32);
        else if (out_p == 64 && in_p == 96) NPM_DW(64, 96);
        else NPM_DW(64, 64);
#undef NPM_DW
        const int count = out_r * in_r;
        hipLaunchKernelGGL(k_dw_reduce, dim3((count + 255) / 256), dim3(256), 0, s, part, blocks,
                           count, grad + L.layer_offset[i]);
    }
    timed_end(ctx, tok, s);
    return hipGetLastError();
}

hipError_t staged_head(npm_ctx *ctx, int64_t n, const float *raw, const float *dir,
                       uint64_t seed, uint32_t stream_id, float *lobes, float *pdf, float *sdir,
                       float *spdf, hipStream_t s, float *sel)
{
    int tok;
    timed_begin(ctx, "staged_head", s, &tok);
    hipLaunchKernelGGL(k_head, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, raw, dir,
                       seed, stream_id, lobes, pdf, sdir, spdf, sel);
    timed_end(ctx, tok, s);
    return hipGetLastError();
}

hipError_t staged_loss_grad(npm_ctx *ctx, int64_t n, const float *raw, const float *dir,
                            const float *rad, const float *spdf, float *draw, double *loss_out,
                            hipStream_t s, const float *bsdf)
{
    constexpr int kMaxBlocks = kPartials / 2;   // the second half holds the selection sums
    const int blocks = (int)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, kMaxBlocks));
    const int sel = ctx->net.cfg.learn_selection;
    double *psel = (sel && bsdf) ? ctx->partials + kMaxBlocks : nullptr;
    int tok;
    timed_begin(ctx, "staged_loss_grad", s, &tok);
    hipLaunchKernelGGL(k_loss_grad, dim3(blocks), dim3(256), 0, s, n, raw, dir, rad, spdf,
                       1.0f / (float)n, draw, ctx->partials, sel, sel ? bsdf : nullptr, psel);
    timed_end(ctx, tok, s);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || !loss_out) return e;
    e = launch_reduce_scaled(ctx->partials, blocks, 1.0 / (double)n, loss_out, s);
    if (e != hipSuccess || !psel) return e;
    return launch_reduce_scaled(psel, blocks, 1.0 / (double)n, loss_out + 1, s);
}

hipError_t staged_scatter(npm_ctx *ctx, int64_t n, const float *pos, const float *dG,
                          float *grad, hipStream_t s)
{
    const GridDesc &g = ctx->net.grid;
    dim3 grid((unsigned)((n * 8 * g.feat + 255) / 256), (unsigned)g.n_levels);
    int tok;
    timed_begin(ctx, "staged_scatter", s, &tok);
    switch (g.feat) {
    case 1: hipLaunchKernelGGL(k_scatter<1>, grid, dim3(256), 0, s, g, n, pos, dG, grad); break;
    case 2: hipLaunchKernelGGL(k_scatter<2>, grid, dim3(256), 0, s, g, n, pos, dG, grad); break;
    case 4: hipLaunchKernelGGL(k_scatter<4>, grid, dim3(256), 0, s, g, n, pos, dG, grad); break;
    default: return hipErrorInvalidValue;
    }
    timed_end(ctx, tok, s);
    return hipGetLastError();
}

}  // namespace npm
