// Per-tile device functions of the fused NPM hot path, shared by the
// single-session fused kernels (k_fused.hip) and the persistent multi-session
// kernels of the serving form (k_serve.hip).
//
// A wave owns a tile of 32 vertices.  Lane l holds vertex l % 32; of a
// feature vector the half-wave h = l / 32 holds the features nf(h, a)
// (device_math.h).  After the output layer half h holds lobes k = 2r + h
// (r = 0..3), components in registers 4r..4r+3, so softmax, log-sum-exp and
// the lobe CDF need one exchange with lane l ^ 32.
//
// Precision form (BF = true): grid features read from an FP16 copy, MLP
// weights and activations in BF16 on v_mfma_f32_32x32x16_bf16 with FP32
// accumulation; mappings, softmax, log-density and sampling in FP32.
#pragma once

#include <type_traits>

#include "device_math.h"

namespace npm {

// One session's grid as a tile sees it: level offsets and resolutions staged
// in LDS, the level flags, and the FP32 or FP16 feature table.
struct GridView {
    const uint32_t *off;
    const int *res;
    uint32_t hashed_mask, table_mask;
    int n_levels;
    const float *g32;
    const __half *g16;
};

// ------------------------------------------------------------------ encode
// Features of the tile vertex for this half-wave: register 4 g + j F + f holds
// feature f of level (8 g + 4 h) / F + j; the registers past the grid
// features are zero.  The half-wave's levels are taken in batches of LBF / F
// (8 LBF floats of corner values): every corner load of a batch is issued
// before any is used, so the gathers of several levels are in flight
// together.  A batch starting at or beyond n_levels is skipped (the branch
// also keeps the compiler from hoisting later batches' loads, which would
// exhaust the registers); a level beyond n_levels inside a batch reads level
// 0 with zero weight.
template <int IN_P, int F, bool BF, int LBF = 8, int IN_G = IN_P>
__device__ __forceinline__ void encode_tile(const GridView &gv, int h, float px, float py,
                                            float pz, float *x)
{
    // IN_G: the grid features' share of the IN_P inputs (NPM-product inputs
    // follow them), rounded up to the 8 features of a register group
    constexpr int GROUPS = (IN_G + 7) / 8;
    constexpr int PER = 4 / F;                // levels per group and half
    constexpr int NLV = GROUPS * PER;         // levels of this half-wave
    constexpr int LB0 = LBF / F < 1 ? 1 : LBF / F;
    constexpr int LB = LB0 < NLV ? LB0 : NLV; // levels per batch
    auto level = [&](int q) { return (8 * (q / PER) + 4 * h) / F + q % PER; };
#pragma unroll
    for (int q0 = 0; q0 < NLV; q0 += LB) {
        if (level(q0) >= gv.n_levels) {
#pragma unroll
            for (int qq = 0; qq < LB && q0 + qq < NLV; ++qq)
#pragma unroll
                for (int f = 0; f < F; ++f) x[4 * ((q0 + qq) / PER) + ((q0 + qq) % PER) * F + f] = 0.0f;
            continue;
        }
        float val[LB][8][F];
        float fr[LB][3];
        bool live[LB];
#pragma unroll
        for (int qq = 0; qq < LB; ++qq) {
            const int q = q0 + qq;
            if (q >= NLV) break;
            const int l = level(q);
            live[qq] = l < gv.n_levels;
            const int lc = live[qq] ? l : 0;
            const int D = gv.res[lc];
            int cx, cy, cz;
            lattice_cell(px, D, cx, fr[qq][0]);
            lattice_cell(py, D, cy, fr[qq][1]);
            lattice_cell(pz, D, cz, fr[qq][2]);
            const uint32_t d1 = (uint32_t)D + 1u;
            const bool hashed = (gv.hashed_mask >> lc) & 1u;
            const uint32_t off = gv.off[lc];
#pragma unroll
            for (int b = 0; b < 8; ++b) {
                const uint32_t X = cx + (b & 1), Y = cy + ((b >> 1) & 1), Z = cz + ((b >> 2) & 1);
                const uint32_t e = off + (hashed ? ((X ^ (Y * 2654435761u) ^ (Z * 805459861u)) & gv.table_mask)
                                                 : X + d1 * (Y + d1 * Z));
                if constexpr (BF) {
                    if constexpr (F == 2) {
                        const __half2 t = *reinterpret_cast<const __half2 *>(gv.g16 + 2 * (size_t)e);
                        val[qq][b][0] = __low2float(t); val[qq][b][1] = __high2float(t);
                    } else {
#pragma unroll
                        for (int f = 0; f < F; ++f) val[qq][b][f] = __half2float(gv.g16[(size_t)e * F + f]);
                    }
                } else {
                    if constexpr (F == 1) {
                        val[qq][b][0] = gv.g32[e];
                    } else if constexpr (F == 2) {
                        const float2 t = *reinterpret_cast<const float2 *>(gv.g32 + 2 * (size_t)e);
                        val[qq][b][0] = t.x; val[qq][b][1] = t.y;
                    } else {
                        const float4 t = *reinterpret_cast<const float4 *>(gv.g32 + 4 * (size_t)e);
                        val[qq][b][0] = t.x; val[qq][b][1] = t.y; val[qq][b][2] = t.z; val[qq][b][3] = t.w;
                    }
                }
            }
        }
#pragma unroll
        for (int qq = 0; qq < LB; ++qq) {
            const int q = q0 + qq;
            if (q >= NLV) break;
            const float fx = fr[qq][0], fy = fr[qq][1], fz = fr[qq][2];
            const float wx[2] = {1.0f - fx, fx}, wy[2] = {1.0f - fy, fy}, wz[2] = {1.0f - fz, fz};
            float acc[F];
#pragma unroll
            for (int f = 0; f < F; ++f) acc[f] = 0.0f;
#pragma unroll
            for (int b = 0; b < 8; ++b) {
                const float w = wx[b & 1] * wy[(b >> 1) & 1] * wz[(b >> 2) & 1];
#pragma unroll
                for (int f = 0; f < F; ++f) acc[f] += w * val[qq][b][f];
            }
#pragma unroll
            for (int f = 0; f < F; ++f) x[4 * (q / PER) + (q % PER) * F + f] = live[qq] ? acc[f] : 0.0f;
        }
    }
#pragma unroll
    for (int a = 4 * GROUPS; a < IN_P / 2; ++a) x[a] = 0.0f;
}

// The grid encoding of a tile split in two, for software pipelining: the
// corner loads of every level of this half-wave are issued for one tile
// (encode_issue) and consumed one round later (encode_finish), so that they
// are in flight while the previous tile's MLP runs.  The loaded words are
// kept as loaded (FP16 pairs in the precision form) and converted when
// consumed, so that nothing waits on them early.
template <int F, bool BF> struct CornerRaw;
template <> struct CornerRaw<1, false> { using T = float; };
template <> struct CornerRaw<2, false> { using T = float2; };
template <> struct CornerRaw<4, false> { using T = float4; };
template <> struct CornerRaw<1, true> { using T = __half; };
template <> struct CornerRaw<2, true> { using T = __half2; };
template <> struct CornerRaw<4, true> { using T = uint2; };

template <int IN_G, int F, bool BF>
struct TileGather {
    static constexpr int GROUPS = (IN_G + 7) / 8;
    static constexpr int PER = 4 / F;
    static constexpr int NLV = GROUPS * PER;
    typename CornerRaw<F, BF>::T raw[NLV][8];
    float fr[NLV][3];
};

template <int IN_G, int F, bool BF>
__device__ __forceinline__ void encode_issue(const GridView &gv, int h, float px, float py,
                                             float pz, TileGather<IN_G, F, BF> &g)
{
    using TG = TileGather<IN_G, F, BF>;
    using RT = typename CornerRaw<F, BF>::T;
#pragma unroll
    for (int q = 0; q < TG::NLV; ++q) {
        const int l = (8 * (q / TG::PER) + 4 * h) / F + q % TG::PER;
        const int lc = l < gv.n_levels ? l : 0;      // a missing level reads level 0 (weight 0)
        const int D = gv.res[lc];
        int cx, cy, cz;
        lattice_cell(px, D, cx, g.fr[q][0]);
        lattice_cell(py, D, cy, g.fr[q][1]);
        lattice_cell(pz, D, cz, g.fr[q][2]);
        const uint32_t d1 = (uint32_t)D + 1u;
        const bool hashed = (gv.hashed_mask >> lc) & 1u;
        const uint32_t off = gv.off[lc];
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const uint32_t X = cx + (b & 1), Y = cy + ((b >> 1) & 1), Z = cz + ((b >> 2) & 1);
            const uint32_t e = off + (hashed ? ((X ^ (Y * 2654435761u) ^ (Z * 805459861u)) & gv.table_mask)
                                             : X + d1 * (Y + d1 * Z));
            if constexpr (BF) g.raw[q][b] = *reinterpret_cast<const RT *>(gv.g16 + (size_t)e * F);
            else g.raw[q][b] = *reinterpret_cast<const RT *>(gv.g32 + (size_t)e * F);
        }
    }
}

template <int IN_P, int IN_G, int F, bool BF>
__device__ __forceinline__ void encode_finish(const GridView &gv, int h,
                                              const TileGather<IN_G, F, BF> &g, float *x)
{
    using TG = TileGather<IN_G, F, BF>;
#pragma unroll
    for (int q = 0; q < TG::NLV; ++q) {
        const int l = (8 * (q / TG::PER) + 4 * h) / F + q % TG::PER;
        const float fx = g.fr[q][0], fy = g.fr[q][1], fz = g.fr[q][2];
        const float wx[2] = {1.0f - fx, fx}, wy[2] = {1.0f - fy, fy}, wz[2] = {1.0f - fz, fz};
        float acc[F];
#pragma unroll
        for (int f = 0; f < F; ++f) acc[f] = 0.0f;
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const float w = wx[b & 1] * wy[(b >> 1) & 1] * wz[(b >> 2) & 1];
            float v[F];
            const auto &r = g.raw[q][b];
            if constexpr (BF) {
                if constexpr (F == 1) {
                    v[0] = __half2float(r);
                } else if constexpr (F == 2) {
                    v[0] = __low2float(r); v[1] = __high2float(r);
                } else {
                    const __half2 lo = *reinterpret_cast<const __half2 *>(&r.x);
                    const __half2 hi = *reinterpret_cast<const __half2 *>(&r.y);
                    v[0] = __low2float(lo); v[1] = __high2float(lo);
                    v[2] = __low2float(hi); v[3] = __high2float(hi);
                }
            } else {
                if constexpr (F == 1) {
                    v[0] = r;
                } else if constexpr (F == 2) {
                    v[0] = r.x; v[1] = r.y;
                } else {
                    v[0] = r.x; v[1] = r.y; v[2] = r.z; v[3] = r.w;
                }
            }
#pragma unroll
            for (int f = 0; f < F; ++f) acc[f] += w * v[f];
        }
        const bool live = l < gv.n_levels;
#pragma unroll
        for (int f = 0; f < F; ++f) x[4 * (q / TG::PER) + (q % TG::PER) * F + f] = live ? acc[f] : 0.0f;
    }
#pragma unroll
    for (int a = 4 * TG::GROUPS; a < IN_P / 2; ++a) x[a] = 0.0f;
}

// NPM-product inputs (Sec. 4.3) of the tile vertex into the feature
// registers: features GF .. GF + 2 SHD^2 hold the spherical harmonics of the
// outgoing direction, then of the normal, then the roughness (a7 = omega_o,
// normal, roughness).  Which register holds which input is fixed at compile
// time for each half-wave, so the fill is one select per register.
template <int NB>
__device__ __forceinline__ float aux_value(int k, const float *yo, const float *yn, float r)
{
    return k < NB ? yo[k] : (k < 2 * NB ? yn[k - NB] : r);
}

template <int IN_P, int GF, int SHD>
__device__ __forceinline__ void aux_fill(int h, const float *a7, float *x)
{
    constexpr int NB = SHD * SHD, NA = 2 * NB + 1;
    float yo[16], yn[16];
    sh_bands4(a7[0], a7[1], a7[2], yo);
    sh_bands4(a7[3], a7[4], a7[5], yn);
#pragma unroll
    for (int a = 0; a < IN_P / 2; ++a) {
        const int k0 = 8 * (a / 4) + (a & 3) - GF, k1 = k0 + 4;   // inputs of half 0 / half 1
        if (k0 >= 0 && k0 < NA && h == 0) x[a] = aux_value<NB>(k0, yo, yn, a7[6]);
        if (k1 >= 0 && k1 < NA && h == 1) x[a] = aux_value<NB>(k1, yo, yn, a7[6]);
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

// Forward of all layers; hidden activations into acts[NH][HID_P/2] when KEEP;
// with SEL also the selection logit *cp (the last hidden layer dotted with the
// selection row wsel in LDS).
template <int IN_P, int HID_P, int NH, bool BF, bool KEEP, bool SEL = false>
__device__ __forceinline__ void mlp_forward(const void *img, const float *x, float (*acts)[HID_P / 2],
                                            float *o, int lane, const float *wsel = nullptr,
                                            float *cp = nullptr)
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
    if constexpr (SEL) *cp = select_logit<HID_P>(wsel, a, lane >> 5);
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
struct QueryIO {
    int64_t n;
    const float *pos, *dir;
    float *lobes, *pdf, *sdir, *spdf;   // requested outputs (null: skipped)
    uint64_t seed;
    uint32_t sid;
    const uint32_t *perm = nullptr;     // visiting order, or null: 0..n-1
    float *stage = nullptr;             // with perm: kStageFloats per slot, AoS
    const float *rec = nullptr;         // with perm: the inputs in visiting order
    const float *aux = nullptr;         // NPM-product inputs [7][n]
    int rec_stride = 8;                 // floats per record (16 with NPM-product)
    float *sel = nullptr;               // selection probability [n] (selection networks)
    const float *wsel = nullptr;        // the selection row in LDS (HID_P floats)
};

// A vertex's inputs in visiting order (written by the spatial sort, 32 bytes
// per slot so that a wave reads its tile coalesced): position, direction,
// radiance, sampling pdf (zeros where the call has none); with NPM-product 64
// bytes, followed by omega_o, the normal and the roughness.
constexpr int kRecFloats = 8;

// The NPM-product inputs of slot v (vertex vv) from the record or the SoA array.
__device__ __forceinline__ void load_aux(const float *rec, int rec_stride, const float *aux,
                                         int64_t n, int64_t v, int64_t vv, float *a7)
{
    if (rec) {
        const f32x4 *r = reinterpret_cast<const f32x4 *>(rec + (size_t)v * rec_stride + 8);
        const f32x4 p = r[0], q = r[1];
        a7[0] = p[0]; a7[1] = p[1]; a7[2] = p[2]; a7[3] = p[3];
        a7[4] = q[0]; a7[5] = q[1]; a7[6] = q[2];
    } else {
#pragma unroll
        for (int j = 0; j < 7; ++j) a7[j] = aux[j * n + vv];
    }
}

// Compile-time shape of the NPM-product inputs (PG: 0 none; 1: 32 grid
// features and 4 SH bands; 2: 4 grid features and 2 bands).
template <int PG> struct ProductShape { static constexpr int GF = 0, SHD = 0; };
template <> struct ProductShape<1> { static constexpr int GF = 32, SHD = 4; };
template <> struct ProductShape<2> { static constexpr int GF = 4, SHD = 2; };

// Staged query outputs of one visiting slot (AoS, 160 bytes), laid out so
// that each half-wave writes whole 16-byte pieces: floats [20 h, 20 h + 16)
// hold the lobes k = 2 r + h of half h (component q of that lobe at
// 20 h + 4 r + q); then pdf at 16, the sample direction at 17..19 and the
// sample pdf at 36.
constexpr int kStageFloats = 40;
constexpr int kStagePdf = 16, kStageSdir = 17, kStageSpdf = 36, kStageSel = 37;

// One 32-vertex tile t of a query: encode, MLP, mappings, pdf at dir, one
// sample per vertex and its pdf.  img: the forward weight image in LDS.
template <int IN_P, int HID_P, int NH, int F, bool BF, int PG = 0, bool SEL = false>
__device__ __forceinline__ void query_tile(const GridView &gv, const void *img, const QueryIO &io,
                                           int64_t t, int lane)
{
    const int h = lane >> 5;
    const int64_t n = io.n;
    const int64_t v = t * 32 + (lane & 31);   // visiting slot
    const bool valid = v < n;
    // the vertex: its inputs, its uniforms and (unstaged) its outputs
    const int64_t vv = io.perm ? (int64_t)io.perm[valid ? v : n - 1] : (valid ? v : n - 1);
    float *st = io.stage ? io.stage + (size_t)(valid ? v : n - 1) * kStageFloats : nullptr;
    float px, py, pz, wx = 0.0f, wy = 0.0f, wz = 0.0f;
    if (io.rec) {
        const f32x4 *r = reinterpret_cast<const f32x4 *>(io.rec + (size_t)(valid ? v : n - 1) * io.rec_stride);
        const f32x4 a = r[0], b = r[1];
        px = a[0]; py = a[1]; pz = a[2]; wx = a[3]; wy = b[0]; wz = b[1];
    } else {
        px = io.pos[vv]; py = io.pos[n + vv]; pz = io.pos[2 * n + vv];
        if (io.pdf) { wx = io.dir[vv]; wy = io.dir[n + vv]; wz = io.dir[2 * n + vv]; }
    }
    float x[IN_P / 2];
    // two levels' corners in flight at F = 2: the query kernel runs three
    // waves per SIMD, which hide the rest
    encode_tile<IN_P, F, BF, 4, (PG > 0 ? ProductShape<PG>::GF : IN_P)>(gv, h, px, py, pz, x);
    if constexpr (PG > 0) {
        float a7[7];
        load_aux(io.rec, io.rec_stride, io.aux, n, valid ? v : n - 1, vv, a7);
        aux_fill<IN_P, ProductShape<PG>::GF, ProductShape<PG>::SHD>(h, a7, x);
    }
    float o[16], cp = 0.0f;
    mlp_forward<IN_P, HID_P, NH, BF, false, SEL>(img, x, nullptr, o, lane, io.wsel, &cp);
    if constexpr (SEL) {
        if (io.sel && valid && h == 0) {
            const float c = sigmoidf(cp);
            if (st) st[kStageSel] = c;
            else io.sel[vv] = c;
        }
    }
    Lobe L[4];
    map_half(o, L);
    if (io.lobes && valid) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int k = 2 * r + h;
            const f32x4 c = {L[r].theta, L[r].phi, L[r].kappa, expf(L[r].loglam)};
            if (st) {
                *reinterpret_cast<f32x4 *>(st + 20 * h + 4 * r) = c;
            } else {
#pragma unroll
                for (int q = 0; q < 4; ++q) io.lobes[(int64_t)(q * kLobes + k) * n + vv] = c[q];
            }
        }
    }
    float pdf_v = 0.0f;
    if (io.pdf) {
        float lt[4];
        const float lv = logpdf_half(L, wx, wy, wz, lt);
        pdf_v = expf(lv);
        if (valid && h == 0 && !st) io.pdf[vv] = pdf_v;
    }
    if (io.sdir || io.spdf) {
        float u[3];
        philox_uniforms((uint64_t)vv, io.seed, io.sid, 0u, u);
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
            if (st) {
                *reinterpret_cast<f32x4 *>(st + kStagePdf) = f32x4{pdf_v, w[0], w[1], w[2]};
                st[kStageSpdf] = expf(lv);
            } else {
                if (io.sdir) { io.sdir[vv] = w[0]; io.sdir[n + vv] = w[1]; io.sdir[2 * n + vv] = w[2]; }
                if (io.spdf) io.spdf[vv] = expf(lv);
            }
        }
    } else if (st && valid && h == 0 && io.pdf) {
        st[kStagePdf] = pdf_v;
    }
}

// Stages a session's grid level table into LDS.
__device__ __forceinline__ void stage_levels(const GridDesc &g, uint32_t *s_off, int *s_res)
{
    if (threadIdx.x < NPM_MAX_LEVELS) {
        s_off[threadIdx.x] = g.offset[threadIdx.x];
        s_res[threadIdx.x] = g.res[threadIdx.x];
    }
}

__device__ __forceinline__ GridView grid_view(const GridDesc &g, const uint32_t *s_off,
                                              const int *s_res, const float *g32,
                                              const __half *g16)
{
    GridView gv;
    gv.off = s_off;
    gv.res = s_res;
    gv.hashed_mask = g.hashed_mask;
    gv.table_mask = g.table_mask;
    gv.n_levels = g.n_levels;
    gv.g32 = g32;
    gv.g16 = g16;
    return gv;
}

// ------------------------------------------------------------------ backward
// A wave's LDS buffer for the in-kernel grid scatter: the tile's dG as rows =
// features (36-float stride), then the aggregation window.
constexpr int kStride = 36;   // LDS row stride (floats) of the buffer

// Writes a T32-layout vector of width 2*REGS into the wave's LDS buffer.
template <int REGS>
__device__ __forceinline__ void t32_to_lds(float *buf, const float *x, int lane)
{
    const int h = lane >> 5, j = lane & 31;
#pragma unroll
    for (int a = 0; a < REGS; ++a) buf[nf(h, a) * kStride + j] = x[a];
}

__device__ __forceinline__ void wave_lds_fence()
{
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

struct TrainIO {
    int64_t n;
    const float *pos, *dir, *rad, *spdf;
    float *grad;      // flat gradient (grid part scattered here), or null: loss only
    float invN;
    const uint32_t *perm;   // visiting order of the vertices, or null: 0..n-1
    const float *rec = nullptr;   // with perm: the inputs in visiting order
    const float *aux = nullptr;   // NPM-product inputs [7][n]
    int rec_stride = 8;           // floats per record (16 with NPM-product)
    const float *bsdf = nullptr;  // BSDF densities [n] (the selection term), or null
};

// The vertex at position v of the visiting order.
__device__ __forceinline__ int64_t visit(const uint32_t *perm, int64_t v)
{
    return perm ? (int64_t)perm[v] : v;
}

// Scatter of a tile's dG into the grid gradient (the transpose of the
// interpolation).  FP32 atomics are limited by the number of distinct 64-byte
// lines per wave instruction, so lanes are assigned to the 8F contributions
// of one (vertex, level) -- corner b = sub / F, feature f = sub % F -- where
// the x-adjacent corners and the F features of an entry are contiguous, and
// the 64 / (8F) vertex-levels of an instruction are consecutive vertices of
// one level.  dGt: the tile's dG in LDS, rows = features, stride kStride.
//
// Window: at a level where the lattice points around the tile's bounding box
// (lo, hi: clamped positions) number at most WIN_PTS, the contributions are
// first summed in a dense LDS window over that box (LDS atomics), and each
// touched lattice point then costs one global atomic per feature, issued in
// window order so that x-neighbours share lines.  In a spatially ordered
// batch this covers the coarse levels, where the 32 vertices of a tile share
// most corners.  The cell lookup is monotone in the position, so every corner
// lies in the window; a corner that did not would take the direct path.
//
// Window sums (WT): FP64, or (WT = int) 32-bit fixed point, which keeps the
// precision form free of FP64 and of FP32 LDS atomics (slow on this chip).
// In fixed point each level gets a power-of-two scale from the largest |dG|
// of its rows in the tile: with max |dG| < 2^e every contribution w dG
// (w <= 1) is below 2^e, at most 32 of them land on one lattice point (one
// per vertex of the tile), so at the scale 2^(25 - e) every sum stays below
// 2^30; each contribution is rounded to a multiple of 2^(e - 25) and the sum
// is exact, independent of the order of the adds.
template <typename WT> struct WinScale {
    __device__ __forceinline__ WT enc(float v) const { return WT(v); }
    __device__ __forceinline__ float dec(WT s) const { return (float)s; }
};
template <> struct WinScale<int> {
    int k = 0;                               // the scale is 2^k (ldexp: no overflow of 2^k itself)
    // the scale of level l from its F rows of the tile's dG (all lanes call
    // it); false when they are all zero
    template <int F>
    __device__ __forceinline__ bool set_level(const float *dGt, int l, int lane)
    {
        float m = 0.0f;
        for (int i = lane; i < F * 32; i += 64) m = fmaxf(m, fabsf(dGt[(l * F + i / 32) * kStride + (i & 31)]));
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) m = fmaxf(m, __shfl_xor(m, o, 64));
        if (!(m > 0.0f)) return false;
        int e;
        frexpf(m, &e);                       // m < 2^e
        k = 25 - e;
        return true;
    }
    __device__ __forceinline__ int enc(float v) const { return (int)rintf(ldexpf(v, k)); }
    __device__ __forceinline__ float dec(int s) const { return ldexpf((float)s, -k); }
};

// fn(integral_constant<int, 0>) ... fn(integral_constant<int, N - 1>), in order
template <int N, typename Fn>
__device__ __forceinline__ void static_for(Fn &&fn)
{
    if constexpr (N > 0) {
        static_for<N - 1>(fn);
        fn(std::integral_constant<int, N - 1>{});
    }
}

// Lane J of each 16-lane row, to every lane of the row (DPP row_newbcast:J);
// a lane the broadcast does not write keeps its own value.
template <int J>
__device__ __forceinline__ int row_bcast(int v)
{
    return __builtin_amdgcn_update_dpp(v, v, 0x150 + J, 0xf, 0xf, false);
}
template <int J>
__device__ __forceinline__ float row_bcast(float v)
{
    return __int_as_float(row_bcast<J>(__float_as_int(v)));
}

template <int F, int WIN_PTS, typename WT = float>
__device__ __forceinline__ void scatter_tile(const GridView &gv, const float *dGt,
                                             const float *__restrict__ pos, const uint32_t *perm,
                                             int64_t n, int64_t t, int lane,
                                             float *__restrict__ grad, const float *lo,
                                             const float *hi, WT *win,
                                             const float *rec = nullptr, int rec_stride = 8,
                                             uint32_t skip_mask = 0u)
{
    constexpr int LPV = 8 * F;              // lanes per vertex-level
    constexpr int VPI = 64 / LPV;           // vertex-levels per instruction
    constexpr int NJ = 32 / VPI;            // vertex-levels per lane and level
    // F >= 2: the LPV lanes of a vertex-level fill whole 16-lane rows, so lane
    // i of a row holds vertex (i mod NJ) VPI + q, forms its lattice cell once
    // per level, and the row reads it by a DPP row broadcast when that
    // vertex's turn comes (F = 1: every lane forms the cells it uses)
    constexpr bool BC = F >= 2;
    const int q = lane / LPV, sub = lane % LPV, b = sub / F, f = sub % F;
    const int bx = b & 1, by = (b >> 1) & 1, bz = (b >> 2) & 1;
    float px[BC ? 1 : NJ], py[BC ? 1 : NJ], pz[BC ? 1 : NJ];
#pragma unroll
    for (int jj = 0; jj < (BC ? 1 : NJ); ++jj) {
        const int64_t v = t * 32 + (BC ? ((lane & 15) % NJ) : jj) * VPI + q;
        if (rec) {
            const f32x4 a = *reinterpret_cast<const f32x4 *>(rec + (size_t)(v < n ? v : n - 1) * rec_stride);
            px[jj] = a[0]; py[jj] = a[1]; pz[jj] = a[2];
        } else {
            const int64_t vv = visit(perm, v < n ? v : n - 1);
            px[jj] = pos[vv]; py[jj] = pos[n + vv]; pz[jj] = pos[2 * n + vv];
        }
    }
    for (int l = 0; l < gv.n_levels; ++l) {
        if ((skip_mask >> l) & 1u) continue;      // scattered by the binned pass
        const int D = gv.res[l];
        const uint32_t d1 = (uint32_t)D + 1u;
        const bool hashed = (gv.hashed_mask >> l) & 1u;
        const uint32_t off = gv.off[l];
        auto entry = [&](uint32_t X, uint32_t Y, uint32_t Z) {
            return off + (hashed ? ((X ^ (Y * 2654435761u) ^ (Z * 805459861u)) & gv.table_mask)
                                 : X + d1 * (Y + d1 * Z));
        };
        int x0 = 0, y0 = 0, z0 = 0, ex = 0, ey = 0, ez = 0;
        bool use_win = false;
        if constexpr (WIN_PTS > 0) {
            float fr;
            int c1;
            lattice_cell(lo[0], D, x0, fr); lattice_cell(hi[0], D, c1, fr); ex = c1 - x0 + 2;
            lattice_cell(lo[1], D, y0, fr); lattice_cell(hi[1], D, c1, fr); ey = c1 - y0 + 2;
            lattice_cell(lo[2], D, z0, fr); lattice_cell(hi[2], D, c1, fr); ez = c1 - z0 + 2;
            // each extent is bounded before the product is formed: at fine
            // levels an unordered tile spans ~2000 cells a side, whose cube
            // overflows 32-bit arithmetic
            use_win = ex <= WIN_PTS && ey <= WIN_PTS && ez <= WIN_PTS &&
                      ex * ey <= WIN_PTS && ex * ey * ez <= WIN_PTS;
        }
        WinScale<WT> sc;
        if constexpr (std::is_same<WT, int>::value) {
            // a level whose dG rows are all zero has nothing to scatter
            if (use_win && !sc.template set_level<F>(dGt, l, lane)) continue;
        }
        if (use_win) {
            const int nw = ex * ey * ez * F;
            for (int i = lane; i < nw; i += 64) win[i] = WT(0);
            wave_lds_fence();
        }
        // corner (bx, by, bz), feature f of vertex j of the tile
        auto corner = [&](int j, int cx, int cy, int cz, float fx, float fy, float fz) {
            if (t * 32 + j >= n) return;
            const float d = dGt[(l * F + f) * kStride + j];
            if (d == 0.0f) return;
            const uint32_t X = cx + bx, Y = cy + by, Z = cz + bz;
            const float w = (bx ? fx : 1.0f - fx) * (by ? fy : 1.0f - fy) * (bz ? fz : 1.0f - fz);
            const uint32_t wx = X - (uint32_t)x0, wy = Y - (uint32_t)y0, wz = Z - (uint32_t)z0;
            if (use_win && wx < (uint32_t)ex && wy < (uint32_t)ey && wz < (uint32_t)ez)
                __hip_atomic_fetch_add(win + ((wz * ey + wy) * ex + wx) * F + f, sc.enc(w * d),
                                       __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
            else
                unsafeAtomicAdd(grad + (size_t)entry(X, Y, Z) * F + f, w * d);
        };
        if constexpr (BC) {
            int cxv, cyv, czv;
            float fxv, fyv, fzv;
            lattice_cell(px[0], D, cxv, fxv);
            lattice_cell(py[0], D, cyv, fyv);
            lattice_cell(pz[0], D, czv, fzv);
            static_for<NJ>([&](auto J) {
                constexpr int jj = decltype(J)::value;
                corner(jj * VPI + q, row_bcast<jj>(cxv), row_bcast<jj>(cyv), row_bcast<jj>(czv),
                       row_bcast<jj>(fxv), row_bcast<jj>(fyv), row_bcast<jj>(fzv));
            });
        } else {
#pragma unroll
            for (int jj = 0; jj < NJ; ++jj) {
                int cx, cy, cz;
                float fx, fy, fz;
                lattice_cell(px[jj], D, cx, fx);
                lattice_cell(py[jj], D, cy, fy);
                lattice_cell(pz[jj], D, cz, fz);
                corner(jj * VPI + q, cx, cy, cz, fx, fy, fz);
            }
        }
        if (use_win) {
            wave_lds_fence();
            const int nw = ex * ey * ez * F;
            for (int i = lane; i < nw; i += 64) {
                const WT s = win[i];
                if (s != WT(0)) {
                    const int p = i / F, pf = i % F;
                    const int pyz = p / ex, wx = p - pyz * ex, wz = pyz / ey, wy = pyz - wz * ey;
                    unsafeAtomicAdd(grad + (size_t)entry(x0 + wx, y0 + wy, z0 + wz) * F + pf,
                                    sc.dec(s));
                }
            }
            wave_lds_fence();
        }
    }
}

// Bounding box of the tile's clamped positions (the lattice lookup clamps to
// the unit cube), over the 32 vertices of a T32 tile.
__device__ __forceinline__ void tile_bbox(float px, float py, float pz, float *lo, float *hi)
{
    const float c[3] = {fminf(fmaxf(px, 0.0f), 1.0f), fminf(fmaxf(py, 0.0f), 1.0f),
                        fminf(fmaxf(pz, 0.0f), 1.0f)};
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        float mn = c[a], mx = c[a];
#pragma unroll
        for (int m = 1; m < 32; m <<= 1) {
            mn = fminf(mn, __shfl_xor(mn, m, 64));
            mx = fmaxf(mx, __shfl_xor(mx, m, 64));
        }
        lo[a] = mn;
        hi[a] = mx;
    }
}

// One tile of the backward: forward with activations in registers, the
// KL-gradient head, the delta chain, the weight gradients into dw, and the
// grid scatter.  lacc accumulates -w log V (FP64) of half 0's vertices.
// STORE_DG: the tile's dG is stored at dg_tiles + t * OUT0 * 32 (row r =
// feature r, 32 vertices of the visiting order) for the aggregated scatter
// kernel; otherwise it is scattered into the grid here.
// A training vertex's inputs: position, direction, radiance estimate and
// sampling pdf of visiting slot v (the vertex vv), from the slot's record or
// the SoA arrays.
struct TrainInputs {
    float px, py, pz, wx, wy, wz, rad, spdf;
};
__device__ __forceinline__ TrainInputs train_inputs(const TrainIO &io, int64_t v, int64_t vv)
{
    TrainInputs in;
    const int64_t n = io.n;
    if (io.rec) {
        const f32x4 *r = reinterpret_cast<const f32x4 *>(io.rec + (size_t)v * io.rec_stride);
        const f32x4 a = r[0], b = r[1];
        in.px = a[0]; in.py = a[1]; in.pz = a[2]; in.wx = a[3];
        in.wy = b[0]; in.wz = b[1]; in.rad = b[2]; in.spdf = b[3];
    } else {
        in.px = io.pos[vv]; in.py = io.pos[n + vv]; in.pz = io.pos[2 * n + vv];
        in.wx = io.dir[vv]; in.wy = io.dir[n + vv]; in.wz = io.dir[2 * n + vv];
        in.rad = io.rad[vv]; in.spdf = io.spdf[vv];
    }
    return in;
}

// The KL-gradient head (Sec. 4.2, eq. mcgradients) of a tile: d = d loss /
// d raw for this half-wave's four lobes, from the raw outputs o; lacc
// accumulates -w log V (FP64) of half 0's vertices.  Returns log V at the
// sample's direction.
__device__ __forceinline__ float kl_head(const float *o, const TrainInputs &in, bool valid,
                                         float invN, int h, float *d, double &lacc)
{
    const float wgt = valid ? sample_weight(in.rad, in.spdf) : 0.0f;
#pragma unroll
    for (int i = 0; i < 16; ++i) d[i] = 0.0f;
    Lobe L[4];
    map_half(o, L);
    float lt[4];
    const float lv = logpdf_half(L, in.wx, in.wy, in.wz, lt);
    if (wgt != 0.0f) {
        const float g = -wgt * invN;
#pragma unroll
        for (int r = 0; r < 4; ++r)
            lobe_grad(L[r], o[4 * r], o[4 * r + 1], o[4 * r + 2], expf(lt[r] - lv),
                      expf(L[r].loglam), g, in.wx, in.wy, in.wz, d + 4 * r);
        if (h == 0) lacc -= (double)wgt * (double)lv;
    }
    return lv;
}

// The MLP input of a tile vertex in the tile layout: the grid encoding, the
// padding rows of a narrow input zero, then the NPM-product inputs.
template <int IN_P, int F, bool BF, int PG>
__device__ __forceinline__ void tile_input(const GridView &gv, const TrainIO &io,
                                           const TrainInputs &in, int64_t v, int64_t vv, int h,
                                           float *x)
{
    constexpr int IN0 = IN_P < 32 ? 32 : IN_P;
    encode_tile<IN_P, F, BF, 8, (PG > 0 ? ProductShape<PG>::GF : IN_P)>(gv, h, in.px, in.py, in.pz,
                                                                       x);
#pragma unroll
    for (int i = IN_P / 2; i < IN0 / 2; ++i) x[i] = 0.0f;
    if constexpr (PG > 0) {
        float a7[7];
        load_aux(io.rec, io.rec_stride, io.aux, io.n, v, vv, a7);
        aux_fill<IN_P, ProductShape<PG>::GF, ProductShape<PG>::SHD>(h, a7, x);
    }
}

// ------------------------------------------------------------------ block-cooperative weight gradients
// The training kernel splits the weight gradients of a block among its WV
// waves.  In every round each wave runs encode, forward, KL-gradient head and
// delta chain for its own 32-vertex tile (the block takes WV tiles at a
// time); per layer, from the output layer back, the waves put
// the layer's deltas and inputs into a shared LDS exchange buffer, transposed
// (rows = features, one column per vertex of the round), and each wave
// accumulates its own share of that layer's 32x32 weight-gradient blocks
// over all 32 WV vertices of the round (the MFMA reduction dimension).  Each
// dW block belongs to one wave, which keeps ceil(blocks / WV) accumulators in
// registers instead of all of them and writes them straight to the block's
// partial at the end: no register spills, no per-wave partial sums.
//
// Layers are numbered 0 (the first, IN0 inputs) to NH (the output layer, 32
// outputs); the phases run from NH down to 0, and the dW blocks are numbered
// in that order, block g belonging to wave g % WV in its slot g / WV.
template <int IN_P, int HID_P, int NH, int WV, bool SPLIT = true>
struct BlockPlan {
    static constexpr int IN0 = IN_P < 32 ? 32 : IN_P;
    static constexpr int out_p(int L) { return L == NH ? 32 : HID_P; }
    static constexpr int in_p(int L) { return L == 0 ? IN0 : HID_P; }
    static constexpr int nbi(int L) { return in_p(L) / 32; }
    static constexpr int blocks(int L) { return (out_p(L) / 32) * nbi(L); }
    // A phase's work items: its blocks, each split into parts(L) ranges of
    // the round's vertices when whole blocks would leave waves idle at the
    // phase's barrier (2 blocks on 4 waves: 4 halves); item it = b parts + p
    static constexpr int parts(int L)
    {
        return !SPLIT || blocks(L) % WV == 0 ? 1 : (2 * blocks(L)) % WV == 0 ? 2 : 1;
    }
    static constexpr int items(int L) { return blocks(L) * parts(L); }
    // the first item of layer L in phase order
    static constexpr int first(int L)
    {
        int g = 0;
        for (int l = NH; l > L; --l) g += items(l);
        return g;
    }
    static constexpr int total() { return first(-1); }
    static constexpr int slots() { return (total() + WV - 1) / WV; }
    // blocks split into parts before layer L in phase order (their partial
    // sums meet in LDS at the end, 1,024 floats each)
    static constexpr int split_before(int L)
    {
        int c = 0;
        for (int l = NH; l > L; --l) c += parts(l) > 1 ? blocks(l) : 0;
        return c;
    }
    static constexpr int splits() { return split_before(-1); }
    // the split blocks' partial sums fit in the exchange buffer
    static constexpr bool scratch_fits(bool bf)
    {
        return splits() * 4096 <= max_rows() * xs(bf) * (bf ? 2 : 4);
    }
    // rows of the exchange buffer in phase L: the deltas, then the inputs
    static constexpr int rows(int L) { return out_p(L) + in_p(L); }
    // with the selection output, the output layer's phase also carries the
    // selection derivative, one row after its deltas and inputs
    static constexpr int sel_row() { return rows(NH); }
    static constexpr int max_rows()
    {
        int r = sel_row() + 1;
        for (int l = 0; l <= NH; ++l) r = rows(l) > r ? rows(l) : r;
        return r;
    }
    // row stride of the exchange buffer (elements): the round's 32 WV
    // vertices plus a pad that puts consecutive rows 4 banks apart, so that
    // the 16-byte reads of 16 lanes on 16 rows hit distinct banks
    static constexpr int xs(bool bf) { return 32 * WV + (bf ? 8 : 4); }
    // FP32 row-major image: layer L's rows are in_p(L) + 1 floats apart
    static constexpr int rm_stride(int L) { return in_p(L) + 1; }
    static constexpr int rm_off(int L)
    {
        int o = 0;
        for (int l = 0; l < L; ++l) o += out_p(l) * rm_stride(l);
        return o;
    }
    static constexpr int rm_elems() { return rm_off(NH + 1); }
};

// fn(std::integral_constant<int, I>) for I = HI, HI - 1, .., LO (nothing if
// HI < LO): a loop whose index is a compile-time constant in the body.
template <int HI, int LO, class Fn>
__device__ __forceinline__ void static_for_down(Fn &&fn)
{
    if constexpr (HI >= LO) {
        fn(std::integral_constant<int, HI>{});
        static_for_down<HI - 1, LO>(fn);
    }
}

// Rows [row0, row0 + 2 REGS) of the exchange buffer, at this wave's 32
// columns, from a tile-layout vector of 2 REGS features.
template <int REGS, int XS, typename XT>
__device__ __forceinline__ void xch_put(XT *xb, int row0, int wave, const float *v, int lane)
{
    const int h = lane >> 5, j = lane & 31;
    XT *p = xb + row0 * XS + 32 * wave + j;
#pragma unroll
    for (int a = 0; a < REGS; ++a) p[nf(h, a) * XS] = XT(v[a]);
}

// acc (a 32x32 dW block) += sum over KV of the round's vertices, from column
// c0 on, of delta[ro + row] input[ri + col], rows of the exchange buffer.
// FP32: 32x32x2 steps, the half-wave h supplying the vertices
// c0 + [KV/2 h, KV/2 (h+1)) in order, four per 16-byte read.  BF16: 32x32x16
// steps, half h supplying the vertices c0 + 16 s + 8 h + e.
template <int KV, int XS>
__device__ __forceinline__ void dw_block(const float *xb, int ro, int ri, int c0, f32x16 &acc,
                                         int lane)
{
    const int i = lane & 31, h = lane >> 5;
    const float *pa = xb + (ro + i) * XS + c0 + (KV / 2) * h;
    const float *pb = xb + (ri + i) * XS + c0 + (KV / 2) * h;
#pragma unroll
    for (int q = 0; q < KV / 8; ++q) {
        const f32x4 A = *reinterpret_cast<const f32x4 *>(pa + 4 * q);
        const f32x4 Bv = *reinterpret_cast<const f32x4 *>(pb + 4 * q);
#pragma unroll
        for (int e = 0; e < 4; ++e) acc = __builtin_amdgcn_mfma_f32_32x32x2f32(A[e], Bv[e], acc, 0, 0, 0);
    }
}
template <int KV, int XS>
__device__ __forceinline__ void dw_block(const __bf16 *xb, int ro, int ri, int c0, f32x16 &acc,
                                         int lane)
{
    const int i = lane & 31, h = lane >> 5;
    const __bf16 *pa = xb + (ro + i) * XS + c0 + 8 * h;
    const __bf16 *pb = xb + (ri + i) * XS + c0 + 8 * h;
#pragma unroll
    for (int s = 0; s < KV / 16; ++s) {
        const bf16x8 A = *reinterpret_cast<const bf16x8 *>(pa + 16 * s);
        const bf16x8 Bv = *reinterpret_cast<const bf16x8 *>(pb + 16 * s);
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(A, Bv, acc, 0, 0, 0);
    }
}

// Phase L of a round: put this wave's deltas dz and layer inputs hin into the
// exchange buffer; after the barrier accumulate this wave's dW items of the
// layer.  The caller runs the next chain step between this and the barrier
// that ends the phase.
template <class Plan, int L, int WV, int XS, typename XT, int NS>
__device__ __forceinline__ void dw_phase(XT *xb, const float *dz, const float *hin, int wave,
                                         f32x16 (&acc)[NS], int lane)
{
    constexpr int OUT = Plan::out_p(L), IN = Plan::in_p(L);
    constexpr int P = Plan::parts(L), KV = 32 * WV / P;
    xch_put<OUT / 2, XS>(xb, 0, wave, dz, lane);
    xch_put<IN / 2, XS>(xb, OUT, wave, hin, lane);
    __syncthreads();
#pragma unroll
    for (int it = 0; it < Plan::items(L); ++it) {
        constexpr int g0 = Plan::first(L);
        if ((g0 + it) % WV == wave) {
            const int b = it / P, p = it % P;
            const int bo = b / Plan::nbi(L), bi = b % Plan::nbi(L);
            dw_block<KV, XS>(xb, 32 * bo, OUT + 32 * bi, KV * p, acc[(g0 + it) / WV], lane);
        }
    }
}

// This block's weight gradients into the flat layout of the MLP weights at
// dst (entries outside the real shapes dropped): stored, or with ATOMIC added
// by FP32 atomics (several blocks add into one buffer).  The parts of a split
// block meet in LDS first: the owners of parts p > 0 leave theirs in `scr`
// (free LDS, 4 KB per split block), and the owner of part 0 adds them and
// writes.  Every thread of the block calls it (two barriers).
template <class Plan, int NH, int WV, bool ATOMIC = false, int NS>
__device__ __forceinline__ void dw_write(float *dst, int n_in, int width, int wave,
                                         f32x16 (&acc)[NS], int lane, float *scr)
{
    const int h = lane >> 5, j = lane & 31;
    if constexpr (Plan::splits() > 0) {
        __syncthreads();                 // the exchange buffer is free
        static_for_down<NH, 0>([&](auto LC) {
            constexpr int L = decltype(LC)::value;
            constexpr int P = Plan::parts(L);
            if constexpr (P > 1) {
#pragma unroll
                for (int it = 0; it < Plan::items(L); ++it) {
                    const int g = Plan::first(L) + it;
                    if (it % P == 0 || g % WV != wave) continue;
                    float *s = scr + (Plan::split_before(L) + it / P) * 1024;
#pragma unroll
                    for (int r = 0; r < 16; ++r) s[r * 64 + lane] = acc[g / WV][r];
                }
            }
        });
        __syncthreads();
    }
    static_for_down<NH, 0>([&](auto LC) {
        constexpr int L = decltype(LC)::value;
        constexpr int P = Plan::parts(L);
        const int out_r = L == NH ? 32 : width, in_r = L == 0 ? n_in : width;
        float *d = dst + (L == 0 ? 0 : width * n_in + (L - 1) * width * width);
#pragma unroll
        for (int it = 0; it < Plan::items(L); ++it) {
            const int g = Plan::first(L) + it;
            if (it % P != 0 || g % WV != wave) continue;
            const int b = it / P;
            const int bo = b / Plan::nbi(L), bi = b % Plan::nbi(L);
            const float *s = scr + (Plan::split_before(L) + b) * 1024;
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                float v = acc[g / WV][r];
                if constexpr (P > 1) v += s[r * 64 + lane];
                const int row = 32 * bo + nf(h, r), col = 32 * bi + j;
                if (row < out_r && col < in_r) {
                    if constexpr (ATOMIC) unsafeAtomicAdd(d + row * in_r + col, v);
                    else d[row * in_r + col] = v;
                }
            }
        }
    });
}

}  // namespace npm
