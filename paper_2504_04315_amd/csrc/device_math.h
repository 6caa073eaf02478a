// Device-side building blocks of the NPM hot path for gfx950: lattice cells
// and corner indices of the multiresolution grid (Sec. 5.1), the Table 1 output
// mappings and the vMF-mixture density and sampler (Preliminary; Sec. 5.3),
// the Monte Carlo KL gradient (Sec. 4.2, eq. mcgradients), Philox4x32-10
// uniforms (Salmon et al., SC'11), and 32-vertex MFMA tiles for the MLP.
#pragma once

#include <hip/hip_bf16.h>
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>

#include <cstdint>

#include "npm_internal.h"

namespace npm {

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

constexpr float kPi = 3.14159265358979323846f;
constexpr float kLog2Pi = 1.83787706640934548356f;   // log(2 pi)

// --------------------------------------------------------------------------
// Tile layout.  A wave holds a tile of 32 vertices: lane l owns vertex l & 31
// and, of a feature vector of width W, the W/2 features nf(l >> 5, a),
// a = 0 .. W/2-1.  This is exactly the row placement of the 32x32 MFMA
// accumulator (row 8*(a/4) + 4*(lane/32) + a%4 in register a), so a layer's
// output can feed the next layer's B operand without moving data.
// --------------------------------------------------------------------------
__device__ __forceinline__ constexpr int nf(int h, int a) { return 8 * (a >> 2) + 4 * h + (a & 3); }

// --------------------------------------------------------------------------
// Grid cell (Sec. 5.1): x clamped into [0, 1] (NaN -> 0), scaled by D_l with
// one float multiply, cell min(floor(p), D_l - 1), fraction p - cell (exact).
// --------------------------------------------------------------------------
__device__ __forceinline__ void lattice_cell(float x, int D, int &c, float &f)
{
    // The fraction must come from the rounded product: without this the
    // compiler fuses the multiply and the subtraction into one FMA.
#pragma clang fp contract(off)
    const float p = __fmul_rn(fminf(fmaxf(x, 0.0f), 1.0f), (float)D);
    int ci = (int)floorf(p);
    ci = ci < D - 1 ? ci : D - 1;
    c = ci;
    f = p - (float)ci;
}

// Table entry of lattice point (x, y, z) of level l: dense x + y(D+1) +
// z(D+1)^2, or the spatial hash (x*1 ^ y*2654435761 ^ z*805459861) mod T.
__device__ __forceinline__ uint32_t corner_entry(const GridDesc &g, int l, uint32_t x, uint32_t y,
                                                 uint32_t z)
{
    const uint32_t d1 = (uint32_t)g.res[l] + 1u;
    const uint32_t dense = x + d1 * (y + d1 * z);
    const uint32_t hash = (x ^ (y * 2654435761u) ^ (z * 805459861u)) & g.table_mask;
    return g.offset[l] + (((g.hashed_mask >> l) & 1u) ? hash : dense);
}

// Eight corners of the enclosing cell at level l: entries and trilinear weights;
// corner b has offsets (b & 1, b >> 1 & 1, b >> 2 & 1).
struct Corners {
    uint32_t e[8];
    float w[8];
};

__device__ __forceinline__ void level_corners(const GridDesc &g, int l, float px, float py,
                                              float pz, Corners &c)
{
    const int D = g.res[l];
    int cx, cy, cz;
    float fx, fy, fz;
    lattice_cell(px, D, cx, fx);
    lattice_cell(py, D, cy, fy);
    lattice_cell(pz, D, cz, fz);
    const float wx[2] = {1.0f - fx, fx}, wy[2] = {1.0f - fy, fy}, wz[2] = {1.0f - fz, fz};
#pragma unroll
    for (int b = 0; b < 8; ++b) {
        const int bx = b & 1, by = (b >> 1) & 1, bz = (b >> 2) & 1;
        c.w[b] = wx[bx] * wy[by] * wz[bz];
        c.e[b] = corner_entry(g, l, (uint32_t)(cx + bx), (uint32_t)(cy + by), (uint32_t)(cz + bz));
    }
}

// --------------------------------------------------------------------------
// Philox4x32-10: counter (vertex lo, vertex hi, stream, sample), key (seed lo,
// seed hi); u = (word >> 8) * 2^-24 in [0, 1), exact in float.
// --------------------------------------------------------------------------
__device__ __forceinline__ void philox_uniforms(uint64_t vertex, uint64_t seed, uint32_t stream,
                                                uint32_t sample, float u[3])
{
    uint32_t c0 = (uint32_t)vertex, c1 = (uint32_t)(vertex >> 32), c2 = stream, c3 = sample;
    uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint32_t hi0 = __umulhi(0xD2511F53u, c0), lo0 = 0xD2511F53u * c0;
        const uint32_t hi1 = __umulhi(0xCD9E8D57u, c2), lo1 = 0xCD9E8D57u * c2;
        const uint32_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
        c0 = n0; c1 = lo1; c2 = n2; c3 = lo0;
        k0 += 0x9E3779B9u; k1 += 0xBB67AE85u;
    }
    u[0] = (float)(c0 >> 8) * 0x1p-24f;
    u[1] = (float)(c1 >> 8) * 0x1p-24f;
    u[2] = (float)(c2 >> 8) * 0x1p-24f;
}

// --------------------------------------------------------------------------
// Table 1 mappings for one lobe from its raw outputs (theta', phi', kappa',
// lambda'); lambda's log-softmax needs the lobe set's log-sum-exp `lse`.
// --------------------------------------------------------------------------
struct Lobe {
    float theta, phi, kappa, loglam;
    float mu[3], t1[3], t2[3];
    float sinT;
};

__device__ __forceinline__ float clamp_kraw(float k) { return fminf(fmaxf(k, -80.0f), 80.0f); }

__device__ __forceinline__ void map_lobe(float th_raw, float ph_raw, float k_raw, float l_raw,
                                         float lse, Lobe &L)
{
    L.theta = 1.0f / (1.0f + expf(-th_raw));
    L.phi = 1.0f / (1.0f + expf(-ph_raw));
    L.kappa = expf(clamp_kraw(k_raw));
    L.loglam = l_raw - lse;
    float sT, cT, sP, cP;
    sincospif(L.theta, &sT, &cT);          // polar angle pi * theta
    sincospif(2.0f * L.phi, &sP, &cP);     // azimuth 2 pi * phi
    L.sinT = sT;
    L.mu[0] = sT * cP; L.mu[1] = sT * sP; L.mu[2] = cT;
    L.t1[0] = cT * cP; L.t1[1] = cT * sP; L.t1[2] = -sT;
    L.t2[0] = -sP;     L.t2[1] = cP;      L.t2[2] = 0.0f;
}

// log( kappa / (2 pi (1 - e^{-2 kappa})) ): the vMF normaliser kappa/(4 pi
// sinh kappa) times e^{kappa}, whose exponent is folded into kappa (mu.w - 1).
__device__ __forceinline__ float log_vmf_norm(float kappa)
{
    return logf(kappa / (-expm1f(-2.0f * kappa))) - kLog2Pi;
}

// log(lambda_k v_k(w)) for one lobe.
__device__ __forceinline__ float lobe_logterm(const Lobe &L, float wx, float wy, float wz)
{
    const float d = L.mu[0] * wx + L.mu[1] * wy + L.mu[2] * wz;
    return L.loglam + log_vmf_norm(L.kappa) + L.kappa * (d - 1.0f);
}

// Direction drawn from one lobe (Jakob 2012): cosine t from the inverse CDF
// of e^{kappa t} on [-1, 1], bounded to [-1, 1], azimuth 2 pi u2 in (t1, t2).
// 1 - t = -log1p((1 - u1) expm1(-2 kappa)) / kappa and
// 1 + t =  log1p(u1 expm1(2 kappa)) / kappa are carried separately (they are
// the same inverse CDF): each is accurate where the other cancels, near the
// lobe axis and near its antipode, and s = sqrt((1 - t)(1 + t)) needs both.
__device__ __forceinline__ void lobe_sample(const Lobe &L, float u1, float u2, float w[3])
{
    const float k = L.kappa;
    const float omt = fminf(2.0f, fmaxf(0.0f, -log1pf((1.0f - u1) * expm1f(-2.0f * k)) / k));
    // expm1(2 kappa) overflows beyond 2 kappa ~ 88; there 1 + t >= 1.6 and
    // 2 - (1 - t) does not cancel
    const float opt = (k < 40.0f) ? fminf(2.0f, fmaxf(0.0f, log1pf(u1 * expm1f(2.0f * k)) / k))
                                  : 2.0f - omt;
    const float t = omt < 1.0f ? 1.0f - omt : opt - 1.0f;
    const float s = sqrtf(omt * opt);
    float sp, cp;
    sincospif(2.0f * u2, &sp, &cp);
#pragma unroll
    for (int d = 0; d < 3; ++d) w[d] = t * L.mu[d] + s * (cp * L.t1[d] + sp * L.t2[d]);
}

// Gradient of log V w.r.t. one lobe's raw outputs, given its responsibility
// r = lambda_k v_k / V and lambda_k; scaled by g = d loss / d log V.
__device__ __forceinline__ void lobe_grad(const Lobe &L, float th_raw, float ph_raw, float k_raw,
                                          float r, float lam, float g, float wx, float wy, float wz,
                                          float out[4])
{
    const float k = L.kappa;
    const float d = L.mu[0] * wx + L.mu[1] * wy + L.mu[2] * wz;
    const float dt1 = L.t1[0] * wx + L.t1[1] * wy + L.t1[2] * wz;
    const float dt2 = L.t2[0] * wx + L.t2[1] * wy;
    // theta (1 - theta) and phi (1 - phi) from the two logistic tails
    const float th1 = 1.0f / (1.0f + expf(th_raw));
    const float ph1 = 1.0f / (1.0f + expf(ph_raw));
    const float dth = k * dt1 * kPi * L.theta * th1;
    const float dph = k * L.sinT * dt2 * 2.0f * kPi * L.phi * ph1;
    const bool clamped = (k_raw < -80.0f) || (k_raw > 80.0f);
    const float dka = clamped ? 0.0f : 1.0f - 2.0f * k / expm1f(2.0f * k) + k * (d - 1.0f);
    out[0] = g * r * dth;
    out[1] = g * r * dph;
    out[2] = g * r * dka;
    out[3] = g * (r - lam);
}

// Weight of a training sample: L / p for finite L > 0 and p > 0, else 0.
__device__ __forceinline__ float sample_weight(float rad, float pdf)
{
    const bool ok = isfinite(rad) && isfinite(pdf) && (pdf > 0.0f) && (rad > 0.0f);
    return ok ? rad / pdf : 0.0f;
}

// --------------------------------------------------------------------------
// MFMA layer tiles.  y (OUT_P wide) = W x for a 32-vertex tile in the tile
// layout, W read from a packed LDS image: FP32 image element
// ((b * IN_P/8 + s/4) * 64 + lane) * 4 + s % 4 holds W[32 b + lane % 32]
// [nf(lane / 32, s)]; BF16 image element ((b * IN_P/16 + s) * 64 + lane) * 8 + e
// holds W[32 b + lane % 32][nf(lane / 32, 8 s + e)].
// --------------------------------------------------------------------------
template <int IN_P, int OUT_P>
__device__ __forceinline__ void mfma_layer_f32(const float *__restrict__ img, const float *x,
                                               float *y, int lane)
{
    constexpr int NB = OUT_P / 32, NS4 = IN_P / 8;
    f32x16 acc[NB];
#pragma unroll
    for (int b = 0; b < NB; ++b)
#pragma unroll
        for (int v = 0; v < 16; ++v) acc[b][v] = 0.0f;
    // weights double-buffered by hand: the next group's LDS reads are issued
    // before this group's MFMAs, and the compiler barrier keeps them there
    // (hoisting every read would cost 4 VGPRs per MFMA group).
    f32x4 wc[NB], wn[NB];
#pragma unroll
    for (int b = 0; b < NB; ++b)
        wc[b] = *reinterpret_cast<const f32x4 *>(img + ((b * NS4 + 0) * 64 + lane) * 4);
#pragma unroll
    for (int s4 = 0; s4 < NS4; ++s4) {
        if (s4 + 1 < NS4) {
#pragma unroll
            for (int b = 0; b < NB; ++b)
                wn[b] = *reinterpret_cast<const f32x4 *>(img + ((b * NS4 + s4 + 1) * 64 + lane) * 4);
        }
        asm volatile("" ::: "memory");
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            acc[b] = __builtin_amdgcn_mfma_f32_32x32x2f32(wc[b][0], x[4 * s4 + 0], acc[b], 0, 0, 0);
            acc[b] = __builtin_amdgcn_mfma_f32_32x32x2f32(wc[b][1], x[4 * s4 + 1], acc[b], 0, 0, 0);
            acc[b] = __builtin_amdgcn_mfma_f32_32x32x2f32(wc[b][2], x[4 * s4 + 2], acc[b], 0, 0, 0);
            acc[b] = __builtin_amdgcn_mfma_f32_32x32x2f32(wc[b][3], x[4 * s4 + 3], acc[b], 0, 0, 0);
        }
#pragma unroll
        for (int b = 0; b < NB; ++b) wc[b] = wn[b];
    }
#pragma unroll
    for (int b = 0; b < NB; ++b)
#pragma unroll
        for (int v = 0; v < 16; ++v) y[16 * b + v] = acc[b][v];
}

template <int IN_P, int OUT_P>
__device__ __forceinline__ void mfma_layer_bf16(const __bf16 *__restrict__ img, const float *x,
                                                float *y, int lane)
{
    constexpr int NB = OUT_P / 32, NS = IN_P / 16;
    f32x16 acc[NB];
#pragma unroll
    for (int b = 0; b < NB; ++b)
#pragma unroll
        for (int v = 0; v < 16; ++v) acc[b][v] = 0.0f;
    bf16x8 wc[NB], wn[NB];
#pragma unroll
    for (int b = 0; b < NB; ++b)
        wc[b] = *reinterpret_cast<const bf16x8 *>(img + ((b * NS + 0) * 64 + lane) * 8);
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        if (s + 1 < NS) {
#pragma unroll
            for (int b = 0; b < NB; ++b)
                wn[b] = *reinterpret_cast<const bf16x8 *>(img + ((b * NS + s + 1) * 64 + lane) * 8);
        }
        asm volatile("" ::: "memory");
        bf16x8 xb;
#pragma unroll
        for (int e = 0; e < 8; ++e) xb[e] = (__bf16)x[8 * s + e];
#pragma unroll
        for (int b = 0; b < NB; ++b)
            acc[b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(wc[b], xb, acc[b], 0, 0, 0);
#pragma unroll
        for (int b = 0; b < NB; ++b) wc[b] = wn[b];
    }
#pragma unroll
    for (int b = 0; b < NB; ++b)
#pragma unroll
        for (int v = 0; v < 16; ++v) y[16 * b + v] = acc[b][v];
}

// y (OUT_P wide) = A x for a 32-vertex tile (x, y in the tile layout), A read
// from a row-major FP32 image in LDS whose rows are S floats apart: TR =
// false, A = W with element (o, i) at o S + i; TR = true, A = W^T, element
// (o, i) of A at i S + o.  One 4-byte read per lane and MFMA (the reads of a
// half-wave fall in distinct banks: S is odd, or the lanes read one row).
template <int IN_P, int OUT_P, int S, bool TR>
__device__ __forceinline__ void mfma_layer_rm(const float *__restrict__ img, const float *x,
                                              float *y, int lane)
{
    constexpr int NB = OUT_P / 32;
    const int i = lane & 31, h = lane >> 5;
    f32x16 acc[NB];
#pragma unroll
    for (int b = 0; b < NB; ++b)
#pragma unroll
        for (int v = 0; v < 16; ++v) acc[b][v] = 0.0f;
    const float *base = TR ? img + 4 * h * S + i : img + i * S + 4 * h;
    auto wt = [&](int a, int b) {
        const int k = 8 * (a >> 2) + (a & 3);     // nf(h, a) - 4 h
        return TR ? base[k * S + 32 * b] : base[32 * b * S + k];
    };
    // the weights of step a + PD are read while the MFMAs of step a run (the
    // compiler barrier keeps the reads ahead of the MFMAs)
    constexpr int NA = IN_P / 2, PD = 4;
    float w[PD][NB];
#pragma unroll
    for (int a = 0; a < PD && a < NA; ++a)
#pragma unroll
        for (int b = 0; b < NB; ++b) w[a][b] = wt(a, b);
#pragma unroll
    for (int a = 0; a < NA; ++a) {
        float cur[NB];
#pragma unroll
        for (int b = 0; b < NB; ++b) cur[b] = w[a % PD][b];
        if (a + PD < NA) {
#pragma unroll
            for (int b = 0; b < NB; ++b) w[a % PD][b] = wt(a + PD, b);
        }
        asm volatile("" ::: "memory");
#pragma unroll
        for (int b = 0; b < NB; ++b)
            acc[b] = __builtin_amdgcn_mfma_f32_32x32x2f32(cur[b], x[a], acc[b], 0, 0, 0);
    }
#pragma unroll
    for (int b = 0; b < NB; ++b)
#pragma unroll
        for (int v = 0; v < 16; ++v) y[16 * b + v] = acc[b][v];
}

// ------------------------------------------------------------------ NPM-product
// Real orthonormal spherical harmonics of the first four bands at the vector
// (x, y, z) (Sec. 4.3 encodes the outgoing direction and the normal with
// them): y[l*l + l + m], m > 0 with cos(m phi), m < 0 with sin(|m| phi), no
// Condon-Shortley phase.  Constants: band 0 1/(2 sqrt(pi)); band 1
// sqrt(3/(4 pi)); band 2 sqrt(15/pi)/2, sqrt(5/pi)/4, sqrt(15/pi)/4; band 3
// sqrt(35/(2 pi))/4, sqrt(105/pi)/2, sqrt(21/(2 pi))/4, sqrt(7/pi)/4,
// sqrt(105/pi)/4.
__device__ __forceinline__ void sh_bands4(float x, float y, float z, float *o)
{
    const float xx = x * x, yy = y * y, zz = z * z;
    o[0] = 0.28209479177387814f;
    o[1] = 0.48860251190291992f * y;
    o[2] = 0.48860251190291992f * z;
    o[3] = 0.48860251190291992f * x;
    o[4] = 1.0925484305920792f * x * y;
    o[5] = 1.0925484305920792f * y * z;
    o[6] = 0.31539156525252005f * (3.0f * zz - 1.0f);
    o[7] = 1.0925484305920792f * x * z;
    o[8] = 0.54627421529603959f * (xx - yy);
    o[9] = 0.59004358992664352f * y * (3.0f * xx - yy);
    o[10] = 2.8906114426405538f * x * y * z;
    o[11] = 0.45704579946446572f * y * (5.0f * zz - 1.0f);
    o[12] = 0.37317633259011540f * z * (5.0f * zz - 3.0f);
    o[13] = 0.45704579946446572f * x * (5.0f * zz - 1.0f);
    o[14] = 1.4453057213202769f * z * (xx - yy);
    o[15] = 0.59004358992664352f * x * (xx - 3.0f * yy);
}

// Wave-wide helpers for the two half-waves of a tile.
__device__ __forceinline__ float xor32(float v) { return __shfl_xor(v, 32, 64); }

// ------------------------------------------------------------------ selection
// Selection term of one sample (the learned selection probability): the
// renderer's one-sample density is p_c = c p_bsdf + (1 - c) V, c = sigmoid(c');
// with V held fixed, d(-(w/N) log p_c)/dc' = g c (1 - c) (p_bsdf - V) / p_c,
// g = -w/N.  With t = log p_bsdf - log V and c / (1 - c) = e^c' this is
//   t <= 0:  g c expm1(t) sigmoid(-(c' + t)),
//   t > 0:   g (1 - c) (-expm1(-t)) sigmoid(c' + t),
// and log p_c = log V - softplus(c') + softplus(c' + t) (t <= 0), or
// log p_bsdf - softplus(-c') + softplus(-c' - t) (t > 0): no cancellation,
// no division, and p_bsdf = 0 (t = -inf) gives -g c and log V + log(1 - c).
// Writes the derivative and returns log p_c.
__device__ __forceinline__ float softplusf(float x)
{
    return x > 0.0f ? x + log1pf(expf(-x)) : log1pf(expf(x));
}

__device__ __forceinline__ float sigmoidf(float x) { return 1.0f / (1.0f + expf(-x)); }

__device__ __forceinline__ float select_term(float cp, float pb, float lv, float g, float &ds)
{
    const float lp = logf(pb);
    const float t = lp - lv;
    if (t <= 0.0f) {
        ds = g * sigmoidf(cp) * expm1f(t) * sigmoidf(-(cp + t));
        return lv - softplusf(cp) + softplusf(cp + t);
    }
    ds = g * sigmoidf(-cp) * -expm1f(-t) * sigmoidf(cp + t);
    return lp - softplusf(-cp) + softplusf(-cp - t);
}

// A BSDF density that takes part in the selection term: finite and >= 0.
__device__ __forceinline__ bool bsdf_valid(float pb) { return isfinite(pb) && pb >= 0.0f; }

// The selection logit of a tile vertex: the last hidden layer hl (tile
// layout, HID_P features; the two half-waves hold the two halves) dotted with
// the selection row wsel (16-byte aligned, HID_P floats, zero past the
// width).  Both halves return the sum.
template <int HID_P>
__device__ __forceinline__ float select_logit(const float *wsel, const float *hl, int h)
{
    float p = 0.0f;
#pragma unroll
    for (int q = 0; q < HID_P / 8; ++q) {
        const f32x4 w = *reinterpret_cast<const f32x4 *>(wsel + 8 * q + 4 * h);
#pragma unroll
        for (int e = 0; e < 4; ++e) p = fmaf(w[e], hl[4 * q + e], p);
    }
    return p + xor32(p);
}


}  // namespace npm
