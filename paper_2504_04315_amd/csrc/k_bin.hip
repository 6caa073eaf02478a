// Binned grid scatter (the gradient of Sec. 4.2 pushed through the
// trilinear interpolation of Sec. 5.1 into the hashed levels).
//
// On a hashed level neighbouring vertices land on unrelated table entries, so
// no spatial order or LDS window brings their corners together, and every
// corner becomes one FP32 atomic request executed at the memory side -- the
// rate that bounds the plain scatter.  Here the corner contributions of those
// levels are instead binned by table slice (kBinSliceFloats floats) and each
// slice is summed by one block.  An item is a pair of x-neighbour corners:
// the hash takes x unmultiplied, so slot(x + 1) = slot(x) ^ (x ^ (x + 1)),
// which stays in the slice of slot(x) while the resolution is below the
// slice's entry count (the plan checks it).  An item holds the key (the
// lower corner's entry within the slice, and above bit 16 the xor to the
// upper one), the x fraction f and the F values wy wz dG; the reduce adds
// (1 - f) times them to the lower entry and f times them to the upper one.
//
//   count   per chunk of kBinChunk visiting slots, the number of items of
//           every (level, slice) bin              -> cnt[bin][chunk]
//   scan    exclusive prefix sum of cnt in bin-major order: the chunk's run
//           of items inside its bin's contiguous range
//   place   the chunk's items, ordered by bin in LDS and written out as
//           contiguous runs of (key, fraction, F values) records
//   reduce  one block per bin: LDS accumulation of its items -- FP64, or in
//           the precision form 64-bit fixed point (no FP64) -- then one
//           coalesced read-add-write of the slice into the gradient
//
// Items are recomputed identically by count and place (same inputs, same
// arithmetic), so place fills each chunk's run exactly; every LDS and global
// index is still checked against its buffer.  The values are the atomic
// scatter's corner weights applied to dG in another grouping (wx (wy wz dG)
// instead of (wx wy wz) dG) and summed in another order.
#include <type_traits>

#include "device_math.h"

namespace npm {

namespace {

__device__ __forceinline__ void slot_position(const float *__restrict__ pos, const uint32_t *perm,
                                              const float *__restrict__ rec, int rec_stride,
                                              int64_t n, int64_t s, float p[3])
{
    if (rec) {
        const f32x4 a = *reinterpret_cast<const f32x4 *>(rec + (size_t)s * rec_stride);
        p[0] = a[0]; p[1] = a[1]; p[2] = a[2];
    } else {
        const int64_t v = perm ? (int64_t)perm[s] : s;
        p[0] = pos[v]; p[1] = pos[n + v]; p[2] = pos[2 * n + v];
    }
}

// dG of slot s, level l, read from the per-tile rows (row l F + f, 32 slots).
// The loads are only issued here: the passes read the next level's values
// while they bin the current level's, and test them when that level comes.
template <int F>
__device__ __forceinline__ void slot_dg(const float *__restrict__ dgt, int rows, int64_t s, int l,
                                        float d[F])
{
    const float *src = dgt + (size_t)(s >> 5) * rows * 32 + (s & 31);
#pragma unroll
    for (int f = 0; f < F; ++f) d[f] = src[(l * F + f) * 32];
}

// Takes the prefetched values into d; true if any is non-zero (a slot whose
// dG is zero at a level adds nothing there and is not binned).
template <int F>
__device__ __forceinline__ bool take_dg(const float dn[F], float d[F])
{
    bool any = false;
#pragma unroll
    for (int f = 0; f < F; ++f) {
        d[f] = dn[f];
        any |= dn[f] != 0.0f;
    }
    return any;
}

// Hashed table slot of the lower corner of pair p (y offset p & 1, z offset
// p >> 1) of the cell, the xor m to its x-neighbour's slot, and the pair's
// weight wy wz (the same hash as the atomic scatter).
__device__ __forceinline__ uint32_t pair_slot(const int c[3], const float fr[3], int p,
                                              uint32_t mask, uint32_t &m, float &wyz)
{
    const int by = p & 1, bz = (p >> 1) & 1;
    const uint32_t X = c[0], Y = c[1] + by, Z = c[2] + bz;
    m = (X ^ (X + 1u)) & mask;
    wyz = (by ? fr[1] : 1.0f - fr[1]) * (bz ? fr[2] : 1.0f - fr[2]);
    return (X ^ (Y * 2654435761u) ^ (Z * 805459861u)) & mask;
}

__device__ __forceinline__ uint32_t wave_inclusive_scan(uint32_t x, int lane)
{
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t t = __shfl_up(x, o, 64);
        if (lane >= o) x += t;
    }
    return x;
}

}  // namespace

template <int F>
__global__ __launch_bounds__(kBinChunk) void k_bin_count(GridDesc g, BinDesc bd, int64_t n,
                                                         const float *__restrict__ pos,
                                                         const uint32_t *perm,
                                                         const float *__restrict__ rec,
                                                         int rec_stride,
                                                         const float *__restrict__ dgt, int rows,
                                                         uint32_t *__restrict__ cnt,
                                                         uint32_t *__restrict__ cmax)
{
    // NC copies of the histogram, lane t counting in copy t mod NC: fewer lanes of
    // one instruction on one counter (the copies sit HS words apart, off each
    // other's banks); the chunk's count is their sum (precision-form step
    // 2.06 -> 2.04 ms, FP32 within noise)
    constexpr int NC = 4, HS = kBinMaxBins + 1;
    __shared__ uint32_t hist[NC * HS];
    __shared__ int s_lv[NPM_MAX_LEVELS], s_res[NPM_MAX_LEVELS];
    __shared__ uint32_t s_max;
    for (int k = threadIdx.x; k < NC * HS; k += kBinChunk) hist[k] = 0u;
    if (threadIdx.x == 0) s_max = 0u;
    if (threadIdx.x < NPM_MAX_LEVELS) {
        s_lv[threadIdx.x] = bd.lv[threadIdx.x];
        s_res[threadIdx.x] = g.res[threadIdx.x];
    }
    // the sentinel after the last bin: the scan turns it into the total
    if (blockIdx.x == 0 && threadIdx.x == 0) cnt[(size_t)bd.nbins * bd.n_chunks] = 0u;
    __syncthreads();
    const int64_t s = blockIdx.x * (int64_t)kBinChunk + threadIdx.x;
    uint32_t *hc = hist + (threadIdx.x & (NC - 1)) * HS;
    float dmax = 0.0f;      // largest |dG| the chunk bins (bounds every item)
    if (s < n) {
        float p[3];
        slot_position(pos, perm, rec, rec_stride, n, s, p);
        float dn[F];
        slot_dg<F>(dgt, rows, s, s_lv[0], dn);
        for (int j = 0; j < bd.nb; ++j) {
            const int l = s_lv[j];
            float d[F];
            const bool any = take_dg<F>(dn, d);
            if (j + 1 < bd.nb) slot_dg<F>(dgt, rows, s, s_lv[j + 1], dn);
            if (!any) continue;
#pragma unroll
            for (int f = 0; f < F; ++f) dmax = fmaxf(dmax, fabsf(d[f]));
            int c[3];
            float fr[3];
#pragma unroll
            for (int a = 0; a < 3; ++a) lattice_cell(p[a], s_res[l], c[a], fr[a]);
#pragma unroll
            for (int pr = 0; pr < 4; ++pr) {
                uint32_t m;
                float wyz;
                const uint32_t slot = pair_slot(c, fr, pr, g.table_mask, m, wyz);
                atomicAdd(&hc[j * bd.ns + (int)(slot >> bd.log2s)], 1u);
            }
        }
    }
    // non-negative floats order as their bit patterns
    atomicMax(&s_max, __float_as_uint(dmax));
    __syncthreads();
    for (int k = threadIdx.x; k < bd.nbins; k += kBinChunk) {
        uint32_t c = 0u;
#pragma unroll
        for (int r = 0; r < NC; ++r) c += hist[r * HS + k];
        cnt[(size_t)k * bd.n_chunks + blockIdx.x] = c;
    }
    if (threadIdx.x == 0) cmax[blockIdx.x] = s_max;
}

// Exclusive prefix sum of m counters: per block of 1024, then over the block
// totals (one block, in segments), then the totals added back.
__global__ __launch_bounds__(1024) void k_bin_scan_local(uint32_t *__restrict__ v, int64_t m,
                                                         uint32_t *__restrict__ totals)
{
    __shared__ uint32_t wsum[16];
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int64_t i = blockIdx.x * (int64_t)1024 + t;
    const uint32_t x = i < m ? v[i] : 0u;
    const uint32_t inc = wave_inclusive_scan(x, lane);
    if (lane == 63) wsum[wave] = inc;
    __syncthreads();
    if (wave == 0) {
        const uint32_t ws = lane < 16 ? wsum[lane] : 0u;
        const uint32_t wi = wave_inclusive_scan(ws, lane);
        if (lane < 16) wsum[lane] = wi - ws;
        if (lane == 15) totals[blockIdx.x] = wi;
    }
    __syncthreads();
    if (i < m) v[i] = wsum[wave] + inc - x;
}

// (The same single block also reduces the chunks' largest |dG| to the
// batch's, cmax[n_chunks], which scales the fixed-point reduce.)
__global__ __launch_bounds__(1024) void k_bin_scan_totals(uint32_t *__restrict__ totals, int nblk,
                                                          uint32_t *__restrict__ cmax,
                                                          int64_t n_chunks)
{
    __shared__ uint32_t wsum[16];
    __shared__ uint32_t carry, bmax;
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    if (t == 0) {
        carry = 0u;
        bmax = 0u;
    }
    __syncthreads();
    uint32_t mx = 0u;
    for (int64_t i = t; i < n_chunks; i += 1024) mx = max(mx, cmax[i]);
    atomicMax(&bmax, mx);
    for (int base = 0; base < nblk; base += 1024) {
        const int i = base + t;
        const uint32_t x = i < nblk ? totals[i] : 0u;
        const uint32_t inc = wave_inclusive_scan(x, lane);
        if (lane == 63) wsum[wave] = inc;
        __syncthreads();
        if (wave == 0) {
            const uint32_t ws = lane < 16 ? wsum[lane] : 0u;
            const uint32_t wi = wave_inclusive_scan(ws, lane);
            if (lane < 16) wsum[lane] = wi - ws;
        }
        __syncthreads();
        const uint32_t c = carry;
        if (i < nblk) totals[i] = c + wsum[wave] + inc - x;
        __syncthreads();
        if (t == 1023) carry = c + wsum[15] + inc;
        __syncthreads();
    }
    if (t == 0) cmax[n_chunks] = bmax;
}

__global__ __launch_bounds__(1024) void k_bin_scan_add(uint32_t *__restrict__ v, int64_t m,
                                                       const uint32_t *__restrict__ totals)
{
    const int64_t i = blockIdx.x * (int64_t)1024 + threadIdx.x;
    if (i < m) v[i] += totals[blockIdx.x];
}

template <int F>
__global__ __launch_bounds__(kBinChunk) void k_bin_place(GridDesc g, BinDesc bd, int64_t n,
                                                         const float *__restrict__ pos,
                                                         const uint32_t *perm,
                                                         const float *__restrict__ rec,
                                                         int rec_stride,
                                                         const float *__restrict__ dgt, int rows,
                                                         const uint32_t *__restrict__ off,
                                                         uint32_t *__restrict__ items)
{
    constexpr int W = 2 + F;                 // words per item: key, fraction, F values
    constexpr int CAP = kBinChunk * 4;       // items (corner pairs) of one chunk and level
    __shared__ __attribute__((aligned(16))) uint32_t st[CAP * W];
    __shared__ uint16_t sb[CAP];
    __shared__ int s_lv[NPM_MAX_LEVELS], s_res[NPM_MAX_LEVELS];
    // sized by the launch: each bin's run start and length, then the level's
    // local bases and ranks (bin_place_lds_bytes)
    extern __shared__ __attribute__((aligned(16))) uint32_t dyn[];
    uint32_t *gd = dyn, *cn = dyn + bd.nbins, *lb = cn + bd.nbins, *rk = lb + bd.ns + 1;
    const int t = threadIdx.x, lane = t & 63;
    if (t < NPM_MAX_LEVELS) {
        s_lv[t] = bd.lv[t];
        s_res[t] = g.res[t];
    }
    const int64_t chunk = blockIdx.x;
    // this chunk's run of every bin (start, length), all fetched at once
    for (int kk = t; kk < bd.nbins; kk += kBinChunk) {
        const size_t idx = (size_t)kk * bd.n_chunks + chunk;
        const uint32_t g0 = off[idx];
        gd[kk] = g0;
        cn[kk] = off[idx + 1] - g0;
    }
    const int64_t s = chunk * kBinChunk + t;
    const bool live = s < n;
    float p[3] = {0.0f, 0.0f, 0.0f};
    if (live) slot_position(pos, perm, rec, rec_stride, n, s, p);
    const uint32_t smask = (1u << bd.log2s) - 1u;
    __syncthreads();
    float dn[F];
#pragma unroll
    for (int f = 0; f < F; ++f) dn[f] = 0.0f;
    if (live) slot_dg<F>(dgt, rows, s, s_lv[0], dn);
    for (int j = 0; j < bd.nb; ++j) {
        // local base of the chunk's run of each bin of the level
        if (t < 64) {
            uint32_t c0 = 0u;
            for (int k0 = 0; k0 < bd.ns; k0 += 64) {
                const int k = k0 + lane;
                uint32_t c = 0u;
                if (k < bd.ns) {
                    c = cn[j * bd.ns + k];
                    rk[k] = 0u;
                }
                const uint32_t inc = wave_inclusive_scan(c, lane);
                if (k < bd.ns) lb[k] = c0 + inc - c;
                c0 += __shfl(inc, 63, 64);
            }
            if (lane == 0) lb[bd.ns] = c0;
        }
        __syncthreads();
        const int l = s_lv[j];
        float d[F];
        const bool any = take_dg<F>(dn, d);
        if (live && j + 1 < bd.nb) slot_dg<F>(dgt, rows, s, s_lv[j + 1], dn);
        if (live && any) {
            int c[3];
            float fr[3];
#pragma unroll
            for (int a = 0; a < 3; ++a) lattice_cell(p[a], s_res[l], c[a], fr[a]);
#pragma unroll
            for (int pr = 0; pr < 4; ++pr) {
                uint32_t m;
                float wyz;
                const uint32_t slot = pair_slot(c, fr, pr, g.table_mask, m, wyz);
                const int k = (int)(slot >> bd.log2s);
                const uint32_t q = lb[k] + atomicAdd(&rk[k], 1u);
                if (q < lb[k + 1] && q < (uint32_t)CAP) {
                    if constexpr (W == 4) {
                        uint4 r;
                        r.x = (slot & smask) | (m << 16);
                        r.y = __float_as_uint(fr[0]);
                        r.z = __float_as_uint(wyz * d[0]);
                        r.w = __float_as_uint(wyz * d[1]);
                        *reinterpret_cast<uint4 *>(st + q * W) = r;
                    } else {
                        st[q * W] = (slot & smask) | (m << 16);
                        st[q * W + 1] = __float_as_uint(fr[0]);
#pragma unroll
                        for (int f = 0; f < F; ++f) st[q * W + 2 + f] = __float_as_uint(wyz * d[f]);
                    }
                    sb[q] = (uint16_t)k;
                }
            }
        }
        __syncthreads();
        const uint32_t tot = min(lb[bd.ns], (uint32_t)CAP);
        for (uint32_t q = t; q < tot; q += kBinChunk) {
            const int k = sb[q];
            if (k >= bd.ns) continue;
            const uint32_t dst = gd[j * bd.ns + k] + (q - lb[k]);
            if (dst < bd.cap) {
                uint32_t *it = items + (size_t)dst * W;
                if constexpr (W == 4) {
                    // nontemporal: the records are read once, by the reduce, after
                    // every chunk has written its own (FP32 step 2.75 -> 2.73 ms,
                    // precision form 2.11 -> 2.07 ms with the reduce's loads below)
                    __builtin_nontemporal_store(*reinterpret_cast<const f32x4 *>(st + q * W),
                                                reinterpret_cast<f32x4 *>(it));
                } else {
#pragma unroll
                    for (int w = 0; w < W; ++w) it[w] = st[q * W + w];
                }
            }
        }
        __syncthreads();
    }
}

// One block per bin: the slice's sums in LDS, then one coalesced
// read-add-write of the slice into the gradient.  The sums are FP64 (LDS
// FP64 atomic adds run several times faster than FP32 ones on this chip, and
// the wider sum rounds once, when it is added to the FP32 gradient), or, in
// the precision form (FIXED), 64-bit fixed point: with every corner value
// below the batch's largest |dG|, M < 2^e, and 2c corner values in the bin of
// c items (2c <= 2^b), the scale 2^(62 - e - b) keeps every entry's sum below
// 2^62; each value is rounded to a multiple of 2^(e + b - 62) (below 1e-12 of
// M for any bin of at most 2^22 items) and the sum is exact in any order.
template <int F, bool FIXED>
__global__ __launch_bounds__(kBinReduceThreads) void k_bin_reduce(GridDesc g, BinDesc bd,
                                                                  const uint32_t *__restrict__ off,
                                                                  const uint32_t *__restrict__ items,
                                                                  const uint32_t *__restrict__ bmax,
                                                                  float *__restrict__ grad)
{
    constexpr int NT = kBinReduceThreads, U = kBinReduceBatch;
    using AccT = typename std::conditional<FIXED, unsigned long long, double>::type;
    __shared__ AccT acc[kBinSliceFloats];
    constexpr int W = 2 + F;                 // words per item: key, fraction, F values
    const int k = blockIdx.x, j = k / bd.ns, slice = k - j * bd.ns;
    const uint32_t S = 1u << bd.log2s;
    const int nf = (int)S * F;
    const uint64_t beg = off[(size_t)k * bd.n_chunks];
    const uint64_t end = min(off[(size_t)(k + 1) * bd.n_chunks], (uint32_t)bd.cap);
    int kx = 0;                                  // fixed point: the scale is 2^kx
    if constexpr (FIXED) {
        const float M = __uint_as_float(*bmax);
        if (!(M > 0.0f) || end <= beg) return;   // nothing to add (block-uniform)
        int e;
        frexpf(M, &e);                           // M < 2^e
        const uint64_t c = 2 * (end - beg);                            // corner values
        const int b = c > 1 ? 64 - __clzll((long long)(c - 1)) : 0;   // c <= 2^b
        kx = 62 - e - b;
    }
    for (int i = threadIdx.x; i < nf; i += NT) acc[i] = AccT(0);
    __syncthreads();
    auto add1 = [&](uint32_t e, float v) {
        if constexpr (FIXED)
            __hip_atomic_fetch_add(&acc[e], (unsigned long long)__float2ll_rn(ldexpf(v, kx)),
                                   __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        else
            __hip_atomic_fetch_add(&acc[e], (double)v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    };
    // item: (1 - fx) v to the lower corner's entry, fx v to the upper one's
    auto add = [&](uint32_t key, float fx, const float *v) {
        const uint32_t e0 = key & 0xffffu, e1 = e0 ^ (key >> 16);
        if (e0 < S && e1 < S) {
            const float w0 = 1.0f - fx;
#pragma unroll
            for (int f = 0; f < F; ++f) {
                add1(e0 * F + f, w0 * v[f]);
                add1(e1 * F + f, fx * v[f]);
            }
        }
    };
    uint64_t i = beg + threadIdx.x;
    // U items in flight per thread: all loads issued before the first add
    // one item: its W words (one 16-byte nontemporal load at F = 2: each record
    // is read once)
    auto load = [&](uint64_t ii, uint32_t &e, float &fx, float *v) {
        const uint32_t *it = items + ii * W;
        if constexpr (W == 4) {
            const f32x4 r = __builtin_nontemporal_load(reinterpret_cast<const f32x4 *>(it));
            e = __float_as_uint(r[0]);
            fx = r[1];
            v[0] = r[2];
            v[1] = r[3];
        } else {
            e = it[0];
            fx = __uint_as_float(it[1]);
#pragma unroll
            for (int f = 0; f < F; ++f) v[f] = __uint_as_float(it[2 + f]);
        }
    };
    for (; i + (uint64_t)(U - 1) * NT < end; i += (uint64_t)U * NT) {
        uint32_t e[U];
        float fx[U], v[U][F];
#pragma unroll
        for (int u = 0; u < U; ++u) load(i + (uint64_t)u * NT, e[u], fx[u], v[u]);
#pragma unroll
        for (int u = 0; u < U; ++u) add(e[u], fx[u], v[u]);
    }
    for (; i < end; i += NT) {
        uint32_t e;
        float fx, v[F];
        load(i, e, fx, v);
        add(e, fx, v);
    }
    __syncthreads();
    float *dst = grad + ((size_t)g.offset[bd.lv[j]] + (size_t)slice * S) * F;
    for (int i2 = threadIdx.x; i2 < nf; i2 += NT) {
        if constexpr (FIXED) {
            const long long a = (long long)acc[i2];
            if (a != 0) dst[i2] += ldexpf(__ll2float_rn(a), -kx);
        } else {
            const double a = acc[i2];
            if (a != 0.0) dst[i2] += (float)a;
        }
    }
}

// Which levels are binned, and the sizes of the pass: every hashed level of
// an unordered batch; of a spatially ordered one, the hashed levels with
// D_l >= kBinMinResOrdered (coarser ones still fit the tile's LDS window).
bool bin_plan(const npm_ctx *ctx, int64_t n, bool ordered, BinDesc *out)
{
    const GridDesc &g = ctx->net.grid;
    const int F = g.feat;
    if (n <= 0 || !g.hashed_mask || (F != 1 && F != 2 && F != 4)) return false;
    BinDesc b{};
    for (int l = 0; l < g.n_levels; ++l)
        if (((g.hashed_mask >> l) & 1u) && (!ordered || g.res[l] >= kBinMinResOrdered))
            b.lv[b.nb++] = l;
    if (b.nb == 0) return false;
    int log2t = 0;
    while ((1u << log2t) <= g.table_mask) ++log2t;
    static_assert(kBinSliceFloats <= 65536, "slice entries and their xor are stored in 16 bits");
    int log2s = 0;
    while ((1 << (log2s + 1)) * F <= kBinSliceFloats) ++log2s;
    b.log2s = std::min(log2s, log2t);
    b.ns = 1 << (log2t - b.log2s);
    b.nbins = b.nb * b.ns;
    if (b.ns > kBinMaxSlices || b.nbins > kBinMaxBins) return false;
    // an x-neighbour pair shares a slice while x + 1 <= D_l < 2^log2s
    for (int j = 0; j < b.nb; ++j)
        if ((int64_t)g.res[b.lv[j]] >= ((int64_t)1 << b.log2s)) return false;
    b.n_chunks = (n + kBinChunk - 1) / kBinChunk;
    b.cap = n * 4 * b.nb;
    if (b.cap >= ((int64_t)1 << 32) - 1 || (int64_t)b.nbins * b.n_chunks + 1 >= ((int64_t)1 << 31))
        return false;
    *out = b;
    return true;
}

// counters (bin-major, and the sentinel), the scan's block totals, then the
// chunks' largest |dG| and the batch's
size_t bin_count_words(const BinDesc &b)
{
    const int64_t m = (int64_t)b.nbins * b.n_chunks + 1;
    return (size_t)m + (size_t)((m + 1023) / 1024) + (size_t)b.n_chunks + 1;
}

// items: cap records of (key, x fraction, F FP32 values)
size_t bin_item_words(const BinDesc &b, int feat)
{
    return (size_t)b.cap * (size_t)(2 + feat);
}

template <int F>
static void launch_bins(const GridDesc &g, const BinDesc &b, int64_t n, const float *pos,
                        const uint32_t *perm, const float *rec, int rec_stride, const float *dgt,
                        int rows, float *grad, uint32_t *cnt, uint32_t *items, int phase,
                        bool fixed, hipStream_t s)
{
    const int64_t m = (int64_t)b.nbins * b.n_chunks + 1;
    const int nblk = (int)((m + 1023) / 1024);
    uint32_t *cmax = cnt + m + nblk;             // n_chunks + 1 words
    switch (phase) {
    case 0:
        hipLaunchKernelGGL(k_bin_count<F>, dim3((unsigned)b.n_chunks), dim3(kBinChunk), 0, s, g, b,
                           n, pos, perm, rec, rec_stride, dgt, rows, cnt, cmax);
        break;
    case 1:
        hipLaunchKernelGGL(k_bin_scan_local, dim3(nblk), dim3(1024), 0, s, cnt, m, cnt + m);
        hipLaunchKernelGGL(k_bin_scan_totals, dim3(1), dim3(1024), 0, s, cnt + m, nblk, cmax,
                           b.n_chunks);
        hipLaunchKernelGGL(k_bin_scan_add, dim3(nblk), dim3(1024), 0, s, cnt, m, cnt + m);
        break;
    case 2:
        hipLaunchKernelGGL(k_bin_place<F>, dim3((unsigned)b.n_chunks), dim3(kBinChunk),
                           (size_t)(2 * b.nbins + 2 * b.ns + 1) * 4, s, g, b, n, pos, perm, rec,
                           rec_stride, dgt, rows, cnt, items);
        break;
    default:
        if (fixed)
            hipLaunchKernelGGL((k_bin_reduce<F, true>), dim3(b.nbins), dim3(kBinReduceThreads), 0, s,
                               g, b, cnt, items, cmax + b.n_chunks, grad);
        else
            hipLaunchKernelGGL((k_bin_reduce<F, false>), dim3(b.nbins), dim3(kBinReduceThreads), 0, s,
                               g, b, cnt, items, cmax + b.n_chunks, grad);
        break;
    }
}

hipError_t binned_scatter(npm_ctx *ctx, const BinDesc &b, int64_t n, const float *pos,
                          const uint32_t *perm, const float *rec, int rec_stride,
                          const float *dgt, int rows, float *grad, uint32_t *cnt,
                          uint32_t *items, hipStream_t s)
{
    const GridDesc &g = ctx->net.grid;
    // the precision form sums in fixed point (no FP64)
    const bool fx = ctx->net.cfg.precision == NPM_PREC_BF16;
    static const char *names[4] = {"bin_count", "bin_scan", "bin_place", "bin_reduce"};
    for (int phase = 0; phase < 4; ++phase) {
        int tok;
        timed_begin(ctx, names[phase], s, &tok);
        switch (g.feat) {
        case 1: launch_bins<1>(g, b, n, pos, perm, rec, rec_stride, dgt, rows, grad, cnt, items, phase, fx, s); break;
        case 2: launch_bins<2>(g, b, n, pos, perm, rec, rec_stride, dgt, rows, grad, cnt, items, phase, fx, s); break;
        default: launch_bins<4>(g, b, n, pos, perm, rec, rec_stride, dgt, rows, grad, cnt, items, phase, fx, s); break;
        }
        timed_end(ctx, tok, s);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace npm
