/*
 * npm_oracle.c -- plain FP64 CPU oracle for the Neural Parametric Mixtures
 * (NPM) hot path: multiresolution grid encoding, decoder MLP, the Table 1
 * output mappings, vMF-mixture pdf and sampling, the Monte Carlo KL
 * gradient, backpropagation with the grid scatter, and Adam.
 *
 * TEST INFRASTRUCTURE.  This file exists only to check the HIP library.  It
 * shares no source, header, table or helper with it; the two agree only
 * through the paper and the flat parameter layout documented below.  Only the
 * test-suite, the smoke check and the benchmark's CPU-baseline leg may load
 * it.  It is deliberately simple: one vertex at a time, in the order the
 * paper states the computation, in double precision.  The only float
 * arithmetic is the position scaling of the grid lookup, which is part of the
 * definition of the lattice cell (see oracle_cell) so that corner indices are
 * comparable bit for bit.
 *
 * Paper sections followed (Dong, Wang, Li, "Neural Parametric Mixtures for
 * Path Guiding", SIGGRAPH 2023):
 *   - Preliminary / "Von Mises-Fisher Mixtures": single-lobe vMF density and
 *     the K-lobe mixture.
 *   - Sec. 4.1 "Radiance-based NPM", eq. npmradiance and Table 1
 *     (tab:activations): exponential kappa, softmax lambda, logistic
 *     (theta, phi) as normalised spherical coordinates of mu.
 *   - Sec. 4.2 "Optimizing NPM": Monte Carlo KL estimator and its gradient,
 *     eq. mcgradients, and the spatially varying objective.
 *   - Sec. 5.1 "Multi-resolution Spatial Embedding": L uniform grids with
 *     exponentially growing resolution, F features per lattice point,
 *     interpolation over the eight cell corners, level concatenation.
 *   - Sec. 5.3 "Guiding Network": ReLU MLP, K = 8 lobes, Adam, and the
 *     numerically stable vMF sampling strategy of Jakob (2012).
 *   - Sec. 4.3 "Full Integrand Learning" (NPM-product): the outgoing
 *     direction and the surface normal, encoded with spherical harmonics, and
 *     the roughness, as extra inputs after G(x); and the moving average of
 *     the weights used for inference (Sec. 5.3).
 *   - Sec. 6.3 "Discussion", path-guiding extensions: the BSDF-selection
 *     probability learned by the network.
 *
 * Readings where the paper is silent (all of them documented in the design
 * notes of the repository, and fixed identically by the library):
 *   - interpolation is trilinear over the 8 corners (the text says
 *     "bilinear" but names eight corners);
 *   - positions live in [0,1]^3, level l has (D_l+1)^3 lattice points, the
 *     cell index is min(floor(x*D_l), D_l-1) with x*D_l one float multiply;
 *   - D_l = floor(D_min * b^l + 1e-6), b = (D_max/D_min)^(1/(L-1)), last
 *     level forced to D_max;
 *   - levels with more than T = 2^log2T lattice points use the spatial hash
 *     of Mueller et al. 2022 (cited by the paper for the embedding): XOR of
 *     (x*1, y*2654435761, z*805459861) in 32-bit arithmetic, modulo T;
 *   - the MLP has no biases; Theta' is lobe-major (theta', phi', kappa',
 *     lambda'); mu = (sin T cos P, sin T sin P, cos T) with T = pi*theta,
 *     P = 2*pi*phi; kappa' is clamped to [-80, 80] before exp;
 *   - the training weight is w = L/p for finite L > 0, p > 0, else 0; the
 *     batch mean divides by N including zero-weight samples;
 *   - Adam: beta1 0.9, beta2 0.999, eps 1e-8 outside the square root, bias
 *     correction with t counted from 1, dense update of every parameter;
 *   - NPM-product inputs: real orthonormal spherical harmonics of
 *     sh_degree bands (no Condon-Shortley phase, index l*l + l + m), of
 *     omega_o then of the normal, then the roughness, all used as given;
 *   - uniforms come from Philox4x32-10 (Salmon et al., SC'11) with counter
 *     (vertex lo, vertex hi, stream, sample) and key (seed lo, seed hi),
 *     u = (word >> 8) * 2^-24; lobe selection takes the first k with
 *     u0*S < C_k over the inclusive prefix sums C of lambda (S = C_{K-1}),
 *     falling back to K-1;
 *   - the learned selection probability (the paper names the extension and
 *     gives no formula) is one more raw output c', c = sigmoid(c'), trained
 *     by the Sec. 4.2 KL estimator applied to the renderer's one-sample
 *     mixture c p_bsdf + (1 - c) V with V held fixed in that term, the
 *     samples weighted as in the mixture's term.
 *
 * Flat parameter layout (the one interface shared with the library): the
 * grid tables first, level after level, entry-major with F features per entry
 * (entry e of level l, feature f at (offset_l + e)*F + f); then the weight
 * matrices W_0 .. W_{n_hidden}, each row-major [out][in]; with the selection
 * output the last matrix has 4K + 1 rows, the selection logit's last.
 *
 * Parity pins: every function here is pinned by a CPU test against the
 * mathematics (closed forms, quadrature, finite differences, invariants,
 * published known-answer vectors).  The resolution-growth rule and the hash
 * are readings, not results; they are pinned only by their properties.
 */
#include <omp.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define NPMO_MAX_LEVELS 32
#define NPMO_MAX_LAYERS 8
#define NPMO_MAX_WIDTH 256
#define NPMO_MAX_LOBES 16
#define NPMO_MAX_OUT (4 * NPMO_MAX_LOBES + 1)   /* lobe outputs, selection logit */

typedef struct {
    int64_t size[NPMO_MAX_LEVELS];    /* table entries of each level          */
    int64_t offset[NPMO_MAX_LEVELS];  /* first entry of each level            */
    int64_t layer_offset[NPMO_MAX_LAYERS]; /* first weight of each matrix     */
    int64_t grid_entries;
    int64_t grid_params;              /* grid_entries * feat                  */
    int64_t n_params;
    int32_t res[NPMO_MAX_LEVELS];
    int32_t hashed[NPMO_MAX_LEVELS];
    int32_t layer_in[NPMO_MAX_LAYERS];
    int32_t layer_out[NPMO_MAX_LAYERS];
    int32_t n_levels, feat, log2_table, dense_only;
    int32_t base_res, max_res;
    int32_t n_in, width, n_hidden, n_lobes, n_layers, n_out;
    int32_t sh_degree;                /* NPM-product: SH bands of omega_o, n   */
    int32_t n_aux;                    /* extra inputs after G(x) (0: radiance) */
    int32_t select;                   /* 1: output 4K is the selection logit  */
} npmo_net;

static const double PI = 3.14159265358979323846264338327950288;

/* MLP shapes and the flat offsets of its matrices (after the grid).        */
static void oracle_layers(npmo_net *net)
{
    net->n_in = net->n_levels * net->feat + net->n_aux;
    int64_t off = net->grid_params;
    for (int i = 0; i < net->n_layers; ++i) {
        net->layer_in[i] = (i == 0) ? net->n_in : net->width;
        net->layer_out[i] = (i == net->n_hidden) ? net->n_out : net->width;
        net->layer_offset[i] = off;
        off += (int64_t)net->layer_in[i] * net->layer_out[i];
    }
    net->n_params = off;
}

/* ------------------------------------------------------------------------ */
/* Level layout: Sec. 5.1, "D_l grows exponentially".                       */
/* ------------------------------------------------------------------------ */
/* Sizes and offsets of the levels from their resolutions: level l has
 * (D_l+1)^3 lattice points, stored densely unless they outnumber the table
 * (then the table of 2^log2T entries, addressed by the hash).              */
static void oracle_levels(npmo_net *net)
{
    net->grid_entries = 0;
    for (int l = 0; l < net->n_levels; ++l) {
        const int D = net->res[l];
        double pts = (double)(D + 1) * (double)(D + 1) * (double)(D + 1);
        if (net->dense_only || pts <= ldexp(1.0, net->log2_table)) {
            net->hashed[l] = 0;
            net->size[l] = (int64_t)(D + 1) * (D + 1) * (D + 1);
        } else {
            net->hashed[l] = 1;
            net->size[l] = (int64_t)1 << net->log2_table;
        }
        net->offset[l] = net->grid_entries;
        net->grid_entries += net->size[l];
    }
    net->grid_params = net->grid_entries * net->feat;
    oracle_layers(net);
}

int npmo_net_init(npmo_net *net, int L, int F, int base_res, int max_res,
                  int log2T, int dense_only, int n_hidden, int width, int K)
{
    if (!net || L < 1 || L > NPMO_MAX_LEVELS || F < 1 || F > 8) return -1;
    if (base_res < 1 || max_res < base_res) return -1;
    if (n_hidden < 1 || n_hidden + 1 > NPMO_MAX_LAYERS) return -1;
    if (width < 1 || width > NPMO_MAX_WIDTH || K < 1 || K > NPMO_MAX_LOBES) return -1;
    if (L * F > NPMO_MAX_WIDTH) return -1;
    if (!dense_only && (log2T < 1 || log2T > 30)) return -1;
    memset(net, 0, sizeof(*net));
    net->n_levels = L; net->feat = F; net->log2_table = log2T;
    net->dense_only = dense_only; net->base_res = base_res; net->max_res = max_res;
    for (int l = 0; l < L; ++l) {
        int D;
        if (l == L - 1) D = max_res;
        else if (l == 0) D = base_res;
        else {
            double b = exp(log((double)max_res / (double)base_res) / (double)(L - 1));
            D = (int)floor((double)base_res * pow(b, (double)l) + 1e-6);
        }
        net->res[l] = D;
    }
    net->width = width; net->n_hidden = n_hidden;
    net->n_lobes = K; net->n_out = 4 * K; net->n_layers = n_hidden + 1;
    net->select = 0;
    oracle_levels(net);
    return 0;
}

/* An explicit resolution table res[0 .. n_levels-1] (each 1..65535,
 * non-decreasing) in place of the exponential growth; the level layout and
 * the flat offsets follow.                                                 */
int npmo_net_set_resolution(npmo_net *net, const int32_t *res)
{
    if (!net || !res) return -1;
    for (int l = 0; l < net->n_levels; ++l)
        if (res[l] < 1 || res[l] > 65535 || (l > 0 && res[l] < res[l - 1])) return -1;
    for (int l = 0; l < net->n_levels; ++l) net->res[l] = res[l];
    net->base_res = res[0];
    net->max_res = res[net->n_levels - 1];
    oracle_levels(net);
    return 0;
}

/* Learned BSDF-selection probability (Sec. 6.3, Discussion, first of the
 * path-guiding extensions): one more raw output c' after the 4K lobe
 * outputs (one more row of the last weight matrix); the probability that
 * the renderer samples the BSDF rather than the mixture is
 * c = 1 / (1 + e^{-c'}).  on = 0 restores the plain network.               */
int npmo_net_set_selection(npmo_net *net, int on)
{
    if (!net) return -1;
    net->select = on ? 1 : 0;
    net->n_out = 4 * net->n_lobes + net->select;
    oracle_layers(net);
    return 0;
}

/* Full integrand learning (Sec. 4.3, NPM-product): the MLP input is G(x)
 * followed by the spherical-harmonics encoding of the outgoing direction and
 * of the surface normal (sh_degree bands each, sh_degree^2 values) and the
 * roughness.  sh_degree 0 restores the radiance-based network.              */
int npmo_net_set_inputs(npmo_net *net, int sh_degree)
{
    if (!net || sh_degree < 0 || sh_degree > 4) return -1;
    int n_aux = sh_degree ? 2 * sh_degree * sh_degree + 1 : 0;
    if (net->n_levels * net->feat + n_aux > NPMO_MAX_WIDTH) return -1;
    net->sh_degree = sh_degree;
    net->n_aux = n_aux;
    oracle_layers(net);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of the      */
/* 4-word S-box with multipliers 0xD2511F53 / 0xCD9E8D57 and key Weyl        */
/* increments 0x9E3779B9 / 0xBB67AE85.                                       */
/* ------------------------------------------------------------------------ */
void npmo_philox(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4])
{
    uint32_t c[4] = {ctr_in[0], ctr_in[1], ctr_in[2], ctr_in[3]};
    uint32_t k0 = key_in[0], k1 = key_in[1];
    for (int r = 0; r < 10; ++r) {
        if (r > 0) { k0 += 0x9E3779B9u; k1 += 0xBB67AE85u; }
        uint64_t p0 = (uint64_t)0xD2511F53u * c[0];
        uint64_t p1 = (uint64_t)0xCD9E8D57u * c[2];
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c[1] ^ k0;
        uint32_t n2 = hi0 ^ c[3] ^ k1;
        c[0] = n0; c[1] = lo1; c[2] = n2; c[3] = lo0;
    }
    out[0] = c[0]; out[1] = c[1]; out[2] = c[2]; out[3] = c[3];
}

static void uniforms3(int64_t vertex, uint64_t seed, uint32_t stream, uint32_t sample, double u[3])
{
    uint32_t ctr[4] = {(uint32_t)((uint64_t)vertex & 0xffffffffu), (uint32_t)((uint64_t)vertex >> 32),
                       stream, sample};
    uint32_t key[2] = {(uint32_t)(seed & 0xffffffffu), (uint32_t)(seed >> 32)};
    uint32_t w[4];
    npmo_philox(ctr, key, w);
    for (int i = 0; i < 3; ++i) u[i] = (double)(w[i] >> 8) * (1.0 / 16777216.0);
}

void npmo_uniforms(int64_t n, const int64_t *vid, uint64_t seed, uint32_t stream,
                   uint32_t sample, double *u /* [n][3] */)
{
    for (int64_t i = 0; i < n; ++i) uniforms3(vid ? vid[i] : i, seed, stream, sample, u + 3 * i);
}

/* ------------------------------------------------------------------------ */
/* Sec. 5.1: the cell of G_l enclosing x, its eight corners and weights.     */
/* ------------------------------------------------------------------------ */
static void oracle_cell(float x, int D, int *c, double *f)
{
    /* Clamp into the unit cube (NaN goes to 0), then one IEEE float multiply. */
    float xc = fminf(fmaxf(x, 0.0f), 1.0f);
    volatile float p = xc * (float)D;
    int ci = (int)floorf(p);
    if (ci > D - 1) ci = D - 1;
    *c = ci;
    *f = (double)(p - (float)ci); /* exact: p and ci are within a factor 2 */
}

static int64_t oracle_corner_index(const npmo_net *net, int l, int64_t x, int64_t y, int64_t z)
{
    int64_t D1 = (int64_t)net->res[l] + 1;
    if (!net->hashed[l]) return net->offset[l] + x + y * D1 + z * D1 * D1;
    uint32_t h = ((uint32_t)x * 1u) ^ ((uint32_t)y * 2654435761u) ^ ((uint32_t)z * 805459861u);
    return net->offset[l] + (int64_t)(h % ((uint32_t)1u << net->log2_table));
}

/* idx[l][8] (global entry index) and w[l][8] for one position; corner b has
 * x offset (b & 1), y offset ((b >> 1) & 1), z offset ((b >> 2) & 1).      */
static void oracle_corners_one(const npmo_net *net, float px, float py, float pz,
                               int64_t *idx, double *w)
{
    for (int l = 0; l < net->n_levels; ++l) {
        int c[3]; double f[3];
        oracle_cell(px, net->res[l], &c[0], &f[0]);
        oracle_cell(py, net->res[l], &c[1], &f[1]);
        oracle_cell(pz, net->res[l], &c[2], &f[2]);
        for (int b = 0; b < 8; ++b) {
            int bx = b & 1, by = (b >> 1) & 1, bz = (b >> 2) & 1;
            double wx = bx ? f[0] : 1.0 - f[0];
            double wy = by ? f[1] : 1.0 - f[1];
            double wz = bz ? f[2] : 1.0 - f[2];
            w[l * 8 + b] = wx * wy * wz;
            idx[l * 8 + b] = oracle_corner_index(net, l, c[0] + bx, c[1] + by, c[2] + bz);
        }
    }
}

void npmo_corners(const npmo_net *net, int64_t n, const float *pos /* [3][n] */,
                  int64_t *idx /* [n][L][8] */, double *w /* [n][L][8] */)
{
    int L = net->n_levels;
    for (int64_t i = 0; i < n; ++i)
        oracle_corners_one(net, pos[i], pos[n + i], pos[2 * n + i], idx + i * L * 8, w + i * L * 8);
}

/* ------------------------------------------------------------------------ */
/* Real spherical harmonics, orthonormal on the unit sphere, bands l < deg,  */
/* index l*l + l + m (m = -l..l): m > 0 goes with cos(m phi), m < 0 with    */
/* sin(|m| phi), written as polynomials in the components of the unit       */
/* vector.  Each function is a list of monomials c x^a y^b z^e; the value    */
/* is their sum and the condition scale the sum of their magnitudes.        */
/* ------------------------------------------------------------------------ */
typedef struct { double c; int a, b, e; } oracle_mono;

static int oracle_sh_monos(int idx, oracle_mono *m)
{
    const double k0 = 0.5 / sqrt(PI);                     /* Y_00            */
    const double k1 = sqrt(3.0 / (4.0 * PI));             /* band 1          */
    const double k2 = 0.5 * sqrt(15.0 / PI), k20 = 0.25 * sqrt(5.0 / PI),
                 k22 = 0.25 * sqrt(15.0 / PI);
    const double k33 = 0.25 * sqrt(35.0 / (2.0 * PI)), k32 = 0.5 * sqrt(105.0 / PI),
                 k31 = 0.25 * sqrt(21.0 / (2.0 * PI)), k30 = 0.25 * sqrt(7.0 / PI),
                 k32c = 0.25 * sqrt(105.0 / PI);
    switch (idx) {
    case 0: m[0] = (oracle_mono){k0, 0, 0, 0}; return 1;
    case 1: m[0] = (oracle_mono){k1, 0, 1, 0}; return 1;                 /* y   */
    case 2: m[0] = (oracle_mono){k1, 0, 0, 1}; return 1;                 /* z   */
    case 3: m[0] = (oracle_mono){k1, 1, 0, 0}; return 1;                 /* x   */
    case 4: m[0] = (oracle_mono){k2, 1, 1, 0}; return 1;                 /* xy  */
    case 5: m[0] = (oracle_mono){k2, 0, 1, 1}; return 1;                 /* yz  */
    case 6: m[0] = (oracle_mono){3.0 * k20, 0, 0, 2};                    /* 3z^2-1 */
            m[1] = (oracle_mono){-k20, 0, 0, 0}; return 2;
    case 7: m[0] = (oracle_mono){k2, 1, 0, 1}; return 1;                 /* xz  */
    case 8: m[0] = (oracle_mono){k22, 2, 0, 0};                          /* x^2-y^2 */
            m[1] = (oracle_mono){-k22, 0, 2, 0}; return 2;
    case 9: m[0] = (oracle_mono){3.0 * k33, 2, 1, 0};                    /* y(3x^2-y^2) */
            m[1] = (oracle_mono){-k33, 0, 3, 0}; return 2;
    case 10: m[0] = (oracle_mono){k32, 1, 1, 1}; return 1;               /* xyz */
    case 11: m[0] = (oracle_mono){5.0 * k31, 0, 1, 2};                   /* y(5z^2-1) */
             m[1] = (oracle_mono){-k31, 0, 1, 0}; return 2;
    case 12: m[0] = (oracle_mono){5.0 * k30, 0, 0, 3};                   /* z(5z^2-3) */
             m[1] = (oracle_mono){-3.0 * k30, 0, 0, 1}; return 2;
    case 13: m[0] = (oracle_mono){5.0 * k31, 1, 0, 2};                   /* x(5z^2-1) */
             m[1] = (oracle_mono){-k31, 1, 0, 0}; return 2;
    case 14: m[0] = (oracle_mono){k32c, 2, 0, 1};                        /* z(x^2-y^2) */
             m[1] = (oracle_mono){-k32c, 0, 2, 1}; return 2;
    case 15: m[0] = (oracle_mono){k33, 3, 0, 0};                         /* x(x^2-3y^2) */
             m[1] = (oracle_mono){-3.0 * k33, 1, 2, 0}; return 2;
    default: return 0;
    }
}

/* out[i] (and scale[i], or NULL) for i < deg*deg at the vector (x, y, z).   */
void npmo_sh(int deg, double x, double y, double z, double *out, double *scale)
{
    for (int i = 0; i < deg * deg; ++i) {
        oracle_mono m[2];
        int k = oracle_sh_monos(i, m);
        double v = 0.0, a = 0.0;
        for (int j = 0; j < k; ++j) {
            double t = m[j].c * pow(x, m[j].a) * pow(y, m[j].b) * pow(z, m[j].e);
            v += t; a += fabs(t);
        }
        out[i] = v;
        if (scale) scale[i] = a;
    }
}

/* The extra inputs of NPM-product for one vertex: aux7 = (omega_o, normal,
 * roughness), as float values; appended after the net's L*F grid features. */
static void oracle_aux_one(const npmo_net *net, const float *aux7, double *G, double *gscale)
{
    int base = net->n_levels * net->feat, d = net->sh_degree, nb = d * d;
    if (!net->n_aux) return;
    npmo_sh(d, aux7[0], aux7[1], aux7[2], G + base, gscale ? gscale + base : NULL);
    npmo_sh(d, aux7[3], aux7[4], aux7[5], G + base + nb, gscale ? gscale + base + nb : NULL);
    G[base + 2 * nb] = aux7[6];
    if (gscale) gscale[base + 2 * nb] = fabs((double)aux7[6]);
}

/* Vertex i's extra inputs from the SoA array aux [7][n] (zeros if NULL).   */
static void oracle_aux_fetch(const float *aux, int64_t n, int64_t i, float aux7[7])
{
    for (int j = 0; j < 7; ++j) aux7[j] = aux ? aux[j * n + i] : 0.0f;
}

/* G(x) = concat_l sum_corners w_c V_l[c]  (level-major, index l*F + f).
 * gscale receives sum_c |w_c V_l[c]| per output, the size of the terms.    */
static void oracle_encode_one(const npmo_net *net, float px, float py, float pz,
                              const double *params, double *G, double *gscale)
{
    int L = net->n_levels, F = net->feat;
    int64_t idx[NPMO_MAX_LEVELS * 8];
    double w[NPMO_MAX_LEVELS * 8];
    oracle_corners_one(net, px, py, pz, idx, w);
    for (int l = 0; l < L; ++l)
        for (int f = 0; f < F; ++f) {
            double s = 0.0, a = 0.0;
            for (int b = 0; b < 8; ++b) {
                double t = w[l * 8 + b] * params[idx[l * 8 + b] * F + f];
                s += t; a += fabs(t);
            }
            G[l * F + f] = s;
            if (gscale) gscale[l * F + f] = a;
        }
}

void npmo_encode(const npmo_net *net, int64_t n, const float *pos, const float *aux /* [7][n] or NULL */,
                 const double *params, double *G /* [n][n_in] */,
                 double *gscale /* [n][n_in] or NULL */)
{
    int ni = net->n_in;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        float a7[7];
        oracle_aux_fetch(aux, n, i, a7);
        oracle_encode_one(net, pos[i], pos[n + i], pos[2 * n + i], params, G + i * ni,
                          gscale ? gscale + i * ni : NULL);
        oracle_aux_one(net, a7, G + i * ni, gscale ? gscale + i * ni : NULL);
    }
}

/* ------------------------------------------------------------------------ */
/* Decoder MLP (Sec. 5.3): z_i = W_i h_i, h_{i+1} = ReLU(z_i) for the hidden */
/* layers, raw output Theta' = W_last h_last.                                */
/* acts[i] holds the input of layer i (acts[0] = G).                        */
/* ------------------------------------------------------------------------ */
static void oracle_mlp_one(const npmo_net *net, const double *G, const double *params,
                           double acts[NPMO_MAX_LAYERS][NPMO_MAX_WIDTH],
                           double *raw, double *rawscale)
{
    for (int j = 0; j < net->n_in; ++j) acts[0][j] = G[j];
    for (int i = 0; i < net->n_layers; ++i) {
        const double *W = params + net->layer_offset[i];
        int nin = net->layer_in[i], nout = net->layer_out[i];
        int last = (i == net->n_layers - 1);
        for (int o = 0; o < nout; ++o) {
            double s = 0.0, a = 0.0;
            for (int k = 0; k < nin; ++k) {
                double t = W[(int64_t)o * nin + k] * acts[i][k];
                s += t; a += fabs(t);
            }
            if (last) {
                raw[o] = s;
                if (rawscale) rawscale[o] = a;
            } else {
                acts[i + 1][o] = s > 0.0 ? s : 0.0;
            }
        }
    }
}

/* The same forward, also carrying the condition scale of every value: the
 * sum of |terms| that an FP32 evaluation rounds, propagated through the
 * layers (cond(z_o) = sum_k |W_ok| cond(h_k); ReLU passes it where z > 0).
 * The tolerance of a float evaluation of z is proportional to cond(z), not
 * to |z|, which cancellation can make arbitrarily small.
 * A hidden pre-activation within 2^-20 cond(z) of zero has a sign that an
 * FP32 evaluation does not determine (its rounding error reaches a fraction
 * of 2^-24 cond(z)), so either side of the ReLU is a correct FP32 result:
 * such a unit is flagged in amb (its output's condition stays cond(z), as
 * FP32 may pass z through), and the backward widens its derivative's
 * condition to cover the other choice.                                     */
#define NPMO_KINK (1.0 / 1048576.0)
static void oracle_mlp_cond_one(const npmo_net *net, const double *G, const double *Gcond,
                                const double *params,
                                double acts[NPMO_MAX_LAYERS][NPMO_MAX_WIDTH],
                                double cacts[NPMO_MAX_LAYERS][NPMO_MAX_WIDTH],
                                unsigned char amb[NPMO_MAX_LAYERS][NPMO_MAX_WIDTH],
                                double *raw, double *rawcond)
{
    for (int j = 0; j < net->n_in; ++j) { acts[0][j] = G[j]; cacts[0][j] = Gcond[j]; }
    for (int i = 0; i < net->n_layers; ++i) {
        const double *W = params + net->layer_offset[i];
        int nin = net->layer_in[i], nout = net->layer_out[i];
        int last = (i == net->n_layers - 1);
        for (int o = 0; o < nout; ++o) {
            double s = 0.0, c = 0.0;
            for (int k = 0; k < nin; ++k) {
                s += W[(int64_t)o * nin + k] * acts[i][k];
                c += fabs(W[(int64_t)o * nin + k]) * cacts[i][k];
            }
            if (last) { raw[o] = s; rawcond[o] = c; }
            else {
                int a = fabs(s) <= NPMO_KINK * c;
                amb[i + 1][o] = (unsigned char)a;
                acts[i + 1][o] = s > 0.0 ? s : 0.0;
                cacts[i + 1][o] = (s > 0.0 || a) ? c : 0.0;
            }
        }
    }
}

void npmo_mlp_forward(const npmo_net *net, int64_t n, const double *G, const double *params,
                      double *raw /* [n][4K] */, double *rawscale /* [n][4K] or NULL */)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        double acts[NPMO_MAX_LAYERS][NPMO_MAX_WIDTH];
        oracle_mlp_one(net, G + i * net->n_in, params, acts, raw + i * net->n_out,
                       rawscale ? rawscale + i * net->n_out : NULL);
    }
}

/* ------------------------------------------------------------------------ */
/* Table 1 mappings and the lobe frames.                                     */
/* ------------------------------------------------------------------------ */
typedef struct {
    double theta, phi, kappa, lambda, loglambda;
    double mu[3], t1[3], t2[3];
    double sinT;
} oracle_lobe;

static double clamp_kappa_raw(double k) { return k < -80.0 ? -80.0 : (k > 80.0 ? 80.0 : k); }

static void oracle_map(const npmo_net *net, const double *raw, oracle_lobe *lob)
{
    int K = net->n_lobes;
    double mx = -INFINITY;
    for (int k = 0; k < K; ++k) if (raw[4 * k + 3] > mx) mx = raw[4 * k + 3];
    double se = 0.0;
    for (int k = 0; k < K; ++k) se += exp(raw[4 * k + 3] - mx);
    double lse = mx + log(se);
    for (int k = 0; k < K; ++k) {
        oracle_lobe *b = &lob[k];
        b->theta = 1.0 / (1.0 + exp(-raw[4 * k + 0]));
        b->phi = 1.0 / (1.0 + exp(-raw[4 * k + 1]));
        b->kappa = exp(clamp_kappa_raw(raw[4 * k + 2]));
        b->loglambda = raw[4 * k + 3] - lse;
        b->lambda = exp(b->loglambda);
        double T = PI * b->theta, P = 2.0 * PI * b->phi;
        double sT = sin(T), cT = cos(T), sP = sin(P), cP = cos(P);
        b->sinT = sT;
        b->mu[0] = sT * cP; b->mu[1] = sT * sP; b->mu[2] = cT;
        b->t1[0] = cT * cP; b->t1[1] = cT * sP; b->t1[2] = -sT;
        b->t2[0] = -sP;     b->t2[1] = cP;      b->t2[2] = 0.0;
    }
}

/* log of the vMF normaliser kappa / (4 pi sinh kappa), written as
 * kappa / (2 pi (1 - e^{-2 kappa})) * e^{-kappa} so that the exponent can be
 * folded into kappa (mu.w - 1); this function returns log of the first
 * factor.  The identity is exact; it only avoids overflow of sinh.         */
static double log_vmf_norm(double kappa)
{
    return log(kappa / (-expm1(-2.0 * kappa))) - log(2.0 * PI);
}

/* Per-lobe log terms log(lambda_k v_k(w)) and the mixture log-density.      */
static double oracle_logpdf(const npmo_net *net, const oracle_lobe *lob, const double w[3],
                            double *terms /* [K] or NULL */)
{
    int K = net->n_lobes;
    double t[NPMO_MAX_LOBES], mx = -INFINITY;
    for (int k = 0; k < K; ++k) {
        double d = lob[k].mu[0] * w[0] + lob[k].mu[1] * w[1] + lob[k].mu[2] * w[2];
        t[k] = lob[k].loglambda + log_vmf_norm(lob[k].kappa) + lob[k].kappa * (d - 1.0);
        if (t[k] > mx) mx = t[k];
    }
    double s = 0.0;
    for (int k = 0; k < K; ++k) s += exp(t[k] - mx);
    if (terms) for (int k = 0; k < K; ++k) terms[k] = t[k];
    return mx + log(s);
}

void npmo_head(const npmo_net *net, int64_t n, const double *raw, double *lobes /* [n][K][4] */)
{
    int K = net->n_lobes;
    for (int64_t i = 0; i < n; ++i) {
        oracle_lobe lob[NPMO_MAX_LOBES];
        oracle_map(net, raw + i * net->n_out, lob);
        for (int k = 0; k < K; ++k) {
            double *o = lobes + (i * K + k) * 4;
            o[0] = lob[k].theta; o[1] = lob[k].phi; o[2] = lob[k].kappa; o[3] = lob[k].lambda;
        }
    }
}

void npmo_logpdf(const npmo_net *net, int64_t n, const double *raw, const double *dir /* [n][3] */,
                 double *logpdf)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        oracle_lobe lob[NPMO_MAX_LOBES];
        oracle_map(net, raw + i * net->n_out, lob);
        logpdf[i] = oracle_logpdf(net, lob, dir + 3 * i, NULL);
    }
}

/* Sampling (Sec. 5.3, Jakob 2012): choose a lobe by the inverse CDF of the
 * weights, draw the cosine t to mu from the marginal density proportional to
 * e^{kappa t} on [-1, 1] by its inverse CDF in the log1p/expm1 form, and the
 * azimuth uniformly in the lobe frame (t1, t2).                            */
static void oracle_sample_one(const npmo_net *net, const oracle_lobe *lob, const double u[3],
                              double w[3], int *lobe_out, double *margin)
{
    int K = net->n_lobes;
    double C[NPMO_MAX_LOBES] = {0.0}, acc = 0.0;
    for (int k = 0; k < K; ++k) { acc += lob[k].lambda; C[k] = acc; }
    double S = C[K - 1], target = u[0] * S;
    int sel = K - 1;
    for (int k = 0; k < K; ++k) if (target < C[k]) { sel = k; break; }
    if (margin) {
        double m = INFINITY;
        for (int k = 0; k < K - 1; ++k) { double d = fabs(target - C[k]) / S; if (d < m) m = d; }
        *margin = m;
    }
    const oracle_lobe *b = &lob[sel];
    double kappa = b->kappa;
    double t = 1.0 + log1p((1.0 - u[1]) * expm1(-2.0 * kappa)) / kappa;
    /* The inverse CDF is -1 at u1 = 0; e^{-2 kappa} underflows for large
     * kappa and the formula then yields -inf, so bound t to [-1, 1].       */
    t = fmin(1.0, fmax(-1.0, t));
    double s = sqrt(fmax(0.0, (1.0 - t) * (1.0 + t)));
    double psi = 2.0 * PI * u[2];
    double cp = cos(psi), sp = sin(psi);
    for (int d = 0; d < 3; ++d) w[d] = t * b->mu[d] + s * (cp * b->t1[d] + sp * b->t2[d]);
    *lobe_out = sel;
}

/* Query: lobes, log pdf at dir, one sample and its log pdf, per vertex.
 * vid gives the vertex number used as the random counter (NULL = 0..n-1). */
void npmo_query(const npmo_net *net, int64_t n, const float *pos, const float *aux /* [7][n] or NULL */,
                const float *dir /* [3][n] or NULL */,
                const int64_t *vid, uint64_t seed, uint32_t stream, const double *params,
                double *G_out /* [n][n_in] or NULL */, double *raw_out /* [n][4K] or NULL */,
                double *lobes /* [n][K][4] or NULL */, double *logpdf /* [n] or NULL */,
                double *sdir /* [n][3] or NULL */, double *slogpdf /* [n] or NULL */,
                int32_t *slobe /* [n] or NULL */, double *smargin /* [n] or NULL */,
                double *sel /* [n] selection probability c, or NULL */)
{
    int K = net->n_lobes;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        double G[NPMO_MAX_WIDTH], raw[NPMO_MAX_OUT];
        double acts[NPMO_MAX_LAYERS][NPMO_MAX_WIDTH];
        oracle_lobe lob[NPMO_MAX_LOBES];
        float a7[7];
        oracle_aux_fetch(aux, n, i, a7);
        oracle_encode_one(net, pos[i], pos[n + i], pos[2 * n + i], params, G, NULL);
        oracle_aux_one(net, a7, G, NULL);
        oracle_mlp_one(net, G, params, acts, raw, NULL);
        oracle_map(net, raw, lob);
        if (G_out) for (int j = 0; j < net->n_in; ++j) G_out[i * net->n_in + j] = G[j];
        if (raw_out) for (int j = 0; j < net->n_out; ++j) raw_out[i * net->n_out + j] = raw[j];
        if (sel && net->select) sel[i] = 1.0 / (1.0 + exp(-raw[4 * K]));
        if (lobes)
            for (int k = 0; k < K; ++k) {
                double *o = lobes + (i * K + k) * 4;
                o[0] = lob[k].theta; o[1] = lob[k].phi; o[2] = lob[k].kappa; o[3] = lob[k].lambda;
            }
        if (logpdf && dir) {
            double w[3] = {dir[i], dir[n + i], dir[2 * n + i]};
            logpdf[i] = oracle_logpdf(net, lob, w, NULL);
        }
        if (sdir || slogpdf || slobe) {
            double u[3], w[3];
            int sel; double mg;
            uniforms3(vid ? vid[i] : i, seed, stream, 0, u);
            oracle_sample_one(net, lob, u, w, &sel, &mg);
            if (sdir) for (int d = 0; d < 3; ++d) sdir[3 * i + d] = w[d];
            if (slogpdf) slogpdf[i] = oracle_logpdf(net, lob, w, NULL);
            if (slobe) slobe[i] = sel;
            if (smargin) smargin[i] = mg;
        }
    }
}

/* Sampling from given raw outputs with explicit uniforms [n][3] (used by
 * the statistical pins, where many draws share one mixture).               */
void npmo_sample_raw(const npmo_net *net, int64_t n, const double *raw /* [n][4K] */,
                     const double *u /* [n][3] */, double *sdir /* [n][3] */, int32_t *slobe)
{
    for (int64_t i = 0; i < n; ++i) {
        oracle_lobe lob[NPMO_MAX_LOBES];
        double w[3]; int sel; double mg;
        oracle_map(net, raw + i * net->n_out, lob);
        oracle_sample_one(net, lob, u + 3 * i, w, &sel, &mg);
        for (int d = 0; d < 3; ++d) sdir[3 * i + d] = w[d];
        if (slobe) slobe[i] = sel;
    }
}

/* ------------------------------------------------------------------------ */
/* Sec. 4.2: the Monte Carlo KL estimate and its gradient (eq. mcgradients).*/
/* Per sample j with weight w_j = L_j / p_j the surrogate loss term is      */
/* -(w_j / N) log V(w_j); its gradient is -(w_j / N) grad V / V, written in */
/* terms of the raw outputs through the Table 1 mappings.                   */
/* ------------------------------------------------------------------------ */
static double oracle_weight(float rad, float pdf)
{
    if (!isfinite(rad) || !isfinite(pdf) || !(pdf > 0.0f) || !(rad > 0.0f)) return 0.0;
    return (double)rad / (double)pdf;
}

/* Returns the sample's loss contribution -(w/N) log V; fills draw[4K].     */
static double oracle_loss_grad_one(const npmo_net *net, const double *raw, const double w3[3],
                                   double wgt, double invN, double *draw)
{
    int K = net->n_lobes;
    for (int j = 0; j < net->n_out; ++j) draw[j] = 0.0;
    if (wgt == 0.0) return 0.0;
    oracle_lobe lob[NPMO_MAX_LOBES];
    double terms[NPMO_MAX_LOBES];
    oracle_map(net, raw, lob);
    double lv = oracle_logpdf(net, lob, w3, terms);
    double g = -wgt * invN;   /* d loss / d log V */
    for (int k = 0; k < K; ++k) {
        const oracle_lobe *b = &lob[k];
        double r = exp(terms[k] - lv);            /* responsibility lambda_k v_k / V */
        double kap = b->kappa;
        double d = b->mu[0] * w3[0] + b->mu[1] * w3[1] + b->mu[2] * w3[2];
        double dt1 = b->t1[0] * w3[0] + b->t1[1] * w3[1] + b->t1[2] * w3[2];
        double dt2 = b->t2[0] * w3[0] + b->t2[1] * w3[1] + b->t2[2] * w3[2];
        /* d log v / d theta' : kappa (t1.w) pi theta (1 - theta)          */
        double dth = kap * dt1 * PI * b->theta * (1.0 - b->theta);
        /* d log v / d phi'   : kappa sinT (t2.w) 2 pi phi (1 - phi)       */
        double dph = kap * b->sinT * dt2 * 2.0 * PI * b->phi * (1.0 - b->phi);
        /* d log v / d kappa' : kappa (1/kappa - 2/(e^{2k}-1) + mu.w - 1),
         * zero where the clamp of kappa' is active.                         */
        double rk = raw[4 * k + 2];
        double dka = (rk < -80.0 || rk > 80.0) ? 0.0
                   : 1.0 - 2.0 * kap / expm1(2.0 * kap) + kap * (d - 1.0);
        draw[4 * k + 0] = g * r * dth;
        draw[4 * k + 1] = g * r * dph;
        draw[4 * k + 2] = g * r * dka;
        /* d log V / d lambda'_k = r_k - lambda_k (softmax Jacobian)        */
        draw[4 * k + 3] = g * (r - b->lambda);
    }
    return g * lv;
}

/* Learned selection probability (Sec. 6.3): the renderer draws a direction
 * from the BSDF with probability c and from the mixture otherwise, so its
 * one-sample MIS density is p_c(w) = c p_bsdf(w) + (1 - c) V(w).  The KL
 * divergence of Sec. 4.2 from the target D to p_c, estimated with the same
 * samples and weights w_j = D_j / p~_j, gives the loss term
 * -(w_j / N) log p_c(w_j) and
 *   d / dc' = -(w_j / N) c (1 - c) (p_bsdf - V) / p_c,
 * with V held fixed: the mixture keeps its own term, and this one moves
 * only c.  A sample whose BSDF density is not finite and >= 0 (a delta
 * lobe, a missing value) contributes nothing to it.                       */
static double oracle_select_weight(double wgt, float bsdf)
{
    return (isfinite(bsdf) && bsdf >= 0.0f) ? wgt : 0.0;
}

static double softplus(double x) { return x > 0.0 ? x + log1p(exp(-x)) : log1p(exp(x)); }

/* Returns the sample's selection loss term; writes d/dc' to *dsel.         */
static double oracle_select_one(const npmo_net *net, const double *raw, const double w3[3],
                                double wsel, float bsdf, double invN, double *dsel)
{
    *dsel = 0.0;
    if (wsel == 0.0) return 0.0;
    oracle_lobe lob[NPMO_MAX_LOBES];
    oracle_map(net, raw, lob);
    double lv = oracle_logpdf(net, lob, w3, NULL);
    double cp = raw[4 * net->n_lobes];
    double c = 1.0 / (1.0 + exp(-cp));
    double lp = log((double)bsdf);                       /* -inf for p_bsdf = 0 */
    double a = lp - softplus(-cp), b = lv - softplus(cp);  /* log c p_bsdf, log (1-c) V */
    double m = a > b ? a : b;
    double lq = m + log(exp(a - m) + exp(b - m));        /* log p_c */
    double g = -wsel * invN;
    *dsel = g * c * (1.0 - c) * (exp(lp - lq) - exp(lv - lq));
    return g * lq;
}

/* d loss / d raw of one sample: the mixture's term, then the selection
 * output's (when the network has one).                                    */
static double oracle_draw_all(const npmo_net *net, const double *raw, const double w3[3],
                              double wgt, float bsdf, double invN, double *draw, double *lsel)
{
    double l = oracle_loss_grad_one(net, raw, w3, wgt, invN, draw);
    double s = 0.0;
    if (net->select)
        s = oracle_select_one(net, raw, w3, oracle_select_weight(wgt, bsdf), bsdf, invN,
                              &draw[4 * net->n_lobes]);
    if (lsel) *lsel = s;
    return l;
}

/* Condition scale of d loss / d raw for one sample: the first-order bound on
 * the error of an FP32 evaluation, in units of the unit roundoff, from two
 * independent sources, which add:
 *   - rounding inside the head with exact raw outputs: each derivative of
 *     oracle_loss_grad_one with its dot products and differences replaced by
 *     sums of absolute values, times the relative error of the
 *     responsibilities r_k = exp(t_k - log V).  The log term t_k carries
 *     kappa_k (mu_k . w - 1), whose dot product rounds with an error of the
 *     order of the unit roundoff, amplified by kappa_k, and log V carries
 *     the r-weighted mean of those: relative error 1 + kappa_k + sum_j r_j
 *     kappa_j;
 *   - the raw outputs' own rounding (condition rawcond_i from the MLP
 *     forward), carried through the head's Jacobian:
 *     sum_i |d draw_j / d raw_i| rawcond_i, the Jacobian taken by central
 *     differences of oracle_draw_all in FP64.
 * The selection output's head rounding: its few products and the sigmoid
 * (a small multiple of |d draw / dc'|), plus the error of the log-ratio
 * t = log p_bsdf - log V through d draw / dt = g c (1 - c) p_bsdf V / p_c^2;
 * t's error (in units of the roundoff) is |log p_bsdf| + |log V| + |t| plus
 * the r-weighted sizes of the log terms that log V sums.                   */
static void oracle_head_cond(const npmo_net *net, const double *raw, const double *rawcond,
                             const double w3[3], double wgt, float bsdf, double invN,
                             double *cdraw)
{
    int K = net->n_lobes;
    for (int j = 0; j < net->n_out; ++j) cdraw[j] = 0.0;
    if (wgt == 0.0) return;
    oracle_lobe lob[NPMO_MAX_LOBES];
    double terms[NPMO_MAX_LOBES];
    oracle_map(net, raw, lob);
    double lv = oracle_logpdf(net, lob, w3, terms);
    double g = fabs(wgt * invN);
    double rk_sum = 0.0;
    for (int k = 0; k < K; ++k) rk_sum += exp(terms[k] - lv) * lob[k].kappa;
    for (int k = 0; k < K; ++k) {
        const oracle_lobe *b = &lob[k];
        double r = exp(terms[k] - lv), kap = b->kappa;
        double a1 = 0.0, a2 = 0.0, am = 0.0;
        for (int d = 0; d < 3; ++d) {
            a1 += fabs(b->t1[d] * w3[d]);
            a2 += fabs(b->t2[d] * w3[d]);
            am += fabs(b->mu[d] * w3[d]);
        }
        double resp = 1.0 + kap + rk_sum;
        cdraw[4 * k + 0] = g * r * kap * PI * b->theta * (1.0 - b->theta) * a1 * resp;
        cdraw[4 * k + 1] = g * r * kap * b->sinT * 2.0 * PI * b->phi * (1.0 - b->phi) * a2 * resp;
        cdraw[4 * k + 2] = g * r * (1.0 + 2.0 * kap / expm1(2.0 * kap) + kap * (am + 1.0)) * resp;
        cdraw[4 * k + 3] = g * (r + b->lambda) * resp;
    }
    double wsel = net->select ? oracle_select_weight(wgt, bsdf) : 0.0;
    if (wsel != 0.0) {
        double cp = raw[4 * K], c = 1.0 / (1.0 + exp(-cp)), dsel;
        oracle_select_one(net, raw, w3, wsel, bsdf, invN, &dsel);
        double tsum = 4.0 + fabs(lv);
        for (int k = 0; k < K; ++k) {
            double d = lob[k].mu[0] * w3[0] + lob[k].mu[1] * w3[1] + lob[k].mu[2] * w3[2];
            tsum += exp(terms[k] - lv) * (fabs(lob[k].loglambda) +
                                          fabs(log_vmf_norm(lob[k].kappa)) +
                                          lob[k].kappa * (fabs(d) + 1.0));
        }
        double tterm = 0.0;
        if (bsdf > 0.0f) {
            double lp = log((double)bsdf);
            double a = lp - softplus(-cp), b = lv - softplus(cp), m = a > b ? a : b;
            double lq = m + log(exp(a - m) + exp(b - m));
            tterm = fabs(wsel * invN) * c * (1.0 - c) * exp(lp + lv - 2.0 * lq) *
                    (tsum + fabs(lp) + fabs(lp - lv));
        }
        cdraw[4 * K] = 8.0 * fabs(dsel) + tterm;
    }
    double rp[NPMO_MAX_OUT], dp[NPMO_MAX_OUT], dm[NPMO_MAX_OUT];
    for (int i = 0; i < net->n_out; ++i) {
        if (rawcond[i] == 0.0) continue;
        double h = 1e-5 * (fabs(raw[i]) > 1.0 ? fabs(raw[i]) : 1.0);
        for (int j = 0; j < net->n_out; ++j) rp[j] = raw[j];
        rp[i] = raw[i] + h;
        oracle_draw_all(net, rp, w3, wgt, bsdf, invN, dp, NULL);
        rp[i] = raw[i] - h;
        oracle_draw_all(net, rp, w3, wgt, bsdf, invN, dm, NULL);
        for (int j = 0; j < net->n_out; ++j)
            cdraw[j] += fabs(dp[j] - dm[j]) / (2.0 * h) * rawcond[i];
    }
}

double npmo_loss_grad(const npmo_net *net, int64_t n, int64_t n_total, const double *raw,
                      const float *dir /* [3][n] */, const float *rad, const float *spdf,
                      const float *bsdf /* [n] or NULL */, double *draw /* [n][n_out] */,
                      double *loss_sel /* or NULL */)
{
    double invN = 1.0 / (double)n_total, loss = 0.0, lsel = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        double w3[3] = {dir[i], dir[n + i], dir[2 * n + i]}, ls;
        loss += oracle_draw_all(net, raw + i * net->n_out, w3, oracle_weight(rad[i], spdf[i]),
                                bsdf ? bsdf[i] : NAN, invN, draw + i * net->n_out, &ls);
        lsel += ls;
    }
    if (loss_sel) *loss_sel = lsel;
    return loss;
}

/* ------------------------------------------------------------------------ */
/* Backpropagation (Fig. 2, dashed path): through the MLP into dG, then the */
/* scatter of dG into the eight corners of every level (the transpose of    */
/* the interpolation), with the encoding recomputed per vertex.  grad and   */
/* gabs accumulate; gabs receives the sum of |contributions| per parameter. */
/* ------------------------------------------------------------------------ */
/* Condition scales of the gradient (gcond, accumulated): the head seed of
 * oracle_head_cond carried back through the layers alongside the values:
 * cond(dz) = cond(dh) where z > 0; cond(dh_k) = sum_o |W_ok| cond(dz_o);
 * cond(dW_ok) += cond(dz_o) |h_k| + |dz_o| cond(h_k); the grid entry of a
 * corner gets w_c cond(dG).                                               */
static void oracle_backward_cond_one(const npmo_net *net, const float *pos3, const float *aux7,
                                     const double w3[3], double wgt, float bsdf, double invN,
                                     const double *params, double *gcond)
{
    int L = net->n_levels, F = net->feat;
    double G[NPMO_MAX_WIDTH], Gc[NPMO_MAX_WIDTH], raw[NPMO_MAX_OUT], rawc[NPMO_MAX_OUT];
    double draw[NPMO_MAX_OUT], cdraw[NPMO_MAX_OUT];
    double acts[NPMO_MAX_LAYERS][NPMO_MAX_WIDTH], cacts[NPMO_MAX_LAYERS][NPMO_MAX_WIDTH];
    unsigned char amb[NPMO_MAX_LAYERS][NPMO_MAX_WIDTH];
    double delta[NPMO_MAX_WIDTH], cdelta[NPMO_MAX_WIDTH], prev[NPMO_MAX_WIDTH], cprev[NPMO_MAX_WIDTH];
    int64_t idx[NPMO_MAX_LEVELS * 8];
    double cw[NPMO_MAX_LEVELS * 8];
    if (wgt == 0.0) return;
    oracle_encode_one(net, pos3[0], pos3[1], pos3[2], params, G, Gc);
    oracle_aux_one(net, aux7, G, Gc);
    oracle_mlp_cond_one(net, G, Gc, params, acts, cacts, amb, raw, rawc);
    oracle_draw_all(net, raw, w3, wgt, bsdf, invN, draw, NULL);
    oracle_head_cond(net, raw, rawc, w3, wgt, bsdf, invN, cdraw);
    for (int j = 0; j < net->n_out; ++j) { delta[j] = draw[j]; cdelta[j] = cdraw[j]; }
    for (int li = net->n_layers - 1; li >= 0; --li) {
        const double *W = params + net->layer_offset[li];
        double *cW = gcond + net->layer_offset[li];
        int nin = net->layer_in[li], nout = net->layer_out[li];
        if (li < net->n_layers - 1)
            for (int o = 0; o < nout; ++o) {
                /* a unit at an undetermined kink: the other choice of the
                 * ReLU derivative moves dz by |dh| (2^24 |dh| in units of
                 * the roundoff)                                          */
                if (amb[li + 1][o]) cdelta[o] += 16777216.0 * fabs(delta[o]);
                else if (!(acts[li + 1][o] > 0.0)) cdelta[o] = 0.0;
                if (!(acts[li + 1][o] > 0.0)) delta[o] = 0.0;
            }
        for (int o = 0; o < nout; ++o)
            for (int k = 0; k < nin; ++k)
                cW[(int64_t)o * nin + k] += cdelta[o] * fabs(acts[li][k]) + fabs(delta[o]) * cacts[li][k];
        for (int k = 0; k < nin; ++k) {
            double sv = 0.0, sc = 0.0;
            for (int o = 0; o < nout; ++o) {
                sv += W[(int64_t)o * nin + k] * delta[o];
                sc += fabs(W[(int64_t)o * nin + k]) * cdelta[o];
            }
            prev[k] = sv; cprev[k] = sc;
        }
        for (int k = 0; k < nin; ++k) { delta[k] = prev[k]; cdelta[k] = cprev[k]; }
    }
    oracle_corners_one(net, pos3[0], pos3[1], pos3[2], idx, cw);
    for (int l = 0; l < L; ++l)
        for (int b = 0; b < 8; ++b)
            for (int f = 0; f < F; ++f)
                gcond[idx[l * 8 + b] * F + f] += cw[l * 8 + b] * cdelta[l * F + f];
}

/* The vertex loops of the backward run over contiguous ranges, one per
 * thread; each thread adds into its own zeroed copy of the m accumulated
 * arrays (thread 0 into the caller's), and the copies are then added to the
 * caller's in thread order, so the sums do not depend on scheduling.  A copy
 * costs time in proportion to the np parameters and a vertex a fixed amount
 * of work (measured: about 4,000 times a parameter's share of allocating,
 * zeroing and adding), so the batch takes about sqrt(4,000 n / (m np))
 * threads, at least 256 vertices each, at most the OpenMP maximum.        */
static int oracle_threads(int64_t n, int64_t np, int m)
{
    int64_t t = omp_get_max_threads();
    if (t > n / 256) t = n / 256;
    const double s = sqrt(4000.0 * (double)n / ((double)m * (double)(np > 0 ? np : 1)));
    if ((double)t > s) t = (int64_t)s;
    return t < 1 ? 1 : (int)t;
}

/* buf holds (T - 1) copies of each of the m accumulated arrays acc[0..m). */
static void oracle_add_copies(int T, int m, double *const *acc, const double *buf, int64_t np)
{
    for (int a = 0; a < m; ++a) {
        const double *b = buf + (size_t)a * (T - 1) * np;
        double *d = acc[a];
#pragma omp parallel for schedule(static)
        for (int64_t k = 0; k < np; ++k) {
            double v = d[k];
            for (int t = 1; t < T; ++t) v += b[(size_t)(t - 1) * np + k];
            d[k] = v;
        }
    }
}

void npmo_backward_cond(const npmo_net *net, int64_t n, int64_t n_total, const float *pos,
                        const float *aux /* [7][n] or NULL */, const float *dir, const float *rad,
                        const float *spdf, const float *bsdf /* [n] or NULL */,
                        const double *params,
                        double *gcond /* [n_params], accumulated */)
{
    double invN = 1.0 / (double)n_total;
    int64_t np = net->n_params;
    int T = oracle_threads(n, np, 1);
    double *buf = T > 1 ? calloc((size_t)(T - 1) * np, sizeof(double)) : NULL;
    if (!buf) T = 1;
#pragma omp parallel num_threads(T)
    {
        int t = omp_get_thread_num();
        double *gc = t == 0 ? gcond : buf + (size_t)(t - 1) * np;
        for (int64_t i = n * t / T; i < n * (t + 1) / T; ++i) {
            float p3[3] = {pos[i], pos[n + i], pos[2 * n + i]}, a7[7];
            double w3[3] = {dir[i], dir[n + i], dir[2 * n + i]};
            oracle_aux_fetch(aux, n, i, a7);
            oracle_backward_cond_one(net, p3, a7, w3, oracle_weight(rad[i], spdf[i]),
                                     bsdf ? bsdf[i] : NAN, invN, params, gc);
        }
    }
    if (T > 1) {
        double *acc[1] = {gcond};
        oracle_add_copies(T, 1, acc, buf, np);
    }
    free(buf);
}

/* One vertex of the backward: returns its loss term, adds its gradient
 * contributions (and their magnitudes) into grad (gabs). */
static double oracle_backward_one(const npmo_net *net, int64_t n, int64_t i, const float *pos,
                                  const float *aux, const float *dir, const float *rad,
                                  const float *spdf, const float *bsdf, const double *params,
                                  double invN, double *grad, double *gabs, double *draw_out,
                                  double *dG_out, double *lsel)
{
    int L = net->n_levels, F = net->feat;
    double G[NPMO_MAX_WIDTH], raw[NPMO_MAX_OUT], draw[NPMO_MAX_OUT];
    double acts[NPMO_MAX_LAYERS][NPMO_MAX_WIDTH];
    double delta[NPMO_MAX_WIDTH], prev[NPMO_MAX_WIDTH];
    int64_t idx[NPMO_MAX_LEVELS * 8];
    double cw[NPMO_MAX_LEVELS * 8];
    float px = pos[i], py = pos[n + i], pz = pos[2 * n + i], a7[7];
    oracle_aux_fetch(aux, n, i, a7);
    oracle_encode_one(net, px, py, pz, params, G, NULL);
    oracle_aux_one(net, a7, G, NULL);
    oracle_mlp_one(net, G, params, acts, raw, NULL);
    double w3[3] = {dir[i], dir[n + i], dir[2 * n + i]};
    double loss = oracle_draw_all(net, raw, w3, oracle_weight(rad[i], spdf[i]),
                                  bsdf ? bsdf[i] : NAN, invN, draw, lsel);
    if (draw_out) for (int j = 0; j < net->n_out; ++j) draw_out[i * net->n_out + j] = draw[j];
    /* delta holds dLoss/d(output of layer i), i from last to first.        */
    for (int j = 0; j < net->n_out; ++j) delta[j] = draw[j];
    for (int li = net->n_layers - 1; li >= 0; --li) {
        const double *W = params + net->layer_offset[li];
        double *dW = grad + net->layer_offset[li];
        double *aW = gabs ? gabs + net->layer_offset[li] : NULL;
        int nin = net->layer_in[li], nout = net->layer_out[li];
        /* hidden layer outputs pass through ReLU: derivative 0 at 0         */
        if (li < net->n_layers - 1)
            for (int o = 0; o < nout; ++o) if (!(acts[li + 1][o] > 0.0)) delta[o] = 0.0;
        for (int o = 0; o < nout; ++o)
            for (int k = 0; k < nin; ++k) {
                double t = delta[o] * acts[li][k];
                dW[(int64_t)o * nin + k] += t;
                if (aW) aW[(int64_t)o * nin + k] += fabs(t);
            }
        for (int k = 0; k < nin; ++k) {
            double s = 0.0;
            for (int o = 0; o < nout; ++o) s += W[(int64_t)o * nin + k] * delta[o];
            prev[k] = s;
        }
        for (int k = 0; k < nin; ++k) delta[k] = prev[k];
    }
    if (dG_out) for (int j = 0; j < net->n_in; ++j) dG_out[i * net->n_in + j] = delta[j];
    oracle_corners_one(net, px, py, pz, idx, cw);
    for (int l = 0; l < L; ++l)
        for (int b = 0; b < 8; ++b)
            for (int f = 0; f < F; ++f) {
                double t = cw[l * 8 + b] * delta[l * F + f];
                grad[idx[l * 8 + b] * F + f] += t;
                if (gabs) gabs[idx[l * 8 + b] * F + f] += fabs(t);
            }
    return loss;
}

double npmo_backward(const npmo_net *net, int64_t n, int64_t n_total, const float *pos,
                     const float *aux /* [7][n] or NULL */, const float *dir, const float *rad,
                     const float *spdf, const float *bsdf /* [n] or NULL */, const double *params,
                     double *grad /* [n_params] */, double *gabs /* [n_params] or NULL */,
                     double *draw_out /* [n][n_out] or NULL */,
                     double *dG_out /* [n][n_in] or NULL */, double *loss_sel /* or NULL */)
{
    double invN = 1.0 / (double)n_total;
    int64_t np = net->n_params;
    int m = gabs ? 2 : 1;
    int T = oracle_threads(n, np, m);
    double tloss[256], tsel[256];
    if (T > 256) T = 256;
    double *buf = T > 1 ? calloc((size_t)m * (T - 1) * np, sizeof(double)) : NULL;
    if (!buf) T = 1;
#pragma omp parallel num_threads(T)
    {
        int t = omp_get_thread_num();
        double *g = t == 0 ? grad : buf + (size_t)(t - 1) * np;
        double *a = !gabs ? NULL : (t == 0 ? gabs : buf + (size_t)(T - 1 + t - 1) * np);
        double l = 0.0, ls = 0.0, s;
        for (int64_t i = n * t / T; i < n * (t + 1) / T; ++i) {
            l += oracle_backward_one(net, n, i, pos, aux, dir, rad, spdf, bsdf, params, invN, g,
                                     a, draw_out, dG_out, &s);
            ls += s;
        }
        tloss[t] = l;
        tsel[t] = ls;
    }
    double loss = 0.0, lsel = 0.0;
    for (int t = 0; t < T; ++t) { loss += tloss[t]; lsel += tsel[t]; }
    if (loss_sel) *loss_sel = lsel;
    if (T > 1) {
        double *acc[2] = {grad, gabs};
        oracle_add_copies(T, m, acc, buf, np);
    }
    free(buf);
    return loss;
}

/* ------------------------------------------------------------------------ */
/* Adam (Kingma and Ba), as the paper trains with it at a fixed rate.        */
/* t is the 1-based step number of this update.                             */
/* ------------------------------------------------------------------------ */
void npmo_adam(int64_t np, double *params, const double *grad, double *m, double *v, int64_t t,
               double lr, double beta1, double beta2, double eps)
{
    double c1 = 1.0 - pow(beta1, (double)t), c2 = 1.0 - pow(beta2, (double)t);
    for (int64_t i = 0; i < np; ++i) {
        double g = grad[i];
        m[i] = beta1 * m[i] + (1.0 - beta1) * g;
        v[i] = beta2 * v[i] + (1.0 - beta2) * g * g;
        double mh = m[i] / c1, vh = v[i] / c2;
        params[i] -= lr * mh / (sqrt(vh) + eps);
    }
}

/* ------------------------------------------------------------------------ */
/* Exponential moving average of the weights (Sec. 5.3: inference uses an    */
/* EMA of the weights of previous training steps).  Called after each        */
/* optimizer step with that step's parameters: ema <- d ema + (1 - d) p.     */
/* ------------------------------------------------------------------------ */
void npmo_ema(int64_t np, double *ema, const double *params, double decay)
{
    for (int64_t i = 0; i < np; ++i) ema[i] = decay * ema[i] + (1.0 - decay) * params[i];
}

/* Threads npmo_backward runs a batch of n vertices on (with_abs: also the
 * magnitudes), and npmo_backward_cond (with_abs = 0).                     */
int npmo_backward_threads(const npmo_net *net, int64_t n, int with_abs)
{
    int T = oracle_threads(n, net->n_params, with_abs ? 2 : 1);
    return T > 256 ? 256 : T;
}

/* Thread count of the OpenMP loops (timing of the oracle on one core);
 * returns the previous maximum.                                            */
int npmo_set_threads(int n)
{
    int old = omp_get_max_threads();
    if (n > 0) omp_set_num_threads(n);
    return old;
}
