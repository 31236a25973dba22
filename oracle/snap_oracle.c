/*
 * SNAP-tFDP CPU oracle -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, obviously-correct FP64 implementation of the edge-centric
 * negative-sampling layout (Algorithm 1 of the paper, forces of Table 1,
 * t-FDP row).  Only the test suite, the smoke check and the CPU-baseline leg of
 * the benchmark may load this library.  It shares no code with the HIP path:
 * the counter-based generator (Philox4x64-10, Salmon et al., SC'11), Lemire's
 * multiply-shift range reduction (ACM TOMACS 2019) and the alias-table sweep
 * (Walker; Vose; Huebschle-Schneider & Sanders) are written here from their
 * published definitions, independently of the device code.
 *
 * Conventions fixed where the paper is silent (each listed in the design notes):
 *   - forces act physically: attraction pulls the pair together, repulsion
 *     pushes it apart (Sec. 3.1: adjacent vertices are drawn together, all
 *     vertices repel).  With d = y_i - y_o and q = |d|^2:
 *         A(d) = alpha * (1 + beta / (1 + q)) * d            (Table 1, t-FDP)
 *         R(d) = d / (1 + q)^gamma                            (Table 1, t-FDP)
 *     edge (i,j):   y_i -= eta*A(y_i - y_j);  y_j += eta*A(y_i - y_j)
 *     negative s:   y_i += eta*R(y_i - y_s);  y_s -= eta*R(y_i - y_s)
 *   - eta_t = eta0 * (1 - t/T), t = 0..T-1 ("decaying over epochs", Sec. 3.3).
 *   - negatives are i.i.d. uniform over V \ {i} (Algorithm 1, Sec. 3.3); the
 *     degree-weighted alias variant is a control, not the paper's method.
 *   - every random number is a pure function of (seed, purpose, indices), so
 *     the order in which edges are processed never changes which samples are
 *     drawn.
 *
 * Random-number layout (identical definition on both sides, separate code):
 *   key     = (seed, KEY_DOMAIN)
 *   counter = (a, b, c, tag)    tag: 1 init, 2 negatives, 3 edge shuffle
 *   one Philox block gives four u64 x0..x3 = eight u32 words
 *       w[2q] = lo32(x_q), w[2q+1] = hi32(x_q)
 *   init of node i:     counter (i, 0, 0, 1); coordinate c (< dim) from x_c:
 *                       v = (int)(x_c >> 40) - 2^23, y = (float)v * 2^-23 * s,
 *                       s = sqrtf((float)n) (FP32, one rounding)
 *   negatives of edge e in epoch t: word stream of blocks (e, t, b, 2), b=0,1,..
 *     UNIFORM: per attempt one word u; p = u*(n-1) (64-bit); reject when
 *              lo32(p) < 2^32 mod (n-1); else s' = hi32(p), s = s' + (s' >= i)
 *     DEGREE:  per attempt two words (u1,u2); p = u1*n; reject when
 *              lo32(p) < 2^32 mod n; c = hi32(p); s = u2 < thr[c] ? c : alias[c];
 *              reject when s == i
 *     after 64 rejected attempts s = (i+1) mod n (probability < 2^-64).
 */
#define _GNU_SOURCE
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define KEY_DOMAIN 0x534E41502D744644ULL /* "SNAP-tFD" */
#define TAG_INIT 1ULL
#define TAG_NEG 2ULL
#define TAG_PERM 3ULL
#define MAX_ATTEMPTS 64

enum { NEG_UNIFORM = 0, NEG_DEGREE = 1 };
enum { ORDER_SHUFFLED = 0, ORDER_CSR = 1 };

/* ---------------------------------------------------------------- Philox */
/* Philox4x64-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy
 * as 1, 2, 3", SC'11): ten rounds of two 64x64->128 multiplies, key bumped by
 * the Weyl constants between rounds. */
static const uint64_t PH_M0 = 0xD2E7470EE14C6C93ULL;
static const uint64_t PH_M1 = 0xCA5A826395121157ULL;
static const uint64_t PH_W0 = 0x9E3779B97F4A7C15ULL;
static const uint64_t PH_W1 = 0xBB67AE8584CAA73BULL;

void oracle_philox4x64(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4])
{
    uint64_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint64_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += PH_W0;
            k1 += PH_W1;
        }
        unsigned __int128 p0 = (unsigned __int128)PH_M0 * x0;
        unsigned __int128 p1 = (unsigned __int128)PH_M1 * x2;
        uint64_t hi0 = (uint64_t)(p0 >> 64), lo0 = (uint64_t)p0;
        uint64_t hi1 = (uint64_t)(p1 >> 64), lo1 = (uint64_t)p1;
        uint64_t n0 = hi1 ^ x1 ^ k0;
        uint64_t n1 = lo1;
        uint64_t n2 = hi0 ^ x3 ^ k1;
        uint64_t n3 = lo0;
        x0 = n0; x1 = n1; x2 = n2; x3 = n3;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* Bulk form used by the generator pin: out[4*r + q] = Philox(ctr0 + r, ...). */
void oracle_philox_bulk(uint64_t k0, uint64_t k1, uint64_t c0, uint64_t c1, uint64_t c2,
                        uint64_t c3, int64_t count, uint64_t *out)
{
    uint64_t key[2] = {k0, k1};
    for (int64_t r = 0; r < count; ++r) {
        uint64_t ctr[4] = {c0 + (uint64_t)r, c1, c2, c3};
        oracle_philox4x64(ctr, key, out + 4 * r);
    }
}

/* The u32 word stream of one (a, b, tag) counter family. */
typedef struct {
    uint64_t key[2];
    uint64_t a, b, tag;
    uint64_t block_index; /* which block is cached in x[] */
    uint64_t x[4];
    int64_t next; /* index of the next word to hand out */
} word_stream;

static void ws_open(word_stream *ws, uint64_t seed, uint64_t a, uint64_t b, uint64_t tag)
{
    ws->key[0] = seed;
    ws->key[1] = KEY_DOMAIN;
    ws->a = a;
    ws->b = b;
    ws->tag = tag;
    ws->block_index = UINT64_MAX;
    ws->next = 0;
}

static uint32_t ws_word(word_stream *ws)
{
    uint64_t blk = (uint64_t)ws->next / 8;
    int within = (int)(ws->next % 8);
    if (blk != ws->block_index) {
        uint64_t ctr[4] = {ws->a, ws->b, blk, ws->tag};
        oracle_philox4x64(ctr, ws->key, ws->x);
        ws->block_index = blk;
    }
    ws->next++;
    uint64_t x = ws->x[within / 2];
    return (within % 2 == 0) ? (uint32_t)x : (uint32_t)(x >> 32);
}

/* ------------------------------------------------------------ init layout */
/* Uniform positions in [-scale, scale]^dim (dim 2 or 3) for nodes [0, n),
 * produced in FP32 (one rounding) and widened exactly to FP64; Y is n*dim. */
void oracle_init_positions_dim(int64_t n, uint64_t seed, float s, int32_t dim, double *Y)
{
    uint64_t key[2] = {seed, KEY_DOMAIN};
    for (int64_t i = 0; i < n; ++i) {
        uint64_t ctr[4] = {(uint64_t)i, 0, 0, TAG_INIT};
        uint64_t x[4];
        oracle_philox4x64(ctr, key, x);
        for (int c = 0; c < dim; ++c) {
            int32_t v = (int32_t)(x[c] >> 40) - (1 << 23);
            float unit = (float)v * 0x1p-23f; /* exact: 24-bit integer times 2^-23 */
            float coord = unit * s;           /* the only rounding */
            Y[dim * i + c] = (double)coord;
        }
    }
}

/* Uniform positions in [-scale, scale]^2. */
void oracle_init_positions_scaled(int64_t n, uint64_t seed, float s, double *Y)
{
    oracle_init_positions_dim(n, seed, s, 2, Y);
}

/* The initial layout: uniform in [-sqrt(n), sqrt(n)]^2. */
void oracle_init_positions(int64_t n, uint64_t seed, double *Y)
{
    oracle_init_positions_scaled(n, seed, sqrtf((float)n), Y);
}

/* The initial positions of listed nodes of an n-node graph only:
 * Y[2q], Y[2q+1] for node nodes[q]. */
void oracle_init_positions_at(int64_t n, uint64_t seed, const int64_t *nodes, int64_t count,
                              double *Y)
{
    float s = sqrtf((float)n);
    uint64_t key[2] = {seed, KEY_DOMAIN};
    for (int64_t q = 0; q < count; ++q) {
        uint64_t ctr[4] = {(uint64_t)nodes[q], 0, 0, TAG_INIT};
        uint64_t x[4];
        oracle_philox4x64(ctr, key, x);
        for (int c = 0; c < 2; ++c) {
            int32_t v = (int32_t)(x[c] >> 40) - (1 << 23);
            float unit = (float)v * 0x1p-23f; /* exact */
            Y[2 * q + c] = (double)(unit * s);
        }
    }
}

/* -------------------------------------------------------------- alias table */
/* Integer alias table for weights w[0..n) (Walker/Vose), built by a
 * deterministic sequential sweep.  Item s has mass M_s = w_s * n against a bin
 * capacity W = sum(w).  Lights (M < W) are visited in index order; each takes
 * its deficit W - M from the current heavy (heavies in index order).  A heavy
 * whose residual r drops below W becomes a partial bin: thr = r, alias = next
 * heavy, and the next heavy absorbs the deficit W - r.  Thresholds are stored
 * as floor(own_mass * 2^32 / W); a full bin stores 0xFFFFFFFF and aliases
 * itself.  Returns 0, or -1 when W == 0 or W >= 2^32 or some M overflows. */
int oracle_alias_build(const int64_t *w, int64_t n, uint32_t *thr, uint32_t *alias)
{
    int64_t W = 0;
    for (int64_t s = 0; s < n; ++s) {
        if (w[s] < 0) return -1;
        W += w[s];
    }
    if (W <= 0 || W >= (1LL << 32)) return -1;
    for (int64_t s = 0; s < n; ++s) {
        thr[s] = 0xFFFFFFFFu;
        alias[s] = (uint32_t)s;
    }
    /* heavies in index order */
    int64_t *heavy = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    int64_t nh = 0;
    for (int64_t s = 0; s < n; ++s)
        if (w[s] * n >= W) heavy[nh++] = s;
    int64_t h = 0;                            /* current heavy */
    __int128 r = nh > 0 ? (__int128)w[heavy[0]] * n : 0; /* its residual mass */
    for (int64_t s = 0; s < n; ++s) {
        __int128 M = (__int128)w[s] * n;
        if (M >= W) continue; /* heavies are handled when they run out */
        /* light bin s: own mass M, the deficit comes from the current heavy */
        thr[s] = (uint32_t)(((unsigned __int128)M << 32) / (unsigned __int128)W);
        alias[s] = (uint32_t)heavy[h];
        r -= (W - M);
        /* the current heavy (and possibly a chain of followers) may now be
         * short of a full bin */
        while (r < W && h + 1 < nh) {
            int64_t cur = heavy[h];
            thr[cur] = (uint32_t)(((unsigned __int128)r << 32) / (unsigned __int128)W);
            alias[cur] = (uint32_t)heavy[h + 1];
            __int128 deficit = W - r;
            h += 1;
            r = (__int128)w[heavy[h]] * n - deficit;
        }
    }
    free(heavy);
    return 0;
}

/* ----------------------------------------------------------------- sampler */
typedef struct {
    int32_t n;
    int32_t mode;
    const uint32_t *thr;
    const uint32_t *alias;
} sampler;

/* Draws the k negatives of directed edge e (source i) in epoch t, following
 * the word-stream definition in the header comment. */
static void draw_negatives(const sampler *sp, uint64_t seed, int64_t e, int64_t t, int32_t i,
                           int32_t k, int32_t *out)
{
    word_stream ws;
    ws_open(&ws, seed, (uint64_t)e, (uint64_t)t, TAG_NEG);
    uint32_t n = (uint32_t)sp->n;
    for (int32_t m = 0; m < k; ++m) {
        int32_t s = -1;
        for (int attempt = 0; attempt < MAX_ATTEMPTS && s < 0; ++attempt) {
            if (sp->mode == NEG_UNIFORM) {
                uint32_t range = n - 1;
                uint32_t reject_below = (uint32_t)((1ULL << 32) % range);
                uint32_t u = ws_word(&ws);
                uint64_t p = (uint64_t)u * range;
                if ((uint32_t)p < reject_below) continue;
                uint32_t sp_ = (uint32_t)(p >> 32);
                s = (int32_t)(sp_ + (sp_ >= (uint32_t)i ? 1u : 0u));
            } else {
                uint32_t reject_below = (uint32_t)((1ULL << 32) % n);
                uint32_t u1 = ws_word(&ws);
                uint32_t u2 = ws_word(&ws);
                uint64_t p = (uint64_t)u1 * n;
                if ((uint32_t)p < reject_below) continue;
                uint32_t c = (uint32_t)(p >> 32);
                uint32_t cand = (u2 < sp->thr[c]) ? c : sp->alias[c];
                if ((int32_t)cand == i) continue;
                s = (int32_t)cand;
            }
        }
        if (s < 0) s = (int32_t)(((uint32_t)i + 1u) % n);
        out[m] = s;
    }
}

/* All negatives of epoch t, out[e*k + m]. */
int oracle_draw_negatives(const int32_t *row_ptr, const int32_t *col, int32_t n, int32_t k,
                          int64_t t, uint64_t seed, int32_t mode, const uint32_t *thr,
                          const uint32_t *alias, int32_t *out)
{
    (void)col;
    sampler sp = {n, mode, thr, alias};
    for (int32_t i = 0; i < n; ++i)
        for (int64_t e = row_ptr[i]; e < row_ptr[i + 1]; ++e)
            draw_negatives(&sp, seed, e, t, i, k, out + e * k);
    return 0;
}

/* The negatives of listed directed edges only: edge edges[q] with source
 * src[q] (the row holding it), out[q*k .. q*k+k).  For graphs too large to
 * draw every edge on the host. */
int oracle_draw_edges(int32_t n, int32_t k, int64_t t, uint64_t seed, int32_t mode,
                      const uint32_t *thr, const uint32_t *alias, const int64_t *edges,
                      const int32_t *src, int64_t count, int32_t *out)
{
    sampler sp = {n, mode, thr, alias};
    for (int64_t q = 0; q < count; ++q)
        draw_negatives(&sp, seed, edges[q], t, src[q], k, out + q * k);
    return 0;
}

/* ------------------------------------------------------------------ forces */
/* Kernel of the forces.  FORCE_T is Table 1's t-FDP row, built on the
 * Student-t kernel 1/(1+q).  FORCE_GAUSSIAN is the Gaussian-based variant the
 * conclusion names as future work without defining it; the reading taken
 * keeps the t-FDP structure and puts the Gaussian kernel exp(-q/2) in place of
 * 1/(1+q) in both forces:
 *   A(d) = alpha * (1 + beta * exp(-q/2)) * d,   R(d) = exp(-gamma*q/2) * d. */
enum { FORCE_T = 0, FORCE_GAUSSIAN = 1 };

/* The kernel used by every following call (set by the Python wrapper before
 * each call). */
static int32_t g_force_kernel = FORCE_T;

void oracle_set_force_kernel(int32_t kernel) { g_force_kernel = kernel; }

typedef struct {
    double alpha, beta, gamma, eta0;
    int32_t kernel;
} force_params;

/* attraction coefficient: A(d) = coef * d (Table 1, t-FDP attractive force) */
static double attr_coef(const force_params *fp, double q)
{
    if (fp->kernel == FORCE_GAUSSIAN) return fp->alpha * (1.0 + fp->beta * exp(-0.5 * q));
    return fp->alpha * (1.0 + fp->beta / (1.0 + q));
}

/* repulsion coefficient: R(d) = coef * d (Table 1, t-FDP repulsive force) */
static double rep_coef(const force_params *fp, double q)
{
    if (fp->kernel == FORCE_GAUSSIAN) return exp(-0.5 * fp->gamma * q);
    return pow(1.0 + q, -fp->gamma);
}

/* Magnitudes |A| and |R| at distance dist, for the closed-form pins. */
void oracle_force_magnitudes(double alpha, double beta, double gamma, double dist, double *fa,
                             double *fr)
{
    force_params fp = {alpha, beta, gamma, 1.0, g_force_kernel};
    double q = dist * dist;
    *fa = attr_coef(&fp, q) * dist;
    *fr = rep_coef(&fp, q) * dist;
}

static double eta_at(const force_params *fp, int64_t t, int64_t T)
{
    return fp->eta0 * (1.0 - (double)t / (double)T);
}

/* --------------------------------------------------------------- serial run */
typedef struct {
    uint64_t key;
    int64_t e;
} perm_item;

static int perm_cmp(const void *a, const void *b)
{
    const perm_item *x = (const perm_item *)a, *y = (const perm_item *)b;
    if (x->key != y->key) return x->key < y->key ? -1 : 1;
    return x->e < y->e ? -1 : (x->e > y->e ? 1 : 0);
}

static int32_t *sources_of(const int32_t *row_ptr, int32_t n)
{
    int64_t nnz = row_ptr[n];
    int32_t *src = (int32_t *)malloc(sizeof(int32_t) * (size_t)(nnz > 0 ? nnz : 1));
    for (int32_t i = 0; i < n; ++i)
        for (int64_t e = row_ptr[i]; e < row_ptr[i + 1]; ++e) src[e] = i;
    return src;
}

/* One stochastic pair step on two points of Y (in place), dim coordinates
 * each; q sums the squared differences over all coordinates. */
static void attract_pair(const force_params *fp, double eta, int dim, double *yi, double *yj)
{
    double d[3], q = 0.0;
    for (int c = 0; c < dim; ++c) {
        d[c] = yi[c] - yj[c];
        q += d[c] * d[c];
    }
    double coef = eta * attr_coef(fp, q);
    for (int c = 0; c < dim; ++c) {
        yi[c] -= coef * d[c];
        yj[c] += coef * d[c];
    }
}

static void repel_pair(const force_params *fp, double eta, int dim, double *yi, double *ys)
{
    double d[3], q = 0.0;
    for (int c = 0; c < dim; ++c) {
        d[c] = yi[c] - ys[c];
        q += d[c] * d[c];
    }
    double coef = eta * rep_coef(fp, q);
    for (int c = 0; c < dim; ++c) {
        yi[c] += coef * d[c];
        ys[c] -= coef * d[c];
    }
}

/* The epochs [t_begin, t_end) of serial Algorithm 1, visiting the directed
 * edges in the order perm[0..nnz): attraction along the edge, then the k
 * negatives one after another, every pair force taken from the current
 * positions and applied at once (Sec. 3.3, "immediate updates"). */
static void serial_epochs(const int32_t *row_ptr, const int32_t *col, int32_t n, int32_t k,
                          int64_t t_begin, int64_t t_end, int64_t T, uint64_t seed,
                          const force_params *fp, const sampler *sp, int32_t dim,
                          const int64_t *perm, double *Y)
{
    int64_t nnz = row_ptr[n];
    int32_t *src = sources_of(row_ptr, n);
    int32_t *neg = (int32_t *)malloc(sizeof(int32_t) * (size_t)(k > 0 ? k : 1));
    for (int64_t t = t_begin; t < t_end; ++t) {
        double eta = eta_at(fp, t, T);
        for (int64_t p = 0; p < nnz; ++p) {
            int64_t e = perm[p];
            int32_t i = src[e], j = col[e];
            attract_pair(fp, eta, dim, Y + (int64_t)dim * i, Y + (int64_t)dim * j);
            draw_negatives(sp, seed, e, t, i, k, neg);
            for (int32_t m = 0; m < k; ++m)
                repel_pair(fp, eta, dim, Y + (int64_t)dim * i, Y + (int64_t)dim * neg[m]);
        }
    }
    free(neg);
    free(src);
}

/* Serial Algorithm 1 in FP64 over epochs [t_begin, t_end) of a T-epoch
 * schedule.  order = ORDER_SHUFFLED: the directed edges are shuffled once
 * (Algorithm 1, first step) by a seeded permutation; ORDER_CSR: rows in index
 * order, each row in CSR order (the visiting order of one bundle-serial
 * worker).  Positions are updated immediately after every pair force
 * (Sec. 3.3, "immediate updates").  Y is n*dim (dim 2 or 3), updated in place. */
int oracle_serial_run(const int32_t *row_ptr, const int32_t *col, int32_t n, int32_t k,
                      int64_t t_begin, int64_t t_end, int64_t T, uint64_t seed, double alpha,
                      double beta, double gamma, double eta0, int32_t order, int32_t mode,
                      const uint32_t *thr, const uint32_t *alias, int32_t dim, double *Y)
{
    int64_t nnz = row_ptr[n];
    force_params fp = {alpha, beta, gamma, eta0, g_force_kernel};
    sampler sp = {n, mode, thr, alias};
    int64_t *perm = (int64_t *)malloc(sizeof(int64_t) * (size_t)(nnz > 0 ? nnz : 1));
    if (order == ORDER_SHUFFLED) {
        perm_item *items = (perm_item *)malloc(sizeof(perm_item) * (size_t)(nnz > 0 ? nnz : 1));
        uint64_t key[2] = {seed, KEY_DOMAIN};
        for (int64_t e = 0; e < nnz; ++e) {
            uint64_t ctr[4] = {(uint64_t)e, 0, 0, TAG_PERM}, x[4];
            oracle_philox4x64(ctr, key, x);
            items[e].key = x[0];
            items[e].e = e;
        }
        qsort(items, (size_t)nnz, sizeof(perm_item), perm_cmp);
        for (int64_t p = 0; p < nnz; ++p) perm[p] = items[p].e;
        free(items);
    } else {
        for (int64_t p = 0; p < nnz; ++p) perm[p] = p;
    }
    serial_epochs(row_ptr, col, n, k, t_begin, t_end, T, seed, &fp, &sp, dim, perm, Y);
    free(perm);
    return 0;
}

/* Serial Algorithm 1 with the directed edges visited in a caller-given order
 * edge_order[0..nnz), which must be a permutation of [0, nnz) (checked; -1
 * otherwise).  Draws stay keyed by CSR position, so only the order of the
 * immediate updates changes. */
int oracle_serial_run_ordered(const int32_t *row_ptr, const int32_t *col, int32_t n, int32_t k,
                              int64_t t_begin, int64_t t_end, int64_t T, uint64_t seed,
                              double alpha, double beta, double gamma, double eta0, int32_t mode,
                              const uint32_t *thr, const uint32_t *alias, int32_t dim,
                              const int64_t *edge_order, double *Y)
{
    int64_t nnz = row_ptr[n];
    unsigned char *seen = (unsigned char *)calloc((size_t)(nnz > 0 ? nnz : 1), 1);
    for (int64_t p = 0; p < nnz; ++p) {
        int64_t e = edge_order[p];
        if (e < 0 || e >= nnz || seen[e]) {
            free(seen);
            return -1;
        }
        seen[e] = 1;
    }
    free(seen);
    force_params fp = {alpha, beta, gamma, eta0, g_force_kernel};
    sampler sp = {n, mode, thr, alias};
    serial_epochs(row_ptr, col, n, k, t_begin, t_end, T, seed, &fp, &sp, dim, edge_order, Y);
    return 0;
}

/* --------------------------------------------------------------- Jacobi epoch */
/* One synchronous epoch t: the same pairs and the same draws as the stochastic
 * epoch, but every pair force is evaluated at the epoch-start positions Y and
 * the contributions are summed into D before Y_out = Y + D.  use_attr /
 * use_rep switch the two force families (for the expectation pins).  When
 * abs_out is non-NULL it receives, per node and coordinate, the sum of the
 * absolute values of the contributions (a rounding-error scale).  Y, Y_out and
 * abs_out are n*dim (dim 2 or 3). */
static void jacobi_pair(double coef, int dim, const double *d, int64_t a, int64_t b, double *D,
                        double *abs_out)
{
    /* D[a] += coef * d, D[b] -= coef * d */
    for (int c = 0; c < dim; ++c) {
        D[a + c] += coef * d[c];
        D[b + c] -= coef * d[c];
        if (abs_out) {
            abs_out[a + c] += fabs(coef * d[c]);
            abs_out[b + c] += fabs(coef * d[c]);
        }
    }
}

int oracle_jacobi_epoch(const int32_t *row_ptr, const int32_t *col, int32_t n, int32_t k,
                        int64_t t, int64_t T, uint64_t seed, double alpha, double beta,
                        double gamma, double eta0, int32_t mode, const uint32_t *thr,
                        const uint32_t *alias, int32_t use_attr, int32_t use_rep, int32_t dim,
                        const double *Y, double *Y_out, double *abs_out)
{
    force_params fp = {alpha, beta, gamma, eta0, g_force_kernel};
    sampler sp = {n, mode, thr, alias};
    double eta = eta_at(&fp, t, T);
    double *D = (double *)calloc((size_t)n * (size_t)dim + 3, sizeof(double));
    int32_t *neg = (int32_t *)malloc(sizeof(int32_t) * (size_t)(k > 0 ? k : 1));
    if (abs_out) memset(abs_out, 0, sizeof(double) * (size_t)n * (size_t)dim);
    for (int32_t i = 0; i < n; ++i) {
        const int64_t yi = (int64_t)dim * i;
        for (int64_t e = row_ptr[i]; e < row_ptr[i + 1]; ++e) {
            const int64_t yj = (int64_t)dim * col[e];
            double d[3], q;
            if (use_attr) {
                q = 0.0;
                for (int c = 0; c < dim; ++c) {
                    d[c] = Y[yi + c] - Y[yj + c];
                    q += d[c] * d[c];
                }
                /* attraction: y_i -= eta*A(d), y_j += eta*A(d) */
                jacobi_pair(-eta * attr_coef(&fp, q), dim, d, yi, yj, D, abs_out);
            }
            if (use_rep && k > 0) {
                draw_negatives(&sp, seed, e, t, i, k, neg);
                for (int32_t m = 0; m < k; ++m) {
                    const int64_t ys = (int64_t)dim * neg[m];
                    q = 0.0;
                    for (int c = 0; c < dim; ++c) {
                        d[c] = Y[yi + c] - Y[ys + c];
                        q += d[c] * d[c];
                    }
                    /* repulsion: y_i += eta*R(d), y_s -= eta*R(d) */
                    jacobi_pair(eta * rep_coef(&fp, q), dim, d, yi, ys, D, abs_out);
                }
            }
        }
    }
    for (int64_t v = 0; v < (int64_t)n * dim; ++v) Y_out[v] = Y[v] + D[v];
    free(neg);
    free(D);
    return 0;
}

/* ----------------------------------------------------------------- energies */
/* Pair energies whose negative gradients are the forces (Eq. (2):
 * F = -grad U), as functions of q = |d|^2 (grad q = 2d):
 *   t-FDP:    U_a(q) = alpha * (q/2 + (beta/2) ln(1+q))
 *             U_r(q) = (1+q)^(1-gamma) / (2(gamma-1))      (gamma != 1)
 *   Gaussian: U_a(q) = alpha * (q/2 + beta (1 - exp(-q/2)))
 *             U_r(q) = exp(-gamma q/2) / gamma                           */
static double energy_attr(const force_params *fp, double q)
{
    if (fp->kernel == FORCE_GAUSSIAN) return fp->alpha * (0.5 * q + fp->beta * -expm1(-0.5 * q));
    return fp->alpha * (0.5 * q + 0.5 * fp->beta * log1p(q));
}

static double energy_rep(const force_params *fp, double q)
{
    if (fp->kernel == FORCE_GAUSSIAN) return exp(-0.5 * fp->gamma * q) / fp->gamma;
    return pow(1.0 + q, 1.0 - fp->gamma) / (2.0 * (fp->gamma - 1.0));
}

/* The two pair energies at distance dist, for the pins of Eq. (2). */
void oracle_pair_energies(double alpha, double beta, double gamma, double dist, double *ua,
                          double *ur)
{
    force_params fp = {alpha, beta, gamma, 1.0, g_force_kernel};
    double q = dist * dist;
    *ua = energy_attr(&fp, q);
    *ur = energy_rep(&fp, q);
}

/* Energy actually sampled in epoch t at fixed Y: the sum over directed edges of
 * the attraction energy plus the repulsion energies of the drawn pairs (the
 * "actual energy" of Sec. 3.3).  parts (nullable) receives {attraction,
 * repulsion}. */
double oracle_sampled_energy(const int32_t *row_ptr, const int32_t *col, int32_t n, int32_t k,
                             int64_t t, uint64_t seed, double alpha, double beta, double gamma,
                             int32_t mode, const uint32_t *thr, const uint32_t *alias,
                             const double *Y, double *parts)
{
    force_params fp = {alpha, beta, gamma, 1.0, g_force_kernel};
    sampler sp = {n, mode, thr, alias};
    int32_t *neg = (int32_t *)malloc(sizeof(int32_t) * (size_t)(k > 0 ? k : 1));
    double ea = 0.0, er = 0.0;
    for (int32_t i = 0; i < n; ++i) {
        for (int64_t e = row_ptr[i]; e < row_ptr[i + 1]; ++e) {
            int32_t j = col[e];
            double dx = Y[2 * i] - Y[2 * j], dy = Y[2 * i + 1] - Y[2 * j + 1];
            ea += energy_attr(&fp, dx * dx + dy * dy);
            draw_negatives(&sp, seed, e, t, i, k, neg);
            for (int32_t m = 0; m < k; ++m) {
                int32_t s = neg[m];
                double sx = Y[2 * i] - Y[2 * s], sy = Y[2 * i + 1] - Y[2 * s + 1];
                er += energy_rep(&fp, sx * sx + sy * sy);
            }
        }
    }
    free(neg);
    if (parts) {
        parts[0] = ea;
        parts[1] = er;
    }
    return ea + er;
}

/* The degree-weighted objective the sampling realises in expectation
 * (Eq. (4) with the weight k(d_i+d_j)/(n-1) of Sec. 3.3):
 *   U_eff = 2 sum_{undirected (i,j)} U_a + (k/(n-1)) sum_{i<j} (d_i+d_j) U_r.
 * O(n^2); for small graphs only.  parts (nullable) receives {attraction,
 * weighted repulsion}. */
double oracle_effective_energy(const int32_t *row_ptr, const int32_t *col, int32_t n, int32_t k,
                               double alpha, double beta, double gamma, const double *Y,
                               double *parts)
{
    force_params fp = {alpha, beta, gamma, 1.0, g_force_kernel};
    double ea = 0.0, er = 0.0;
    for (int32_t i = 0; i < n; ++i)
        for (int64_t e = row_ptr[i]; e < row_ptr[i + 1]; ++e) {
            int32_t j = col[e];
            double dx = Y[2 * i] - Y[2 * j], dy = Y[2 * i + 1] - Y[2 * j + 1];
            ea += energy_attr(&fp, dx * dx + dy * dy); /* each undirected edge twice */
        }
    for (int32_t i = 0; i < n; ++i)
        for (int32_t j = i + 1; j < n; ++j) {
            double di = row_ptr[i + 1] - row_ptr[i], dj = row_ptr[j + 1] - row_ptr[j];
            double dx = Y[2 * i] - Y[2 * j], dy = Y[2 * i + 1] - Y[2 * j + 1];
            er += (di + dj) * energy_rep(&fp, dx * dx + dy * dy);
        }
    er *= n > 1 ? (double)k / (double)(n - 1) : 0.0;
    if (parts) {
        parts[0] = ea;
        parts[1] = er;
    }
    return ea + er;
}

/* ------------------------------------------------ threaded bundle scheme */
/* The paper's lock-free bundle scheme (Sec. 3.4) on host threads: the rows
 * (bundles: all out-edges of one source) are visited in a seeded shuffled
 * order, handed out dynamically, one bundle per thread at a time, with
 * unsynchronised read-modify-writes of the shared FP64 positions (relaxed
 * atomic loads/stores of the bit patterns, so the races are benign in C).
 * Used as the timed CPU baseline and as the large-graph quality reference. */
typedef struct {
    const int32_t *row_ptr, *col;
    int32_t n, k;
    int64_t t_begin, t_end, T;
    uint64_t seed;
    force_params fp;
    sampler sp;
    const int32_t *order; /* shuffled row order */
    double *Y;
    int64_t next_bundle; /* shared work counter, atomic, reset every epoch */
    pthread_barrier_t *barrier;
} thread_job;

typedef struct {
    thread_job *job;
    int32_t index;
} thread_arg;

static inline double ld(const double *p)
{
    uint64_t b = __atomic_load_n((const uint64_t *)p, __ATOMIC_RELAXED);
    double d;
    memcpy(&d, &b, sizeof d);
    return d;
}

static inline void st(double *p, double v)
{
    uint64_t b;
    memcpy(&b, &v, sizeof b);
    __atomic_store_n((uint64_t *)p, b, __ATOMIC_RELAXED);
}

static void *thread_main(void *arg)
{
    thread_arg *ta = (thread_arg *)arg;
    thread_job *job = ta->job;
    int32_t *neg = (int32_t *)malloc(sizeof(int32_t) * (size_t)(job->k > 0 ? job->k : 1));
    for (int64_t t = job->t_begin; t < job->t_end; ++t) {
        double eta = eta_at(&job->fp, t, job->T);
        for (;;) {
            int64_t b = __atomic_fetch_add(&job->next_bundle, 1, __ATOMIC_RELAXED);
            if (b >= job->n) break;
            int32_t i = job->order[b];
            double *Y = job->Y;
            for (int64_t e = job->row_ptr[i]; e < job->row_ptr[i + 1]; ++e) {
                int32_t j = job->col[e];
                double yi[2] = {ld(Y + 2 * i), ld(Y + 2 * i + 1)};
                double yj[2] = {ld(Y + 2 * j), ld(Y + 2 * j + 1)};
                attract_pair(&job->fp, eta, 2, yi, yj);
                st(Y + 2 * i, yi[0]); st(Y + 2 * i + 1, yi[1]);
                st(Y + 2 * j, yj[0]); st(Y + 2 * j + 1, yj[1]);
                draw_negatives(&job->sp, job->seed, e, t, i, job->k, neg);
                for (int32_t m = 0; m < job->k; ++m) {
                    int32_t s = neg[m];
                    double ys[2] = {ld(Y + 2 * s), ld(Y + 2 * s + 1)};
                    yi[0] = ld(Y + 2 * i); yi[1] = ld(Y + 2 * i + 1);
                    repel_pair(&job->fp, eta, 2, yi, ys);
                    st(Y + 2 * i, yi[0]); st(Y + 2 * i + 1, yi[1]);
                    st(Y + 2 * s, ys[0]); st(Y + 2 * s + 1, ys[1]);
                }
            }
        }
        /* every thread finishes epoch t before the counter is reset and any
         * thread starts epoch t+1 (eta changes between epochs) */
        pthread_barrier_wait(job->barrier);
        if (ta->index == 0) __atomic_store_n(&job->next_bundle, 0, __ATOMIC_RELAXED);
        pthread_barrier_wait(job->barrier);
    }
    free(neg);
    return NULL;
}

int oracle_threaded_run(const int32_t *row_ptr, const int32_t *col, int32_t n, int32_t k,
                        int64_t t_begin, int64_t t_end, int64_t T, uint64_t seed, double alpha,
                        double beta, double gamma, double eta0, int32_t mode, const uint32_t *thr,
                        const uint32_t *alias, int32_t nthreads, double *Y)
{
    if (nthreads < 1) nthreads = 1;
    int32_t *order = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    perm_item *items = (perm_item *)malloc(sizeof(perm_item) * (size_t)(n > 0 ? n : 1));
    uint64_t key[2] = {seed, KEY_DOMAIN};
    for (int32_t i = 0; i < n; ++i) {
        uint64_t ctr[4] = {(uint64_t)i, 1, 0, TAG_PERM}, x[4];
        oracle_philox4x64(ctr, key, x);
        items[i].key = x[0];
        items[i].e = i;
    }
    qsort(items, (size_t)n, sizeof(perm_item), perm_cmp);
    for (int32_t p = 0; p < n; ++p) order[p] = (int32_t)items[p].e;
    free(items);

    pthread_barrier_t barrier;
    pthread_barrier_init(&barrier, NULL, (unsigned)nthreads);
    thread_job job;
    job.row_ptr = row_ptr;
    job.col = col;
    job.n = n;
    job.k = k;
    job.t_begin = t_begin;
    job.t_end = t_end;
    job.T = T;
    job.seed = seed;
    job.fp = (force_params){alpha, beta, gamma, eta0, g_force_kernel};
    job.sp = (sampler){n, mode, thr, alias};
    job.order = order;
    job.Y = Y;
    job.next_bundle = 0;
    job.barrier = &barrier;
    pthread_t *th = (pthread_t *)malloc(sizeof(pthread_t) * (size_t)nthreads);
    thread_arg *args = (thread_arg *)malloc(sizeof(thread_arg) * (size_t)nthreads);
    for (int32_t w = 0; w < nthreads; ++w) {
        args[w].job = &job;
        args[w].index = w;
        pthread_create(&th[w], NULL, thread_main, &args[w]);
    }
    for (int32_t w = 0; w < nthreads; ++w) pthread_join(th[w], NULL);
    free(args);
    free(th);
    pthread_barrier_destroy(&barrier);
    free(order);
    return 0;
}
