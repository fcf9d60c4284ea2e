/*
 * FP64 CPU oracle for SNeCT (Choi & Sael, "SNeCT: Scalable network
 * constrained Tucker decomposition for integrative multi-platform data
 * analysis", arXiv:1711.08095).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the tests, the smoke check and the benchmark's CPU
 * baseline do.  It shares no source with the HIP path.
 *
 * What it computes, with the paper passage each part follows:
 *   - the Tucker model value, Eq. (2) written elementwise:
 *       xt(i,j,k) = sum_{a,b,c} G[a,b,c] A[i,a] B[j,b] C[k,c]
 *   - the objective f_opt = f + lambda_g f_g, Eq. (3) with the L2 term in the
 *     per-nonzero split of Section 2.3.2 and the network term Eq. (4);
 *   - the stratified SGD iteration ("SNeCT-S") that replaces the lock-free
 *     random-order loop of Algorithm 1 by a seeded, deterministic schedule:
 *       plan: seeded row permutations put patients into P row blocks and genes
 *             into P column blocks; block (p,q) lists its nonzeros in
 *             ascending (k, i, j) order, cut into tiles of at most T entries
 *             that never straddle a change of k;
 *       each epoch: one Jacobi step of the network gradient (Eq. 5, third
 *             line, summed over all edges, Algorithm 1 network update),
 *             then P strata, stratum s holding the blocks (p, (p+s) mod P);
 *             in every tile all nonzeros use the factor rows as they were
 *             before the tile (factor-row update of Algorithm 1 with the
 *             gradients of Eq. 5), duplicate rows summing their terms;
 *             after each stratum one core/platform step with the stratum's
 *             mean gradient (Algorithm 1 core update; the paper gives no
 *             rule for a stratum, this is the reading used);
 *       loss and training RMSE at the end of every epoch.
 *
 * Readings of the paper where it is silent or garbled (also listed in the
 * design notes):
 *   - Collapse(D,n) and D (/) G in Algorithm 1 are taken as the true Eq. (5)
 *     gradients, never dividing by G.
 *   - every mode of one nonzero uses the values from before its update;
 *   - the edge update of Algorithm 1 is simultaneous on both endpoints and
 *     applied once per epoch to all edges at once (Jacobi), in n_sub equal
 *     sub-steps, n_sub = max(1, ceil(2 eta lambda_g d_max));
 *   - R in Eq. (3) counts only rows with at least one nonzero (the
 *     per-nonzero split gives empty rows no weight);
 *   - the random order of Algorithm 1 is replaced by SplitMix64 streams
 *     driving Fisher-Yates shuffles (see oracle_stream_state).
 *
 * Random numbers: SplitMix64 (Steele, Lea & Flood, OOPSLA 2014), with the
 * published increment 0x9e3779b97f4a7c15 and finaliser constants
 * 0xbf58476d1ce4e5b9 / 0x94d049bb133111eb and shifts 30/27/31.  Stream t of a
 * seed starts from the t-th output (t = 0, 1, ...) of SplitMix64 seeded with
 * the seed.  A shuffle of n items walks r = n-1 down to 1, draws one 64-bit
 * value u and swaps item r with item floor(u * (r+1) / 2^64).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_OK 0
#define ORC_E_ARG -1
#define ORC_E_INDEX -2
#define ORC_E_DUPLICATE -3
#define ORC_E_OOM -5

/* ------------------------------------------------------------------ */
/* SplitMix64 and shuffles                                            */
/* ------------------------------------------------------------------ */
static uint64_t orc_sm64(uint64_t *s)
{
    uint64_t z = (*s += 0x9e3779b97f4a7c15ULL);
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
    return z ^ (z >> 31);
}

/* n-th output (0-based) of SplitMix64 seeded with `seed`.  The generator's
   state only ever grows by the increment, so before output n it holds
   seed + n * increment (mod 2^64); one step from there gives output n. */
uint64_t oracle_splitmix64_at(uint64_t seed, uint64_t n)
{
    uint64_t s = seed + n * 0x9e3779b97f4a7c15ULL;
    return orc_sm64(&s);
}

uint64_t oracle_stream_state(uint64_t seed, uint64_t stream)
{
    return oracle_splitmix64_at(seed, stream);
}

/* In-place Fisher-Yates of a[0..n) driven by the given stream. */
void oracle_shuffle(int32_t *a, int64_t n, uint64_t seed, uint64_t stream)
{
    uint64_t s = oracle_stream_state(seed, stream);
    for (int64_t r = n - 1; r >= 1; --r) {
        uint64_t u = orc_sm64(&s);
        int64_t j = (int64_t)(((unsigned __int128)u * (unsigned __int128)(uint64_t)(r + 1)) >> 64);
        int32_t t = a[r];
        a[r] = a[j];
        a[j] = t;
    }
}

/* ------------------------------------------------------------------ */
/* Problem description                                                */
/* ------------------------------------------------------------------ */
typedef struct {
    int32_t I1, I2, I3;
    int32_t J1, J2, J3;
    int64_t nnz;
    const int32_t *i, *j, *k;
    const double *x;
    int64_t E;
    const int32_t *eu, *ev;
    const double *ew; /* NULL -> all weights 1 */
    double lam, lam_g, lr, core_lr_scale;
    int32_t P, T;
    uint64_t seed;
} oracle_problem;

/* The plan: block membership and the ordered, tiled nonzero lists. */
typedef struct {
    int32_t P;
    int32_t *perm1, *perm2;     /* row permutations: perm[position] = row */
    int32_t *blk1, *blk2;       /* row -> block */
    int64_t *block_start;       /* [P*P+1] offsets into order[] */
    int64_t *order;             /* nonzero ids, block-major, (k,i,j) inside */
    int64_t ntiles;
    int64_t *tile_start;        /* [ntiles+1] offsets into order[] */
    int64_t *block_tile;        /* [P*P+1] offsets into tile_start[] */
    int64_t *n1, *n2, *n3;      /* slice counts */
    /* symmetric network: CSR of neighbours with summed weights */
    int64_t *adj_start;         /* [I2+1] */
    int32_t *adj_nbr;
    double *adj_w;
    double *deg;                /* weighted degree */
    double dmax;
} oracle_plan_t;

static const oracle_problem *g_sort_prob; /* qsort context (single-threaded plan) */

static int orc_cmp_kij(const void *pa, const void *pb)
{
    int64_t a = *(const int64_t *)pa, b = *(const int64_t *)pb;
    const oracle_problem *pr = g_sort_prob;
    if (pr->k[a] != pr->k[b]) return pr->k[a] < pr->k[b] ? -1 : 1;
    if (pr->i[a] != pr->i[b]) return pr->i[a] < pr->i[b] ? -1 : 1;
    if (pr->j[a] != pr->j[b]) return pr->j[a] < pr->j[b] ? -1 : 1;
    return 0;
}

typedef struct { int32_t a, b; double w; } orc_edge;

static int orc_cmp_edge(const void *pa, const void *pb)
{
    const orc_edge *a = (const orc_edge *)pa, *b = (const orc_edge *)pb;
    if (a->a != b->a) return a->a < b->a ? -1 : 1;
    if (a->b != b->b) return a->b < b->b ? -1 : 1;
    return 0;
}

void oracle_plan_free(oracle_plan_t *pl)
{
    if (!pl) return;
    free(pl->perm1); free(pl->perm2); free(pl->blk1); free(pl->blk2);
    free(pl->block_start); free(pl->order); free(pl->tile_start); free(pl->block_tile);
    free(pl->n1); free(pl->n2); free(pl->n3);
    free(pl->adj_start); free(pl->adj_nbr); free(pl->adj_w); free(pl->deg);
    free(pl);
}

static int orc_validate(const oracle_problem *pr)
{
    if (pr->I1 <= 0 || pr->I2 <= 0 || pr->I3 <= 0) return ORC_E_ARG;
    if (pr->J1 <= 0 || pr->J2 <= 0 || pr->J3 <= 0) return ORC_E_ARG;
    if (pr->nnz < 0 || pr->E < 0) return ORC_E_ARG;
    if (pr->P < 1 || pr->P > pr->I1 || pr->P > pr->I2) return ORC_E_ARG;
    if (pr->T < 1) return ORC_E_ARG;
    if (!(pr->lam >= 0) || !(pr->lam_g >= 0) || !(pr->lr > 0) || !(pr->core_lr_scale >= 0))
        return ORC_E_ARG;
    for (int64_t t = 0; t < pr->nnz; ++t) {
        if (pr->i[t] < 0 || pr->i[t] >= pr->I1 || pr->j[t] < 0 || pr->j[t] >= pr->I2 ||
            pr->k[t] < 0 || pr->k[t] >= pr->I3)
            return ORC_E_INDEX;
        if (!isfinite(pr->x[t])) return ORC_E_ARG;
    }
    for (int64_t e = 0; e < pr->E; ++e) {
        if (pr->eu[e] < 0 || pr->eu[e] >= pr->I2 || pr->ev[e] < 0 || pr->ev[e] >= pr->I2)
            return ORC_E_INDEX;
        if (pr->eu[e] == pr->ev[e]) return ORC_E_ARG;
        if (pr->ew && (!(pr->ew[e] >= 0) || !isfinite(pr->ew[e]))) return ORC_E_ARG;
    }
    return ORC_OK;
}

/* Build the plan.  Returns 0 or a negative error code. */
int oracle_plan_build(const oracle_problem *pr, oracle_plan_t **out)
{
    int rc = orc_validate(pr);
    if (rc) return rc;
    oracle_plan_t *pl = (oracle_plan_t *)calloc(1, sizeof(oracle_plan_t));
    if (!pl) return ORC_E_OOM;
    const int64_t P = pr->P;
    pl->P = pr->P;
    pl->perm1 = (int32_t *)malloc(sizeof(int32_t) * pr->I1);
    pl->perm2 = (int32_t *)malloc(sizeof(int32_t) * pr->I2);
    pl->blk1 = (int32_t *)malloc(sizeof(int32_t) * pr->I1);
    pl->blk2 = (int32_t *)malloc(sizeof(int32_t) * pr->I2);
    pl->n1 = (int64_t *)calloc(pr->I1, sizeof(int64_t));
    pl->n2 = (int64_t *)calloc(pr->I2, sizeof(int64_t));
    pl->n3 = (int64_t *)calloc(pr->I3, sizeof(int64_t));
    pl->block_start = (int64_t *)calloc(P * P + 1, sizeof(int64_t));
    pl->order = (int64_t *)malloc(sizeof(int64_t) * (pr->nnz > 0 ? pr->nnz : 1));
    if (!pl->perm1 || !pl->perm2 || !pl->blk1 || !pl->blk2 || !pl->n1 || !pl->n2 || !pl->n3 ||
        !pl->block_start || !pl->order) {
        oracle_plan_free(pl);
        return ORC_E_OOM;
    }
    /* slice counts |Omega^{n,i}| */
    for (int64_t t = 0; t < pr->nnz; ++t) {
        pl->n1[pr->i[t]]++;
        pl->n2[pr->j[t]]++;
        pl->n3[pr->k[t]]++;
    }
    /* seeded permutations and block membership: the row at position r of
       the permutation goes to block floor(r * P / I) */
    for (int32_t r = 0; r < pr->I1; ++r) pl->perm1[r] = r;
    for (int32_t r = 0; r < pr->I2; ++r) pl->perm2[r] = r;
    oracle_shuffle(pl->perm1, pr->I1, pr->seed, 0);
    oracle_shuffle(pl->perm2, pr->I2, pr->seed, 1);
    for (int64_t r = 0; r < pr->I1; ++r) pl->blk1[pl->perm1[r]] = (int32_t)(r * P / pr->I1);
    for (int64_t r = 0; r < pr->I2; ++r) pl->blk2[pl->perm2[r]] = (int32_t)(r * P / pr->I2);
    /* bucket nonzeros by block, then order each block by (k, i, j) */
    for (int64_t t = 0; t < pr->nnz; ++t)
        pl->block_start[(int64_t)pl->blk1[pr->i[t]] * P + pl->blk2[pr->j[t]] + 1]++;
    for (int64_t b = 0; b < P * P; ++b) pl->block_start[b + 1] += pl->block_start[b];
    {
        int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * P * P);
        if (!fill) { oracle_plan_free(pl); return ORC_E_OOM; }
        memcpy(fill, pl->block_start, sizeof(int64_t) * P * P);
        for (int64_t t = 0; t < pr->nnz; ++t) {
            int64_t b = (int64_t)pl->blk1[pr->i[t]] * P + pl->blk2[pr->j[t]];
            pl->order[fill[b]++] = t;
        }
        free(fill);
    }
    g_sort_prob = pr;
    for (int64_t b = 0; b < P * P; ++b) {
        int64_t s = pl->block_start[b], e = pl->block_start[b + 1];
        if (e - s > 1) qsort(pl->order + s, (size_t)(e - s), sizeof(int64_t), orc_cmp_kij);
        for (int64_t t = s + 1; t < e; ++t)
            if (orc_cmp_kij(&pl->order[t - 1], &pl->order[t]) == 0) {
                oracle_plan_free(pl);
                return ORC_E_DUPLICATE;
            }
    }
    /* tiles: runs of at most T entries, a new tile whenever k changes */
    pl->tile_start = (int64_t *)malloc(sizeof(int64_t) * (pr->nnz + 1));
    pl->block_tile = (int64_t *)malloc(sizeof(int64_t) * (P * P + 1));
    if (!pl->tile_start || !pl->block_tile) { oracle_plan_free(pl); return ORC_E_OOM; }
    int64_t nt = 0;
    for (int64_t b = 0; b < P * P; ++b) {
        pl->block_tile[b] = nt;
        int64_t s = pl->block_start[b], e = pl->block_start[b + 1];
        int64_t t = s;
        while (t < e) {
            pl->tile_start[nt++] = t;
            int32_t kk = pr->k[pl->order[t]];
            int64_t u = t;
            while (u < e && u - t < pr->T && pr->k[pl->order[u]] == kk) ++u;
            t = u;
        }
    }
    pl->block_tile[P * P] = nt;
    pl->tile_start[nt] = pr->nnz;
    pl->ntiles = nt;
    /* symmetric weighted adjacency: each undirected edge in both rows,
       repeated pairs merged by summing their weights */
    {
        int64_t m = 2 * pr->E;
        orc_edge *ed = (orc_edge *)malloc(sizeof(orc_edge) * (m > 0 ? m : 1));
        if (!ed) { oracle_plan_free(pl); return ORC_E_OOM; }
        for (int64_t e = 0; e < pr->E; ++e) {
            double w = pr->ew ? pr->ew[e] : 1.0;
            ed[2 * e].a = pr->eu[e]; ed[2 * e].b = pr->ev[e]; ed[2 * e].w = w;
            ed[2 * e + 1].a = pr->ev[e]; ed[2 * e + 1].b = pr->eu[e]; ed[2 * e + 1].w = w;
        }
        if (m > 1) qsort(ed, (size_t)m, sizeof(orc_edge), orc_cmp_edge);
        int64_t u = 0;
        for (int64_t e = 0; e < m; ++e) {
            if (u > 0 && ed[u - 1].a == ed[e].a && ed[u - 1].b == ed[e].b)
                ed[u - 1].w += ed[e].w;
            else
                ed[u++] = ed[e];
        }
        pl->adj_start = (int64_t *)calloc(pr->I2 + 1, sizeof(int64_t));
        pl->adj_nbr = (int32_t *)malloc(sizeof(int32_t) * (u > 0 ? u : 1));
        pl->adj_w = (double *)malloc(sizeof(double) * (u > 0 ? u : 1));
        pl->deg = (double *)calloc(pr->I2, sizeof(double));
        if (!pl->adj_start || !pl->adj_nbr || !pl->adj_w || !pl->deg) {
            free(ed); oracle_plan_free(pl); return ORC_E_OOM;
        }
        for (int64_t e = 0; e < u; ++e) {
            pl->adj_start[ed[e].a + 1]++;
            pl->adj_nbr[e] = ed[e].b;
            pl->adj_w[e] = ed[e].w;
            pl->deg[ed[e].a] += ed[e].w;
        }
        for (int32_t r = 0; r < pr->I2; ++r) pl->adj_start[r + 1] += pl->adj_start[r];
        pl->dmax = 0.0;
        for (int32_t r = 0; r < pr->I2; ++r) if (pl->deg[r] > pl->dmax) pl->dmax = pl->deg[r];
        free(ed);
    }
    *out = pl;
    return ORC_OK;
}

/* ------------------------------------------------------------------ */
/* Plain definitions                                                  */
/* ------------------------------------------------------------------ */

/* Eq. (2) elementwise: model value at one cell. */
static double orc_model_value(const oracle_problem *pr, const double *A, const double *B,
                              const double *C, const double *G, int32_t i, int32_t j, int32_t k)
{
    const int J1 = pr->J1, J2 = pr->J2, J3 = pr->J3;
    double s = 0.0;
    for (int a = 0; a < J1; ++a)
        for (int b = 0; b < J2; ++b)
            for (int c = 0; c < J3; ++c)
                s += G[((int64_t)a * J2 + b) * J3 + c] * A[(int64_t)i * J1 + a] *
                     B[(int64_t)j * J2 + b] * C[(int64_t)k * J3 + c];
    return s;
}

void oracle_model_values(const oracle_problem *pr, const double *A, const double *B,
                         const double *C, const double *G, double *out)
{
#pragma omp parallel for schedule(static)
    for (int64_t t = 0; t < pr->nnz; ++t)
        out[t] = orc_model_value(pr, A, B, C, G, pr->i[t], pr->j[t], pr->k[t]);
}

#define ORC_CHUNK 4096

/* f_opt = 1/2 sum e^2 + lambda/2 (|G|^2 + sum over observed rows |u|^2)
 *       + lambda_g/2 sum_edges w |b_u - b_v|^2   (Eq. 3, Sec. 2.3.2, Eq. 4)
 * Fills parts[0] = 1/2 sum e^2, parts[1] = L2 term (with lambda/2),
 * parts[2] = network term (with lambda_g/2).  Chunked sums added in a fixed
 * order, so the result does not depend on the thread count. */
double oracle_loss(const oracle_problem *pr, const double *A, const double *B, const double *C,
                   const double *G, double *rmse, double *parts)
{
    const int64_t nch = (pr->nnz + ORC_CHUNK - 1) / ORC_CHUNK;
    double *cs = (double *)calloc(nch > 0 ? nch : 1, sizeof(double));
#pragma omp parallel for schedule(static)
    for (int64_t c = 0; c < nch; ++c) {
        int64_t s = c * ORC_CHUNK, e = s + ORC_CHUNK;
        if (e > pr->nnz) e = pr->nnz;
        double acc = 0.0;
        for (int64_t t = s; t < e; ++t) {
            double r = pr->x[t] - orc_model_value(pr, A, B, C, G, pr->i[t], pr->j[t], pr->k[t]);
            acc += r * r;
        }
        cs[c] = acc;
    }
    double sse = 0.0;
    for (int64_t c = 0; c < nch; ++c) sse += cs[c];
    free(cs);
    /* which rows are observed */
    char *o1 = (char *)calloc(pr->I1, 1), *o2 = (char *)calloc(pr->I2, 1), *o3 = (char *)calloc(pr->I3, 1);
    for (int64_t t = 0; t < pr->nnz; ++t) { o1[pr->i[t]] = 1; o2[pr->j[t]] = 1; o3[pr->k[t]] = 1; }
    double reg = 0.0;
    for (int64_t q = 0; q < (int64_t)pr->J1 * pr->J2 * pr->J3; ++q) reg += G[q] * G[q];
    for (int32_t r = 0; r < pr->I1; ++r)
        if (o1[r]) for (int a = 0; a < pr->J1; ++a) reg += A[(int64_t)r * pr->J1 + a] * A[(int64_t)r * pr->J1 + a];
    for (int32_t r = 0; r < pr->I2; ++r)
        if (o2[r]) for (int b = 0; b < pr->J2; ++b) reg += B[(int64_t)r * pr->J2 + b] * B[(int64_t)r * pr->J2 + b];
    for (int32_t r = 0; r < pr->I3; ++r)
        if (o3[r]) for (int c = 0; c < pr->J3; ++c) reg += C[(int64_t)r * pr->J3 + c] * C[(int64_t)r * pr->J3 + c];
    free(o1); free(o2); free(o3);
    double net = 0.0;
    for (int64_t e = 0; e < pr->E; ++e) {
        double w = pr->ew ? pr->ew[e] : 1.0, d2 = 0.0;
        for (int b = 0; b < pr->J2; ++b) {
            double d = B[(int64_t)pr->eu[e] * pr->J2 + b] - B[(int64_t)pr->ev[e] * pr->J2 + b];
            d2 += d * d;
        }
        net += w * d2;
    }
    if (rmse) *rmse = pr->nnz > 0 ? sqrt(sse / (double)pr->nnz) : 0.0;
    double f = 0.5 * sse + 0.5 * pr->lam * reg + 0.5 * pr->lam_g * net;
    if (parts) { parts[0] = 0.5 * sse; parts[1] = 0.5 * pr->lam * reg; parts[2] = 0.5 * pr->lam_g * net; }
    return f;
}

/* ------------------------------------------------------------------ */
/* The SNeCT-S iteration                                              */
/* ------------------------------------------------------------------ */

/* Network step for one epoch: B <- B - (eta lambda_g / n_sub) L B, n_sub
 * times, each a Jacobi step over all rows (Eq. 5, edge gradient, summed). */
static void orc_graph_step(const oracle_problem *pr, const oracle_plan_t *pl, double *B, double *tmp)
{
    if (!(pr->lam_g > 0) || pr->E == 0) return;
    const int J2 = pr->J2;
    int64_t nsub = (int64_t)ceil(2.0 * pr->lr * pr->lam_g * pl->dmax);
    if (nsub < 1) nsub = 1;
    const double alpha = pr->lr * pr->lam_g / (double)nsub;
    for (int64_t it = 0; it < nsub; ++it) {
#pragma omp parallel for schedule(static)
        for (int32_t r = 0; r < pr->I2; ++r) {
            for (int b = 0; b < J2; ++b) {
                double lb = pl->deg[r] * B[(int64_t)r * J2 + b];
                for (int64_t e = pl->adj_start[r]; e < pl->adj_start[r + 1]; ++e)
                    lb -= pl->adj_w[e] * B[(int64_t)pl->adj_nbr[e] * J2 + b];
                tmp[(int64_t)r * J2 + b] = B[(int64_t)r * J2 + b] - alpha * lb;
            }
        }
        memcpy(B, tmp, sizeof(double) * (size_t)pr->I2 * J2);
    }
}

/* One block's tiles.  S (I3 x J1 x J2) and m (I3) receive the block's sums
 * of e * a (x) b and of nonzero counts per platform.  dA / dB are zeroed
 * scratch rows (indexed by global row) owned by this block's rows. */
static void orc_block(const oracle_problem *pr, const oracle_plan_t *pl, int64_t blk,
                      const double *H, double *A, double *B, double *S, double *m,
                      double *dA, double *dB, double *wa, double *wb)
{
    const int J1 = pr->J1, J2 = pr->J2;
    for (int64_t tl = pl->block_tile[blk]; tl < pl->block_tile[blk + 1]; ++tl) {
        const int64_t s = pl->tile_start[tl], e = pl->tile_start[tl + 1];
        const int32_t k = pr->k[pl->order[s]];
        const double *Hk = H + (int64_t)k * J1 * J2;
        double *Sk = S + (int64_t)k * J1 * J2;
        /* every nonzero of the tile reads the rows as they were before it */
        for (int64_t t = s; t < e; ++t) {
            const int64_t z = pl->order[t];
            const int32_t i = pr->i[z], j = pr->j[z];
            const double *a = A + (int64_t)i * J1, *b = B + (int64_t)j * J2;
            /* wa = H_k b  (= G x2 b x3 c_k), wb = H_k^T a (= G x1 a x3 c_k) */
            for (int r = 0; r < J1; ++r) {
                double acc = 0.0;
                for (int c = 0; c < J2; ++c) acc += Hk[r * J2 + c] * b[c];
                wa[r] = acc;
            }
            for (int c = 0; c < J2; ++c) {
                double acc = 0.0;
                for (int r = 0; r < J1; ++r) acc += a[r] * Hk[r * J2 + c];
                wb[c] = acc;
            }
            double xt = 0.0;
            for (int r = 0; r < J1; ++r) xt += a[r] * wa[r];
            const double err = pr->x[z] - xt;
            /* minus the Eq. (5) gradients: e * [G x2 b x3 c] - lambda/n1 a */
            for (int r = 0; r < J1; ++r)
                dA[(int64_t)i * J1 + r] += err * wa[r] - pr->lam / (double)pl->n1[i] * a[r];
            for (int c = 0; c < J2; ++c)
                dB[(int64_t)j * J2 + c] += err * wb[c] - pr->lam / (double)pl->n2[j] * b[c];
            for (int r = 0; r < J1; ++r)
                for (int c = 0; c < J2; ++c) Sk[r * J2 + c] += err * a[r] * b[c];
        }
        m[k] += (double)(e - s);
        /* apply, then clear the scratch rows */
        for (int64_t t = s; t < e; ++t) {
            const int64_t z = pl->order[t];
            const int32_t i = pr->i[z], j = pr->j[z];
            for (int r = 0; r < J1; ++r) {
                A[(int64_t)i * J1 + r] += pr->lr * dA[(int64_t)i * J1 + r];
                dA[(int64_t)i * J1 + r] = 0.0;
            }
            for (int c = 0; c < J2; ++c) {
                B[(int64_t)j * J2 + c] += pr->lr * dB[(int64_t)j * J2 + c];
                dB[(int64_t)j * J2 + c] = 0.0;
            }
        }
    }
}

/* Run `epochs` epochs starting at absolute epoch index `start_epoch`.
 * A, B, C, G are read and overwritten.  loss / rmse (may be NULL) receive
 * one value per epoch.  nthreads <= 0 keeps the OpenMP default. */
int oracle_run(const oracle_problem *pr, double *A, double *B, double *C, double *G,
               int32_t start_epoch, int32_t epochs, double *loss, double *rmse, int32_t nthreads)
{
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
    oracle_plan_t *pl = NULL;
    int rc = oracle_plan_build(pr, &pl);
    if (rc) return rc;
    const int64_t P = pr->P;
    const int J1 = pr->J1, J2 = pr->J2, J3 = pr->J3, I3 = pr->I3;
    const int64_t JJ = (int64_t)J1 * J2;
    double *H = (double *)malloc(sizeof(double) * I3 * JJ);
    double *S = (double *)calloc((size_t)(P * I3 * JJ), sizeof(double));
    double *M = (double *)calloc((size_t)(P * I3), sizeof(double));
    double *dA = (double *)calloc((size_t)pr->I1 * J1, sizeof(double));
    double *dB = (double *)calloc((size_t)pr->I2 * J2, sizeof(double));
    double *tmp = (double *)malloc(sizeof(double) * (size_t)pr->I2 * J2);
    double *C0 = (double *)malloc(sizeof(double) * (size_t)I3 * J3);
    double *G0 = (double *)malloc(sizeof(double) * (size_t)JJ * J3);
    int32_t *ord = (int32_t *)malloc(sizeof(int32_t) * P);
    if (!H || !S || !M || !dA || !dB || !tmp || !C0 || !G0 || !ord) {
        rc = ORC_E_OOM;
        goto done;
    }
    for (int32_t ep = start_epoch; ep < start_epoch + epochs; ++ep) {
        orc_graph_step(pr, pl, B, tmp);
        for (int64_t s = 0; s < P; ++s) ord[s] = (int32_t)s;
        oracle_shuffle(ord, P, pr->seed, 2 + (uint64_t)ep);
        for (int64_t si = 0; si < P; ++si) {
            const int64_t st = ord[si];
            memcpy(C0, C, sizeof(double) * (size_t)I3 * J3);
            memcpy(G0, G, sizeof(double) * (size_t)JJ * J3);
            /* H_k = G x3 c_k, frozen for the stratum */
            for (int k = 0; k < I3; ++k)
                for (int64_t ab = 0; ab < JJ; ++ab) {
                    double acc = 0.0;
                    for (int c = 0; c < J3; ++c) acc += G0[ab * J3 + c] * C0[(int64_t)k * J3 + c];
                    H[k * JJ + ab] = acc;
                }
            memset(S, 0, sizeof(double) * (size_t)(P * I3 * JJ));
            memset(M, 0, sizeof(double) * (size_t)(P * I3));
#pragma omp parallel
            {
                double *wa = (double *)malloc(sizeof(double) * J1);
                double *wb = (double *)malloc(sizeof(double) * J2);
#pragma omp for schedule(dynamic, 1)
                for (int64_t p = 0; p < P; ++p) {
                    const int64_t q = (p + st) % P;
                    orc_block(pr, pl, p * P + q, H, A, B, S + p * I3 * JJ, M + p * I3, dA, dB, wa, wb);
                }
                free(wa);
                free(wb);
            }
            /* reduce over blocks in ascending p */
            double msum = 0.0;
            for (int k = 0; k < I3; ++k) {
                double mk = 0.0;
                for (int64_t p = 0; p < P; ++p) mk += M[p * I3 + k];
                M[k] = mk; /* slot p = 0 now holds the total */
                msum += mk;
                for (int64_t ab = 0; ab < JJ; ++ab) {
                    double acc = 0.0;
                    for (int64_t p = 0; p < P; ++p) acc += S[(p * I3 + k) * JJ + ab];
                    S[k * JJ + ab] = acc;
                }
            }
            if (msum > 0) {
                const double etac = pr->lr * pr->core_lr_scale;
                /* mean platform-factor gradient */
                for (int k = 0; k < I3; ++k) {
                    for (int c = 0; c < J3; ++c) {
                        double g = 0.0;
                        for (int64_t ab = 0; ab < JJ; ++ab) g -= G0[ab * J3 + c] * S[k * JJ + ab];
                        if (M[k] > 0) g += pr->lam * (M[k] / (double)pl->n3[k]) * C0[(int64_t)k * J3 + c];
                        C[(int64_t)k * J3 + c] = C0[(int64_t)k * J3 + c] - etac * g / msum;
                    }
                }
                /* mean core gradient */
                for (int64_t ab = 0; ab < JJ; ++ab)
                    for (int c = 0; c < J3; ++c) {
                        double g = 0.0;
                        for (int k = 0; k < I3; ++k) g -= S[k * JJ + ab] * C0[(int64_t)k * J3 + c];
                        g += pr->lam * (msum / (double)pr->nnz) * G0[ab * J3 + c];
                        G[ab * J3 + c] = G0[ab * J3 + c] - etac * g / msum;
                    }
            }
        }
        double r = 0.0;
        double f = oracle_loss(pr, A, B, C, G, &r, NULL);
        if (loss) loss[ep - start_epoch] = f;
        if (rmse) rmse[ep - start_epoch] = r;
    }
done:
    free(H); free(S); free(M); free(dA); free(dB); free(tmp); free(C0); free(G0); free(ord);
    oracle_plan_free(pl);
    return rc;
}

/* ------------------------------------------------------------------ */
/* Algorithm 1 read literally (comparison run, not the library's       */
/* schedule)                                                          */
/* ------------------------------------------------------------------ */

/* Stream offset of the literal run's per-epoch visiting order; far from the
 * streams of the SNeCT-S plan (0, 1 and 2 + epoch). */
#define ORC_LITERAL_STREAM 0x100000000ull

/* Algorithm 1 on one core: each epoch visits the nnz nonzeros and the E
 * edges once, in one random interleaving (a Fisher-Yates shuffle of item ids
 * 0..nnz+E-1, id < nnz a nonzero, else edge id - nnz, drawn from stream
 * ORC_LITERAL_STREAM + epoch).  A nonzero updates a_i, b_j, c_k and G at
 * once with the Eq. (5) gradients evaluated at the values before the item,
 * step eta for every mode and for the core (one core, so the paper's
 * eta * P core step is eta); an edge (u, v, w) moves b_u and b_v towards
 * each other, both from their values before the item.  Loss and RMSE at
 * the end of every epoch.  P and T of the problem are not used. */
int oracle_run_literal(const oracle_problem *pr, double *A, double *B, double *C, double *G,
                       int32_t start_epoch, int32_t epochs, double *loss, double *rmse)
{
    oracle_plan_t *pl = NULL;
    int rc = oracle_plan_build(pr, &pl); /* validation and slice counts */
    if (rc) return rc;
    const int J1 = pr->J1, J2 = pr->J2, J3 = pr->J3;
    const int64_t NG = (int64_t)J1 * J2 * J3, nit = pr->nnz + pr->E;
    int32_t *items = (int32_t *)malloc(sizeof(int32_t) * (size_t)(nit > 0 ? nit : 1));
    double *wa = (double *)malloc(sizeof(double) * J1), *wb = (double *)malloc(sizeof(double) * J2);
    double *wc = (double *)malloc(sizeof(double) * J3), *a0 = (double *)malloc(sizeof(double) * J1);
    double *b0 = (double *)malloc(sizeof(double) * J2), *c0 = (double *)malloc(sizeof(double) * J3);
    double *G0 = (double *)malloc(sizeof(double) * NG);
    if (!items || !wa || !wb || !wc || !a0 || !b0 || !c0 || !G0 || nit >= (int64_t)1 << 31) {
        rc = ORC_E_OOM;
        goto done;
    }
    for (int32_t ep = start_epoch; ep < start_epoch + epochs; ++ep) {
        for (int64_t t = 0; t < nit; ++t) items[t] = (int32_t)t;
        oracle_shuffle(items, nit, pr->seed, ORC_LITERAL_STREAM + (uint64_t)ep);
        for (int64_t t = 0; t < nit; ++t) {
            const int64_t id = items[t];
            if (id < pr->nnz) {
                const int32_t i = pr->i[id], j = pr->j[id], k = pr->k[id];
                double *a = A + (int64_t)i * J1, *b = B + (int64_t)j * J2, *c = C + (int64_t)k * J3;
                memcpy(a0, a, sizeof(double) * J1);
                memcpy(b0, b, sizeof(double) * J2);
                memcpy(c0, c, sizeof(double) * J3);
                memcpy(G0, G, sizeof(double) * NG);
                /* partial products of G with two of the three rows */
                for (int r = 0; r < J1; ++r) wa[r] = 0.0;
                for (int q = 0; q < J2; ++q) wb[q] = 0.0;
                for (int s = 0; s < J3; ++s) wc[s] = 0.0;
                for (int r = 0; r < J1; ++r)
                    for (int q = 0; q < J2; ++q)
                        for (int s = 0; s < J3; ++s) {
                            const double g = G0[((int64_t)r * J2 + q) * J3 + s];
                            wa[r] += g * b0[q] * c0[s];
                            wb[q] += g * a0[r] * c0[s];
                            wc[s] += g * a0[r] * b0[q];
                        }
                double xt = 0.0;
                for (int r = 0; r < J1; ++r) xt += a0[r] * wa[r];
                const double err = pr->x[id] - xt, eta = pr->lr;
                for (int r = 0; r < J1; ++r) a[r] = a0[r] + eta * (err * wa[r] - pr->lam / (double)pl->n1[i] * a0[r]);
                for (int q = 0; q < J2; ++q) b[q] = b0[q] + eta * (err * wb[q] - pr->lam / (double)pl->n2[j] * b0[q]);
                for (int s = 0; s < J3; ++s) c[s] = c0[s] + eta * (err * wc[s] - pr->lam / (double)pl->n3[k] * c0[s]);
                for (int r = 0; r < J1; ++r)
                    for (int q = 0; q < J2; ++q)
                        for (int s = 0; s < J3; ++s) {
                            const int64_t g = ((int64_t)r * J2 + q) * J3 + s;
                            G[g] = G0[g] + eta * (err * a0[r] * b0[q] * c0[s] - pr->lam / (double)pr->nnz * G0[g]);
                        }
            } else {
                const int64_t e = id - pr->nnz;
                const double w = pr->ew ? pr->ew[e] : 1.0, al = pr->lr * pr->lam_g * w;
                double *bu = B + (int64_t)pr->eu[e] * J2, *bv = B + (int64_t)pr->ev[e] * J2;
                for (int q = 0; q < J2; ++q) {
                    const double d = bu[q] - bv[q];
                    bu[q] -= al * d;
                    bv[q] += al * d;
                }
            }
        }
        double r = 0.0;
        double f = oracle_loss(pr, A, B, C, G, &r, NULL);
        if (loss) loss[ep - start_epoch] = f;
        if (rmse) rmse[ep - start_epoch] = r;
    }
done:
    free(items); free(wa); free(wb); free(wc); free(a0); free(b0); free(c0); free(G0);
    oracle_plan_free(pl);
    return rc;
}

/* Export the plan for cross-checks: perm1[I1], perm2[I2], order[nnz] (ids in
 * plan order), tile_start[ntiles+1] (needs room for nnz+1), block_tile[P*P+1],
 * strata[P] = stratum order of `epoch`.  *ntiles receives the tile count. */
int oracle_plan_export(const oracle_problem *pr, int32_t epoch, int32_t *perm1, int32_t *perm2,
                       int64_t *order, int64_t *tile_start, int64_t *block_tile, int32_t *strata,
                       int64_t *ntiles)
{
    oracle_plan_t *pl = NULL;
    int rc = oracle_plan_build(pr, &pl);
    if (rc) return rc;
    const int64_t P = pr->P;
    if (perm1) memcpy(perm1, pl->perm1, sizeof(int32_t) * pr->I1);
    if (perm2) memcpy(perm2, pl->perm2, sizeof(int32_t) * pr->I2);
    if (order) memcpy(order, pl->order, sizeof(int64_t) * pr->nnz);
    if (tile_start) memcpy(tile_start, pl->tile_start, sizeof(int64_t) * (pl->ntiles + 1));
    if (block_tile) memcpy(block_tile, pl->block_tile, sizeof(int64_t) * (P * P + 1));
    if (strata) {
        for (int64_t s = 0; s < P; ++s) strata[s] = (int32_t)s;
        oracle_shuffle(strata, P, pr->seed, 2 + (uint64_t)epoch);
    }
    if (ntiles) *ntiles = pl->ntiles;
    oracle_plan_free(pl);
    return ORC_OK;
}

/* Default random start of Algorithm 1 (its first step initialises the
 * factors randomly; the paper names no distribution).  Reading: every entry
 * of A, B, C and G, in that order and each row-major, is drawn i.i.d. from
 * N(0, sigma^2) with sigma = (mean of x^2 / (J1 J2 J3))^(1/8), so that a
 * model value, a sum of J1 J2 J3 products of four such entries, starts with
 * the second moment of the data; sigma = 1 when there are no nonzeros or
 * every value is 0.  Normal deviates by the Box-Muller transform (Box &
 * Muller, Ann. Math. Statist. 29, 1958): a pair of uniforms (u1, u2) on
 * (0, 1) gives sqrt(-2 ln u1) cos(2 pi u2), then sqrt(-2 ln u1) sin(2 pi u2).
 * Uniforms take the top 53 bits of consecutive 64-bit draws r of stream
 * 2^40 of the seed, u = (floor(r / 2^11) + 1/2) 2^-53. */
#define ORC_INIT_STREAM (1ULL << 40)

void oracle_random_start(const oracle_problem *pr, double *A, double *B, double *C, double *G)
{
    double ss = 0.0;
    for (int64_t t = 0; t < pr->nnz; ++t) ss += pr->x[t] * pr->x[t];
    const double ms = pr->nnz > 0 ? ss / (double)pr->nnz : 0.0;
    const double sigma = ms > 0.0 ? pow(ms / ((double)pr->J1 * pr->J2 * pr->J3), 0.125) : 1.0;
    const int64_t nA = (int64_t)pr->I1 * pr->J1, nB = (int64_t)pr->I2 * pr->J2;
    const int64_t nC = (int64_t)pr->I3 * pr->J3, nG = (int64_t)pr->J1 * pr->J2 * pr->J3;
    double *out[4] = {A, B, C, G};
    const int64_t len[4] = {nA, nB, nC, nG};
    uint64_t st = oracle_stream_state(pr->seed, ORC_INIT_STREAM);
    const double pi = 3.14159265358979323846264338327950288;
    int part = 0;
    int64_t at = 0;
    const int64_t n = nA + nB + nC + nG;
    for (int64_t t = 0; t < n; t += 2) {
        const double u1 = ((double)(orc_sm64(&st) >> 11) + 0.5) / 9007199254740992.0;
        const double u2 = ((double)(orc_sm64(&st) >> 11) + 0.5) / 9007199254740992.0;
        const double rad = sqrt(-2.0 * log(u1));
        const double z[2] = {rad * cos(2.0 * pi * u2), rad * sin(2.0 * pi * u2)};
        for (int h = 0; h < 2 && t + h < n; ++h) {
            while (at >= len[part]) { ++part; at = 0; }
            out[part][at++] = sigma * z[h];
        }
    }
}

int oracle_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
