/*
 * FUnc-SNE CPU oracle -- TEST INFRASTRUCTURE ONLY (see fsne_oracle.h).
 *
 * Plain double-precision C.  Loops over points may run under OpenMP; every
 * point writes only its own outputs and reads a snapshot of the state, so the
 * result does not depend on the thread count.  Sums over points run in index
 * order on one thread.
 *
 * Build: gcc -O2 -std=c11 -fopenmp -ffp-contract=off -shared -fPIC
 * (contraction stays off so that the one single-precision decision, the
 * clustering's eps test, is exactly the stated operation sequence).
 */
#include "fsne_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------------ */
/* Counter-based generator: Philox4x32 with 10 rounds (Salmon, Moraes, Dror, */
/* Shaw, "Parallel random numbers: as easy as 1, 2, 3", SC 2011).  A round   */
/* multiplies counter words 0 and 2 by two fixed odd constants, and the new  */
/* counter is (hi(c2*M1) ^ c1 ^ k0, lo(c2*M1), hi(c0*M0) ^ c3 ^ k1,          */
/* lo(c0*M0)); the key is bumped by two Weyl constants between rounds.       */
/* ------------------------------------------------------------------------ */
void fsneo_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
    const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += W0;
            k1 += W1;
        }
        uint64_t p0 = (uint64_t)M0 * c0;
        uint64_t p1 = (uint64_t)M1 * c2;
        uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
        uint32_t n1 = (uint32_t)p1;
        uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
        uint32_t n3 = (uint32_t)p0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* Draw block for (point, iteration, stream, slot) under key = seed. */
static void draw(uint64_t seed, uint32_t i, uint32_t t, uint32_t stream, uint32_t slot,
                 uint32_t out[4])
{
    uint32_t ctr[4] = {i, t, stream, slot};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    fsneo_philox4x32_10(ctr, key, out);
}

/* floor(u * K / 2^32): a uniform index in [0, K). */
static int64_t uniform_index(uint32_t u, int64_t K)
{
    return (int64_t)(((uint64_t)u * (uint64_t)K) >> 32);
}

/* A uniform point of {0..N-1} other than i. */
static int64_t uniform_other(uint32_t u, int64_t i, int64_t N)
{
    int64_t j = uniform_index(u, N - 1);
    return j + (j >= i);
}

/* ------------------------------------------------------------------------ */
/* Refinement probability (Sec. 3, paragraph on skipping the HD refinement): */
/* p = p_min + (1 - p_min) E with the paper's p_min = 0.05.  The iteration   */
/* refines when its 32-bit draw u satisfies u < p 2^32, compared in double   */
/* (u is an integer below 2^32 and scaling p by 2^32 is exact).              */
/* ------------------------------------------------------------------------ */
static uint32_t coin_draw(uint32_t t, uint64_t seed)
{
    uint32_t u[4];
    draw(seed, 0xFFFFFFFFu, t, FSNEO_S_COIN, 0, u);
    return u[0];
}

int fsneo_coin(double E, uint32_t t, uint64_t seed, int32_t hd_mode, double p_min)
{
    if (hd_mode == 1) return 1;
    if (hd_mode == 2) return 0;
    double p = p_min + (1.0 - p_min) * E;
    if (p >= 1.0) return 1;
    if (p <= 0.0) return 0;
    return (double)coin_draw(t, seed) < p * 4294967296.0;
}

/* u - p 2^32 for iteration t: how far the draw lies from the threshold (a  */
/* single-precision implementation of the same rule can only decide          */
/* otherwise when this is within its rounding of p 2^32).                    */
double fsneo_coin_margin(double E, uint32_t t, uint64_t seed, double p_min)
{
    double p = p_min + (1.0 - p_min) * E;
    return (double)coin_draw(t, seed) - p * 4294967296.0;
}

/* E <- (1 - lambda) E + lambda N_new / N. */
double fsneo_E_next(double E, int64_t n_new, int64_t N, double lam)
{
    return (1.0 - lam) * E + lam * (double)n_new / (double)N;
}

/* ------------------------------------------------------------------------ */
/* Distances.                                                                */
/* ------------------------------------------------------------------------ */
static double xval(const void *X, int32_t xdtype, int64_t k)
{
    if (xdtype == 0) return (double)((const float *)X)[k];
    uint32_t u = (uint32_t)((const uint16_t *)X)[k] << 16;
    float f;
    memcpy(&f, &u, sizeof f);
    return (double)f;
}

/* Squared Euclidean HD distance delta_ij^2 (Sec. 2.2), in double. */
double fsneo_hd_dist2(const void *X, int32_t xdtype, int32_t D, int64_t a, int64_t b)
{
    double s = 0.0;
    for (int32_t k = 0; k < D; ++k) {
        double v = xval(X, xdtype, a * D + k) - xval(X, xdtype, b * D + k);
        s += v * v;
    }
    return s;
}

/* HD distance of either metric (the paper names the HD metric as a setting  */
/* that can change during optimisation, Sec. 3).  metric 0: the squared      */
/* Euclidean distance.  metric 1 (angular): the squared Euclidean distance   */
/* between the rows scaled to unit length, sum_k (x_k/|x| - y_k/|y|)^2,      */
/* which is 2 (1 - cos) of the angle between them; a zero row stays zero.    */
/* The affinities of eq. (1) take this value in place of delta^2.            */
double fsneo_hd_dist2_metric(const void *X, int32_t xdtype, int32_t D, int32_t metric,
                             int64_t a, int64_t b)
{
    if (metric == 0) return fsneo_hd_dist2(X, xdtype, D, a, b);
    double na = 0.0, nb = 0.0;
    for (int32_t k = 0; k < D; ++k) {
        double u = xval(X, xdtype, a * D + k), v = xval(X, xdtype, b * D + k);
        na += u * u;
        nb += v * v;
    }
    double sa = na > 0.0 ? 1.0 / sqrt(na) : 0.0, sb = nb > 0.0 ? 1.0 / sqrt(nb) : 0.0;
    double s = 0.0;
    for (int32_t k = 0; k < D; ++k) {
        double v = xval(X, xdtype, a * D + k) * sa - xval(X, xdtype, b * D + k) * sb;
        s += v * v;
    }
    return s;
}

static double state_dist2(const fsneo_state *S, int64_t a, int64_t b)
{
    return fsneo_hd_dist2_metric(S->X, S->xdtype, S->D, S->metric, a, b);
}

/* Squared distance of the clustering's eps test: single precision on the  */
/* single-precision coordinates, summed over c in index order, each         */
/* operation rounded, no fused multiply-add.                                */
static float cluster_dist2(const double *Y, int32_t d, int64_t i, int64_t j)
{
    volatile float acc = 0.0f;
    for (int32_t c = 0; c < d; ++c) {
        volatile float diff = (float)Y[j * d + c] - (float)Y[i * d + c];
        volatile float sq = diff * diff;
        acc = acc + sq;
    }
    return acc;
}

/* Squared LD distance |y_i - y_j|^2 (the distance of eq. (4)), in double.  */
/* It both decides LD list membership and enters the kernel.                */
static double ld_dist2(const double *Y, int32_t d, int64_t i, int64_t j)
{
    double s = 0.0;
    for (int32_t c = 0; c < d; ++c) {
        double v = Y[i * d + c] - Y[j * d + c];
        s += v * v;
    }
    return s;
}

/* ------------------------------------------------------------------------ */
/* Sorted key lists: ascending squared distance, ties broken by index.       */
/* ------------------------------------------------------------------------ */
typedef struct {
    double key;
    int64_t idx;
} entry;

static int entry_less(const entry *a, const entry *b)
{
    if (a->key < b->key) return 1;
    if (a->key > b->key) return 0;
    return a->idx < b->idx;
}

static void sort_entries(entry *e, int n)
{
    for (int a = 1; a < n; ++a) {
        entry v = e[a];
        int b = a - 1;
        while (b >= 0 && entry_less(&v, &e[b])) {
            e[b + 1] = e[b];
            --b;
        }
        e[b + 1] = v;
    }
}

static int contains(const int32_t *list, int n, int64_t v)
{
    for (int k = 0; k < n; ++k)
        if (list[k] == v) return 1;
    return 0;
}

static int contains64(const int64_t *list, int n, int64_t v)
{
    for (int k = 0; k < n; ++k)
        if (list[k] == v) return 1;
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Bandwidth calibration (eq. (1), Sec. 2.2): beta_i = 1/(2 sigma_i^2) is    */
/* set so that the entropy of p_{.|i}, restricted to the row's HD            */
/* neighbours, equals ln(perplexity).  With e_k = exp(-beta (d2_k - m)):     */
/*   H(beta) = ln S + beta sum_k p_k (d2_k - m),  p_k = e_k / S.             */
/* H decreases strictly from ln K (beta = 0) towards ln(#ties at the        */
/* minimum), so the root is unique; it is found by bracketing and bisection */
/* in double.  With #ties >= perplexity H never reaches the target at a     */
/* finite beta: then beta = 1e30 (the row is uniform over the ties).         */
/* out = {beta, m, r, invS}.  Returns 1 when the row has no root.            */
/* ------------------------------------------------------------------------ */
static double row_entropy(const double *d2, int32_t K, double m, double beta, double *S_out)
{
    double S = 0.0, T = 0.0;
    for (int32_t k = 0; k < K; ++k) {
        double e = exp(-beta * (d2[k] - m));
        S += e;
        T += e * (d2[k] - m);
    }
    if (S_out) *S_out = S;
    return log(S) + beta * T / S;
}

static int32_t count_ties(const double *d2, int32_t K, double m)
{
    int32_t n = 0;
    for (int32_t k = 0; k < K; ++k) n += d2[k] == m;
    return n;
}

int fsneo_calibrate(const double *d2, int32_t K, double perplexity, double out[4])
{
    const double beta_max = 1e30;
    double m = d2[0], r = d2[0];
    for (int32_t k = 1; k < K; ++k) {
        if (d2[k] < m) m = d2[k];
        if (d2[k] > r) r = d2[k];
    }
    double target = log(perplexity);
    double beta, S;
    int noroot = 0;
    if (!(r > m)) {
        beta = 0.0; /* all distances equal: the row is uniform for every beta */
        noroot = !(log((double)K) <= target);
    } else if (count_ties(d2, K, m) >= perplexity) {
        beta = beta_max;
        noroot = 1;
    } else {
        double lo = 0.0, hi = 1.0;
        while (row_entropy(d2, K, m, hi, NULL) > target) {
            lo = hi;
            hi *= 2.0;
        }
        for (int it = 0; it < 400 && hi - lo > 1e-15 * hi; ++it) {
            double mid = 0.5 * (lo + hi);
            if (row_entropy(d2, K, m, mid, NULL) > target)
                lo = mid;
            else
                hi = mid;
        }
        beta = 0.5 * (lo + hi);
    }
    row_entropy(d2, K, m, beta, &S);
    out[0] = beta;
    out[1] = m;
    out[2] = r;
    out[3] = 1.0 / S;
    return noroot;
}

static void calibrate_point(fsneo_state *S, int64_t i, double perplexity)
{
    double rec[4];
    fsneo_calibrate(S->hd_d2 + i * S->K_hd, S->K_hd, perplexity, rec);
    S->beta[i] = rec[0];
    S->m[i] = rec[1];
    S->r[i] = rec[2];
    S->invS[i] = rec[3];
}

/* ------------------------------------------------------------------------ */
/* Symmetrised sparse affinities (eq. (1)), with both conditionals taken    */
/* over the approximate HD neighbour sets.  For j = HD list of i, entry k:  */
/*   p_{j|i} = exp(-beta_i (d2_ij - m_i)) invS_i                              */
/*   p_{i|j} = exp(-beta_j (d2_ij - m_j)) invS_j  if i is in j's HD list,     */
/*             0 otherwise                                                    */
/*   P_ik    = (p_{j|i} + p_{i|j}) / (2N)                                     */
/* Pairs where only i is in j's list (not j in i's) do not act on i.         */
/* ------------------------------------------------------------------------ */
static void psym_row_from(int64_t i, const int32_t *idx, const double *d2, int32_t K, int64_t N,
                          const double rec_i[4], const int32_t *const *rows_j,
                          const double *const *rec_j, double *out)
{
    for (int32_t k = 0; k < K; ++k) {
        double pji = exp(-rec_i[0] * (d2[k] - rec_i[1])) * rec_i[3];
        double pij = 0.0;
        if (contains(rows_j[k], K, i)) pij = exp(-rec_j[k][0] * (d2[k] - rec_j[k][1])) * rec_j[k][3];
        out[k] = (pji + pij) / (2.0 * (double)N);
        (void)idx;
    }
}

void fsneo_psym_row(const fsneo_state *S, int64_t i, double *out)
{
    const int32_t K = S->K_hd;
    const int32_t *rows[FSNEO_KMAX];
    double recs[FSNEO_KMAX][4];
    const double *recp[FSNEO_KMAX];
    for (int32_t k = 0; k < K; ++k) {
        int64_t j = S->hd_idx[i * K + k];
        rows[k] = S->hd_idx + j * K;
        recs[k][0] = S->beta[j]; recs[k][1] = S->m[j];
        recs[k][2] = S->r[j]; recs[k][3] = S->invS[j];
        recp[k] = recs[k];
    }
    double rec_i[4] = {S->beta[i], S->m[i], S->r[i], S->invS[i]};
    psym_row_from(i, S->hd_idx + i * K, S->hd_d2 + i * K, K, S->N, rec_i, rows, recp, out);
}

/* ------------------------------------------------------------------------ */
/* Candidate generation (Sec. 3, interleaved KNN refinement): neighbours of  */
/* neighbours in the list's own space, neighbours and neighbours of          */
/* neighbours in the other space, and uniform random points.  Slot s of      */
/* point i at iteration t draws the block (i, t, stream, s).                 */
/* ------------------------------------------------------------------------ */
/* Rows of a neighbour list, either a full N x K array or a few rows by id. */
typedef struct {
    const int32_t *full;   /* N x K, or NULL                                   */
    int32_t K;
    int n;                 /* number of sparse rows                             */
    const int64_t *ids;    /* ids of the sparse rows                            */
    const int32_t *rows;   /* n x K                                             */
} rows_t;

static const int32_t *row_of(const rows_t *L, int64_t j)
{
    if (L->full) return L->full + j * L->K;
    for (int k = 0; k < L->n; ++k)
        if (L->ids[k] == j) return L->rows + (int64_t)k * L->K;
    abort(); /* a row outside the dependency set was read */
}

static int64_t candidate(int s, const uint32_t u[4], int64_t i, const rows_t *L,
                         const rows_t *Lx, int64_t N)
{
    const int32_t K = L->K, Kx = Lx->K;
    if (s < FSNEO_SAME_NON) {
        int64_t j = row_of(L, i)[uniform_index(u[0], K)];
        return row_of(L, j)[uniform_index(u[1], K)];
    }
    if (s < FSNEO_SAME_NON + FSNEO_CROSS_DIR) return row_of(Lx, i)[uniform_index(u[0], Kx)];
    if (s < FSNEO_SAME_NON + FSNEO_CROSS_DIR + FSNEO_CROSS_NON) {
        int64_t j = row_of(Lx, i)[uniform_index(u[0], Kx)];
        return row_of(Lx, j)[uniform_index(u[1], Kx)];
    }
    return uniform_other(u[0], i, N);
}

/* Candidates of point i, with those equal to i, already in i's list, or     */
/* equal to an earlier slot removed (removed slots are not redrawn).         */
static int gather_candidates(int64_t i, uint32_t t, uint32_t stream, uint64_t seed,
                             const rows_t *L, const rows_t *Lx, int64_t N,
                             int64_t cand[FSNEO_C])
{
    int nc = 0;
    const int32_t *own = row_of(L, i);
    for (int s = 0; s < FSNEO_C; ++s) {
        uint32_t u[4];
        draw(seed, (uint32_t)i, t, stream, (uint32_t)s, u);
        int64_t c = candidate(s, u, i, L, Lx, N);
        if (c == i || contains(own, L->K, c) || contains64(cand, nc, c)) continue;
        cand[nc++] = c;
    }
    return nc;
}

/* ------------------------------------------------------------------------ */
/* HD refinement of one point: merge the candidates into the sorted HD list, */
/* keep the K_hd closest; changed = some candidate entered the list.         */
/* ------------------------------------------------------------------------ */
void fsneo_hd_refine_point(const fsneo_state *S, int64_t i, uint32_t t, int32_t *idx_out,
                           double *d2_out, uint8_t *changed)
{
    const int32_t K = S->K_hd;
    int64_t cand[FSNEO_C];
    rows_t L = {S->hd_idx, K, 0, NULL, NULL}, Lx = {S->ld_idx, S->K_ld, 0, NULL, NULL};
    int nc = gather_candidates(i, t, FSNEO_S_HDC, S->seed, &L, &Lx, S->N, cand);
    entry e[FSNEO_KMAX + FSNEO_C];
    for (int32_t k = 0; k < K; ++k) {
        e[k].key = S->hd_d2[i * K + k];
        e[k].idx = S->hd_idx[i * K + k];
    }
    for (int c = 0; c < nc; ++c) {
        e[K + c].key = state_dist2(S, i, cand[c]);
        e[K + c].idx = cand[c];
    }
    sort_entries(e, K + nc);
    uint8_t ch = 0;
    for (int32_t k = 0; k < K; ++k) {
        ch |= (uint8_t)contains64(cand, nc, e[k].idx);
        idx_out[k] = (int32_t)e[k].idx;
        d2_out[k] = e[k].key;
    }
    *changed = ch;
}

/* ------------------------------------------------------------------------ */
/* LD refinement and gradient partials of one point (eqs. (4)-(6); the split */
/* of attraction and repulsion of Sec. 3).  hd_next / P_next are the HD list */
/* rows and i's affinity row after this iteration's HD phase.               */
/*   w      = (1 + d^2/alpha)^(-alpha)     w^(1/alpha) = 1 / (1 + d^2/alpha)  */
/*   A_i    = sum_{k} P_ik w^(1/a) (y_i - y_j)            j over the HD list  */
/*   R_i    = sum_{j in U} w^(1+1/a) (y_i - y_j) + negatives                  */
/*   Zh_i   = sum_{j in U} w + negatives                                      */
/* U = HD list union new LD list.  Each of the n_neg negatives is a uniform  */
/* other point; one that falls in U adds nothing, the rest are weighted      */
/* (N-1)/n_neg so that the sum is unbiased for the terms outside U.          */
/* ------------------------------------------------------------------------ */
static void ld_point(const fsneo_state *S, const fsneo_hp *hp, int64_t i, uint32_t t,
                     const rows_t *hd_next, const double *P_row, int32_t *ld_out, double *A,
                     double *R, double *Zh)
{
    const int32_t K = S->K_ld, Kh = S->K_hd, d = S->d;
    const double alpha = hp->alpha;
    int64_t cand[FSNEO_C];
    rows_t L = {S->ld_idx, K, 0, NULL, NULL};
    int nc = gather_candidates(i, t, FSNEO_S_LDC, S->seed, &L, hd_next, S->N, cand);
    entry e[FSNEO_KMAX + FSNEO_C];
    for (int32_t k = 0; k < K; ++k) {
        e[k].idx = S->ld_idx[i * K + k];
        e[k].key = ld_dist2(S->Y, d, i, e[k].idx);
    }
    for (int c = 0; c < nc; ++c) {
        e[K + c].idx = cand[c];
        e[K + c].key = ld_dist2(S->Y, d, i, cand[c]);
    }
    sort_entries(e, K + nc);
    for (int32_t k = 0; k < K; ++k) ld_out[k] = (int32_t)e[k].idx;

    for (int32_t c = 0; c < d; ++c) A[c] = R[c] = 0.0;
    *Zh = 0.0;
    const int32_t *hl = row_of(hd_next, i);
    const double *yi = S->Y + i * d;
    /* attraction over the HD list, and the HD part of U */
    for (int32_t k = 0; k < Kh; ++k) {
        int64_t j = hl[k];
        double q2 = ld_dist2(S->Y, d, i, j);
        double wa = 1.0 / (1.0 + q2 / alpha);
        double w = pow(1.0 + q2 / alpha, -alpha);
        for (int32_t c = 0; c < d; ++c) {
            double dy = yi[c] - S->Y[j * d + c];
            A[c] += P_row[k] * wa * dy;
            R[c] += w * wa * dy;
        }
        *Zh += w;
    }
    /* LD neighbours that are not HD neighbours */
    for (int32_t k = 0; k < K; ++k) {
        int64_t j = ld_out[k];
        if (contains(hl, Kh, j)) continue;
        double q2 = ld_dist2(S->Y, d, i, j);
        double wa = 1.0 / (1.0 + q2 / alpha);
        double w = pow(1.0 + q2 / alpha, -alpha);
        for (int32_t c = 0; c < d; ++c) R[c] += w * wa * (yi[c] - S->Y[j * d + c]);
        *Zh += w;
    }
    /* negative samples for the rest */
    if (hp->n_neg > 0) {
        double scale = (double)(S->N - 1) / (double)hp->n_neg;
        for (int s = 0; s < hp->n_neg; ++s) {
            uint32_t u[4];
            draw(S->seed, (uint32_t)i, t, FSNEO_S_NEG, (uint32_t)s, u);
            int64_t j = uniform_other(u[0], i, S->N);
            if (contains(hl, Kh, j) || contains(ld_out, K, j)) continue;
            double q2 = ld_dist2(S->Y, d, i, j);
            double wa = 1.0 / (1.0 + q2 / alpha);
            double w = pow(1.0 + q2 / alpha, -alpha);
            for (int32_t c = 0; c < d; ++c) R[c] += scale * w * wa * (yi[c] - S->Y[j * d + c]);
            *Zh += scale * w;
        }
    }
}

void fsneo_ld_refine_grad_point(const fsneo_state *S, const fsneo_hp *hp, int64_t i, uint32_t t,
                                const int32_t *hd_next, const double *P_next, int32_t *ld_out,
                                double *A, double *R, double *Zh)
{
    rows_t H = {hd_next, S->K_hd, 0, NULL, NULL};
    ld_point(S, hp, i, t, &H, P_next + i * S->K_hd, ld_out, A, R, Zh);
}

/* ------------------------------------------------------------------------ */
/* Initial state: for each point, the first K distinct other points drawn    */
/* from the INIT streams (after 64K draws, the next indices i+1, i+2, ...    */
/* fill the rest); HD lists sorted by distance; every point calibrated;      */
/* E = 1 so the first iteration refines the HD lists; V = 0; t = 0.          */
/* ------------------------------------------------------------------------ */
/* out[0..n_have) already holds list ids; fill up to K with the first      */
/* distinct other points among the draws (i, t, stream, s), s = 0, 1, ...  */
/* < 64K, then the next indices i+1, i+2, ... (initial lists: t = 0 and    */
/* n_have = 0).                                                             */
static void random_list(int64_t i, int64_t N, int32_t K, uint32_t stream, uint32_t t,
                        uint64_t seed, int32_t *out, int n_have)
{
    int n = n_have;
    for (uint32_t s = 0; n < K && s < 64u * (uint32_t)K; ++s) {
        uint32_t u[4];
        draw(seed, (uint32_t)i, t, stream, s, u);
        int64_t c = uniform_other(u[0], i, N);
        if (!contains(out, n, c)) out[n++] = (int32_t)c;
    }
    for (int64_t c = (i + 1) % N; n < K; c = (c + 1) % N)
        if (c != i && !contains(out, n, c)) out[n++] = (int32_t)c;
}

static void init_point_lists(fsneo_state *S, int64_t i, int64_t N)
{
    const int32_t K = S->K_hd;
    random_list(i, N, K, FSNEO_S_INIT_HD, 0, S->seed, S->hd_idx + i * K, 0);
    random_list(i, N, S->K_ld, FSNEO_S_INIT_LD, 0, S->seed, S->ld_idx + i * S->K_ld, 0);
    entry e[FSNEO_KMAX];
    for (int32_t k = 0; k < K; ++k) {
        e[k].idx = S->hd_idx[i * K + k];
        e[k].key = state_dist2(S, i, e[k].idx);
    }
    sort_entries(e, K);
    for (int32_t k = 0; k < K; ++k) {
        S->hd_idx[i * K + k] = (int32_t)e[k].idx;
        S->hd_d2[i * K + k] = e[k].key;
    }
}

static void all_psym(fsneo_state *S)
{
    const int64_t N = S->N;
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t i = 0; i < N; ++i) fsneo_psym_row(S, i, S->P + i * S->K_hd);
}

int fsneo_init(fsneo_state *S, const fsneo_hp *hp)
{
    const int64_t N = S->N;
    if (S->K_hd < 2 || S->K_hd > FSNEO_KMAX || S->K_ld < 1 || S->K_ld > FSNEO_KMAX ||
        S->K_hd >= N ||
        S->K_ld >= N || S->d < 1 || S->d > 64)
        return -1;
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t i = 0; i < N; ++i) {
        init_point_lists(S, i, N);
        calibrate_point(S, i, hp->perplexity);
        S->flags[i] = 1;
    }
    all_psym(S);
    for (int64_t k = 0; k < N * S->d; ++k) S->V[k] = 0.0;
    *S->E = 1.0;
    *S->t = 0;
    return 0;
}

/* ------------------------------------------------------------------------ */
/* The end of the HD phase (Sec. 3, flags paragraph; eq. (1)): the points   */
/* whose list changed (flag set) are recalibrated, then P is recomputed for */
/* every point from the new lists and records.                              */
/* ------------------------------------------------------------------------ */
void fsneo_hd_finish(fsneo_state *S, const fsneo_hp *hp)
{
    const int64_t N = S->N;
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t i = 0; i < N; ++i)
        if (S->flags[i]) calibrate_point(S, i, hp->perplexity);
    all_psym(S);
}

/* The LD phase of every point (LD refinement at the current Y and gradient */
/* partials) against given HD lists and affinities of this iteration.       */
void fsneo_ld_phase(const fsneo_state *S, const fsneo_hp *hp, uint32_t t, const int32_t *hd_next,
                    const double *P_next, int32_t *ld_out, double *A, double *R, double *Zh)
{
    const int64_t N = S->N;
    const int32_t Kl = S->K_ld, d = S->d;
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t i = 0; i < N; ++i)
        fsneo_ld_refine_grad_point(S, hp, i, t, hd_next, P_next, ld_out + i * Kl, A + i * d,
                                   R + i * d, Zh + i);
}

/* ------------------------------------------------------------------------ */
/* One iteration, in this order (Sec. 3): coin; if it fires, refine every HD */
/* list from the current HD and LD lists, recalibrate the points whose list  */
/* changed (their flags), recompute P; refine every LD list at the current  */
/* Y from the current LD list and the new HD list; gradient partials; Z;    */
/* g = 4 (attr A - rep R / Z); V <- momentum V - lr g; Y <- Y + V; update E */
/* after an HD refinement; t <- t + 1.  Every phase reads the state as it   */
/* was before the phase.                                                     */
/* ------------------------------------------------------------------------ */
int fsneo_step(fsneo_state *S, const fsneo_hp *hp, fsneo_stats *st, double *A_out,
               double *R_out, double *Zh_out)
{
    const int64_t N = S->N;
    const int32_t Kh = S->K_hd, Kl = S->K_ld, d = S->d;
    const uint32_t t = *S->t;
    int fired = fsneo_coin(*S->E, t, S->seed, hp->hd_mode, hp->p_min);
    int64_t n_new = 0;
    if (fired) {
        int32_t *ni = malloc(sizeof(int32_t) * N * Kh);
        double *nd = malloc(sizeof(double) * N * Kh);
        if (!ni || !nd) {
            free(ni);
            free(nd);
            return -2;
        }
#pragma omp parallel for schedule(dynamic, 256)
        for (int64_t i = 0; i < N; ++i)
            fsneo_hd_refine_point(S, i, t, ni + i * Kh, nd + i * Kh, S->flags + i);
        memcpy(S->hd_idx, ni, sizeof(int32_t) * N * Kh);
        memcpy(S->hd_d2, nd, sizeof(double) * N * Kh);
        free(ni);
        free(nd);
        for (int64_t i = 0; i < N; ++i) n_new += S->flags[i];
        fsneo_hd_finish(S, hp);
    }
    int32_t *nl = malloc(sizeof(int32_t) * N * Kl);
    double *A = malloc(sizeof(double) * N * d);
    double *R = malloc(sizeof(double) * N * d);
    double *Zh = malloc(sizeof(double) * N);
    if (!nl || !A || !R || !Zh) {
        free(nl);
        free(A);
        free(R);
        free(Zh);
        return -2;
    }
    fsneo_ld_phase(S, hp, t, S->hd_idx, S->P, nl, A, R, Zh);
    double Z = 0.0;
    for (int64_t i = 0; i < N; ++i) Z += Zh[i];
    for (int64_t k = 0; k < N * d; ++k) {
        double g = 4.0 * (hp->attr * A[k] - hp->rep * R[k] / Z);
        S->V[k] = hp->momentum * S->V[k] - hp->lr * g;
        S->Y[k] += S->V[k];
    }
    memcpy(S->ld_idx, nl, sizeof(int32_t) * N * Kl);
    if (A_out) memcpy(A_out, A, sizeof(double) * N * d);
    if (R_out) memcpy(R_out, R, sizeof(double) * N * d);
    if (Zh_out) memcpy(Zh_out, Zh, sizeof(double) * N);
    free(nl);
    free(A);
    free(R);
    free(Zh);
    if (fired) *S->E = fsneo_E_next(*S->E, n_new, N, hp->e_smooth);
    *S->t = t + 1;
    if (st) {
        st->fired = fired;
        st->n_new = n_new;
        st->Z = Z;
        st->E = *S->E;
        st->t = *S->t;
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* The same iteration for one point i, for checks at sizes where the full   */
/* step is too slow.  It refines i and the members of i's new HD list (their */
/* records and HD lists feed i's affinities and LD candidates), then i's LD  */
/* phase.  Outputs are i's: new HD row, flag, record {beta, m, r, invS},     */
/* P row, new LD row and gradient partials.  Z is not formed.                */
/* ------------------------------------------------------------------------ */
typedef struct {
    int32_t idx[FSNEO_KMAX];
    double d2[FSNEO_KMAX];
    double rec[4];
} point_next;

/* Planted mistakes, compiled in only by the test which shows that comparing */
/* fsneo_point_step with fsneo_step catches them (0: none).  1: a changed    */
/* neighbour keeps its old record; 2: the LD phase reads the neighbours'     */
/* HD rows from before the refinement; 3: the affinities test membership in  */
/* the neighbours' old rows; 4: i's affinities use its own old record.     */
#ifndef FSNEO_PLANT
#define FSNEO_PLANT 0
#endif

/* HD row and record of point j after the HD phase; returns j's flag. */
static uint8_t next_of(const fsneo_state *S, const fsneo_hp *hp, int64_t j, int32_t fired,
                       point_next *pn)
{
    const int32_t K = S->K_hd;
    uint8_t ch = 0;
    if (fired) {
        fsneo_hd_refine_point(S, j, *S->t, pn->idx, pn->d2, &ch);
    } else {
        memcpy(pn->idx, S->hd_idx + j * K, sizeof(int32_t) * K);
        memcpy(pn->d2, S->hd_d2 + j * K, sizeof(double) * K);
    }
    if (ch && FSNEO_PLANT != 1) {
        fsneo_calibrate(pn->d2, K, hp->perplexity, pn->rec);
    } else {
        pn->rec[0] = S->beta[j];
        pn->rec[1] = S->m[j];
        pn->rec[2] = S->r[j];
        pn->rec[3] = S->invS[j];
    }
    return ch;
}

int fsneo_point_step(const fsneo_state *S, const fsneo_hp *hp, int64_t i, int32_t fired,
                     int32_t *hd_idx_out, double *hd_d2_out, uint8_t *flag_out, double rec_out[4],
                     double *P_out, int32_t *ld_out, double *A, double *R, double *Zh)
{
    const int32_t K = S->K_hd;
    const int64_t N = S->N;
    point_next *pn = malloc(sizeof(point_next) * (size_t)(K + 1));
    int64_t *ids = malloc(sizeof(int64_t) * (size_t)(K + 1));
    int32_t *rows = malloc(sizeof(int32_t) * (size_t)(K + 1) * K);
    if (!pn || !ids || !rows) {
        free(pn); free(ids); free(rows);
        return -2;
    }
    uint8_t ch = next_of(S, hp, i, fired, &pn[0]);
    for (int32_t k = 0; k < K; ++k) next_of(S, hp, pn[0].idx[k], fired, &pn[1 + k]);
    /* affinities of i from the next rows and records of its neighbours */
    {
        const int32_t *rows_j[FSNEO_KMAX] = {0};
        const double *rec_j[FSNEO_KMAX] = {0};
        for (int32_t k = 0; k < K; ++k) {
            rows_j[k] = FSNEO_PLANT == 3 ? S->hd_idx + (int64_t)pn[0].idx[k] * K : pn[1 + k].idx;
            rec_j[k] = pn[1 + k].rec;
        }
        double rec_old[4] = {S->beta[i], S->m[i], S->r[i], S->invS[i]};
        psym_row_from(i, pn[0].idx, pn[0].d2, K, N, FSNEO_PLANT == 4 ? rec_old : pn[0].rec,
                      rows_j, rec_j, P_out);
    }
    /* the LD phase of i reads the next HD rows of i and of its members only */
    ids[0] = i;
    memcpy(rows, pn[0].idx, sizeof(int32_t) * K);
    for (int32_t k = 0; k < K; ++k) {
        ids[1 + k] = pn[0].idx[k];
        memcpy(rows + (int64_t)(1 + k) * K,
               FSNEO_PLANT == 2 ? S->hd_idx + (int64_t)pn[0].idx[k] * K : pn[1 + k].idx,
               sizeof(int32_t) * K);
    }
    rows_t H = {NULL, K, K + 1, ids, rows};
    ld_point(S, hp, i, *S->t, &H, P_out, ld_out, A, R, Zh);
    memcpy(hd_idx_out, pn[0].idx, sizeof(int32_t) * K);
    memcpy(hd_d2_out, pn[0].d2, sizeof(double) * K);
    *flag_out = ch;
    memcpy(rec_out, pn[0].rec, sizeof(double) * 4);
    free(pn);
    free(ids);
    free(rows);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Dynamic data (Sec. 3, paragraph on online use; Sec. 5).                   */
/* Insert: rows N..N+n-1 of X are already in place; they get Y from the     */
/* caller, V = 0, random lists, calibration and a set flag; N grows; P is   */
/* recomputed for every point (its 1/(2N) factor changed).                   */
/* Drift: rows ids of X already hold the new coordinates; each drifted      */
/* point gets V = 0 and optionally a new y; every HD list entry whose pair   */
/* involves a drifted point has its distance recomputed; affected rows are  */
/* re-sorted, flagged and recalibrated; P is recomputed.                     */
/* ------------------------------------------------------------------------ */
int fsneo_insert(fsneo_state *S, const fsneo_hp *hp, int64_t n_new, const double *Y_new)
{
    const int64_t N0 = S->N, N1 = S->N + n_new;
    const int32_t d = S->d;
    S->N = N1;
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t i = N0; i < N1; ++i) {
        init_point_lists(S, i, N1);
        calibrate_point(S, i, hp->perplexity);
        S->flags[i] = 1;
        for (int32_t c = 0; c < d; ++c) {
            S->Y[i * d + c] = Y_new[(i - N0) * d + c];
            S->V[i * d + c] = 0.0;
        }
    }
    all_psym(S);
    return 0;
}

int fsneo_drift(fsneo_state *S, const fsneo_hp *hp, const int64_t *ids, int64_t n,
                const double *Y_new)
{
    const int64_t N = S->N;
    const int32_t K = S->K_hd, d = S->d;
    uint8_t *moved = calloc((size_t)N, 1);
    if (!moved) return -2;
    for (int64_t k = 0; k < n; ++k) {
        int64_t i = ids[k];
        moved[i] = 1;
        for (int32_t c = 0; c < d; ++c) {
            if (Y_new) S->Y[i * d + c] = Y_new[k * d + c];
            S->V[i * d + c] = 0.0;
        }
    }
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t i = 0; i < N; ++i) {
        int touched = moved[i];
        entry e[FSNEO_KMAX];
        for (int32_t k = 0; k < K; ++k) {
            int64_t j = S->hd_idx[i * K + k];
            e[k].idx = j;
            if (moved[i] || moved[j]) {
                e[k].key = state_dist2(S, i, j);
                touched = 1;
            } else {
                e[k].key = S->hd_d2[i * K + k];
            }
        }
        S->flags[i] = (uint8_t)touched;
        if (!touched) continue;
        sort_entries(e, K);
        for (int32_t k = 0; k < K; ++k) {
            S->hd_idx[i * K + k] = (int32_t)e[k].idx;
            S->hd_d2[i * K + k] = e[k].key;
        }
        calibrate_point(S, i, hp->perplexity);
    }
    all_psym(S);
    free(moved);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Change of the HD metric during optimisation (Sec. 3: the scheme adapts   */
/* to changes of HD-side settings such as the metric).  The lists keep      */
/* their members; every stored distance is recomputed in the new metric,    */
/* each row is re-sorted by (d2, id), flagged and recalibrated, P is        */
/* recomputed, and E restarts at 1: the lists are not yet the new metric's  */
/* neighbours, so the coin refines at once, as at the start.                */
/* ------------------------------------------------------------------------ */
int fsneo_set_metric(fsneo_state *S, const fsneo_hp *hp, int32_t metric)
{
    if (metric < 0 || metric > 1) return -1;
    S->metric = metric;
    const int64_t N = S->N;
    const int32_t K = S->K_hd;
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t i = 0; i < N; ++i) {
        entry e[FSNEO_KMAX];
        for (int32_t k = 0; k < K; ++k) {
            e[k].idx = S->hd_idx[i * K + k];
            e[k].key = state_dist2(S, i, e[k].idx);
        }
        sort_entries(e, K);
        for (int32_t k = 0; k < K; ++k) {
            S->hd_idx[i * K + k] = (int32_t)e[k].idx;
            S->hd_d2[i * K + k] = e[k].key;
        }
        S->flags[i] = 1;
        calibrate_point(S, i, hp->perplexity);
    }
    all_psym(S);
    *S->E = 1.0;
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Point deletion (Sec. 3: points can be removed on the fly).  The caller   */
/* has already compacted the per-point rows (survivors at or beyond the new */
/* N moved into the freed ids below it) and set N; newid maps every old id  */
/* to its new one, or to -1 for a deleted point.  For each survivor i:      */
/*   LD list: surviving entries (new ids) in their order, then refills from */
/*   the draws (i, t, 11, s);                                               */
/*   HD list: if any entry was deleted or renumbered, surviving entries keep */
/*   their distances, refills from the draws (i, t, 10, s) get theirs, the  */
/*   row is sorted by (d2, id), and if an entry was deleted it is          */
/*   recalibrated and flagged.                                              */
/* P is then recomputed for every point.                                    */
/* ------------------------------------------------------------------------ */
void fsneo_delete_fix(fsneo_state *S, const fsneo_hp *hp, const int32_t *newid)
{
    const int64_t N = S->N;
    const int32_t Kh = S->K_hd, Kl = S->K_ld;
    const uint32_t t = *S->t;
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t i = 0; i < N; ++i) {
        int32_t ids[FSNEO_KMAX];
        int nk = 0;
        for (int32_t k = 0; k < Kl; ++k) {
            int32_t nj = newid[S->ld_idx[i * Kl + k]];
            if (nj >= 0) ids[nk++] = nj;
        }
        random_list(i, N, Kl, FSNEO_S_DEL_LD, t, S->seed, ids, nk);
        for (int32_t k = 0; k < Kl; ++k) S->ld_idx[i * Kl + k] = ids[k];

        entry e[FSNEO_KMAX];
        int changed = 0;
        nk = 0;
        for (int32_t k = 0; k < Kh; ++k) {
            int32_t j = S->hd_idx[i * Kh + k], nj = newid[j];
            changed |= nj != j;
            if (nj >= 0) {
                ids[nk] = nj;
                e[nk].idx = nj;
                e[nk].key = S->hd_d2[i * Kh + k];
                ++nk;
            }
        }
        if (!changed) continue;
        random_list(i, N, Kh, FSNEO_S_DEL_HD, t, S->seed, ids, nk);
        for (int32_t k = nk; k < Kh; ++k) {
            e[k].idx = ids[k];
            e[k].key = state_dist2(S, i, ids[k]);
        }
        sort_entries(e, Kh);
        for (int32_t k = 0; k < Kh; ++k) {
            S->hd_idx[i * Kh + k] = (int32_t)e[k].idx;
            S->hd_d2[i * Kh + k] = e[k].key;
        }
        if (nk < Kh) {
            calibrate_point(S, i, hp->perplexity);
            S->flags[i] = 1;
        }
    }
    all_psym(S);
}

/* ------------------------------------------------------------------------ */
/* Clustering for the hierarchy graph (Sec. 4.2): DBSCAN (Ester, Kriegel,   */
/* Sander, Xu 1996) with each point's eps-neighbourhood taken from its LD   */
/* list: N(i) = {i} + {j in L_i : d2(i, j) <= eps^2} (d2 as the LD          */
/* decision distance), core points have |N(i)| >= min_pts, clusters are the */
/* connected components of the core points (linked when either is in the   */
/* other's N), a non-core point within eps of a core point (in either list) */
/* joins the cluster of the nearest one (ties: smaller cluster), the rest   */
/* is noise (-1).  Clusters are numbered 0, 1, ... by the smallest index  */
/* among their core points.  Returns the number of clusters (-2: out of   */
/* memory).                                                                 */
/* ------------------------------------------------------------------------ */
static int64_t uf_find(int64_t *parent, int64_t a)
{
    while (parent[a] != a) {
        parent[a] = parent[parent[a]];
        a = parent[a];
    }
    return a;
}

int32_t fsneo_cluster(const fsneo_state *S, float eps, int32_t min_pts, int32_t *labels)
{
    const int64_t N = S->N;
    const int32_t K = S->K_ld, d = S->d;
    volatile float e = eps;
    const float eps2 = e * e;
    uint8_t *core = calloc((size_t)N, 1);
    int64_t *parent = malloc(sizeof(int64_t) * (size_t)N);
    float *bd = malloc(sizeof(float) * (size_t)N);
    int64_t *bl = malloc(sizeof(int64_t) * (size_t)N);
    int64_t *dense = malloc(sizeof(int64_t) * (size_t)N);
    if (!core || !parent || !bd || !bl || !dense) {
        free(core);
        free(parent);
        free(bd);
        free(bl);
        free(dense);
        return -2;
    }
    for (int64_t i = 0; i < N; ++i) {
        int cnt = 1;
        for (int32_t k = 0; k < K; ++k)
            cnt += cluster_dist2(S->Y, d, i, S->ld_idx[i * K + k]) <= eps2;
        core[i] = cnt >= min_pts;
        parent[i] = i;
    }
    /* union by smaller root: every root is its component's smallest index */
    for (int64_t i = 0; i < N; ++i) {
        if (!core[i]) continue;
        for (int32_t k = 0; k < K; ++k) {
            int64_t j = S->ld_idx[i * K + k];
            if (!core[j] || cluster_dist2(S->Y, d, i, j) > eps2) continue;
            int64_t a = uf_find(parent, i), b = uf_find(parent, j);
            if (a < b) parent[b] = a;
            else if (b < a) parent[a] = b;
        }
    }
    for (int64_t i = 0; i < N; ++i) {
        bd[i] = INFINITY;
        bl[i] = -1;
    }
    for (int64_t i = 0; i < N; ++i)
        for (int32_t k = 0; k < K; ++k) {
            int64_t j = S->ld_idx[i * K + k];
            if (core[i] == core[j]) continue;
            float q = cluster_dist2(S->Y, d, i, j);
            if (q > eps2) continue;
            int64_t border = core[i] ? j : i, owner = core[i] ? i : j;
            int64_t lab = uf_find(parent, owner);
            if (q < bd[border] || (q == bd[border] && lab < bl[border])) {
                bd[border] = q;
                bl[border] = lab;
            }
        }
    int32_t nc = 0;
    for (int64_t i = 0; i < N; ++i) dense[i] = (core[i] && uf_find(parent, i) == i) ? nc++ : -1;
    for (int64_t i = 0; i < N; ++i) {
        int64_t root = core[i] ? uf_find(parent, i) : bl[i];
        labels[i] = root >= 0 ? (int32_t)dense[root] : -1;
    }
    free(core);
    free(parent);
    free(bd);
    free(bl);
    free(dense);
    return nc;
}

/* ------------------------------------------------------------------------ */
/* Jump start (Sec. 3, paragraph on helping the first iterations): the       */
/* embedding becomes a random linear projection of the centred data,        */
/*   y_ic = s sum_k (x_ik - mu_k) r_kc,                                      */
/* r_kc = -1 if bit 0 of the first word of block (k, c, 9, projection) is   */
/* set, else +1 (a Rademacher projection, Achlioptas 2003); s = sigma /      */
/* sqrt(tr Sigma) with tr Sigma = (1/N) sum_i |x_i - mu|^2 (s = 0 when it is */
/* 0), so every coordinate has variance about sigma^2.  V = 0.               */
/* ------------------------------------------------------------------------ */
int fsneo_jump_start(fsneo_state *S, int32_t projection, double sigma)
{
    const int64_t N = S->N;
    const int32_t D = S->D, d = S->d;
    double *mu = calloc((size_t)D, sizeof(double));
    double *r = malloc(sizeof(double) * (size_t)D * (size_t)d);
    if (!mu || !r) {
        free(mu);
        free(r);
        return -2;
    }
    for (int64_t i = 0; i < N; ++i)
        for (int32_t k = 0; k < D; ++k) mu[k] += xval(S->X, S->xdtype, i * D + k);
    for (int32_t k = 0; k < D; ++k) mu[k] /= (double)N;
    double tr = 0.0;
    for (int32_t k = 0; k < D; ++k) {
        double v = 0.0;
        for (int64_t i = 0; i < N; ++i) {
            double e = xval(S->X, S->xdtype, i * D + k) - mu[k];
            v += e * e;
        }
        tr += v / (double)N;
    }
    const double scale = tr > 0.0 ? sigma / sqrt(tr) : 0.0;
    for (int32_t k = 0; k < D; ++k)
        for (int32_t c = 0; c < d; ++c) {
            uint32_t u[4];
            draw(S->seed, (uint32_t)k, (uint32_t)c, FSNEO_S_JUMP, (uint32_t)projection, u);
            r[k * d + c] = (u[0] & 1u) ? -1.0 : 1.0;
        }
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < N; ++i)
        for (int32_t c = 0; c < d; ++c) {
            double y = 0.0;
            for (int32_t k = 0; k < D; ++k)
                y += (xval(S->X, S->xdtype, i * D + k) - mu[k]) * r[k * d + c];
            S->Y[i * d + c] = scale * y;
            S->V[i * d + c] = 0.0;
        }
    free(mu);
    free(r);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Exact references, O(N^2), used to pin the method.                          */
/* ------------------------------------------------------------------------ */

/* Full eq. (1): conditional affinities over all k != i with beta_i set to   */
/* the perplexity, symmetrised; P is N x N with a zero diagonal.             */
void fsneo_exact_P(const void *X, int32_t xdtype, int64_t N, int32_t D, double perplexity,
                   double *P, double *beta)
{
    double *cond = malloc(sizeof(double) * (size_t)(N * N));
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < N; ++i) {
        double *d2 = malloc(sizeof(double) * (size_t)(N - 1));
        int64_t n = 0;
        for (int64_t j = 0; j < N; ++j)
            if (j != i) d2[n++] = fsneo_hd_dist2(X, xdtype, D, i, j);
        double rec[4];
        fsneo_calibrate(d2, (int32_t)(N - 1), perplexity, rec);
        beta[i] = rec[0];
        double S = 0.0;
        for (int64_t j = 0; j < N; ++j) {
            if (j == i) {
                cond[i * N + j] = 0.0;
                continue;
            }
            double v = exp(-rec[0] * (fsneo_hd_dist2(X, xdtype, D, i, j) - rec[1]));
            cond[i * N + j] = v;
            S += v;
        }
        for (int64_t j = 0; j < N; ++j) cond[i * N + j] /= S;
        free(d2);
    }
    for (int64_t i = 0; i < N; ++i)
        for (int64_t j = 0; j < N; ++j)
            P[i * N + j] = (cond[j * N + i] + cond[i * N + j]) / (2.0 * (double)N);
    free(cond);
}

static double wkern(double q2, double alpha) { return pow(1.0 + q2 / alpha, -alpha); }

/* KL(P || Q) with Q from eq. (4). */
double fsneo_exact_cost(const double *P, const double *Y, int64_t N, int32_t d, double alpha)
{
    double Z = 0.0;
    for (int64_t k = 0; k < N; ++k)
        for (int64_t l = 0; l < N; ++l)
            if (k != l) Z += wkern(ld_dist2(Y, d, k, l), alpha);
    double C = 0.0;
    for (int64_t k = 0; k < N; ++k)
        for (int64_t l = 0; l < N; ++l) {
            double p = P[k * N + l];
            if (k == l || p <= 0.0) continue;
            double q = wkern(ld_dist2(Y, d, k, l), alpha) / Z;
            C += p * log(p / q);
        }
    return C;
}

/* Gradient of eq. (5): 4 sum_j (p_ij - q_ij) w_ij^(1/alpha) (y_i - y_j). */
void fsneo_exact_grad(const double *P, const double *Y, int64_t N, int32_t d, double alpha,
                      double *G)
{
    double Z = 0.0;
    for (int64_t k = 0; k < N; ++k)
        for (int64_t l = 0; l < N; ++l)
            if (k != l) Z += wkern(ld_dist2(Y, d, k, l), alpha);
    for (int64_t i = 0; i < N; ++i) {
        for (int32_t c = 0; c < d; ++c) G[i * d + c] = 0.0;
        for (int64_t j = 0; j < N; ++j) {
            if (j == i) continue;
            double q2 = ld_dist2(Y, d, i, j);
            double w = wkern(q2, alpha);
            double wa = 1.0 / (1.0 + q2 / alpha);
            double coef = 4.0 * (P[i * N + j] - w / Z) * wa;
            for (int32_t c = 0; c < d; ++c) G[i * d + c] += coef * (Y[i * d + c] - Y[j * d + c]);
        }
    }
}

/* Exact K nearest neighbours of the query points (self excluded), sorted by */
/* (d2, idx), by brute force over all N points.                              */
void fsneo_knn_exact(const void *X, int32_t xdtype, int64_t N, int32_t D, const int64_t *q,
                     int64_t nq, int32_t K, int32_t *idx, double *d2)
{
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t a = 0; a < nq; ++a) {
        int64_t i = q[a];
        entry *best = malloc(sizeof(entry) * (size_t)(K + 1));
        int n = 0;
        for (int64_t j = 0; j < N; ++j) {
            if (j == i) continue;
            entry e = {fsneo_hd_dist2(X, xdtype, D, i, j), j};
            if (n == K && !entry_less(&e, &best[K - 1])) continue;
            int b = (n < K) ? n++ : K - 1;
            while (b > 0 && entry_less(&e, &best[b - 1])) {
                best[b] = best[b - 1];
                --b;
            }
            best[b] = e;
        }
        for (int32_t k = 0; k < K; ++k) {
            idx[a * K + k] = (int32_t)best[k].idx;
            d2[a * K + k] = best[k].key;
        }
        free(best);
    }
}

int fsneo_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Threads used by the loops over points from now on (results do not depend */
/* on it).                                                                    */
void fsneo_set_num_threads(int n)
{
#ifdef _OPENMP
    omp_set_num_threads(n);
#else
    (void)n;
#endif
}
