/*
 * FUnc-SNE CPU oracle -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, double-precision reference of the FUnc-SNE iteration
 * (Lambert, Couplet, Verleysen, Lee: "FUnc-SNE: A flexible, Fast, and
 * Unconstrained algorithm for neighbour embeddings").  It exists to check the
 * HIP library; only the tests, the smoke check and the benchmark's CPU
 * baseline may load it.  It shares no code, header, table or helper with the
 * HIP path.
 *
 * Readings of the paper where it is silent are fixed in the functions that
 * apply them; every reading is applied identically by the HIP library.
 */
#ifndef FSNE_ORACLE_H
#define FSNE_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Longest neighbour list (HD or LD). */
#define FSNEO_KMAX 256

/* Number of candidate slots per point and refinement, and their kinds. */
#define FSNEO_C 32
#define FSNEO_SAME_NON 16   /* slots  0..15: neighbour of neighbour, same space   */
#define FSNEO_CROSS_DIR 4   /* slots 16..19: direct neighbour, other space         */
#define FSNEO_CROSS_NON 8   /* slots 20..27: neighbour of neighbour, other space   */
#define FSNEO_RANDOM 4      /* slots 28..31: uniform random point                  */

/* Counter-stream ids of the random draws (third counter word). */
enum { FSNEO_S_HDC = 1, FSNEO_S_LDC = 2, FSNEO_S_NEG = 3, FSNEO_S_INIT_HD = 4,
       FSNEO_S_INIT_LD = 5, FSNEO_S_COIN = 7, FSNEO_S_JUMP = 9, FSNEO_S_DEL_HD = 10,
       FSNEO_S_DEL_LD = 11 };

typedef struct {
    int64_t N;          /* live number of points                              */
    int32_t D, d, K_hd, K_ld;
    int32_t xdtype;     /* 0: X is float32, 1: X holds bfloat16 bit patterns   */
    uint64_t seed;      /* key of the counter-based generator                  */
    const void *X;      /* N x D, row-major                                    */
    double *Y, *V;      /* N x d                                               */
    int32_t *hd_idx;    /* N x K_hd, sorted by (d2, idx)                       */
    double *hd_d2;      /* N x K_hd                                            */
    int32_t *ld_idx;    /* N x K_ld                                            */
    double *beta;       /* N: 1 / (2 sigma_i^2)                                 */
    double *m;          /* N: smallest HD d2 of row i (exponent shift)         */
    double *r;          /* N: largest HD d2 of row i                           */
    double *invS;       /* N: 1 / sum_k exp(-beta_i (d2_ik - m_i))             */
    double *P;          /* N x K_hd symmetrised affinities aligned with hd_idx */
    uint8_t *flags;     /* N: 1 if the last HD refinement changed row i        */
    double *E;          /* smoothed fraction of points that gained neighbours  */
    uint32_t *t;        /* iteration counter                                   */
    int32_t metric;     /* HD distance: 0 squared Euclidean, 1 angular (the    */
                        /* squared Euclidean distance of the unit rows)        */
} fsneo_state;

typedef struct {
    double alpha, perplexity, lr, momentum, attr, rep;
    int32_t n_neg;
    int32_t hd_mode;    /* 0 auto (coin), 1 always, 2 never                    */
    double e_smooth;    /* smoothing weight lambda of E                        */
    double p_min;       /* floor of the refinement probability                 */
} fsneo_hp;

typedef struct {
    int32_t fired;
    int64_t n_new;
    double Z;
    double E;           /* E after the step                                    */
    uint32_t t;         /* t after the step                                    */
} fsneo_stats;

void fsneo_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
int fsneo_coin(double E, uint32_t t, uint64_t seed, int32_t hd_mode, double p_min);
double fsneo_coin_margin(double E, uint32_t t, uint64_t seed, double p_min);
double fsneo_E_next(double E, int64_t n_new, int64_t N, double lam);
int fsneo_calibrate(const double *d2, int32_t K, double perplexity, double out[4]);
double fsneo_hd_dist2(const void *X, int32_t xdtype, int32_t D, int64_t a, int64_t b);
double fsneo_hd_dist2_metric(const void *X, int32_t xdtype, int32_t D, int32_t metric,
                             int64_t a, int64_t b);
int fsneo_set_metric(fsneo_state *S, const fsneo_hp *hp, int32_t metric);
int fsneo_init(fsneo_state *S, const fsneo_hp *hp);
int fsneo_step(fsneo_state *S, const fsneo_hp *hp, fsneo_stats *st,
               double *A, double *R, double *Zh);
void fsneo_hd_refine_point(const fsneo_state *S, int64_t i, uint32_t t,
                           int32_t *idx_out, double *d2_out, uint8_t *changed);
void fsneo_psym_row(const fsneo_state *S, int64_t i, double *out);
void fsneo_ld_refine_grad_point(const fsneo_state *S, const fsneo_hp *hp, int64_t i,
                                uint32_t t, const int32_t *hd_next, const double *P_next,
                                int32_t *ld_out, double *A, double *R, double *Zh);
void fsneo_hd_finish(fsneo_state *S, const fsneo_hp *hp);
void fsneo_ld_phase(const fsneo_state *S, const fsneo_hp *hp, uint32_t t, const int32_t *hd_next,
                    const double *P_next, int32_t *ld_out, double *A, double *R, double *Zh);
int fsneo_point_step(const fsneo_state *S, const fsneo_hp *hp, int64_t i, int32_t fired,
                     int32_t *hd_idx_out, double *hd_d2_out, uint8_t *flag_out,
                     double rec_out[4], double *P_out, int32_t *ld_out,
                     double *A, double *R, double *Zh);
void fsneo_exact_P(const void *X, int32_t xdtype, int64_t N, int32_t D, double perplexity,
                   double *P, double *beta);
double fsneo_exact_cost(const double *P, const double *Y, int64_t N, int32_t d, double alpha);
void fsneo_exact_grad(const double *P, const double *Y, int64_t N, int32_t d, double alpha,
                      double *G);
void fsneo_knn_exact(const void *X, int32_t xdtype, int64_t N, int32_t D,
                     const int64_t *q, int64_t nq, int32_t K, int32_t *idx, double *d2);
int fsneo_insert(fsneo_state *S, const fsneo_hp *hp, int64_t n_new, const double *Y_new);
int fsneo_drift(fsneo_state *S, const fsneo_hp *hp, const int64_t *ids, int64_t n,
                const double *Y_new);
int fsneo_jump_start(fsneo_state *S, int32_t projection, double sigma);
void fsneo_delete_fix(fsneo_state *S, const fsneo_hp *hp, const int32_t *newid);
int32_t fsneo_cluster(const fsneo_state *S, float eps, int32_t min_pts, int32_t *labels);
int fsneo_num_threads(void);
void fsneo_set_num_threads(int n);

#ifdef __cplusplus
}
#endif
#endif
