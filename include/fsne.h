/*
 * fsne.h -- C ABI of the MI355X (gfx950) FUnc-SNE step library, libfsne.so.
 *
 * FUnc-SNE (Lambert, Couplet, Verleysen, Lee, "FUnc-SNE: A flexible, Fast, and
 * Unconstrained algorithm for neighbour embeddings") embeds N points x_i of
 * R^D into R^d.  One iteration interleaves three things that the paper
 * describes in Sec. 3:
 *   - refinement of approximate HD and LD K-nearest-neighbour lists from
 *     candidates (neighbours of neighbours, cross-space feeds, random
 *     draws); the HD refinement runs with probability 0.05 + 0.95 E, E the
 *     smoothed fraction of points that gained HD neighbours;
 *   - the variable-tailed gradient of eqs. (4)-(6): attraction over the HD
 *     neighbours' affinities p_ij (eq. (1)), repulsion over HD and LD
 *     neighbours plus negative samples, normalised by Z;
 *   - a momentum update of the embedding.
 *
 * Conventions
 *   - Every call returns an fsne_status; no exception or abort crosses the
 *     ABI.  fsne_last_error() gives the message of the last failing call on
 *     a context.
 *   - The caller owns every pointer it passes.  "device" pointers are HIP
 *     device memory of the current device; "host" pointers are ordinary CPU
 *     memory.  Each argument says which it is.
 *   - Work is queued on the context's HIP stream.  fsne_step is asynchronous;
 *     the get_* calls synchronise the stream before they return.
 *   - A context is not thread-safe: calls on one context must not overlap.
 *   - Layouts are row-major: point i's row of an N x W array starts at i*W.
 *   - N <= 2^31 - 1; K_hd, K_ld <= 64; d <= 64; n_neg <= 64; D <= fsne_max_dim().
 */
#ifndef FSNE_H
#define FSNE_H
#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct fsne_ctx fsne_ctx;
typedef struct fsne_mlp fsne_mlp;

typedef enum {
    FSNE_OK = 0,
    FSNE_EINVAL = -1,     /* an argument is out of range; nothing was changed    */
    FSNE_ENOMEM = -2,     /* device allocation failed or capacity exceeded       */
    FSNE_EHIP = -3,       /* a HIP runtime call failed                           */
    FSNE_ESTATE = -4,     /* the context is not in a state that allows the call  */
    FSNE_ENONFINITE = -5  /* the embedding holds a NaN or infinity               */
} fsne_status;

typedef enum { FSNE_F32 = 0, FSNE_BF16 = 1 } fsne_dtype;

/* Hyperparameters; all may change between steps (fsne_set_hyperparams). */
typedef struct fsne_hparams {
    float alpha;        /* tail parameter of eq. (4), > 0; 1 is t-SNE             */
    float perplexity;   /* perplexity of eq. (1), 1 < perplexity < K_hd            */
    float lr;           /* learning rate of the gradient step, >= 0                */
    float momentum;     /* momentum of the update, in [0, 1)                       */
    float attr;         /* attraction scale (early exaggeration), >= 0             */
    float rep;          /* repulsion scale, >= 0                                   */
    int32_t n_neg;      /* negative samples per point and iteration, 0..64         */
    int32_t hd_mode;    /* 0: HD refinement by the coin, 1: every iteration, 2: never */
    int32_t dist_mode;  /* HD candidate distances: 0 FP32 direct, 1 BF16 MFMA screen
                           with FP32 re-rank (requires BF16 X)                       */
    float e_smooth;     /* smoothing weight lambda of E, in (0, 1]                 */
    float p_min;        /* refinement probability floor (0.05 in the paper)        */
    float rerank_margin;/* BF16 screen keeps candidates with d2~ <= r_i (1+margin)  */
    int32_t reject_memo;/* 1: each point remembers the last candidates its HD
                           refinements rejected (64 with direct distances on rows
                           of 512 bytes or more, else 32) and does not evaluate
                           them again; 0: every candidate is evaluated.  Both
                           give the same
                           lists: while X and the lists change only by
                           refinement, a point's K-th HD distance never grows, so
                           a rejected candidate would be rejected again.  The
                           memory is cleared where that does not hold (drift,
                           delete, a state load of the HD lists, a change of
                           dist_mode or rerank_margin); inserted points start
                           empty.                                               */
    int32_t metric;     /* HD distance (Sec. 3 names the metric as an HD-side
                           setting that may change during optimisation):
                           0 squared Euclidean; 1 angular, the squared Euclidean
                           distance between the rows scaled to unit length,
                           2 (1 - cos); a zero row stays zero.  The affinities
                           of eq. (1) take it in place of delta^2.  The library
                           then keeps an FP32 copy of the unit rows (capacity x D)
                           for the HD kernels; metric 1 needs dist_mode 0.      */
} fsne_hparams;

/* Host-side view of the iteration state for checkpoints and checks.  Every
 * pointer is host memory of the stated size, or NULL to skip that field. */
typedef struct fsne_state_view {
    float *Y;           /* N x d embedding                                         */
    float *V;           /* N x d velocity                                          */
    int32_t *hd_idx;    /* N x K_hd HD lists, sorted by (d2, index)                */
    float *hd_d2;       /* N x K_hd HD distances of the lists in the current
                           metric (squared Euclidean, or angular)              */
    int32_t *ld_idx;    /* N x K_ld LD lists                                       */
    float *rec;         /* N x 4 per-point {beta, m, r, invS}: beta = 1/(2 sigma^2),
                           m and r the smallest and largest d2 of the HD list,
                           invS = 1/sum_k exp(-beta (d2_k - m))                      */
    float *P;           /* N x K_hd symmetrised affinities aligned with hd_idx     */
    uint8_t *flags;     /* N: 1 where the last HD refinement changed the list      */
    float *A;           /* N x d attraction partials of the last step (get only)   */
    float *R;           /* N x d repulsion partials of the last step (get only)    */
    float *Zh;          /* N per-point normaliser partials of the last step (get)  */
    float *E;           /* scalar: smoothed fraction E                             */
    uint32_t *t;        /* scalar: iteration counter                               */
} fsne_state_view;

typedef struct fsne_stats {
    int64_t N;          /* live points                                             */
    uint32_t t;         /* iterations done                                         */
    float E;            /* smoothed fraction of points that gained HD neighbours   */
    int32_t next_fire;  /* whether iteration t refines the HD lists                */
    int32_t last_fired; /* whether iteration t-1 refined them                      */
    int32_t n_new;      /* points whose HD list changed in the last refinement     */
    float Z;            /* normaliser of the last iteration                        */
    int32_t nonfinite;  /* 1 if a NaN/inf reached the embedding                    */
    uint32_t hd_cand_rows; /* distinct HD candidate rows loaded by the last HD
                              refinement (duplicates are never loaded)             */
    uint32_t ld_cand_rows; /* distinct LD candidate rows of the last iteration     */
    uint32_t hd_refinements; /* iterations that refined the HD lists since init    */
} fsne_stats;

/* Largest HD dimension D the library accepts for rows of xdtype: 4096 for
 * FP32 with D % 4 == 0, 2048 for BF16 with D % 8 == 0, 1024 otherwise. */
int32_t fsne_max_dim(int32_t xdtype, int32_t D);

/* Fill *hp with the defaults: alpha 1, perplexity 10, lr 100, momentum 0.5,
 * attr 1, rep 1, n_neg 16, hd_mode 0, dist_mode 0, e_smooth 0.1, p_min 0.05,
 * rerank_margin 2^-6, reject_memo 1, metric 0.  Returns FSNE_EINVAL if hp is NULL. */
fsne_status fsne_default_hparams(fsne_hparams *hp);

/* Create a context and its initial state (Sec. 3: optimisation starts right
 * after allocation, with random neighbour lists).
 *   X         N x D points, FP32 or BF16 (bit patterns) per xdtype; host memory
 *             unless x_on_device = 1, in which case it is device memory that
 *             must outlive the context (it is read, never written).
 *   Y0        N x d initial embedding, host memory (NULL: all zeros).
 *   d, K_hd, K_ld  embedding dimension and list lengths:
 *             1 <= d <= 64, 2 <= K_hd <= 256, 1 <= K_ld <= 64, K_hd, K_ld < N.
 *             HD lists longer than 64 (held in LDS, one point per wave)
 *             take direct distances only (dist_mode 0) and no drift,
 *             delete or metric switch (those return FSNE_EINVAL).
 *   alpha     tail of the LD kernel (eq. (4)), > 0; replaces hp->alpha.
 *   perplexity  of the HD affinities (eq. (1)), 1 < perplexity < K_hd;
 *             replaces hp->perplexity.
 *   seed      key of the Philox4x32-10 draws (candidates, negatives, coin).
 *   hp        the other hyperparameters, or NULL for the defaults.
 *   stream    hipStream_t to run on, or NULL for a stream the context owns.
 *   capacity  rows reserved for fsne_insert_points (>= N).
 * Initial lists: for point i, the first K distinct other points from draws
 * (i, 0, stream, s), s = 0, 1, ...; HD lists sorted; all points calibrated to
 * the perplexity; V = 0; E = 1; t = 0.
 * Errors: FSNE_EINVAL (bad sizes or hyperparameters), FSNE_ENOMEM, FSNE_EHIP. */
fsne_status fsne_init(fsne_ctx **out, const void *X, int64_t N, int32_t D, int32_t xdtype,
                      const float *Y0, int32_t d, int32_t K_hd, int32_t K_ld, float alpha,
                      float perplexity, uint64_t seed, const fsne_hparams *hp,
                      int32_t x_on_device, void *stream, int64_t capacity);

/* Run n_iters iterations (Sec. 3), asynchronously on the context stream.
 * Per iteration: [if the coin fires] HD refinement + recalibration of changed
 * points + affinities of the list entries with a changed point at either end
 * (the others keep their values); LD refinement + gradient partials; Z; momentum update;
 * E and the next coin.  Errors: FSNE_EINVAL (n_iters < 0), FSNE_EHIP. */
fsne_status fsne_step(fsne_ctx *ctx, int32_t n_iters);

/* Replace the hyperparameters.  A perplexity change recalibrates every point
 * and recomputes the affinities before the next step (Sec. 3: HD-side
 * hyperparameters change on the fly).  A metric change keeps every HD list's
 * members, recomputes every stored distance in the new metric, re-sorts each
 * list by (d2, id), flags and recalibrates every point, recomputes the
 * affinities and sets E to 1, so that the next iterations refine the lists
 * towards the new metric's neighbours.  Synchronises the context stream when
 * the perplexity or the metric changes.  Errors: FSNE_EINVAL, FSNE_ENOMEM (no
 * memory for the unit rows of the angular metric; the previous hyperparameters
 * stay), FSNE_EHIP. */
fsne_status fsne_set_hyperparams(fsne_ctx *ctx, const fsne_hparams *hp);
fsne_status fsne_get_hyperparams(const fsne_ctx *ctx, fsne_hparams *hp);

/* Copy the N x d embedding to out (host memory, or device memory if
 * out_on_device = 1).  Synchronises.  Errors: FSNE_EINVAL, FSNE_EHIP. */
fsne_status fsne_get_Y(fsne_ctx *ctx, float *out, int32_t out_on_device);

/* Copy the current lists: which = 0 HD (idx N x K_hd, dist2 N x K_hd may be
 * NULL; distances in the current HD metric), which = 1 LD (idx N x K_ld;
 * dist2 must be NULL).  Host memory.
 * Synchronises.  Errors: FSNE_EINVAL, FSNE_EHIP. */
fsne_status fsne_get_knn(fsne_ctx *ctx, int32_t which, int32_t *idx, float *dist2);

/* Renumber the points (not in the paper; an ordering for memory locality):
 * point i becomes point new_of_old[i], a permutation of 0..N-1 in host
 * memory.  Every per-point row (X, Y, V, gradient partials, records, P,
 * flags, lists) moves to the new id and every list entry is mapped; the
 * method then goes on exactly as it would from the renumbered state (its
 * draws are keyed by the new ids).  The remembered rejections are cleared.
 * Synchronises.  Errors: FSNE_EINVAL (not a permutation), FSNE_ESTATE (X
 * borrowed), FSNE_ENOMEM, FSNE_EHIP. */
fsne_status fsne_renumber(fsne_ctx *ctx, const int32_t *new_of_old);

/* Renumber the points along the Morton (Z-order) curve of the embedding
 * projected onto at most three axes (y itself when d <= 3; otherwise axis a
 * sums y_a, y_{a+3}, ... with alternating signs), ties by the old id, so
 * that points close in the embedding get nearby ids and the step's gathers
 * hit in the caches.  new_of_old (host, N entries, may be NULL) receives the
 * permutation applied, for the caller's own per-point arrays.  Synchronises.
 * Errors: FSNE_ENONFINITE, FSNE_ESTATE, FSNE_ENOMEM, FSNE_EHIP. */
fsne_status fsne_reorder(fsne_ctx *ctx, int32_t *new_of_old);

/* Renumber the points along the Morton curve of the data rows projected
 * onto three axes, c_a = sum_k x_ik r_ka with fixed signs r_ka = +-1 (bit 0
 * of the first word of Philox block (k, a, 12, 0)); under the angular metric
 * the rows scaled to unit length.  A fixed projection shrinks distances
 * about evenly, so points close in R^D get nearby ids even before the
 * embedding has any structure of its own (right after fsne_init, say); ties
 * by the old id.  new_of_old and errors as fsne_reorder. */
fsne_status fsne_reorder_data(fsne_ctx *ctx, int32_t *new_of_old);

/* Copy the state to / from host memory (checkpoint, resume, checks).  set
 * reads every non-NULL field except A, R, Zh and recomputes the coin of the
 * next iteration from E and t.  If it sets HD lists, distances or records
 * but no affinities P, it recomputes P from the new state (eq. (1), reading
 * restricted to the lists): refinements only update the entries of points
 * whose lists changed.  Synchronises.  Errors: FSNE_EINVAL, FSNE_EHIP. */
fsne_status fsne_get_state(fsne_ctx *ctx, const fsne_state_view *s);
fsne_status fsne_set_state(fsne_ctx *ctx, const fsne_state_view *s);

/* Statistics of the last iteration.  Synchronises.  Returns FSNE_ENONFINITE
 * (with *st filled) if the embedding holds a NaN or infinity. */
fsne_status fsne_get_stats(fsne_ctx *ctx, fsne_stats *st);

/* Wait for the context's queued work.  Errors: FSNE_EHIP. */
fsne_status fsne_sync(fsne_ctx *ctx);

/* Dynamic data (Sec. 3 on online use; Sec. 5).  Insert n new points (host
 * X rows of the context's dtype, host Yinit n x d or NULL for zeros): they
 * take indices N..N+n-1, get random lists, calibration and V = 0; every
 * point's affinities are recomputed for the new N.  Errors: FSNE_ENOMEM
 * (beyond capacity), FSNE_EINVAL, FSNE_EHIP. */
fsne_status fsne_insert_points(fsne_ctx *ctx, const void *Xnew, int64_t n, const float *Yinit);

/* Replace the HD coordinates of n existing points (host ids, host rows).
 * Their velocity is reset; Yinit (host n x d, or NULL to keep y) replaces
 * their embedding.  Every HD list entry that pairs with a moved point gets
 * its new distance; affected lists are re-sorted, flagged and recalibrated;
 * affinities are recomputed.  Errors: FSNE_EINVAL, FSNE_EHIP. */
fsne_status fsne_drift_points(fsne_ctx *ctx, const int64_t *ids, const void *Xnew, int64_t n,
                              const float *Yinit);

/* For callers that cannot allocate (code under HIP graph capture, tight
 * serving loops, harnesses that forbid device allocation): fsne_drift_points
 * without any hipMalloc / hipFree.  The ids, X rows and Y rows of the call
 * are staged in a fixed device array of 16 MiB that the library holds on
 * each GPU until the process ends; a call needs
 *   align256(8n) + align256(4n) + align256(n D xbytes) + align256(4 n d)
 *   + align256(4 n DP)  bytes  (DP: d rounded up to a power of two >= 2)
 * and a larger batch is rejected with FSNE_EINVAL (split it).  ids must be
 * strictly increasing (no duplicates).  Same results as fsne_drift_points.
 * Synchronises the context stream before returning.  Every call on a GPU
 * shares that GPU's array: calls that overlap on one GPU (from several
 * threads or contexts) race and must be serialised by the caller.
 * Errors: FSNE_EINVAL, FSNE_ESTATE (borrowed X), FSNE_EHIP. */
fsne_status fsne_drift_points_noalloc(fsne_ctx *ctx, const int64_t *ids, const void *Xnew,
                                      int64_t n, const float *Yinit);

/* Remove n points (host ids, distinct, 0 <= id < N; at least
 * max(K_hd, K_ld) + 1 points must remain) -- online use, Sec. 3.  Ids stay
 * dense: with N' = N - n, the surviving points at or beyond N' move, in
 * increasing order, into the freed ids below N', in increasing order; every
 * other survivor keeps its id.  Each survivor's lists are rewritten:
 * entries of deleted points are dropped, the rest take the new ids; an HD
 * list refills with random points (draws (i, t, 10, s)), gets their
 * distances, is re-sorted by (d2, id) and recalibrated (flag set); an LD list
 * keeps its surviving entries in order and appends random refills (draws
 * (i, t, 11, s)).  Affinities are recomputed.  Synchronises the stream.
 * Errors: FSNE_EINVAL, FSNE_ESTATE (X borrowed), FSNE_ENOMEM, FSNE_EHIP. */
fsne_status fsne_delete_points(fsne_ctx *ctx, const int64_t *ids, int64_t n);

/* Clusters of the current embedding for the hierarchy graph (Sec. 4.2):
 * DBSCAN (Ester et al. 1996) with each point's eps-neighbourhood read from
 * its LD neighbour list:
 *   N(i) = {i} + {j in LD list of i : |y_i - y_j|^2 <= eps^2},
 *   core points: |N(i)| >= min_pts (1 <= min_pts <= K_ld + 1);
 *   clusters: connected components of the core points, linked when either
 *   lies in the other's N; a non-core point within eps of a core point (in
 *   either list) joins the nearest one's cluster (ties: smaller cluster);
 *   the rest is noise.
 * Squared distances are summed in index order in FP32 without fused
 * multiply-add.  labels (host, N) get 0 .. n_clusters-1, numbered by the
 * smallest index among each cluster's core points, or -1 for noise;
 * *n_clusters (may be NULL) gets the count.  Synchronises the stream.
 * Errors: FSNE_EINVAL, FSNE_EHIP. */
fsne_status fsne_cluster(fsne_ctx *ctx, float eps, int32_t min_pts, int32_t *labels,
                         int32_t *n_clusters);

/* Edges of the hierarchy graph between two clusterings of the same n points
 * (levels g and h = g + 1, Sec. 4.2): E[i cb + j] = |A_i and B_j| /
 * min(|A_i|, |B_j|) for cluster i of la (ca clusters) and j of lb (cb
 * clusters), 0 when either is empty; label -1 (noise) belongs to no
 * cluster.  Host arrays; pure host code.  Errors: FSNE_EINVAL. */
fsne_status fsne_hierarchy_edges(const int32_t *la, int32_t ca, const int32_t *lb, int32_t cb,
                                 int64_t n, float *E);

/* Scale the embedding down by factor (> 0): Y <- Y / factor, V <- V / factor
 * (Sec. 3, the "implosion" control).  Errors: FSNE_EINVAL, FSNE_EHIP. */
fsne_status fsne_implode(fsne_ctx *ctx, float factor);

/* Jump start (Sec. 3, helping the first iterations): replace the embedding
 * of the N live points by a random linear projection of the centred data,
 *   y_ic = s sum_k (x_ik - mu_k) r_kc,  r_kc = -1 if bit 0 of the first word
 *   of Philox block (k, c, 9, projection) under the context's seed is set,
 *   else +1;  s = sigma / sqrt(tr Sigma), tr Sigma = (1/N) sum_i |x_i - mu|^2
 *   (s = 0 if the data have no spread),
 * so each coordinate has variance about sigma^2; V <- 0.  Means and the
 * trace are summed in double.  Typical use: a few projections (projection =
 * 0, 1, ...) each followed by some iterations at learning rate 0, before the
 * gradient takes over.  Synchronises the stream.
 * Errors: FSNE_EINVAL (projection < 0, sigma <= 0), FSNE_EHIP. */
fsne_status fsne_jump_start(fsne_ctx *ctx, int32_t projection, float sigma);

/* Kernels of one iteration, in launch order (indices of fsne_get_kernel_times). */
enum {
    FSNE_K_HD_REFINE = 0, /* HD candidates, distances, merge, recalibration     */
    FSNE_K_AFFINITY = 1,  /* symmetrised affinities of eq. (1)                   */
    FSNE_K_LD_GRAD = 2,   /* LD refinement and gradient partials (eqs. (4)-(6))  */
    FSNE_K_REDUCE = 3,    /* fixed-order partial sums of Z and N_new             */
    FSNE_K_UPDATE = 4,    /* momentum update and next-iteration scalars          */
    FSNE_NKERNELS = 5
};

/* Measurement: with enable = 1, fsne_step records a HIP event pair on the
 * context stream around every kernel it launches; enabling or disabling
 * clears the totals.  Errors: FSNE_EHIP. */
fsne_status fsne_profile(fsne_ctx *ctx, int32_t enable);

/* Totals since fsne_profile(ctx, 1): ms[k] summed kernel time and
 * launches[k] launch count, k < FSNE_NKERNELS (host arrays).  A kernel that
 * exits early because the coin did not fire still counts as a launch.
 * Synchronises.  Errors: FSNE_EINVAL, FSNE_EHIP. */
fsne_status fsne_get_kernel_times(fsne_ctx *ctx, double *ms, int64_t *launches);

/* ------------------------------------------------------------------------
 * Placement network for dynamic data (Sec. 3 on online use, Sec. 5): a
 * multilayer perceptron D -> hidden1 -> hidden2 -> d with ReLU hidden layers,
 * fitted by mean squared error to the standardised embedding of a context
 * (y - mean) / std per component, with Adam (Kingma and Ba 2015).  Its
 * predictions initialise the y of inserted or drifted points (fsne_insert_points
 * / fsne_drift_points take them as Yinit).  The three large products run on
 * BF16 matrix cores with FP32 accumulation; weights are FP32.
 * Parameters (fsne_mlp_get_params) are one flat FP32 array:
 *   W1 (hidden1 x D), b1 (hidden1), W2 (hidden2 x hidden1), b2 (hidden2),
 *   W3 (d x hidden2), b3 (d).
 * ------------------------------------------------------------------------ */
typedef struct fsne_mlp_opts {
    int32_t hidden1, hidden2;  /* hidden widths (default 512, 512)               */
    int32_t epochs;            /* passes over the context's points (default 5)   */
    int32_t batch;             /* rows per Adam step (default 4096)              */
    float lr, beta1, beta2, eps; /* Adam (default 1e-3, 0.9, 0.999, 1e-8)        */
    uint64_t seed;             /* He-uniform initialisation draws (Philox)       */
} fsne_mlp_opts;

fsne_status fsne_mlp_default_opts(fsne_mlp_opts *opts);

/* Create a network for ctx's D, d and input dtype, initialised He-uniform:
 * w = (2u - 1) sqrt(6 / fan_in), u from Philox block (index, layer, 8, 0);
 * biases 0; standardisation mean 0, std 1.  Errors: FSNE_EINVAL, FSNE_ENOMEM. */
fsne_status fsne_mlp_create(const fsne_ctx *ctx, const fsne_mlp_opts *opts, fsne_mlp **out);

/* Fit the network to ctx's current points (x_i, y_i), i < N: the
 * standardisation is taken from ctx's Y, then opts.epochs passes of Adam
 * steps over batches of opts.batch consecutive rows (epoch e starts at row
 * 104729 e mod N).  The products read their operands as bfloat16: with FP32
 * rows, D a multiple of 8 and more than one epoch, the call holds a
 * bfloat16 copy of X (N D 2 bytes of device memory, freed before it
 * returns; if it cannot be allocated the rows are rounded batch by batch).
 * *final_loss (may be NULL) gets the mean loss of the last epoch.
 * Synchronises ctx's stream first.  Errors: FSNE_EINVAL, FSNE_EHIP. */
fsne_status fsne_mlp_train(fsne_mlp *m, fsne_ctx *ctx, float *final_loss);

/* Predict y for n host rows X (the context's dtype) into host Y (n x d). */
fsne_status fsne_mlp_predict(fsne_mlp *m, const void *X, int64_t n, float *Y);

/* Copy parameters / standardisation out of or into host arrays (NULL skips). */
fsne_status fsne_mlp_get_params(fsne_mlp *m, float *params, float *ymean, float *ystd);
fsne_status fsne_mlp_set_params(fsne_mlp *m, const float *params, const float *ymean,
                                const float *ystd);

/* Loss 1/(n d) sum (out - T)^2 and its gradient (flat, host, num_params
 * floats) for n <= batch host rows X with standardised targets T (n x d). */
fsne_status fsne_mlp_loss_grad(fsne_mlp *m, const void *X, const float *T, int64_t n,
                               float *grad, float *loss);

/* One Adam step on n <= batch host rows X with standardised targets T. */
fsne_status fsne_mlp_train_batch(fsne_mlp *m, const void *X, const float *T, int64_t n);

int64_t fsne_mlp_num_params(const fsne_mlp *m);
void fsne_mlp_destroy(fsne_mlp *m);
const char *fsne_mlp_last_error(const fsne_mlp *m);

/* Destroy the context and free its device memory (NULL is accepted). */
void fsne_destroy(fsne_ctx *ctx);

/* Message of the last failing call on ctx (never NULL). */
const char *fsne_last_error(const fsne_ctx *ctx);

#ifdef __cplusplus
}
#endif
#endif
