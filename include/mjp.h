/*
 * mjp.h -- C ABI of libmjp: the R-MJP (restricted Markov-jump-process)
 * expansion of rho(0) exp(A_theta t) on one MI355X (gfx950).
 *
 * Method (Pessoa, Schweiger, Presse, "Avoiding matrix exponentials for large
 * transition rate matrices", arXiv 2312.05647):
 *   A_theta   generator (Eq. A_def): a_nm = rate n->m (n != m),
 *             a_nn = -(total rate out of n); row = from-state.
 *   Omega     omega_factor * max_n |a_nn|, omega_factor > 1 (Eq. B_def; the
 *             paper uses 1.1).
 *   B         I + A/Omega, a stochastic matrix (Eq. B_def).
 *   rho(t)    = sum_k rho(0) B^k Poisson(k | Omega t)   (Eq. ME_uniform),
 *             truncated after K products, the dropped weight placed on
 *             rho(0) B^K (Algorithm 2; Sec. 2.2.3, Eq. R-MJP_expansion).
 *   loglik    sum_i log rho(T^i)_{s^i} over snapshot observations
 *             (Sec. 2.1.2).
 * The surrogate entry points (an MLP over log-parameters trained on exact
 * log-likelihoods, used for delayed-acceptance sampling) are an addition to
 * the paper's method; they are documented where declared.
 *
 * Conventions for every entry point:
 *   - Every function returns mjp_status; nothing throws across the ABI.
 *     On failure mjp_last_error() returns a thread-local message.
 *   - Arguments named *_d are device pointers (memory on the GPU that was
 *     current when the plan or surrogate was created); *_h are host pointers.
 *     All buffers are owned by the caller unless stated otherwise.
 *   - All argument checks run on the host before any GPU work is enqueued, so
 *     an invalid call never launches a kernel.
 *   - Calls are asynchronous on the given stream (a hipStream_t passed as
 *     mjp_stream_t; NULL = the null stream) unless an info_h pointer is
 *     given, which makes the call wait for its own work to finish.
 *   - A plan or surrogate must not be used by two streams at the same time.
 *     Handles are opaque and freed by their *_destroy function.
 *   - Scratch memory (ping-pong vectors, compensation terms, weight tables)
 *     is owned by the plan and grows on demand with hipMalloc.
 */
#ifndef MJP_H
#define MJP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* A hipStream_t. */
typedef void* mjp_stream_t;

typedef enum {
    MJP_OK = 0,
    MJP_E_INVALID_ARG = 1,    /* null pointer, size <= 0, t < 0 or not finite, bad option, ... */
    MJP_E_NOT_GENERATOR = 2,  /* negative off-diagonal rate, or a row sum that breaks the truncation rule */
    MJP_E_K_LIMIT = 3,        /* the jump count K needed for (t, tol) exceeds opts.k_cap */
    MJP_E_WORKSPACE = 4,      /* a size exceeds what the chosen kernel supports */
    MJP_E_DEVICE = 5,         /* a HIP runtime call failed (no GPU, out of memory, launch error) */
    MJP_E_NUMERIC = 6,        /* (synchronous calls only) NaN/Inf or a negative entry was detected */
    MJP_E_UNSUPPORTED = 7     /* a valid request this build does not implement */
} mjp_status;

/* ---------------------------------------------------------------- options */

enum { MJP_K_TOL = 0,      /* K, L from the Poisson tails: eps_right = eps_left = tol/4 */
       MJP_K_PAPER = 1 };  /* K = floor(W + 6 sqrt W) + 1, L = 0: the loop bound of
                              Algorithm 2 (while k <= W + 6 sqrt W, increment first) */

enum { MJP_CONSERVATIVE = 0, /* transitions that would leave the state space are dropped,
                                so rows of A sum to 0 and rows of B to 1 (Eq. B_def) */
       MJP_LEAKY = 1 };      /* the exit rate still counts them (the m_theta of the
                                birth-death example, Sec. 3.1.1); mass leaks */

enum { MJP_VARIANT_AUTO = 0,       /* the plan picks the launch strategy */
       MJP_VARIANT_STEPWISE = 1,   /* one kernel per jump, launched in a loop */
       MJP_VARIANT_PERSISTENT = 2, /* all K jumps in one cooperative launch; the
                                      iterate moves between XCDs through
                                      device-scope loads and stores.  Where
                                      the operator is a grid (every column of
                                      row m in {m, m +- 1, m +- S1}, width <=
                                      5, at least 128 workgroups of 4096 rows,
                                      at most 2 windows open at once) and
                                      renorm_every is a multiple of 8 (else 4),
                                      each workgroup owns a 2-D tile and
                                      computes eight (else four) jumps per
                                      synchronisation where the rings of cells
                                      around its tile fit its LDS, recomputing
                                      those rings; else, where the reach is short
                                      (at most 2048 rows of halo per 4096-row
                                      block, width <= 5) and renorm_every is
                                      even, two jumps per synchronisation;
                                      both bit-identical to one jump per
                                      synchronisation */
       MJP_VARIANT_PERSISTENT_FENCED = 3, /* one jump per synchronisation,
                                      synchronised with agent-scope
                                      release/acquire fences (L2 write-back and
                                      invalidate per workgroup and jump):
                                      slower, bit-identical; kept as the
                                      reference protocol */
       MJP_VARIANT_PERSISTENT_ONEJUMP = 4, /* one jump per synchronisation,
                                      device-scope protocol: bit-identical */
       MJP_VARIANT_PERSISTENT_TWOJUMP = 5 /* two jumps per synchronisation on
                                      row blocks where they fit, else one:
                                      bit-identical */ };

typedef struct {
    double  omega_factor;  /* Omega = omega_factor * max|a_nn|; must be > 1 (Eq. B_def: 1.1) */
    double  tol;           /* L1 truncation budget of the series, 0 < tol < 1.  With lumping the
                              L1 distance to rho(0)exp(At) from truncation is at most
                              2 (eps_left + eps_right) = tol. */
    int32_t k_rule;        /* MJP_K_TOL | MJP_K_PAPER */
    int32_t truncation;    /* MJP_CONSERVATIVE | MJP_LEAKY */
    int32_t renorm_every;  /* 0 = off; m > 0: every m jumps rescale rho to the initial mass
                              (valid only for conservative truncation; rejected otherwise) */
    int32_t lump;          /* 1 = add (1 - sum_{L..K} w_k) rho(0)B^K (last line of Algorithm 2) */
    int64_t k_cap;         /* largest K accepted; larger -> MJP_E_K_LIMIT */
    int32_t variant;       /* MJP_VARIANT_* */
    int32_t barrier_timeout_us; /* deadline of one grid or neighbour wait of the persistent
                              kernels: 0 = 2 s; > 0 microseconds.  < 0 exercises the
                              abort path: the two-jump kernel runs in a form whose waits
                              give up at their first unready read, so every workgroup
                              leaves and a call with info_h fails (other paths keep 2 s) */
    int32_t reserved[6];   /* must be zero */
} mjp_opts;

/* Fill *o with the defaults: omega_factor 1.1, tol 1e-9, MJP_K_TOL,
 * MJP_CONSERVATIVE, renorm_every 32, lump 1, k_cap 10^7, MJP_VARIANT_AUTO. */
void mjp_opts_default(mjp_opts* o);

/* ----------------------------------------------------------- result info */

enum { MJP_FLAG_NAN = 1,           /* a NaN/Inf appeared in rho(0) or in the iterate */
       MJP_FLAG_NEG = 2,           /* rho(0) had a negative entry */
       MJP_FLAG_UNDERFLOW_OBS = 4, /* an observed state had probability <= 0 in FP32 */
       MJP_FLAG_OUT_OF_GRID = 8,   /* an observation lies outside the state space */
       MJP_FLAG_K_LIMIT = 16,      /* (log-likelihood) an item needed K > k_cap; its value is -inf */
       MJP_FLAG_SUBNORMAL_OBS = 32 };/* (log-likelihood) an observed state's FP32 probability lay below
                                        FP32's normal range (1.18e-38): that log term has fewer than
                                        24 significant bits */

typedef struct {
    double  omega;          /* Omega */
    double  W;              /* Omega * t */
    double  eps_left;       /* sum_{k<L} w_k (FP64) */
    double  eps_right;      /* sum_{k>K} w_k (FP64) */
    double  residual;       /* 1 - sum_{k=L..K} w_k, lumped onto rho(0)B^K when opts.lump */
    double  mass_in;        /* sum of rho(0) (FP64 sum on the GPU) */
    double  mass_out;       /* sum of the result (FP64 sum on the GPU) */
    int32_t K;              /* number of products rho <- rho B */
    int32_t L;              /* first accumulated jump index */
    int32_t flags;          /* MJP_FLAG_* */
    int32_t path;           /* mjp_expv(_batched): the sweep that ran (MJP_PATH_*); 0 elsewhere */
} mjp_info;

enum { MJP_PATH_STEPWISE = 1,            /* one launch per jump */
       MJP_PATH_PERSISTENT = 2,          /* one launch, one jump per synchronisation */
       MJP_PATH_PERSISTENT_FENCED = 3,   /* the same, fenced protocol */
       MJP_PATH_PERSISTENT_TWOJUMP = 4,  /* one launch, two jumps per synchronisation */
       MJP_PATH_BATCHED_ITEM = 5,        /* mjp_expv_batched: one workgroup ran the item */
       MJP_PATH_PERSISTENT_MULTIJUMP = 6 };/* one launch, eight (else four) jumps per synchronisation on tiles */

/* ------------------------------------------------------------ operators */

/* Generator A in CSR form, on the host, FP64.  Row = from-state.  Column
 * indices strictly increasing within a row; the diagonal entry may be absent
 * only in a row with no off-diagonal entries. */
typedef struct {
    int32_t        n;        /* number of states N >= 1 */
    int32_t        nnz;      /* row_ptr[n] */
    const int32_t* row_ptr;  /* [n+1], row_ptr[0] = 0, non-decreasing */
    const int32_t* col_idx;  /* [nnz], 0 <= col < n */
    const double*  val;      /* [nnz], a_nm */
} mjp_csr;

/* Built-in reaction networks whose generator is computed on the fly.
 *   MJP_MODEL_BD: immigration-death (Eq. BD_def), theta = {beta, gamma},
 *     dims = {N, 1}, state n = count; n -> n+1 at beta, n -> n-1 at gamma n.
 *   MJP_MODEL_CASCADE2: two species on an S1 x S2 grid, theta = {k1, g1, k2, g2},
 *     dims = {S1, S2}, state n = n1 + S1 n2 (first coordinate fastest, as the
 *     paper linearises multi-index states, Sec. 3.1.2);
 *     (n1,n2) -> (n1+1,n2) at k1, -> (n1-1,n2) at g1 n1, -> (n1,n2+1) at k2 n1,
 *     -> (n1,n2-1) at g2 n2.
 *   MJP_MODEL_TWOSTATE: two-state birth-death (Sec. 3.1.2, Eq. 2S_chem),
 *     theta = {beta, gamma, lambda_act, lambda_ina}, dims = {N_R, 1}, state
 *     n = n_R + g N_R (g = 0 active, 1 inactive; N = 2 N_R); active births at
 *     beta, deaths at gamma n_R, active -> inactive at lambda_ina, inactive ->
 *     active at lambda_act.
 *   MJP_MODEL_AUTOREG: autoregulatory gene network (Sec. 3.1.3, Eq. STS_chem),
 *     theta = {beta_R, beta_P, gamma_R, gamma_P, lambda_act, lambda_ina},
 *     dims = {N_R, N_P}, state n = n_R + n_P N_R + g N_R N_P (N = 2 N_R N_P);
 *     active R births at beta_R, P births at beta_P n_R, deaths at gamma_R n_R
 *     and gamma_P n_P, active + P -> inactive at lambda_ina n_P, inactive ->
 *     active + P at lambda_act.
 * Stencil plans (mjp_plan_create_stencil) cover all four: the kernels form
 * each row's entries from theta and the state's coordinates (no matrix). */
enum { MJP_MODEL_BD = 0, MJP_MODEL_CASCADE2 = 1, MJP_MODEL_TWOSTATE = 2, MJP_MODEL_AUTOREG = 3 };

typedef struct {
    int32_t model;     /* MJP_MODEL_* */
    int32_t dims[2];
    double  theta[8];  /* rates, >= 0 and finite; unused entries ignored */
} mjp_model;

/* Number of states and stored entries of a model's generator under the given
 * truncation (host only, no GPU needed). */
mjp_status mjp_model_csr_size(const mjp_model* m, int32_t truncation, int32_t* n_h, int32_t* nnz_h);

/* Write the model's generator (Eq. A_def) into caller-allocated host CSR
 * arrays sized by mjp_model_csr_size (host only, no GPU needed).  Zero rates
 * are not stored. */
mjp_status mjp_model_csr(const mjp_model* m, int32_t truncation, int32_t* row_ptr_h,
                         int32_t* col_idx_h, double* val_h);

typedef struct mjp_plan mjp_plan;

/* Build a plan from a generator in CSR (Eq. A_def): checks it is a generator
 * (off-diagonals >= 0; row sums 0 within 1e-12 max|a_nn| under
 * MJP_CONSERVATIVE, <= that under MJP_LEAKY), computes Omega (Eq. B_def),
 * forms B^T in FP32 on the GPU in a sliced-ELL layout, and under
 * MJP_CONSERVATIVE sets each diagonal b_nn to 1 minus the FP64 sum of that
 * row's FP32 off-diagonals so every FP32 row of B sums to 1 to within one
 * rounding.  Copies what it needs; the caller's arrays may be freed after. */
mjp_status mjp_plan_create_csr(const mjp_csr* A, const mjp_opts* opts, mjp_plan** out);

/* Build a plan for a built-in model (any of the four): no matrix is stored,
 * the kernels compute each entry of B from theta when they need it -- the
 * same FP32 values a CSR plan of mjp_model_csr would hold up to the rounding
 * of rate/Omega * count (products of FP32 factors here), with the diagonal as
 * an FP32 pair so rows sum to their exact sum.  Omega comes from the same
 * FP64 maximum exit rate as for the CSR generator. */
mjp_status mjp_plan_create_stencil(const mjp_model* m, const mjp_opts* opts, mjp_plan** out);

/* Free a plan and its device memory.  NULL is accepted. */
void mjp_plan_destroy(mjp_plan* p);

/* Number of states of a plan (0 for NULL). */
int32_t mjp_plan_n(const mjp_plan* p);

/* ------------------------------------------------------------- solvers */

/* rho(t_j) for n_t times in one sweep of jumps (Algorithm 2 per time, all
 * times sharing the iterates rho(0)B^k).
 *   rho0_d   [N] FP32 on the device, entries >= 0 (the map is linear, so any
 *            total mass is allowed).
 *   t_h      [n_t] times on the host, finite and >= 0, any order.
 *   out_d    [n_t x N] FP32 on the device; row j is rho(t_h[j]).  Must not
 *            overlap rho0_d.
 *   info_h   [n_t] or NULL.  Non-NULL makes the call synchronous and returns
 *            MJP_E_NUMERIC if a NaN/Inf or negative entry was detected, or
 *            MJP_E_DEVICE if a wait of the persistent kernel missed its
 *            deadline (opts.barrier_timeout_us; every workgroup then left the
 *            kernel and out_d is not valid).
 * t = 0 and Omega = 0 (all rates zero) return rho0 unchanged.
 * Precision: the products run in FP32; the weighted series is accumulated
 * with Kahan compensation in FP32; the Poisson weights are FP64. */
mjp_status mjp_expv(mjp_plan* p, const float* rho0_d, int32_t n_t, const double* t_h,
                    float* out_d, mjp_info* info_h, mjp_stream_t stream);

/* B independent solves of Algorithm 2, item b: plans[b], rho0_d[b], n_t[b]
 * times t_h[b], outputs out_d[b] ([n_t[b] x N_b], the layout of mjp_expv).
 * info_h, if not NULL, holds sum_b n_t[b] entries in item order (path
 * MJP_PATH_BATCHED_ITEM for items of the batched sweep) and makes the call
 * synchronous, with mjp_expv's error rules.  Plans may repeat (the same
 * operator with several initial vectors).
 * Items whose vector one workgroup holds (N up to 512 R rows, R = 1..8 by
 * the row width; at most 48 times and 4 windows open at once) on the first
 * item's device, with opts.variant AUTO, PERSISTENT or PERSISTENT_ONEJUMP,
 * run in one launch per operator class (kind, rows per thread, entries per
 * row) after one launch that forms every item's Poisson weights: each
 * workgroup takes every grid-th item of the longest-first order and sweeps it with its
 * vector in LDS.  Such an item's output equals its own mjp_expv call's bit
 * for bit.  Every other item runs its own sweep (mjp_expv), in item order.
 * The batched sweep's workspace belongs to the library, one per (device,
 * stream); concurrent calls on one stream from several host threads are
 * not allowed. */
mjp_status mjp_expv_batched(int32_t B, mjp_plan* const* plans, const float* const* rho0_d,
                            const int32_t* n_t, const double* const* t_h, float* const* out_d,
                            mjp_info* info_h, mjp_stream_t stream);

/* Measurement aid, not a computation of the method: the floor that the
 * synchronisation of the plan's sweep sets (the tiled sweep with several
 * jumps per synchronisation where the plan's variant allows it, else the
 * two-jump sweep).  Runs `rounds` rounds of exactly its per-round
 * communication on this plan's launch configuration -- each workgroup loads
 * its halo rows of the iterate from global memory into LDS with
 * device-scope loads, stores its own rows with device-scope stores, drains
 * them, publishes its flag and waits for its neighbours' -- without the
 * arithmetic, and returns the mean time per round (HIP events on `stream`,
 * after one warm-up run) in *us_per_round_h, and (probe_exchange2) the
 * sweep's jumps per round in *jumps_h.  Synchronous.  MJP_E_UNSUPPORTED
 * when the plan's sweep synchronises every jump; MJP_E_INVALID_ARG for
 * rounds outside [1, 10^6]; MJP_E_DEVICE if a wait missed its 2 s deadline.
 * Overwrites the plan's iterate buffers. */
mjp_status mjp_probe_exchange(mjp_plan* p, int32_t rounds, double* us_per_round_h, mjp_stream_t stream);
mjp_status mjp_probe_exchange2(mjp_plan* p, int32_t rounds, double* us_per_round_h, int32_t* jumps_h,
                               mjp_stream_t stream);

/* Snapshot observations shared by every item of a log-likelihood batch
 * (Sec. 2.1.2): each observation is one system observed at one collection
 * time.  States are given as grid coordinates so items with different grid
 * sizes can share them; for MJP_MODEL_BD x2 must be 0. */
typedef struct {
    int32_t        n_t;      /* number of collection times */
    const double*  T_h;      /* [n_t] collection times, host, >= 0 */
    int32_t        n_obs;    /* number of (time, state) records */
    const int32_t* obs_h;    /* [n_obs x 4] host: (time index, x1, x2, count >= 1); the
                                observed counts: (n, 0) BD, (n1, n2) cascade, (n_R, 0)
                                two-state, (n_R, n_P) autoregulatory */
    int32_t        x0[2];    /* initial state, a point mass: (n, 0), (n1, n2), (n_R, gene
                                state 0/1) two-state, (n_R, n_P) autoregulatory (active) */
} mjp_obs;

/* Log-likelihoods of B parameter draws of one built-in model (any of the
 * four; for the two gene-state models the gene state is not observed and a
 * record's probability is the sum over it, Secs. 3.1.2-3.1.3):
 *   loglik_d[b] = sum_i count_i log rho_b(T_{j_i})_{(x1_i, x2_i)}
 * where rho_b solves the model with theta_d[b*4 .. b*4+3] on the grid
 * dims_d[b*2], dims_d[b*2+1] (conservative truncation).  Items are grouped
 * by size class (states <= mjp_loglik_class_limit(c), c < MJP_LL_CLASSES)
 * and each class runs in one persistent launch, longest item first, with the
 * class's launch shape (a default, or set by mjp_loglik_tune /
 * mjp_loglik_set_shapes); each item keeps its whole state vector in the LDS
 * of one workgroup, so S1*S2 <= mjp_loglik_max_states().
 * Only observed states are accumulated.  An observation outside an item's
 * grid, or with FP32 probability 0, gives -inf for that item (and a flag).
 *   theta_d  [B x P] FP64 device, P = 6 for MJP_MODEL_AUTOREG and 4 otherwise
 *            (BD uses the first 2 of each 4)
 *   dims_d   [B x 2] int32 device: {N, 1}, {S1, S2}, {N_R, 1} or {N_R, N_P}
 *   loglik_d [B] FP64 device
 *   info_d   [B] device or NULL (omega, W of the last time, K, L of the last
 *            time, flags, mass_out = final mass of the iterate)
 * Asynchronous on `stream`.  Buffers (library-owned, per device):
 *   - each distinct observation set (records and times) is uploaded once, by
 *     copies enqueued on the stream of the first call that uses it, into
 *     device buffers that are never rewritten, so kernels still in flight and
 *     captured graphs keep the records they were given; the 256 most recently
 *     used sets are kept (an older one is freed after a device
 *     synchronisation);
 *   - the work tables (windows, costs, order, queue counters) are kept per
 *     stream (64 streams; an older stream's are freed likewise), so calls on
 *     different streams never share them; a call with more items than its
 *     stream had before grows them (hipMalloc/hipFree);
 *   - with them, three streams of default priority per caller stream: the
 *     call forks its size classes onto them after the preparation kernels
 *     and joins them back into `stream` before it returns (events), so the
 *     call stays ordered on `stream` and a capture on it records the fork
 *     and the join.
 * A call on a stream that already ran one with at least this B and the same
 * observation set only enqueues kernels, so it may be captured in a hipGraph.
 * The graph uses that stream's work tables: it is invalidated by a later call
 * on the stream that grows them, and must not be replayed while another call
 * on that stream runs. */
mjp_status mjp_loglik(int32_t model, int32_t B, const double* theta_d, const int32_t* dims_d,
                      const mjp_obs* obs, const mjp_opts* opts, double* loglik_d,
                      mjp_info* info_d, mjp_stream_t stream);

/* mjp_loglik without any allocation, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight sampling loops, harnesses that
 * forbid hipMalloc).  Same arguments, kernels, launch shapes and results
 * (bit for bit) as mjp_loglik.  The call's tables (records, times, windows,
 * costs, order, queue counters) live in one fixed array of
 * mjp_loglik_noalloc_capacity() bytes (6 MiB) of device memory per GPU,
 * part of the library and held until the process ends; a call needs
 * mjp_loglik_noalloc_bytes(B, n_t, n_obs) of it (B (32 n_t + 8) + 16 n_obs +
 * 8 n_t plus alignment: for example B <= 8192 at 20 times and 1000 records)
 * and returns MJP_E_WORKSPACE, before any GPU work, when that exceeds the
 * capacity.  The records and times are copied from obs's host arrays by
 * copies enqueued on `stream`: keep those arrays unchanged until the stream
 * has passed the call (for a captured graph, while it is replayed).  Every
 * call on a GPU uses that GPU's one array, which keeps the last call's
 * contents: calls that overlap on one GPU (on different streams, or a graph
 * replayed while another call runs) race and give wrong results.  Calls no
 * hipMalloc, hipFree or allocating routine; the first call on a device looks
 * up the array's device address and sets kernel attributes. */
mjp_status mjp_loglik_noalloc(int32_t model, int32_t B, const double* theta_d, const int32_t* dims_d,
                              const mjp_obs* obs, const mjp_opts* opts, double* loglik_d,
                              mjp_info* info_d, mjp_stream_t stream);
/* Bytes of the array a mjp_loglik_noalloc call with these sizes needs (-1 for
 * negative sizes), and the array's size. */
int64_t mjp_loglik_noalloc_bytes(int32_t B, int32_t n_t, int32_t n_obs);
int64_t mjp_loglik_noalloc_capacity(void);

/* Which kernel computes the items of a model in mjp_loglik (and its tuner,
 * and mjp_loglik_noalloc) on the current device:
 *   MJP_LL_KERNEL_AUTO  (default) cascade items whose grid fits the column
 *       kernel -- S1 <= 992 columns, the S2 rows cut into at most 992 / S1
 *       segments of at most 64 rows, a column-major LDS mirror of at most
 *       40,256 floats -- run in it (each lane keeps one column segment in
 *       registers; left and right neighbours by cross-lane moves); every
 *       other item in the cell kernel;
 *   MJP_LL_KERNEL_CELLS every item in the cell kernel, whose launch shapes
 *       mjp_loglik_set_shapes and mjp_loglik_tune choose.
 * The other models always use the cell kernel. */
enum { MJP_LL_KERNEL_AUTO = 0, MJP_LL_KERNEL_CELLS = 1 };
mjp_status mjp_loglik_set_kernel(int32_t model, int32_t kernel);

/* Items of the cascade and birth-death models with more states than one
 * workgroup's LDS holds (S1*S2 > mjp_loglik_max_states()) run in clusters
 * of *group_h workgroups of one cooperative launch (each workgroup owns a
 * contiguous range of states and recomputes a halo three boundary rows
 * deep, so the boundary rows are exchanged every four jumps where the item
 * allows -- renorm_every a multiple of 4, S1 <= 512, at least four rows per
 * workgroup -- and every jump otherwise or when opts->variant is
 * MJP_VARIANT_PERSISTENT_ONEJUMP; the results are bit-identical either
 * way), up to *max_states_h states and, for the cascade, S1 <= 1024; larger items
 * (and any large item of the other models, or in mjp_loglik_noalloc) get
 * -inf with MJP_FLAG_OUT_OF_GRID.  Reports, for the current device, the
 * clusters that run co-resident (0: none, large items then get -inf), the
 * cluster workgroups that fit one CU and whether cooperative launches are
 * supported.  Any pointer may be NULL. */
mjp_status mjp_loglik_cluster_config(int32_t* clusters_h, int32_t* per_cu_h, int32_t* coop_h, int32_t* group_h,
                                     int32_t* max_states_h);

/* Largest S1*S2 a log-likelihood item may have (LDS capacity of one CU). */
int32_t mjp_loglik_max_states(void);

/* Launch shapes of the batched log-likelihood (not in the paper: how the
 * batch maps onto the chip).  A shape is T threads per workgroup, each
 * owning C cells of the item's state vector; it holds up to
 * max_states = min(T*C, mjp_loglik_max_states()) states in lds_bytes of LDS,
 * so smaller shapes let several workgroups share a CU, and a shape with T
 * threads takes at most 4*T observation records.  Size class c holds the
 * items with mjp_loglik_class_limit(c-1) < S1*S2 <= mjp_loglik_class_limit(c);
 * a shape may run class c if max_states >= mjp_loglik_class_limit(c). */
#define MJP_LL_CLASSES 4
#define MJP_LL_MAX_SHAPES 16

typedef struct {
    int32_t threads, cells, max_states, lds_bytes;
    int32_t reserved[4];
} mjp_ll_shape;

typedef struct {
    int32_t items[MJP_LL_CLASSES];                    /* items of the batch per class */
    int32_t chosen[MJP_LL_CLASSES];                   /* shape now used per class */
    float   ms[MJP_LL_CLASSES][MJP_LL_MAX_SHAPES];    /* fastest of reps runs of (class,
                                                         shape) in ms; -1 = not timed */
} mjp_ll_tune_report;

int32_t    mjp_loglik_num_shapes(void);
/* MJP_E_INVALID_ARG for id outside [0, mjp_loglik_num_shapes()). */
mjp_status mjp_loglik_shape(int32_t id, mjp_ll_shape* out_h);
/* Largest S1*S2 of class cls (0 for cls outside [0, MJP_LL_CLASSES)). */
int32_t    mjp_loglik_class_limit(int32_t cls);

/* Shapes per class for a model on the current device: ids_h[MJP_LL_CLASSES],
 * -1 = the default.  MJP_E_INVALID_ARG if a shape cannot hold its class.
 * A call whose records exceed a chosen shape's 4*T uses the default. */
mjp_status mjp_loglik_set_shapes(int32_t model, const int32_t* ids_h);
/* The shapes a call with n_rec records would use now (defaults resolved). */
mjp_status mjp_loglik_get_shapes(int32_t model, int32_t n_rec, int32_t* ids_h);

/* On-disk cache of the autotuner's choices (a build aid, not in the paper):
 * mjp_loglik_save_shapes writes the shape chosen for every (model, size
 * class) on the current device -- by mjp_loglik_tune, mjp_loglik_set_shapes
 * or the defaults (-1) -- to the text file `path`, keyed by the device's
 * architecture, compute-unit count and product name and by this library's
 * shape table (number of shapes, class limits).  mjp_loglik_load_shapes reads
 * such a file and applies it to the current device; the whole file is
 * checked first and nothing changes on an error: MJP_E_INVALID_ARG if it
 * cannot be read or is not a complete, valid cache; MJP_E_UNSUPPORTED if it
 * was written on another GPU or by a build with another shape table (tune
 * again there); MJP_E_DEVICE if no device can be queried. */
mjp_status mjp_loglik_save_shapes(const char* path);
mjp_status mjp_loglik_load_shapes(const char* path);

/* Autotuner: runs the batch of mjp_loglik (same arguments) once per
 * eligible shape and size class (after one warm-up run each, reps timed
 * runs, HIP events on `stream`), keeps the fastest shape per class for this
 * model on the current device, and reruns the chosen shapes, so loglik_d and
 * info_d hold what mjp_loglik now returns.  Synchronous; do not call it
 * while a graph is being captured.  report_h (host, may be NULL) gets the
 * class sizes, the timings and the choice.  Results of different shapes
 * differ only in the rounding of the mass renormalisation's block sums. */
mjp_status mjp_loglik_tune(int32_t model, int32_t B, const double* theta_d, const int32_t* dims_d,
                           const mjp_obs* obs, const mjp_opts* opts, double* loglik_d, mjp_info* info_d,
                           int32_t reps, mjp_ll_tune_report* report_h, mjp_stream_t stream);

/* J-MJP state probabilities (Method #2, Sec. 2.2.2, the algorithm of the
 * state probabilities for J-MJP): for each draw b and observation i,
 *   logphi_d[b*I + i] = log p(s_i | k_i, theta_b) = log (rho(0) B_b^{k_i})_{s_i}
 * with B_b = I + A_b / Omega_b, Omega_b = omega_factor * max|a_nn| (the same
 * Omega as mjp_loglik), k_i = k_d[b*I + i] the observation's own number of
 * virtual jumps, I = obs->n_obs, and s_i the record's state (for the two
 * gene-state models summed over the hidden gene state).  Every record's
 * count must be 1 (each observation has its own jump count); the record's
 * time index is not used here (the caller needs T for the jump-count prior
 * Poisson(k | Omega_b T)).  One sweep per draw to max_i k_i, the iterate in
 * LDS as in mjp_loglik (same size classes, default shapes), FP32 jumps and
 * mass renormalisation, FP64 logs.
 *   k_d      [B x I] int32 device; a draw with some k_i < 0 or > opts->k_cap
 *            gets -inf everywhere and MJP_FLAG_K_LIMIT
 *   logphi_d [B x I] FP64 device; -inf where the FP32 probability is 0 or the
 *            state is off the draw's grid
 *   omega_d  [B] FP64 device or NULL: Omega_b
 * Asynchronous; opts->tol and variant are not used. */
mjp_status mjp_jump_probs(int32_t model, int32_t B, const double* theta_d, const int32_t* dims_d,
                          const mjp_obs* obs, const int32_t* k_d, const mjp_opts* opts, double* logphi_d,
                          double* omega_d, mjp_stream_t stream);

/* ------------------------------------------------ surrogate (not in paper) */

typedef struct mjp_surrogate mjp_surrogate;

typedef struct {
    int32_t in_dim;   /* inputs (standardised log-parameters), 1..16 */
    int32_t width;    /* hidden width, multiple of 64, <= 512 */
    int32_t depth;    /* number of hidden layers (Linear+GELU), 1..8 */
} mjp_mlp_cfg;

typedef struct {
    int32_t epochs;
    int32_t batch;        /* minibatch, multiple of 512 in [512, 65536]; the last one of an epoch may be short */
    float   lr;           /* Adam step size */
    float   beta1, beta2, eps_adam;
    float   weight_decay; /* decoupled, 0 = off */
    uint64_t seed;        /* minibatch shuffling */
} mjp_train_cfg;

/* Create an MLP in->width->...->width->1 with GELU z*Phi(z) between the
 * Linear layers, FP32 master weights initialised from seed (uniform in
 * +-1/sqrt(fan_in)), BF16 copies used by the matrix-core kernels.  Not part
 * of the paper: a learned stand-in for the log-likelihood over log-rates,
 * screening proposals in delayed-acceptance sampling. */
mjp_status mjp_surrogate_create(const mjp_mlp_cfg* cfg, uint64_t seed, mjp_surrogate** out);
void       mjp_surrogate_destroy(mjp_surrogate* s);

/* Mean-squared-error training with Adam on x_d [n x in_dim] FP32 and targets
 * y_d [n] FP32 (device).  loss_h [epochs] receives the mean training loss of
 * each epoch (the call is synchronous when loss_h is not NULL).  For width
 * <= 256 a step is three launches (forward, loss and backward-data products
 * of 16 rows per workgroup with activations in LDS; every layer's
 * weight-gradient partials; Adam); wider nets run one launch per product.
 * Both are deterministic: the same seed and data give the same parameters. */
mjp_status mjp_surrogate_train(mjp_surrogate* s, const float* x_d, const float* y_d, int32_t n,
                               const mjp_train_cfg* cfg, float* loss_h, mjp_stream_t stream);

/* Mean-squared-error loss and its gradient with respect to every parameter
 * for one batch of n <= 65536 rows, without updating anything (for checking
 * the backward kernels).  grad_h [num_params] FP32 in the packing of
 * mjp_surrogate_get_params; loss_h [1] or NULL.  Synchronous. */
mjp_status mjp_surrogate_grad(const mjp_surrogate* s, const float* x_d, const float* y_d, int32_t n, float* grad_h,
                              float* loss_h, mjp_stream_t stream);

/* y_d[i] = MLP(x_d[i]) for n inputs (device FP32). */
mjp_status mjp_surrogate_infer(const mjp_surrogate* s, const float* x_d, int32_t n, float* y_d,
                               mjp_stream_t stream);

/* Copy the FP32 master parameters to/from host memory: layer l weight
 * [out x in] row-major then bias [out], layers in order.  Count = params_h
 * size, checked against mjp_surrogate_num_params. */
int64_t    mjp_surrogate_num_params(const mjp_surrogate* s);
mjp_status mjp_surrogate_get_params(const mjp_surrogate* s, float* params_h, int64_t count);
mjp_status mjp_surrogate_set_params(mjp_surrogate* s, const float* params_h, int64_t count);

/* Save / load the configuration and FP32 master parameters (little-endian
 * binary, magic "MJPS"). */
mjp_status mjp_surrogate_save(const mjp_surrogate* s, const char* path);
mjp_status mjp_surrogate_load(const char* path, mjp_surrogate** out);

/* ------------------------------------------------------ device samplers */

/* Metropolis-Hastings and delayed-acceptance chains on the GPU (SI:
 * sampling scheme and prior; Christen and Fox 2005 for delayed acceptance).
 * C chains random-walk in log-rates psi = log(theta), proposal psi' = psi +
 * L z with z ~ Normal(0, I) (L: lower Cholesky factor of the proposal
 * covariance), prior Normal(prior_mu, prior_sigma) on every log-rate.  Each
 * scored proposal's log-likelihood is mjp_loglik's (model, grid, obs, opts).
 *   Plain MH:  accept with min(1, exp(post(psi') - post(psi))).
 *   Delayed acceptance (a screen is set): stage 1 accepts with min(1,
 *     exp(s(psi') - s(psi))), s = the surrogate's log-likelihood (its
 *     standardised output times ll_std plus ll_mean, inputs (psi - mean) /
 *     std) plus the exact log-prior; only stage-1 survivors are scored
 *     exactly, and stage 2 accepts with min(1, exp((post(psi') - post(psi))
 *     - (s(psi') - s(psi)))), so the exact posterior stays invariant.
 * Random numbers: Philox4x32-10 (Salmon et al., SC 2011) keyed by cfg.seed
 * with counter (chain, step mod 2^32, step / 2^32, block): blocks 0-2 give
 * the normals (Box-Muller on 53-bit uniforms), block 3 the uniforms u1
 * (stage 1) and u2 (MH test, stage 2).  The same seed, covariance and start
 * give the same chains on every run, and plain MH equals delayed acceptance
 * whose screen is constant.
 * A step is a fixed sequence of kernel launches on the stream with no host
 * read (the masked likelihood skips stage-1 rejects on the device), so a
 * step may be captured in a graph once the same call has run eagerly on
 * the same stream (which sizes the likelihood's tables). */
typedef struct mjp_sampler mjp_sampler;

typedef struct {
    int32_t  model;        /* MJP_MODEL_*: the chains sample its 2, 4 or 6 log-rates */
    int32_t  dims[2];      /* the grid of every likelihood (mjp_loglik's dims; dims[1] unused for BD) */
    int32_t  chains;       /* C, 1 .. 2^24 */
    uint64_t seed;         /* Philox key */
    double   prior_mu;     /* Normal prior on every log-rate */
    double   prior_sigma;
} mjp_sampler_cfg;

void       mjp_sampler_cfg_default(mjp_sampler_cfg* cfg);  /* cascade, 256 chains, seed 1, prior (1, 1e5) */
/* Copies obs (host arrays) and opts; device buffers for cfg->chains chains
 * on the current device.  MJP_E_INVALID_ARG on a bad model, grid, chain
 * count, prior or empty observations. */
mjp_status mjp_sampler_create(const mjp_sampler_cfg* cfg, const mjp_obs* obs, const mjp_opts* opts,
                              mjp_sampler** out);
void       mjp_sampler_destroy(mjp_sampler* s);
/* chol_h [d x d] row-major, lower triangular, finite (d = the model's
 * log-rate count). */
mjp_status mjp_sampler_set_proposal(mjp_sampler* s, const double* chol_h);
/* screen NULL: plain MH.  Otherwise delayed acceptance with this surrogate
 * (borrowed, must outlive the runs) and its standardisation: psi_mean_h,
 * psi_std_h [d] (std > 0), output scale ll_mean, ll_std > 0.  Takes effect
 * at the next mjp_sampler_init. */
mjp_status mjp_sampler_set_screen(mjp_sampler* s, const mjp_surrogate* screen, const double* psi_mean_h,
                                  const double* psi_std_h, double ll_mean, double ll_std);
/* psi0_d [C x d] device: the chains' states; scores them (and screens them)
 * and zeroes the step and the counters. */
mjp_status mjp_sampler_init(mjp_sampler* s, const double* psi0_d, mjp_stream_t stream);
/* steps steps; samples_d [ring_rows x C x d] device or NULL: after step h
 * the states go to row h mod ring_rows (h counts from 0 since init). */
mjp_status mjp_sampler_run(mjp_sampler* s, int32_t steps, double* samples_d, int32_t ring_rows,
                           mjp_stream_t stream);
/* Checkpoint: states psi_h [C x d], log-posteriors lp_h [C], screened
 * log-posteriors sc_h [C] and counters_h [4] = (steps, accepted, stage-1
 * accepted, exact evaluations), host, synchronous.  set_state restores them
 * (same cfg, proposal and screen): the continued chains equal the
 * uninterrupted ones. */
mjp_status mjp_sampler_get_state(const mjp_sampler* s, double* psi_h, double* lp_h, double* sc_h,
                                 uint64_t* counters_h, mjp_stream_t stream);
mjp_status mjp_sampler_set_state(mjp_sampler* s, const double* psi_h, const double* lp_h, const double* sc_h,
                                 const uint64_t* counters_h, mjp_stream_t stream);
/* The generator itself: out4 = Philox4x32-10(ctr4, key2) on the host, and
 * out_d[4i .. 4i+3] = Philox4x32-10((i, c1, c2, c3), key) on the device for
 * i < n. */
void       mjp_philox4x32_10(const uint32_t* ctr4, const uint32_t* key2, uint32_t* out4);
mjp_status mjp_philox_fill(uint64_t key, uint32_t c1, uint32_t c2, uint32_t c3, int32_t n, uint32_t* out_d,
                           mjp_stream_t stream);

/* Device Poisson draws: out_d[i] ~ Poisson(lam_d[i]) from the generator
 * keyed by key with counter (i, c1, 0, attempt): inversion below mean 10,
 * the transformed rejection method of Hoermann (1993) above. */
mjp_status mjp_poisson_fill(uint64_t key, uint32_t c1, const double* lam_d, int32_t n, int32_t* out_d,
                            mjp_stream_t stream);

/* J-MJP Gibbs chains on the device (Method #2, Sec. 2.2.2, Eq.
 * sample_J-MJP): per step every jump count k_i is proposed from
 * Poisson(Omega_theta T_i) (its prior, the SI's proposal) and accepted with
 * min(1, phi(k') / phi(k)), phi = mjp_jump_probs; then theta takes a
 * Gaussian random-walk step in log space (mjp_sampler's proposal and prior)
 * with target p(theta) prod_i Poisson(k_i | Omega_theta T_i) phi_i.  Every
 * record's count must be 1 (one jump count per observation).  Random
 * numbers: the sampler's Philox generator keyed by cfg.seed (counters
 * (chain, observation, step, attempt) for the counts, (chain, 2^32 - 1,
 * step, block) for theta).  No host read inside a step. */
typedef struct mjp_jmjp mjp_jmjp;
mjp_status mjp_jmjp_create(const mjp_sampler_cfg* cfg, const mjp_obs* obs, const mjp_opts* opts, mjp_jmjp** out);
void       mjp_jmjp_destroy(mjp_jmjp* s);
mjp_status mjp_jmjp_set_proposal(mjp_jmjp* s, const double* chol_h);
/* psi0_d [C x d] device; the jump counts start from their prior at psi0 and
 * take k_burn sweeps at fixed psi0; the step and the counters restart. */
mjp_status mjp_jmjp_init(mjp_jmjp* s, const double* psi0_d, int32_t k_burn, mjp_stream_t stream);
/* as mjp_sampler_run */
mjp_status mjp_jmjp_run(mjp_jmjp* s, int32_t steps, double* samples_d, int32_t ring_rows, mjp_stream_t stream);
/* counters_h [4]: steps, theta accepted, jump counts accepted, jump counts proposed (synchronous) */
mjp_status mjp_jmjp_counters(const mjp_jmjp* s, uint64_t* counters_h, mjp_stream_t stream);

/* --------------------------------------- Krylov propagator (Method #5) */

/* rho(0) exp(A t) by Krylov-subspace steps (Sec. 2.2.5, Algorithm
 * ArnoldiKrylov and Eq. Krylov_expansion), in FP64: per step of length dt
 * an orthonormal basis q_1 = rho/||rho||, q_i from q_{i-1} A (kappa - 1
 * products, H kappa x kappa with a zero last column), and
 * rho(t + dt) = ||rho|| sum_i [exp(H dt)]_{i,1} q_i.  dt = dt_factor * kappa
 * / max|a_nn|; the last step before each requested time is shortened so the
 * propagation lands on it.  The paper's choice dt_factor = 2 is stable but
 * leaves an L1 error of order 1e-3 on stiff problems; dt_factor = 0.5 is
 * accurate to ~1e-11 on the same problems (4x the steps). */
typedef struct mjp_krylov mjp_krylov;

typedef struct {
    int32_t kappa;       /* basis size, 2..32 (the paper: 20) */
    int32_t variant;     /* MJP_KRYLOV_AUTO | MJP_KRYLOV_PASSES | MJP_KRYLOV_FUSED */
    double  dt_factor;   /* > 0 (the paper: 2) */
    int32_t reserved[6];
} mjp_krylov_opts;

/* How a step runs.  PASSES: one launch per pass over the vectors (three per
 * Arnoldi iteration, the exponential, the combination).  FUSED: the whole
 * step in one cooperative launch with grid barriers between the passes
 * (needs cooperative launch, every workgroup co-resident and N <= 8 rows per
 * thread of the grid, i.e. N <= 1,048,576 on 256 CUs).  AUTO: PASSES -- a
 * grid-wide sum inside the fused step (block sums, a grid barrier, every
 * workgroup adding the partials) costs about what the kernel boundary it
 * replaces does, so the fused step is slower at N = 10^6.  Both compute the
 * same arithmetic; the sums across workgroups add the same per-workgroup
 * partials in different fixed orders, so the two agree to rounding, and
 * each is deterministic. */
enum { MJP_KRYLOV_AUTO = 0, MJP_KRYLOV_PASSES = 1, MJP_KRYLOV_FUSED = 2 };

typedef struct {
    double  m_theta;     /* max |a_nn| */
    double  dt;          /* full step length */
    int64_t steps;       /* steps taken over all requested times */
    int32_t kappa;
    int32_t fused;       /* 1 if the steps ran as one cooperative launch each */
    int32_t reserved[4];
} mjp_krylov_info;

/* Defaults: kappa 20, dt_factor 2. */
void mjp_krylov_opts_default(mjp_krylov_opts* o);

/* Builds A^T (FP64 sliced ELL) and the kappa x N basis workspace on the
 * current device.  A is checked like mjp_plan_create_csr (conservative rows:
 * MJP_E_NOT_GENERATOR on a negative rate or a row sum off 0).  A variant
 * outside the enum is MJP_E_INVALID_ARG; MJP_KRYLOV_FUSED where the fused
 * step does not fit is MJP_E_UNSUPPORTED.  The handle owns all device memory
 * until mjp_krylov_destroy. */
mjp_status mjp_krylov_create(const mjp_csr* A, const mjp_krylov_opts* opts, mjp_krylov** out);
void       mjp_krylov_destroy(mjp_krylov* k);
int32_t    mjp_krylov_n(const mjp_krylov* k);

/* out_d[j*N .. j*N+N-1] = rho0_d exp(A t_h[j]) for j < n_t (times in any
 * order, >= 0; one propagation through the sorted times).  rho0_d and out_d
 * are FP64 device vectors owned by the caller; rho0_d is only read.
 * Asynchronous on `stream`; info_h (host, may be NULL) gets the step count.
 * With info_h on the fused path the call waits for the stream and returns
 * MJP_E_DEVICE if a grid barrier missed its deadline (every workgroup then
 * left the step; the output is not valid).  A handle must not be used on two
 * streams at once. */
mjp_status mjp_krylov_expv(mjp_krylov* k, const double* rho0_d, int32_t n_t, const double* t_h, double* out_d,
                           mjp_krylov_info* info_h, mjp_stream_t stream);

/* ----------------------------- Runge-Kutta propagator (Method #4) */

/* rho(0) propagated by the classical fourth-order Runge-Kutta step
 * (Sec. 2.2.4, Eqs. RKstep and RKintermediate), in FP64, with rates that may
 * change in time: A(t) = sum_c g_c(t) A_c over 1..8 channels.  Each channel
 * A_c is a generator (checked like mjp_plan_create_csr, conservative rows)
 * and g_c(t) >= 0 is piecewise linear through the knots set with
 * mjp_rk4_set_schedule, constant outside them (default: g_c = 1).  Step
 * dt = dt_factor / m with m = max over the knots of max_n |a_nn(t)|
 * (dt_factor 1 is the paper's stability bound); the last step before each
 * requested time is shortened to land on it.  Error O(dt^4). */
typedef struct mjp_rk4 mjp_rk4;

typedef struct {
    double  dt_factor;   /* > 0 (the paper's bound: 1) */
    int32_t reserved[6];
} mjp_rk4_opts;

typedef struct {
    double  m;           /* max over the schedule of max |a_nn(t)| */
    double  dt;          /* full step length (inf when m = 0) */
    int64_t steps;       /* steps taken over all requested times */
    int32_t reserved[6];
} mjp_rk4_info;

/* Defaults: dt_factor 1. */
void mjp_rk4_opts_default(mjp_rk4_opts* o);

/* Merges the channels' A_c^T into one FP64 sliced-ELL operator (entry:
 * source state, rate, channel) on the current device; every channel has the
 * same n.  MJP_E_INVALID_ARG on n_channels outside 1..8 or mismatched sizes,
 * MJP_E_NOT_GENERATOR as for a CSR plan.  The handle owns its device memory
 * (operator + five N-vectors) until mjp_rk4_destroy. */
mjp_status mjp_rk4_create(int32_t n_channels, const mjp_csr* channels, const mjp_rk4_opts* opts, mjp_rk4** out);

/* The same propagator for a built-in model given as rates (mjp_model, as
 * for mjp_model_csr): the channels are the model's reactions in the order of
 * its theta, each with its own schedule (mjp_rk4_set_schedule) --
 *   birth-death: 0 birth (theta[0]), 1 death (theta[1] n);
 *   cascade at (x, y): 0 birth of x (theta[0]), 1 death of x (theta[1] x),
 *     2 birth of y (theta[2] x), 3 death of y (theta[3] y);
 *   two-state (Sec. 3.1.2): 0 birth (theta[0], active gene), 1 death
 *     (theta[1] n), 2 activation (theta[2]), 3 inactivation (theta[3]);
 *   autoregulatory (Sec. 3.1.3): 0 R birth (theta[0], active), 1 P birth
 *     (theta[1] n_R), 2 R death (theta[2] n_R), 3 P death (theta[3] n_P),
 *     4 unbinding (theta[4]), 5 binding (theta[5] n_P).
 * Births that would leave the grid are dropped, as in mjp_model_csr.  The
 * stage kernel forms A(t)'s entries from the state's coordinates, so a stage
 * streams only the N-vectors.  MJP_E_INVALID_ARG as for mjp_model_csr.  The
 * handle owns five FP64 N-vectors until mjp_rk4_destroy. */
mjp_status mjp_rk4_create_stencil(const mjp_model* model, const mjp_rk4_opts* opts, mjp_rk4** out);
void       mjp_rk4_destroy(mjp_rk4* k);
int32_t    mjp_rk4_n(const mjp_rk4* k);

/* g_c(t) through (t_knots[i], g_knots[i]), i < n_knots (host arrays, copied):
 * times strictly increasing and finite, values finite and >= 0. */
mjp_status mjp_rk4_set_schedule(mjp_rk4* k, int32_t channel, int32_t n_knots, const double* t_knots,
                                const double* g_knots);

/* out_d[j*N .. j*N+N-1] = rho(t_h[j]) for j < n_t (times in any order, >= 0;
 * one propagation through the sorted times).  rho0_d and out_d are FP64
 * device vectors owned by the caller; rho0_d is only read.  Asynchronous on
 * `stream`; info_h (host, may be NULL) gets m, dt and the step count.  A
 * handle must not be used on two streams at once. */
mjp_status mjp_rk4_expv(mjp_rk4* k, const double* rho0_d, int32_t n_t, const double* t_h, double* out_d,
                        mjp_rk4_info* info_h, mjp_stream_t stream);

/* ---------------------------------------------------------------- misc */

/* Message describing the last failure on this thread ("" if none). */
const char* mjp_last_error(void);

/* Library version string. */
const char* mjp_version(void);

/* Waits for every device the library used and frees the device memory,
 * pinned host memory and events the library itself owns (the
 * log-likelihood's observation sets and work tables, the batched sweep's
 * workspaces); later calls rebuild them.  Handles the caller owns (plans,
 * Krylov, RK4 and surrogate handles) are not touched, and the fixed array
 * of mjp_loglik_noalloc stays.  For a clean process exit (the Python
 * binding calls it at interpreter exit); not thread-safe with other calls.
 * MJP_E_DEVICE if a device call fails. */
mjp_status mjp_shutdown(void);

#ifdef __cplusplus
}
#endif
#endif /* MJP_H */
