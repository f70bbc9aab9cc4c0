/*
 * tca.h -- C ABI of the MI355X (gfx950) traveling cluster approximation
 * library (libtca.so).
 *
 * The method is the parallelized traveling cluster approximation (TCA) of
 * Mukherjee, Patel, Bishop and Dagotto, arXiv:1502.07028.  A Monte Carlo
 * sweep visits every site of an L x L periodic lattice of classical unit
 * spins; for each site it diagonalizes a small periodic cluster Hamiltonian
 * before and after a random change of that site's spin and accepts the
 * change by Metropolis (Sec. II(c), Fig. 2).  The sweep is split into four
 * quadrant blocks whose clusters are independent and are all solved in one
 * batched launch (Sec. III(a), Fig. 3 and Fig. 4).
 *
 * Model (double exchange, classical spins S_i, |S_i| = 1):
 *   H = -t sum_<ij>,s c+_is c_js - (J_H/2) sum_i S_i.(c+_i sigma c_i)
 *       + J_AF sum_<ij> S_i.S_j
 * Cluster: the Lc x Lc patch whose corner (0,0) is the update site, periodic
 * in itself; basis index 2*(a + Lc*b) + spin.  Cluster energy: the fermionic
 * grand potential F = -T sum_i ln(1 + exp(-(eps_i - mu)/T)); the classical
 * term uses the four lattice neighbours of the update site.
 *
 * Conventions for every entry point
 *   - Every function returns a tca_status (0 = TCA_OK, negative = error) and
 *     never aborts or throws across the ABI; tca_last_error() gives a
 *     thread-local message for the last failure on the calling thread.
 *   - Pointers documented as "host" are ordinary host memory, read or written
 *     before the call returns.  The library owns all device memory it
 *     allocates; it is released by tca_destroy().
 *   - Spins are stored as N x 3 doubles (x, y, z), site p = x + L*y.
 *   - All work of one context is issued on the context's HIP stream; calls on
 *     one context must not overlap (one context per host thread).
 *   - Random numbers: Philox4x64-10 with key (seed, 0) and counter
 *     (sweep, site, stream, attempt); results do not depend on batching.
 */
#ifndef TCA_H
#define TCA_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define TCA_ABI_VERSION 2

typedef enum {
  TCA_OK = 0,
  TCA_E_INVAL = -1,        /* invalid argument (sizes, NULL, non-unit spin, ...) */
  TCA_E_NOMEM = -2,        /* device or host allocation failed */
  TCA_E_DEVICE = -3,       /* a HIP runtime call or kernel launch failed */
  TCA_E_UNSUPPORTED = -4,  /* valid request the library does not implement */
} tca_status;

enum { TCA_FP64 = 0, TCA_MIXED = 1 };  /* precision of the tridiagonal reduction */
enum { TCA_INIT_RANDOM = 0, TCA_INIT_FERRO = 1, TCA_INIT_NEEL = 2, TCA_INIT_USER = 3 };
/* tca_params.flags bits */
enum {
  TCA_FLAG_PROFILE = 1,      /* time every kernel launch of a sweep with HIP events */
  TCA_FLAG_NO_GRAPH = 2,     /* issue every launch directly instead of replaying a captured sweep */
  TCA_FLAG_NO_AUTOTUNE = 4,  /* keep the default reducer variants (no timing at init) */
  TCA_FLAG_EXACT_METROPOLIS = 8, /* evaluate every Metropolis test in its exact form (u < exp(-dE/T),
                                    or the delayed-acceptance quotient) instead of comparing ln u with
                                    -dE/T outside a relative 1e-10 band; the decisions are the same */
};

typedef struct {
  int32_t abi_version;   /* must be TCA_ABI_VERSION */
  int32_t L;             /* lattice linear size, even, >= 4 */
  int32_t Lc;            /* cluster linear size when n_classes == 0: 2 <= Lc <= L/2+1, Lc <= 10 */
  int32_t n_classes;     /* 0: every update uses Lc; 1..4: size drawn per update from Lc_classes */
  int32_t Lc_classes[4]; /* cluster sizes to draw from (each obeys the Lc bounds) */
  double t, JH, JAF, mu; /* hopping, Hund coupling, superexchange, chemical potential */
  uint64_t seed;         /* Philox key word 0 */
  int32_t precision;     /* TCA_FP64 or TCA_MIXED */
  int32_t init;          /* TCA_INIT_*; USER takes spins_xyz */
  int32_t flags;         /* TCA_FLAG_* bits; other bits must be 0 */
  int32_t reserved;
} tca_params;

/* One Monte Carlo update, in visiting order (block-major, raster in block). */
typedef struct {
  int32_t site;   /* lattice site p */
  int16_t Lc;     /* cluster linear size used */
  uint8_t accept; /* 1 if the proposal was accepted */
  uint8_t flags;  /* bit 0: near-threshold of the exact test (|T ln u - rhs| <= 1e-9 max(|dE|,1e-3));
                     bit 1: the update reached the exact stage (always set without a surrogate);
                     bit 2: near-threshold of the surrogate stage */
  double dF;      /* F_new - F_old of the cluster (NaN if the surrogate stage rejected it) */
  double dE;      /* dF + classical change (NaN likewise) */
  double u;       /* the Metropolis uniform */
  float dS_f;     /* surrogate dF of the move (0 without a surrogate) */
  float dS_r;     /* surrogate dF of the reverse move */
} tca_update_record;

typedef struct {
  int64_t updates;
  int64_t accepted;
  int64_t near_threshold;
  double elapsed_ms;        /* device time of the sweeps (HIP events) */
  /* filled only with TCA_FLAG_PROFILE (else 0): summed durations and counts
   * of the per-block phases -- Householder reductions of all cluster matrices
   * of a block (one launch, or one per size class, timed together),
   * tridiagonal eigenvalues + free energies, and Metropolis decisions */
  double reduce_ms;
  double eig_ms;
  double decide_ms;
  int64_t reduce_launches;
  int64_t eig_launches;
  int64_t decide_launches;
  int64_t stage1_passed;    /* updates that reached the exact stage (= updates without a surrogate) */
  double surrogate_ms;      /* with TCA_FLAG_PROFILE: delayed-acceptance stage 1 (features, MLP, flags) */
  int64_t surrogate_launches;
} tca_sweep_stats;

typedef struct tca_ctx tca_ctx;
typedef struct tca_surrogate tca_surrogate;

/* Create a lattice context on the current HIP device.
 *   p          host; validated (TCA_E_INVAL on a bad size, precision or flag)
 *   spins_xyz  host N x 3 initial spins when p->init == TCA_INIT_USER (each
 *              |S| within 1e-12 of 1, else TCA_E_INVAL), otherwise ignored
 *   hip_stream hipStream_t to issue all work on; NULL: a stream the context
 *              creates and owns (default priority)
 *   out        receives the context (NULL on failure)
 * Random initial spins are uniform on the sphere (Philox stream 3).
 * Unless TCA_FLAG_NO_AUTOTUNE is set, the first context of the process that
 * uses a cluster size (per precision) times every reducer variant of that
 * size on its own block-0 clusters and records the fastest for the process
 * (tca_tuning_report shows the timings).  Sweeps without a log, collection or
 * profiling are captured once as a HIP graph and replayed per sweep (the
 * kernels read the sweep counter and T from device memory) unless
 * TCA_FLAG_NO_GRAPH is set. */
int tca_init_lattice(const tca_params* p, const double* spins_xyz, void* hip_stream,
                     tca_ctx** out);

/* Run nsweeps Monte Carlo sweeps (Sec. II(c) Fig. 2 semantics, executed as the
 * four-block schedule of Sec. III(a)).  Sweep s uses temperature T[s] (host,
 * length nsweeps, each > 0) and Philox sweep counter (context counter + s);
 * the context counter then advances by nsweeps.
 *   log  host, NULL or nsweeps * L*L records in visiting order
 *   st   host, NULL or receives totals over the call
 * Blocks until the work is done. */
int tca_sweep(tca_ctx* c, const double* T, int32_t nsweeps, tca_update_record* log,
              tca_sweep_stats* st);

/* Eigenvalues (ascending) of the cluster matrices around `sites` in the
 * current state, computed by the same kernels as tca_sweep (Sec. II(b),
 * Fig. 2 steps (b) and (d)).
 *   sites        host, count lattice sites
 *   Lc           host, count cluster sizes, or NULL for the context's Lc
 *   proposed_xyz host, count x 3 spins placed at the cluster corner, or NULL
 *   eig          host, count x ld doubles; row r holds 2*Lc[r]^2 values
 * TCA_E_INVAL if ld < 2*Lc^2 for some row or a size is out of range. */
int tca_cluster_eigvals(tca_ctx* c, const int32_t* sites, const int32_t* Lc,
                        const double* proposed_xyz, int32_t count, double* eig, int32_t ld);

/* Snapshot of the state and its observables (Eq. (2) for one configuration).
 *   spins_out host N x 3 or NULL
 *   Sq        host L x L or NULL: S(q) = (1/N^2) |sum_i S_i e^{i q.r_i}|^2,
 *             q = 2 pi (qx, qy)/L stored at [qy*L + qx]
 *   m         host 3 doubles or NULL: mean spin */
int tca_observables(tca_ctx* c, double* spins_out, double* Sq, double* m);

/* Replace the state (checkpoint resume): spins host N x 3 (unit norm within
 * 1e-12) and the Philox sweep counter of the next sweep. */
int tca_set_state(tca_ctx* c, const double* spins_xyz, uint64_t sweep_counter);

/* Philox sweep counter of the next sweep (host out). */
int tca_get_sweep_counter(tca_ctx* c, uint64_t* sweep_counter);

/* Eigenvalues of `batch` dense complex Hermitian n x n matrices with the
 * production reduction + eigenvalue kernels.
 *   A  host, batch * n * n complex numbers as interleaved (re, im) doubles,
 *      row-major; only the lower triangle (i >= j) is read
 *   w  host, batch * n doubles, ascending per matrix
 *   precision TCA_FP64 or TCA_MIXED;  2 <= n <= 200.
 * If F is not NULL it receives batch free energies at (T, mu). */
int tca_heevals_batched(const double* A, int32_t n, int32_t batch, int32_t precision,
                        double T, double mu, double* w, double* F);

/* Same as tca_heevals_batched with device pointers (A: batch*n*n*2 doubles,
 * w: batch*n doubles or NULL, F: batch doubles or NULL), issued on
 * hip_stream without synchronization; used for timing. */
int tca_heevals_batched_dev(const double* A, int32_t n, int32_t batch, int32_t precision,
                            double T, double mu, double* w, double* F, void* hip_stream);

/* ------------------------------------------------------------------------
 * Learned first stage of delayed-acceptance Metropolis.
 *
 * The paper has no learned component: this is the delayed-acceptance scheme
 * of Christen & Fox (2005) put in front of the exact cluster energy of
 * Sec. II(c) (Fig. 2 steps (b)-(e)), which stays the second stage, so the
 * chain keeps the stationary law of the plain TCA sweep for any surrogate.
 * The surrogate is an MLP n_in -> H -> H -> 1 with SiLU after the first two
 * layers, n_in = 3 Lc^2 + 4: the cluster spins in cluster order (x, y, z),
 * the proposed spin, and T/0.1; it predicts F_new - F_old of the cluster.
 * Weights are FP32 (trained by the library's own FP32 kernels: forward,
 * backward of the mean squared error, Adam with beta1 0.9, beta2 0.999,
 * eps 1e-8); inference inside a sweep runs in BF16 on the matrix cores
 * (inputs, W1, W2 and the two hidden activations rounded to bfloat16, FP32
 * accumulation).
 * Flat parameter layout (FP32): W1 [H][n_in] row-major, b1 [H], W2 [H][H],
 * b2 [H], W3 [H], b3 [1].
 * A surrogate's device memory belongs to the library until
 * tca_surrogate_destroy(); all work is issued on its stream and finished
 * before a call returns.  Errors as for the lattice entry points.
 * ---------------------------------------------------------------------- */

/* New surrogate for clusters of linear size Lc (2..10) and hidden width
 * `hidden` (16..1024, multiple of 16); weights uniform in +-sqrt(6/(fan_in +
 * fan_out)) from Philox(seed), biases 0; dataset capacity `capacity` rows
 * (>= 0) in device memory. */
int tca_surrogate_create(int32_t Lc, int32_t hidden, uint64_t seed, int64_t capacity,
                         void* hip_stream, tca_surrogate** out);

/* Release the surrogate (NULL accepted).  Detach it from every context that
 * uses it first. */
int tca_surrogate_destroy(tca_surrogate* s);

/* Host out: number of parameters, input width, rows held in the dataset. */
int tca_surrogate_info(tca_surrogate* s, int64_t* nparams, int32_t* n_in, int64_t* rows);

/* Copy the FP32 parameters out to / in from host memory (nparams floats). */
int tca_surrogate_save(tca_surrogate* s, float* params);
int tca_surrogate_load(tca_surrogate* s, const float* params);

/* Training data from the exact method: run nsweeps plain sweeps of context c
 * (Sec. II(c) semantics, as tca_sweep without a surrogate) and append one row
 * per update -- features of the proposed move in the block-start state and
 * the exact F_new - F_old -- to the dataset.  c must use a fixed cluster size
 * equal to the surrogate's Lc, and nsweeps * L*L rows must fit the remaining
 * capacity (else TCA_E_INVAL).  T as for tca_sweep; st NULL or filled. */
int tca_surrogate_collect(tca_surrogate* s, tca_ctx* c, const double* T, int32_t nsweeps,
                          tca_sweep_stats* st);

/* Copy dataset rows [r0, r0 + rows) out to host memory (X: rows x n_in,
 * y: rows); TCA_E_INVAL if the range is not inside the dataset. */
int tca_surrogate_get_rows(tca_surrogate* s, int64_t r0, int64_t rows, float* X, float* y);

/* Append host rows (rows x n_in features, rows targets) to the dataset. */
int tca_surrogate_add_rows(tca_surrogate* s, const float* X, const float* y, int64_t rows);

/* `steps` Adam steps on minibatches of `batch` rows drawn (Philox, with
 * replacement) from the first rows - n_hold rows of the dataset, where
 * n_hold = floor(holdout * rows) rows at the end are held out (0 <= holdout
 * < 1).  Host out (each may be NULL): mean training loss of the last
 * min(steps, 50) steps, RMSE of the FP32 and of the BF16 network on the
 * held-out rows (0 if none). */
int tca_surrogate_train(tca_surrogate* s, int32_t steps, int32_t batch, float lr, double holdout,
                        double* train_mse, double* holdout_rmse_fp32,
                        double* holdout_rmse_bf16);

/* Loss mean((f(X) - y)^2) and its gradient (nparams floats, parameter
 * layout) for host rows; the weights are not changed. */
int tca_surrogate_grad(tca_surrogate* s, const float* X, const float* y, int32_t rows,
                       float* grad, double* loss);

/* One Adam step with a host gradient (nparams floats). */
int tca_surrogate_adam_step(tca_surrogate* s, const float* grad, float lr);

/* Predictions for host rows (rows x n_in): bf16 = 0 the FP32 network,
 * bf16 = 1 the BF16 inference path used inside sweeps. */
int tca_surrogate_eval(tca_surrogate* s, const float* X, int32_t rows, int32_t bf16, float* out);

/* Make s the first stage of delayed acceptance in every later tca_sweep on c
 * (NULL: plain Metropolis again).  Needs a fixed cluster size equal to the
 * surrogate's Lc (TCA_E_UNSUPPORTED with size classes).  Per update: stage 1
 * passes iff u1 == 0 or ln u1 < min(0, -dS_f/T); only survivors are solved
 * exactly, and a survivor is accepted iff u == 0 or
 * ln u < -dE/T + min(0, -dS_r/T) - min(0, -dS_f/T), where dS_f and dS_r are
 * the surrogate on the move and on its reverse (corner spin = proposal,
 * proposing the old spin), u and u1 words 0 and 1 of the update's Metropolis
 * Philox block.  The context keeps a pointer: the surrogate must outlive the
 * attachment. */
int tca_attach_surrogate(tca_ctx* c, tca_surrogate* s);

/* Reducer variants for matrices of dimension n (2..200) at a precision:
 * host out count (>= 1) and, if name is not NULL, a static name of `variant`
 * (NULL if out of range). */
int tca_reducer_variants(int32_t n, int32_t precision, int32_t variant, int32_t* count,
                         const char** name);

/* Use `variant` for every later reduction of dimension class n at this
 * precision in the process (overrides and disables the autotuner for that
 * class; meant for tests and tuning studies). */
int tca_select_reducer_variant(int32_t n, int32_t precision, int32_t variant);

/* Text of the autotuner's timings and choices for this context's cluster
 * sizes (host buf of len bytes, NUL-terminated, truncated if needed). */
int tca_tuning_report(tca_ctx* c, char* buf, int32_t len);

/* Release the context and its device memory (NULL is accepted). */
int tca_destroy(tca_ctx* c);

/* Sizes of the ABI structs as compiled into the library (host out, 3 values:
 * sizeof(tca_params), sizeof(tca_update_record), sizeof(tca_sweep_stats));
 * needs no GPU, lets bindings check their struct layouts. */
int tca_abi_sizes(int32_t* out3);

/* Static text for a status code. */
const char* tca_strerror(int status);

/* Thread-local description of the last failure on this thread ("" if none). */
const char* tca_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* TCA_H */
