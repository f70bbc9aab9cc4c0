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

#define TCA_ABI_VERSION 1

typedef enum {
  TCA_OK = 0,
  TCA_E_INVAL = -1,        /* invalid argument (sizes, NULL, non-unit spin, ...) */
  TCA_E_NOMEM = -2,        /* device or host allocation failed */
  TCA_E_DEVICE = -3,       /* a HIP runtime call or kernel launch failed */
  TCA_E_UNSUPPORTED = -4,  /* valid request this build does not implement */
} tca_status;

enum { TCA_FP64 = 0, TCA_MIXED = 1 };  /* precision of the tridiagonal reduction */
enum { TCA_INIT_RANDOM = 0, TCA_INIT_FERRO = 1, TCA_INIT_NEEL = 2, TCA_INIT_USER = 3 };
/* tca_params.flags bits */
enum { TCA_FLAG_PROFILE = 1 };  /* time every kernel launch of a sweep with HIP events */

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
  uint8_t flags;  /* bit 0: near-threshold (|dE + T ln u| <= 1e-9 max(|dE|,1e-3)) */
  double dF;      /* F_new - F_old of the cluster */
  double dE;      /* dF + classical change */
  double u;       /* the Metropolis uniform */
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
} tca_sweep_stats;

typedef struct tca_ctx tca_ctx;

/* Create a lattice context on the current HIP device.
 *   p          host; validated (TCA_E_INVAL on a bad size, precision or flag)
 *   spins_xyz  host N x 3 initial spins when p->init == TCA_INIT_USER (each
 *              |S| within 1e-12 of 1, else TCA_E_INVAL), otherwise ignored
 *   hip_stream hipStream_t to issue all work on, NULL = the null stream
 *   out        receives the context (NULL on failure)
 * Random initial spins are uniform on the sphere (Philox stream 3). */
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
