/*
 * rsl.h -- resultants of bivariate integer polynomials on MI355X (gfx950).
 *
 * Computes R^(y) = res(f, g, y) in Z[x] and R^(x) = res(f, g, x) in Z[y] for
 * f, g in Z[x, y] by the modular route of the paper's Sec. 4.1 (Collins'
 * divide-conquer-combine scheme): reduce the coefficients modulo many 31-bit
 * primes, evaluate at many integer points, take univariate resultants over
 * Z_p, interpolate in x, and lift the coefficients to Z by Chinese
 * remaindering.  Every stage after the host-side plan runs in HIP kernels on
 * the device.  The resultant itself is the determinant of the Sylvester matrix
 * S^(y)(f, g) of Sec. 3.1 (f rows first, highest power of y first, actual
 * y-degrees m_y, n_y); the result is exact, bit for bit.
 *
 * Conventions where the paper is silent:
 *   - either input is the zero polynomial          -> R = 0  (deg = -1)
 *   - m_y = n_y = 0 (both constant in y)           -> R = 1
 *   - a common factor                              -> R = 0  (not an error;
 *     the paper assumes none, Sec. 2)
 *   - zero rows/columns of the input arrays are trimmed: degrees are actual.
 *
 * Error convention: every call returns an int; RSL_OK (0) on success, a
 * negative RSL_E* code otherwise.  rsl_strerror() maps codes to text and
 * rsl_last_error() returns the context's last detailed message.
 *
 * Threading: one rsl_ctx per host thread and stream.  Server calls are
 * thread-safe.  Inputs and outputs are host memory owned by the caller.
 */
#ifndef RSL_H
#define RSL_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ----------------------------------------------------------------- codes */
#define RSL_OK 0
#define RSL_EINVAL (-1)   /* null pointer, negative dims, limbs < 1, bad var/mode;
                             a problem beyond the supported sizes: more than 4096
                             primes, more than 3800 points, degree in the
                             eliminated variable above 255, or more than 256
                             primes in the persistent schedule             */
#define RSL_ERANGE (-2)   /* output buffer too small: nothing written              */
#define RSL_ENOMEM (-3)   /* workspace or budget smaller than the footprint        */
#define RSL_EPRIMES (-4)  /* prime table exhausted (too many bad primes)           */
#define RSL_EDEVICE (-5)  /* HIP error: the context is poisoned, destroy it        */
#define RSL_EAGAIN (-6)   /* server queue full, try again later                    */
#define RSL_ETIMEDOUT (-7)/* rsl_server_wait timed out, request still in flight    */

/* which variable is eliminated */
#define RSL_Y 0 /* res(f, g, y) in Z[x] */
#define RSL_X 1 /* res(f, g, x) in Z[y] */

/* execution modes of rsl_batch / rsl_job_run */
#define RSL_PLAIN 0   /* one pipeline (reduce, eval+ures, interp, crt) per problem          */
#define RSL_BATCHED 1 /* all problems in one persistent launch (device task queue); a wave
                         waits at most RSL_QUEUE_WAIT_MS (environment, read by
                         rsl_ctx_create; default 10000) for its next task, after which
                         the launch ends and the run returns RSL_EDEVICE             */
#define RSL_STAGED 2  /* one launch per stage, each over the work items of all problems     */
#define RSL_AUTO 3    /* the schedule the autotuner chose for this shape (RSL_STAGED if none) */

/* Environment read by rsl_ctx_create (test hooks): RSL_CRT_GARNER=1 makes the
 * CRT stage use Garner's mixed-radix digits for every coefficient instead of
 * the direct form (whose quotient estimate falls back to Garner only when it
 * cannot be decided); RSL_WIDE_VALU=1 runs the wide CRT's contraction on the
 * vector ALUs instead of the int8 matrix cores; RSL_EVAL_HORNER=1 keeps the
 * register-form evaluation on Horner's rule (vector ALUs) instead of the
 * int8 matrix-core sums.  In every case the results are identical. */

/* rsl_job_run only: OR into the mode to replay the run (status reset and every
 * launch of the schedule) as a HIP graph captured on the context stream on first
 * use and re-captured when the context's constant tables move.  Runs with
 * profiling enabled are not captured. */
#define RSL_GRAPH 0x100

/* point policy (rsl_opts.points) */
#define RSL_POINTS_REPLACE 0 /* bad points skipped: first D+1 good points of 0..D+s */
#define RSL_POINTS_FORMAL 1  /* all points 0..D used (formal-degree values)          */

/*
 * A dense bivariate polynomial f = sum_{i<=dx, j<=dy} c_ij x^i y^j.
 * coeff holds (dy+1)*(dx+1) coefficients, row-major by the power of y:
 * coefficient c_ij starts at coeff[(j*(dx+1) + i) * limbs] and is stored as
 * `limbs` little-endian 32-bit words in two's complement.  Zero padding
 * (rows/columns) is allowed and trimmed.  Paper Sec. 2, Eq. (2.1).
 */
typedef struct {
  int32_t dx;
  int32_t dy;
  int32_t limbs;
  const uint32_t *coeff;
} rsl_poly;

/*
 * Output: coefficient k of R (k = 0..deg) is written to
 * coeff[k*limbs .. k*limbs+limbs-1], two's complement little-endian words.
 * cap_deg is the highest degree the buffer holds (coeff has
 * (cap_deg+1)*limbs words).  deg is set to the actual degree (-1 for R = 0).
 * If R does not fit (deg > cap_deg or a coefficient needs more limbs) the
 * call returns RSL_ERANGE, sets deg and needed_limbs, and writes no
 * coefficient.
 */
typedef struct {
  int32_t cap_deg;
  int32_t limbs;
  uint32_t *coeff;
  int32_t deg;          /* out */
  int32_t needed_limbs; /* out: limbs of the widest coefficient (signed) */
} rsl_result;

/* Sizing of one problem, computed on the host without device work. */
typedef struct {
  int32_t D;            /* degree bound used for interpolation (paper Sec. 3.1: deg R <= m n) */
  int32_t bound_bits;   /* bits of the Hadamard bound B with |coeff of R| <= B */
  int32_t n_primes;     /* number of primes (2^30 < p < 2^32/3), prod p > 2B */
  int32_t n_points;     /* evaluation points per prime: D + 1 + s */
  int32_t out_limbs;    /* limbs that always suffice for every coefficient */
  int32_t my, ny;       /* actual degrees in the eliminated variable */
  int32_t bad_primes;   /* primes skipped because they divide a leading coefficient */
  size_t footprint_bytes; /* device workspace one rsl_res call needs */
  size_t table_bytes;     /* bytes of the context's constant tables that cover this problem
                             (primes, factorials, checkpoint rows of the Stirling triangle,
                             CRT constants), rounded up as the context grows them */
  int32_t origin;         /* first evaluation point (default options: see point_origin) */
} rsl_info;

/* Per-call options (zero-initialise for the defaults). */
typedef struct {
  int32_t points;      /* RSL_POINTS_REPLACE (default) or RSL_POINTS_FORMAL */
  int32_t prime_start; /* skip this many primes of the table (self-consistency tests) */
  int32_t extra_primes;/* use this many primes beyond the bound (self-consistency tests) */
  int32_t point_origin;/* > 0: evaluate at origin, origin+1, ... instead of 0, 1, ...;
                          0 (default): 0, unless a leading coefficient in the eliminated
                          variable vanishes at 0 over Z (point 0 bad for every prime) --
                          then the first origin in 1..16 where neither vanishes, so that
                          the primes keep the consecutive-point interpolation (followed by
                          a Taylor shift back to x); -1: 0 regardless (the gapped path) */
  int32_t extra_points;/* evaluate at this many points beyond D + s */
  int32_t prime_limit; /* test hook: treat the prime table as having only this many entries */
  int32_t eval_lanes;  /* lanes per (prime, point) pair in evaluation: 1, 2 or 4 (an upper
                          bound: problems of low degree use fewer); 0 = chosen from the job
                          size or by the autotuner */
  int32_t eval_regs;   /* 0: keep both polynomials of a pair in registers when the shape
                          allows (degrees <= 32 differing by at most one); -1: never */
  int32_t eval_schur;  /* 1: univariate resultants by the generalised Schur algorithm on
                          the displacement generators of the Sylvester matrix (paper
                          Sec. 4.1), one wave per (prime, point), for problems with
                          m_y, n_y >= 1 and m_y + n_y <= 64 (others keep the remainder
                          sequence); staged and plain schedules only; 0 = remainder
                          sequence unless the autotuner chose Schur */
  int32_t interp_mm;   /* 1: interpolation on the matrix cores -- the columns of all problems
                          sharing a prime as two matrix products with the Vandermonde
                          system's triangular factors (forward differences, Stirling
                          basis change); staged schedule (plain runs take the vector
                          path on the same layout); 0 = vector path unless the
                          autotuner chose the matrix cores */
  int32_t interp_newton;/* 1: every prime interpolates by the Vandermonde solve of the gapped
                          path -- divided differences, then the Newton form expanded to
                          monomials (the triangular factors of the Vandermonde matrix,
                          paper Sec. 4.1), D + 1 parallel steps per prime -- instead of the
                          consecutive-point products; 0 = only primes with a bad point */
} rsl_opts;

/* Counters of the last call on a context (or of a server). */
typedef struct {
  int64_t problems;
  int64_t pairs;        /* (prime, point) univariate resultants computed */
  int64_t bad_pairs;    /* of which had a vanishing leading coefficient */
  int64_t bad_primes;
  int64_t slow_primes;  /* primes interpolated on a non-consecutive point set */
  double ms_device;     /* device time of the last call (HIP events) */
  double ms_total;      /* host wall time of the last call */
  double ms_build;      /* of ms_total: planning and job layout (host) */
  double ms_bind;       /* of ms_total: writing the upload image (host) */
  double ms_transfer;   /* of ms_total: copies and launch overhead outside the device time */
  double ms_decode;     /* of ms_total: results into the callers' buffers (host) */
} rsl_counters;

typedef struct rsl_ctx rsl_ctx;

/*
 * Create a context on HIP device `device`.  All device memory the library
 * uses is the caller's (e.g. torch uint8 tensors); it must stay alive until
 * rsl_ctx_destroy.
 *   d_workspace / ws_bytes: per-call scratch (the job of rsl_res, rsl_batch,
 *     rsl_gcd ... and the server's arena).
 *   d_tables / table_bytes: the region of the context's constant tables
 *     (primes, Montgomery constants, factorials, every 32nd row of the
 *     Stirling triangle, CRT tables).  With d_tables = NULL the top
 *     table_bytes of the workspace are used instead (and the rest is scratch).
 *     rsl_query's table_bytes gives what a problem needs; a call whose
 *     problems need more gets RSL_ENOMEM.  The tables grow on demand inside
 *     the region (after waiting for this context's streams only).
 *   stream: the hipStream_t all work is ordered on (NULL = the null stream).
 * The library allocates no device memory of its own besides rsl_res_static's
 * fixed array; pinned host staging is allocated with hipHostMalloc.
 */
int rsl_ctx_create(int device, void *d_workspace, size_t ws_bytes, void *d_tables, size_t table_bytes,
                   void *stream, rsl_ctx **out);
int rsl_ctx_destroy(rsl_ctx *ctx);

/* Sizing only; no device work, no context needed.  var = RSL_Y or RSL_X. */
int rsl_query(const rsl_poly *f, const rsl_poly *g, int var, rsl_info *info);

/*
 * res(f, g, var): synchronous with respect to the context stream (the result
 * is in `out` when the call returns).  opts may be NULL.
 */
int rsl_res(rsl_ctx *ctx, const rsl_poly *f, const rsl_poly *g, int var, const rsl_opts *opts,
            rsl_result *out);

/*
 * rsl_res_static: the same resultant as rsl_res, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  It calls no hipMalloc, hipHostMalloc,
 * hipFree or other allocating device routine: the job is laid out in a fixed
 * device array of this library (64 MiB, held on every device the library runs
 * on until the process ends; the context's workspace is not used), and the
 * inputs and outputs travel through ordinary host memory.  Limits: a problem
 * whose footprint (rsl_query's footprint_bytes) exceeds 64 MiB gives
 * RSL_ENOMEM, and so does one that the context's constant tables do not cover
 * yet (an earlier rsl_res or rsl_batch on the context of a problem with at
 * least as many primes and points grows them).  Every call on a device shares
 * that device's array: calls that overlap on one GPU (from any context or
 * thread) race and must be serialised by the caller.  Arguments, results and
 * the other errors are those of rsl_res.
 */
int rsl_res_static(rsl_ctx *ctx, const rsl_poly *f, const rsl_poly *g, int var, const rsl_opts *opts,
                   rsl_result *out);
int rsl_res_y(rsl_ctx *ctx, const rsl_poly *f, const rsl_poly *g, rsl_result *out);
int rsl_res_x(rsl_ctx *ctx, const rsl_poly *f, const rsl_poly *g, rsl_result *out);

/*
 * Both projections of one system, R^(y) = res(f, g, y) into out_y and
 * R^(x) = res(f, g, x) into out_x (the solver needs both, paper Sec. 3), as
 * one job whose stage launches carry both problems (and share the
 * basis-change table reads where the two use the same primes).  Synchronous
 * like rsl_res; opts (may be NULL) applies to both; returns the first nonzero
 * status of the two.
 */
int rsl_res_xy(rsl_ctx *ctx, const rsl_poly *f, const rsl_poly *g, const rsl_opts *opts, rsl_result *out_y,
               rsl_result *out_x);
/* The x problem of such a pair also takes its residues of the common primes
 * from the y problem's reduction (the tiles are each other's transposes). */

/* ------------------------------------------- gcd and square-free part in Z[x]
 * The step after the resultant: the solver's Project step (paper Sec. 3.2)
 * takes a square-free factorisation of R by Yun's algorithm, i.e. gcds of R
 * and its derivatives, and the paper's outlook (Sec. 6) proposes the modular
 * route for it.
 *
 * A univariate input: deg + 1 coefficients, lowest power first, each `limbs`
 * little-endian 32-bit limbs in two's complement (deg -1 or all-zero: the zero
 * polynomial; leading zero coefficients are trimmed).  Host memory, caller
 * owned, read during the call only.
 */
typedef struct {
  int32_t deg;
  int32_t limbs;
  const uint32_t *coeff;
} rsl_upoly;

/*
 * G = gcd(pp(u), pp(v)) in Z[x] (primitive, positive leading coefficient; the
 * zero polynomial when u = v = 0) and the exact cofactors u / G and v / G, by
 * the modular route: per prime (not dividing a leading coefficient) Euclid's
 * algorithm over Z_p on the device, the gcd made monic and scaled by
 * gcd(lc u, lc v); the primes of least gcd degree kept; Chinese remaindering,
 * the content of the scaled gcd removed modulo each prime, the cofactors by
 * exact long division modulo each prime.  The kept primes' product exceeds
 * twice (deg u + deg v + 2) times Mignotte's bounds on G and on the cofactors,
 * and every reconstructed coefficient is checked against its bound, so the
 * identities G (u/G) = u and G (v/G) = v hold over Z (the result is certified,
 * not probabilistic).  Synchronous; uses the context workspace (RSL_ENOMEM
 * when it is too small).  Any of g, ug, vg may be NULL.  Output buffers as in
 * rsl_res (RSL_ERANGE with deg and needed_limbs set when too small).
 */
int rsl_gcd(rsl_ctx *ctx, const rsl_upoly *u, const rsl_upoly *v, rsl_result *g, rsl_result *ug,
            rsl_result *vg);

/*
 * Square-free part: g = gcd(pp(r), pp(r)') and q = r / g (the content and sign
 * of r stay in q; pp(q) is the square-free part of r).  Computed as
 * rsl_gcd(r, r').  Either output may be NULL.
 */
int rsl_sqfree_part(rsl_ctx *ctx, const rsl_upoly *r, rsl_result *q, rsl_result *g);

/*
 * Square-free factorisation pp(r) = prod_{i>=1} r_i^i (Yun's algorithm, the
 * one the paper's Project step names): r_i primitive, positive leading
 * coefficient, square-free and pairwise coprime; each gcd with its cofactors
 * by rsl_gcd's certified modular route on the device, the differences
 * c - b' on the host.  factors[i] receives r_{i+1} for i < *nfactors
 * (trailing factors equal to 1 are dropped; zero or constant r gives none).
 * RSL_ERANGE when *nfactors > max_factors (nothing written) or a buffer is too
 * small.
 */
int rsl_sqfree_factor(rsl_ctx *ctx, const rsl_upoly *r, int max_factors, rsl_result *factors, int *nfactors);

/*
 * A batch of n independent problems (f[k], g[k], var[k]) -> out[k].
 * mode RSL_PLAIN runs one pipeline per problem on the context stream;
 * RSL_BATCHED plans all problems together and runs them in one persistent
 * launch; RSL_STAGED runs one launch per stage over all problems.  All modes
 * give bit-identical results.  Per-problem status codes go to
 * status[k] (may be NULL); the call returns the first nonzero one.
 */
int rsl_batch(rsl_ctx *ctx, int n, const rsl_poly *f, const rsl_poly *g, const int *var,
              rsl_result *out, int *status, int mode);

/* Counters of the last rsl_res / rsl_batch on this context. */
int rsl_last_counters(rsl_ctx *ctx, rsl_counters *c);

/* ---------------------------------------------------------- resident jobs */
/*
 * A job is a planned batch whose inputs stay resident in device memory, so
 * that the device pipeline can be run repeatedly without host work (used for
 * throughput measurement and by the autotuner).  rsl_job_create plans and lays
 * the job out on the host only; rsl_job_bind then points it at device memory
 * owned by the caller (at least rsl_job_info.device_bytes, alive until
 * rsl_job_destroy or the next bind) and uploads the inputs.  A job must be used
 * with the context it was created on.
 */
typedef struct rsl_job rsl_job;

typedef struct {
  int32_t n_problems;     /* problems submitted */
  int32_t n_live;         /* problems with device work (non-zero inputs) */
  int64_t pairs;          /* (prime, point) univariate resultants per run */
  int64_t mulmods;        /* algorithmic multiply-adds of evaluation + remainder sequences per run */
  size_t device_bytes;    /* device memory the job's current layout needs */
  size_t upload_bytes;    /* host -> device bytes at creation */
  size_t download_bytes;  /* device -> host bytes per rsl_job_results */
  int32_t layout_mode;    /* schedule the layout was tuned for (RSL_STAGED or RSL_BATCHED) */
  int32_t chunk_target;   /* interpolation chunking of the layout */
  int32_t grid_mult;      /* persistent grid multiplier */
  int32_t eval_lanes;     /* most lanes per (prime, point) pair used by any problem */
  int32_t eval_mfma;      /* problems whose evaluation sums run on the matrix cores (register form,
                             one lane or a lane pair per pair, x-degrees up to 32: x-powers
                             0..31 on the matrix cores, x-power 32 on the vector ALUs) */
  int64_t mulmods_sums_mfma;  /* of mulmods: evaluation sums taken on the matrix cores */
  int64_t mulmods_valu;       /* of mulmods: the rest (remainder sequences, Horner sums) on the vector ALUs */
  int64_t mfma_int8_macs;     /* int8 multiply-adds the matrix cores issue per run for those sums
                                 (padded tiles, 25 digit products per residue product) */
  int64_t interp_mulmods;     /* interpolation products per run: N_p (D+1)(D+2) over problems */
} rsl_job_info;

/* Plan and lay out n problems (status per problem in `status`, may be NULL); host work only.
 * The context's constant tables are grown to cover the job. */
int rsl_job_create(rsl_ctx *ctx, int n, const rsl_poly *f, const rsl_poly *g, const int *var,
                   const rsl_opts *opts, int *status, rsl_job **out);
/* Bind `bytes` of caller-owned device memory at d_mem (256-byte aligned) and upload the inputs
 * (synchronous).  RSL_ENOMEM when the layout needs more; rsl_job_run, rsl_job_results and
 * rsl_job_tune return RSL_EINVAL until a bind succeeds. */
int rsl_job_bind(rsl_ctx *ctx, rsl_job *job, void *d_mem, size_t bytes);
/* Run the device pipeline on the resident inputs; asynchronous on the context stream. */
int rsl_job_run(rsl_ctx *ctx, rsl_job *job, int mode);
/* Wait for the last run, copy the results back and decode them. */
int rsl_job_results(rsl_ctx *ctx, rsl_job *job, rsl_result *out, int *status);
int rsl_job_info_get(const rsl_job *job, rsl_job_info *info);
int rsl_job_destroy(rsl_job *job);

/* --------------------------------------------------------------- autotuner */
/*
 * The autotuner times candidate schedules of a job -- staged or persistent
 * launch, interpolation chunking (blocks kept in flight), persistent grid size
 * -- on the job itself, checks that every candidate produces the same output
 * bytes as the first (a candidate that differs is an error, RSL_EDEVICE), keeps
 * the fastest, re-lays the job out with it (candidates whose layout needs more
 * than the bound memory are skipped), and records it in the context's
 * cache under the job's shape bucket (problems, max degree bound, max primes,
 * max degree, all rounded to powers of two).  Jobs created later with the
 * same bucket are laid out with the cached choice; RSL_AUTO runs it.
 */
typedef struct {
  int32_t mode;          /* RSL_STAGED or RSL_BATCHED */
  int32_t chunk_target;  /* interpolation blocks kept in flight */
  int32_t grid_mult;     /* persistent workgroups per resident slot */
  int32_t evk;           /* lanes per (prime, point) pair in evaluation: 1, 2 or 4 */
  int32_t conv_whole;    /* 1: convolution sums taken whole, 0: split like the basis change */
  int32_t schur;         /* 1: evaluation by the Schur algorithm (see rsl_opts.eval_schur) */
  int32_t interp_mm;     /* 1: interpolation on the matrix cores (see rsl_opts.interp_mm) */
  int32_t candidates;    /* candidates timed */
  double ms;             /* device time of one run of the chosen schedule */
  double ms_worst;       /* device time of the slowest candidate */
} rsl_tune_result;

int rsl_job_tune(rsl_ctx *ctx, rsl_job *job, int reps, rsl_tune_result *best);
/* Save / load the tuning cache as text lines
 * "key mode chunk_target grid_mult evk conv_whole schur interp_mm ms" (lines without
 * interp_mm are read as 0). */
int rsl_tune_save(rsl_ctx *ctx, const char *path);
int rsl_tune_load(rsl_ctx *ctx, const char *path);

/* --------------------------------------------------------------- profiling */
/* Stages: 0 reduce, 1 eval+ures, 2 interp (convolution), 3 interp (basis
 * change), 4 interp (gapped points, shifted origin), 5 CRT. */
#define RSL_NUM_STAGES 6
/* While enabled, every batched launch records HIP events on the context
 * stream at each stage boundary. */
int rsl_profile_enable(rsl_ctx *ctx, int on);
/* Synchronise, add up the stage durations of all launches recorded since the
 * last call into stage_ms[RSL_NUM_STAGES], and reset.  A stage that launched
 * no kernel for a job reads 0; the time of its boundary markers is counted in
 * the stage before it.  A persistent launch is reported as stage 0. */
int rsl_profile_take(rsl_ctx *ctx, double *stage_ms, int *runs);

/* ---------------------------------------------------------------- serving */
typedef struct rsl_server rsl_server;

typedef struct {
  int64_t submitted, completed, rejected, in_flight;
  double p50_ms, p99_ms, mean_ms; /* submit -> completion latency of completed requests */
  double throughput;              /* completed requests per second since creation */
  int64_t admitted_bytes_peak;    /* peak sum of footprints admitted at once */
  int64_t launches;               /* device iterations run by the scheduler */
  int64_t max_batch;              /* most requests that shared one device iteration */
} rsl_stats;

/*
 * Start a server on a context (the server owns the context's workspace until
 * rsl_server_destroy: meanwhile rsl_res, rsl_res_xy, rsl_batch and the gcd
 * calls on that context return RSL_EINVAL, and a second server is refused).
 * Requests are admitted in FIFO order while slots are free and the sum of
 * their device footprints stays within budget_bytes (<= workspace size);
 * admitted requests run together in one batched device iteration, and
 * requests arriving while an iteration runs join the next one (continuous
 * batching).  max_queue bounds the host queue (RSL_EAGAIN beyond it).  A
 * request whose constant tables would not fit the context's table region is
 * refused at submit with RSL_ENOMEM.
 */
int rsl_server_create(rsl_ctx *ctx, size_t budget_bytes, int max_slots, int max_queue,
                      rsl_server **out);
/* Copy the inputs, plan and enqueue; `out` must stay valid until completion. */
int rsl_server_submit(rsl_server *s, const rsl_poly *f, const rsl_poly *g, int var,
                      rsl_result *out, uint64_t *ticket);
/* The same in two steps, for a caller that sizes `out` from the plan: copy the
 * inputs and plan the request (info as rsl_query's; RSL_ENOMEM when its tables
 * would not fit the context's table region), then queue it under `handle`
 * with its result buffer.  The request is planned once; the scheduler lays
 * out its batches from those plans.  A handle is used by one successful
 * enqueue; after RSL_EAGAIN (queue full) it stays valid for a later one, after
 * any other error it is spent.  Handles never enqueued are freed with the server. */
int rsl_server_plan(rsl_server *s, const rsl_poly *f, const rsl_poly *g, int var, rsl_info *info,
                    uint64_t *handle);
int rsl_server_enqueue(rsl_server *s, uint64_t handle, rsl_result *out, uint64_t *ticket);
/* 1 if done (status in *status), 0 if still in flight. */
int rsl_server_poll(rsl_server *s, uint64_t ticket, int *status);
/* Wait up to timeout_ms (< 0: forever); returns the request status or RSL_ETIMEDOUT. */
int rsl_server_wait(rsl_server *s, uint64_t ticket, int timeout_ms);
int rsl_server_stats(rsl_server *s, rsl_stats *st);
int rsl_server_destroy(rsl_server *s);

/* ---------------------------------------------------------------- errors */
const char *rsl_strerror(int code);
const char *rsl_last_error(rsl_ctx *ctx);
/* Library version string. */
const char *rsl_version(void);

#ifdef __cplusplus
}
#endif
#endif /* RSL_H */
