/*
 * esnufft — type 1, 2 and 3 nonuniform FFTs on one AMD MI355X (gfx950) GPU
 * with the "exponential of semicircle" (ES) spreading kernel.
 *
 * The transforms approximate, to a requested relative tolerance eps, the
 * exponential sums of Sec. 1 of Barnett, Magland & af Klinteberg,
 * "A parallel non-uniform fast Fourier transform library based on an
 * 'exponential of semicircle' kernel" (arXiv:1808.06736):
 *
 *   type 1 (eq. (1)):  f_k = sum_{j=1..M} c_j exp(isign * i k.x_j),  k in I
 *   type 2 (eq. (2)):  c_j = sum_{k in I} f_k exp(isign * i k.x_j),  j = 1..M
 *   type 3 (eq. (3)):  f_k = sum_{j=1..M} c_j exp(isign * i s_k.x_j), k = 1..N
 *                      (any real sources x_j and target frequencies s_k; see
 *                      esn_setpts3)
 *
 * with d = 1, 2 or 3, mode set I = I_{N1} x ... x I_{Nd},
 * I_N = {-floor(N/2), ..., -floor(N/2) + N - 1}, points x_j anywhere in
 * [-3pi, 3pi]^d (the sums are 2pi-periodic in each coordinate), complex c_j, f_k.
 * No normalisation.  The method (Sec. 3): spread onto an upsampled fine grid
 * with the ES kernel phi(z) = exp(beta(sqrt(1 - z^2) - 1)) (eq. (ES)), FFT, and
 * divide by the kernel's Fourier transform (eqs. (pb1), (pk)); type 2 runs the
 * steps in reverse (Sec. 3.2).
 *
 * Memory: every data pointer below is a DEVICE pointer (hipMalloc'd or a
 * torch CUDA tensor's data_ptr) unless the argument says "host".  The caller
 * owns x, y, z, c and f; the library reads/writes them only during the call
 * that receives them.  esn_setpts copies the points, bin-sorted and rescaled,
 * into plan-owned device memory, so the caller may free or overwrite the
 * coordinate arrays once it returns.  The plan owns its fine grid, correction
 * factors, sort arrays, rocFFT plan and work buffer until esn_destroy.
 *
 * Layouts: complex data are interleaved (re, im) pairs of float (ESN_SINGLE)
 * or double (ESN_DOUBLE).  Strengths c are [ntransf][M].  Mode arrays f are
 * [ntransf][N3][N2][N1] (N1 fastest); within a dimension the modes run in
 * increasing k from -floor(N/2) (modeord 0) or in FFT order 0,1,..,-1
 * (modeord 1).  Outputs are overwritten, never accumulated.
 *
 * Streams: all work of a plan is enqueued on the hipStream_t given to
 * esn_makeplan (NULL = the null stream).  Calls return once the work is
 * enqueued, except where stated; errors found on the host are returned
 * before anything is enqueued.  One plan must not be used from two host
 * threads at once.  A plan's device memory comes from the stream-ordered
 * allocator on that stream (allocation and freeing do not wait for the
 * rest of the device; freed memory stays in the device's default pool up to
 * 16 GiB), so the stream must stay valid until esn_destroy.
 *
 * Status codes: 0 = success, 1 = warning (computed, but eps is beyond what
 * the precision supports), >= 2 = error (nothing was computed).
 */
#ifndef ESNUFFT_H
#define ESNUFFT_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- precision codes ---------------------------------------------------- */
#define ESN_SINGLE 1 /* complex64 data, FP32 spread/interp/FFT */
#define ESN_DOUBLE 2 /* complex128 data, FP64 everywhere */

/* ---- status codes -------------------------------------------------------- */
#define ESN_OK 0
#define ESN_WARN_EPS_TOO_SMALL 1   /* eps < 1e-6 in single or < 1e-15; w clamped */
#define ESN_ERR_BAD_ARG 2          /* invalid type, dim, sizes, sign, pointer */
#define ESN_ERR_PTS_OUT_OF_RANGE 3 /* chkbnds: a coordinate outside [-3pi, 3pi] */
#define ESN_ERR_NAN_PTS 4          /* a coordinate is NaN or infinite */
#define ESN_ERR_BUDGET 5           /* request exceeds the HBM budget */
#define ESN_ERR_ALLOC 6            /* device allocation failed */
#define ESN_ERR_FFT_PLAN 7         /* rocFFT refused the plan */
#define ESN_ERR_HIP 8              /* a HIP runtime call failed */
#define ESN_ERR_UNSUPPORTED 9      /* a valid request this build does not do */
#define ESN_ERR_NO_POINTS 10       /* execute before setpts */
#define ESN_ERR_QUEUE 11           /* server: unknown ticket or server stopped */

/* ---- options (paper Sec. 2: an opts struct with defaults) ----------------- */
typedef struct esn_opts {
  int debug;          /* 1: time each stage with HIP events (esn_get_stats) */
  int chkbnds;        /* 1: setpts rejects coordinates outside [-3pi, 3pi] */
  int modeord;        /* 0: increasing k from -floor(N/2); 1: FFT order */
  double upsampfac;   /* fine grid / modes ratio sigma: 2.0 (eq. (params)) or
                         1.25 (low upsampling: w = ceil(1.7136 log10(1/eps)
                         + 0.6), beta = 1.8397 w; types 1 and 2 only) */
  int sort;           /* bin-sort the points (Sec. 5.1): 1 (default) choose by
                         size; 2 stable radix sort of the point records by cell;
                         3 counting sort by cell (atomic per point, no order
                         inside a cell); 0: keep the caller's order */
  int spread_method;  /* 0 auto; 1 LDS tile per subproblem; 2 global atomics;
                         3 matrix cores (3D, single precision, w <= 7) */
  int interp_method;  /* 0 auto; 1 LDS tile per subproblem; 2 direct gather;
                         3 matrix cores (3D, single precision, w <= 7) */
  int bin[3];         /* bin size in fine-grid cells per dim; 0 = default */
  int maxsubprob;     /* max points per subproblem (Sec. 5.2); 0 = default
                         (on the matrix cores 1024 for type 1 and 512 for
                         type 2, 1024 otherwise) */
  int ntransf_chunk;  /* transforms per fused launch; 0 = as many as fit */
  int block;          /* threads per workgroup for spread/interp; 0 = 256 */
  int kerevalmeth;    /* kernel evaluation: 0 auto (the table in double
                         precision, exp and sqrt in single); 1 exp and sqrt
                         at every weight (eq. (ES)); 2 piecewise polynomial
                         table (Sec. 5.3, esn_kernel_poly) */
} esn_opts;

/* Fill *o with the defaults (debug 0, chkbnds 1, modeord 0, upsampfac 2.0,
 * sort 1, everything else 0 = automatic). */
void esn_default_opts(esn_opts* o);

/* ---- parameter choice (host only, no GPU needed) --------------------------- */
typedef struct esn_params {
  int w;             /* kernel width in fine-grid cells, eq. (params) */
  double beta;       /* ES shape parameter 2.30 w, eq. (params) */
  int nquad;         /* positive Gauss-Legendre nodes p >= 1.5 w + 2 (Sec. 3.1) */
  int64_t nf[3];     /* fine grid per dim: smallest 2^a 3^b 5^c >= max(sigma N, 2w) */
} esn_params;

/* Kernel and grid parameters for tolerance eps (Sec. 3, eq. (params) and
 * Sec. 3.1): sigma = upsampfac = 2: w = ceil(log10(1/eps)) + 1, beta = 2.30 w;
 * sigma = 1.25: w = ceil(1.7136 log10(1/eps) + 0.6), beta = 1.8397 w (eqs.
 * (gam) and (ESerr) with the safety factor 0.976 of the sigma = 2 rule); w
 * clamped to [2, 16]; n_i = smallest 2^a 3^b 5^c >= max(sigma N_i, 2w)
 * (unused dims: 1).  nmodes: host array of 3 (entries beyond dim ignored).
 * Returns ESN_OK, ESN_WARN_EPS_TOO_SMALL (w clamped, eps < 1e-15, or eps <
 * 1e-6 in single precision) or ESN_ERR_BAD_ARG (other sigma too). */
int esn_choose_params(double eps, int prec, int dim, const int64_t* nmodes,
                      double upsampfac, esn_params* out);

/* The p positive nodes (decreasing) and their weights of the 2p-node
 * Gauss-Legendre rule on [-1, 1], FP64 Newton iteration on P_2p (the rule of
 * eq. (quad)).  nodes, weights: host arrays of p >= 1.  Host only. */
int esn_gauss_legendre(int p, double* nodes, double* weights);

/* Host FP64 twin of the GPU correction factors of one dimension:
 * out[k] = 1 / (w sum_{j<=p} w_j phi(q_j) cos(alpha k q_j)), k = 0..floor(N/2),
 * alpha = pi w / nf, p = nquad (eqs. (pk1), (quad)).  out: host array of
 * floor(N/2) + 1 doubles.  Host only; used to check the GPU values. */
int esn_correction_factors(int w, double beta, int nquad, int64_t nf, int64_t N, double* out);

/* Piecewise polynomial form of the kernel phi(z) = exp(beta (sqrt(1 - z^2) - 1))
 * (Sec. 5.3): w equal intervals of [-1, 1], one per window cell, each a
 * polynomial of degree w + 3 in a local t in [-1, 1], with
 * z = (k + (t + 1) / 2 - w / 2) (2 / w) on interval k.  coeffs: host array of
 * w (w + 4) doubles, coefficient of t^j on interval k at coeffs[k (w + 4) + j]
 * (Chebyshev interpolation converted to monomials).  w in 2..16, beta > 0;
 * ESN_ERR_BAD_ARG otherwise.  Host only. */
int esn_kernel_poly(int w, double beta, double* coeffs);

/* ---- plan interface -------------------------------------------------------- */
typedef struct esn_plan_s* esn_plan;

/* Make a plan for ntransf transforms of one type that share one point set
 * (Sec. 2, remark on repeated small problems: a plan stage and multiple
 * inputs).  type 1, 2 or 3; dim 1..3; nmodes host[3] (N_i >= 1; not read
 * for type 3); isign +1/-1; ntransf >= 1; prec ESN_SINGLE/ESN_DOUBLE; opts
 * may be NULL (defaults); stream is a hipStream_t or NULL.  Types 1 and 2:
 * computes the correction factors p_k (eqs. (pk1), (quad), (pk)) on the GPU
 * in FP64 and builds the rocFFT plan; type 3 sizes its grids in esn_setpts3.
 * Synchronises the stream before returning.  *out is NULL on error. */
int esn_makeplan(int type, int dim, const int64_t* nmodes, int isign, int ntransf,
                 double eps, int prec, esn_plan* out, const esn_opts* opts,
                 void* stream);

/* Give the plan M points, 0 <= M <= 2^31 - 2^16 (ESN_ERR_BAD_ARG above; the
 * same limit holds for the sources and targets of esn_setpts3): coordinate
 * arrays x[, y[, z]] of M values, float if coord_prec == ESN_SINGLE else
 * double; unused dims may be NULL.
 * Folds each coordinate into [0, 2pi) and rescales it to fine-grid units in
 * FP64, bin-sorts the points (Sec. 5.1) and builds the subproblem list
 * (Sec. 5.2).  Synchronises the stream (it reads back the subproblem count
 * and the bounds/NaN flags).  On ESN_ERR_NAN_PTS or (with chkbnds)
 * ESN_ERR_PTS_OUT_OF_RANGE the plan is left without points, so a following
 * esn_execute returns ESN_ERR_NO_POINTS until a successful esn_setpts. */
int esn_setpts(esn_plan p, int64_t M, int coord_prec, const void* x, const void* y,
               const void* z);

/* Type 3 plans (esn_makeplan with type 3; nmodes is not read and may be NULL):
 * give the M source points x[, y[, z]] and the N target frequencies s[, t[, u]]
 * of eq. (3), f_k = sum_j c_j exp(isign i s_k.x_j), any finite real values
 * (float if coord_prec == ESN_SINGLE else double; unused dims may be NULL).
 * Centres both sets (eq. (trans)), sizes the fine grid and the dilation from
 * their half-widths (eq. (ng) of Sec. 3.3, step 0), bin-sorts the rescaled
 * sources for spreading and the rescaled targets for the inner type 2 NUFFT,
 * and evaluates the per-target correction (d p FP64 cosines) and phases.
 * Synchronises the stream.  Errors: ESN_ERR_BAD_ARG, ESN_ERR_NAN_PTS (a NaN or
 * infinite coordinate), ESN_ERR_BUDGET (a fine grid of more than 2^31 cells),
 * ESN_ERR_ALLOC; on error the plan has no points.  esn_execute then reads c
 * [ntransf][M] and writes f [ntransf][N]; esn_execute_adjoint returns
 * ESN_ERR_UNSUPPORTED for type 3. */
int esn_setpts3(esn_plan p, int64_t M, int coord_prec, const void* x, const void* y,
                const void* z, int64_t N, const void* s, const void* t, const void* u);

/* Run the transforms.  type 1: reads c [ntransf][M], writes f
 * [ntransf][N3][N2][N1] (steps of Sec. 3.1: spread eq. (bl), FFT eq. (dft1),
 * truncate and correct eq. (pb1)); type 2: reads f, writes c (Sec. 3.2:
 * amplify and zero-pad, FFT eq. (dft), interpolate eq. (interp)).
 * Asynchronous on the plan's stream. */
int esn_execute(esn_plan p, void* c, void* f);

/* The adjoint of the plan's transform on the same sorted points (Sec. 1: the
 * type 2 sum with sign -isign is the adjoint of the type 1 sum with sign
 * isign, and the type 2 algorithm of Sec. 3.2 is the exact adjoint of the
 * type 1 algorithm of Sec. 3.1).  A type 1 plan reads f [ntransf][N3][N2][N1]
 * and writes c [ntransf][M] (c_j = sum_k f_k e^{-isign i k.x_j}); a type 2
 * plan reads c and writes f (f_k = sum_j c_j e^{-isign i k.x_j}).  Same
 * tolerance, bins and subproblems as the plan's own transform, so one
 * esn_setpts serves both directions.  The first call makes the rocFFT plans
 * of the opposite sign (device allocation); later calls allocate nothing.
 * Asynchronous on the plan's stream; errors as esn_execute. */
int esn_execute_adjoint(esn_plan p, void* c, void* f);

/* The spreading step alone, eq. (bl): grid[t] = sum_j c[t][j] psi~(l h - x_j)
 * for the plan's points, into a caller buffer of ntransf * n1*n2*n3 complex
 * values (n1 fastest, fine-grid cell l at l*h).  Type 1 plans only. */
int esn_spread(esn_plan p, const void* c, void* grid);

/* The interpolation step alone, eq. (interp): c[t][j] = sum_l grid[t][l]
 * psi~(l h - x_j).  Type 2 plans only. */
int esn_interp(esn_plan p, const void* grid, void* c);

typedef struct esn_info {
  int type, dim, isign, ntransf, prec, w, nquad, modeord;
  double beta, eps;
  int64_t nmodes[3], nf[3], M;
  int bin[3], maxsubprob, nsubprob, nbins_nonempty, ntransf_chunk;
  int spread_method, interp_method, point_code; /* point_code 1: fixed point u32, 2: f64 */
  int64_t device_bytes;  /* device memory the plan holds */
  int ndense_units;      /* subproblems run on the matrix cores (method 3) */
  int kerevalmeth;       /* 1 exp and sqrt, 2 piecewise polynomial table */
} esn_info;

/* Describe a plan (host struct filled). */
int esn_get_info(esn_plan p, esn_info* out);

typedef struct esn_stats {
  /* milliseconds of the last setpts / execute, by stage (debug = 1 only).
   * Types 1 and 2 record HIP events around the stages and read them only
   * here, so timing adds no host synchronisation to the calls; reading waits
   * for the calls timed.
   * 3D single-precision plans whose FFT runs as column FFTs carry the
   * correction (deconvolution / amplification) inside the FFT: t_fft then
   * includes it and t_deconv_or_amplify is only the gap between the stages.
   * Type 3 plans: t_spread_or_interp = spreading (step 1), t_fft = the inner
   * type 2 transform (step 2), t_deconv_or_amplify = that transform's
   * interpolation alone. */
  double t_setpts, t_spread_or_interp, t_fft, t_deconv_or_amplify, t_execute;
} esn_stats;

/* Stage times of the plan's most recent setpts and execute calls (types 1
 * and 2, debug = 1), oldest first: up to max entries (at most 256 are kept)
 * into out, their number into *count.  A setpts entry has t_setpts only, an
 * execute entry the other fields.  Waits for the calls timed.  Lets a caller
 * time a loop of calls without a synchronisation in it. */
int esn_get_stats_history(esn_plan p, esn_stats* out, int max, int* count);

/* esn_setpts for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc).
 * Same arguments and result as esn_setpts, with the radix bin sort always
 * (esn_opts.sort 0 keeps the caller's order as usual).  Allocates nothing:
 *   - the sort's scratch is one static device array of 128 MiB per GPU, shared
 *     by every call on that GPU; the call clears what must start at zero, and
 *     calls that overlap on one GPU (other threads, other streams) race on it;
 *   - the plan must already hold room for M points: an earlier esn_setpts of
 *     at least M points on this plan (whose device memory the plan keeps).
 * Returns ESN_ERR_BAD_ARG when M exceeds that room or the sort's scratch for
 * M points exceeds the static array (about 5.5e6 points in single precision,
 * 3.3e6 in double precision), ESN_ERR_HIP if the array's address cannot be
 * found; otherwise as esn_setpts. */
int esn_setpts_noalloc(esn_plan p, int64_t M, int coord_prec, const void* x, const void* y,
                       const void* z);

/* Debug view of the bin sort (Sec. 5.1) and the subproblems (Sec. 5.2) of
 * the plan's current points (types 1 and 2), for tests of the sort's
 * invariants.  geom (host, 5 values) gets {M, number of bins, cells per bin,
 * number of subproblems, sort method (0 none, 2 radix, 3 counting)}; with
 * every array NULL only geom is filled.  Otherwise each non-NULL host array
 * is filled:
 *   perm[M]           original index of the i-th sorted point;
 *   key[M]            its cell key, bin * cells_per_bin + index of the cell in
 *                     the bin (window cells, see esn_setpts);
 *   bin_start[nbins+1] first sorted position of every bin, bin_start[nbins] = M;
 *   sub[3 * nsub]     subproblems {bin, first sorted position, length}.
 * bin_start and sub need a sorted plan (BAD_ARG otherwise).  Allocates
 * temporary device memory and synchronises the plan's stream. */
int esn_debug_sort(esn_plan p, int64_t* geom, int32_t* perm, uint32_t* key, int32_t* bin_start,
                   int32_t* sub);

/* Copy the plan's GPU-computed correction factors of dimension m (0-based,
 * floor(N_m/2) + 1 doubles) into the host array out of length len.
 * Synchronises the plan's stream. */
int esn_plan_correction(esn_plan p, int m, double* out, int64_t len);

/* Per-stage times of the last calls; requires opts.debug = 1.  Synchronises. */
int esn_get_stats(esn_plan p, esn_stats* out);

/* Free everything the plan owns (waits for its stream first).  NULL is ok. */
int esn_destroy(esn_plan p);

/* ---- one-shot calls in the paper's style (Sec. 2: status = finufft1d1(...)) */
/* Coordinates are device doubles; c and f device complex of precision prec;
 * opts may be NULL; stream as above.  Each call plans, sets points, executes
 * and destroys; it returns after the result is complete. */
int esn_1d1(int64_t M, const double* x, const void* c, int isign, double eps,
            int64_t N1, void* f, int prec, const esn_opts* opts, void* stream);
int esn_1d2(int64_t M, const double* x, void* c, int isign, double eps, int64_t N1,
            const void* f, int prec, const esn_opts* opts, void* stream);
int esn_2d1(int64_t M, const double* x, const double* y, const void* c, int isign,
            double eps, int64_t N1, int64_t N2, void* f, int prec,
            const esn_opts* opts, void* stream);
int esn_2d2(int64_t M, const double* x, const double* y, void* c, int isign,
            double eps, int64_t N1, int64_t N2, const void* f, int prec,
            const esn_opts* opts, void* stream);
int esn_3d1(int64_t M, const double* x, const double* y, const double* z,
            const void* c, int isign, double eps, int64_t N1, int64_t N2,
            int64_t N3, void* f, int prec, const esn_opts* opts, void* stream);
int esn_3d2(int64_t M, const double* x, const double* y, const double* z, void* c,
            int isign, double eps, int64_t N1, int64_t N2, int64_t N3,
            const void* f, int prec, const esn_opts* opts, void* stream);

/* ---- normal operator in Toeplitz form (inverse NUFFT by conjugate gradients
 * on the normal equations, Sec. 1 remark on the inverse NUFFT) -------------- */
typedef struct esn_toeplitz_s* esn_toeplitz;

/* T = A^H W A for A the type 2 transform of sign isign with N modes on the M
 * points x, y, z (eq. (2)), W = diag(weights): (T f)_k = sum_k' t_{k-k'} f_k',
 * t_m = sum_j w_j exp(-isign i m.x_j).  Set-up runs one type 1 transform of the
 * weights on 2 N_i modes per dimension (tolerance eps) and the FFT of the
 * result; esn_toeplitz_apply then costs two FFTs of prod(2 N_i) points.
 * dim 1..3; nmodes host[3]; prec ESN_SINGLE/ESN_DOUBLE; coordinates: device
 * arrays of M values in coord_prec (as esn_setpts); weights: device array of M
 * complex values in prec, or NULL for all ones; opts: modeord sets the order of
 * the mode arrays of esn_toeplitz_apply (other fields as for esn_makeplan);
 * stream: hipStream_t or NULL.  Synchronises the stream.  Returns ESN_OK or a
 * warning with *out set, else an error code with *out NULL. */
int esn_toeplitz_makeplan(int dim, const int64_t* nmodes, int isign, double eps, int prec,
                          int64_t M, int coord_prec, const void* x, const void* y, const void* z,
                          const void* weights, esn_toeplitz* out, const esn_opts* opts,
                          void* stream);
/* g = T f; f, g: device arrays of N1 N2 N3 complex values (may not alias).
 * Enqueued on the plan's stream; ESN_ERR_BAD_ARG on NULL pointers. */
int esn_toeplitz_apply(esn_toeplitz t, const void* f, void* g);
int esn_toeplitz_destroy(esn_toeplitz t);

/* ---- serving: a request loop for many independent transforms -------------
 * Not from the paper (its remark on repeated small problems, Sec. 2, is what
 * plan reuse answers); this is the library's own continuous-batching front
 * end.  Worker threads, each with its own HIP stream (default priority), take
 * requests from one FIFO queue; a request starts as soon as a worker is free
 * and its estimated device memory fits the budget, evicting idle cached plans
 * (least recently used first) when needed.  Requests that can never fit fail
 * with ESN_ERR_BUDGET.  Plans are cached by (type, dim, modes, isign, eps,
 * prec); a cached plan remembers the points_id it last sorted, and a request
 * naming the same nonzero points_id (the caller promises the same points)
 * skips setpts.  Data pointers are device pointers that must stay valid until
 * esn_server_wait returns for the ticket; once it has returned, the outputs
 * are complete on the device.  Kernels of concurrent requests
 * overlap on the device; results do not depend on what else is running. */
typedef struct esn_request {
  int type;                /* 1 or 2 */
  int dim;                 /* 1..3 */
  int64_t nmodes[3];       /* entries beyond dim ignored */
  int isign;               /* +1 / -1 */
  double eps;
  int prec;                /* ESN_SINGLE / ESN_DOUBLE: dtype of c and f */
  int64_t M;
  int coord_prec;          /* ESN_SINGLE / ESN_DOUBLE: dtype of x, y, z */
  const void* x;
  const void* y;
  const void* z;
  void* c;                 /* [M] strengths (type 1 input, type 2 output) */
  void* f;                 /* [N3][N2][N1] modes (type 1 output, type 2 input) */
  long long points_id;     /* 0, or an id shared by requests with identical points */
  void* stream;            /* hipStream_t that wrote the inputs (x, y, z, and c for
                              type 1 or f for type 2), or NULL for the null stream:
                              submit records an event on it and the request's work
                              waits for that event, so inputs still being written
                              by work queued there are complete before they are read */
} esn_request;

typedef struct esn_serve_stats {
  long long submitted, completed, failed, rejected, queued, running;
  long long plan_cache_hits, plan_cache_misses, point_cache_hits, cached_plans;
  long long hbm_in_use, hbm_peak;      /* bytes counted against the budget */
  double p50_ms, p99_ms, mean_ms, max_ms; /* submit-to-done latency of completed requests */
  double pts_per_s;                    /* completed NU points / (last done - first submit) */
} esn_serve_stats;

typedef struct esn_server_s* esn_server;

/* Start a server with nslots workers (1..64) and an HBM budget in bytes on
 * the current device.  opts (may be NULL) apply to every plan it makes. */
int esn_server_create(const esn_opts* opts, int nslots, long long hbm_budget_bytes,
                      esn_server* out);
/* Queue a request (host struct, copied); *ticket identifies it.  Returns
 * ESN_ERR_BAD_ARG for malformed requests, ESN_ERR_QUEUE after destroy began. */
int esn_server_submit(esn_server s, const esn_request* r, long long* ticket);
/* Block until the request is done; *status is its status, *latency_ms its
 * submit-to-done time (either may be NULL).  A ticket can be waited once. */
int esn_server_wait(esn_server s, long long ticket, int* status, double* latency_ms);
/* Counters and latency percentiles since creation or the last reset. */
int esn_server_stats(esn_server s, esn_serve_stats* out);
int esn_server_reset_stats(esn_server s);
/* Finish every queued request, then free all plans, streams and threads. */
int esn_server_destroy(esn_server s);

/* Text for a status code (static string). */
const char* esn_strerror(int status);

#ifdef __cplusplus
}
#endif
#endif /* ESNUFFT_H */
