/*
 * Plain FP64 CPU oracle for the type 1, type 2 and type 3 NUFFT sums.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg load this code.  It shares nothing with the GPU
 * library: it evaluates the exponential sums by their definitions, term by term,
 * in double precision, with no kernel, grid, FFT or approximation of any kind.
 *
 * Definitions followed (Sec. 1, eqs. (1) and (2)):
 *   mode set per dimension  I_N = { -floor(N/2), ..., -floor(N/2)+N-1 }
 *     (N even: -N/2..N/2-1;  N odd: -(N-1)/2..(N-1)/2)
 *   type 1:  f_k = sum_{j=1..M} c_j exp(+/- i k.x_j),   k in I_{N1} x ... x I_{Nd}
 *   type 2:  c_j = sum_{k in I}  f_k exp(+/- i k.x_j),   j = 1..M
 *   type 3:  f_k = sum_{j=1..M} c_j exp(+/- i s_k.x_j),  k = 1..N  (eq. (3):
 *            arbitrary real source points x_j and target frequencies s_k)
 * The sign of i is the caller's isign (+1 or -1); the paper's defaults are +1
 * for type 1 and -1 for type 2.  No normalisation is applied.
 *
 * exp(i k.x) is formed as the product over dimensions of exp(i k_m x_m), an
 * exact identity, so that one sin/cos pair per (point, mode index, dimension)
 * suffices.  Complex numbers are interleaved (re, im) doubles.  Output arrays are
 * ordered with the first dimension's index fastest.
 *
 * Threads only split independent work: type 1 splits the points (each thread
 * sums its own points for every requested mode; partial sums are then added in
 * thread order, so results do not depend on scheduling); types 2 and 3 split
 * the outputs.  Every sum is accumulated in blocks of at most ORACLE_BLOCK
 * terms: a block's terms are summed on their own and the block sums added
 * to the running total, which keeps the rounding of long sums (up to 1e7
 * terms) near that of a 4096-term sum plus the number of blocks.  Type 3 forms each phase s_k.x_j in FP64 and takes its cosine
 * and sine directly (the targets are not a grid, so there is no product form).
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* Terms per block of every accumulation. */
#define ORACLE_BLOCK 4096

typedef struct {
  int dim;
  int64_t j0, j1;                 /* point range [j0, j1) */
  const double *x[3];
  const double *c;                /* type 1: strengths (2*M) */
  const double *f;                /* type 2: coefficients (2*N) */
  int isign;
  int64_t nk[3];                  /* number of mode indices per dim */
  const int64_t *k[3];            /* mode index values per dim */
  double *out;                    /* type 1: private partial sums; type 2: c */
} job_t;

/* e[a] = exp(i*isign*k[a]*x) for a = 0..n-1 (interleaved re, im). */
static void phases(double x, int isign, int64_t n, const int64_t *k, double *e) {
  for (int64_t a = 0; a < n; a++) {
    double th = (double)isign * (double)k[a] * x;
    e[2 * a] = cos(th);
    e[2 * a + 1] = sin(th);
  }
}

static void *type1_worker(void *arg) {
  job_t *jb = (job_t *)arg;
  int64_t n1 = jb->nk[0], n2 = jb->nk[1], n3 = jb->nk[2];
  int64_t K = n1 * n2 * n3;
  double *e1 = malloc(sizeof(double) * 2 * n1);
  double *e2 = malloc(sizeof(double) * 2 * n2);
  double *e3 = malloc(sizeof(double) * 2 * n3);
  double *blk = calloc(2 * K, sizeof(double));   /* sum over the current block of points */
  double *acc = jb->out;                          /* sum of the finished blocks */
  for (int64_t b0 = jb->j0; b0 < jb->j1; b0 += ORACLE_BLOCK) {
    int64_t b1 = b0 + ORACLE_BLOCK < jb->j1 ? b0 + ORACLE_BLOCK : jb->j1;
    memset(blk, 0, sizeof(double) * 2 * K);
    for (int64_t j = b0; j < b1; j++) {
      phases(jb->x[0][j], jb->isign, n1, jb->k[0], e1);
      if (jb->dim >= 2) phases(jb->x[1][j], jb->isign, n2, jb->k[1], e2);
      else { e2[0] = 1.0; e2[1] = 0.0; }
      if (jb->dim >= 3) phases(jb->x[2][j], jb->isign, n3, jb->k[2], e3);
      else { e3[0] = 1.0; e3[1] = 0.0; }
      double cr = jb->c[2 * j], ci = jb->c[2 * j + 1];
      for (int64_t a3 = 0; a3 < n3; a3++) {
        /* c_j * exp(i k3 z_j) */
        double u3r = cr * e3[2 * a3] - ci * e3[2 * a3 + 1];
        double u3i = cr * e3[2 * a3 + 1] + ci * e3[2 * a3];
        for (int64_t a2 = 0; a2 < n2; a2++) {
          /* ... * exp(i k2 y_j) */
          double u2r = u3r * e2[2 * a2] - u3i * e2[2 * a2 + 1];
          double u2i = u3r * e2[2 * a2 + 1] + u3i * e2[2 * a2];
          double *row = blk + 2 * n1 * (a2 + n2 * a3);
          for (int64_t a1 = 0; a1 < n1; a1++) {
            /* ... * exp(i k1 x_j), accumulated into f_k */
            row[2 * a1] += u2r * e1[2 * a1] - u2i * e1[2 * a1 + 1];
            row[2 * a1 + 1] += u2r * e1[2 * a1 + 1] + u2i * e1[2 * a1];
          }
        }
      }
    }
    for (int64_t q = 0; q < 2 * K; q++) acc[q] += blk[q];
  }
  free(e1); free(e2); free(e3); free(blk);
  return NULL;
}

static void *type2_worker(void *arg) {
  job_t *jb = (job_t *)arg;
  int64_t n1 = jb->nk[0], n2 = jb->nk[1], n3 = jb->nk[2];
  double *e1 = malloc(sizeof(double) * 2 * n1);
  double *e2 = malloc(sizeof(double) * 2 * n2);
  double *e3 = malloc(sizeof(double) * 2 * n3);
  for (int64_t j = jb->j0; j < jb->j1; j++) {
    phases(jb->x[0][j], jb->isign, n1, jb->k[0], e1);
    if (jb->dim >= 2) phases(jb->x[1][j], jb->isign, n2, jb->k[1], e2);
    else { e2[0] = 1.0; e2[1] = 0.0; }
    if (jb->dim >= 3) phases(jb->x[2][j], jb->isign, n3, jb->k[2], e3);
    else { e3[0] = 1.0; e3[1] = 0.0; }
    double sr = 0.0, si = 0.0;     /* sum of the finished blocks of modes */
    double br = 0.0, bi = 0.0;     /* sum over the current block */
    int64_t nb = 0;                /* terms in the current block */
    for (int64_t a3 = 0; a3 < n3; a3++) {
      for (int64_t a2 = 0; a2 < n2; a2++) {
        /* exp(i (k2 y + k3 z)) */
        double p23r = e3[2 * a3] * e2[2 * a2] - e3[2 * a3 + 1] * e2[2 * a2 + 1];
        double p23i = e3[2 * a3] * e2[2 * a2 + 1] + e3[2 * a3 + 1] * e2[2 * a2];
        const double *frow = jb->f + 2 * n1 * (a2 + n2 * a3);
        for (int64_t a1 = 0; a1 < n1; a1++) {
          double pr = p23r * e1[2 * a1] - p23i * e1[2 * a1 + 1];
          double pi = p23r * e1[2 * a1 + 1] + p23i * e1[2 * a1];
          double fr = frow[2 * a1], fi = frow[2 * a1 + 1];
          br += fr * pr - fi * pi;
          bi += fr * pi + fi * pr;
          if (++nb == ORACLE_BLOCK) {
            sr += br; si += bi;
            br = bi = 0.0;
            nb = 0;
          }
        }
      }
    }
    jb->out[2 * j] = sr + br;
    jb->out[2 * j + 1] = si + bi;
  }
  free(e1); free(e2); free(e3);
  return NULL;
}

static int clamp_threads(int nthreads, int64_t work) {
  if (nthreads < 1) nthreads = 1;
  if (nthreads > 256) nthreads = 256;
  if ((int64_t)nthreads > work) nthreads = work > 0 ? (int)work : 1;
  return nthreads;
}

/*
 * Type 1 at the product set of the given mode indices.
 *   dim 1..3; M points with coordinates x[0..dim-1][M]; c: 2*M doubles.
 *   nk[m], k[m]: number and values of the requested mode indices of dimension m
 *   (for dim < 3 the unused dimensions must have nk = 1, k = {0}).
 *   f: 2*nk[0]*nk[1]*nk[2] doubles, overwritten; k[0] index fastest.
 * Returns 0, or -1 on bad arguments / allocation failure.
 */
int oracle_type1(int dim, int64_t M, const double *x, const double *y,
                 const double *z, const double *c, int isign, int64_t nk1,
                 const int64_t *k1, int64_t nk2, const int64_t *k2, int64_t nk3,
                 const int64_t *k3, double *f, int nthreads) {
  if (dim < 1 || dim > 3 || M < 0 || nk1 < 1 || nk2 < 1 || nk3 < 1) return -1;
  if ((dim < 2 && nk2 != 1) || (dim < 3 && nk3 != 1)) return -1;
  int64_t K = nk1 * nk2 * nk3;
  memset(f, 0, sizeof(double) * 2 * K);
  if (M == 0) return 0;
  int T = clamp_threads(nthreads, M);
  job_t *jobs = calloc(T, sizeof(job_t));
  pthread_t *th = calloc(T, sizeof(pthread_t));
  if (!jobs || !th) return -1;
  for (int t = 0; t < T; t++) {
    job_t *jb = &jobs[t];
    jb->dim = dim;
    jb->j0 = M * t / T;
    jb->j1 = M * (t + 1) / T;
    jb->x[0] = x; jb->x[1] = y; jb->x[2] = z;
    jb->c = c;
    jb->isign = isign;
    jb->nk[0] = nk1; jb->nk[1] = nk2; jb->nk[2] = nk3;
    jb->k[0] = k1; jb->k[1] = k2; jb->k[2] = k3;
    jb->out = calloc(2 * K, sizeof(double));
    if (!jb->out) return -1;
    pthread_create(&th[t], NULL, type1_worker, jb);
  }
  for (int t = 0; t < T; t++) pthread_join(th[t], NULL);
  for (int t = 0; t < T; t++) {
    for (int64_t q = 0; q < 2 * K; q++) f[q] += jobs[t].out[q];
    free(jobs[t].out);
  }
  free(jobs); free(th);
  return 0;
}

/*
 * Type 2 at M target points from the full coefficient array.
 *   f: 2*N1*N2*N3 doubles, k1 fastest, each dimension in increasing mode
 *   order starting at -floor(N_m/2).  c: 2*M doubles, overwritten.
 * Returns 0, or -1 on bad arguments / allocation failure.
 */
int oracle_type2(int dim, int64_t M, const double *x, const double *y,
                 const double *z, const double *f, int64_t N1, int64_t N2,
                 int64_t N3, int isign, double *c, int nthreads) {
  if (dim < 1 || dim > 3 || M < 0 || N1 < 1 || N2 < 1 || N3 < 1) return -1;
  if ((dim < 2 && N2 != 1) || (dim < 3 && N3 != 1)) return -1;
  if (M == 0) return 0;
  int64_t Ns[3] = {N1, N2, N3};
  int64_t *ks[3];
  for (int m = 0; m < 3; m++) {
    ks[m] = malloc(sizeof(int64_t) * Ns[m]);
    if (!ks[m]) return -1;
    for (int64_t a = 0; a < Ns[m]; a++) ks[m][a] = a - Ns[m] / 2;
  }
  int T = clamp_threads(nthreads, M);
  job_t *jobs = calloc(T, sizeof(job_t));
  pthread_t *th = calloc(T, sizeof(pthread_t));
  if (!jobs || !th) return -1;
  for (int t = 0; t < T; t++) {
    job_t *jb = &jobs[t];
    jb->dim = dim;
    jb->j0 = M * t / T;
    jb->j1 = M * (t + 1) / T;
    jb->x[0] = x; jb->x[1] = y; jb->x[2] = z;
    jb->f = f;
    jb->isign = isign;
    for (int m = 0; m < 3; m++) { jb->nk[m] = Ns[m]; jb->k[m] = ks[m]; }
    jb->out = c;
    pthread_create(&th[t], NULL, type2_worker, jb);
  }
  for (int t = 0; t < T; t++) pthread_join(th[t], NULL);
  for (int m = 0; m < 3; m++) free(ks[m]);
  free(jobs); free(th);
  return 0;
}

typedef struct {
  int dim;
  int64_t k0, k1;                 /* target range [k0, k1) */
  int64_t M;
  const double *x[3], *s[3];
  const double *c;
  int isign;
  double *f;
} job3_t;

static void *type3_worker(void *arg) {
  job3_t *jb = (job3_t *)arg;
  for (int64_t k = jb->k0; k < jb->k1; k++) {
    double fr = 0.0, fi = 0.0;     /* sum of the finished blocks of sources */
    double br = 0.0, bi = 0.0;     /* sum over the current block */
    for (int64_t j = 0; j < jb->M; j++) {
      double ph = 0.0;
      for (int m = 0; m < jb->dim; m++) ph += jb->s[m][k] * jb->x[m][j];
      ph *= (double)jb->isign;
      double cr = jb->c[2 * j], ci = jb->c[2 * j + 1];
      double er = cos(ph), ei = sin(ph);
      br += cr * er - ci * ei;
      bi += cr * ei + ci * er;
      if ((j + 1) % ORACLE_BLOCK == 0) {
        fr += br; fi += bi;
        br = bi = 0.0;
      }
    }
    jb->f[2 * k] = fr + br;
    jb->f[2 * k + 1] = fi + bi;
  }
  return NULL;
}

/*
 * Type 3 (eq. (3)): f_k = sum_j c_j exp(isign i s_k.x_j), k = 0..N-1.
 *   sources x[0..dim-1][M], strengths c: 2*M doubles; targets s[0..dim-1][N];
 *   f: 2*N doubles, overwritten.
 * Returns 0, or -1 on bad arguments / allocation failure.
 */
int oracle_type3(int dim, int64_t M, const double *x, const double *y, const double *z,
                 const double *c, int64_t N, const double *s, const double *t,
                 const double *u, int isign, double *f, int nthreads) {
  if (dim < 1 || dim > 3 || M < 0 || N < 0) return -1;
  if (N == 0) return 0;
  int T = clamp_threads(nthreads, N);
  job3_t *jobs = calloc(T, sizeof(job3_t));
  pthread_t *th = calloc(T, sizeof(pthread_t));
  if (!jobs || !th) return -1;
  for (int q = 0; q < T; q++) {
    job3_t *jb = &jobs[q];
    jb->dim = dim;
    jb->k0 = N * q / T;
    jb->k1 = N * (q + 1) / T;
    jb->M = M;
    jb->x[0] = x; jb->x[1] = y; jb->x[2] = z;
    jb->s[0] = s; jb->s[1] = t; jb->s[2] = u;
    jb->c = c;
    jb->isign = isign;
    jb->f = f;
    pthread_create(&th[q], NULL, type3_worker, jb);
  }
  for (int q = 0; q < T; q++) pthread_join(th[q], NULL);
  free(jobs); free(th);
  return 0;
}
