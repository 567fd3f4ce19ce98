/*
 * sigk_oracle.c -- plain, slow, CPU reference for the signature kernel.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the oracle that the GPU library is
 * checked against.  Only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark may load it; the product path never does.  It shares no
 * code, header, table or constant generator with the GPU library.
 *
 * What it computes (arXiv 2502.20392, Sec. 2):
 *   k(x, y) = K(1, 1), where K solves the Goursat problem of Definition 2.1
 *   (equivalently the Volterra equation of Sec. 2.1) with the tilewise constant
 *   coefficient rho = <x', y'> of the affine interpolants.
 *
 * How: tiles are swept cell by cell in raster order (row l outer, column k
 * inner).  On each cell the solution is the tile-centred power series of
 * Proposition 2.8, C = A o B o W, written in the monomial basis, with the
 * entries exactly as in the proof of Proposition 2.8:
 *     C[i][j] = c^min(i,j) * w_ij * (i >= j ? alpha[i-j] : beta[j-i]),
 *     w_ij    = (max(i,j) - min(i,j))! / (max(i,j)! * min(i,j)!),
 * alpha = bottom-edge series (a function of the x-direction coordinate) and
 * beta = left-edge series.  The next cell's boundary series are C evaluated on
 * the top and right edges (the alpha/beta recursion of Proposition 2.8).
 *
 * Readings of the paper taken here (each is listed in the design notes):
 *   - cell coefficient c = <dx_k, dy_l> with k indexing x-segments (columns)
 *     and l indexing y-segments (rows);
 *   - every cell is mapped to unit coordinates [0,1]^2, so the evaluation
 *     vector eta(.) of Proposition 2.8 is the all-ones vector and c is the raw
 *     increment inner product (reparametrisation invariance of K);
 *   - alpha sits on the entries with i >= j (the bottom edge), as in the proof
 *     of Proposition 2.8 (its statement has the two swapped);
 *   - the corner value is taken from alpha (C[0][0] = alpha[0]).
 *
 * Truncation: per cell, N = max(len alpha, len beta) + n_c coefficients are
 * kept, where n_c is the least n with |c|^n/(n!)^2 < 2^-64; afterwards
 * trailing coefficients below 2^-64 * max(1, max|coef|) are dropped.  If N
 * would exceed NCAP the call fails (never silently).
 *
 * The file is compiled twice: REAL = double (suffix _f64) and
 * REAL = long double (suffix _ld), the second bounding the first's rounding.
 * Build with -ffp-contract=off.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <unistd.h>

#ifndef REAL
#define REAL double
#endif
#ifndef SFX
#define SFX _f64
#endif
#define CAT_(a, b) a##b
#define CAT(a, b) CAT_(a, b)
#define FN(name) CAT(name, SFX)
#define ST(name) CAT(name, CAT(SFX, _s))

#define NCAP 160

enum {
    ORC_OK = 0,
    ORC_EINVAL = -1,
    ORC_ENOMEM = -2,
    ORC_ECAP = -5 /* more than NCAP coefficients would be needed */
};

static REAL ST(ifact)[2 * NCAP + 2];          /* 1/i!                 */
static REAL ST(qfm)[NCAP][NCAP];              /* q!/M!  for q <= M    */
static pthread_once_t ST(once) = PTHREAD_ONCE_INIT;

static void ST(init_tables)(void)
{
    ST(ifact)[0] = 1;
    for (int i = 1; i < 2 * NCAP + 2; ++i) ST(ifact)[i] = ST(ifact)[i - 1] / (REAL)i;
    for (int M = 0; M < NCAP; ++M) {
        ST(qfm)[M][M] = 1;
        for (int q = M - 1; q >= 0; --q) ST(qfm)[q][M] = ST(qfm)[q + 1][M] / (REAL)(q + 1);
    }
}

/* w_ij = (max-min)!/(max! min!)   (matrix W of Proposition 2.8) */
static REAL ST(w)(int i, int j)
{
    int mn = i < j ? i : j, mx = i < j ? j : i;
    return ST(qfm)[mx - mn][mx] * ST(ifact)[mn];
}

static REAL ST(absr)(REAL v) { return v < 0 ? -v : v; }

/* least n with |c|^n/(n!)^2 < 2^-64 */
static int ST(neumann_terms)(REAL c)
{
    REAL ac = ST(absr)(c), t = 1;
    const REAL thr = (REAL)5.421010862427522e-20; /* 2^-64 */
    int n = 0;
    while (t >= thr && n < 2 * NCAP) {
        ++n;
        t = t * ac / ((REAL)n * (REAL)n);
    }
    return n;
}

/* Coefficient matrix of one cell (Proposition 2.8), N x N, row-major. */
static void ST(cell_matrix)(const REAL* a, int la, const REAL* b, int lb, REAL c, int N,
                            REAL* C)
{
    REAL cp[NCAP];
    cp[0] = 1;
    for (int n = 1; n < N; ++n) cp[n] = cp[n - 1] * c;
    for (int i = 0; i < N; ++i)
        for (int j = 0; j < N; ++j) {
            int mn = i < j ? i : j, dd = i < j ? j - i : i - j;
            REAL coef;
            if (i >= j)
                coef = dd < la ? a[dd] : 0;
            else
                coef = dd < lb ? b[dd] : 0;
            C[(size_t)i * N + j] = cp[mn] * ST(w)(i, j) * coef;
        }
}

/* Trim trailing coefficients below 2^-64 * max(1, max|v|); returns new length. */
static int ST(trim)(const REAL* v, int len)
{
    REAL mx = 1;
    for (int i = 0; i < len; ++i)
        if (ST(absr)(v[i]) > mx) mx = ST(absr)(v[i]);
    const REAL thr = (REAL)5.421010862427522e-20 * mx;
    while (len > 1 && ST(absr)(v[len - 1]) <= thr) --len;
    return len;
}

/*
 * One cell: given bottom-edge series a (la coefficients) and left-edge series
 * b (lb coefficients) in the monomial basis of the unit cell, and the cell
 * coefficient c, write the top-edge series (a_out) and the right-edge series
 * (b_out), trimmed.  Work array C must hold NCAP*NCAP values.
 */
static int ST(cell)(const REAL* a, int la, const REAL* b, int lb, REAL c, REAL* a_out,
                    int* la_out, REAL* b_out, int* lb_out, REAL* C, int* n_used)
{
    int N = (la > lb ? la : lb) + ST(neumann_terms)(c);
    if (N > NCAP) return ORC_ECAP;
    ST(cell_matrix)(a, la, b, lb, c, N, C);
    for (int i = 0; i < N; ++i) {
        REAL s = 0;
        for (int j = 0; j < N; ++j) s += C[(size_t)i * N + j];
        a_out[i] = s; /* top edge: expansion evaluated at v = 1 */
    }
    for (int j = 0; j < N; ++j) {
        REAL s = 0;
        for (int i = 0; i < N; ++i) s += C[(size_t)i * N + j];
        b_out[j] = s; /* right edge: expansion evaluated at u = 1 */
    }
    *la_out = ST(trim)(a_out, N);
    *lb_out = ST(trim)(b_out, N);
    if (*la_out == N && N == NCAP) return ORC_ECAP;
    if (*lb_out == N && N == NCAP) return ORC_ECAP;
    if (n_used) *n_used = N;
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Raster sweep over one pair.                                              */

typedef struct {
    /* optional per-cell storage of the cell inputs, for the adjoint */
    REAL* pool;
    size_t pool_len, pool_cap;
    size_t* off;   /* [cells]  offset of (a, b) in pool */
    int* la;       /* [cells]  */
    int* lb;       /* [cells]  */
} ST(store);

static int ST(store_push)(ST(store) * s, size_t cell, const REAL* a, int la, const REAL* b,
                          int lb)
{
    size_t need = s->pool_len + (size_t)la + (size_t)lb;
    if (need > s->pool_cap) {
        size_t cap = s->pool_cap ? s->pool_cap : 1024;
        while (cap < need) cap *= 2;
        REAL* p = (REAL*)realloc(s->pool, cap * sizeof(REAL));
        if (!p) return ORC_ENOMEM;
        s->pool = p;
        s->pool_cap = cap;
    }
    s->off[cell] = s->pool_len;
    s->la[cell] = la;
    s->lb[cell] = lb;
    memcpy(s->pool + s->pool_len, a, (size_t)la * sizeof(REAL));
    memcpy(s->pool + s->pool_len + la, b, (size_t)lb * sizeof(REAL));
    s->pool_len = need;
    return ORC_OK;
}

/*
 * Sweep the (m x n) grid of cells with coefficients c(k, l) = <dx_k, dy_l>.
 * dx: [m][d], dy: [n][d] (increments).  Returns K(1,1) in *k_out.
 * diag (optional, 4 values): [0] max corner mismatch |alpha0-beta0|/max(1,|alpha0|),
 * [1] max N used, [2] |top-sum - right-sum|/max(1,|k|) at the last cell,
 * [3] max trimmed edge length.
 */
static int ST(sweep)(const REAL* dx, int64_t m, const REAL* dy, int64_t n, int64_t d,
                     REAL* k_out, double* diag, ST(store) * st)
{
    pthread_once(&ST(once), ST(init_tables));
    int rc = ORC_OK;
    REAL* bot = (REAL*)malloc((size_t)m * NCAP * sizeof(REAL));
    int* blen = (int*)malloc((size_t)m * sizeof(int));
    REAL* C = (REAL*)malloc((size_t)NCAP * NCAP * sizeof(REAL));
    REAL left[NCAP], aout[NCAP], bout[NCAP];
    if (!bot || !blen || !C) {
        rc = ORC_ENOMEM;
        goto done;
    }
    for (int64_t k = 0; k < m; ++k) {
        bot[(size_t)k * NCAP] = 1;
        blen[k] = 1;
    }
    double mism = 0, maxn = 0, maxlen = 0, lastdiff = 0;
    for (int64_t l = 0; l < n; ++l) {
        int llen = 1;
        left[0] = 1;
        for (int64_t k = 0; k < m; ++k) {
            REAL c = 0;
            for (int64_t ch = 0; ch < d; ++ch) c += dx[k * d + ch] * dy[l * d + ch];
            REAL* a = bot + (size_t)k * NCAP;
            REAL a0 = a[0], b0 = left[0];
            REAL den = ST(absr)(a0) > 1 ? ST(absr)(a0) : 1;
            double mm = (double)(ST(absr)(a0 - b0) / den);
            if (mm > mism) mism = mm;
            if (st) {
                rc = ST(store_push)(st, (size_t)l * m + k, a, blen[k], left, llen);
                if (rc) goto done;
            }
            int la2, lb2, nu;
            rc = ST(cell)(a, blen[k], left, llen, c, aout, &la2, bout, &lb2, C, &nu);
            if (rc) goto done;
            if (nu > maxn) maxn = nu;
            if (la2 > maxlen) maxlen = la2;
            if (lb2 > maxlen) maxlen = lb2;
            memcpy(a, aout, (size_t)la2 * sizeof(REAL));
            blen[k] = la2;
            memcpy(left, bout, (size_t)lb2 * sizeof(REAL));
            llen = lb2;
        }
        if (l == n - 1) {
            REAL kt = 0, kr = 0;
            const REAL* a = bot + (size_t)(m - 1) * NCAP;
            for (int i = 0; i < blen[m - 1]; ++i) kt += a[i];
            for (int j = 0; j < llen; ++j) kr += left[j];
            *k_out = kt; /* top edge of the last cell evaluated at u = 1 */
            REAL den = ST(absr)(kt) > 1 ? ST(absr)(kt) : 1;
            lastdiff = (double)(ST(absr)(kt - kr) / den);
        }
    }
    if (diag) {
        diag[0] = mism;
        diag[1] = maxn;
        diag[2] = lastdiff;
        diag[3] = maxlen;
    }
done:
    free(bot);
    free(blen);
    free(C);
    return rc;
}

static int ST(increments)(const double* z, int64_t len, int64_t d, REAL** out)
{
    int64_t m = len - 1;
    REAL* dz = (REAL*)malloc((size_t)(m > 0 ? m : 1) * (size_t)d * sizeof(REAL));
    if (!dz) return ORC_ENOMEM;
    for (int64_t k = 0; k < m; ++k)
        for (int64_t ch = 0; ch < d; ++ch)
            dz[k * d + ch] = (REAL)z[(k + 1) * d + ch] - (REAL)z[k * d + ch];
    *out = dz;
    return ORC_OK;
}

/*
 * k(x, y) for one pair.  x: [lx][d], y: [ly][d], row-major, double.
 * k_out: result rounded to double; k_ext (optional): result in REAL.
 * diag (optional): see sweep().
 */
int FN(sigk_oracle_pair)(const double* x, int64_t lx, const double* y, int64_t ly, int64_t d,
                         double* k_out, REAL* k_ext, double* diag)
{
    if (!x || !y || !k_out || d < 1 || lx < 0 || ly < 0) return ORC_EINVAL;
    if (diag) diag[0] = diag[1] = diag[2] = diag[3] = 0;
    if (lx < 2 || ly < 2) { /* no cells: K = 1 on the axes */
        *k_out = 1.0;
        if (k_ext) *k_ext = 1;
        return ORC_OK;
    }
    REAL *dx = NULL, *dy = NULL, k = 0;
    int rc = ST(increments)(x, lx, d, &dx);
    if (!rc) rc = ST(increments)(y, ly, d, &dy);
    if (!rc) rc = ST(sweep)(dx, lx - 1, dy, ly - 1, d, &k, diag, NULL);
    free(dx);
    free(dy);
    if (!rc) {
        *k_out = (double)k;
        if (k_ext) *k_ext = k;
    }
    return rc;
}

/*
 * The fixed-order kernel of the paper's error analysis (App. C, first display;
 * the same approximant as in Proposition A.3): every tile keeps the
 * (N+1) x (N+1) coefficient matrix C~ = A o B o W with 0 <= i, j <= N and the
 * entries of Proposition 2.8 (cell_matrix above); the next tiles' edge series
 * are its row and column sums, kept to N+1 coefficients, with no adaptive
 * order and no trimming.  Returns k^[N](x, y) in *k_out.
 */
int FN(sigk_oracle_pair_fixed)(const double* x, int64_t lx, const double* y, int64_t ly,
                               int64_t d, int N, double* k_out)
{
    if (!x || !y || !k_out || d < 1 || lx < 0 || ly < 0 || N < 0 || N + 1 > NCAP)
        return ORC_EINVAL;
    if (lx < 2 || ly < 2) {
        *k_out = 1.0;
        return ORC_OK;
    }
    pthread_once(&ST(once), ST(init_tables));
    const int n1 = N + 1;
    const int64_t m = lx - 1, n = ly - 1;
    REAL *dx = NULL, *dy = NULL;
    REAL* bot = (REAL*)malloc((size_t)m * n1 * sizeof(REAL));
    REAL* C = (REAL*)malloc((size_t)n1 * n1 * sizeof(REAL));
    REAL left[NCAP], right[NCAP];
    int rc = (bot && C) ? ORC_OK : ORC_ENOMEM;
    if (!rc) rc = ST(increments)(x, lx, d, &dx);
    if (!rc) rc = ST(increments)(y, ly, d, &dy);
    if (rc) goto done;
    for (int64_t k = 0; k < m; ++k)
        for (int i = 0; i < n1; ++i) bot[(size_t)k * n1 + i] = i == 0 ? 1 : 0;
    for (int64_t l = 0; l < n; ++l) {
        for (int j = 0; j < n1; ++j) left[j] = j == 0 ? 1 : 0;
        for (int64_t k = 0; k < m; ++k) {
            REAL rho = 0;
            for (int64_t ch = 0; ch < d; ++ch) rho += dx[k * d + ch] * dy[l * d + ch];
            REAL* col = bot + (size_t)k * n1; /* bottom edge in, top edge out */
            ST(cell_matrix)(col, n1, left, n1, rho, n1, C);
            for (int i = 0; i < n1; ++i) {
                REAL sum = 0;
                for (int j = 0; j < n1; ++j) sum += C[(size_t)i * n1 + j];
                col[i] = sum; /* top edge, kept to N+1 coefficients */
            }
            for (int j = 0; j < n1; ++j) {
                REAL sum = 0;
                for (int i = 0; i < n1; ++i) sum += C[(size_t)i * n1 + j];
                right[j] = sum; /* right edge */
            }
            for (int j = 0; j < n1; ++j) left[j] = right[j];
        }
    }
    {
        REAL kt = 0;
        for (int i = 0; i < n1; ++i) kt += bot[(size_t)(m - 1) * n1 + i];
        *k_out = (double)kt;
    }
done:
    free(dx);
    free(dy);
    free(bot);
    free(C);
    return rc;
}

/*
 * One cell in isolation (for unit tests of the cell map): inputs a (la), b (lb)
 * monomial coefficients, c; outputs the N x N matrix C (N given) and the top
 * and right edge series of length N (untrimmed).
 */
int FN(sigk_oracle_cell)(const double* a, int la, const double* b, int lb, double c, int N,
                         double* C_out, double* top_out, double* right_out)
{
    if (N < 1 || N > NCAP || la < 1 || lb < 1 || la > NCAP || lb > NCAP) return ORC_EINVAL;
    pthread_once(&ST(once), ST(init_tables));
    REAL A[NCAP], B[NCAP];
    for (int i = 0; i < la; ++i) A[i] = a[i];
    for (int i = 0; i < lb; ++i) B[i] = b[i];
    REAL* C = (REAL*)malloc((size_t)N * N * sizeof(REAL));
    if (!C) return ORC_ENOMEM;
    ST(cell_matrix)(A, la, B, lb, (REAL)c, N, C);
    for (int i = 0; i < N; ++i) {
        REAL s = 0;
        for (int j = 0; j < N; ++j) s += C[(size_t)i * N + j];
        if (top_out) top_out[i] = (double)s;
    }
    for (int j = 0; j < N; ++j) {
        REAL s = 0;
        for (int i = 0; i < N; ++i) s += C[(size_t)i * N + j];
        if (right_out) right_out[j] = (double)s;
    }
    if (C_out)
        for (int i = 0; i < N * N; ++i) C_out[i] = (double)C[i];
    free(C);
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Many pairs on a thread pool (one pair per task, raster sweep inside).    */

typedef struct {
    const double* pool;
    const int64_t* offsets;
    const int32_t* pairs;
    int64_t npairs, d;
    double* out;
    int64_t next;
    int rc;
    pthread_mutex_t mu;
} ST(job);

static void* ST(worker)(void* arg)
{
    ST(job)* J = (ST(job)*)arg;
    for (;;) {
        pthread_mutex_lock(&J->mu);
        int64_t p = J->next++;
        int stop = J->rc != 0;
        pthread_mutex_unlock(&J->mu);
        if (p >= J->npairs || stop) break;
        int32_t px = J->pairs[2 * p], py = J->pairs[2 * p + 1];
        const double* x = J->pool + J->offsets[px] * J->d;
        const double* y = J->pool + J->offsets[py] * J->d;
        int64_t lx = J->offsets[px + 1] - J->offsets[px];
        int64_t ly = J->offsets[py + 1] - J->offsets[py];
        int rc = FN(sigk_oracle_pair)(x, lx, y, ly, J->d, &J->out[p], NULL, NULL);
        if (rc) {
            pthread_mutex_lock(&J->mu);
            J->rc = rc;
            pthread_mutex_unlock(&J->mu);
        }
    }
    return NULL;
}

/*
 * Ragged batch: pool [sum len][d] of concatenated paths, offsets[npaths+1] in
 * points, pairs[npairs][2] path ids; out[npairs].  nthreads <= 0: all cores.
 */
int FN(sigk_oracle_ragged)(const double* pool, const int64_t* offsets, int64_t npaths, int64_t d,
                           const int32_t* pairs, int64_t npairs, double* out, int nthreads)
{
    if (!pool || !offsets || !pairs || !out || d < 1 || npaths < 0 || npairs < 0)
        return ORC_EINVAL;
    for (int64_t p = 0; p < npairs; ++p)
        if (pairs[2 * p] < 0 || pairs[2 * p] >= npaths || pairs[2 * p + 1] < 0 ||
            pairs[2 * p + 1] >= npaths)
            return ORC_EINVAL;
    if (nthreads <= 0) nthreads = (int)sysconf(_SC_NPROCESSORS_ONLN);
    if (nthreads < 1) nthreads = 1;
    if (nthreads > 256) nthreads = 256;
    ST(job) J;
    J.pool = pool;
    J.offsets = offsets;
    J.pairs = pairs;
    J.npairs = npairs;
    J.d = d;
    J.out = out;
    J.next = 0;
    J.rc = 0;
    pthread_mutex_init(&J.mu, NULL);
    pthread_t th[256];
    for (int t = 0; t < nthreads; ++t) pthread_create(&th[t], NULL, ST(worker), &J);
    for (int t = 0; t < nthreads; ++t) pthread_join(th[t], NULL);
    pthread_mutex_destroy(&J.mu);
    return J.rc;
}

/* ------------------------------------------------------------------------ */
/* Continuous adjoint: dk/dx, dk/dy.                                        */
/*
 * Perturbing the cell coefficient c_kl changes K(1,1) by
 *     dk/dc_kl = int_cell K(u,v) R(u,v) du dv,
 * where R is the Riemann function of the Goursat operator at (1,1): the
 * solution of the same equation on [u,1]x[v,1] with R = 1 on the lines u = 1
 * and v = 1 (the adjoint of the Volterra equation of Sec. 2.1).  R is the
 * kernel of the two reversed paths, so it is obtained by sweeping the grid of
 * reversed increments; cell (k,l) of the original grid is cell
 * (m-1-k, n-1-l) there, expanded about the original cell's top-right corner
 * in the coordinates (1-u, 1-v).  With K = sum C_ij u^i v^j and
 * R = sum D_pq (1-u)^p (1-v)^q the integral is
 *     sum_{ijpq} C_ij D_pq Beta(i+1,p+1) Beta(j+1,q+1),
 * Beta(i+1,p+1) = i! p!/(i+p+1)!.  The chain rule through c_kl = <dx_k, dy_l>
 * and dx_k = x_{k+1} - x_k gives the gradients with respect to the points.
 */

static REAL ST(beta_ip)(int i, int p)
{
    /* i! p! / (i+p+1)! = 1/(i+p+1) * prod_{q=1..p} q/(i+q) */
    REAL v = 1;
    for (int q = 1; q <= p; ++q) v = v * (REAL)q / (REAL)(i + q);
    return v / (REAL)(i + p + 1);
}

int FN(sigk_oracle_grad)(const double* x, int64_t lx, const double* y, int64_t ly, int64_t d,
                         double* k_out, double* gx, double* gy)
{
    if (!x || !y || !k_out || !gx || !gy || d < 1 || lx < 0 || ly < 0) return ORC_EINVAL;
    memset(gx, 0, (size_t)lx * d * sizeof(double));
    memset(gy, 0, (size_t)ly * d * sizeof(double));
    if (lx < 2 || ly < 2) {
        *k_out = 1.0;
        return ORC_OK;
    }
    pthread_once(&ST(once), ST(init_tables));
    int64_t m = lx - 1, n = ly - 1;
    size_t cells = (size_t)m * (size_t)n;
    REAL *dx = NULL, *dy = NULL, *rdx = NULL, *rdy = NULL, *g = NULL, *C = NULL, *D = NULL,
         *T = NULL, *Bt = NULL;
    ST(store) sf, sr;
    memset(&sf, 0, sizeof sf);
    memset(&sr, 0, sizeof sr);
    int rc = ST(increments)(x, lx, d, &dx);
    if (!rc) rc = ST(increments)(y, ly, d, &dy);
    if (rc) goto done;
    rdx = (REAL*)malloc((size_t)m * d * sizeof(REAL));
    rdy = (REAL*)malloc((size_t)n * d * sizeof(REAL));
    g = (REAL*)calloc(cells, sizeof(REAL));
    C = (REAL*)malloc((size_t)NCAP * NCAP * sizeof(REAL));
    D = (REAL*)malloc((size_t)NCAP * NCAP * sizeof(REAL));
    T = (REAL*)malloc((size_t)NCAP * NCAP * sizeof(REAL));
    Bt = (REAL*)malloc((size_t)NCAP * NCAP * sizeof(REAL));
    sf.off = (size_t*)malloc(cells * sizeof(size_t));
    sf.la = (int*)malloc(cells * sizeof(int));
    sf.lb = (int*)malloc(cells * sizeof(int));
    sr.off = (size_t*)malloc(cells * sizeof(size_t));
    sr.la = (int*)malloc(cells * sizeof(int));
    sr.lb = (int*)malloc(cells * sizeof(int));
    if (!rdx || !rdy || !g || !C || !D || !T || !Bt || !sf.off || !sf.la || !sf.lb || !sr.off ||
        !sr.la || !sr.lb) {
        rc = ORC_ENOMEM;
        goto done;
    }
    /* reversed paths: z_rev[k] = z[len-1-k], so dz_rev[k] = -dz[len-2-k] */
    for (int64_t k = 0; k < m; ++k)
        for (int64_t ch = 0; ch < d; ++ch) rdx[k * d + ch] = -dx[(m - 1 - k) * d + ch];
    for (int64_t l = 0; l < n; ++l)
        for (int64_t ch = 0; ch < d; ++ch) rdy[l * d + ch] = -dy[(n - 1 - l) * d + ch];
    REAL kf = 0, kr = 0;
    rc = ST(sweep)(dx, m, dy, n, d, &kf, NULL, &sf);
    if (!rc) rc = ST(sweep)(rdx, m, rdy, n, d, &kr, NULL, &sr);
    if (rc) goto done;
    for (int i = 0; i < NCAP; ++i)
        for (int p = 0; p < NCAP; ++p) Bt[(size_t)i * NCAP + p] = ST(beta_ip)(i, p);
    for (int64_t l = 0; l < n; ++l)
        for (int64_t k = 0; k < m; ++k) {
            size_t cf = (size_t)l * m + k;
            size_t cr = (size_t)(n - 1 - l) * m + (m - 1 - k);
            REAL c = 0;
            for (int64_t ch = 0; ch < d; ++ch) c += dx[k * d + ch] * dy[l * d + ch];
            int laf = sf.la[cf], lbf = sf.lb[cf], lar = sr.la[cr], lbr = sr.lb[cr];
            int Nf = (laf > lbf ? laf : lbf) + ST(neumann_terms)(c);
            int Nr = (lar > lbr ? lar : lbr) + ST(neumann_terms)(c);
            if (Nf > NCAP || Nr > NCAP) {
                rc = ORC_ECAP;
                goto done;
            }
            ST(cell_matrix)(sf.pool + sf.off[cf], laf, sf.pool + sf.off[cf] + laf, lbf, c, Nf, C);
            ST(cell_matrix)(sr.pool + sr.off[cr], lar, sr.pool + sr.off[cr] + lar, lbr, c, Nr, D);
            /* T = Bt[0:Nf, 0:Nr] * D  (Nf x Nr) */
            for (int i = 0; i < Nf; ++i)
                for (int q = 0; q < Nr; ++q) {
                    REAL s = 0;
                    for (int p = 0; p < Nr; ++p)
                        s += Bt[(size_t)i * NCAP + p] * D[(size_t)p * Nr + q];
                    T[(size_t)i * Nr + q] = s;
                }
            /* g = sum_ij C_ij * (T * Bt^T)_ij */
            REAL gs = 0;
            for (int i = 0; i < Nf; ++i)
                for (int j = 0; j < Nf; ++j) {
                    REAL s = 0;
                    for (int q = 0; q < Nr; ++q)
                        s += T[(size_t)i * Nr + q] * Bt[(size_t)j * NCAP + q];
                    gs += C[(size_t)i * Nf + j] * s;
                }
            g[cf] = gs;
        }
    /* chain rule: dk/ddx_k = sum_l g_kl dy_l ; dk/ddy_l = sum_k g_kl dx_k */
    for (int64_t k = 0; k < m; ++k)
        for (int64_t ch = 0; ch < d; ++ch) {
            REAL s = 0;
            for (int64_t l = 0; l < n; ++l) s += g[(size_t)l * m + k] * dy[l * d + ch];
            /* dx_k = x_{k+1} - x_k */
            gx[(k + 1) * d + ch] += (double)s;
            gx[k * d + ch] -= (double)s;
        }
    for (int64_t l = 0; l < n; ++l)
        for (int64_t ch = 0; ch < d; ++ch) {
            REAL s = 0;
            for (int64_t k = 0; k < m; ++k) s += g[(size_t)l * m + k] * dx[k * d + ch];
            gy[(l + 1) * d + ch] += (double)s;
            gy[l * d + ch] -= (double)s;
        }
    *k_out = (double)kf;
done:
    free(dx);
    free(dy);
    free(rdx);
    free(rdy);
    free(g);
    free(C);
    free(D);
    free(T);
    free(Bt);
    free(sf.pool);
    free(sf.off);
    free(sf.la);
    free(sf.lb);
    free(sr.pool);
    free(sr.off);
    free(sr.la);
    free(sr.lb);
    return rc;
}
