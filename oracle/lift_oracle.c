/*
 * Reference oracle for the BLAS pattern compositions of Steuwer, Fensch and
 * Dubach, "Patterns and Rewrite Rules for Systematic Code Generation"
 * (arXiv 1502.02389).  TEST INFRASTRUCTURE ONLY: the tests, the smoke check
 * and the CPU-baseline leg of the benchmark call this code; the GPU library
 * never does, and the two share no source.
 *
 * Everything is evaluated in IEEE binary64 with no fusion, blocking or
 * reordering beyond what the pattern definitions state:
 *
 *   map(f)         T[n] -> U[n], f applied to every element     (Table 1)
 *   zip(a, b)      a:T[n], b:U[n] -> <T,U>[n]                    (Table 1)
 *   reduce(f, z)   T[] -> T[1]; evaluated as the sequential left fold
 *                  acc = z; acc = f(acc, a_i) for i = 0..n-1, which is the
 *                  one reduction the paper lowers to (reduce-seq, Table 2
 *                  and the reduction lowering rule of Fig. 4b)
 *
 * and the four linear-algebra programs are the literal compositions of the
 * BLAS figure (Fig. 5, Section 5.1):
 *
 *   abs(x)            = if x < 0 then -x else x
 *   scal(a, x)        = map(mult(a), x)
 *   asum(x)           = reduce(add, 0) . map(abs, x)
 *   dot(x, y)         = reduce(add, 0) . map(mult) . zip(x, y)
 *   gemv(A, x, y, a, b):
 *       z  = map(scal(a) . dot(x), A)            (one dot per row of A)
 *       y' = map(add) . zip(z, scal(b, y))
 *
 * Readings where the paper is silent:
 *   - storage types f32 / bf16 / f16 are widened EXACTLY to binary64 as the
 *     first map; every result is binary64 (the caller rounds if it wants);
 *   - gemv follows the BLAS convention that beta == 0 means y is not read
 *     (NaN/Inf in y do not propagate); for beta != 0 it is the literal
 *     composition above;
 *   - A is row-major with leading dimension lda >= n (map over rows).
 *
 * For timing on a multi-core host there is also the split-join form of
 * scal, asum and dot on p threads (rule 3d of Section 4: a reduction may be
 * split into partial reductions whose results are reduced again, valid when
 * z is the identity of f): split the input into p chunks, run the sequential
 * composition above on each chunk on its own thread (a map over the chunks),
 * then reduce the p partial results in chunk order.  A shorter last chunk is
 * the same as padding with z.  On integer-valued inputs it equals the
 * sequential form exactly; in floating point it is another association.
 *
 * Pins (see tests/test_oracle_blas.py): closed forms, exact integer sums,
 * math.fsum (correctly rounded) within the sequential-fold error bound,
 * Hadamard orthogonality, brute force with Python Fractions, and the
 * decoders against numpy / torch for all 65536 16-bit patterns.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>
#include <pthread.h>

enum { OR_F32 = 0, OR_BF16 = 1, OR_F16 = 2, OR_F64 = 3 };
enum { OR_OK = 0, OR_EINVAL = -1, OR_ENOMEM = -2 };

/* ------------------------------------------------------------------ */
/* exact storage decoders (IEEE 754 binary32 / binary16, bfloat16)     */
/* ------------------------------------------------------------------ */

static double decode_f32(uint32_t bits)
{
    float f;
    memcpy(&f, &bits, sizeof f);
    return (double)f; /* binary32 -> binary64 is exact */
}

/* bfloat16 is the upper half of a binary32 encoding. */
static double decode_bf16(uint16_t h)
{
    return decode_f32((uint32_t)h << 16);
}

/* binary16: 1 sign bit, 5 exponent bits (bias 15), 10 fraction bits. */
static double decode_f16(uint16_t h)
{
    int sign = (h >> 15) & 1;
    int e = (h >> 10) & 0x1f;
    int m = h & 0x3ff;
    double v;
    if (e == 0)
        v = ldexp((double)m, -24);              /* zero / subnormal */
    else if (e == 31)
        v = m ? NAN : INFINITY;
    else
        v = ldexp((double)(1024 + m), e - 25);  /* (1.m) * 2^(e-15) */
    return sign ? -v : v;
}

static double load_elem(int dtype, const void *base, int64_t i)
{
    switch (dtype) {
    case OR_F32: {
        uint32_t b;
        memcpy(&b, (const char *)base + 4 * i, 4);
        return decode_f32(b);
    }
    case OR_BF16: {
        uint16_t b;
        memcpy(&b, (const char *)base + 2 * i, 2);
        return decode_bf16(b);
    }
    case OR_F16: {
        uint16_t b;
        memcpy(&b, (const char *)base + 2 * i, 2);
        return decode_f16(b);
    }
    default:
        return ((const double *)base)[i];
    }
}

static int valid_dtype(int t) { return t >= OR_F32 && t <= OR_F64; }

/* ------------------------------------------------------------------ */
/* high-level patterns (Table 1) over binary64 arrays                  */
/* ------------------------------------------------------------------ */

typedef double (*unary_fn)(double v, const void *env);
typedef double (*binary_fn)(double a, double b, const void *env);
typedef struct { double a, b; } pair_t;

/* map(f): out[i] = f(in[i]) */
static void map1(int64_t n, const double *in, double *out, unary_fn f, const void *env)
{
    for (int64_t i = 0; i < n; ++i)
        out[i] = f(in[i], env);
}

/* zip(a, b): out[i] = <a[i], b[i]> */
static void zip(int64_t n, const double *a, const double *b, pair_t *out)
{
    for (int64_t i = 0; i < n; ++i) {
        out[i].a = a[i];
        out[i].b = b[i];
    }
}

/* map(f) over an array of pairs, f taking the pair's two components */
static void map_pairs(int64_t n, const pair_t *in, double *out, binary_fn f, const void *env)
{
    for (int64_t i = 0; i < n; ++i)
        out[i] = f(in[i].a, in[i].b, env);
}

/* reduce(f, z): sequential left fold from index 0 */
static double reduce(int64_t n, const double *in, binary_fn f, double z, const void *env)
{
    double acc = z;
    for (int64_t i = 0; i < n; ++i)
        acc = f(acc, in[i], env);
    return acc;
}

/* widening map: the exact conversion of the stored type to binary64 */
static void widen(int64_t n, int dtype, const void *src, int64_t stride, double *dst)
{
    for (int64_t i = 0; i < n; ++i)
        dst[i] = load_elem(dtype, src, i * stride);
}

/* ------------------------------------------------------------------ */
/* user functions of the BLAS figure                                    */
/* ------------------------------------------------------------------ */

static double fn_add(double x, double y, const void *env) { (void)env; return x + y; }
static double fn_mult(double x, double y, const void *env) { (void)env; return x * y; }
static double fn_abs(double x, const void *env) { (void)env; return (x < 0) ? -x : x; }
/* mult(a) with a bound as the first argument (partial application) */
static double fn_mult_bound(double x, const void *env) { return *(const double *)env * x; }
/* |a*b|: used only for the error-bound denominators below */
static double fn_absmult(double x, double y, const void *env)
{
    (void)env;
    double p = x * y;
    return (p < 0) ? -p : p;
}

/* ------------------------------------------------------------------ */
/* exported entry points                                                */
/* ------------------------------------------------------------------ */

int oracle_widen(int64_t n, int dtype, const void *x, double *out)
{
    if (n < 0 || !valid_dtype(dtype) || (n > 0 && (!x || !out)))
        return OR_EINVAL;
    widen(n, dtype, x, 1, out);
    return OR_OK;
}

/* scal(a, x) = map(mult(a), x) */
int oracle_scal(int64_t n, double alpha, int xt, const void *x, double *out)
{
    if (n < 0 || !valid_dtype(xt) || (n > 0 && (!x || !out)))
        return OR_EINVAL;
    double *w = malloc((size_t)(n ? n : 1) * sizeof *w);
    if (!w)
        return OR_ENOMEM;
    widen(n, xt, x, 1, w);
    map1(n, w, out, fn_mult_bound, &alpha);
    free(w);
    return OR_OK;
}

/* asum(x) = reduce(add, 0) . map(abs, x) */
int oracle_asum(int64_t n, int xt, const void *x, double *result)
{
    if (n < 0 || !valid_dtype(xt) || !result || (n > 0 && !x))
        return OR_EINVAL;
    double *w = malloc((size_t)(n ? n : 1) * sizeof *w);
    double *t = malloc((size_t)(n ? n : 1) * sizeof *t);
    if (!w || !t) {
        free(w);
        free(t);
        return OR_ENOMEM;
    }
    widen(n, xt, x, 1, w);
    map1(n, w, t, fn_abs, NULL);
    *result = reduce(n, t, fn_add, 0.0, NULL);
    free(w);
    free(t);
    return OR_OK;
}

/* reduce(add, 0) . map(g) . zip(x, y) on already-widened operands */
static double dot_widened(int64_t n, const double *wx, const double *wy, binary_fn g,
                          pair_t *zbuf, double *pbuf)
{
    zip(n, wx, wy, zbuf);
    map_pairs(n, zbuf, pbuf, g, NULL);
    return reduce(n, pbuf, fn_add, 0.0, NULL);
}

static int dot_common(int64_t n, int xt, const void *x, int yt, const void *y,
                      binary_fn g, double *result)
{
    if (n < 0 || !valid_dtype(xt) || !valid_dtype(yt) || !result || (n > 0 && (!x || !y)))
        return OR_EINVAL;
    size_t m = (size_t)(n ? n : 1);
    double *wx = malloc(m * sizeof *wx);
    double *wy = malloc(m * sizeof *wy);
    pair_t *z = malloc(m * sizeof *z);
    double *p = malloc(m * sizeof *p);
    int rc = OR_OK;
    if (!wx || !wy || !z || !p) {
        rc = OR_ENOMEM;
    } else {
        widen(n, xt, x, 1, wx);
        widen(n, yt, y, 1, wy);
        *result = dot_widened(n, wx, wy, g, z, p);
    }
    free(wx);
    free(wy);
    free(z);
    free(p);
    return rc;
}

/* dot(x, y) = reduce(add, 0) . map(mult) . zip(x, y) */
int oracle_dot(int64_t n, int xt, const void *x, int yt, const void *y, double *result)
{
    return dot_common(n, xt, x, yt, y, fn_mult, result);
}

/* sum_i |x_i * y_i|: the condition denominator used to state dot's error */
int oracle_dot_absmass(int64_t n, int xt, const void *x, int yt, const void *y, double *result)
{
    return dot_common(n, xt, x, yt, y, fn_absmult, result);
}

static int gemv_common(int64_t m, int64_t n, double alpha, int at, const void *A, int64_t lda,
                       int xt, const void *x, double beta, int yt, const void *y,
                       binary_fn g, int absolute, double *out)
{
    if (m < 0 || n < 0 || lda < (n > 1 ? n : 1) || !valid_dtype(at) || !valid_dtype(xt) ||
        !valid_dtype(yt) || (m > 0 && !out) || (m > 0 && n > 0 && (!A || !x)) ||
        (m > 0 && beta != 0.0 && !y))
        return OR_EINVAL;
    size_t nn = (size_t)(n ? n : 1);
    double *wx = malloc(nn * sizeof *wx);
    double *row = malloc(nn * sizeof *row);
    pair_t *zb = malloc(nn * sizeof *zb);
    double *pb = malloc(nn * sizeof *pb);
    size_t mm = (size_t)(m ? m : 1);
    double *z = malloc(mm * sizeof *z);
    double *wy = malloc(mm * sizeof *wy);
    double *by = malloc(mm * sizeof *by);
    pair_t *zz = malloc(mm * sizeof *zz);
    int rc = OR_OK;
    if (!wx || !row || !zb || !pb || !z || !wy || !by || !zz) {
        rc = OR_ENOMEM;
        goto done;
    }
    widen(n, xt, x, 1, wx);
    /* z = map(scal(a) . dot(x), A): one dot per row, then multiply by a */
    size_t esz = (at == OR_F32) ? 4 : (at == OR_F64) ? 8 : 2;
    for (int64_t i = 0; i < m; ++i) {
        if (n > 0)
            widen(n, at, (const char *)A + (size_t)i * (size_t)lda * esz, 1, row);
        double d = dot_widened(n, wx, row, g, zb, pb);
        double a = absolute ? fabs(alpha) : alpha;
        double one[1] = {d}, scaled[1];
        map1(1, one, scaled, fn_mult_bound, &a); /* scal(a) of the length-1 dot */
        z[i] = scaled[0];
    }
    /* y' = map(add) . zip(z, scal(b, y)); beta == 0 leaves y unread */
    if (beta == 0.0) {
        for (int64_t i = 0; i < m; ++i)
            by[i] = 0.0;
    } else {
        double b = absolute ? fabs(beta) : beta;
        widen(m, yt, y, 1, wy);
        if (absolute)
            map1(m, wy, wy, fn_abs, NULL);
        map1(m, wy, by, fn_mult_bound, &b);
    }
    zip(m, z, by, zz);
    map_pairs(m, zz, out, fn_add, NULL);
done:
    free(wx);
    free(row);
    free(zb);
    free(pb);
    free(z);
    free(wy);
    free(by);
    free(zz);
    return rc;
}

/* gemv: y' = alpha * A x + beta * y, row-major A with leading dimension lda */
int oracle_gemv(int64_t m, int64_t n, double alpha, int at, const void *A, int64_t lda,
                int xt, const void *x, double beta, int yt, const void *y, double *out)
{
    return gemv_common(m, n, alpha, at, A, lda, xt, x, beta, yt, y, fn_mult, 0, out);
}

/* |alpha| * sum_j |A_ij x_j| + |beta y_i|: per-row error denominator for gemv */
int oracle_gemv_absmass(int64_t m, int64_t n, double alpha, int at, const void *A, int64_t lda,
                        int xt, const void *x, double beta, int yt, const void *y, double *out)
{
    return gemv_common(m, n, alpha, at, A, lda, xt, x, beta, yt, y, fn_absmult, 1, out);
}

/* ------------------------------------------------------------------ */
/* split-join form on p threads (rule 3d)                               */
/* ------------------------------------------------------------------ */

enum { PAR_SCAL = 0, PAR_ASUM = 1, PAR_DOT = 2 };
enum { PAR_MAX_THREADS = 256 };

typedef struct {
    int op;
    int64_t n;          /* this chunk's length */
    int xt, yt;
    const void *x, *y;  /* this chunk's first elements */
    double alpha;
    double *out;        /* scal: this chunk's first output */
    double partial;     /* asum / dot: the chunk's reduction */
    int rc;
} par_chunk;

static size_t elem_size(int dtype)
{
    return dtype == OR_F64 ? 8 : dtype == OR_F32 ? 4 : 2;
}

static void *par_worker(void *arg)
{
    par_chunk *c = arg;
    switch (c->op) {
    case PAR_SCAL:
        c->rc = oracle_scal(c->n, c->alpha, c->xt, c->x, c->out);
        break;
    case PAR_ASUM:
        c->rc = oracle_asum(c->n, c->xt, c->x, &c->partial);
        break;
    default:
        c->rc = oracle_dot(c->n, c->xt, c->x, c->yt, c->y, &c->partial);
        break;
    }
    return NULL;
}

/* map over the p chunks on p threads, then (asum, dot) reduce(add, 0) over
   the chunk results in chunk order */
static int split_join(int op, int64_t n, int xt, const void *x, int yt, const void *y, double alpha,
                      double *out, double *result, int threads)
{
    if (n < 0 || threads < 1 || threads > PAR_MAX_THREADS || !valid_dtype(xt) ||
        (op == PAR_DOT && !valid_dtype(yt)))
        return OR_EINVAL;
    if (n > 0 && (!x || (op == PAR_DOT && !y) || (op == PAR_SCAL && !out)))
        return OR_EINVAL;
    if (op != PAR_SCAL && !result)
        return OR_EINVAL;
    int64_t p = threads;
    int64_t k = n > 0 ? (n + p - 1) / p : 0;   /* chunk length of split(k) */
    if (k > 0)
        p = (n + k - 1) / k;                    /* chunks actually formed */
    else
        p = 0;
    par_chunk c[PAR_MAX_THREADS];
    pthread_t tid[PAR_MAX_THREADS];
    int started[PAR_MAX_THREADS];
    for (int64_t i = 0; i < p; ++i) {
        int64_t lo = i * k, len = (n - lo < k) ? n - lo : k;
        c[i].op = op;
        c[i].n = len;
        c[i].xt = xt;
        c[i].yt = yt;
        c[i].x = (const char *)x + (size_t)lo * elem_size(xt);
        c[i].y = op == PAR_DOT ? (const char *)y + (size_t)lo * elem_size(yt) : NULL;
        c[i].alpha = alpha;
        c[i].out = op == PAR_SCAL ? out + lo : NULL;
        c[i].partial = 0.0;
        c[i].rc = OR_OK;
        started[i] = pthread_create(&tid[i], NULL, par_worker, &c[i]) == 0;
        if (!started[i])
            par_worker(&c[i]);                  /* no thread: run the chunk here */
    }
    int rc = OR_OK;
    for (int64_t i = 0; i < p; ++i) {
        if (started[i])
            pthread_join(tid[i], NULL);
        if (c[i].rc != OR_OK)
            rc = c[i].rc;
    }
    if (rc != OR_OK)
        return rc;
    if (op != PAR_SCAL) {
        double acc = 0.0;
        for (int64_t i = 0; i < p; ++i)
            acc = fn_add(acc, c[i].partial, NULL);
        *result = acc;
    }
    return OR_OK;
}

int oracle_scal_par(int64_t n, double alpha, int xt, const void *x, double *out, int threads)
{
    return split_join(PAR_SCAL, n, xt, x, OR_F64, NULL, alpha, out, NULL, threads);
}

int oracle_asum_par(int64_t n, int xt, const void *x, double *result, int threads)
{
    return split_join(PAR_ASUM, n, xt, x, OR_F64, NULL, 0.0, NULL, result, threads);
}

int oracle_dot_par(int64_t n, int xt, const void *x, int yt, const void *y, double *result, int threads)
{
    return split_join(PAR_DOT, n, xt, x, yt, y, 0.0, NULL, result, threads);
}

/* ------------------------------------------------------------------ */
/* BlackScholes: map(BSComputation) over stock prices (Section 5.2)    */
/* ------------------------------------------------------------------ */
/*
 * The paper maps BSComputation over a vector of stock prices s; for each s
 * it computes d1 = compD1(s), d2 = compD2(d1, s) and returns the pair
 * {compCall(d1, d2, s), compPut(d1, d2, s)}.  The four helpers are not
 * printed; they are the closed-form Black-Scholes model for a European
 * option with strike K, time to expiry T (years), risk-free rate r and
 * volatility v, the same for every element:
 *
 *   d1   = (ln(s / K) + (r + v^2 / 2) T) / (v sqrt(T))
 *   d2   = d1 - v sqrt(T)
 *   call = s N(d1) - K exp(-r T) N(d2)
 *   put  = K exp(-r T) N(-d2) - s N(-d1)
 *
 * with N the standard normal distribution function, N(x) = erfc(-x/sqrt 2)/2.
 * Output: pairs {call, put}, element i at out[2i], out[2i + 1].
 */
typedef struct { double K, r, v, T; } bs_params;

static double cnd(double x) { return 0.5 * erfc(-x / sqrt(2.0)); }

static double comp_d1(double s, const bs_params *q)
{
    return (log(s / q->K) + (q->r + 0.5 * q->v * q->v) * q->T) / (q->v * sqrt(q->T));
}

static double comp_d2(double d1, double s, const bs_params *q)
{
    (void)s;
    return d1 - q->v * sqrt(q->T);
}

static double comp_call(double d1, double d2, double s, const bs_params *q)
{
    return s * cnd(d1) - q->K * exp(-q->r * q->T) * cnd(d2);
}

static double comp_put(double d1, double d2, double s, const bs_params *q)
{
    return q->K * exp(-q->r * q->T) * cnd(-d2) - s * cnd(-d1);
}

/* BSComputation(s) = {compCall(d1, d2, s), compPut(d1, d2, s)} */
static pair_t bs_computation(double s, const bs_params *q)
{
    double d1 = comp_d1(s, q);
    double d2 = comp_d2(d1, s, q);
    pair_t r = {comp_call(d1, d2, s, q), comp_put(d1, d2, s, q)};
    return r;
}

int oracle_blackscholes(int64_t n, int st, const void *s, double strike, double rate, double volatility,
                        double years, double *out)
{
    if (n < 0 || !valid_dtype(st) || (n > 0 && (!s || !out)))
        return OR_EINVAL;
    if (!(strike > 0) || !(volatility > 0) || !(years > 0) || !isfinite(rate))
        return OR_EINVAL;
    double *w = malloc((size_t)(n ? n : 1) * sizeof *w);
    if (!w)
        return OR_ENOMEM;
    widen(n, st, s, 1, w);
    bs_params q = {strike, rate, volatility, years};
    for (int64_t i = 0; i < n; ++i) {   /* map(BSComputation) */
        pair_t cp = bs_computation(w[i], &q);
        out[2 * i] = cp.a;
        out[2 * i + 1] = cp.b;
    }
    free(w);
    return OR_OK;
}

/* ------------------------------------------------------------------ */
/* MD: map over particles of a reduce over neighbour indices (Fig. 7)  */
/* ------------------------------------------------------------------ */
/*
 *   md(ps, N, t) = map(lambda (p, ns): reduce(lambda (f, nId):
 *                         updateF(f, nId, p, ps, t), 0, ns)) . zip(ps, N)
 *   updateF(f, nId, p, ps, t): q = ps[nId]; d = distance(p, q);
 *                              if d < t then f + calculateForce(p, q) else f
 *
 * The paper gives neither calculateForce nor the neighbour lists.  Readings:
 *   - the force of q on p is the Lennard-Jones pair force
 *       F = 24 eps / r^2 * (2 (sigma^2/r^2)^6 - (sigma^2/r^2)^3) * (p - q),
 *     r = |p - q|, i.e. minus the gradient of 4 eps ((sigma/r)^12 - (sigma/r)^6);
 *   - positions are 4 floats per particle (x, y, z, unused), forces 3 values;
 *   - N is an n x k row-major matrix of int32 indices; an index outside
 *     [0, n) is an empty slot and leaves f unchanged (lists of uneven length);
 *   - "d < t" is the plain definition: the Euclidean distance of the two
 *     stored binary32 positions, evaluated in binary64 (the differences are
 *     exact there, the distance is within a few binary64 ulps), compared
 *     with t.  The force is evaluated in binary64 from the same positions;
 *   - reduce is the sequential fold over the list in order (the fused lambda
 *     is valid only for reduce-seq).
 */
typedef struct { double x, y, z; } vec3_t;
typedef struct { double eps24, sigma2, t; } md_params;

/* updateF's test: distance(p, q) < t */
static int md_within(const float *p, const float *q, double t)
{
    double d0 = (double)p[0] - q[0], d1 = (double)p[1] - q[1], d2 = (double)p[2] - q[2];
    return sqrt(d0 * d0 + d1 * d1 + d2 * d2) < t;
}

/* calculateForce: the pair force on p from q (binary64 from binary32 input) */
static vec3_t calculate_force(const float *p, const float *q, const md_params *m, vec3_t *mass)
{
    double dx = (double)p[0] - q[0], dy = (double)p[1] - q[1], dz = (double)p[2] - q[2];
    double r2 = dx * dx + dy * dy + dz * dz;
    double s2 = m->sigma2 / r2;
    double s6 = s2 * s2 * s2;
    double a = m->eps24 / r2 * s6 * 2.0 * s6;  /* repulsive term */
    double b = m->eps24 / r2 * s6;             /* attractive term */
    vec3_t f = {(a - b) * dx, (a - b) * dy, (a - b) * dz};
    if (mass) {  /* |terms|: the scale of the rounding error of f */
        mass->x += (a + b) * fabs(dx);
        mass->y += (a + b) * fabs(dy);
        mass->z += (a + b) * fabs(dz);
    }
    return f;
}

static vec3_t update_f(vec3_t f, int32_t nid, const float *p, const float *ps, int64_t n, const md_params *m,
                       vec3_t *mass)
{
    if (nid < 0 || (int64_t)nid >= n)
        return f;  /* empty slot */
    const float *q = ps + 4 * (int64_t)nid;
    if (md_within(p, q, m->t)) {
        vec3_t g = calculate_force(p, q, m, mass);
        f.x += g.x;
        f.y += g.y;
        f.z += g.z;
    }
    return f;
}

int oracle_md(int64_t n, const float *pos, int64_t k, const int32_t *nbr, double cutoff, double epsilon,
              double sigma, double *force, double *mass)
{
    if (n < 0 || k < 0 || (n > 0 && (!pos || !force)) || (n > 0 && k > 0 && !nbr))
        return OR_EINVAL;
    if (!(cutoff >= 0) || !isfinite(cutoff) || !(sigma > 0) || !isfinite(sigma) || !isfinite(epsilon))
        return OR_EINVAL;
    md_params m = {24.0 * epsilon, sigma * sigma, cutoff};
    for (int64_t i = 0; i < n; ++i) {  /* map over zip(ps, N) */
        const float *p = pos + 4 * i;
        vec3_t f = {0.0, 0.0, 0.0};    /* reduce(..., 0, ns): fold in list order */
        vec3_t ms = {0.0, 0.0, 0.0};
        for (int64_t j = 0; j < k; ++j)
            f = update_f(f, nbr[i * k + j], p, pos, n, &m, mass ? &ms : NULL);
        force[3 * i] = f.x;
        force[3 * i + 1] = f.y;
        force[3 * i + 2] = f.z;
        if (mass) {
            mass[3 * i] = ms.x;
            mass[3 * i + 1] = ms.y;
            mass[3 * i + 2] = ms.z;
        }
    }
    return OR_OK;
}
