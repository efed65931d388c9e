/*
 * Oracle: plain FP64 direct-summation two-point correlations and their
 * exact adjoint.  TEST INFRASTRUCTURE ONLY -- nothing in the product path
 * may link, load or call this file.  Only the test suite, the smoke check
 * and the CPU-baseline leg of the benchmark use it.
 *
 * What it computes (Seibert et al., "Reconstructing random heterogeneous
 * media through differentiable optimization"):
 *
 *   Two-point correlation, Sec. 3.2.1 (probability that a vector r starts in
 *   phase a and ends in phase b), evaluated over every pixel as a starting
 *   point, Sec. 3.2.2 (n_r = I*J realisations, linear ensemble average), with
 *   periodic wrap-around as in the convolution of eq. (convdef), indices
 *   written 0-based:
 *
 *       S_ab(r) = (1/N) * sum_x  a(x) * b((x + r) mod n)
 *
 *   For a soft field this is the corrected descriptor of Appendix A with the
 *   identity threshold (Sec. 5.1 runs the method without the threshold and
 *   states the Appendix A corrections still hold).
 *
 *   Adjoint (the exact derivative the method back-propagates, Sec. 3.1 and
 *   Appendix B): for a cotangent G(r) over the displacement list,
 *
 *       d/da(x) sum_r G(r) S_ab(r) = (1/N) sum_r G(r) b(x + r)
 *       d/db(y) sum_r G(r) S_ab(r) = (1/N) sum_r G(r) a(y - r)
 *
 * Fields are dense row-major arrays of shape n0 x n1 x n2 (axis 2 fastest);
 * a 2-D field is passed with n0 = 1.  Displacements are K triples (r0,r1,r2).
 * Nothing here is blocked, fused or reordered: every sum is the definition
 * written out.  OpenMP only splits independent outputs across threads.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

static inline int64_t wrap(int64_t i, int64_t n)
{
    int64_t m = i % n;
    return m < 0 ? m + n : m;
}

static inline int64_t lin(int64_t i0, int64_t i1, int64_t i2,
                          int64_t n1, int64_t n2)
{
    return (i0 * n1 + i1) * n2 + i2;
}

int ora_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void ora_set_num_threads(int t)
{
#ifdef _OPENMP
    if (t > 0) omp_set_num_threads(t);
#else
    (void)t;
#endif
}

/* S[k] = (1/N) sum_x a[x] b[(x + r_k) mod n]  for k = 0..K-1. */
void ora_corr(int n0, int n1, int n2, const double *a, const double *b,
              int K, const int *r, double *S)
{
    const int64_t N = (int64_t)n0 * n1 * n2;
    int k;
#pragma omp parallel for schedule(dynamic, 1)
    for (k = 0; k < K; ++k) {
        const int r0 = r[3 * k], r1 = r[3 * k + 1], r2 = r[3 * k + 2];
        double acc = 0.0;
        for (int64_t i0 = 0; i0 < n0; ++i0) {
            const int64_t j0 = wrap(i0 + r0, n0);
            for (int64_t i1 = 0; i1 < n1; ++i1) {
                const int64_t j1 = wrap(i1 + r1, n1);
                for (int64_t i2 = 0; i2 < n2; ++i2) {
                    const int64_t j2 = wrap(i2 + r2, n2);
                    acc += a[lin(i0, i1, i2, n1, n2)] * b[lin(j0, j1, j2, n1, n2)];
                }
            }
        }
        S[k] = acc / (double)N;
    }
}

/* Gradient of sum_k G[k] S_ab(r_k) over the whole grid:
 *   ga[x] += (1/N) sum_k G[k] b[x + r_k]
 *   gb[x] += (1/N) sum_k G[k] a[x - r_k]
 * ga and gb may be the same array (auto-correlation: a == b). */
void ora_corr_adjoint(int n0, int n1, int n2, const double *a, const double *b,
                      int K, const int *r, const double *G,
                      double *ga, double *gb)
{
    const int64_t N = (int64_t)n0 * n1 * n2;
    int64_t x;
#pragma omp parallel for schedule(static)
    for (x = 0; x < N; ++x) {
        const int64_t i0 = x / ((int64_t)n1 * n2);
        const int64_t i1 = (x / n2) % n1;
        const int64_t i2 = x % n2;
        double sa = 0.0, sb = 0.0;
        for (int k = 0; k < K; ++k) {
            const int r0 = r[3 * k], r1 = r[3 * k + 1], r2 = r[3 * k + 2];
            sa += G[k] * b[lin(wrap(i0 + r0, n0), wrap(i1 + r1, n1), wrap(i2 + r2, n2), n1, n2)];
            sb += G[k] * a[lin(wrap(i0 - r0, n0), wrap(i1 - r1, n1), wrap(i2 - r2, n2), n1, n2)];
        }
        ga[x] += sa / (double)N;
        gb[x] += sb / (double)N;
    }
}

/* Same adjoint, evaluated only at nv listed voxels (v triples):
 *   ga_v[m] = (1/N) sum_k G[k] b[v_m + r_k],  gb_v[m] = (1/N) sum_k G[k] a[v_m - r_k]. */
void ora_corr_adjoint_at(int n0, int n1, int n2, const double *a, const double *b,
                         int K, const int *r, const double *G,
                         int nv, const int *v, double *ga_v, double *gb_v)
{
    const int64_t N = (int64_t)n0 * n1 * n2;
    int m;
#pragma omp parallel for schedule(dynamic, 1)
    for (m = 0; m < nv; ++m) {
        const int64_t i0 = v[3 * m], i1 = v[3 * m + 1], i2 = v[3 * m + 2];
        double sa = 0.0, sb = 0.0;
        for (int k = 0; k < K; ++k) {
            const int r0 = r[3 * k], r1 = r[3 * k + 1], r2 = r[3 * k + 2];
            sa += G[k] * b[lin(wrap(i0 + r0, n0), wrap(i1 + r1, n1), wrap(i2 + r2, n2), n1, n2)];
            sb += G[k] * a[lin(wrap(i0 - r0, n0), wrap(i1 - r1, n1), wrap(i2 - r2, n2), n1, n2)];
        }
        ga_v[m] = sa / (double)N;
        gb_v[m] = sb / (double)N;
    }
}

/*
 * Soft-threshold ensemble (Sec. 3.2.4, eq. softthreshold) on the two-point
 * masks of Sec. 3.2.3.  The mask of r != 0 holds 1/2 at the tip and at the
 * end of r, so the convolution of eq. (convdef) gives
 *     u_r(x) = (a(x) + b(x + r)) / 2;
 * the mask of r = 0 holds a single 1, which gives u_0(x) = a(x) -- the same
 * expression when a == b.  (For a cross pair, a != b, the same expression is
 * used at r = 0 as well.)  The threshold step applies the logistic
 *     f(u) = c1 / (1 + exp(-alpha (u + c2))) + c3,
 * and the quadratic reduction of eq. (s3) with r_a = r_b gives
 *     Sbar[k] = (1/N) sum_x f(u_{r_k}(x))^2.
 * coef = {alpha, c1, c2, c3}.
 */
#include <math.h>

static inline double soft_f(double u, const double *c)
{
    return c[1] / (1.0 + exp(-c[0] * (u + c[2]))) + c[3];
}

/* f(u) f'(u): the derivative of f(u)^2 with respect to either end value,
 * since du/da = du/db = 1/2 and d(f^2)/du = 2 f f'. */
static inline double soft_ffp(double u, const double *c)
{
    const double s = 1.0 / (1.0 + exp(-c[0] * (u + c[2])));
    const double f = c[1] * s + c[3];
    const double fp = c[1] * c[0] * s * (1.0 - s);
    return f * fp;
}

void ora_sbar(int n0, int n1, int n2, const double *a, const double *b,
              int K, const int *r, const double *coef, double *S)
{
    const int64_t N = (int64_t)n0 * n1 * n2;
    int k;
#pragma omp parallel for schedule(dynamic, 1)
    for (k = 0; k < K; ++k) {
        const int r0 = r[3 * k], r1 = r[3 * k + 1], r2 = r[3 * k + 2];
        double acc = 0.0;
        for (int64_t i0 = 0; i0 < n0; ++i0) {
            const int64_t j0 = wrap(i0 + r0, n0);
            for (int64_t i1 = 0; i1 < n1; ++i1) {
                const int64_t j1 = wrap(i1 + r1, n1);
                for (int64_t i2 = 0; i2 < n2; ++i2) {
                    const int64_t j2 = wrap(i2 + r2, n2);
                    const double u = 0.5 * (a[lin(i0, i1, i2, n1, n2)] + b[lin(j0, j1, j2, n1, n2)]);
                    const double e = soft_f(u, coef);
                    acc += e * e;
                }
            }
        }
        S[k] = acc / (double)N;
    }
}

/* Gradient of sum_k G[k] Sbar_ab(r_k):
 *   ga[x] += (1/N) sum_k G[k] (f f')((a[x] + b[x + r_k]) / 2)
 *   gb[y] += (1/N) sum_k G[k] (f f')((a[y - r_k] + b[y]) / 2)
 * ga and gb may be the same array (auto-correlation: a == b). */
void ora_sbar_adjoint(int n0, int n1, int n2, const double *a, const double *b,
                      int K, const int *r, const double *coef, const double *G,
                      double *ga, double *gb)
{
    const int64_t N = (int64_t)n0 * n1 * n2;
    int64_t x;
#pragma omp parallel for schedule(static)
    for (x = 0; x < N; ++x) {
        const int64_t i0 = x / ((int64_t)n1 * n2);
        const int64_t i1 = (x / n2) % n1;
        const int64_t i2 = x % n2;
        double sa = 0.0, sb = 0.0;
        for (int k = 0; k < K; ++k) {
            const int r0 = r[3 * k], r1 = r[3 * k + 1], r2 = r[3 * k + 2];
            const double bf = b[lin(wrap(i0 + r0, n0), wrap(i1 + r1, n1), wrap(i2 + r2, n2), n1, n2)];
            const double ab = a[lin(wrap(i0 - r0, n0), wrap(i1 - r1, n1), wrap(i2 - r2, n2), n1, n2)];
            sa += G[k] * soft_ffp(0.5 * (a[x] + bf), coef);
            sb += G[k] * soft_ffp(0.5 * (ab + b[x]), coef);
        }
        ga[x] += sa / (double)N;
        gb[x] += sb / (double)N;
    }
}

/* Same adjoint at nv listed voxels (v triples), written (not accumulated). */
void ora_sbar_adjoint_at(int n0, int n1, int n2, const double *a, const double *b,
                         int K, const int *r, const double *coef, const double *G,
                         int nv, const int *v, double *ga_v, double *gb_v)
{
    const int64_t N = (int64_t)n0 * n1 * n2;
    int m;
#pragma omp parallel for schedule(dynamic, 1)
    for (m = 0; m < nv; ++m) {
        const int64_t i0 = v[3 * m], i1 = v[3 * m + 1], i2 = v[3 * m + 2];
        const int64_t x = lin(i0, i1, i2, n1, n2);
        double sa = 0.0, sb = 0.0;
        for (int k = 0; k < K; ++k) {
            const int r0 = r[3 * k], r1 = r[3 * k + 1], r2 = r[3 * k + 2];
            const double bf = b[lin(wrap(i0 + r0, n0), wrap(i1 + r1, n1), wrap(i2 + r2, n2), n1, n2)];
            const double ab = a[lin(wrap(i0 - r0, n0), wrap(i1 - r1, n1), wrap(i2 - r2, n2), n1, n2)];
            sa += G[k] * soft_ffp(0.5 * (a[x] + bf), coef);
            sb += G[k] * soft_ffp(0.5 * (ab + b[x]), coef);
        }
        ga_v[m] = sa / (double)N;
        gb_v[m] = sb / (double)N;
    }
}

/*
 * Three-point correlation of one phase (Sec. 3.2.2, eq. s3): the quadratic
 * reduction of two realisations of the same start point x,
 *     S3(r_a, r_b) = (1/N) sum_x e_a(x) e_b(x).
 * mode 0 (product form, the exact three-point probability on binary fields):
 *     e_a(x) e_b(x) is replaced by phi(x) phi(x + r_a) phi(x + r_b);
 * mode 1 (soft threshold, Sec. 3.2.4): e_c(x) = f((phi(x) + phi(x + r_c)) / 2)
 *     with the logistic f (coef = {alpha, c1, c2, c3}); e_0(x) = f(phi(x)).
 * `vec` holds M displacement triples, `pa`/`pb` the K3 index pairs (a, b).
 */
static inline double s3_term(const double *f, int64_t x, int64_t xa, int64_t xb, int mode, const double *coef)
{
    if (mode == 0) return f[x] * f[xa] * f[xb];
    return soft_f(0.5 * (f[x] + f[xa]), coef) * soft_f(0.5 * (f[x] + f[xb]), coef);
}

void ora_s3(int n0, int n1, int n2, const double *f, const int *vec, int K3, const int *pa, const int *pb,
            int mode, const double *coef, double *S)
{
    const int64_t N = (int64_t)n0 * n1 * n2;
    int k;
#pragma omp parallel for schedule(dynamic, 1)
    for (k = 0; k < K3; ++k) {
        const int *a = vec + 3 * pa[k], *b = vec + 3 * pb[k];
        double acc = 0.0;
        for (int64_t i0 = 0; i0 < n0; ++i0)
            for (int64_t i1 = 0; i1 < n1; ++i1)
                for (int64_t i2 = 0; i2 < n2; ++i2) {
                    const int64_t x = lin(i0, i1, i2, n1, n2);
                    const int64_t xa = lin(wrap(i0 + a[0], n0), wrap(i1 + a[1], n1), wrap(i2 + a[2], n2), n1, n2);
                    const int64_t xb = lin(wrap(i0 + b[0], n0), wrap(i1 + b[1], n1), wrap(i2 + b[2], n2), n1, n2);
                    acc += s3_term(f, x, xa, xb, mode, coef);
                }
        S[k] = acc / (double)N;
    }
}

/* Gradient of sum_k G[k] S3_k with respect to f, accumulated into g: every
 * voxel y collects the derivative of each term in which it appears as the start
 * x, as x + r_a or as x + r_b (terms where two roles coincide collect both). */
void ora_s3_adjoint(int n0, int n1, int n2, const double *f, const int *vec, int K3, const int *pa,
                    const int *pb, int mode, const double *coef, const double *G, double *g)
{
    const int64_t N = (int64_t)n0 * n1 * n2;
    int64_t y;
#pragma omp parallel for schedule(static)
    for (y = 0; y < N; ++y) {
        const int64_t i0 = y / ((int64_t)n1 * n2), i1 = (y / n2) % n1, i2 = y % n2;
        double acc = 0.0;
        for (int k = 0; k < K3; ++k) {
            const int *a = vec + 3 * pa[k], *b = vec + 3 * pb[k];
            /* the three start points x whose term reads f(y): x = y, y - r_a, y - r_b */
            for (int role = 0; role < 3; ++role) {
                const int *s = role == 0 ? NULL : (role == 1 ? a : b);
                const int64_t j0 = s ? wrap(i0 - s[0], n0) : i0;
                const int64_t j1 = s ? wrap(i1 - s[1], n1) : i1;
                const int64_t j2 = s ? wrap(i2 - s[2], n2) : i2;
                const int64_t x = lin(j0, j1, j2, n1, n2);
                const int64_t xa = lin(wrap(j0 + a[0], n0), wrap(j1 + a[1], n1), wrap(j2 + a[2], n2), n1, n2);
                const int64_t xb = lin(wrap(j0 + b[0], n0), wrap(j1 + b[1], n1), wrap(j2 + b[2], n2), n1, n2);
                /* derivative of the term at x with respect to the factor(s) at position `role` */
                double d = 0.0;
                if (mode == 0) {
                    if (role == 0) d = f[xa] * f[xb];
                    if (role == 1) d = f[x] * f[xb];
                    if (role == 2) d = f[x] * f[xa];
                } else {
                    const double ua = 0.5 * (f[x] + f[xa]), ub = 0.5 * (f[x] + f[xb]);
                    const double ea = soft_f(ua, coef), eb = soft_f(ub, coef);
                    const double sa = 1.0 / (1.0 + exp(-coef[0] * (ua + coef[2])));
                    const double sb = 1.0 / (1.0 + exp(-coef[0] * (ub + coef[2])));
                    const double da = 0.5 * coef[1] * coef[0] * sa * (1.0 - sa);   /* d e_a / d f(x) = d e_a / d f(x + r_a) */
                    const double db = 0.5 * coef[1] * coef[0] * sb * (1.0 - sb);
                    if (role == 0) d = da * eb + ea * db;
                    if (role == 1) d = da * eb;
                    if (role == 2) d = ea * db;
                }
                acc += G[k] * d;
            }
        }
        g[y] += acc / (double)N;
    }
}
