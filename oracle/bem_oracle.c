/*
 * bem_oracle.c -- plain, slow, FP64 CPU oracle for the discretised single-layer
 * Helmholtz boundary operator T(k) whose node sweep the library accelerates.
 *
 * TEST INFRASTRUCTURE.  Only the tests, the smoke check and the benchmark's CPU
 * baseline leg load this library; the product path never does.  It shares no code,
 * header, table or constant with the HIP implementation.
 *
 * What it computes (all complex values interleaved re,im; all arithmetic FP64):
 *
 *   Kernel: the free-space Green's function g(r) = exp(i k r)/(4 pi r) of the Helmholtz
 *   equation (paper, Section 1, eq. GreenFun), with complex wavenumber k.
 *
 *   Discretisation (the operator T(z) of eq. NEVPHelmholtz specialised to a Dirichlet
 *   problem, single layer, piecewise-constant collocation at triangle centroids):
 *     T_ab(k) = sum_{q<7} A_b w_q g(|x_a - y_bq|)               (a != b)
 *     T_aa(k) = integral over triangle a of g(|x_a - y|) dA_y     (exact, polar form)
 *   with x_a the centroid of triangle a, A_b the area of triangle b and (y_bq, w_q) the
 *   degree-5 seven-point rule of Radon (1948) mapped to triangle b.
 *
 *   Self term in polar coordinates around the centroid: for each edge e at distance d_e
 *   from x_a, with the angle phi measured from the foot of the perpendicular,
 *     T_aa(k) = 1/(4 pi) sum_e int_{phi_e-}^{phi_e+} F(k, d_e/cos(phi)) dphi,
 *     F(k, rho) = int_0^rho exp(i k t) dt = (exp(i k rho) - 1)/(i k).
 *   The deriv argument d (>= 0) returns the d-th derivative in k instead: the kernel
 *   becomes (i r)^d g(r) and F becomes int_0^rho (i t)^d exp(i k t) dt.
 *
 *   The angular integral is evaluated by composite Gauss-Legendre quadrature whose panel
 *   count is doubled until two successive values agree to 1e-15 relative.
 */
#include <complex.h>
#include <float.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef double complex cplx;

static const double PI = 3.14159265358979323846264338327950288;

/* ---------------------------------------------------------------- quadrature --- */

/* Radon's 7-point degree-5 rule on a triangle: barycentric points and weights that sum
 * to one (Stroud 1971, T2:5-1).  Centroid weight 9/40; two orbits of three points
 * (a1,b1,b1) and (a2,b2,b2) with a = (9 -+ 2 sqrt 15)/21, b = (6 +- sqrt 15)/21 and
 * weights (155 +- sqrt 15)/1200. */
void or_radon7(double *bary, double *w)
{
    const double s = sqrt(15.0);
    const double a1 = (9.0 - 2.0 * s) / 21.0, b1 = (6.0 + s) / 21.0;
    const double a2 = (9.0 + 2.0 * s) / 21.0, b2 = (6.0 - s) / 21.0;
    const double w1 = (155.0 + s) / 1200.0, w2 = (155.0 - s) / 1200.0;
    const double pts[7][3] = {
        {1.0 / 3.0, 1.0 / 3.0, 1.0 / 3.0},
        {a1, b1, b1}, {b1, a1, b1}, {b1, b1, a1},
        {a2, b2, b2}, {b2, a2, b2}, {b2, b2, a2},
    };
    const double ww[7] = {9.0 / 40.0, w1, w1, w1, w2, w2, w2};
    for (int q = 0; q < 7; ++q) {
        for (int c = 0; c < 3; ++c) bary[3 * q + c] = pts[q][c];
        w[q] = ww[q];
    }
}

/* Gauss-Legendre nodes and weights on [-1,1]: roots of P_n found by Newton's method on
 * the three-term Legendre recurrence, weights 2/((1-x^2) P_n'(x)^2). */
void or_gauss_legendre(int n, double *x, double *w)
{
    for (int i = 0; i < (n + 1) / 2; ++i) {
        double z = cos(PI * (i + 0.75) / (n + 0.5)), z1, pp;
        do {
            double p1 = 1.0, p2 = 0.0;
            for (int j = 1; j <= n; ++j) {
                double p3 = p2;
                p2 = p1;
                p1 = ((2.0 * j - 1.0) * z * p2 - (j - 1.0) * p3) / j;
            }
            pp = n * (z * p1 - p2) / (z * z - 1.0);
            z1 = z;
            z = z1 - p1 / pp;
        } while (fabs(z - z1) > 1e-15);
        {
            double p1 = 1.0, p2 = 0.0;
            for (int j = 1; j <= n; ++j) {
                double p3 = p2;
                p2 = p1;
                p1 = ((2.0 * j - 1.0) * z * p2 - (j - 1.0) * p3) / j;
            }
            pp = n * (z * p1 - p2) / (z * z - 1.0);
        }
        x[i] = -z;
        x[n - 1 - i] = z;
        w[i] = w[n - 1 - i] = 2.0 / ((1.0 - z * z) * pp * pp);
    }
}

/* ------------------------------------------------------------------ geometry --- */

typedef struct {
    int64_t n;
    double *cen;  /* n x 3 centroids (collocation points) */
    double *area; /* n */
    double *qp;   /* n x 7 x 3 quadrature points */
    double *qw;   /* n x 7 physical weights A_b w_q */
    double *vtx;  /* n x 9 vertex coordinates */
} geom_t;

static void geom_free(geom_t *g)
{
    free(g->cen); free(g->area); free(g->qp); free(g->qw); free(g->vtx);
}

/* Builds centroids, areas and mapped quadrature points.  Returns 0, or -1 on a bad
 * index, -2 on a degenerate (zero-area) triangle, -3 on allocation failure. */
static int geom_build(const double *xyz, int64_t nv, const int32_t *tri, int64_t n, geom_t *g)
{
    double bary[21], w[7];
    or_radon7(bary, w);
    g->n = n;
    g->cen = malloc(sizeof(double) * 3 * (size_t)n);
    g->area = malloc(sizeof(double) * (size_t)n);
    g->qp = malloc(sizeof(double) * 21 * (size_t)n);
    g->qw = malloc(sizeof(double) * 7 * (size_t)n);
    g->vtx = malloc(sizeof(double) * 9 * (size_t)n);
    if (!g->cen || !g->area || !g->qp || !g->qw || !g->vtx) { geom_free(g); return -3; }
    for (int64_t b = 0; b < n; ++b) {
        double P[3][3];
        for (int v = 0; v < 3; ++v) {
            int32_t id = tri[3 * b + v];
            if (id < 0 || id >= nv) { geom_free(g); return -1; }
            for (int c = 0; c < 3; ++c) P[v][c] = xyz[3 * id + c];
        }
        double e1[3], e2[3], cr[3];
        for (int c = 0; c < 3; ++c) { e1[c] = P[1][c] - P[0][c]; e2[c] = P[2][c] - P[0][c]; }
        cr[0] = e1[1] * e2[2] - e1[2] * e2[1];
        cr[1] = e1[2] * e2[0] - e1[0] * e2[2];
        cr[2] = e1[0] * e2[1] - e1[1] * e2[0];
        double A = 0.5 * sqrt(cr[0] * cr[0] + cr[1] * cr[1] + cr[2] * cr[2]);
        if (!(A > 0.0)) { geom_free(g); return -2; }
        g->area[b] = A;
        for (int c = 0; c < 3; ++c) {
            g->cen[3 * b + c] = (P[0][c] + P[1][c] + P[2][c]) / 3.0;
            for (int v = 0; v < 3; ++v) g->vtx[9 * b + 3 * v + c] = P[v][c];
        }
        for (int q = 0; q < 7; ++q) {
            for (int c = 0; c < 3; ++c)
                g->qp[21 * b + 3 * q + c] =
                    bary[3 * q] * P[0][c] + bary[3 * q + 1] * P[1][c] + bary[3 * q + 2] * P[2][c];
            g->qw[7 * b + q] = A * w[q];
        }
    }
    return 0;
}

int or_geometry(const double *xyz, int64_t nv, const int32_t *tri, int64_t n,
                double *area, double *cen, double *qp, double *qw)
{
    geom_t g;
    int rc = geom_build(xyz, nv, tri, n, &g);
    if (rc) return rc;
    memcpy(area, g.area, sizeof(double) * (size_t)n);
    memcpy(cen, g.cen, sizeof(double) * 3 * (size_t)n);
    memcpy(qp, g.qp, sizeof(double) * 21 * (size_t)n);
    memcpy(qw, g.qw, sizeof(double) * 7 * (size_t)n);
    geom_free(&g);
    return 0;
}

/* ----------------------------------------------------------------- self term --- */

/* J_d(w) = int_0^1 u^d exp(w u) du.  Power series sum_n w^n / (n! (n+d+1)) for small
 * |w| (no cancellation there); otherwise the integration-by-parts recursion
 * J_0 = (e^w - 1)/w, J_d = (e^w - d J_{d-1})/w, which is stable for |w| > d. */
static cplx jmoment(cplx w, int d)
{
    double aw = cabs(w);
    if (aw <= 2.0 || aw <= (double)d) {
        cplx term = 1.0, sum = 0.0;
        for (int k = 0; k < 200; ++k) {
            cplx t = term / (double)(k + d + 1);
            sum += t;
            if (cabs(t) < 1e-20 * cabs(sum) && k > 2) break;
            term *= w / (double)(k + 1);
        }
        return sum;
    }
    cplx ew = cexp(w);
    cplx j = (ew - 1.0) / w;
    for (int k = 1; k <= d; ++k) j = (ew - (double)k * j) / w;
    return j;
}

/* F_d(k, rho) = int_0^rho (i t)^d exp(i k t) dt = i^d rho^(d+1) J_d(i k rho). */
static cplx radial(cplx k, double rho, int d)
{
    cplx id = 1.0;
    for (int j = 0; j < d; ++j) id *= I;
    return id * pow(rho, d + 1) * jmoment(I * k * rho, d);
}

#define GL_ORDER 16
static double gl_x[GL_ORDER], gl_w[GL_ORDER];
static int gl_ready = 0;

static void gl_init(void)
{
    if (!gl_ready) {
        or_gauss_legendre(GL_ORDER, gl_x, gl_w);
        gl_ready = 1;
    }
}

/* int_{p0}^{p1} F_d(k, dist/cos(phi)) dphi on `panels` equal panels. */
static cplx edge_panels(cplx k, double dist, double p0, double p1, int d, int panels)
{
    cplx s = 0.0;
    double h = (p1 - p0) / panels;
    for (int p = 0; p < panels; ++p) {
        double lo = p0 + p * h, mid = lo + 0.5 * h;
        for (int i = 0; i < GL_ORDER; ++i) {
            double phi = mid + 0.5 * h * gl_x[i];
            s += (0.5 * h * gl_w[i]) * radial(k, dist / cos(phi), d);
        }
    }
    return s;
}

static cplx self_term_tri(const double P[3][3], cplx k, int d)
{
    double x[3];
    for (int c = 0; c < 3; ++c) x[c] = (P[0][c] + P[1][c] + P[2][c]) / 3.0;
    cplx total = 0.0;
    for (int e = 0; e < 3; ++e) {
        const double *A = P[e], *B = P[(e + 1) % 3];
        double t[3], len = 0.0;
        for (int c = 0; c < 3; ++c) { t[c] = B[c] - A[c]; len += t[c] * t[c]; }
        len = sqrt(len);
        for (int c = 0; c < 3; ++c) t[c] /= len;
        double s = 0.0; /* (x - A).t */
        for (int c = 0; c < 3; ++c) s += (x[c] - A[c]) * t[c];
        double foot2 = 0.0;
        for (int c = 0; c < 3; ++c) {
            double f = A[c] + s * t[c] - x[c];
            foot2 += f * f;
        }
        double dist = sqrt(foot2);
        double lminus = -s, lplus = len - s; /* tangential coordinates of A and B */
        double p0 = atan2(lminus, dist), p1 = atan2(lplus, dist);
        cplx prev = edge_panels(k, dist, p0, p1, d, 1), cur = prev;
        for (int panels = 2; panels <= 4096; panels *= 2) {
            cur = edge_panels(k, dist, p0, p1, d, panels);
            if (cabs(cur - prev) <= 1e-15 * cabs(cur)) break;
            prev = cur;
        }
        total += cur;
    }
    return total / (4.0 * PI);
}

/* Self term of one triangle P (9 doubles: three vertices) at wavenumber k, derivative
 * order d; result written to out[0..1]. */
void or_self_term_tri(const double *P9, double kr, double ki, int d, double *out)
{
    gl_init();
    double P[3][3];
    for (int v = 0; v < 3; ++v)
        for (int c = 0; c < 3; ++c) P[v][c] = P9[3 * v + c];
    cplx r = self_term_tri(P, kr + I * ki, d);
    out[0] = creal(r);
    out[1] = cimag(r);
}

/* ------------------------------------------------------------------- entries --- */

static cplx offdiag(const geom_t *g, int64_t a, int64_t b, cplx k, int d)
{
    const double *x = g->cen + 3 * a;
    cplx s = 0.0;
    for (int q = 0; q < 7; ++q) {
        const double *y = g->qp + 21 * b + 3 * q;
        double dx = x[0] - y[0], dy = x[1] - y[1], dz = x[2] - y[2];
        double r = sqrt(dx * dx + dy * dy + dz * dz);
        cplx kern = cexp(I * k * r) / (4.0 * PI * r);
        for (int j = 0; j < d; ++j) kern *= I * r;
        s += g->qw[7 * b + q] * kern;
    }
    return s;
}

static cplx entry(const geom_t *g, int64_t a, int64_t b, cplx k, int d)
{
    if (a != b) return offdiag(g, a, b, k, d);
    double P[3][3];
    for (int v = 0; v < 3; ++v)
        for (int c = 0; c < 3; ++c) P[v][c] = g->vtx[9 * a + 3 * v + c];
    return self_term_tri(P, k, d);
}

/* Self terms T_aa(kappa_j) for all triangles and nk wavenumbers: out is nk x n complex. */
int or_self_terms(const double *xyz, int64_t nv, const int32_t *tri, int64_t n,
                  const double *kappa, int64_t nk, int d, double *out)
{
    gl_init();
    geom_t g;
    int rc = geom_build(xyz, nv, tri, n, &g);
    if (rc) return rc;
#pragma omp parallel for schedule(dynamic, 16) collapse(2)
    for (int64_t j = 0; j < nk; ++j)
        for (int64_t a = 0; a < n; ++a) {
            cplx v = entry(&g, a, a, kappa[2 * j] + I * kappa[2 * j + 1], d);
            out[2 * (j * n + a)] = creal(v);
            out[2 * (j * n + a) + 1] = cimag(v);
        }
    geom_free(&g);
    return 0;
}

/* Dense T(k) (or its d-th derivative), n x n complex, row-major. For small n only. */
int or_dense(const double *xyz, int64_t nv, const int32_t *tri, int64_t n,
             double kr, double ki, int d, double *T)
{
    gl_init();
    geom_t g;
    int rc = geom_build(xyz, nv, tri, n, &g);
    if (rc) return rc;
    cplx k = kr + I * ki;
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t a = 0; a < n; ++a)
        for (int64_t b = 0; b < n; ++b) {
            cplx v = entry(&g, a, b, k, d);
            T[2 * (a * n + b)] = creal(v);
            T[2 * (a * n + b) + 1] = cimag(v);
        }
    geom_free(&g);
    return 0;
}

/* Neumaier's compensated summation step: adds x into (s, c). */
static inline void nsum(double *s, double *c, double x)
{
    double t = *s + x;
    if (fabs(*s) >= fabs(x)) *c += (*s - t) + x;
    else *c += (x - t) + *s;
    *s = t;
}

/* Matrix-free rows of Y = T(k) V: for each requested row a (rows[0..nrows)),
 * Y[i, :] = sum_b T_ab(k) V[b, :], summed in natural b order with Neumaier
 * compensation.  V is n x m complex with row stride ldv (complex elements); Y is
 * nrows x m complex, contiguous. */
int or_apply_rows(const double *xyz, int64_t nv, const int32_t *tri, int64_t n,
                  double kr, double ki, int d, const int64_t *rows, int64_t nrows,
                  const double *V, int64_t m, int64_t ldv, double *Y)
{
    gl_init();
    geom_t g;
    int rc = geom_build(xyz, nv, tri, n, &g);
    if (rc) return rc;
    for (int64_t i = 0; i < nrows; ++i)
        if (rows[i] < 0 || rows[i] >= n) { geom_free(&g); return -1; }
    cplx k = kr + I * ki;
    int bad = 0;
#pragma omp parallel
    {
        cplx *trow = malloc(sizeof(cplx) * (size_t)n);
        double *acc = malloc(sizeof(double) * 4 * (size_t)m);
        if (!trow || !acc) {
#pragma omp atomic write
            bad = 1;
        }
#pragma omp for schedule(dynamic, 1)
        for (int64_t i = 0; i < nrows; ++i) {
            if (!trow || !acc) continue;
            int64_t a = rows[i];
            for (int64_t b = 0; b < n; ++b) trow[b] = entry(&g, a, b, k, d);
            memset(acc, 0, sizeof(double) * 4 * (size_t)m);
            for (int64_t b = 0; b < n; ++b) {
                double tr = creal(trow[b]), ti = cimag(trow[b]);
                const double *v = V + 2 * b * ldv;
                for (int64_t c = 0; c < m; ++c) {
                    double vr = v[2 * c], vi = v[2 * c + 1];
                    nsum(&acc[4 * c], &acc[4 * c + 1], tr * vr);
                    nsum(&acc[4 * c], &acc[4 * c + 1], -ti * vi);
                    nsum(&acc[4 * c + 2], &acc[4 * c + 3], tr * vi);
                    nsum(&acc[4 * c + 2], &acc[4 * c + 3], ti * vr);
                }
            }
            for (int64_t c = 0; c < m; ++c) {
                Y[2 * (i * m + c)] = acc[4 * c] + acc[4 * c + 1];
                Y[2 * (i * m + c) + 1] = acc[4 * c + 2] + acc[4 * c + 3];
            }
        }
        free(trow);
        free(acc);
    }
    geom_free(&g);
    return bad ? -3 : 0;
}

/* ---------------------------------------------------------------- near field --- */
/*
 * Near-field quadrature: the entries T_ab, a != b, whose collocation point x_a is close
 * to triangle b are redefined as the integral itself,
 *     T_ab(k) = integral over triangle b of g(|x_a - y|) dA_y,
 * instead of its 7-point approximation (the same boundary integral of Section 1, eq.
 * GreenFun, that the 7-point rule approximates; the rule loses accuracy when x_a is
 * within a few triangle diameters of triangle b).  A pair (a, b), a != b, is near when
 *     |x_a - x_b|^2 < eta^2 h_b^2,
 * with h_b the longest edge of triangle b; every quantity in that test is formed in the
 * order written below (centroid ((P0 + P1) + P2)/3 per coordinate, squared lengths as
 * dx*dx + dy*dy + dz*dz, then (eta*eta)*h2), so the list is reproducible bit for bit.
 *
 * The integral is evaluated by adaptive cubature: a collapsed Gauss-Legendre product
 * rule (Stroud's conical product, 10 x 10 points, exact for polynomials of degree 18 on
 * the triangle) on a triangle and on its four midpoint children; where the two estimates
 * differ by more than the tolerance (an absolute bound, the relative tolerance times the
 * first estimate, the same at every level) the children are refined in turn.  All wavenumbers
 * share one refinement (the near-singularity at x_a does not depend on k), and the
 * acceptance test takes the largest difference over them.
 */

#define NQ_COLLAPSED 10
#define ADAPT_DEPTH 40

static double cq_x[NQ_COLLAPSED], cq_w[NQ_COLLAPSED];
static int cq_ready = 0;

static void cq_init(void)
{
    if (!cq_ready) {
        or_gauss_legendre(NQ_COLLAPSED, cq_x, cq_w);
        cq_ready = 1;
    }
}

/* Collapsed product rule on triangle (V0, V1, V2): y = V0 + s (V1 - V0) + t (V2 - V0) with
 * s = u (1 - v), t = u v on the unit square, dA = 2 A u du dv.  out[j] = sum of g over
 * the rule for wavenumber k[j]. */
static void collapsed_rule(const double x[3], const double V0[3], const double V1[3],
                           const double V2[3], const cplx *k, int nk, cplx *out)
{
    double e1[3], e2[3];
    for (int c = 0; c < 3; ++c) { e1[c] = V1[c] - V0[c]; e2[c] = V2[c] - V0[c]; }
    double cr0 = e1[1] * e2[2] - e1[2] * e2[1];
    double cr1 = e1[2] * e2[0] - e1[0] * e2[2];
    double cr2 = e1[0] * e2[1] - e1[1] * e2[0];
    double twoA = sqrt(cr0 * cr0 + cr1 * cr1 + cr2 * cr2);
    for (int j = 0; j < nk; ++j) out[j] = 0.0;
    for (int i = 0; i < NQ_COLLAPSED; ++i) {
        double u = 0.5 * (1.0 + cq_x[i]);
        for (int l = 0; l < NQ_COLLAPSED; ++l) {
            double v = 0.5 * (1.0 + cq_x[l]);
            double s = u * (1.0 - v), t = u * v;
            double w = twoA * u * 0.25 * cq_w[i] * cq_w[l];
            double dx = x[0] - (V0[0] + s * e1[0] + t * e2[0]);
            double dy = x[1] - (V0[1] + s * e1[1] + t * e2[1]);
            double dz = x[2] - (V0[2] + s * e1[2] + t * e2[2]);
            double r = sqrt(dx * dx + dy * dy + dz * dz);
            double wr = w / (4.0 * PI * r);
            for (int j = 0; j < nk; ++j) out[j] += wr * cexp(I * k[j] * r);
        }
    }
}

/* Refines triangle (V0, V1, V2) whose rule value is `whole`; adds the accepted value of
 * every leaf to acc.  work holds 5 nk complex values per remaining level. */
static void adapt_tri(const double x[3], const double V0[3], const double V1[3], const double V2[3],
                      const cplx *k, int nk, const cplx *whole, double tol, int depth, cplx *work,
                      cplx *acc)
{
    double m01[3], m12[3], m20[3];
    for (int c = 0; c < 3; ++c) {
        m01[c] = 0.5 * (V0[c] + V1[c]);
        m12[c] = 0.5 * (V1[c] + V2[c]);
        m20[c] = 0.5 * (V2[c] + V0[c]);
    }
    const double *ch[4][3] = {{V0, m01, m20}, {m01, V1, m12}, {m20, m12, V2}, {m01, m12, m20}};
    cplx *cv = work, *sum = work + 4 * nk;
    for (int q = 0; q < 4; ++q) collapsed_rule(x, ch[q][0], ch[q][1], ch[q][2], k, nk, cv + q * nk);
    double err = 0.0, mag = 0.0;
    for (int j = 0; j < nk; ++j) {
        sum[j] = cv[j] + cv[nk + j] + cv[2 * nk + j] + cv[3 * nk + j];
        double e = cabs(sum[j] - whole[j]);
        if (e > err) err = e;
        for (int q = 0; q < 4; ++q)
            if (cabs(cv[q * nk + j]) > mag) mag = cabs(cv[q * nk + j]);
    }
    /* accept below the tolerance, or once the difference is at the rounding level of the
     * children's own sums (further refinement cannot reduce it) */
    if (err <= tol || err <= 256.0 * DBL_EPSILON * mag || depth >= ADAPT_DEPTH) {
        for (int j = 0; j < nk; ++j) acc[j] += sum[j];
        return;
    }
    for (int q = 0; q < 4; ++q)
        adapt_tri(x, ch[q][0], ch[q][1], ch[q][2], k, nk, cv + q * nk, tol, depth + 1,
                  work + 5 * nk, acc);
}

/* Integral of g(|x - y|) over triangle P (9 doubles) for the nk wavenumbers k (interleaved
 * complex); out is nk complex.  The refinement stops where the children change the value
 * by at most rtol times the largest first estimate.  Returns 0 or -3 (allocation). */
int or_tri_integral(const double *x, const double *P9, const double *kappa, int64_t nk, double rtol,
                    double *out)
{
    cq_init();
    cplx *k = malloc(sizeof(cplx) * (size_t)(nk > 0 ? nk : 1));
    cplx *work = malloc(sizeof(cplx) * (size_t)(nk > 0 ? nk : 1) * (5 * (ADAPT_DEPTH + 1) + 2));
    if (!k || !work) { free(k); free(work); return -3; }
    for (int64_t j = 0; j < nk; ++j) k[j] = kappa[2 * j] + I * kappa[2 * j + 1];
    const double *V0 = P9, *V1 = P9 + 3, *V2 = P9 + 6;
    cplx *whole = work + 5 * (ADAPT_DEPTH + 1) * nk, *acc = whole + nk;
    collapsed_rule(x, V0, V1, V2, k, (int)nk, whole);
    double scale = 0.0;
    for (int64_t j = 0; j < nk; ++j) {
        acc[j] = 0.0;
        if (cabs(whole[j]) > scale) scale = cabs(whole[j]);
    }
    adapt_tri(x, V0, V1, V2, k, (int)nk, whole, rtol * scale, 0, work, acc);
    for (int64_t j = 0; j < nk; ++j) {
        out[2 * j] = creal(acc[j]);
        out[2 * j + 1] = cimag(acc[j]);
    }
    free(k);
    free(work);
    return 0;
}

/* Centroids and squared longest edges in the order stated above. */
static void near_geometry(const double *xyz, const int32_t *tri, int64_t n, double *cen, double *h2)
{
    for (int64_t b = 0; b < n; ++b) {
        const double *P[3];
        for (int v = 0; v < 3; ++v) P[v] = xyz + 3 * (int64_t)tri[3 * b + v];
        for (int c = 0; c < 3; ++c) cen[3 * b + c] = ((P[0][c] + P[1][c]) + P[2][c]) / 3.0;
        double best = 0.0;
        for (int e = 0; e < 3; ++e) {
            const double *A = P[e], *B = P[(e + 1) % 3];
            double dx = B[0] - A[0], dy = B[1] - A[1], dz = B[2] - A[2];
            double l2 = dx * dx + dy * dy + dz * dz;
            if (l2 > best) best = l2;
        }
        h2[b] = best;
    }
}

/* Near pairs by brute force over all (a, b): row a lists its near b in increasing order.
 * rowptr has n + 1 entries; col (capacity cap) may be NULL to count only.  Returns the
 * number of pairs, -1 on a bad index, -3 on allocation failure, -4 if cap is too small. */
int64_t or_near_pairs(const double *xyz, int64_t nv, const int32_t *tri, int64_t n, double eta,
                      int64_t *rowptr, int32_t *col, int64_t cap)
{
    for (int64_t i = 0; i < 3 * n; ++i)
        if (tri[i] < 0 || tri[i] >= nv) return -1;
    double *cen = malloc(sizeof(double) * 3 * (size_t)n), *h2 = malloc(sizeof(double) * (size_t)n);
    if (!cen || !h2) { free(cen); free(h2); return -3; }
    near_geometry(xyz, tri, n, cen, h2);
    int64_t count = 0;
    rowptr[0] = 0;
    for (int64_t a = 0; a < n; ++a) {
        for (int64_t b = 0; b < n; ++b) {
            if (b == a) continue;
            double dx = cen[3 * a] - cen[3 * b], dy = cen[3 * a + 1] - cen[3 * b + 1],
                   dz = cen[3 * a + 2] - cen[3 * b + 2];
            double d2 = dx * dx + dy * dy + dz * dz;
            if (d2 < eta * eta * h2[b]) {
                if (col) {
                    if (count >= cap) { free(cen); free(h2); return -4; }
                    col[count] = (int32_t)b;
                }
                ++count;
            }
        }
        rowptr[a + 1] = count;
    }
    free(cen);
    free(h2);
    return count;
}

/* Near-field corrections dT[j][i] = (integral - 7-point value) for pair i = (a, col[i]) of
 * the list (rowptr, col) and wavenumber kappa[j]; dT is nk x nnz complex.  rtol as in
 * or_tri_integral.  Returns 0, -1 (bad index or list), -3 (allocation). */
int or_nearfield_correction(const double *xyz, int64_t nv, const int32_t *tri, int64_t n,
                            const int64_t *rowptr, const int32_t *col, const double *kappa, int64_t nk,
                            double rtol, double *dT)
{
    geom_t g;
    int rc = geom_build(xyz, nv, tri, n, &g);
    if (rc) return rc;
    const int64_t nnz = rowptr[n];
    for (int64_t i = 0; i < nnz; ++i)
        if (col[i] < 0 || col[i] >= n) { geom_free(&g); return -1; }
    int bad = 0;
#pragma omp parallel
    {
        double *res = malloc(sizeof(double) * 2 * (size_t)(nk > 0 ? nk : 1));
#pragma omp for schedule(dynamic, 8)
        for (int64_t a = 0; a < n; ++a) {
            for (int64_t i = rowptr[a]; i < rowptr[a + 1]; ++i) {
                int64_t b = col[i];
                if (!res || b == a || or_tri_integral(g.cen + 3 * a, g.vtx + 9 * b, kappa, nk, rtol, res)) {
#pragma omp atomic write
                    bad = 1;
                    continue;
                }
                for (int64_t j = 0; j < nk; ++j) {
                    cplx seven = offdiag(&g, a, b, kappa[2 * j] + I * kappa[2 * j + 1], 0);
                    dT[2 * (j * nnz + i)] = res[2 * j] - creal(seven);
                    dT[2 * (j * nnz + i) + 1] = res[2 * j + 1] - cimag(seven);
                }
            }
        }
        free(res);
    }
    geom_free(&g);
    return bad ? -1 : 0;
}

int or_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
