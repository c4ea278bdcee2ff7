/*
 * bemrat.h -- C ABI of libbemrat.so: the node sweep of the contour / Chebyshev rational
 * approximation method for boundary-element acoustic eigenproblems T(kappa) x = 0
 * (El-Guide, Miedlar, Saad, arXiv 1906.03938), on AMD Instinct MI355X (gfx950).
 *
 * The operator.  T(kappa) is the single-layer Helmholtz operator of a closed surface made
 * of n flat triangles, discretised by piecewise-constant collocation at the centroids
 * x_a (paper, Section 1: Green's function, eq. GreenFun; the matrix T(z) of
 * eq. NEVPHelmholtz for a Dirichlet problem):
 *     T_ab(kappa) = sum_{q<7} A_b w_q exp(i kappa r)/(4 pi r),  r = |x_a - y_bq|  (a != b)
 *     T_aa(kappa) = integral over triangle a of exp(i kappa |x_a - y|)/(4 pi |x_a - y|)
 * where (y_bq, w_q) is Radon's degree-5 seven-point rule mapped to triangle b and A_b its
 * area; the self term is integrated exactly (polar coordinates around x_a).  kappa may be
 * complex.  Entries are regenerated on the device for every use and never stored.
 *
 * Conventions shared by every entry point:
 *   - complex numbers are interleaved (re, im) pairs of double, the layout of
 *     std::complex<double>, C99 double _Complex and torch.complex128;
 *   - pointers marked [host] are host memory read (or written) before the call returns;
 *     every other array pointer is device memory owned by the caller;
 *   - matrices are row-major; "ld" arguments are row strides in complex elements;
 *   - calls are asynchronous on the given stream (0 = the null stream); host-side
 *     argument checks happen before anything is launched, and an argument error launches
 *     nothing;
 *   - results are bitwise reproducible for identical inputs on the same device (fixed
 *     reduction orders, no floating-point atomics);
 *   - a mesh handle owns its device geometry and a workspace that grows on demand (the
 *     first call of a given size may allocate device memory); one handle must not be
 *     used from two host threads or on two streams concurrently;
 *   - no C++ exception crosses this interface; on failure bem_last_error() describes the
 *     most recent error of the calling thread.
 */
#ifndef BEMRAT_H
#define BEMRAT_H

#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct bem_mesh *bem_mesh_t;
typedef struct bem_batch *bem_batch_t;

typedef enum {
    BEM_OK = 0,
    BEM_EINVAL = 1,       /* bad argument: null pointer, size <= 0, ld < m, non-finite value */
    BEM_EMESH = 2,        /* bad mesh: index out of range, degenerate (zero-area) triangle */
    BEM_ENOMEM = 3,       /* device allocation failed */
    BEM_EDEVICE = 4,      /* HIP runtime or kernel error */
    BEM_EUNSUPPORTED = 5  /* option not built (e.g. a reduced-precision flag) */
} bem_status;

/* Sweep forms, passed in `flags`.
 *   BEM_FORM_DIRECT: one regenerated operator per node, T(z_j) V for every node.
 *   BEM_FORM_EXPAND: T(z) = sum_l t^l T_l with t = (z - c)/R about the centre c and
 *     radius R of the node set (Taylor expansion of exp(i z r) in z; for cheb_moments the
 *     nodes are the real Chebyshev points, c = (a+b)/2, R ~ (b-a)/2); the library
 *     generates L coefficient operators, truncated where the remainder bound falls below
 *     1e-14 relative to the smallest kernel value at the nodes, and recombines them per
 *     node or weight set.
 *   BEM_FORM_CHEB: for node sets on the real axis only: T(alpha + beta xi) =
 *     sum_l eps_l i^l T_l(xi) B_l with alpha, beta the centre and half-width of the nodes
 *     and B_l the operators of the Chebyshev (Jacobi-Anger) expansion of exp(i kappa r),
 *     entries w/r exp(i alpha r) J_l(beta r); truncated where the tail bound falls below
 *     1e-14 (|T_l| <= 1 on the interval, so recombination does not amplify errors).
 *     Complex nodes return BEM_EUNSUPPORTED.
 *   BEM_FORM_AUTO: the form with the fewest generated operators among those that apply
 *     (CHEB before EXPAND before DIRECT on ties).
 * Bits 4..7 select the arithmetic:
 *   BEM_PREC_F64 (0): FP64 throughout.
 *   BEM_PREC_F32, BEM_PREC_BF16, BEM_PREC_F16: operator entries generated in FP64, scaled
 *     and rounded to FP32 / BF16 / FP16 together with the probe block, contracted on the
 *     matrix cores with FP32 accumulation; the self terms (diagonal) are added in FP64
 *     afterwards; expansion lengths follow the looser tolerance of the type.  With these,
 *     BEM_FORM_AUTO takes CHEB for real node sets and DIRECT otherwise (EXPAND amplifies
 *     rounding errors by up to e^{2 R diam} on complex nodes and is used only on request).
 *     Results are accurate to about the unit roundoff of the type (see the tests for
 *     the tolerances), not to FP64.
 *   Other values return BEM_EUNSUPPORTED. */
#define BEM_FORM_AUTO 0u
#define BEM_FORM_DIRECT 1u
#define BEM_FORM_EXPAND 2u
#define BEM_FORM_CHEB 3u
#define BEM_FORM_MASK 3u
#define BEM_PREC_MASK 0xF0u
#define BEM_PREC_F64 0x00u
#define BEM_PREC_F32 0x10u
#define BEM_PREC_BF16 0x20u
#define BEM_PREC_F16 0x30u

/* ---------------------------------------------------------------- mesh handle --- */

/* Creates a mesh handle: uploads the surface, builds centroids, areas and quadrature
 * points on the device (sweep step "geometry staging").  xyz [host]: nv x 3 vertex
 * coordinates; tri [host]: n x 3 vertex indices (0-based).  Synchronises `stream` once
 * (to check triangle areas).  Errors: BEM_EINVAL (null pointers, nv < 3, n < 1,
 * non-finite coordinates), BEM_EMESH (index outside [0, nv), zero-area triangle),
 * BEM_ENOMEM, BEM_EDEVICE.  On error *out is set to NULL. */
bem_status bem_mesh_create(const double *xyz, int64_t nv, const int32_t *tri, int64_t n,
                           hipStream_t stream, bem_mesh_t *out);

/* Releases the handle and all its device memory (synchronises the device first).
 * NULL is accepted. */
void bem_mesh_destroy(bem_mesh_t mesh);

/* Number of triangles (= degrees of freedom) of the mesh, or -1 for NULL. */
int64_t bem_mesh_size(bem_mesh_t mesh);

/* Geometry as built on the device, copied to host arrays (any may be NULL):
 * area [host] n, centroid [host] n x 3, quad_xyz [host] n x 7 x 3,
 * quad_w [host] n x 7 physical weights A_b w_q.  Synchronises `stream`. */
bem_status bem_mesh_geometry(bem_mesh_t mesh, double *area, double *centroid,
                             double *quad_xyz, double *quad_w, hipStream_t stream);

/* ------------------------------------------------------------ nodes, weights --- */

/* Trapezoidal rule for the Cauchy integral (paper, eq. Tz and eq. TzApp) on the circle
 * |z - c| = radius with N nodes z_j = c + radius e^{i theta_j}, theta_j = 2 pi (j + 1/2)/N,
 * and weights w_j = -(z_j - c)/N so that T(z) ~ sum_j w_j T(z_j)/(z - z_j).  If P > 0
 * also writes the moment weights W[j][p] = w_j (z_j - shift)^{-(p+1)}, p < P, which turn
 * the node sweep into the blocks sum_j B_j (z_j - shift)^{-(p+1)}, B_j = w_j T(z_j), of one
 * inverse-power step (Algorithm 1).  z, w [host]: N complex; W [host]: N x P complex
 * (may be NULL when P == 0).  Errors: BEM_EINVAL (N < 1, radius <= 0, P < 0, null
 * outputs, a node equal to the shift). */
bem_status bem_contour_nodes(double c_re, double c_im, double radius, int64_t N,
                             double shift_re, double shift_im, int64_t P,
                             double *z, double *w, double *W);

/* First-kind Chebyshev points on [a, b] (paper, eq. Chebyshev) kappa_k = alpha + beta
 * cos(pi (k + 1/2)/N), alpha = (a+b)/2, beta = (b-a)/2, and the DCT-II matrix
 * coef[l][k] = (eps_l/N) cos(pi l (k + 1/2)/N), eps_0 = 1, eps_l = 2, of the degree N-1
 * interpolant sum_l C_l T_l((kappa - alpha)/beta).  kappa [host]: N doubles;
 * coef [host]: N x N doubles (may be NULL).  Errors: BEM_EINVAL (N < 1, a >= b). */
bem_status bem_cheb_nodes(double a, double b, int64_t N, double *kappa, double *coef);

/* ----------------------------------------------------------------- the sweep --- */

/* Self terms S[k][a] = T_aa(kappa_k) (the exact singular integral over triangle a, see
 * above), for nk wavenumbers.  kappa [host]: nk complex; S: device, nk x n complex,
 * contiguous.  Errors: BEM_EINVAL (null, nk < 1, non-finite kappa), BEM_EDEVICE. */
bem_status bem_self_terms(bem_mesh_t mesh, const double *kappa, int64_t nk, double *S,
                          hipStream_t stream);

/* Y[k] = T(kappa_k) V for k < nk: the operator regenerated at each wavenumber and
 * applied to the probe block (paper, the products with B_i of Example 3).
 * kappa [host]: nk complex.  V: device, n x m complex, row stride ldv >= m.
 * Y: device, nk blocks of n x m complex; block k starts at Y + 2*k*n*ldy doubles, row
 * stride ldy >= m.  flags: BEM_FORM_DIRECT (AUTO means DIRECT here).
 * Errors: BEM_EINVAL, BEM_EUNSUPPORTED, BEM_ENOMEM, BEM_EDEVICE. */
bem_status bem_assemble_apply(bem_mesh_t mesh, const double *kappa, int64_t nk,
                              const double *V, int64_t m, int64_t ldv, double *Y, int64_t ldy,
                              uint32_t flags, hipStream_t stream);

/* Contour moments M[p] = sum_j W[j][p] T(z_j) V, p < P (paper, eq. TzApp with
 * B_j = w_j T(z_j), folded with the per-node weights of eq. linsyssim; with
 * W[j][0] = w_j/(z_j - c) the sum is -S V, S = T~(c) the Schur complement).
 * z [host]: N complex nodes; W [host]: N x P complex.  V: device n x m (ldv >= m).
 * M: device, P blocks of n x m; block p starts at M + 2*p*n*ldm doubles, row stride
 * ldm >= m.  The EXPAND form generates only the Taylor operators the weight sets reach
 * (those whose largest possible contribution exceeds the expansion's truncation tolerance
 * times the largest term of some set; moment weights of a circle about its centre reach one
 * operator per order).  In FP64 with at most four weight sets and the DIRECT or EXPAND form,
 * the sweep folds the weights into the generated entries and contracts only the P
 * combinations (same sums, different rounding order); otherwise every generated operator is
 * contracted and the results recombined.  Errors: BEM_EINVAL, BEM_EUNSUPPORTED, BEM_ENOMEM,
 * BEM_EDEVICE. */
bem_status contour_moments(bem_mesh_t mesh, const double *z, int64_t N, const double *W,
                           int64_t P, const double *V, int64_t m, int64_t ldv, double *M,
                           int64_t ldm, uint32_t flags, hipStream_t stream);

/* contour_moments for callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same arguments, results
 * and kernels as contour_moments, but every piece of device workspace (parameter block, self
 * terms, probe copy, folded diagonal, generated products) is taken from the library's static
 * scratch array of 128 MiB per device instead of the handle's buffers, and nothing is
 * allocated (no hipMalloc, hipFree or allocating library routine; the parameter block is
 * staged through the handle's pinned buffer of 1 MiB, sized when the handle was created).
 * Sizes whose workspace exceeds the array (e.g. n = 81920 with m = 64 in the folded form needs
 * about 212 MB) or whose parameter block exceeds the staging buffer return BEM_EINVAL and
 * launch nothing.  All calls of this entry point on one GPU share that GPU's array, which keeps
 * the last call's contents: calls that overlap in time on one device (two streams, two host
 * threads) race and must be avoided by the caller.  Errors: those of contour_moments. */
bem_status contour_moments_noalloc(bem_mesh_t mesh, const double *z, int64_t N, const double *W,
                                   int64_t P, const double *V, int64_t m, int64_t ldv, double *M,
                                   int64_t ldm, uint32_t flags, hipStream_t stream);

/* Chebyshev coefficient blocks C[l] = sum_k coef[l][k] T(kappa_k) V, l < L <= N, on the
 * first-kind points of [a, b] (paper, eq. Chebyshev; nodes and coef as in
 * bem_cheb_nodes).  a < b real.  flags: BEM_FORM_* as for contour_moments.  V: device n x m (ldv >= m).  C: device, L blocks of
 * n x m, block l at C + 2*l*n*ldc doubles, row stride ldc >= m.
 * Errors: BEM_EINVAL, BEM_EUNSUPPORTED, BEM_ENOMEM, BEM_EDEVICE. */
bem_status cheb_moments(bem_mesh_t mesh, double a, double b, int64_t N, int64_t L,
                        const double *V, int64_t m, int64_t ldv, double *C, int64_t ldc,
                        uint32_t flags, hipStream_t stream);

/* Rayleigh-Ritz projections Pout[j] = U^H T(z_j) U, j < N, each m x m row-major
 * contiguous (paper, Section 3: B^_j = w_j U^H T(z_j) U), optionally fused with the
 * moments M[p] = sum_j W[j][p] T(z_j) U, p < Pw, of the same sweep (W [host] N x Pw, M
 * device with row stride ldm >= m; pass W = NULL, Pw = 0, M = NULL to skip them; in the
 * EXPAND form the moments combine the Taylor operators their weights reach, as
 * contour_moments does, although the projections take them all).
 * z [host]: N complex.  U: device n x m (ldu >= m).  Pout: device, N x m x m complex.
 * Errors: BEM_EINVAL, BEM_EUNSUPPORTED, BEM_ENOMEM, BEM_EDEVICE. */
bem_status rr_project(bem_mesh_t mesh, const double *z, int64_t N, const double *U,
                      int64_t m, int64_t ldu, double *Pout, const double *W, int64_t Pw,
                      double *M, int64_t ldm, uint32_t flags, hipStream_t stream);

/* Near-field quadrature (a refinement of the operator's discretisation, not a step of the
 * paper's method: the same boundary integral of Section 1, eq. GreenFun, evaluated more
 * accurately where the 7-point rule is poor).  A pair (a, b), a != b, is near when
 * |x_a - x_b|^2 < (eta*eta) h_b^2, with x the triangle centroids ((P0 + P1) + P2)/3 and h_b
 * the longest edge of triangle b, all formed in that order without fused multiply-adds.
 * For near pairs the corrected operator uses the integral of g(|x_a - y|) over triangle b
 * (semi-analytic: polar form around the foot of x_a on the plane of b, radial part in closed
 * form, angular part by sinh-transformed Gauss-Legendre panels of 16 or 10 points; accurate to about
 * 1e-14 relative while |kappa| h_b <~ 2) in place of the 7-point value.
 *
 * bem_mesh_set_nearfield builds the near-pair list of the mesh on the host and uploads it
 * (a set-up call: synchronises the device).  eta = 0 removes it; 0 <= eta <= 16, else
 * BEM_EINVAL.  Errors: BEM_EINVAL, BEM_ENOMEM, BEM_EDEVICE. */
bem_status bem_mesh_set_nearfield(bem_mesh_t mesh, double eta);

/* The near-pair list: *pairs = its length; rowptr [host, n + 1 entries, may be NULL] and col
 * [host, *pairs entries, may be NULL]: row a lists its near b in increasing order at
 * col[rowptr[a] .. rowptr[a+1]).  Synchronous.  Errors: BEM_EINVAL, BEM_EDEVICE. */
bem_status bem_mesh_nearfield(bem_mesh_t mesh, int64_t *pairs, int64_t *rowptr, int32_t *col);

/* How the near-field calls below evaluate the corrections of a node set.
 * BEM_NF_AUTO (the default): when x = max_j |z_j| R_max is small enough that x^L e^x / L! <=
 * 1e-17 for some L in {12, 16, 24, 32} (R_max a bound on the distance from a pair's target to
 * any point of its triangle, fixed by the list), each pair's correction is expanded as the
 * power series dT_ab(kappa) = sum_{n<L} c_n (i kappa)^n -- the closed-form radial integral
 * int e^{i kappa r} dr of the polar form and each 7-point term e^{i kappa r}/r expanded term by
 * term, over the same angular points -- and folded with the weights' moments
 * sum_j W[j][p] (i z_j)^n: one pass over the pairs per call instead of one per node; the
 * result equals the per-node evaluation to rounding (the truncation is below 1e-17 relative).
 * Otherwise, and with BEM_NF_NODES always, every pair is integrated at every node.
 * Errors: BEM_EINVAL (mesh NULL, mode not one of these). */
#define BEM_NF_AUTO 0
#define BEM_NF_NODES 1
bem_status bem_mesh_set_nearfield_mode(bem_mesh_t mesh, int mode);

/* Series length L the last near-field call on the mesh used (0: per node, or no call yet).
 * Errors: BEM_EINVAL. */
bem_status bem_nearfield_last_terms(bem_mesh_t mesh, int *terms);

/* Adds the near-field correction to moments of the 7-point operator:
 *   M[p] += sum_j W[j][p] dT(z_j) V,  p < P,
 * dT(z) = (near-field operator - 7-point operator) at z, nonzero only on the near pairs, so
 * contour_moments followed by this call gives the moments of the corrected operator (the
 * same sums with W[j][p] = delta_jp give T(z_j) V).  Arguments and layout as for
 * contour_moments (z, W [host]; V, M device; block p at M + 2*p*n*ldm doubles); M is read
 * and written.  Without a near-pair list M is left unchanged.  Each entry dT_ab(z_j) (or its
 * series, bem_mesh_set_nearfield_mode) is generated on the device per call; results are
 * deterministic.  Errors: BEM_EINVAL,
 * BEM_ENOMEM, BEM_EDEVICE. */
bem_status bem_nearfield_moments(bem_mesh_t mesh, const double *z, int64_t N, const double *W,
                                 int64_t P, const double *V, int64_t m, int64_t ldv, double *M,
                                 int64_t ldm, hipStream_t stream);

/* Adds the near-field correction to a dense node combination: S[a][b] += sum_j c_j
 * dT_ab(z_j) for every near pair (a, b) of the mesh's list, so that bem_assemble_sum followed
 * by this call gives sum_j c_j T(z_j) of the corrected operator (the matrix the inverse
 * iteration solves with).  z, c [host]: N complex.  S: device, n x lds complex (lds >= n), read
 * and written.  Without a near-pair list S is left unchanged.  Errors: BEM_EINVAL, BEM_ENOMEM,
 * BEM_EDEVICE. */
bem_status bem_nearfield_sum(bem_mesh_t mesh, const double *z, int64_t N, const double *c, double *S,
                             int64_t lds, hipStream_t stream);

/* Dense node combination S = sum_j c_j T(z_j), n x n row-major (row stride lds >= n): the
 * matrix the inverse iteration solves with -- for the Cauchy form the Schur complement
 * S = sum_j w_j T(z_j)/(z_j - s) of the linearisation at the shift s (paper, eq. sc2-sc5:
 * c_j = W[j][0] of bem_contour_nodes), for the Chebyshev form G = sum_l B_l T_l(s) (c_j the
 * DCT weights times T_l(s), summed over l).  Each entry is generated once on the device
 * from the same operators as the sweep (flags: BEM_FORM_* as for contour_moments, FP64
 * only), so S V equals contour_moments with the weights c to rounding.  z, c [host]: N
 * complex.  S: device, n x lds complex.  Timed by bem_set_timing like a sweep.  Errors:
 * BEM_EINVAL, BEM_EUNSUPPORTED (reduced precision, CHEB on complex nodes), BEM_ENOMEM,
 * BEM_EDEVICE. */
bem_status bem_assemble_sum(bem_mesh_t mesh, const double *z, int64_t N, const double *c, double *S,
                            int64_t lds, uint32_t flags, hipStream_t stream);

/* ------------------------------------------------- learned near-field correction --- */

/* A surrogate for the near-field quadrature (not a step of the paper's method): a perceptron
 * with three hidden layers of 128 tanh units maps a near pair's source triangle, target point
 * and wavenumber to the correction dT = (integral of g over the triangle) - (its 7-point value),
 * trained on the GPU by the kernels below on triples labelled by bem_nf_labels; the quadrature
 * of bem_nearfield_moments stays the fallback outside the network's trust region and its reference.
 *
 * Inputs (19, padded to BEM_NET_INPUTS floats per row): in the unit frame of the source
 * triangle (its longest edge A -> B on the x axis, the first longest of P0P1, P1P2, P2P0;
 * lengths divided by h = |B - A|; third vertex C = (p, q), q > 0; mirrored across u = 1/2 when
 * p > 1/2) the target is (u, v, w), and the inputs are (p - 0.25)/0.25, (q - 0.5)/0.4,
 * (u - 0.5)/1.5, (v - 0.3)/1.5, |w|, 2 Re(kappa h) - 1, Im(kappa h)/0.3, r0 - 1, 0.5/r0,
 * 0.3/r_k (k < 7), 0.5/s_k (k < 3); r0 is the distance to the centroid, r_k to the points of
 * Radon's rule (centroid; barycentric weight (9 - 2 sqrt 15)/21 on A, B, C; weight
 * (9 + 2 sqrt 15)/21 on A, B, C), s_k to A, B, C.  The outputs y (2) give
 * dT = h (S_re y_0 + i S_im y_1) / (4 pi r0^4), S the model's output scales.
 * Parameters: BEM_NET_PARAMS floats (device), row-major out x in: W1 [128 x 32] (input columns
 * 19..31 unused), b1 [128], W2 [128 x 128], b2, W3 [128 x 128], b3, W4 [2 x 128], b4 [2]. */
#define BEM_NET_PARAMS 37506
#define BEM_NET_INPUTS 32
#define BEM_NET_BINS 8

/* Number of network parameters (BEM_NET_PARAMS), for binding checks. */
int64_t bem_net_params(void);

/* Training labels from the library's near-field quadrature: out[s] = (integral over triangle
 * P9[s] of g(|x[s] - y|), g(r) = exp(i kappa[s] r)/(4 pi r)) - (Radon's 7-point value of the same
 * integral), s < S.  P9: device S x 9 doubles (three vertices); x: device S x 3; kappa, out:
 * device S complex.  The integral is the polar form of bem_nearfield_moments (accurate to about
 * 1e-14 relative while |kappa| h <~ 2).  Errors: BEM_EINVAL, BEM_EDEVICE. */
bem_status bem_nf_labels(const double *P9, const double *x, const double *kappa, int64_t S, double *out,
                         hipStream_t stream);

/* Network inputs of the triples (P9[s], x[s], kappa[s]): X device S x BEM_NET_INPUTS floats
 * (columns 19.. zero), aux device S x 4 doubles (h, r0, Re kappa h, Im kappa h).
 * Errors: BEM_EINVAL, BEM_EDEVICE. */
bem_status bem_net_features(const double *P9, const double *x, const double *kappa, int64_t S, float *X,
                            double *aux, hipStream_t stream);

/* FP32 forward pass of B rows of inputs X (device B x BEM_NET_INPUTS): Y device B x 2.
 * Errors: BEM_EINVAL, BEM_EDEVICE. */
bem_status bem_net_forward(const float *params, const float *X, int64_t B, float *Y, hipStream_t stream);

/* Device workspace (floats) bem_net_gradient needs for a batch of B rows; -1 if B < 1. */
int64_t bem_net_work_floats(int64_t B);

/* Loss (1/B) sum_b sum_o (Y_bo - T_bo)^2 of the batch (targets T device B x 2) and its gradient
 * with respect to the parameters, by back-propagation on the FP32 matrix cores: grad device
 * BEM_NET_PARAMS floats, loss device 1 float, work device bem_net_work_floats(B) floats (caller
 * owned; the call allocates nothing).  Per-tile gradients are summed in a fixed order: results
 * are bitwise reproducible.  Errors: BEM_EINVAL, BEM_EDEVICE. */
bem_status bem_net_gradient(const float *params, const float *X, const float *T, int64_t B, float *work,
                            float *grad, float *loss, hipStream_t stream);

/* One Adam update (Kingma and Ba, 2015; beta1 0.9, beta2 0.999, eps 1e-8) of the parameters
 * with gradient grad and moment estimates m, v (all device BEM_NET_PARAMS floats), step >= 1
 * (bias corrections 1 - beta^step), learning rate lr > 0.  Errors: BEM_EINVAL, BEM_EDEVICE. */
bem_status bem_net_adam(float *params, const float *grad, float *m, float *v, int64_t step, double lr,
                        hipStream_t stream);

/* A trained network and its trust region: pairs whose target lies at least dmin (in units of
 * the source triangle's longest edge h) from the triangle, whose triangle has every angle at
 * least min_angle_deg, with max_j |Re kappa_j| h <= kh_re_max, max_j |Im kappa_j| h <= kh_im_max,
 * every Re kappa_j >= 0, and whose distance falls in a bin [bin_edges[i], bin_edges[i+1]) with
 * bin_trusted[i] != 0, use the network; every other pair the quadrature.
 * freeze_tol: 0 evaluates the network at every node z_j.  A positive value evaluates it once
 * per pair, at the centre c of the nodes' bounding box, for the pairs (inside the region above)
 * with s k h^2 <= freeze_tol, s = max_j |z_j - c|, k = max_j |z_j|: the correction is then
 * dT(c) at every node (dT depends on kappa only through the 7-point rule's error on the
 * smooth part of the kernel, so s k h^2 estimates its relative change over the nodes), and it
 * folds as dT(c) sum_j W[j][p]; the other pairs take the quadrature.  One evaluation per pair
 * instead of one per node. */
typedef struct {
    const float *params;               /* device, BEM_NET_PARAMS floats */
    double out_scale[2];               /* S_re, S_im */
    double dmin, min_angle_deg, kh_re_max, kh_im_max;
    double bin_edges[BEM_NET_BINS + 1];
    int bin_trusted[BEM_NET_BINS];
    double freeze_tol;
} bem_net_model;

/* As bem_nearfield_moments, with the corrections of the pairs inside the model's trust region
 * taken from the network (FP16 on the matrix cores, FP32 accumulation; accurate to the model's
 * validation error, not to FP64) and the others from the quadrature:
 *   M[p] += sum_j W[j][p] dT(z_j) V.
 * The network's corrections of a pair are folded with the weights in FP64, the pairs are
 * applied in a fixed order: results are deterministic.  fallback_pairs [host, may be NULL]:
 * receives the number of pairs the quadrature handled (the call then synchronises `stream`).
 * Workspace (packed FP16 weights, one folded correction per pair and weight set, one flag per
 * pair) is the handle's, allocated on first use of a size.  Errors: BEM_EINVAL, BEM_ENOMEM,
 * BEM_EDEVICE. */
bem_status bem_nearfield_moments_net(bem_mesh_t mesh, const bem_net_model *model, const double *z, int64_t N,
                                     const double *W, int64_t P, const double *V, int64_t m, int64_t ldv,
                                     double *M, int64_t ldm, int64_t *fallback_pairs, hipStream_t stream);

/* Near-field corrections of the Rayleigh-Ritz projections (paper, Section 3, B^_j = U^H B_j U):
 *   Pout[j] += U^H dT(z_j) U,  j < N <= 4096,
 * dT the mesh's near-field correction (the quadrature when model is NULL; else the model's
 * network inside its trust region and the quadrature outside), so rr_project followed by this
 * call gives the projections of the corrected operator.  The per-node corrections dT(z_j) U are
 * formed in the handle's workspace (N x n x m complex, allocated on first use of a size) and
 * projected with rr_project's fixed-order reduction.  z [host]: N complex.  U: device n x m
 * (ldu >= m).  Pout: device N x m x m, read and written.  Without a near-pair list Pout is left
 * unchanged.  Errors: BEM_EINVAL, BEM_ENOMEM, BEM_EDEVICE. */
bem_status bem_nearfield_project(bem_mesh_t mesh, const bem_net_model *model, const double *z, int64_t N,
                                 const double *U, int64_t m, int64_t ldu, double *Pout, hipStream_t stream);

/* ------------------------------------------------------------- batched form --- */

/* A batch of meshes, each with its own node set and moment weights, whose contour moments
 * M_i[p] = sum_j W_i[j][p] T_i(z_ij) V_i (as contour_moments, per mesh i) are computed by
 * one persistent generate-and-contract launch over every mesh's tiles (work items taken
 * from a device queue, longest first), followed by the per-mesh recombination.
 * meshes [host]: count handles on the current device (they must outlive the batch and keep
 * their geometry; the batch holds its own self terms and workspace, so calls on a mesh
 * handle do not disturb it).  z [host]: count x N complex (row i = nodes of mesh i).
 * W [host]: count x N x P complex.  m: probe columns of every mesh.  flags: BEM_FORM_AUTO,
 * BEM_FORM_DIRECT or BEM_FORM_EXPAND with any BEM_PREC_*; one form serves the whole batch
 * (AUTO in FP64: EXPAND when every mesh admits it and it generates fewer operator entries in
 * total, else DIRECT; AUTO at reduced precision: DIRECT); BEM_FORM_CHEB returns
 * BEM_EUNSUPPORTED.  At reduced precision each mesh's probe block is scaled by its own
 * largest modulus and its self terms are added in FP64, as in the per-mesh calls.
 * tune != 0: the column tile (16 to 64 columns in FP64, 16 to 128 at reduced precision, at
 * most what m fills) is chosen by timing the persistent launch on an even sample of the
 * batch's own work; tune == 0 takes the per-call sweep's rule.  Computes every self term, uploads the parameter table and
 * the work list, and synchronises `stream`; all device memory of the batch is allocated
 * here.  Errors: BEM_EINVAL (null or non-finite arguments, a mesh on another device),
 * BEM_EUNSUPPORTED, BEM_ENOMEM, BEM_EDEVICE.  On error *out is NULL. */
bem_status bem_batch_create(const bem_mesh_t *meshes, int64_t count, const double *z, int64_t N,
                            const double *W, int64_t P, int64_t m, uint32_t flags, int tune,
                            hipStream_t stream, bem_batch_t *out);

/* Releases the batch and its device memory (synchronises the device first); NULL is
 * accepted.  The meshes are not released. */
void bem_batch_destroy(bem_batch_t batch);

/* Layout of the packed blocks (any output may be NULL): rows [host] count + 1 offsets, mesh
 * i owning packed rows rows[i] .. rows[i+1]-1 (rows[i+1] - rows[i] = its triangle count);
 * operators [host] count generated operators per mesh; *form the form in use
 * (BEM_FORM_DIRECT or BEM_FORM_EXPAND); *col_tile the probe columns per tile. */
bem_status bem_batch_layout(bem_batch_t batch, int64_t *rows, int64_t *operators, uint32_t *form,
                            int *col_tile);

/* The batch's contour moments.  V: device, rows[count] x m complex, contiguous rows (mesh
 * i's probe block is rows rows[i] .. rows[i+1]-1).  M: device; mesh i's P blocks of
 * n_i x m (contiguous, row stride m) start at M + 2 * P * rows[i] * m doubles, block p of
 * it at + 2 * p * n_i * m more.  Launches kernels only (no allocation, no host
 * synchronisation, no memset), so the call may be captured into a HIP graph; the batch's
 * workspace is shared by its calls, which must not overlap in time (one stream at a
 * time).  Errors: BEM_EINVAL (null batch, V or M not device memory), BEM_EDEVICE. */
bem_status bem_batch_moments(bem_batch_t batch, const double *V, double *M, hipStream_t stream);

/* Timing of the persistent launch, as bem_set_timing / bem_last_kernel_ms for a mesh. */
bem_status bem_batch_set_timing(bem_batch_t batch, int on);
bem_status bem_batch_last_kernel_ms(bem_batch_t batch, float *ms);

/* ------------------------------------------------- dense LU of the inverse iteration --- */

/* Inverse iteration on the linearised Cauchy approximation (Section 3, eq. sc2-sc5, the
 * step of Algorithm 1) solves with one n x n matrix, the Schur complement S = M_1 (for the
 * Chebyshev form, the matrix G of its linearisation), factorised once: P S = L U with
 * partial (row) pivoting.  These calls factorise and solve with a dense complex matrix held
 * in device memory; every index is formed in 64 bits, so n is limited only by memory
 * (n = 81920 takes 107 GB).  Each is a sequence of kernel launches on `stream`; they
 * allocate nothing.  The pivot of column j is the row i >= j with the largest
 * |Re a_ij| + |Im a_ij| (LAPACK's zgetrf measure; ties to the smaller row).  The trailing
 * updates run on the FP64 matrix cores (Gauss's three-multiplication complex product), so L
 * and U agree with zgetrf's to rounding, with the same pivots except where two candidates
 * are within rounding of each other.  Results are bitwise reproducible. */

/* Device workspace in bytes of bem_lu_factor (m = 0) or of bem_lu_solve with m right-hand
 * sides; -1 if n < 1 or m < 0. */
int64_t bem_lu_work_bytes(int64_t n, int64_t m);

/* In-place factorisation of A (device, n x n, row stride lda >= n): on return the strictly
 * lower part holds L's multipliers, the upper part U.  ipiv (device, n int64): row ipiv[j]
 * (0-based, >= j) was swapped with row j at step j, LAPACK's order; perm (device, n int64):
 * their product, row i of P A is row perm[i] of A.  info (device, 1 int64) is set to 0, or
 * to j + 1 for the first column j without a nonzero finite pivot candidate (the matrix is
 * singular to working precision, or holds a NaN; U[j][j] is then that column's diagonal
 * value and the factorisation continues).  work: bem_lu_work_bytes(n, 0) bytes (device).
 * Errors: BEM_EINVAL (n < 1, lda < n, null or host pointers, work too small), BEM_EDEVICE. */
bem_status bem_lu_factor(double *A, int64_t n, int64_t lda, int64_t *ipiv, int64_t *perm, int64_t *info,
                         void *work, int64_t work_bytes, hipStream_t stream);

/* X = A^-1 B from the factors of bem_lu_factor (LU, lda, perm) for m right-hand sides:
 * B device n x m (row stride ldb >= m), X device n x m (row stride ldx >= m; must not
 * overlap B); the row permutation, then forward substitution with L and backward with U.
 * work: bem_lu_work_bytes(n, m) bytes (device).  A zero diagonal entry of U gives
 * non-finite values in X (check the factorisation's info).
 * Errors: BEM_EINVAL (sizes, strides, null or host pointers, work too small), BEM_EDEVICE. */
bem_status bem_lu_solve(const double *LU, int64_t n, int64_t lda, const int64_t *perm, const double *B, int64_t ldb,
                        double *X, int64_t ldx, int64_t m, void *work, int64_t work_bytes, hipStream_t stream);

/* Column-scaled sum of device blocks, out[r][c] = sum_{b < nb} coef[b][c] X_b[r][c], summed
 * in the order b = 0, 1, ... (Algorithm 1 in moment-recurrence form: the right-hand side of
 * each Schur-complement solve, S u = sum_i B_i v_i / d_i, is a sum of swept moment blocks
 * M_p a_1, plus on restarts the block (M_1 + R_lam) x times rho^j per column, Section 3.2).
 * blocks [host]: nb (1 <= nb <= 64) device pointers to n x m complex blocks of row stride
 * ldx >= m.  coef: device, nb x m complex (block b's factor for column c at coef[b*m + c]).
 * out: device n x m complex, row stride ldo >= m; it may be one of the blocks when
 * ldo == ldx, and must not otherwise overlap one.
 * Errors: BEM_EINVAL (sizes, strides, host pointers, overlap), BEM_EDEVICE. */
bem_status bem_block_combine(const double *const *blocks, int64_t nb, const double *coef, int64_t n, int64_t m,
                             int64_t ldx, double *out, int64_t ldo, hipStream_t stream);

/* ---------------------------------------------------------------- diagnostics --- */

/* Form the last sweep call on this handle used: BEM_FORM_DIRECT, BEM_FORM_EXPAND or
 * BEM_FORM_CHEB, and the number of generated operators (nodes for DIRECT, expansion terms
 * for EXPAND and CHEB).
 * Either output may be NULL.  Returns BEM_EINVAL for a NULL handle. */
bem_status bem_last_form(bem_mesh_t mesh, uint32_t *form, int64_t *operators);

/* Enables (on != 0) or disables timing of the generate-and-contract kernel: when on,
 * every sweep call records HIP events around that kernel on the call's stream. */
bem_status bem_set_timing(bem_mesh_t mesh, int on);

/* Device time in milliseconds of the generate-and-contract kernel of the most recent
 * timed sweep call (synchronises on its end event).  BEM_EINVAL if none was timed. */
bem_status bem_last_kernel_ms(bem_mesh_t mesh, float *ms);

/* Synchronises `stream` and reports any asynchronous device error as BEM_EDEVICE. */
bem_status bem_stream_status(hipStream_t stream);

/* Message describing the most recent error of the calling thread ("" if none). */
const char *bem_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* BEMRAT_H */
