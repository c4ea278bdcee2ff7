// Internal declarations shared by the HIP translation units of libbemrat.so.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace bemrat {

constexpr int kQuad = 7;        // points of the triangle rule
constexpr int kPad = 64;        // n is padded to a multiple of this on the device
constexpr int kSelfGL = 32;     // Gauss-Legendre points per edge for the self term
constexpr int kMaxTaylor = 96;  // largest expansion length supported

// Device geometry of one mesh (all arrays padded to n_pad entries).
struct DeviceMesh {
    int64_t n = 0, n_pad = 0;
    double4 *colloc = nullptr;  // n_pad: collocation point (centroid), w unused
    double4 *quad = nullptr;    // n_pad * 7: (x, y, z, A_b w_q / (4 pi)); pads have weight 0
    double *vtx = nullptr;      // n_pad * 9: vertex coordinates (self terms)
    double *area = nullptr;     // n_pad
    double *gl = nullptr;       // 2 * kSelfGL: Gauss-Legendre nodes then weights on [-1, 1]
};

// Generator of the coefficient operators of one sweep.  DirectSym is the direct form on node
// sets made of quadruples {x + iy, x - iy, x' + iy, x' - iy}, stored consecutively in that
// order: the four share one exp(-y r) (and its reciprocal) per quadrature point, and each
// conjugate pair one sincos.
enum class Gen : int { Direct = 0, Taylor = 1, Cheb = 2, DirectSym = 3 };

// Arithmetic of the contraction (bits 4..7 of the flags): FP64 throughout, or FP64
// generation with an FP32 / BF16 / FP16 matrix-core contraction and FP32 accumulation.
enum class Prec : int { F64 = 0, F32 = 1, BF16 = 2, F16 = 3 };

struct SweepArgs {
    const double4 *colloc;
    const double4 *quad;
    const double2 *self;  // L x n_pad: diagonal entry of each generated operator
    const double2 *V;     // caller's probe block (row stride ldv)
    int64_t ldv;
    const double2 *Vp2;   // zero-padded copy n_pad x m_pad
    int64_t m_pad;
    double2 *Z;           // operator l writes n x m block at Z + l * zstride, row stride ldz
    int64_t ldz, zstride;
    int64_t n, n_pad, m;
    int L;                // number of generated operators
    int decay;            // some wavenumber (Direct) or the centre (Taylor) has Im != 0
    // Direct: wavenumbers of the L nodes
    const double2 *kappa;
    // Taylor: exp(i (c + R t) r) = exp(i c r) sum_l (i R r t)^l / l!
    // Cheb:   exp(i (alpha + beta xi) r) = exp(i alpha r) sum_l eps_l i^l J_l(beta r) T_l(xi),
    //         alpha in c_re, beta in R
    double c_re, c_im, R;
    const double *inv_fact;  // 1/l!, l < kMaxTaylor
    const double *inv_int;   // 1/l, l < kMaxTaylor (entry 0 unused)
    int miller_M;            // Cheb: start index of the Bessel recurrence (multiple of 8)
    double a_scale;          // reduced precision: entries are scaled by this before rounding
    const unsigned long long *vmax;  // reduced precision: bits of max |V| (probe scale)
    // Folded form (the sweep contracts L folded operators sum_l fcoef[l][p] T_l, p < L, out of
    // Lgen generated ones; self then holds the folded diagonal)
    int Lgen;
    const double2 *fcoef;  // Lgen x L
};

// One mesh of the persistent batched sweep: its arguments (the operator family, a
// BatchVariant, is common to the launch; `variant` records it per mesh for checking).
enum BatchVariant : int {
    kBatchDirectDecay = 0,
    kBatchDirect = 1,
    kBatchTaylorDecay = 2,
    kBatchTaylor = 3,
    kBatchDirectSym = 4,  // Gen::DirectSym (complex nodes: always with decay)
};
struct BatchEntry {
    SweepArgs args;
    int variant;  // BatchVariant
    int pad_;
};

// Launchers (asynchronous on `stream`; return hipSuccess or the launch error).
hipError_t launch_prepare_mesh(const double *xyz, const int32_t *tri, int64_t n, int64_t n_pad,
                               DeviceMesh mesh, const double *rule, hipStream_t stream);
hipError_t launch_self_terms(const DeviceMesh &mesh, const double2 *kappa, int64_t nk,
                             double2 *S, int64_t lds, hipStream_t stream);
hipError_t launch_sweep(Gen gen, const SweepArgs &args, hipStream_t stream);
// Reduced-precision sweep (diagonal entries zero) and the FP64 diagonal pass that completes it.
hipError_t launch_sweep_lp(Prec prec, Gen gen, const SweepArgs &args, hipStream_t stream);
hipError_t launch_absmax(const double2 *V, int64_t ldv, int64_t n, int64_t m, unsigned long long *out,
                         hipStream_t stream);
hipError_t launch_add_diag(const double2 *S, int64_t n_pad, const double2 *V, int64_t ldv, double2 *Z, int64_t ldz,
                           int64_t zstride, int64_t n, int64_t m, int L, hipStream_t stream);
int sweep_lp_ops_per_block(Gen gen, int64_t m);
int64_t sweep_lp_m_pad(int64_t m);  // column padding of the probe copy for the reduced-precision sweep
// Folded FP64 sweep for the moments of Direct or Taylor plans: the producer generates all
// args.Lgen operators of each entry and folds them into args.L <= kFoldMax combinations,
// the consumers contract only those and write them to args.Z like operators.  The fold
// runs at the width KL = fold_width(args.L) (1, 2 or 4) over args.fcoef, Lgen rows of KL
// (zero from column L on), at most kFoldCoef entries: the block keeps them in LDS.  For
// Taylor plans fcoef[l][k] carries the operator's own factor i^l / l! (the generator folds
// the plain power sums sum_q y_q x_q^l).
constexpr int kFoldMax = 4;
constexpr int kFoldCoef = 512;
constexpr int fold_width(int P) { return P <= 2 ? P : 4; }
hipError_t launch_sweep_fold(Gen gen, const SweepArgs &args, hipStream_t stream);

// Length unit of the expansion forms (their L is a multiple of it): 8.  The FP64 sweep
// generates 8 operators per block, or 16 for the expansion form up to 32 columns.
int sweep_ops_per_block(Gen gen, int64_t m);
int batch_ops_per_item_f64(Gen gen, int cb);  // the same for a batched work item of cb column groups
// Persistent batched FP64 sweep: clears `counter` (a kernel, not a memset), then `grid` blocks
// take the `nitems` items (mesh, row block, column block, operator block) of `table` meshes,
// all of operator family `variant`.
// cb = 16-column groups per tile (1, 2 or 4; batch_col_tile(m) is the per-call kernel's choice).
hipError_t launch_sweep_batch(int variant, int cb, const BatchEntry *table, const int4 *items, int nitems,
                              unsigned *counter, int grid, hipStream_t stream);
int batch_variant(Gen gen, bool decay);  // BatchVariant of an operator family, -1 if none
// Folded batch (FP64, P <= kFoldBatchMax = 4 weight sets per mesh, fold width fold_width(P)):
// items (mesh, row block, column block, 0); each mesh's args carry L = P, Lgen, fcoef (Lgen
// rows of the fold width, at most kFoldCoef entries) and its folded diagonal in self, and the
// folds land in its Z like operators.
constexpr int kFoldBatchMax = 4;
hipError_t launch_sweep_fold_batch(int variant, int cb, int P, const BatchEntry *table, const int4 *items, int nitems,
                                   unsigned *counter, int grid, hipStream_t stream);
// The same at reduced precision (each table entry carries its mesh's a_scale and probe-scale
// pointer); cb = 1, 2, 4 or 8 16-column groups, operators per item lp_batch_ops_per_block.
hipError_t launch_sweep_lp_batch(Prec prec, int variant, int cb, const BatchEntry *table, const int4 *items,
                                 int nitems, unsigned *counter, int grid, hipStream_t stream);
int lp_batch_col_tile(int64_t m);              // the per-call reduced-precision column rule
int lp_batch_ops_per_block(Gen gen, int cb);   // operators per work item
int batch_col_tile(int64_t m);
// Column padding of the probe copy the sweep reads (a multiple of its column tile).
int64_t sweep_m_pad(int64_t m);
hipError_t launch_prep_probe(const double2 *V, int64_t ldv, int64_t n, int64_t m, int64_t n_pad, int64_t m_pad,
                             double2 *Vp2, hipStream_t stream);
hipError_t launch_combine(const double2 *Z, int64_t zstride, int64_t ldz, int L,
                          const double2 *coef, int P, int64_t n, int64_t m, double2 *out,
                          int64_t ldo, hipStream_t stream);
// Dense S[a][b] = sum_l d[l] T_l[a][b] (a != b), S[a][a] = sum_l d[l] self_l[a], for the
// plan's generated operators (row stride lds); operators are generated in blocks of
// assemble_ops_per_block(), so the plan's L must be a multiple of it for the expansion forms.
hipError_t launch_assemble_sum(Gen gen, const SweepArgs &p, const double2 *d, double2 *S, int64_t lds,
                               hipStream_t stream);
int assemble_ops_per_block();
hipError_t launch_coef_dft(const double2 *samples, int64_t n_pad, int K, const double2 *F,
                           int L, double2 *out, hipStream_t stream);
hipError_t launch_project_partial(const double2 *U, int64_t ldu, const double2 *Z,
                                  int64_t zstride, int64_t ldz, int L, int64_t n, int64_t m,
                                  int64_t rows_per_chunk, int nchunks, double2 *partial,
                                  hipStream_t stream);
hipError_t launch_project_finish(const double2 *partial, int nchunks, int L, int64_t m,
                                 const double2 *coef, int N, double2 *out,
                                 hipStream_t stream, bool accumulate = false);
// out[l] += sum over the chunks of partial[l] (the projections U^H Z_l themselves, added)
hipError_t launch_project_add(const double2 *partial, int nchunks, int L, int64_t m, double2 *out,
                              hipStream_t stream);

// Near-field correction (nearfield.hip): M[p0 + p][a, :] += sum_j W[j][p0 + p] sum_{b in
// row a of (rowptr, col)} (integral - 7-point value of T_ab(kappa_j)) V[b, :], p < P <= kNfFold;
// one workgroup per row of the mesh.  gl16: 16-point Gauss-Legendre nodes then weights,
// followed by the 10-point rule's nodes then weights.  With S non-null (and P = 1) the folded
// corrections are added to the dense matrix S (row stride lds) instead: S[a][b] += sum_j
// W[j][p0] dT_ab(kappa_j); V and M are then unused.
constexpr int kNfFold = 8;
hipError_t launch_nearfield(const DeviceMesh &mesh, const double *gl16, const int64_t *rowptr,
                            const int32_t *col, const double2 *kappa, int N, const double2 *W, int Pstride,
                            int p0, int P, double kmax, const double2 *V, int64_t ldv, int64_t m,
                            double2 *M, int64_t ldm, double2 *S, int64_t lds, const int *nodes, int nnodes,
                            hipStream_t stream);

// Near-field fold mode: the corrections of the pairs k with flag[k] != 0 only, folded with
// weight columns p0 .. p0 + P - 1 and written to F[k * Pstride + p0 + p] (F pairs x Pstride).
// nodes (device, nnodes entries) lists the nodes with a nonzero weight in those columns (all N
// when null); launch_nearfield takes the same list.
hipError_t launch_nearfield_fold(const DeviceMesh &mesh, const double *gl16, const int64_t *rowptr,
                                 const int32_t *col, const unsigned char *flag, const double2 *kappa, int N,
                                 const double2 *W, int Pstride, int p0, int P, double kmax, double2 *F,
                                 const int *nodes, int nnodes, hipStream_t stream);
// Series form of the near-field corrections: for each pair k (row[k], col[k]) with flag[k] != 0
// (every pair when flag is null), F[k * Fstride + p0 + p] = sum_{n<L} c_n mu[n * P + p], p < P,
// c_n the coefficients of dT_ab(kappa) = sum_n c_n (i kappa)^n and mu[n][p] = sum_j W[j][p]
// (i kappa_j)^n (device, L x P); kmax sets the angular panels as in launch_nearfield.
// L in {12, 16, 24, 32}.  nf_series_terms(x): the smallest of these with x^L e^x / L! <= 1e-17
// for x = kappa_max R_max, or 0 when none is (then the per-node kernel is used).
int nf_series_terms(double x);
hipError_t launch_nearfield_series(const DeviceMesh &mesh, const double *gl16, const int32_t *row, const int32_t *col,
                                   int64_t npairs, const unsigned char *flag, double kmax, const double2 *mu, int L,
                                   int P, double2 *F, int Fstride, int p0, hipStream_t stream);
// S[row[k]][col[k]] += F[k], k < npairs (dense mode of the series form).
hipError_t launch_pair_dense_add(const int32_t *row, const int32_t *col, const double2 *F, int64_t npairs, double2 *S,
                                 int64_t lds, hipStream_t stream);
// Labels of the learned correction: out[s] = integral - 7-point value of triangle P9[s] (9
// doubles) at target x[s] (3 doubles) and wavenumber kappa[s]; gl52 the 16- and 10-point
// Gauss-Legendre rules (nodes then weights of each), rule28 Radon's rule (3 barycentric weights
// and the weight, per point).  Host pointers gl52 and rule28 are read before the call returns.
hipError_t launch_nf_labels(const double *P9, const double *x, const double2 *kappa, int64_t S, double2 *out,
                            const double *gl52, const double *rule28, hipStream_t stream);

// The learned near-field correction (nfnet.hip): a perceptron 19 -> 128 -> 128 -> 128 -> 2
// (tanh), FP32 parameters in one array (W1 [128 x 32], b1, W2 [128 x 128], b2, W3, b3,
// W4 [2 x 128], b4).
constexpr int kNetHidden = 128, kNetIn = 19, kNetInPad = 32, kNetOut = 2;
constexpr int64_t kNetParams = (int64_t)kNetHidden * kNetInPad + kNetHidden +
                               2 * ((int64_t)kNetHidden * kNetHidden + kNetHidden) + (int64_t)kNetOut * kNetHidden +
                               kNetOut;
constexpr int kNetBins = 8;   // distance bins of the trust region
constexpr int kNetMaxP = 2;   // weight sets per fold launch (the host loops over chunks)
hipError_t launch_net_features(const double *P9, const double *x, const double2 *kappa, int64_t S, float *X, double *aux,
                               hipStream_t stream);
int64_t net_slots(int64_t B);  // gradient slots of a batch of B samples
hipError_t launch_net_forward(const float *params, const float *X, int64_t B, float *Y, hipStream_t stream);
hipError_t launch_net_gradient(const float *params, const float *X, const float *T, int64_t B, float *partial,
                               float *loss_part, float *grad, float *loss, hipStream_t stream);
hipError_t launch_net_adam(float *params, const float *grad, float *m, float *v, float lr, float beta1, float beta2,
                           float eps, float c1, float c2, hipStream_t stream);
int64_t net_frag_bytes();
hipError_t launch_net_pack(const float *params, void *frag, hipStream_t stream);
struct NetFoldParams {
    const DeviceMesh *mesh;
    const int64_t *rowptr;
    const int32_t *col;
    int64_t npairs;
    const double2 *kappa;
    int N;
    const double2 *W;  // N x Pstride; this launch folds columns p0 .. p0 + P - 1 (P <= kNetMaxP) into F
    int Pstride, p0, P;
    const void *frag;
    const float *params;
    double S_re, S_im;
    double dmin, tan_min, kh_re_max, kh_im_max, kre_max, kim_max;
    double bin_edges[kNetBins + 1];
    int bin_ok[kNetBins];
    double2 *F;
    unsigned char *flag;
    const int *nodes;  // nodes with a nonzero weight in this launch's columns (all N when null)
    int nnodes;
    // frozen wavenumber (Wsum non-null): one evaluation per pair at kc, for pairs with
    // h^2 <= h2max, folded with Wsum[p] = sum_j W[j][p] for every p < P (any P)
    const double2 *Wsum;
    double2 kc;
    double h2max;
};
hipError_t launch_net_fold(const NetFoldParams &q, hipStream_t stream);
// M[p][a, :] += sum over the pairs k of row a of F[k * P + p] V[col[k], :], p < P (block p at
// M + p * n * ldm; launched in chunks of kNfFold sets, one wave per row).
hipError_t launch_pair_apply(const DeviceMesh &mesh, const int64_t *rowptr, const int32_t *col, const double2 *F, int P,
                             const double2 *V, int64_t ldv, int64_t m, double2 *M, int64_t ldm, hipStream_t stream);

// Dense complex LU with partial pivoting and its solves (lu.hip).
int64_t lu_factor_work_bytes();
int64_t lu_solve_work_bytes(int64_t n, int64_t m);
hipError_t lu_factor(double2 *A, int64_t n, int64_t lda, int64_t *ipiv, int64_t *perm, int64_t *info, void *work,
                     hipStream_t stream);
hipError_t lu_solve(const double2 *LU, int64_t n, int64_t lda, const int64_t *perm, const double2 *B, int64_t ldb,
                    double2 *X, int64_t ldx, int64_t m, void *work, hipStream_t stream);

// Static device scratch array of the allocation-free entry point (scratch.hip): 128 MiB per
// device.  scratch_region returns the current device's copy (its address is looked up once per
// device) and its size.
constexpr size_t kScratchBytes = size_t(128) << 20;
hipError_t scratch_region(void **ptr, size_t *bytes);

}  // namespace bemrat
