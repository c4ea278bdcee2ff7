// Dense complex LU factorisation with partial (row) pivoting, P A = L U, and the solves with it,
// for the matrix that inverse iteration solves with: the Schur complement S = M_1 of the
// linearised Cauchy approximation (paper Section 3, eq. sc2-sc5), factorised once and used
// for every step.
//
// Storage: row-major, element (i, j) at A[i lda + j] (double2), every index formed in 64 bits,
// so n = 81920 (107 GB) is fine.  L is unit lower triangular (its multipliers below the
// diagonal), U upper triangular, both in place.  ipiv[j] (0-based) is the row swapped with
// row j at step j; perm is their product: row i of P A is row perm[i] of A.
//
// Factorisation (right-looking, two levels of blocking, the structure of LAPACK's getrf):
//   for each outer panel of kPanel = 256 columns k .. k + kb:
//     for each sub-panel of kSub = 32 columns s0 .. s1:
//       for each column j: the pivot is the largest |Re a_ij| + |Im a_ij| over rows i >= j
//       (LAPACK's izamax measure; ties to the smaller row; the search runs fused into the
//       previous column's elimination); rows j and ipiv[j] are swapped across the outer panel; rows i > j get
//       l_ij = a_ij / a_jj and a_ic -= l_ij a_jc for the sub-panel's columns c > j;
//       then the sub-panel's rows of the outer panel's remaining columns by forward
//       substitution, and the rows below by a complex GEMM with K = 32;
//     the panel's swaps are applied to every column outside it;
//     U12 = L11^-1 A12 by blocked forward substitution (32 rows at a time);
//     A22 -= L21 U12: complex GEMM with K = kb.
// The GEMM forms each complex product with Gauss's three real multiplications
// (P1 = Ar Br, P2 = Ai Bi, P3 = (Ar + Ai)(Br + Bi); Re = P1 - P2, Im = P3 - P1 - P2) on
// v_mfma_f64_16x16x4f64, through LDS in stages of 16 k with the next stage's global loads in
// flight during the current stage's MFMAs.
//
// Solves (forward with the unit lower L, then backward with U, 32 rows at a time): the rows'
// product with the solved part is a split-K MFMA GEMM into partial sums, and one kernel per
// 32-row block adds the partial sums and solves with the diagonal block (one thread per
// right-hand side column, the block in LDS).
#include <algorithm>

#include "internal.h"

namespace bemrat {

namespace {

typedef double v4d __attribute__((ext_vector_type(4)));

__device__ __forceinline__ v4d mfma(double a, double b, v4d c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

constexpr int kSub = 32;         // sub-panel width, triangular block size of the solves
constexpr int64_t kPanel = 256;  // outer panel width (the trailing GEMM's K)
constexpr int kStageK = 16;      // k per LDS stage of the GEMM
constexpr int kPivotBlocks = 1024;
constexpr int64_t kSolveChunk = 1024;  // split-K chunk of the solves

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

__device__ __forceinline__ double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }

// ------------------------------------------------------------------------ GEMM

struct ZgemmArgs {
    double2 *C;  // C -= A B (when part is null)
    int64_t ldc;
    const double2 *A;  // M x K
    int64_t lda;
    const double2 *B;  // K x N
    int64_t ldb;
    int64_t M, N, K;
    int64_t kchunk;  // k per blockIdx.z (K when not split)
    double2 *part;   // split-K: part[z][M][N] = A[:, chunk z] B[chunk z, :]
};

// One workgroup of 4 waves per BM x BN output tile (blockIdx.y, blockIdx.x) and k chunk
// (blockIdx.z); waves on a WGM x WGN grid, each owning TM x TN MFMA tiles of 16 x 16.
// MFMA operand layout: lane (ci = lane & 15, ck = lane >> 4) holds A[ci][ck] and B[ck][ci]; the
// result's register q holds row ck + 4 q, column ci.
template <int WGM, int WGN, int TM, int TN>
__global__ __launch_bounds__(256) void zgemm_kernel(ZgemmArgs g) {
    static_assert(WGM * WGN == 4, "4 waves");
    constexpr int BM = WGM * 16 * TM, BN = WGN * 16 * TN, KS = kStageK;
    constexpr int LA = BM * KS / 256, LB = KS * BN / 256;
    static_assert(LA * 256 == BM * KS && LB * 256 == KS * BN, "whole staging loads");
    __shared__ double2 sA[BM][KS + 1];
    __shared__ double2 sB[KS][BN];
    const int t = threadIdx.x, w = t >> 6, lane = t & 63, ci = lane & 15, ck = lane >> 4;
    const int wm = w / WGN, wn = w % WGN;
    const int64_t row0 = (int64_t)blockIdx.y * BM, col0 = (int64_t)blockIdx.x * BN;
    const int64_t ka = (int64_t)blockIdx.z * g.kchunk;
    const int64_t kz = ka + g.kchunk < g.K ? ka + g.kchunk : g.K;

    v4d P1[TM][TN], P2[TM][TN], P3[TM][TN];
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) P1[i][j] = P2[i][j] = P3[i][j] = v4d{0.0, 0.0, 0.0, 0.0};

    double2 ra[LA], rb[LB];
    auto load = [&](int64_t k0) {
#pragma unroll
        for (int l = 0; l < LA; ++l) {
            const int idx = t + 256 * l, r = idx / KS, kk = idx % KS;
            const int64_t gr = row0 + r, gk = k0 + kk;
            ra[l] = (gr < g.M && gk < kz) ? g.A[gr * g.lda + gk] : make_double2(0.0, 0.0);
        }
#pragma unroll
        for (int l = 0; l < LB; ++l) {
            const int idx = t + 256 * l, kk = idx / BN, c = idx % BN;
            const int64_t gk = k0 + kk, gc = col0 + c;
            rb[l] = (gk < kz && gc < g.N) ? g.B[gk * g.ldb + gc] : make_double2(0.0, 0.0);
        }
    };
    load(ka);
    for (int64_t k0 = ka; k0 < kz; k0 += KS) {
        __syncthreads();  // the previous stage's reads of sA, sB are done
#pragma unroll
        for (int l = 0; l < LA; ++l) {
            const int idx = t + 256 * l;
            sA[idx / KS][idx % KS] = ra[l];
        }
#pragma unroll
        for (int l = 0; l < LB; ++l) {
            const int idx = t + 256 * l;
            sB[idx / BN][idx % BN] = rb[l];
        }
        __syncthreads();
        if (k0 + KS < kz) load(k0 + KS);
#pragma unroll
        for (int ks = 0; ks < KS; ks += 4) {
            double ar[TM], ai[TM], as[TM], br[TN], bi[TN], bs[TN];
#pragma unroll
            for (int i = 0; i < TM; ++i) {
                const double2 a = sA[wm * 16 * TM + 16 * i + ci][ks + ck];
                ar[i] = a.x;
                ai[i] = a.y;
                as[i] = a.x + a.y;
            }
#pragma unroll
            for (int j = 0; j < TN; ++j) {
                const double2 b = sB[ks + ck][wn * 16 * TN + 16 * j + ci];
                br[j] = b.x;
                bi[j] = b.y;
                bs[j] = b.x + b.y;
            }
#pragma unroll
            for (int i = 0; i < TM; ++i)
#pragma unroll
                for (int j = 0; j < TN; ++j) {
                    P1[i][j] = mfma(ar[i], br[j], P1[i][j]);
                    P2[i][j] = mfma(ai[i], bi[j], P2[i][j]);
                    P3[i][j] = mfma(as[i], bs[j], P3[i][j]);
                }
        }
    }
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int64_t r = row0 + wm * 16 * TM + 16 * i + ck + 4 * q;
                const int64_t c = col0 + wn * 16 * TN + 16 * j + ci;
                if (r < g.M && c < g.N) {
                    const double p1 = P1[i][j][q], p2 = P2[i][j][q], p3 = P3[i][j][q];
                    const double2 v = make_double2(p1 - p2, p3 - p1 - p2);
                    if (g.part) {
                        g.part[((int64_t)blockIdx.z * g.M + r) * g.N + c] = v;
                    } else {
                        double2 &o = g.C[r * g.ldc + c];
                        o = csub(o, v);
                    }
                }
            }
}

// Trailing updates: 128 x 64 tiles, waves 2 x 2 of 64 x 32.
constexpr int kBigWGM = 2, kBigWGN = 2, kBigTM = 4, kBigTN = 2;
constexpr int kBigBM = kBigWGM * 16 * kBigTM, kBigBN = kBigWGN * 16 * kBigTN;
// Split-K products of the solves: 32 x 64 tiles, waves 2 x 2 of 16 x 32.
constexpr int kSolWGM = 2, kSolWGN = 2, kSolTM = 1, kSolTN = 2;
constexpr int kSolBM = kSolWGM * 16 * kSolTM, kSolBN = kSolWGN * 16 * kSolTN;
static_assert(kSolBM == kSub, "a solve block is one tile row");

hipError_t gemm_sub(double2 *C, int64_t ldc, const double2 *A, int64_t lda, const double2 *B, int64_t ldb, int64_t M,
                    int64_t N, int64_t K, hipStream_t s) {
    if (M <= 0 || N <= 0 || K <= 0) return hipSuccess;
    ZgemmArgs g{C, ldc, A, lda, B, ldb, M, N, K, K, nullptr};
    dim3 grid((unsigned)((N + kBigBN - 1) / kBigBN), (unsigned)((M + kBigBM - 1) / kBigBM), 1);
    hipLaunchKernelGGL((zgemm_kernel<kBigWGM, kBigWGN, kBigTM, kBigTN>), grid, dim3(256), 0, s, g);
    return hipGetLastError();
}

// part[z] = A[0:M, chunk z] B[chunk z, 0:N] for the kSolveChunk chunks of [0, K); M <= kSub.
hipError_t gemm_part(double2 *part, const double2 *A, int64_t lda, const double2 *B, int64_t ldb, int64_t M,
                     int64_t N, int64_t K, int nz, hipStream_t s) {
    ZgemmArgs g{nullptr, 0, A, lda, B, ldb, M, N, K, kSolveChunk, part};
    dim3 grid((unsigned)((N + kSolBN - 1) / kSolBN), 1, (unsigned)nz);
    hipLaunchKernelGGL((zgemm_kernel<kSolWGM, kSolWGN, kSolTM, kSolTN>), grid, dim3(256), 0, s, g);
    return hipGetLastError();
}

// --------------------------------------------------------------- pivoting

// Block reduction of (value, row) pairs to the largest value, ties to the smaller row; thread 0
// writes the block's pair.
__device__ void reduce_pivot(double v, int64_t r, double *sv, int64_t *sr, double *pval, int64_t *prow) {
    sv[threadIdx.x] = v;
    sr[threadIdx.x] = r;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
            const double v2 = sv[threadIdx.x + s];
            const int64_t r2 = sr[threadIdx.x + s];
            if (v2 > sv[threadIdx.x] || (v2 == sv[threadIdx.x] && r2 < sr[threadIdx.x])) {
                sv[threadIdx.x] = v2;
                sr[threadIdx.x] = r2;
            }
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        pval[blockIdx.x] = sv[0];
        prow[blockIdx.x] = sr[0];
    }
}

// Partial pivot search of column j over rows [j, n): per-block (largest |Re a_ij| + |Im a_ij|,
// row).  Rows
// without a finite value never win (a NaN compares false).
__global__ __launch_bounds__(256) void pivot_partial_kernel(const double2 *__restrict__ A, int64_t lda, int64_t n,
                                                            int64_t j, double *__restrict__ pval,
                                                            int64_t *__restrict__ prow) {
    __shared__ double sv[256];
    __shared__ int64_t sr[256];
    double best = -1.0;
    int64_t brow = n;
    for (int64_t i = j + (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
        const double2 a = A[i * lda + j];
        const double v = fabs(a.x) + fabs(a.y);
        if (v > best) {
            best = v;
            brow = i;
        }
    }
    reduce_pivot(best, brow, sv, sr, pval, prow);
}

// Final reduction of the nparts partials of column j, ipiv[j] = the pivot row, and the swap of
// rows j and ipiv[j] over columns [c0, c1) (one workgroup).  A column without a nonzero
// finite candidate keeps row j and records info = j + 1 (the first such column).
__global__ __launch_bounds__(256) void pivot_swap_kernel(double2 *__restrict__ A, int64_t lda, int64_t j,
                                                         const double *__restrict__ pval,
                                                         const int64_t *__restrict__ prow, int nparts,
                                                         int64_t *__restrict__ ipiv, int64_t c0, int64_t c1,
                                                         int64_t *__restrict__ info) {
    __shared__ double sv[256];
    __shared__ int64_t sr[256];
    __shared__ int64_t sp;
    double best = -1.0;
    int64_t r = j;
    for (int b = threadIdx.x; b < nparts; b += 256) {
        const double v = pval[b];
        const int64_t q = prow[b];
        if (v > best || (v == best && q < r)) {
            best = v;
            r = q;
        }
    }
    sv[threadIdx.x] = best;
    sr[threadIdx.x] = r;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
            const double v2 = sv[threadIdx.x + s];
            const int64_t r2 = sr[threadIdx.x + s];
            if (v2 > sv[threadIdx.x] || (v2 == sv[threadIdx.x] && r2 < sr[threadIdx.x])) {
                sv[threadIdx.x] = v2;
                sr[threadIdx.x] = r2;
            }
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        int64_t p = sr[0];
        if (!(sv[0] > 0.0)) {
            p = j;
            if (*info == 0) *info = j + 1;
        }
        ipiv[j] = p;
        sp = p;
    }
    __syncthreads();
    const int64_t p = sp;
    if (p == j) return;
    for (int64_t c = c0 + threadIdx.x; c < c1; c += 256) {
        const double2 x = A[j * lda + c], y = A[p * lda + c];
        A[j * lda + c] = y;
        A[p * lda + c] = x;
    }
}

// Elimination of column j within the sub-panel ending at column s1: rows i > j get
// l = a_ij / a_jj (stored in place) and a_ic -= l a_jc for j < c < s1.  Each 32-lane half-wave
// owns one row (lane = column offset from j, so a row's segment is one coalesced access);
// with search set, lane 1 also keeps the largest updated a_i,j+1 (same measure) and the block writes its
// partial pivot of column j + 1.
__global__ __launch_bounds__(256) void eliminate_kernel(double2 *__restrict__ A, int64_t lda, int64_t n, int64_t j,
                                                        int64_t s1, int search, double *__restrict__ pval,
                                                        int64_t *__restrict__ prow) {
    __shared__ double sv[256];
    __shared__ int64_t sr[256];
    const int lane = threadIdx.x & 31, grp = threadIdx.x >> 5;
    const int64_t c = j + lane;
    const bool col_ok = c < s1;
    const double2 piv = A[j * lda + j];
    const double den = piv.x * piv.x + piv.y * piv.y;
    const double2 inv = den > 0.0 ? make_double2(piv.x / den, -piv.y / den) : make_double2(0.0, 0.0);
    const double2 u = col_ok ? A[j * lda + c] : make_double2(0.0, 0.0);
    double best = -1.0;
    int64_t brow = n;
    for (int64_t i = j + 1 + (int64_t)blockIdx.x * 8 + grp; i < n; i += (int64_t)gridDim.x * 8) {
        double2 a = col_ok ? A[i * lda + c] : make_double2(0.0, 0.0);
        const double2 head = make_double2(__shfl(a.x, 0, 32), __shfl(a.y, 0, 32));
        const double2 l = cmul(head, inv);
        if (lane == 0) {
            A[i * lda + j] = l;
        } else if (col_ok) {
            a = csub(a, cmul(l, u));
            A[i * lda + c] = a;
            if (lane == 1) {
                const double v = fabs(a.x) + fabs(a.y);
                if (v > best) {
                    best = v;
                    brow = i;
                }
            }
        }
    }
    if (search) reduce_pivot(best, brow, sv, sr, pval, prow);
}

// Row swaps j <-> ipiv[j], j = k .. k + kb - 1 in order, on columns [0, k) and [k + kb, n), one
// thread per column; the thread after the last column applies them to perm.
__global__ __launch_bounds__(256) void laswp_kernel(double2 *__restrict__ A, int64_t lda, int64_t n, int64_t k,
                                                    int64_t kb, const int64_t *__restrict__ ipiv,
                                                    int64_t *__restrict__ perm) {
    const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t cols = n - kb;
    if (idx > cols) return;
    if (idx == cols) {
        for (int64_t j = k; j < k + kb; ++j) {
            const int64_t p = ipiv[j];
            const int64_t x = perm[j];
            perm[j] = perm[p];
            perm[p] = x;
        }
        return;
    }
    const int64_t c = idx < k ? idx : idx + kb;
    for (int64_t j = k; j < k + kb; ++j) {
        const int64_t p = ipiv[j];
        if (p != j) {
            const double2 x = A[j * lda + c], y = A[p * lda + c];
            A[j * lda + c] = y;
            A[p * lda + c] = x;
        }
    }
}

__global__ __launch_bounds__(256) void lu_init_kernel(int64_t *__restrict__ perm, int64_t n,
                                                      int64_t *__restrict__ info) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) perm[i] = i;
    if (i == 0) *info = 0;
}

// Forward substitution with the unit lower rb x rb block L (rb <= kSub) on rows 0 .. rb of B,
// columns [c0, c1): one thread per column, the block in LDS.  With part set, B's rows first
// lose the sum of the nz split-K partial products part[z][r][c - c0].
__global__ __launch_bounds__(256) void trsm_lower_kernel(const double2 *__restrict__ L, int64_t ldl,
                                                         double2 *__restrict__ B, int64_t ldb, int rb, int64_t c0,
                                                         int64_t c1, const double2 *__restrict__ part, int nz) {
    __shared__ double2 sL[kSub][kSub];
    for (int i = threadIdx.x; i < kSub * kSub; i += 256) {
        const int r = i / kSub, q = i % kSub;
        sL[r][q] = (r < rb && q < r) ? L[r * ldl + q] : make_double2(0.0, 0.0);
    }
    __syncthreads();
    const int64_t c = c0 + (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (c >= c1) return;
    const int64_t m = c1 - c0;
    double2 x[kSub];
#pragma unroll
    for (int r = 0; r < kSub; ++r) {
        x[r] = r < rb ? B[r * ldb + c] : make_double2(0.0, 0.0);
        if (part && r < rb)
            for (int z = 0; z < nz; ++z) x[r] = csub(x[r], part[((int64_t)z * rb + r) * m + (c - c0)]);
    }
#pragma unroll
    for (int r = 1; r < kSub; ++r) {
#pragma unroll
        for (int q = 0; q < r; ++q) x[r] = csub(x[r], cmul(sL[r][q], x[q]));
        if (r - 1 < rb) B[(r - 1) * ldb + c] = x[r - 1];
    }
    if (rb == kSub) B[(kSub - 1) * ldb + c] = x[kSub - 1];
}

// Backward substitution with the upper rb x rb block U (diagonal included, rb <= kSub) on rows
// 0 .. rb of B, columns [0, m), after subtracting the nz split-K partials (as above).
__global__ __launch_bounds__(256) void trsm_upper_kernel(const double2 *__restrict__ U, int64_t ldu,
                                                         double2 *__restrict__ B, int64_t ldb, int rb, int64_t m,
                                                         const double2 *__restrict__ part, int nz) {
    __shared__ double2 sU[kSub][kSub];
    for (int i = threadIdx.x; i < kSub * kSub; i += 256) {
        const int r = i / kSub, q = i % kSub;
        sU[r][q] = (r < rb && q < rb && q >= r) ? U[r * ldu + q] : make_double2(r == q ? 1.0 : 0.0, 0.0);
    }
    __syncthreads();
    const int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (c >= m) return;
    double2 x[kSub];
#pragma unroll
    for (int r = 0; r < kSub; ++r) {
        x[r] = r < rb ? B[r * ldb + c] : make_double2(0.0, 0.0);
        if (part && r < rb)
            for (int z = 0; z < nz; ++z) x[r] = csub(x[r], part[((int64_t)z * rb + r) * m + c]);
    }
#pragma unroll
    for (int r = kSub - 1; r >= 0; --r) {
#pragma unroll
        for (int q = r + 1; q < kSub; ++q) x[r] = csub(x[r], cmul(sU[r][q], x[q]));
        const double2 d = sU[r][r];
        const double den = d.x * d.x + d.y * d.y;
        x[r] = make_double2((x[r].x * d.x + x[r].y * d.y) / den, (x[r].y * d.x - x[r].x * d.y) / den);
    }
#pragma unroll
    for (int r = 0; r < kSub; ++r)
        if (r < rb) B[r * ldb + c] = x[r];
}

// X[i][c] = B[perm[i]][c]
__global__ __launch_bounds__(256) void permute_rows_kernel(const double2 *__restrict__ B, int64_t ldb,
                                                           const int64_t *__restrict__ perm, int64_t n, int64_t m,
                                                           double2 *__restrict__ X, int64_t ldx) {
    const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (idx >= n * m) return;
    const int64_t i = idx / m, c = idx % m;
    X[i * ldx + c] = B[perm[i] * ldb + c];
}

unsigned blocks(int64_t items) { return (unsigned)((items + 255) / 256); }

}  // namespace

int64_t lu_factor_work_bytes() { return kPivotBlocks * (int64_t)(sizeof(double) + sizeof(int64_t)); }

int64_t lu_solve_work_bytes(int64_t n, int64_t m) {
    const int64_t nz = (n + kSolveChunk - 1) / kSolveChunk;
    return nz * kSub * m * (int64_t)sizeof(double2);
}

hipError_t lu_factor(double2 *A, int64_t n, int64_t lda, int64_t *ipiv, int64_t *perm, int64_t *info, void *work,
                     hipStream_t s) {
    double *pval = static_cast<double *>(work);
    int64_t *prow = reinterpret_cast<int64_t *>(pval + kPivotBlocks);
    hipError_t e;
    hipLaunchKernelGGL(lu_init_kernel, dim3(blocks(n)), dim3(256), 0, s, perm, n, info);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    for (int64_t k = 0; k < n; k += kPanel) {
        const int64_t kb = std::min(kPanel, n - k);
        for (int64_t s0 = k; s0 < k + kb; s0 += kSub) {
            const int64_t s1 = std::min<int64_t>(s0 + kSub, k + kb);
            // pivot search of the sub-panel's first column (the others run fused below)
            int parts = (int)std::min<int64_t>((n - s0 + 255) / 256, kPivotBlocks);
            hipLaunchKernelGGL(pivot_partial_kernel, dim3(parts), dim3(256), 0, s, A, lda, n, s0, pval, prow);
            for (int64_t j = s0; j < s1; ++j) {
                hipLaunchKernelGGL(pivot_swap_kernel, dim3(1), dim3(256), 0, s, A, lda, j, pval, prow, parts, ipiv, k,
                                   k + kb, info);
                const int64_t rows = n - j - 1;
                if (rows > 0) {
                    const int eb = (int)std::min<int64_t>((rows + 7) / 8, kPivotBlocks);
                    const int search = j + 1 < s1 ? 1 : 0;
                    hipLaunchKernelGGL(eliminate_kernel, dim3(eb), dim3(256), 0, s, A, lda, n, j, s1, search, pval,
                                       prow);
                    if (search) parts = eb;
                }
                if ((e = hipGetLastError()) != hipSuccess) return e;
            }
            // the sub-panel's rows of the outer panel's remaining columns, then the rows below
            const int64_t c1 = k + kb;
            if (c1 > s1) {
                hipLaunchKernelGGL(trsm_lower_kernel, dim3(blocks(c1 - s1)), dim3(256), 0, s, A + s0 * lda + s0, lda,
                                   A + s0 * lda, lda, (int)(s1 - s0), s1, c1, (const double2 *)nullptr, 0);
                if ((e = hipGetLastError()) != hipSuccess) return e;
                if ((e = gemm_sub(A + s1 * lda + s1, lda, A + s1 * lda + s0, lda, A + s0 * lda + s1, lda, n - s1,
                                  c1 - s1, s1 - s0, s)) != hipSuccess)
                    return e;
            }
        }
        hipLaunchKernelGGL(laswp_kernel, dim3(blocks(n - kb + 1)), dim3(256), 0, s, A, lda, n, k, kb, ipiv, perm);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        const int64_t c0 = k + kb;
        if (c0 < n) {
            // U12 = L11^-1 A12, 32 rows at a time
            for (int64_t r0 = k; r0 < c0; r0 += kSub) {
                const int64_t r1 = std::min<int64_t>(r0 + kSub, c0);
                hipLaunchKernelGGL(trsm_lower_kernel, dim3(blocks(n - c0)), dim3(256), 0, s, A + r0 * lda + r0, lda,
                                   A + r0 * lda, lda, (int)(r1 - r0), c0, n, (const double2 *)nullptr, 0);
                if ((e = hipGetLastError()) != hipSuccess) return e;
                if ((e = gemm_sub(A + r1 * lda + c0, lda, A + r1 * lda + r0, lda, A + r0 * lda + c0, lda, c0 - r1,
                                  n - c0, r1 - r0, s)) != hipSuccess)
                    return e;
            }
            // A22 -= L21 U12
            if ((e = gemm_sub(A + c0 * lda + c0, lda, A + c0 * lda + k, lda, A + k * lda + c0, lda, n - c0, n - c0, kb,
                              s)) != hipSuccess)
                return e;
        }
    }
    return hipSuccess;
}

hipError_t lu_solve(const double2 *LU, int64_t n, int64_t lda, const int64_t *perm, const double2 *B, int64_t ldb,
                    double2 *X, int64_t ldx, int64_t m, void *work, hipStream_t s) {
    double2 *part = static_cast<double2 *>(work);
    hipError_t e;
    hipLaunchKernelGGL(permute_rows_kernel, dim3(blocks(n * m)), dim3(256), 0, s, B, ldb, perm, n, m, X, ldx);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    // L Y = P B
    for (int64_t r0 = 0; r0 < n; r0 += kSub) {
        const int rb = (int)std::min<int64_t>(kSub, n - r0);
        int nz = 0;
        if (r0 > 0) {
            nz = (int)((r0 + kSolveChunk - 1) / kSolveChunk);
            if ((e = gemm_part(part, LU + r0 * lda, lda, X, ldx, rb, m, r0, nz, s)) != hipSuccess) return e;
        }
        hipLaunchKernelGGL(trsm_lower_kernel, dim3(blocks(m)), dim3(256), 0, s, LU + r0 * lda + r0, lda, X + r0 * ldx,
                           ldx, rb, (int64_t)0, m, nz ? part : nullptr, nz);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    // U X = Y, from the bottom
    for (int64_t r0 = (n - 1) / kSub * kSub; r0 >= 0; r0 -= kSub) {
        const int rb = (int)std::min<int64_t>(kSub, n - r0);
        const int64_t k0 = r0 + rb;
        int nz = 0;
        if (k0 < n) {
            nz = (int)((n - k0 + kSolveChunk - 1) / kSolveChunk);
            if ((e = gemm_part(part, LU + r0 * lda + k0, lda, X + k0 * ldx, ldx, rb, m, n - k0, nz, s)) != hipSuccess)
                return e;
        }
        hipLaunchKernelGGL(trsm_upper_kernel, dim3(blocks(m)), dim3(256), 0, s, LU + r0 * lda + r0, lda, X + r0 * ldx,
                           ldx, rb, m, nz ? part : nullptr, nz);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace bemrat
