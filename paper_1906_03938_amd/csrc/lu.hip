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
//       previous column's elimination); rows j and ipiv[j] are swapped across the outer
//       panel; rows i > j get l_ij = a_ij / a_jj and a_ic -= l_ij a_jc for the sub-panel's
//       columns c > j;
//       then the sub-panel's rows of the outer panel's remaining columns by forward
//       substitution, and the rows below by a complex GEMM with K = 32;
//     the panel's swaps are applied to every column outside it;
//     U12 = L11^-1 A12 by blocked forward substitution;
//     A22 -= L21 U12: complex GEMM with K = kb.
// The GEMM forms each complex product with Gauss's three real multiplications
// (P1 = Ar Br, P2 = Ai Bi, P3 = (Ar + Ai)(Br + Bi); Re = P1 - P2, Im = P3 - P1 - P2) on
// v_mfma_f64_16x16x4f64: 128 x 96 output tiles, 8 waves of 32 x 48 (two waves per SIMD, so
// one wave's barrier waits and LDS reads hide behind the other's MFMAs), double-buffered LDS
// stages of 16 k with the next stage's global loads in flight during the current MFMAs.
//
// Triangular blocks (U12 above, and the solves): up to 256 rows at a time, one workgroup per
// 8 right-hand-side columns holding the block's rows in LDS; 32-row diagonal sub-blocks are
// solved by 32 lanes per column with shuffles, and each solved sub-block updates the block's
// remaining rows.  The solves take the rows' product with the already solved part as a
// split-K MFMA GEMM into partial sums, summed in a fixed order.
#include <algorithm>

#include "internal.h"

namespace bemrat {

namespace {

typedef double v4d __attribute__((ext_vector_type(4)));

__device__ __forceinline__ v4d mfma(double a, double b, v4d c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

constexpr int kSub = 32;         // sub-panel width, diagonal sub-block of the triangular blocks
constexpr int64_t kPanel = 256;  // outer panel width (the trailing GEMM's K)
constexpr int kBlock = 256;      // rows of a triangular block
constexpr int kBlockCols = 8;    // right-hand-side columns per triangular-block workgroup
constexpr int kStageK = 16;      // k per LDS stage of the GEMM
constexpr int kPivotBlocks = 1024;
constexpr int64_t kSolveChunk = 512;  // split-K chunk of the solves with more than 32 columns
constexpr int64_t kSolveChunkNarrow = 128;  // ... and with at most 32

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

// One workgroup of WGM x WGN waves per BM x BN output tile (blockIdx.y, blockIdx.x) and k chunk
// (blockIdx.z); each wave owns TM x TN MFMA tiles of 16 x 16.  MFMA operand layout: lane
// (ci = lane & 15, ck = lane >> 4) holds A[ci][ck] and B[ck][ci]; the result's register q
// holds row ck + 4 q, column ci.
template <int WGM, int WGN, int TM, int TN>
__global__ __launch_bounds__(64 * WGM * WGN) void zgemm_kernel(ZgemmArgs g) {
    constexpr int NT = 64 * WGM * WGN;
    constexpr int BM = WGM * 16 * TM, BN = WGN * 16 * TN, KS = kStageK;
    constexpr int LA = BM * KS / NT, LB = KS * BN / NT;
    static_assert(LA * NT == BM * KS && LB * NT == KS * BN, "whole staging loads");
    __shared__ double2 sA[2][BM][KS + 1];
    __shared__ double2 sB[2][KS][BN];
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
            const int idx = t + NT * l, r = idx / KS, kk = idx % KS;
            const int64_t gr = row0 + r, gk = k0 + kk;
            ra[l] = (gr < g.M && gk < kz) ? g.A[gr * g.lda + gk] : make_double2(0.0, 0.0);
        }
#pragma unroll
        for (int l = 0; l < LB; ++l) {
            const int idx = t + NT * l, kk = idx / BN, c = idx % BN;
            const int64_t gk = k0 + kk, gc = col0 + c;
            rb[l] = (gk < kz && gc < g.N) ? g.B[gk * g.ldb + gc] : make_double2(0.0, 0.0);
        }
    };
    auto store = [&](int b) {
#pragma unroll
        for (int l = 0; l < LA; ++l) {
            const int idx = t + NT * l;
            sA[b][idx / KS][idx % KS] = ra[l];
        }
#pragma unroll
        for (int l = 0; l < LB; ++l) {
            const int idx = t + NT * l;
            sB[b][idx / BN][idx % BN] = rb[l];
        }
    };
    // Stage s is computed from buffer s & 1; after computing it a wave stores stage s + 1
    // (loaded during stage s - 1) into the other buffer, which every wave finished reading
    // before the previous barrier, and issues the loads of stage s + 2.
    load(ka);
    store(0);
    if (ka + KS < kz) load(ka + KS);
    __syncthreads();
    int b = 0;
    for (int64_t k0 = ka; k0 < kz; k0 += KS) {
#pragma unroll
        for (int ks = 0; ks < KS; ks += 4) {
            double ar[TM], ai[TM], as[TM], br[TN], bi[TN], bs[TN];
#pragma unroll
            for (int i = 0; i < TM; ++i) {
                const double2 a = sA[b][wm * 16 * TM + 16 * i + ci][ks + ck];
                ar[i] = a.x;
                ai[i] = a.y;
                as[i] = a.x + a.y;
            }
#pragma unroll
            for (int j = 0; j < TN; ++j) {
                const double2 v = sB[b][ks + ck][wn * 16 * TN + 16 * j + ci];
                br[j] = v.x;
                bi[j] = v.y;
                bs[j] = v.x + v.y;
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
        if (k0 + KS < kz) {
            store(b ^ 1);
            if (k0 + 2 * KS < kz) load(k0 + 2 * KS);
        }
        __syncthreads();
        b ^= 1;
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

// Factorisation updates: 128 x 96 tiles, 8 waves of 32 x 48 (measured 0.69 of MFMA-issued peak
// on M = N = 32512, K = 256, against 0.67 for 32 x 32 waves and 0.45 for 4 waves of 64 x 32).
constexpr int kWGM = 4, kWGN = 2, kTM = 2, kTN = 3;
constexpr int kBM = kWGM * 16 * kTM, kBN = kWGN * 16 * kTN;
// Split-K products of the solves: 128 x 64 tiles (the right-hand sides come in 64s), 8 waves
// of 32 x 32; with at most 32 right-hand sides 64 x 32 tiles of 4 waves of 16 x 32 over
// chunks of 128 (the wide tile would leave half its waves on zero columns, and a chunk of 512
// gives too few workgroups to stream the panel at the rate of the chip: sphere-81920, 32
// columns, 131 us per product).
constexpr int kPTN = 2, kPBN = kWGN * 16 * kPTN;
constexpr int64_t solve_chunk(int64_t m) { return m <= 32 ? kSolveChunkNarrow : kSolveChunk; }

hipError_t gemm_sub(double2 *C, int64_t ldc, const double2 *A, int64_t lda, const double2 *B, int64_t ldb, int64_t M,
                    int64_t N, int64_t K, hipStream_t s) {
    if (M <= 0 || N <= 0 || K <= 0) return hipSuccess;
    ZgemmArgs g{C, ldc, A, lda, B, ldb, M, N, K, K, nullptr};
    dim3 grid((unsigned)((N + kBN - 1) / kBN), (unsigned)((M + kBM - 1) / kBM), 1);
    hipLaunchKernelGGL((zgemm_kernel<kWGM, kWGN, kTM, kTN>), grid, dim3(64 * kWGM * kWGN), 0, s, g);
    return hipGetLastError();
}

// part[z] = A[0:M, chunk z] B[chunk z, 0:N] for the solve_chunk(N) chunks z < nz of [0, K).
hipError_t gemm_part(double2 *part, const double2 *A, int64_t lda, const double2 *B, int64_t ldb, int64_t M,
                     int64_t N, int64_t K, int nz, hipStream_t s) {
    ZgemmArgs g{nullptr, 0, A, lda, B, ldb, M, N, K, solve_chunk(N), part};
    if (N <= 32) {
        constexpr int NBM = kWGM * 16;
        dim3 grid(1u, (unsigned)((M + NBM - 1) / NBM), (unsigned)nz);
        hipLaunchKernelGGL((zgemm_kernel<kWGM, 1, 1, kPTN>), grid, dim3(64 * kWGM), 0, s, g);
        return hipGetLastError();
    }
    dim3 grid((unsigned)((N + kPBN - 1) / kPBN), (unsigned)((M + kBM - 1) / kBM), (unsigned)nz);
    hipLaunchKernelGGL((zgemm_kernel<kWGM, kWGN, kTM, kPTN>), grid, dim3(64 * kWGM * kWGN), 0, s, g);
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

// Triangular block solve in place: rows [0, rb) (rb <= kBlock) of X, columns [c0, c1), with the
// rb x rb diagonal block T: unit lower (forward substitution, UPPER false) or upper with its
// diagonal (backward substitution, UPPER true).  One workgroup per kBlockCols columns holds
// the block's rows in LDS.  Per 32-row diagonal sub-block (top down, or bottom up): lane
// r < 32 of column group c keeps row r of column c; for each q in order, the solved value
// x_q is shuffled from lane q and lanes on the unsolved side subtract T[r][q] x_q (for U,
// lane q first divides by T[q][q]).  Then each thread takes one row of the block's unsolved
// side and subtracts its product with the sub-block's 32 solved rows, for all the columns.
template <bool UPPER>
__global__ __launch_bounds__(256) void block_trsm_kernel(const double2 *__restrict__ T, int64_t ldt,
                                                         double2 *__restrict__ X, int64_t ldx, int rb, int64_t c0,
                                                         int64_t c1) {
    __shared__ double2 sX[kBlock][kBlockCols];
    __shared__ double2 sD[kSub][kSub + 1];
    const int t = threadIdx.x;
    const int64_t cb = c0 + (int64_t)blockIdx.x * kBlockCols;
    const int nc = (int)(c1 - cb < kBlockCols ? c1 - cb : kBlockCols);
    for (int i = t; i < rb * kBlockCols; i += 256) {
        const int r = i / kBlockCols, c = i % kBlockCols;
        sX[r][c] = c < nc ? X[r * ldx + cb + c] : make_double2(0.0, 0.0);
    }
    const int nsub = (rb + kSub - 1) / kSub;
    const int lane = t & 31, col = t >> 5;
    for (int it = 0; it < nsub; ++it) {
        const int s0 = (UPPER ? nsub - 1 - it : it) * kSub;
        const int sn = rb - s0 < kSub ? rb - s0 : kSub;
        __syncthreads();
        for (int i = t; i < kSub * kSub; i += 256) {
            const int r = i / kSub, q = i % kSub;
            sD[r][q] = (r < sn && q < sn) ? T[(int64_t)(s0 + r) * ldt + s0 + q] : make_double2(r == q ? 1.0 : 0.0, 0.0);
        }
        __syncthreads();
        // diagonal sub-block: 32 lanes per column (8 columns = 256 threads)
        double2 x = lane < sn ? sX[s0 + lane][col] : make_double2(0.0, 0.0);
        if (!UPPER) {
            for (int q = 0; q < kSub - 1; ++q) {
                const double2 xq = make_double2(__shfl(x.x, q, 32), __shfl(x.y, q, 32));
                if (lane > q) x = csub(x, cmul(sD[lane][q], xq));
            }
        } else {
            for (int q = kSub - 1; q >= 0; --q) {
                if (lane == q) {
                    const double2 d = sD[q][q];
                    const double den = d.x * d.x + d.y * d.y;
                    x = make_double2((x.x * d.x + x.y * d.y) / den, (x.y * d.x - x.x * d.y) / den);
                }
                const double2 xq = make_double2(__shfl(x.x, q, 32), __shfl(x.y, q, 32));
                if (lane < q) x = csub(x, cmul(sD[lane][q], xq));
            }
        }
        if (lane < sn) sX[s0 + lane][col] = x;
        __syncthreads();
        // the block's unsolved rows lose their product with the solved sub-block
        const int ra = UPPER ? 0 : s0 + sn, rz = UPPER ? s0 : rb;
        for (int r = ra + t; r < rz; r += 256) {
            double2 acc[kBlockCols];
#pragma unroll
            for (int c = 0; c < kBlockCols; ++c) acc[c] = make_double2(0.0, 0.0);
            const double2 *Tr = T + (int64_t)r * ldt + s0;
            for (int q = 0; q < sn; ++q) {
                const double2 l = Tr[q];
#pragma unroll
                for (int c = 0; c < kBlockCols; ++c) {
                    const double2 v = sX[s0 + q][c];
                    acc[c].x += l.x * v.x - l.y * v.y;
                    acc[c].y += l.x * v.y + l.y * v.x;
                }
            }
#pragma unroll
            for (int c = 0; c < kBlockCols; ++c) sX[r][c] = csub(sX[r][c], acc[c]);
        }
    }
    __syncthreads();
    for (int i = t; i < rb * kBlockCols; i += 256) {
        const int r = i / kBlockCols, c = i % kBlockCols;
        if (c < nc) X[r * ldx + cb + c] = sX[r][c];
    }
}

// X[r][c] -= sum over z < nz of part[z][r][c], r < rb, c < m.  A workgroup takes 32 items
// (consecutive in memory) and splits z into kSumSlices interleaved slices, one per 32 threads;
// each slice sums in z order and the slices are added in slice order (a fixed order: the
// result does not depend on the launch).  Enough workgroups to stream the partials however
// many chunks there are.
constexpr int kSumSlices = 8;
__global__ __launch_bounds__(256) void part_sum_kernel(double2 *__restrict__ X, int64_t ldx, int rb, int64_t m,
                                                       const double2 *__restrict__ part, int nz) {
    __shared__ double2 acc[kSumSlices][32];
    const int lane = threadIdx.x & 31, slice = threadIdx.x >> 5;
    const int64_t item = (int64_t)blockIdx.x * 32 + lane, items = (int64_t)rb * m;
    double sr = 0.0, si = 0.0;
    if (item < items) {
        for (int z = slice; z < nz; z += kSumSlices) {
            const double2 p = part[(int64_t)z * items + item];
            sr += p.x;
            si += p.y;
        }
    }
    acc[slice][lane] = make_double2(sr, si);
    __syncthreads();
    if (slice == 0 && item < items) {
        for (int k = 1; k < kSumSlices; ++k) {
            sr += acc[k][lane].x;
            si += acc[k][lane].y;
        }
        const int64_t r = item / m, c = item % m;
        double2 &o = X[r * ldx + c];
        o = make_double2(o.x - sr, o.y - si);
    }
}

hipError_t block_trsm(bool upper, const double2 *T, int64_t ldt, double2 *X, int64_t ldx, int rb, int64_t c0,
                      int64_t c1, hipStream_t s) {
    const unsigned nb = (unsigned)((c1 - c0 + kBlockCols - 1) / kBlockCols);
    if (upper)
        hipLaunchKernelGGL(block_trsm_kernel<true>, dim3(nb), dim3(256), 0, s, T, ldt, X, ldx, rb, c0, c1);
    else
        hipLaunchKernelGGL(block_trsm_kernel<false>, dim3(nb), dim3(256), 0, s, T, ldt, X, ldx, rb, c0, c1);
    return hipGetLastError();
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
    const int64_t nz = (n + solve_chunk(m) - 1) / solve_chunk(m);
    return nz * kBlock * m * (int64_t)sizeof(double2);
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
                if ((e = block_trsm(false, A + s0 * lda + s0, lda, A + s0 * lda, lda, (int)(s1 - s0), s1, c1, s)) !=
                    hipSuccess)
                    return e;
                if ((e = gemm_sub(A + s1 * lda + s1, lda, A + s1 * lda + s0, lda, A + s0 * lda + s1, lda, n - s1,
                                  c1 - s1, s1 - s0, s)) != hipSuccess)
                    return e;
            }
        }
        hipLaunchKernelGGL(laswp_kernel, dim3(blocks(n - kb + 1)), dim3(256), 0, s, A, lda, n, k, kb, ipiv, perm);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        const int64_t c0 = k + kb;
        if (c0 < n) {
            // U12 = L11^-1 A12, then A22 -= L21 U12
            if ((e = block_trsm(false, A + k * lda + k, lda, A + k * lda, lda, (int)kb, c0, n, s)) != hipSuccess)
                return e;
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
    // L Y = P B, kBlock rows at a time: the rows' product with the solved part (split-K
    // partials, then their sum), then the diagonal block
    for (int64_t r0 = 0; r0 < n; r0 += kBlock) {
        const int rb = (int)std::min<int64_t>(kBlock, n - r0);
        if (r0 > 0) {
            const int nz = (int)((r0 + solve_chunk(m) - 1) / solve_chunk(m));
            if ((e = gemm_part(part, LU + r0 * lda, lda, X, ldx, rb, m, r0, nz, s)) != hipSuccess) return e;
            hipLaunchKernelGGL(part_sum_kernel, dim3((unsigned)(((int64_t)rb * m + 31) / 32)), dim3(256), 0, s, X + r0 * ldx, ldx, rb,
                               m, (const double2 *)part, nz);
        }
        if ((e = block_trsm(false, LU + r0 * lda + r0, lda, X + r0 * ldx, ldx, rb, 0, m, s)) != hipSuccess) return e;
    }
    // U X = Y, from the bottom
    for (int64_t r0 = (n - 1) / kBlock * kBlock; r0 >= 0; r0 -= kBlock) {
        const int rb = (int)std::min<int64_t>(kBlock, n - r0);
        const int64_t k0 = r0 + rb;
        if (k0 < n) {
            const int nz = (int)((n - k0 + solve_chunk(m) - 1) / solve_chunk(m));
            if ((e = gemm_part(part, LU + r0 * lda + k0, lda, X + k0 * ldx, ldx, rb, m, n - k0, nz, s)) != hipSuccess)
                return e;
            hipLaunchKernelGGL(part_sum_kernel, dim3((unsigned)(((int64_t)rb * m + 31) / 32)), dim3(256), 0, s, X + r0 * ldx, ldx, rb,
                               m, (const double2 *)part, nz);
        }
        if ((e = block_trsm(true, LU + r0 * lda + r0, lda, X + r0 * ldx, ldx, rb, 0, m, s)) != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace bemrat
