// Combination of the generated-operator products Z_l = T_l V into the sweep outputs.
//
// combine:  out_p = sum_l coef[l][p] Z_l  (contour moments, Chebyshev coefficient blocks,
//           or per-node products when the operators are expansion terms);
//           HBM-bound: every Z_l element is read once, outputs written once.
// project:  Q_l = U^H Z_l over row chunks (partials in a fixed order, no atomics), then
//           out_j = sum_l coef[j][l] Q_l.
// block combine: out = sum_b coef[b] (per column) X_b over separate device blocks.
#include "internal.h"
#include "block_combine.h"

namespace bemrat {

namespace {

constexpr int kCombineP = 8;  // outputs accumulated per pass

__global__ void combine_kernel(const double2 *__restrict__ Z, int64_t zstride, int64_t ldz, int L,
                               const double2 *__restrict__ coef, int P, int p0, int64_t n,
                               int64_t m, double2 *__restrict__ out, int64_t ldo) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= n * m) return;
    const int64_t a = idx / m, c = idx % m;
    double sr[kCombineP], si[kCombineP];
#pragma unroll
    for (int p = 0; p < kCombineP; ++p) sr[p] = si[p] = 0.0;
    const int np = min(kCombineP, P - p0);
    for (int l = 0; l < L; ++l) {
        const double2 z = Z[(int64_t)l * zstride + a * ldz + c];
#pragma unroll
        for (int p = 0; p < kCombineP; ++p) {
            if (p < np) {
                const double2 w = coef[(int64_t)l * P + p0 + p];
                sr[p] += w.x * z.x - w.y * z.y;
                si[p] += w.x * z.y + w.y * z.x;
            }
        }
    }
#pragma unroll
    for (int p = 0; p < kCombineP; ++p)
        if (p < np) out[(int64_t)(p0 + p) * n * ldo + a * ldo + c] = make_double2(sr[p], si[p]);
}

// partial[l][chunk][c][d] = sum_{a in chunk} conj(U[a][c]) Z_l[a][d] for a 64 x 64 tile
__global__ __launch_bounds__(256) void project_partial_kernel(
    const double2 *__restrict__ U, int64_t ldu, const double2 *__restrict__ Z, int64_t zstride,
    int64_t ldz, int64_t n, int64_t m, int64_t rows_per_chunk, int nchunks,
    double2 *__restrict__ partial) {
    __shared__ double2 sU[16][64 + 1];
    __shared__ double2 sZ[16][64 + 1];
    const int l = blockIdx.x;
    const int chunk = blockIdx.y;
    const int tiles = (int)((m + 63) / 64);
    const int tc = blockIdx.z / tiles, td = blockIdx.z % tiles;
    const int64_t c0 = (int64_t)tc * 64, d0 = (int64_t)td * 64;
    const int tid = threadIdx.x;
    const int ic = (tid >> 4) * 4, id = (tid & 15) * 4;
    double ar[4][4], ai[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) ar[i][j] = ai[i][j] = 0.0;
    const int64_t a_begin = (int64_t)chunk * rows_per_chunk;
    const int64_t a_end = min(n, a_begin + rows_per_chunk);
    const double2 *Zl = Z + (int64_t)l * zstride;
    for (int64_t a0 = a_begin; a0 < a_end; a0 += 16) {
        __syncthreads();
        for (int i = tid; i < 16 * 64; i += 256) {
            const int r = i >> 6, c = i & 63;
            const int64_t arow = a0 + r;
            const bool ok = arow < a_end;
            sU[r][c] = (ok && c0 + c < m) ? U[arow * ldu + c0 + c] : make_double2(0.0, 0.0);
            sZ[r][c] = (ok && d0 + c < m) ? Zl[arow * ldz + d0 + c] : make_double2(0.0, 0.0);
        }
        __syncthreads();
#pragma unroll 4
        for (int r = 0; r < 16; ++r) {
            double2 u[4], z[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                u[i] = sU[r][ic + i];
                z[i] = sZ[r][id + i];
            }
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    // conj(u) * z
                    ar[i][j] += u[i].x * z[j].x + u[i].y * z[j].y;
                    ai[i][j] += u[i].x * z[j].y - u[i].y * z[j].x;
                }
        }
    }
    double2 *dst = partial + ((int64_t)l * nchunks + chunk) * m * m;
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int64_t c = c0 + ic + i, d = d0 + id + j;
            if (c < m && d < m) dst[c * m + d] = make_double2(ar[i][j], ai[i][j]);
        }
}

// partial[l][0] <- sum over chunks, in chunk order
__global__ void project_reduce_kernel(double2 *__restrict__ partial, int nchunks, int L, int64_t mm) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)L * mm) return;
    const int64_t l = idx / mm, e = idx % mm;
    double2 *base = partial + l * nchunks * mm + e;
    double sr = 0.0, si = 0.0;
    for (int c = 0; c < nchunks; ++c) {
        sr += base[c * mm].x;
        si += base[c * mm].y;
    }
    base[0] = make_double2(sr, si);
}

// out[j] (+)= sum_l coef[j][l] Q_l, Q_l = partial[l][0]
__global__ void project_mix_kernel(const double2 *__restrict__ partial, int nchunks, int L,
                                   int64_t mm, const double2 *__restrict__ coef, int N,
                                   double2 *__restrict__ out, int accumulate) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)N * mm) return;
    const int64_t j = idx / mm, e = idx % mm;
    double sr = 0.0, si = 0.0;
    for (int l = 0; l < L; ++l) {
        const double2 w = coef[j * L + l];
        const double2 q = partial[(int64_t)l * nchunks * mm + e];
        sr += w.x * q.x - w.y * q.y;
        si += w.x * q.y + w.y * q.x;
    }
    if (accumulate) {
        const double2 o = out[j * mm + e];
        sr = o.x + sr;
        si = o.y + si;
    }
    out[j * mm + e] = make_double2(sr, si);
}

// out[l] += sum over chunks of partial[l][chunk], in chunk order
__global__ void project_add_kernel(const double2 *__restrict__ partial, int nchunks, int L, int64_t mm,
                                   double2 *__restrict__ out) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)L * mm) return;
    const int64_t l = idx / mm, e = idx % mm;
    const double2 *base = partial + l * nchunks * mm + e;
    double sr = 0.0, si = 0.0;
    for (int c = 0; c < nchunks; ++c) {
        sr += base[c * mm].x;
        si += base[c * mm].y;
    }
    const double2 o = out[idx];
    out[idx] = make_double2(o.x + sr, o.y + si);
}

// out[r][c] = sum over b < nb of coef[b][c] X_b[r][c], in the order b = 0, 1, ... (the
// block pointers travel in the kernel's arguments).
struct BlockList {
    const double2 *x[kBlockCombineMax];
};

__global__ __launch_bounds__(256) void block_combine_kernel(BlockList bl, int nb, const double2 *__restrict__ coef,
                                                            int64_t n, int64_t m, int64_t ldx, double2 *out,
                                                            int64_t ldo) {
    const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (idx >= n * m) return;
    const int64_t r = idx / m, c = idx % m;
    double sr = 0.0, si = 0.0;
    for (int b = 0; b < nb; ++b) {
        const double2 w = coef[(int64_t)b * m + c];
        const double2 v = bl.x[b][r * ldx + c];
        sr = fma(w.x, v.x, fma(-w.y, v.y, sr));
        si = fma(w.x, v.y, fma(w.y, v.x, si));
    }
    out[r * ldo + c] = make_double2(sr, si);
}

}  // namespace

hipError_t launch_block_combine(const double2 *const *blocks, int nb, const double2 *coef, int64_t n, int64_t m,
                                int64_t ldx, double2 *out, int64_t ldo, hipStream_t stream) {
    if (nb < 1 || nb > kBlockCombineMax) return hipErrorInvalidValue;
    BlockList bl{};
    for (int b = 0; b < nb; ++b) bl.x[b] = blocks[b];
    const unsigned grid = (unsigned)((n * m + 255) / 256);
    hipLaunchKernelGGL(block_combine_kernel, dim3(grid), dim3(256), 0, stream, bl, nb, coef, n, m, ldx, out, ldo);
    return hipGetLastError();
}

hipError_t launch_project_add(const double2 *partial, int nchunks, int L, int64_t m, double2 *out,
                              hipStream_t stream) {
    const int64_t mm = m * m;
    const int bs = 256;
    hipLaunchKernelGGL(project_add_kernel, dim3((unsigned)((L * mm + bs - 1) / bs)), dim3(bs), 0, stream, partial,
                       nchunks, L, mm, out);
    return hipGetLastError();
}

hipError_t launch_combine(const double2 *Z, int64_t zstride, int64_t ldz, int L, const double2 *coef,
                          int P, int64_t n, int64_t m, double2 *out, int64_t ldo, hipStream_t stream) {
    const int bs = 256;
    const unsigned grid = (unsigned)((n * m + bs - 1) / bs);
    for (int p0 = 0; p0 < P; p0 += kCombineP) {
        hipLaunchKernelGGL(combine_kernel, dim3(grid), dim3(bs), 0, stream, Z, zstride, ldz, L, coef,
                           P, p0, n, m, out, ldo);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_project_partial(const double2 *U, int64_t ldu, const double2 *Z, int64_t zstride,
                                  int64_t ldz, int L, int64_t n, int64_t m, int64_t rows_per_chunk,
                                  int nchunks, double2 *partial, hipStream_t stream) {
    const int tiles = (int)((m + 63) / 64);
    dim3 grid((unsigned)L, (unsigned)nchunks, (unsigned)(tiles * tiles));
    hipLaunchKernelGGL(project_partial_kernel, grid, dim3(256), 0, stream, U, ldu, Z, zstride, ldz, n,
                       m, rows_per_chunk, nchunks, partial);
    return hipGetLastError();
}

hipError_t launch_project_finish(const double2 *partial, int nchunks, int L, int64_t m,
                                 const double2 *coef, int N, double2 *out, hipStream_t stream, bool accumulate) {
    const int64_t mm = m * m;
    const int bs = 256;
    hipLaunchKernelGGL(project_reduce_kernel, dim3((unsigned)((L * mm + bs - 1) / bs)), dim3(bs), 0,
                       stream, const_cast<double2 *>(partial), nchunks, L, mm);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(project_mix_kernel, dim3((unsigned)((N * mm + bs - 1) / bs)), dim3(bs), 0,
                       stream, partial, nchunks, L, mm, coef, N, out, accumulate ? 1 : 0);
    return hipGetLastError();
}

}  // namespace bemrat
