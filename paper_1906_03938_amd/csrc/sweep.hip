// Generate-and-contract sweep: Z_l = T_l V for a group of coefficient operators T_l.
//
// On gfx950 the FP64 MFMA and the FP64 vector ALU share one pipe (they do not overlap),
// and the LDS is the next scarcest resource, so the kernel generates every operator
// entry exactly once, moves few bytes through the LDS, and keeps the pipe fed from two
// instruction streams:
//
// * Block = 8 waves on 16 target rows (the M dimension of v_mfma_f64_16x16x4f64) and
//   16*CB probe columns, for the NOPS = 4 G operators L0 .. L0 + NOPS - 1
//   (L0 = NOPS blockIdx.z).  The K loop runs over the source triangles in stages of
//   kStage = 16.
// * Producer waves 0-3: thread t generates, for target row t & 15 and source triangle
//   t >> 4 of stage s, the entries of all NOPS operators (the 7 quadrature terms and their
//   transcendental parts once, then the operator sequence) into LDS, in the layout of
//   the MFMA A operand; the diagonal entry is the precomputed self term.  They also
//   stage the probe rows of stage s (from a zero-padded copy made once per call, so no
//   bounds checks are repeated) and the quadrature points of stage s + 1.
// * Consumer waves 4-7: wave w contracts operators L0 + G w .. L0 + G w + G - 1 of stage
//   s - 1 while the producers work on stage s (double-buffered LDS).  Per k-step
//   (4 source triangles) lane (i = lane & 15, k = lane >> 4) reads its entry of each
//   operator (16 bytes) and the probe rows, and accumulates with Gauss's
//   three-multiplication complex product: P1 += Gr Vr, P2 += Gi Vi,
//   P3 += (Gr + Gi)(Vr + Vi); at the end Re Z = P1 - P2, Im Z = P3 - P1 - P2.
//   Generated tiles never reach HBM.
// * Every SIMD runs one producer and one consumer wave, so the vector work of one fills
//   the gaps of the other's MFMA stream.
//
// Operator families (entry of T_l at a != b, summed over the 7 points, with the weight
// A_b w_q / (4 pi) folded into the staged points):
//   Direct: T_l = T(kappa_l):              w/r exp(i kappa_l r)
//   DirectSym: the same on quadruples of nodes {x +- iy, x' +- iy}, sharing transcendentals
//   Taylor: T(c + R t) = sum_l t^l T_l:    w/r exp(i c r) (i R r)^l / l!
#include "generators.h"

namespace bemrat {

namespace {

typedef double v4d __attribute__((ext_vector_type(4)));

__device__ __forceinline__ v4d mfma(double a, double b, v4d c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// Producer / consumer form: waves 0-3 generate the entries of stage s + 1 while waves
// 4-7 contract stage s, through double-buffered LDS; every SIMD then runs one wave of
// each kind, so the vector work of one fills the gaps of the other's MFMA stream on the
// shared FP64 pipe.  Both kinds pass one barrier before their loop and run the same
// nstages + 1 iterations, each ending in exactly one barrier (and none after the loop).
// LDS of one tile (double-buffered probe rows, entries and quadrature points).
template <int G, int CB>
struct TileLds {
    double2 sV[2][kStage * 16 * CB];      // (Vr, Vi) [triangle][column]
    double2 sA[2][4 * G * kStage * 16];   // entries [(operator * kStage + triangle) * 16 + row]
    double4 sQ[2][kStage * kQuad];        // quadrature points [triangle][q]
};

// Operators per consumer wave: 2 (8 per block), except for the expansion form up to 32
// columns: 4 (16 per block, the two-pass generator), where the matrix work per generated
// entry is small and sharing each point's transcendental work over 16 operators pays; with
// 64 columns the 16-operator tiles would not fit the LDS.
constexpr int ops_g(Gen gen, int cb) { return gen == Gen::Taylor && cb <= 2 ? 4 : 2; }

// One tile: 16 target rows from row0, 16 CB columns from col0, operators L0 .. L0 + 4 G - 1,
// by the 512 threads of the block.  Used by the per-call kernel (one tile per block) and by
// the batched persistent kernel (tiles of several meshes taken from a work queue).
template <int G, int CB, Gen GEN, bool DECAY, bool CAST, int FOLDK = 0>
__device__ __forceinline__ void sweep_tile(const SweepArgs &p, int64_t row0, int64_t col0, int L0,
                                           TileLds<G, CB> &lds, double2 *sFc = nullptr) {
    constexpr int NC = 16 * CB;
    constexpr int NOPS = 4 * G;
    constexpr int VPT = kStage * NC / 256;  // staged probe elements per producer thread (1, 2, 4)
    auto &sV = lds.sV;
    auto &sA = lds.sA;
    auto &sQ = lds.sQ;

    const int tid = threadIdx.x;
    const int64_t nstages = p.n_pad / kStage;
    constexpr bool FOLD = FOLDK > 0;
    if constexpr (FOLD) {
        // the fold coefficients (Lgen rows of FOLDK, at most kFoldCoef) into LDS; the first
        // barrier of both roles below publishes them
        for (int i = tid; i < p.Lgen * FOLDK; i += 512) sFc[i] = ld<CAST>(p.fcoef, i);
    }

    if (tid < 256) {
        // ---- producer: thread t generates row t & 15, stage triangle t >> 4
        constexpr int QN = kStage * kQuad;  // quadrature points per stage (112)
        const int brow = tid & 15, btri = tid >> 4;
        const int64_t grow = row0 + brow;
        const double4 xa = ld<CAST>(p.colloc, grow);
        std::conditional_t<FOLD, FoldGenerator<NOPS, GEN, DECAY, FOLDK>, Generator<NOPS, GEN, DECAY>> gen;
        gen.init(p, L0);
        if constexpr (FOLD) gen.set_coef(sFc);
        int64_t voff[VPT];
#pragma unroll
        for (int i = 0; i < VPT; ++i) {
            const int idx = tid + 256 * i;
            voff[i] = (int64_t)(idx / NC) * p.m_pad + col0 + idx % NC;
        }
        const int64_t vstride = (int64_t)kStage * p.m_pad;
        // prologue: probe rows of stage 0 in registers, points of stage 0 in LDS, points
        // of stage 1 in registers
        double2 rv[VPT];
#pragma unroll
        for (int i = 0; i < VPT; ++i) rv[i] = ld<CAST>(p.Vp2, voff[i]);
        double4 rq = make_double4(0.0, 0.0, 0.0, 0.0);
        if (tid < QN) {
            sQ[0][tid] = ld<CAST>(p.quad, tid);
            if (nstages > 1) rq = ld<CAST>(p.quad, QN + tid);
        }
        __syncthreads();
        for (int64_t it = 0; it <= nstages; ++it) {
            if (it < nstages) {
                const int buf = (int)(it & 1);
#pragma unroll
                for (int i = 0; i < VPT; ++i) sV[buf][tid + 256 * i] = rv[i];
                if (tid < QN && it + 1 < nstages) sQ[buf ^ 1][tid] = rq;
                const bool diag = it * kStage + btri == grow;
                double r[kQuad], wr[kQuad];
#pragma unroll
                for (int q = 0; q < kQuad; ++q) {
                    const double4 y = sQ[buf][btri * kQuad + q];
                    const double dx = xa.x - y.x, dy = xa.y - y.y, dz = xa.z - y.z;
                    double r2 = fma(dx, dx, fma(dy, dy, dz * dz));
                    r2 = diag ? 1.0 : r2;  // the diagonal is replaced by the self term below
                    const double rinv = rsqrt_pos(r2);
                    r[q] = r2 * rinv;
                    wr[q] = y.w * rinv;
                }
                // next stage's probe rows and the points of the stage after: they land
                // during the generation below
                if (it + 1 < nstages) {
#pragma unroll
                    for (int i = 0; i < VPT; ++i) rv[i] = ld<CAST>(p.Vp2, voff[i] + (it + 1) * vstride);
                }
                if (tid < QN && it + 2 < nstages) rq = ld<CAST>(p.quad, (it + 2) * QN + tid);
                double2 a[NOPS];
                gen.entries(r, wr, p, a);
                if (diag) {
#pragma unroll
                    for (int j = 0; j < NOPS; ++j) a[j] = ld<CAST>(p.self, (int64_t)min(L0 + j, p.L - 1) * p.n_pad + grow);
                }
#pragma unroll
                for (int j = 0; j < NOPS; ++j) sA[buf][(j * kStage + btri) * 16 + brow] = a[j];
            }
            __syncthreads();
        }
    } else {
        // ---- consumer: wave w contracts operators L0 + G w ... of stage it - 1
        const int w = (tid >> 6) - 4;
        const int lane = tid & 63;
        const int ci = lane & 15, ck = lane >> 4;
        v4d P1[G][CB], P2[G][CB], P3[G][CB];
#pragma unroll
        for (int g = 0; g < G; ++g)
#pragma unroll
            for (int cb = 0; cb < CB; ++cb) {
                P1[g][cb] = v4d{0.0, 0.0, 0.0, 0.0};
                P2[g][cb] = v4d{0.0, 0.0, 0.0, 0.0};
                P3[g][cb] = v4d{0.0, 0.0, 0.0, 0.0};
            }
        __syncthreads();  // pairs with the producers' prologue barrier
        // with 16-operator blocks, a wave whose operators all lie beyond L (the last block of
        // an odd number of 8-operator halves) only keeps the barrier rhythm, as does a wave
        // past the folds of a folded tile
        const bool active = G == 2 || L0 + w * G < p.L;
        for (int64_t it = 0; it <= nstages; ++it) {
            if (it >= 1 && active) {
                const int buf = (int)((it - 1) & 1);
#pragma unroll 2
                for (int ks = 0; ks < kStageSteps; ++ks) {
                    const int tri = 4 * ks + ck;
                    double gr[G], gi[G], gs[G];
#pragma unroll
                    for (int g = 0; g < G; ++g) {
                        const double2 a = sA[buf][((w * G + g) * kStage + tri) * 16 + ci];
                        gr[g] = a.x;
                        gi[g] = a.y;
                        gs[g] = a.x + a.y;
                    }
#pragma unroll
                    for (int cb = 0; cb < CB; ++cb) {
                        const double2 v = sV[buf][tri * NC + cb * 16 + ci];
                        const double vs = v.x + v.y;
#pragma unroll
                        for (int g = 0; g < G; ++g) {
                            P1[g][cb] = mfma(gr[g], v.x, P1[g][cb]);
                            P2[g][cb] = mfma(gi[g], v.y, P2[g][cb]);
                            P3[g][cb] = mfma(gs[g], vs, P3[g][cb]);
                        }
                    }
                }
            }
            __syncthreads();
        }
        // D layout of the 16x16x4 f64 MFMA: register i of a lane holds row (lane >> 4) + 4 i,
        // column lane & 15.
        const int l0 = L0 + w * G;
#pragma unroll
        for (int g = 0; g < G; ++g) {
            if (l0 + g >= p.L) break;
            double2 *Z = p.Z + (int64_t)(l0 + g) * p.zstride;
#pragma unroll
            for (int cb = 0; cb < CB; ++cb) {
                const int64_t col = col0 + cb * 16 + ci;
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int64_t row = row0 + ck + 4 * i;
                    const double p1 = P1[g][cb][i], p2 = P2[g][cb][i], p3 = P3[g][cb][i];
                    if (row < p.n && col < p.m) st<CAST>(Z, row * p.ldz + col, make_double2(p1 - p2, p3 - p1 - p2));
                }
            }
        }
    }
}

template <int G, int CB, Gen GEN, bool DECAY>
__global__ __launch_bounds__(512, 1) void sweep_kernel(SweepArgs p) {
    __shared__ TileLds<G, CB> lds;
    sweep_tile<G, CB, GEN, DECAY, false>(p, (int64_t)blockIdx.x * 16, (int64_t)blockIdx.y * 16 * CB,
                                  (int)blockIdx.z * 4 * G, lds);
}

// Folded form: one block per (row block, column block) generates every operator of its
// entries and contracts its p.L folds, at the fold width KL = 1, 2 or 4, on a tile of 4
// operators.
template <int CB, Gen GEN, bool DECAY, int KL>
__global__ __launch_bounds__(512, 1) void sweep_fold_kernel(SweepArgs p) {
    __shared__ TileLds<1, CB> lds;
    __shared__ double2 sFc[kFoldCoef];
    sweep_tile<1, CB, GEN, DECAY, false, KL>(p, (int64_t)blockIdx.x * 16, (int64_t)blockIdx.y * 16 * CB, 0, lds, sFc);
}

template <int CB, Gen GEN, bool DECAY, int KL>
hipError_t launch_fold_t(const SweepArgs &p, hipStream_t stream) {
    constexpr int NC = 16 * CB;
    dim3 grid((unsigned)(p.n_pad / 16), (unsigned)((p.m + NC - 1) / NC), 1u);
    hipLaunchKernelGGL((sweep_fold_kernel<CB, GEN, DECAY, KL>), grid, dim3(512), 0, stream, p);
    return hipGetLastError();
}

template <Gen GEN, bool DECAY, int KL>
hipError_t launch_fold_k(const SweepArgs &p, hipStream_t stream) {
    const int cb = p.m <= 16 ? 1 : (p.m <= 32 ? 2 : 4);
    switch (cb) {
        case 1: return launch_fold_t<1, GEN, DECAY, KL>(p, stream);
        case 2: return launch_fold_t<2, GEN, DECAY, KL>(p, stream);
        default: return launch_fold_t<4, GEN, DECAY, KL>(p, stream);
    }
}

template <Gen GEN, bool DECAY>
hipError_t launch_fold_gen(const SweepArgs &p, hipStream_t stream) {
    switch (fold_width(p.L)) {
        case 1: return launch_fold_k<GEN, DECAY, 1>(p, stream);
        case 2: return launch_fold_k<GEN, DECAY, 2>(p, stream);
        default: return launch_fold_k<GEN, DECAY, 4>(p, stream);
    }
}

template <int G, int CB, Gen GEN, bool DECAY>
hipError_t launch_t(const SweepArgs &p, hipStream_t stream) {
    constexpr int NC = 16 * CB;
    dim3 grid((unsigned)(p.n_pad / 16), (unsigned)((p.m + NC - 1) / NC), (unsigned)((p.L + 4 * G - 1) / (4 * G)));
    hipLaunchKernelGGL((sweep_kernel<G, CB, GEN, DECAY>), grid, dim3(512), 0, stream, p);
    return hipGetLastError();
}

template <Gen GEN, bool DECAY>
hipError_t launch_gen(const SweepArgs &p, hipStream_t stream) {
    if (p.m <= 16) return launch_t<ops_g(GEN, 1), 1, GEN, DECAY>(p, stream);
    if (p.m <= 32) return launch_t<ops_g(GEN, 2), 2, GEN, DECAY>(p, stream);
    return launch_t<2, 4, GEN, DECAY>(p, stream);
}

// Persistent batched form: one block per compute unit takes tiles of several meshes from a
// work queue (an atomic counter cleared by batch_reset_kernel before the launch); each item
// names (mesh, row block, column block, operator block) and the mesh's arguments come from
// a table in device memory.  Every mesh of one launch uses the same operator family.  Items
// are ordered longest first by the host, so the tail of the launch holds the shortest tiles.  Every block leaves the
// loop once the counter passes the item count.
template <int CB, Gen GEN, bool DECAY>
__global__ __launch_bounds__(512, 1) void sweep_batch_kernel(const BatchEntry *__restrict__ table,
                                                             const int4 *__restrict__ items, int nitems,
                                                             unsigned *__restrict__ counter) {
    constexpr int G = ops_g(GEN, CB);
    __shared__ TileLds<G, CB> lds;
    __shared__ int s_next;
    for (;;) {
        if (threadIdx.x == 0) s_next = (int)atomicAdd(counter, 1u);
        // the tile's own barriers keep this write behind every read of the previous value
        __syncthreads();
        const int idx = __builtin_amdgcn_readfirstlane(s_next);
        if (idx >= nitems) break;
        const int4 item = items[idx];
        const int mesh = __builtin_amdgcn_readfirstlane(item.x);
        const SweepArgs p = table[mesh].args;
        sweep_tile<G, CB, GEN, DECAY, true>(p, (int64_t)__builtin_amdgcn_readfirstlane(item.y) * 16,
                                            (int64_t)__builtin_amdgcn_readfirstlane(item.z) * 16 * CB,
                                            __builtin_amdgcn_readfirstlane(item.w) * 4 * G, lds);
    }
}

// Folded persistent batch: as sweep_batch_kernel with the folded tile (each mesh's P <= 4 weight
// sets at the fold width KL = 1, 2 or 4: every operator of an entry generated and folded, only the folds contracted);
// the items carry no operator block.  A tile copies its mesh's fold coefficients into LDS
// behind the previous tile's last barrier.
template <int CB, Gen GEN, bool DECAY, int KL>
__global__ __launch_bounds__(512, 1) void sweep_fold_batch_kernel(const BatchEntry *__restrict__ table,
                                                                  const int4 *__restrict__ items, int nitems,
                                                                  unsigned *__restrict__ counter) {
    __shared__ TileLds<1, CB> lds;
    __shared__ double2 sFc[kFoldCoef];
    __shared__ int s_next;
    for (;;) {
        if (threadIdx.x == 0) s_next = (int)atomicAdd(counter, 1u);
        // the tile's own barriers keep this write behind every read of the previous value
        __syncthreads();
        const int idx = __builtin_amdgcn_readfirstlane(s_next);
        if (idx >= nitems) break;
        const int4 item = items[idx];
        const int mesh = __builtin_amdgcn_readfirstlane(item.x);
        const SweepArgs p = table[mesh].args;
        sweep_tile<1, CB, GEN, DECAY, true, KL>(p, (int64_t)__builtin_amdgcn_readfirstlane(item.y) * 16,
                                                (int64_t)__builtin_amdgcn_readfirstlane(item.z) * 16 * CB, 0, lds,
                                                sFc);
    }
}

__global__ void batch_reset_kernel(unsigned *counter) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *counter = 0u;
}

// Zero-padded copy of the probe block: Vp2[b][c] = V[b][c] for b < n_pad, c < m_pad
// (zeros outside n x m).
__global__ void prep_probe_kernel(const double2 *__restrict__ V, int64_t ldv, int64_t n, int64_t m,
                                  int64_t n_pad, int64_t m_pad, double2 *__restrict__ Vp2) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= n_pad * m_pad) return;
    const int64_t b = idx / m_pad, c = idx % m_pad;
    Vp2[idx] = (b < n && c < m) ? V[b * ldv + c] : make_double2(0.0, 0.0);
}

}  // namespace

// Expansion lengths are whole multiples of 8 whatever the block: a 16-operator block whose
// second half lies beyond L skips that half (generator pass and contraction).  Rounding L up
// to 16 instead would add terms whose self-term coefficients are rounding noise, which the
// Chebyshev eigen-route's highest coefficient blocks are sensitive to.
int sweep_ops_per_block(Gen, int64_t) { return 8; }

int batch_ops_per_item_f64(Gen gen, int cb) { return 4 * ops_g(gen, cb); }

int64_t sweep_m_pad(int64_t m) {
    const int nc = m <= 16 ? 16 : (m <= 32 ? 32 : 64);
    return (m + nc - 1) / nc * nc;
}

hipError_t launch_prep_probe(const double2 *V, int64_t ldv, int64_t n, int64_t m, int64_t n_pad, int64_t m_pad,
                             double2 *Vp2, hipStream_t stream) {
    const int bs = 256;
    const unsigned grid = (unsigned)((n_pad * m_pad + bs - 1) / bs);
    hipLaunchKernelGGL(prep_probe_kernel, dim3(grid), dim3(bs), 0, stream, V, ldv, n, m, n_pad, m_pad, Vp2);
    return hipGetLastError();
}

int batch_variant(Gen gen, bool decay) {
    switch (gen) {
        case Gen::Direct: return decay ? kBatchDirectDecay : kBatchDirect;
        case Gen::Taylor: return decay ? kBatchTaylorDecay : kBatchTaylor;
        case Gen::DirectSym: return decay ? kBatchDirectSym : -1;
        default: return -1;
    }
}

int batch_col_tile(int64_t m) { return m <= 16 ? 1 : (m <= 32 ? 2 : 4); }

template <Gen GEN, bool DECAY>
hipError_t launch_batch_gen(int cb, const BatchEntry *table, const int4 *items, int nitems, unsigned *counter,
                            int grid, hipStream_t stream) {
    switch (cb) {
        case 1: hipLaunchKernelGGL((sweep_batch_kernel<1, GEN, DECAY>), dim3(grid), dim3(512), 0, stream, table, items, nitems, counter); break;
        case 2: hipLaunchKernelGGL((sweep_batch_kernel<2, GEN, DECAY>), dim3(grid), dim3(512), 0, stream, table, items, nitems, counter); break;
        case 4: hipLaunchKernelGGL((sweep_batch_kernel<4, GEN, DECAY>), dim3(grid), dim3(512), 0, stream, table, items, nitems, counter); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_sweep_batch(int variant, int cb, const BatchEntry *table, const int4 *items, int nitems,
                              unsigned *counter, int grid, hipStream_t stream) {
    if (grid < 1 || nitems < 0) return hipErrorInvalidValue;
    hipLaunchKernelGGL(batch_reset_kernel, dim3(1), dim3(64), 0, stream, counter);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    switch (variant) {
        case kBatchDirectDecay: return launch_batch_gen<Gen::Direct, true>(cb, table, items, nitems, counter, grid, stream);
        case kBatchDirect: return launch_batch_gen<Gen::Direct, false>(cb, table, items, nitems, counter, grid, stream);
        case kBatchTaylorDecay: return launch_batch_gen<Gen::Taylor, true>(cb, table, items, nitems, counter, grid, stream);
        case kBatchTaylor: return launch_batch_gen<Gen::Taylor, false>(cb, table, items, nitems, counter, grid, stream);
        case kBatchDirectSym: return launch_batch_gen<Gen::DirectSym, true>(cb, table, items, nitems, counter, grid, stream);
        default: return hipErrorInvalidValue;
    }
}

template <Gen GEN, bool DECAY, int KL>
hipError_t launch_fold_batch_gen(int cb, const BatchEntry *table, const int4 *items, int nitems, unsigned *counter,
                                 int grid, hipStream_t stream) {
    const dim3 g(grid), b(512);
    switch (cb) {
        case 1: hipLaunchKernelGGL((sweep_fold_batch_kernel<1, GEN, DECAY, KL>), g, b, 0, stream, table, items, nitems, counter); break;
        case 2: hipLaunchKernelGGL((sweep_fold_batch_kernel<2, GEN, DECAY, KL>), g, b, 0, stream, table, items, nitems, counter); break;
        case 4: hipLaunchKernelGGL((sweep_fold_batch_kernel<4, GEN, DECAY, KL>), g, b, 0, stream, table, items, nitems, counter); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <int KL>
hipError_t launch_fold_batch_k(int variant, int cb, const BatchEntry *table, const int4 *items, int nitems,
                               unsigned *counter, int grid, hipStream_t stream) {
    switch (variant) {
        case kBatchDirectDecay: return launch_fold_batch_gen<Gen::Direct, true, KL>(cb, table, items, nitems, counter, grid, stream);
        case kBatchDirect: return launch_fold_batch_gen<Gen::Direct, false, KL>(cb, table, items, nitems, counter, grid, stream);
        case kBatchTaylorDecay: return launch_fold_batch_gen<Gen::Taylor, true, KL>(cb, table, items, nitems, counter, grid, stream);
        case kBatchTaylor: return launch_fold_batch_gen<Gen::Taylor, false, KL>(cb, table, items, nitems, counter, grid, stream);
        case kBatchDirectSym: return launch_fold_batch_gen<Gen::DirectSym, true, KL>(cb, table, items, nitems, counter, grid, stream);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_sweep_fold_batch(int variant, int cb, int P, const BatchEntry *table, const int4 *items, int nitems,
                                   unsigned *counter, int grid, hipStream_t stream) {
    if (grid < 1 || nitems < 0 || P < 1 || P > kFoldBatchMax) return hipErrorInvalidValue;
    hipLaunchKernelGGL(batch_reset_kernel, dim3(1), dim3(64), 0, stream, counter);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    switch (fold_width(P)) {
        case 1: return launch_fold_batch_k<1>(variant, cb, table, items, nitems, counter, grid, stream);
        case 2: return launch_fold_batch_k<2>(variant, cb, table, items, nitems, counter, grid, stream);
        default: return launch_fold_batch_k<4>(variant, cb, table, items, nitems, counter, grid, stream);
    }
}

hipError_t launch_sweep_fold(Gen gen, const SweepArgs &args, hipStream_t stream) {
    if (args.L < 1 || args.L > kFoldMax || args.Lgen < 1 || args.Lgen * fold_width(args.L) > kFoldCoef)
        return hipErrorInvalidValue;
    const bool decay = args.decay != 0;
    switch (gen) {
        case Gen::Direct:
            return decay ? launch_fold_gen<Gen::Direct, true>(args, stream) : launch_fold_gen<Gen::Direct, false>(args, stream);
        case Gen::Taylor:
            return decay ? launch_fold_gen<Gen::Taylor, true>(args, stream) : launch_fold_gen<Gen::Taylor, false>(args, stream);
        case Gen::DirectSym:  // quadruples have Im != 0
            return decay ? launch_fold_gen<Gen::DirectSym, true>(args, stream) : hipErrorInvalidValue;
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_sweep(Gen gen, const SweepArgs &args, hipStream_t stream) {
    const bool decay = args.decay != 0;
    switch (gen) {
        case Gen::Direct:
            return decay ? launch_gen<Gen::Direct, true>(args, stream) : launch_gen<Gen::Direct, false>(args, stream);
        case Gen::Taylor:
            return decay ? launch_gen<Gen::Taylor, true>(args, stream) : launch_gen<Gen::Taylor, false>(args, stream);
        case Gen::Cheb:
            return decay ? hipErrorInvalidValue : launch_gen<Gen::Cheb, false>(args, stream);
        case Gen::DirectSym:  // quadruples have Im != 0
            return decay ? launch_gen<Gen::DirectSym, true>(args, stream) : hipErrorInvalidValue;
        default: return hipErrorInvalidValue;
    }
}

}  // namespace bemrat
