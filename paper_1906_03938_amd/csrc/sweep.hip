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
template <int G, int CB, Gen GEN, bool DECAY>
__global__ __launch_bounds__(512, 1) void sweep_kernel(SweepArgs p) {
    constexpr int NC = 16 * CB;
    constexpr int NOPS = 4 * G;
    constexpr int VPT = kStage * NC / 256;  // staged probe elements per producer thread (1, 2, 4)
    __shared__ double2 sV[2][kStage * NC];         // (Vr, Vi) [triangle][column]
    __shared__ double2 sA[2][NOPS * kStage * 16];  // entries [(operator * kStage + triangle) * 16 + row]
    __shared__ double4 sQ[2][kStage * kQuad];      // quadrature points [triangle][q]

    const int tid = threadIdx.x;
    const int64_t row0 = (int64_t)blockIdx.x * 16;
    const int64_t col0 = (int64_t)blockIdx.y * NC;
    const int L0 = blockIdx.z * NOPS;
    const int64_t nstages = p.n_pad / kStage;

    if (tid < 256) {
        // ---- producer: thread t generates row t & 15, stage triangle t >> 4
        constexpr int QN = kStage * kQuad;  // quadrature points per stage (112)
        const int brow = tid & 15, btri = tid >> 4;
        const int64_t grow = row0 + brow;
        const double4 xa = p.colloc[grow];
        Generator<NOPS, GEN, DECAY> gen;
        gen.init(p, L0);
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
        for (int i = 0; i < VPT; ++i) rv[i] = p.Vp2[voff[i]];
        double4 rq = make_double4(0.0, 0.0, 0.0, 0.0);
        if (tid < QN) {
            sQ[0][tid] = p.quad[tid];
            if (nstages > 1) rq = p.quad[QN + tid];
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
                    for (int i = 0; i < VPT; ++i) rv[i] = p.Vp2[voff[i] + (it + 1) * vstride];
                }
                if (tid < QN && it + 2 < nstages) rq = p.quad[(it + 2) * QN + tid];
                double2 a[NOPS];
                gen.entries(r, wr, p, a);
                if (diag) {
#pragma unroll
                    for (int j = 0; j < NOPS; ++j) a[j] = p.self[(int64_t)min(L0 + j, p.L - 1) * p.n_pad + grow];
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
        for (int64_t it = 0; it <= nstages; ++it) {
            if (it >= 1) {
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
                    if (row < p.n && col < p.m) Z[row * p.ldz + col] = make_double2(p1 - p2, p3 - p1 - p2);
                }
            }
        }
    }
}

template <int G, int CB, Gen GEN, bool DECAY>
hipError_t launch_t(const SweepArgs &p, hipStream_t stream) {
    constexpr int NC = 16 * CB;
    dim3 grid((unsigned)(p.n_pad / 16), (unsigned)((p.m + NC - 1) / NC), (unsigned)((p.L + 4 * G - 1) / (4 * G)));
    hipLaunchKernelGGL((sweep_kernel<G, CB, GEN, DECAY>), grid, dim3(512), 0, stream, p);
    return hipGetLastError();
}

// Operators per consumer wave: 2 (8 per block) for every column count; the producer's
// generation of 8 operators fits two waves per SIMD without spilling.
template <Gen GEN, bool DECAY>
hipError_t launch_gen(const SweepArgs &p, hipStream_t stream) {
    if (p.m <= 16) return launch_t<2, 1, GEN, DECAY>(p, stream);
    if (p.m <= 32) return launch_t<2, 2, GEN, DECAY>(p, stream);
    return launch_t<2, 4, GEN, DECAY>(p, stream);
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

int sweep_ops_per_block(int64_t) { return 8; }

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

hipError_t launch_sweep(Gen gen, const SweepArgs &args, hipStream_t stream) {
    const bool decay = args.decay != 0;
    switch (gen) {
        case Gen::Direct:
            return decay ? launch_gen<Gen::Direct, true>(args, stream) : launch_gen<Gen::Direct, false>(args, stream);
        case Gen::Taylor:
            return decay ? launch_gen<Gen::Taylor, true>(args, stream) : launch_gen<Gen::Taylor, false>(args, stream);
        case Gen::Cheb:
            return decay ? hipErrorInvalidValue : launch_gen<Gen::Cheb, false>(args, stream);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace bemrat
