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
#include "devmath.h"
#include "internal.h"

namespace bemrat {

namespace {

typedef double v4d __attribute__((ext_vector_type(4)));

constexpr int kStage = 16;               // source triangles per stage
constexpr int kStageSteps = kStage / 4;  // k-steps per stage

__device__ __forceinline__ v4d mfma(double a, double b, v4d c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// 1/sqrt(a) for finite a > 0 (squared distances between distinct points, or 1 on the
// diagonal): hardware estimate and one Newton step y (3 - a y^2) / 2, written as
// y + y/2 (1 - a y^2) with fused multiply-adds.
__device__ __forceinline__ double rsqrt_pos(double a) {
    const double y = __builtin_amdgcn_rsq(a);
    const double e = fma(-a * y, y, 1.0);
    return fma(0.5 * y, e, y);
}

// Entries of the NOPS operators L0 .. L0 + NOPS - 1 at one (row, triangle) off the
// diagonal, from the distances r_q and weights w_q / r_q of the 7 quadrature points.
template <int NOPS, Gen GEN, bool DECAY>
struct Generator;

template <int NOPS, bool DECAY>
struct Generator<NOPS, Gen::Direct, DECAY> {
    double kr[NOPS], ki[NOPS];
    __device__ void init(const SweepArgs &p, int L0) {
#pragma unroll
        for (int j = 0; j < NOPS; ++j) {
            const int l = min(L0 + j, p.L - 1);
            kr[j] = p.kappa[l].x;
            ki[j] = p.kappa[l].y;
        }
    }
    __device__ __forceinline__ void entries(const double (&r)[kQuad], const double (&wr)[kQuad],
                                            const SweepArgs &, double2 (&out)[NOPS]) const {
#pragma unroll
        for (int j = 0; j < NOPS; ++j) {
            double gr = 0.0, gi = 0.0;
#pragma unroll
            for (int q = 0; q < kQuad; ++q) {
                const double e = DECAY ? exp_cw(-ki[j] * r[q]) * wr[q] : wr[q];
                double sn, cs;
                sincos_cw(kr[j] * r[q], sn, cs);
                gr = fma(e, cs, gr);
                gi = fma(e, sn, gi);
            }
            out[j] = make_double2(gr, gi);
        }
    }
};

// Term of operator L0 + j at one point: w/r exp(i c r) (i x)^(L0 + j) / (L0 + j)!, x = R r.
// L0 is a multiple of 4, so (i x)^L0 = x^L0; the rest is y0 i^j x^j c_j with
// y0 = w/r exp(i c r) x^L0 / L0! and the block-uniform c_j = L0! / (L0 + j)!, which with
// i^j is applied once to the sum over the points.  The power x^j is a running product, so
// no per-operator factor can be hoisted out of the point loop and kept live.
template <int NOPS, bool DECAY>
struct Generator<NOPS, Gen::Taylor, DECAY> {
    static constexpr int B = NOPS;  // L0 = z B
    int z;
    double inv_fact;                // 1 / L0!
    double cj[NOPS];                // L0! / (L0 + j)!
    __device__ void init(const SweepArgs &p, int L0) {
        z = L0 / B;
        inv_fact = p.inv_fact[min(L0, kMaxTaylor - 1)];
        double c = 1.0;
#pragma unroll
        for (int j = 0; j < NOPS; ++j) {
            cj[j] = c;
            c *= p.inv_int[min(L0 + j + 1, kMaxTaylor - 1)];
        }
    }
    __device__ __forceinline__ void entries(const double (&r)[kQuad], const double (&wr)[kQuad],
                                            const SweepArgs &p, double2 (&out)[NOPS]) const {
        double gr[NOPS], gi[NOPS];
#pragma unroll
        for (int j = 0; j < NOPS; ++j) gr[j] = gi[j] = 0.0;
        // x^L0 / L0! = (x^B)^z / L0! for all points together: z is uniform over the block,
        // so the loop over its bits does not diverge and costs two products per point and bit
        double xq[kQuad], base[kQuad], pwq[kQuad];
#pragma unroll
        for (int q = 0; q < kQuad; ++q) {
            xq[q] = p.R * r[q];
            const double x2 = xq[q] * xq[q], x4 = x2 * x2;
            base[q] = B == 8 ? x4 * x4 : x4 * x4 * x4;
            pwq[q] = inv_fact;
        }
        for (int zz = z; zz != 0; zz >>= 1) {
            if (zz & 1) {
#pragma unroll
                for (int q = 0; q < kQuad; ++q) pwq[q] *= base[q];
            }
#pragma unroll
            for (int q = 0; q < kQuad; ++q) base[q] *= base[q];
        }
#pragma unroll
        for (int q = 0; q < kQuad; ++q) {
            const double x = xq[q], pw = pwq[q];
            const double e = (DECAY ? exp_cw(-p.c_im * r[q]) * wr[q] : wr[q]) * pw;
            double sn, cs;
            sincos_cw(p.c_re * r[q], sn, cs);
            const double yr = e * cs, yi = e * sn;
            // sum_q y x^j (c_j and i^j are applied once per operator below)
            double xp = x;
            gr[0] += yr;
            gi[0] += yi;
#pragma unroll
            for (int j = 1; j < NOPS; ++j) {
                gr[j] = fma(yr, xp, gr[j]);
                gi[j] = fma(yi, xp, gi[j]);
                xp *= x;
            }
        }
#pragma unroll
        for (int j = 1; j < NOPS; ++j) {
            const double a = gr[j] * cj[j], b = gi[j] * cj[j];
            switch (j & 3) {  // times i^j (compile-time rotation)
                case 0: gr[j] = a; gi[j] = b; break;
                case 1: gr[j] = -b; gi[j] = a; break;
                case 2: gr[j] = -a; gi[j] = -b; break;
                default: gr[j] = b; gi[j] = -a; break;
            }
        }
#pragma unroll
        for (int j = 0; j < NOPS; ++j) out[j] = make_double2(gr[j], gi[j]);
    }
};

// Chebyshev (Jacobi-Anger) form for real nodes kappa = alpha + beta xi, xi in [-1, 1]:
// exp(i kappa r) = exp(i alpha r) sum_l eps_l i^l J_l(beta r) T_l(xi), so with the factors
// eps_l i^l left to the host's recombination, operator l has entries
// sum_q w_q / r_q exp(i alpha r_q) J_l(beta r_q).  The J_l come from Miller's backward
// recurrence J_{l-1} = (2 l / x) J_l - J_{l+1}, started at J_{M+1} = 0, J_M = 2^-1000 (M a
// multiple of 8, at least the block's top index, chosen by the host) and normalised by
// J_0 + 2 sum_k J_{2k} = 1.  The recurrence runs eight steps per trip; after each trip the
// values are scaled down by 2^-400 if they exceed 2^400 (they grow like M! (2/x)^M for
// small x; eight steps grow them by less than 2^250 for x >= 1e-7 and M <= 96), and a
// factor f carries that scaling to the block's values stored earlier.
template <int NOPS, bool DECAY>
struct Generator<NOPS, Gen::Cheb, DECAY> {
    int L0, M;
    __device__ void init(const SweepArgs &p, int L0_) {
        L0 = L0_;
        M = p.miller_M;
    }
    // eight steps from index l (a multiple of 8) down to l - 8; S gains 2 J at each even index
    __device__ __forceinline__ static void steps8(int l, double tx, double &jp, double &jc, double &S) {
        double t = l * tx;
#pragma unroll
        for (int i = 1; i <= 8; ++i) {
            const double jn = fma(t, jc, -jp);  // J_{l-i}
            jp = jc;
            jc = jn;
            t -= tx;
            if ((i & 1) == 0) S = fma(2.0, jc, S);
        }
    }
    __device__ __forceinline__ static double rescale(double &jp, double &jc, double &S) {
        const double sc = fabs(jc) > 0x1p400 ? 0x1p-400 : 1.0;
        jp *= sc;
        jc *= sc;
        S *= sc;
        return sc;
    }
    __device__ __forceinline__ void entries(const double (&r)[kQuad], const double (&wr)[kQuad],
                                            const SweepArgs &p, double2 (&out)[NOPS]) const {
        double gr[NOPS], gi[NOPS];
#pragma unroll
        for (int j = 0; j < NOPS; ++j) gr[j] = gi[j] = 0.0;
#pragma unroll
        for (int q = 0; q < kQuad; ++q) {
            const double x = p.R * r[q];
            // 2 / x by the reciprocal estimate and two Newton steps (x > 0)
            double tx = __builtin_amdgcn_rcp(x);
            tx = fma(fma(-x, tx, 1.0), tx, tx);
            tx = 2.0 * fma(fma(-x, tx, 1.0), tx, tx);
            double sn, cs;
            sincos_cw(p.c_re * r[q], sn, cs);
            const double yr = wr[q] * cs, yi = wr[q] * sn;
            double jp = 0.0, jc = 0x1p-1000, S = 2.0 * jc;  // J_{M+1}, J_M (M even, > 0)
            for (int l = M; l > L0 + NOPS; l -= 8) {
                steps8(l, tx, jp, jc, S);
                rescale(jp, jc, S);
            }
            // the block's indices L0 + NOPS - 1 .. L0 (jc is J_{L0+NOPS} here)
            double jb[NOPS];
            double t = (L0 + NOPS) * tx;
#pragma unroll
            for (int j = NOPS - 1; j >= 0; --j) {
                const double jn = fma(t, jc, -jp);
                jp = jc;
                jc = jn;
                t -= tx;
                jb[j] = jc;
                if ((j & 1) == 0) S = fma(2.0, jc, S);  // L0 is even
            }
            double f = 1.0;
            for (int l = L0; l > 0; l -= 8) {
                steps8(l, tx, jp, jc, S);
                f *= rescale(jp, jc, S);
            }
            S -= jc;  // J_0 was counted twice
            const double nrm = f / S;
#pragma unroll
            for (int j = 0; j < NOPS; ++j) {
                const double v = jb[j] * nrm;
                gr[j] = fma(yr, v, gr[j]);
                gi[j] = fma(yi, v, gi[j]);
            }
        }
#pragma unroll
        for (int j = 0; j < NOPS; ++j) out[j] = make_double2(gr[j], gi[j]);
    }
};

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
