// Operator-entry generators shared by the FP64 sweep and the reduced-precision sweep:
// for one (target row, source triangle) and the 7 quadrature points, the entries of a block
// of NOPS consecutive coefficient operators (Direct, Taylor or Chebyshev family), in FP64.
// With LOWP (entries bound for a BF16 or FP16 contraction) the sines and cosines come from
// the FP32 hardware after an FP64 reduction (sincos_lowp), 1.2e-7 absolute.
#pragma once

#include <type_traits>

#include "devmath.h"
#include "internal.h"

namespace bemrat {
namespace {

// Loads and stores through the global address space, for pointers read from a table in
// device memory (the batched form): the compiler takes those as generic, and generic (flat)
// accesses also count against the LDS wait counter, so the producers' LDS waits would wait
// for their prefetches too.  Kernel-argument pointers are known to be global already.
typedef double gv2 __attribute__((ext_vector_type(2)));
typedef double gv4 __attribute__((ext_vector_type(4)));
#define BEMRAT_GLOBAL __attribute__((address_space(1)))
__device__ __forceinline__ double gld(const double *p, int64_t i) { return ((const BEMRAT_GLOBAL double *)p)[i]; }
__device__ __forceinline__ double2 gld(const double2 *p, int64_t i) {
    const gv2 v = ((const BEMRAT_GLOBAL gv2 *)p)[i];
    return make_double2(v[0], v[1]);
}
__device__ __forceinline__ double4 gld(const double4 *p, int64_t i) {
    const gv4 v = ((const BEMRAT_GLOBAL gv4 *)p)[i];
    return make_double4(v[0], v[1], v[2], v[3]);
}
__device__ __forceinline__ void gst(double2 *p, int64_t i, double2 v) {
    ((BEMRAT_GLOBAL gv2 *)p)[i] = gv2{v.x, v.y};
}
#undef BEMRAT_GLOBAL

// Memory accesses of a sweep tile: plain for kernel-argument pointers, explicitly global for
// pointers taken from the batched form's table (CAST).
template <bool CAST, class T>
__device__ __forceinline__ T ld(const T *p, int64_t i) {
    if constexpr (CAST) return gld(p, i);
    else return p[i];
}
template <bool CAST>
__device__ __forceinline__ void st(double2 *p, int64_t i, double2 v) {
    if constexpr (CAST) gst(p, i, v);
    else p[i] = v;
}

constexpr int kStage = 16;               // source triangles per stage
constexpr int kStageSteps = kStage / 4;  // k-steps per stage

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
template <int NOPS, Gen GEN, bool DECAY, bool LOWP = false>
struct Generator;

// In FP64 a block whose operators run past L (the last block of a ragged L) generates only
// those below L (the others are zero and never written); a full block takes the unrolled
// loop over all NOPS.
template <int NOPS, bool DECAY, bool LOWP>
struct Generator<NOPS, Gen::Direct, DECAY, LOWP> {
    double kr[NOPS], ki[NOPS];
    int nact;  // operators of the block below L (uniform)
    __device__ void init(const SweepArgs &p, int L0) {
        nact = min(NOPS, p.L - L0);
#pragma unroll
        for (int j = 0; j < NOPS; ++j) {
            const int l = min(L0 + j, p.L - 1);
            kr[j] = p.kappa[l].x;
            ki[j] = p.kappa[l].y;
        }
    }
    __device__ __forceinline__ double2 entry(int j, const double (&r)[kQuad], const double (&wr)[kQuad]) const {
        double gr = 0.0, gi = 0.0;
#pragma unroll
        for (int q = 0; q < kQuad; ++q) {
            const double e = DECAY ? exp_cw(-ki[j] * r[q]) * wr[q] : wr[q];
            double sn, cs;
            sincos_gen<LOWP>(kr[j] * r[q], sn, cs);
            gr = fma(e, cs, gr);
            gi = fma(e, sn, gi);
        }
        return make_double2(gr, gi);
    }
    __device__ __forceinline__ void entries(const double (&r)[kQuad], const double (&wr)[kQuad],
                                            const SweepArgs &, double2 (&out)[NOPS]) const {
        if constexpr (!LOWP) {
            if (nact < NOPS) {
#pragma unroll
                for (int j = 0; j < NOPS; ++j) {
                    out[j] = make_double2(0.0, 0.0);
                    if (j < nact) out[j] = entry(j, r, wr);
                }
                return;
            }
        }
#pragma unroll
        for (int j = 0; j < NOPS; ++j) out[j] = entry(j, r, wr);
    }
};

// Direct form on quadruples of nodes {x + iy, x - iy, x' + iy, x' - iy} (operators 4g .. 4g + 3
// of the block, in that order) whose real parts are mirror images about one centre c on the
// real axis, x' = 2c - x (a circle centred on the real axis with N a multiple of 4 and the
// half-step offset is made of them; c in c_re): per quadrature point the block takes
// exp(2icr) once, and each quadruple one exp(-y r), its reciprocal exp(+y r) (hardware
// estimate and two Newton steps) and the sincos of x r, with exp(i x' r) = exp(2icr) times
// the conjugate of exp(i x r) -- four operators for what one node of the plain direct form
// costs.  Every node is still its own operator, contracted on its own.
template <int NOPS, bool DECAY, bool LOWP>
struct Generator<NOPS, Gen::DirectSym, DECAY, LOWP> {
    static_assert(NOPS % 4 == 0, "whole quadruples per block");
    static constexpr int NQ = NOPS / 4;
    double xa[NQ], y[NQ];
    double c2;
    __device__ void init(const SweepArgs &p, int L0) {
        c2 = 2.0 * p.c_re;
#pragma unroll
        for (int g = 0; g < NQ; ++g) {
            // a quadruple beyond L (L a multiple of 4) repeats the first: its operators are
            // not written
            const int l = L0 + 4 * g < p.L ? L0 + 4 * g : L0;
            xa[g] = p.kappa[l].x;
            y[g] = p.kappa[l].y;
        }
    }
    __device__ __forceinline__ void entries(const double (&r)[kQuad], const double (&wr)[kQuad],
                                            const SweepArgs &, double2 (&out)[NOPS]) const {
        double gr[NOPS], gi[NOPS];
#pragma unroll
        for (int j = 0; j < NOPS; ++j) gr[j] = gi[j] = 0.0;
#pragma unroll
        for (int q = 0; q < kQuad; ++q) {
            double sc, cc;  // exp(2icr)
            sincos_gen<LOWP>(c2 * r[q], sc, cc);
#pragma unroll
            for (int g = 0; g < NQ; ++g) {
                const double E = exp_cw(-y[g] * r[q]);
                double Ei = __builtin_amdgcn_rcp(E);
                Ei = fma(fma(-E, Ei, 1.0), Ei, Ei);
                Ei = fma(fma(-E, Ei, 1.0), Ei, Ei);
                const double e1 = E * wr[q], e2 = Ei * wr[q];
                double s1, c1;
                sincos_gen<LOWP>(xa[g] * r[q], s1, c1);
                const double c2v = fma(cc, c1, sc * s1), s2v = fma(sc, c1, -(cc * s1));
                gr[4 * g] = fma(e1, c1, gr[4 * g]);
                gi[4 * g] = fma(e1, s1, gi[4 * g]);
                gr[4 * g + 1] = fma(e2, c1, gr[4 * g + 1]);
                gi[4 * g + 1] = fma(e2, s1, gi[4 * g + 1]);
                gr[4 * g + 2] = fma(e1, c2v, gr[4 * g + 2]);
                gi[4 * g + 2] = fma(e1, s2v, gi[4 * g + 2]);
                gr[4 * g + 3] = fma(e2, c2v, gr[4 * g + 3]);
                gi[4 * g + 3] = fma(e2, s2v, gi[4 * g + 3]);
            }
        }
#pragma unroll
        for (int j = 0; j < NOPS; ++j) out[j] = make_double2(gr[j], gi[j]);
    }
};

// Term of operator L0 + j at one point: w/r exp(i c r) (i x)^(L0 + j) / (L0 + j)!, x = R r.
// L0 is a multiple of 4, so (i x)^L0 = x^L0; the rest is y0 i^j x^j c_j with
// y0 = w/r exp(i c r) x^L0 / L0! and the block-uniform c_j = L0! / (L0 + j)!, which with
// i^j is applied once to the sum over the points.  The power x^j is a running product, so
// no per-operator factor can be hoisted out of the point loop and kept live.
template <int NOPS, bool DECAY, bool LOWP>
struct Generator<NOPS, Gen::Taylor, DECAY, LOWP> {
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
            sincos_gen<LOWP>(p.c_re * r[q], sn, cs);
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

// Sixteen Taylor operators per block (L0 a multiple of 16) in two passes of eight that share
// each point's distance, exp(i c r) and x^L0 / L0!: after the first pass the point term is
// advanced by x^8 (the chain's last power times x) and the factorial ratios continue, so
// the transcendental work per point is paid once for 16 operators.  When the second half
// lies beyond L (L a multiple of 8) it is skipped and returned as zeros.
template <bool DECAY, bool LOWP>
struct Generator<16, Gen::Taylor, DECAY, LOWP> {
    int z, L0;
    double inv_fact;  // 1 / L0!
    __device__ void init(const SweepArgs &p, int L0_) {
        L0 = L0_;
        z = L0 / 16;
        inv_fact = p.inv_fact[min(L0, kMaxTaylor - 1)];
    }
    __device__ __forceinline__ void entries(const double (&r)[kQuad], const double (&wr)[kQuad],
                                            const SweepArgs &p, double2 (&out)[16]) const {
        double xq[kQuad], yr[kQuad], yi[kQuad];
#pragma unroll
        for (int q = 0; q < kQuad; ++q) {
            const double x = p.R * r[q];
            const double x2 = x * x, x4 = x2 * x2, x8 = x4 * x4;
            double base = x8 * x8, pw = inv_fact;
            for (int zz = z; zz != 0; zz >>= 1) {  // z is uniform: no divergence
                if (zz & 1) pw *= base;
                base *= base;
            }
            const double e = (DECAY ? exp_cw(-p.c_im * r[q]) * wr[q] : wr[q]) * pw;
            double sn, cs;
            sincos_gen<LOWP>(p.c_re * r[q], sn, cs);
            xq[q] = x;
            yr[q] = e * cs;
            yi[q] = e * sn;
        }
        double c = 1.0;  // L0! / (L0 + 8 h + j)!
        const int passes = L0 + 8 < p.L ? 2 : 1;  // uniform over the block
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            if (h >= passes) {
#pragma unroll
                for (int j = 0; j < 8; ++j) out[8 * h + j] = make_double2(0.0, 0.0);
                break;
            }
            double gr[8], gi[8];
#pragma unroll
            for (int j = 0; j < 8; ++j) gr[j] = gi[j] = 0.0;
#pragma unroll
            for (int q = 0; q < kQuad; ++q) {
                const double x = xq[q];
                double xp = x;
                gr[0] += yr[q];
                gi[0] += yi[q];
#pragma unroll
                for (int j = 1; j < 8; ++j) {
                    gr[j] = fma(yr[q], xp, gr[j]);
                    gi[j] = fma(yi[q], xp, gi[j]);
                    xp *= x;
                }
                if (h == 0) {  // advance the point term to x^(L0 + 8)
                    yr[q] *= xp;
                    yi[q] *= xp;
                }
            }
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                if (h + j > 0) c *= p.inv_int[min(L0 + 8 * h + j, kMaxTaylor - 1)];
                const double a = gr[j] * c, b = gi[j] * c;
                switch (j & 3) {  // times i^(8 h + j) = i^j
                    case 0: out[8 * h + j] = make_double2(a, b); break;
                    case 1: out[8 * h + j] = make_double2(-b, a); break;
                    case 2: out[8 * h + j] = make_double2(-a, -b); break;
                    default: out[8 * h + j] = make_double2(b, -a); break;
                }
            }
        }
    }
};

// Folded generators: all p.Lgen operators of one entry, combined into the outputs
// out[k] = sum_l fcoef[l][k] T_l, k < KL (zero beyond, up to NOPS), the coefficients read
// from the block's LDS copy (set_coef), rows of KL (zero from column p.L on).  The Taylor form computes each point's distance, exp(i c r)
// and weight once and runs the power chain through all the operators in passes of eight
// (the point term advanced by x^8 between passes; the factors i^l / l! are in the
// coefficients); the direct form generates its nodes in passes of eight (of quadruples for
// DirectSym).
typedef const __attribute__((address_space(3))) double lds_double;
struct FoldCoef {
    const double2 *fc = nullptr;  // LDS, Lgen rows of the fold width
    __device__ void set_coef(const double2 *c) { fc = c; }
    // the row length: KL, which is p.L for KL <= 2 (taken from the arguments there, which
    // the compiler schedules better, 442 against 489 ms on sphere-81920 with P = 2)
    template <int KL>
    __device__ __forceinline__ static int row(const SweepArgs &p) { return KL <= 2 ? p.L : KL; }
    __device__ __forceinline__ double2 coef(int i) const {
        lds_double *d = (lds_double *)fc;
        return make_double2(d[2 * i], d[2 * i + 1]);
    }
};

template <int NOPS, Gen GEN, bool DECAY, int KL>
struct FoldGenerator;

template <int NOPS, bool DECAY, int KL>
struct FoldGenerator<NOPS, Gen::Taylor, DECAY, KL> : FoldCoef {
    __device__ void init(const SweepArgs &, int) {}
    __device__ __forceinline__ void fold(const SweepArgs &p, int l, double er, double ei, double (&ar)[NOPS],
                                         double (&ai)[NOPS]) const {
#pragma unroll
        for (int k = 0; k < KL; ++k) {
            {
                const double2 w = coef(l * row<KL>(p) + k);
                ar[k] = fma(w.x, er, fma(-w.y, ei, ar[k]));
                ai[k] = fma(w.x, ei, fma(w.y, er, ai[k]));
            }
        }
    }
    __device__ __forceinline__ void entries(const double (&r)[kQuad], const double (&wr)[kQuad],
                                            const SweepArgs &p, double2 (&out)[NOPS]) const {
        double xq[kQuad], yr[kQuad], yi[kQuad];
#pragma unroll
        for (int q = 0; q < kQuad; ++q) {
            const double e = DECAY ? exp_cw(-p.c_im * r[q]) * wr[q] : wr[q];
            double sn, cs;
            sincos_cw(p.c_re * r[q], sn, cs);
            xq[q] = p.R * r[q];
            yr[q] = e * cs;
            yi[q] = e * sn;
        }
        double ar[NOPS], ai[NOPS];
#pragma unroll
        for (int k = 0; k < NOPS; ++k) ar[k] = ai[k] = 0.0;
#pragma unroll 1
        for (int h = 0; h < p.Lgen; h += 8) {  // uniform over the block
            double gr[8], gi[8];
#pragma unroll
            for (int j = 0; j < 8; ++j) gr[j] = gi[j] = 0.0;
#pragma unroll
            for (int q = 0; q < kQuad; ++q) {
                const double x = xq[q];
                double xp = x;
                gr[0] += yr[q];
                gi[0] += yi[q];
#pragma unroll
                for (int j = 1; j < 8; ++j) {
                    gr[j] = fma(yr[q], xp, gr[j]);
                    gi[j] = fma(yi[q], xp, gi[j]);
                    xp *= x;
                }
                yr[q] *= xp;  // x^8: the next pass starts at x^(h + 8)
                yi[q] *= xp;
            }
#pragma unroll
            for (int j = 0; j < 8; ++j) fold(p, h + j, gr[j], gi[j], ar, ai);
        }
#pragma unroll
        for (int k = 0; k < NOPS; ++k) out[k] = make_double2(ar[k], ai[k]);
    }
};

template <int NOPS, bool DECAY, int KL>
struct FoldGenerator<NOPS, Gen::Direct, DECAY, KL> : FoldCoef {
    __device__ void init(const SweepArgs &, int) {}
    __device__ __forceinline__ void entries(const double (&r)[kQuad], const double (&wr)[kQuad],
                                            const SweepArgs &p, double2 (&out)[NOPS]) const {
        double ar[NOPS], ai[NOPS];
#pragma unroll
        for (int k = 0; k < NOPS; ++k) ar[k] = ai[k] = 0.0;
        for (int h = 0; h < p.Lgen; h += 8) {  // uniform over the block
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                if (h + j >= p.Lgen) break;
                const double2 kap = p.kappa[h + j];
                double gr = 0.0, gi = 0.0;
#pragma unroll
                for (int q = 0; q < kQuad; ++q) {
                    const double e = DECAY ? exp_cw(-kap.y * r[q]) * wr[q] : wr[q];
                    double sn, cs;
                    sincos_cw(kap.x * r[q], sn, cs);
                    gr = fma(e, cs, gr);
                    gi = fma(e, sn, gi);
                }
#pragma unroll
                for (int k = 0; k < KL; ++k) {
                    {
                        const double2 w = coef((h + j) * row<KL>(p) + k);
                        ar[k] = fma(w.x, gr, fma(-w.y, gi, ar[k]));
                        ai[k] = fma(w.x, gi, fma(w.y, gr, ai[k]));
                    }
                }
            }
        }
#pragma unroll
        for (int k = 0; k < NOPS; ++k) out[k] = make_double2(ar[k], ai[k]);
    }
};

// Direct form on node quadruples (as Generator<.., DirectSym, ..>), folded: each quadruple's
// four entries are formed with one exp(-y r), its reciprocal and one sincos of x r per point
// (exp(2icr) once per point for the whole entry) and folded with the weights at once.
template <int NOPS, bool DECAY, int KL>
struct FoldGenerator<NOPS, Gen::DirectSym, DECAY, KL> : FoldCoef {
    static_assert(DECAY, "quadruples have Im != 0");
    __device__ void init(const SweepArgs &, int) {}
    __device__ __forceinline__ void fold(const SweepArgs &p, int l, double er, double ei, double (&ar)[NOPS],
                                         double (&ai)[NOPS]) const {
#pragma unroll
        for (int k = 0; k < KL; ++k) {
            {
                const double2 w = coef(l * row<KL>(p) + k);
                ar[k] = fma(w.x, er, fma(-w.y, ei, ar[k]));
                ai[k] = fma(w.x, ei, fma(w.y, er, ai[k]));
            }
        }
    }
    __device__ __forceinline__ void entries(const double (&r)[kQuad], const double (&wr)[kQuad],
                                            const SweepArgs &p, double2 (&out)[NOPS]) const {
        const double c2 = 2.0 * p.c_re;
        double sc[kQuad], cc[kQuad];  // exp(2icr)
#pragma unroll
        for (int q = 0; q < kQuad; ++q) sincos_cw(c2 * r[q], sc[q], cc[q]);
        double ar[NOPS], ai[NOPS];
#pragma unroll
        for (int k = 0; k < NOPS; ++k) ar[k] = ai[k] = 0.0;
        for (int g = 0; g < p.Lgen; g += 4) {  // uniform over the block; Lgen is a multiple of 4
            const double2 kap = p.kappa[g];
            double gr[4], gi[4];
#pragma unroll
            for (int j = 0; j < 4; ++j) gr[j] = gi[j] = 0.0;
#pragma unroll
            for (int q = 0; q < kQuad; ++q) {
                const double E = exp_cw(-kap.y * r[q]);
                double Ei = __builtin_amdgcn_rcp(E);
                Ei = fma(fma(-E, Ei, 1.0), Ei, Ei);
                Ei = fma(fma(-E, Ei, 1.0), Ei, Ei);
                const double e1 = E * wr[q], e2 = Ei * wr[q];
                double s1, c1;
                sincos_cw(kap.x * r[q], s1, c1);
                const double c2v = fma(cc[q], c1, sc[q] * s1), s2v = fma(sc[q], c1, -(cc[q] * s1));
                gr[0] = fma(e1, c1, gr[0]);
                gi[0] = fma(e1, s1, gi[0]);
                gr[1] = fma(e2, c1, gr[1]);
                gi[1] = fma(e2, s1, gi[1]);
                gr[2] = fma(e1, c2v, gr[2]);
                gi[2] = fma(e1, s2v, gi[2]);
                gr[3] = fma(e2, c2v, gr[3]);
                gi[3] = fma(e2, s2v, gi[3]);
            }
#pragma unroll
            for (int j = 0; j < 4; ++j) fold(p, g + j, gr[j], gi[j], ar, ai);
        }
#pragma unroll
        for (int k = 0; k < NOPS; ++k) out[k] = make_double2(ar[k], ai[k]);
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
template <int NOPS, bool DECAY, bool LOWP>
struct Generator<NOPS, Gen::Cheb, DECAY, LOWP> {
    int L0, M;
    __device__ void init(const SweepArgs &p, int L0_) {
        L0 = L0_;
        M = p.miller_M;
    }
    // The points advance in two groups (4 and 3) whose recurrences run side by side, so the
    // serial dependence of each is hidden by the others without running out of registers.
    template <int Q0, int QN>
    __device__ __forceinline__ void group(const double (&r)[kQuad], const double (&wr)[kQuad], const SweepArgs &p,
                                          double (&gr)[NOPS], double (&gi)[NOPS]) const {
        double tx[QN], jp[QN], jc[QN], S[QN], f[QN];
#pragma unroll
        for (int q = 0; q < QN; ++q) {
            const double x = p.R * r[Q0 + q];
            // 2 / x by the reciprocal estimate and two Newton steps (x > 0)
            double t = __builtin_amdgcn_rcp(x);
            t = fma(fma(-x, t, 1.0), t, t);
            tx[q] = 2.0 * fma(fma(-x, t, 1.0), t, t);
            jp[q] = 0.0;        // J_{M+1}
            jc[q] = 0x1p-1000;  // J_M (M even, > 0)
            S[q] = 2.0 * jc[q];
            f[q] = 1.0;
        }
        // eight steps from index l (a multiple of 8) down to l - 8 for every point; S gains
        // 2 J at each even index; then the rescale check
        auto steps8 = [&](int l, bool track) {
#pragma unroll
            for (int q = 0; q < QN; ++q) {
                double t = l * tx[q];
#pragma unroll
                for (int i = 1; i <= 8; ++i) {
                    const double jn = fma(t, jc[q], -jp[q]);  // J_{l-i}
                    jp[q] = jc[q];
                    jc[q] = jn;
                    t -= tx[q];
                    if ((i & 1) == 0) S[q] = fma(2.0, jc[q], S[q]);
                }
                const double sc = fabs(jc[q]) > 0x1p400 ? 0x1p-400 : 1.0;
                jp[q] *= sc;
                jc[q] *= sc;
                S[q] *= sc;
                if (track) f[q] *= sc;
            }
        };
        for (int l = M; l > L0 + NOPS; l -= 8) steps8(l, false);
        // the block's indices L0 + NOPS - 1 .. L0 (jc is J_{L0+NOPS} here)
        double jb[QN][NOPS];
#pragma unroll
        for (int q = 0; q < QN; ++q) {
            double t = (L0 + NOPS) * tx[q];
#pragma unroll
            for (int j = NOPS - 1; j >= 0; --j) {
                const double jn = fma(t, jc[q], -jp[q]);
                jp[q] = jc[q];
                jc[q] = jn;
                t -= tx[q];
                jb[q][j] = jc[q];
                if ((j & 1) == 0) S[q] = fma(2.0, jc[q], S[q]);  // L0 is even
            }
        }
        for (int l = L0; l > 0; l -= 8) steps8(l, true);
#pragma unroll
        for (int q = 0; q < QN; ++q) {
            S[q] -= jc[q];  // J_0 was counted twice
            // f / S by the reciprocal estimate and two Newton steps (S > 0)
            double rs = __builtin_amdgcn_rcp(S[q]);
            rs = fma(fma(-S[q], rs, 1.0), rs, rs);
            rs = fma(fma(-S[q], rs, 1.0), rs, rs);
            const double nrm = f[q] * rs;
            double sn, cs;
            sincos_gen<LOWP>(p.c_re * r[Q0 + q], sn, cs);
            const double yr = wr[Q0 + q] * cs * nrm, yi = wr[Q0 + q] * sn * nrm;
#pragma unroll
            for (int j = 0; j < NOPS; ++j) {
                gr[j] = fma(yr, jb[q][j], gr[j]);
                gi[j] = fma(yi, jb[q][j], gi[j]);
            }
        }
    }
    __device__ __forceinline__ void entries(const double (&r)[kQuad], const double (&wr)[kQuad],
                                            const SweepArgs &p, double2 (&out)[NOPS]) const {
        static_assert(kQuad == 7, "two groups of 4 and 3 points");
        double gr[NOPS], gi[NOPS];
#pragma unroll
        for (int j = 0; j < NOPS; ++j) gr[j] = gi[j] = 0.0;
        group<0, 4>(r, wr, p, gr, gi);
        group<4, 3>(r, wr, p, gr, gi);
#pragma unroll
        for (int j = 0; j < NOPS; ++j) out[j] = make_double2(gr[j], gi[j]);
    }
};

}  // namespace
}  // namespace bemrat
