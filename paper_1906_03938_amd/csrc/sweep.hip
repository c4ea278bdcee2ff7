// Generate-and-contract sweep: Z_l = T_l V for a group of coefficient operators T_l.
//
// On gfx950 the FP64 MFMA and the FP64 vector ALU share one pipe (they do not overlap),
// so the kernel minimises the total FP64 work per (entry, operator):
//
// * Block = 4 waves (256 threads), all owning the same 16 target rows (the M dimension
//   of v_mfma_f64_16x16x4f64) and 16*CB probe columns; wave w handles the G operators
//   l0 = 4 G blockIdx.z + G w, ..., so a block covers 4 G operators.
// * The K loop runs over the source triangles in stages of kStage = 16.  For a stage the
//   probe rows (Vr, Vi) and Vr + Vi -- read from a zero-padded copy made once per call, so
//   no bounds checks or additions are repeated per block -- and the 7 quadrature points of
//   each triangle are staged in LDS (prefetched into registers during the previous stage).
// * Base phase: thread t computes, for target row t & 15 and source triangle t >> 4 of
//   the stage, the operator-independent part of all 7 quadrature terms (the distance,
//   the weight over 4 pi r, and for the expansion the factor exp(i c r)) once, into LDS.
//   The expensive transcendental work is thus shared by all 4 G operators of the block.
// * Contract phase: per k-step (4 source triangles) lane (i = lane & 15, k = lane >> 4)
//   reads the 7 base terms of entry (row i, triangle 4 ks + k), forms the entries of its
//   wave's G operators -- exactly the A-operand elements it feeds to the MFMA, so
//   generated tiles never reach HBM -- and accumulates with Gauss's three-multiplication
//   complex product: P1 += Gr Vr, P2 += Gi Vi, P3 += (Gr + Gi)(Vr + Vi); at the end
//   Re Z = P1 - P2, Im Z = P3 - P1 - P2.
//
// Operator families (entry of T_l at a != b, summed over the 7 points, with the weight
// A_b w_q / (4 pi) folded into the staged points):
//   Direct: T_l = T(kappa_l):              w/r exp(i kappa_l r)
//   Taylor: T(c + R t) = sum_l t^l T_l:    w/r exp(i c r) (i R r)^l / l!
// The diagonal entry of T_l comes from a precomputed table (exact self terms or their
// expansion coefficients).
#include "devmath.h"
#include "internal.h"

namespace bemrat {

namespace {

typedef double v4d __attribute__((ext_vector_type(4)));

constexpr int kStage = 16;                  // source triangles per stage
constexpr int kStageSteps = kStage / 4;     // k-steps per stage
constexpr int kBase = kQuad * kStage * 16;  // base terms per stage (q, triangle, row)

__device__ __forceinline__ v4d mfma(double a, double b, v4d c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// Base terms of one quadrature point, stored as one double4 per (q, triangle, row):
//   Direct: (r, w/r, -, -)
//   Taylor: (x = R r, y = w/r exp(i c r) (i x)^L0 / L0!) for the block's first operator L0.
template <Gen GEN, bool DECAY>
struct Base;

template <bool DECAY>
struct Base<Gen::Direct, DECAY> {
    __device__ void init(const SweepArgs &, int, int) {}
    __device__ __forceinline__ double4 make(double r, double wr, const SweepArgs &) const {
        return make_double4(r, wr, 0.0, 0.0);
    }
};

template <bool DECAY>
struct Base<Gen::Taylor, DECAY> {
    int L0, z, B;  // L0 = z B: block z of B operators
    double inv_fact;
    __device__ void init(const SweepArgs &p, int L0_, int B_) {
        L0 = L0_;
        B = B_;
        z = L0 / B;
        inv_fact = p.inv_fact[min(L0, kMaxTaylor - 1)];
    }
    __device__ __forceinline__ double4 make(double r, double wr, const SweepArgs &p) const {
        const double e = DECAY ? exp_cw(-p.c_im * r) * wr : wr;
        double s, c;
        sincos_cw(p.c_re * r, s, c);
        const double x = p.R * r;
        // x^L0 / L0! = (x^B)^z / L0!: x^B by squaring (B = 8 or 12), then the at most 4
        // bits of the block-uniform z by selects (no branches)
        const double x2 = x * x, x4 = x2 * x2, x8 = x4 * x4;
        double base = B == 8 ? x8 : x8 * x4;
        double pw = inv_fact;
#pragma unroll
        for (int bit = 0; bit < 4; ++bit) {
            pw = ((z >> bit) & 1) ? pw * base : pw;
            base *= base;
        }
        double yr = e * c * pw, yi = e * s * pw;
        // times i^L0 (L0 is a multiple of 4 when B = 8 or 12: i^L0 = 1) -- kept general
        const double t = yr;
        yr = (L0 & 1) ? -yi : yr;
        yi = (L0 & 1) ? t : yi;
        yr = (L0 & 2) ? -yr : yr;
        yi = (L0 & 2) ? -yi : yi;
        return make_double4(x, yr, yi, 0.0);
    }
};

// Entries of a wave's G operators from the base terms.
template <int G, Gen GEN, bool DECAY>
struct Ops;

template <int G, bool DECAY>
struct Ops<G, Gen::Direct, DECAY> {
    double kr[G], ki[G];
    __device__ void init(const SweepArgs &p, int L0, int wave) {
#pragma unroll
        for (int g = 0; g < G; ++g) {
            const int l = min(L0 + G * wave + g, p.L - 1);
            kr[g] = p.kappa[l].x;
            ki[g] = p.kappa[l].y;
        }
    }
    __device__ __forceinline__ void term(const double4 &b, double (&gr)[G], double (&gi)[G]) const {
        const double r = b.x, wr = b.y;
#pragma unroll
        for (int g = 0; g < G; ++g) {
            const double e = DECAY ? exp_cw(-ki[g] * r) * wr : wr;
            double s, c;
            sincos_cw(kr[g] * r, s, c);
            gr[g] = fma(e, c, gr[g]);
            gi[g] = fma(e, s, gi[g]);
        }
    }
};

// Wave w's operators are l = L0 + G w + g: term = y (i x)^(G w) L0!/(L0 + G w)! then
// times i x / (l + 1) per further operator.
template <int G, bool DECAY>
struct Ops<G, Gen::Taylor, DECAY> {
    static constexpr int kBits = G <= 2 ? 3 : 4;  // bits of the wave offset G w <= 3 G
    int e;                                        // G w (uniform)
    double cw;                                    // i^(G w) L0! / (L0 + G w)! (real: G w even or sign folded below)
    bool rot;                                     // G w odd: one more factor i
    double inv_int[G];
    __device__ void init(const SweepArgs &p, int L0, int wave) {
        e = G * wave;
        double f = 1.0;
        for (int j = 1; j <= e; ++j) f *= p.inv_int[min(L0 + j, kMaxTaylor - 1)];
        // i^e = (-1)^(e/2) for even e, i (-1)^((e-1)/2) for odd e
        cw = ((e >> 1) & 1) ? -f : f;
        rot = e & 1;
#pragma unroll
        for (int g = 0; g < G; ++g) inv_int[g] = p.inv_int[min(L0 + e + g + 1, kMaxTaylor - 1)];
    }
    __device__ __forceinline__ void term(const double4 &b, double (&gr)[G], double (&gi)[G]) const {
        const double x = b.x;
        // x^e with selects (e uniform, at most kBits bits)
        double pw = cw, base = x;
#pragma unroll
        for (int bit = 0; bit < kBits; ++bit) {
            pw = ((e >> bit) & 1) ? pw * base : pw;
            base *= base;
        }
        double tr = b.y * pw, ti = b.z * pw;
        const double t0 = tr;
        tr = rot ? -ti : tr;
        ti = rot ? t0 : ti;
#pragma unroll
        for (int g = 0; g < G; ++g) {
            gr[g] += tr;
            gi[g] += ti;
            const double f = x * inv_int[g];  // next term: times i x / (l + 1)
            const double t = tr;
            tr = -ti * f;
            ti = t * f;
        }
    }
};

template <int G, int CB, Gen GEN, bool DECAY>
__global__ __launch_bounds__(256, 1) void sweep_kernel(SweepArgs p) {
    constexpr int NC = 16 * CB;
    constexpr int VPT = kStage * NC / 256;  // staged probe elements per thread (1, 2, 4)
    constexpr int QN = kStage * kQuad;      // staged points per stage (112)
    // double2 + double arrays keep every LDS read and write free of bank conflicts
    __shared__ double2 sV2[kStage * NC];  // (Vr, Vi)
    __shared__ double sVs[kStage * NC];   // Vr + Vi
    __shared__ double4 sQ[QN];
    __shared__ double2 sB2[kBase];        // base terms [(q * kStage + triangle) * 16 + row]
    __shared__ double sB1[kBase];

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int64_t row0 = (int64_t)blockIdx.x * 16;
    const int64_t col0 = (int64_t)blockIdx.y * NC;
    const int L0 = blockIdx.z * 4 * G;
    const int l0 = L0 + wave * G;

    Base<GEN, DECAY> basef;
    basef.init(p, L0, 4 * G);
    Ops<G, GEN, DECAY> ops;
    ops.init(p, L0, wave);
    // base phase coordinates: row t & 15, stage triangle t >> 4
    const int brow = tid & 15, btri = tid >> 4;
    const double4 xa = p.colloc[row0 + brow];
    // contract phase coordinates
    const int ci = lane & 15, ck = lane >> 4;
    const int64_t arow = row0 + ci;
    double2 self[G];
#pragma unroll
    for (int g = 0; g < G; ++g) self[g] = p.self[(int64_t)min(l0 + g, p.L - 1) * p.n_pad + arow];

    v4d P1[G][CB], P2[G][CB], P3[G][CB];
#pragma unroll
    for (int g = 0; g < G; ++g)
#pragma unroll
        for (int cb = 0; cb < CB; ++cb) {
            P1[g][cb] = v4d{0.0, 0.0, 0.0, 0.0};
            P2[g][cb] = v4d{0.0, 0.0, 0.0, 0.0};
            P3[g][cb] = v4d{0.0, 0.0, 0.0, 0.0};
        }

    // stage staging through registers, from the zero-padded probe copy (n_pad x m_pad)
    double2 rv[VPT];
    double rs[VPT];
    double4 rq = make_double4(0.0, 0.0, 0.0, 0.0);
    const double2 *vsrc2[VPT];
    const double *vsrcs[VPT];
#pragma unroll
    for (int i = 0; i < VPT; ++i) {
        const int idx = tid + 256 * i;
        const int64_t off = (int64_t)(idx / NC) * p.m_pad + col0 + idx % NC;
        vsrc2[i] = p.Vp2 + off;
        vsrcs[i] = p.Vps + off;
    }
    const int64_t vstride = (int64_t)kStage * p.m_pad;
    auto fetch = [&](int64_t st) {
#pragma unroll
        for (int i = 0; i < VPT; ++i) {
            rv[i] = vsrc2[i][st * vstride];
            rs[i] = vsrcs[i][st * vstride];
        }
        if (tid < QN) rq = p.quad[st * kStage * kQuad + tid];
    };
    auto stash = [&]() {
#pragma unroll
        for (int i = 0; i < VPT; ++i) {
            sV2[tid + 256 * i] = rv[i];
            sVs[tid + 256 * i] = rs[i];
        }
        if (tid < QN) sQ[tid] = rq;
    };

    const int64_t nstages = p.n_pad / kStage;
    fetch(0);
    stash();
    __syncthreads();
    for (int64_t st = 0; st < nstages; ++st) {
        const int64_t b0 = st * kStage;
        // base phase
        {
            const bool diag = b0 + btri == row0 + brow;
#pragma unroll
            for (int q = 0; q < kQuad; ++q) {
                const double4 y = sQ[btri * kQuad + q];
                const double dx = xa.x - y.x, dy = xa.y - y.y, dz = xa.z - y.z;
                double r2 = fma(dx, dx, fma(dy, dy, dz * dz));
                r2 = diag ? 1.0 : r2;  // the diagonal is replaced by the self term
                const double rinv = rsqrt(r2);
                const double4 bt = basef.make(r2 * rinv, diag ? 0.0 : y.w * rinv, p);
                sB2[(q * kStage + btri) * 16 + brow] = make_double2(bt.x, bt.y);
                sB1[(q * kStage + btri) * 16 + brow] = bt.z;
            }
        }
        __syncthreads();
        if (st + 1 < nstages) fetch(st + 1);
        // contract phase
#pragma unroll 1
        for (int ks = 0; ks < kStageSteps; ++ks) {
            const int tri = 4 * ks + ck;
            double gr[G], gi[G];
#pragma unroll
            for (int g = 0; g < G; ++g) gr[g] = gi[g] = 0.0;
#pragma unroll
            for (int q = 0; q < kQuad; ++q) {
                const int bi = (q * kStage + tri) * 16 + ci;
                const double2 b2 = sB2[bi];
                ops.term(make_double4(b2.x, b2.y, sB1[bi], 0.0), gr, gi);
            }
            const bool diag = b0 + tri == arow;
            double gs[G];
#pragma unroll
            for (int g = 0; g < G; ++g) {
                gr[g] = diag ? self[g].x : gr[g];
                gi[g] = diag ? self[g].y : gi[g];
                gs[g] = gr[g] + gi[g];
            }
#pragma unroll
            for (int cb = 0; cb < CB; ++cb) {
                const double2 v = sV2[tri * NC + cb * 16 + ci];
                const double vr_ = v.x, vi_ = v.y, vs_ = sVs[tri * NC + cb * 16 + ci];
#pragma unroll
                for (int g = 0; g < G; ++g) {
                    P1[g][cb] = mfma(gr[g], vr_, P1[g][cb]);
                    P2[g][cb] = mfma(gi[g], vi_, P2[g][cb]);
                    P3[g][cb] = mfma(gs[g], vs_, P3[g][cb]);
                }
            }
        }
        __syncthreads();  // stage fully consumed
        if (st + 1 < nstages) {
            stash();
            __syncthreads();
        }
    }

    // D layout of the 16x16x4 f64 MFMA: register i of a lane holds row (lane >> 4) + 4 i,
    // column lane & 15.
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

template <int G, int CB, Gen GEN, bool DECAY>
hipError_t launch_t(const SweepArgs &p, hipStream_t stream) {
    constexpr int NC = 16 * CB;
    dim3 grid((unsigned)(p.n_pad / 16), (unsigned)((p.m + NC - 1) / NC), (unsigned)((p.L + 4 * G - 1) / (4 * G)));
    hipLaunchKernelGGL((sweep_kernel<G, CB, GEN, DECAY>), grid, dim3(256), 0, stream, p);
    return hipGetLastError();
}

// Operators per wave: 3 while the three accumulator sets (12 G CB doubles per lane) leave
// room for the generator, 2 at 64 columns.
template <Gen GEN, bool DECAY>
hipError_t launch_gen(const SweepArgs &p, hipStream_t stream) {
    if (p.m <= 16) return launch_t<3, 1, GEN, DECAY>(p, stream);
    if (p.m <= 32) return launch_t<3, 2, GEN, DECAY>(p, stream);
    return launch_t<2, 4, GEN, DECAY>(p, stream);
}

// Zero-padded copy of the probe block: Vp2[b][c] = (Vr, Vi), Vps[b][c] = Vr + Vi for
// b < n_pad, c < m_pad (zeros outside n x m).
__global__ void prep_probe_kernel(const double2 *__restrict__ V, int64_t ldv, int64_t n, int64_t m,
                                  int64_t n_pad, int64_t m_pad, double2 *__restrict__ Vp2,
                                  double *__restrict__ Vps) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= n_pad * m_pad) return;
    const int64_t b = idx / m_pad, c = idx % m_pad;
    const double2 v = (b < n && c < m) ? V[b * ldv + c] : make_double2(0.0, 0.0);
    Vp2[idx] = v;
    Vps[idx] = v.x + v.y;
}

}  // namespace

int sweep_ops_per_block(int64_t m) { return m <= 32 ? 12 : 8; }

int64_t sweep_m_pad(int64_t m) {
    const int nc = m <= 16 ? 16 : (m <= 32 ? 32 : 64);
    return (m + nc - 1) / nc * nc;
}

hipError_t launch_prep_probe(const double2 *V, int64_t ldv, int64_t n, int64_t m, int64_t n_pad, int64_t m_pad,
                             double2 *Vp2, double *Vps, hipStream_t stream) {
    const int bs = 256;
    const unsigned grid = (unsigned)((n_pad * m_pad + bs - 1) / bs);
    hipLaunchKernelGGL(prep_probe_kernel, dim3(grid), dim3(bs), 0, stream, V, ldv, n, m, n_pad, m_pad, Vp2, Vps);
    return hipGetLastError();
}

hipError_t launch_sweep(Gen gen, const SweepArgs &args, hipStream_t stream) {
    const bool decay = args.decay != 0;
    switch (gen) {
        case Gen::Direct:
            return decay ? launch_gen<Gen::Direct, true>(args, stream) : launch_gen<Gen::Direct, false>(args, stream);
        case Gen::Taylor:
            return decay ? launch_gen<Gen::Taylor, true>(args, stream) : launch_gen<Gen::Taylor, false>(args, stream);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace bemrat
