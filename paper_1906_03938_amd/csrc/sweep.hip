// Generate-and-contract sweep: Z_l = T_l V for a group of coefficient operators T_l.
//
// Block = 4 waves (256 threads) owning 64 target rows (16 per wave, the M dimension of
// v_mfma_f64_16x16x4f64) and 16*CB probe columns, for G consecutive operators l.
// The K loop runs over all source triangles b in chunks of kChunk = 32: a chunk's probe
// rows V[b, cols] and the 7 quadrature points of its triangles are staged in LDS and
// shared by the four waves.  Each k-step covers 4 source triangles; lane
// (i = lane & 15, k = lane >> 4) of a wave generates the entry T_l[row0 + i, b0 + k] of
// the G operators in registers -- exactly the A-operand element it feeds to the MFMA --
// so generated tiles never touch LDS or HBM.  Two blocks run on every CU (one wave of
// each per SIMD): while one wave generates entries on the vector ALU, the other one's
// MFMAs keep the matrix core busy, and a block waiting at a chunk barrier leaves the
// SIMDs to the other block.
//
// Complex product with four real MFMAs: Re += Gr Vr - Gi Vi, Im += Gr Vi + Gi Vr.
//
// Operator generators (entry of T_l at a != b, summed over the 7 points; the weight
// A_b w_q / (4 pi) is folded into the staged points):
//   Direct: T_l = T(kappa_l):              w/r exp(i kappa_l r)
//   Taylor: T(c + R t) = sum_l t^l T_l:    w/r exp(i c r) (i R r)^l / l!
// The diagonal entry of T_l comes from a precomputed table (exact self terms or their
// expansion coefficients).
#include "devmath.h"
#include "internal.h"

namespace bemrat {

namespace {

typedef double v4d __attribute__((ext_vector_type(4)));

__device__ __forceinline__ v4d mfma(double a, double b, v4d c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

template <int G, Gen GEN, bool DECAY>
struct Generator;

// T(kappa_l): w/r exp(-Im(kappa) r) (cos(Re(kappa) r) + i sin(Re(kappa) r))
template <int G, bool DECAY>
struct Generator<G, Gen::Direct, DECAY> {
    double kr[G], ki[G];
    __device__ void init(const SweepArgs &p, int g0) {
#pragma unroll
        for (int g = 0; g < G; ++g) {
            const int l = min(g0 + g, p.L - 1);
            kr[g] = p.kappa[l].x;
            ki[g] = p.kappa[l].y;
        }
    }
    __device__ __forceinline__ void point(double r, double wr, double (&gr)[G], double (&gi)[G]) const {
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

// Taylor terms l0 .. l0+G-1 of exp(i (c + R t) r) in t: w/r exp(i c r) (i R r)^l / l!
template <int G, bool DECAY>
struct Generator<G, Gen::Taylor, DECAY> {
    double cr, ci, R, inv_fact0;
    int l0;
    double inv_int[G];
    __device__ void init(const SweepArgs &p, int g0) {
        cr = p.c_re;
        ci = p.c_im;
        R = p.R;
        l0 = g0;
        inv_fact0 = p.inv_fact[g0];
#pragma unroll
        for (int g = 0; g < G; ++g) inv_int[g] = p.inv_int[min(g0 + g + 1, kMaxTaylor - 1)];
    }
    __device__ __forceinline__ void point(double r, double wr, double (&gr)[G], double (&gi)[G]) const {
        const double e = DECAY ? exp_cw(-ci * r) * wr : wr;
        double s, c;
        sincos_cw(cr * r, s, c);
        const double x = R * r;
        // x^l0 / l0! by binary powering; l0 is uniform across the block, so the bit tests
        // are scalar branches
        double pw = inv_fact0, base = x;
        for (int e2 = l0; e2; e2 >>= 1) {
            if (e2 & 1) pw *= base;
            base *= base;
        }
        const double m = e * pw;
        double tr = m * c, ti = m * s;
        // times i^l0 (uniform)
        if (l0 & 1) {
            const double t = tr;
            tr = -ti;
            ti = t;
        }
        if (l0 & 2) {
            tr = -tr;
            ti = -ti;
        }
#pragma unroll
        for (int g = 0; g < G; ++g) {
            gr[g] += tr;
            gi[g] += ti;
            // next term: times i x / (l0 + g + 1)
            const double f = x * inv_int[g];
            const double t = tr;
            tr = -ti * f;
            ti = t * f;
        }
    }
};

// Entries of the G operators at (a, b) from the 7 staged points of triangle b.
template <int G, class GenT>
__device__ __forceinline__ void generate(const GenT &gen, const double4 *__restrict__ q7, const double4 &xa,
                                         bool diag, const double2 (&self)[G], double (&gr)[G], double (&gi)[G]) {
#pragma unroll
    for (int g = 0; g < G; ++g) gr[g] = gi[g] = 0.0;
#pragma unroll
    for (int q = 0; q < kQuad; ++q) {
        const double4 y = q7[q];
        const double dx = xa.x - y.x, dy = xa.y - y.y, dz = xa.z - y.z;
        double r2 = fma(dx, dx, fma(dy, dy, dz * dz));
        r2 = diag ? 1.0 : r2;  // the diagonal is replaced below; keep it finite
        const double rinv = rsqrt(r2);
        gen.point(r2 * rinv, y.w * rinv, gr, gi);
    }
#pragma unroll
    for (int g = 0; g < G; ++g) {
        gr[g] = diag ? self[g].x : gr[g];
        gi[g] = diag ? self[g].y : gi[g];
    }
}

template <int G, int CB, Gen GEN, bool DECAY>
__global__ __launch_bounds__(256, 2) void sweep_kernel(SweepArgs p) {
    constexpr int NC = 16 * CB;
    constexpr int VPT = kChunk * NC / 256;  // staged probe elements per thread
    constexpr int QN = kChunk * kQuad;      // staged points per chunk (224 <= 256)
    constexpr int KSTEPS = kChunk / 4;
    __shared__ double2 sV[kChunk * NC];
    __shared__ double4 sQ[QN];

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int64_t row0 = (int64_t)blockIdx.x * kRowTile + wave * 16;
    const int64_t a = row0 + (lane & 15);
    const int kq = lane >> 4;
    const int64_t col0 = (int64_t)blockIdx.y * NC;
    const int g0 = blockIdx.z * G;

    Generator<G, GEN, DECAY> gen;
    gen.init(p, g0);
    const double4 xa = p.colloc[a];
    double2 self[G];
#pragma unroll
    for (int g = 0; g < G; ++g) self[g] = p.self[(int64_t)min(g0 + g, p.L - 1) * p.n_pad + a];

    v4d acc_r[G][CB], acc_i[G][CB];
#pragma unroll
    for (int g = 0; g < G; ++g)
#pragma unroll
        for (int cb = 0; cb < CB; ++cb) {
            acc_r[g][cb] = v4d{0.0, 0.0, 0.0, 0.0};
            acc_i[g][cb] = v4d{0.0, 0.0, 0.0, 0.0};
        }

    const int64_t nchunks = p.n_pad / kChunk;
    for (int64_t ch = 0; ch < nchunks; ++ch) {
        const int64_t b0 = ch * kChunk;
        __syncthreads();  // every wave has consumed the previous chunk
#pragma unroll
        for (int i = 0; i < VPT; ++i) {
            const int idx = tid + 256 * i;
            const int r = idx / NC, c = idx % NC;
            const int64_t b = b0 + r, col = col0 + c;
            sV[idx] = (b < p.n && col < p.m) ? p.V[b * p.ldv + col] : make_double2(0.0, 0.0);
        }
        if (tid < QN) sQ[tid] = p.quad[b0 * kQuad + tid];
        __syncthreads();
#pragma unroll 2
        for (int ks = 0; ks < KSTEPS; ++ks) {
            const int bl = 4 * ks + kq;
            double gr[G], gi[G];
            generate<G>(gen, &sQ[bl * kQuad], xa, b0 + bl == a, self, gr, gi);
            double2 v[CB];
#pragma unroll
            for (int cb = 0; cb < CB; ++cb) v[cb] = sV[bl * NC + cb * 16 + (lane & 15)];
            // first the products that start each accumulator's update, then the ones that
            // finish it, so dependent MFMAs are 2 G CB apart
#pragma unroll
            for (int cb = 0; cb < CB; ++cb)
#pragma unroll
                for (int g = 0; g < G; ++g) {
                    acc_r[g][cb] = mfma(gr[g], v[cb].x, acc_r[g][cb]);
                    acc_i[g][cb] = mfma(gi[g], v[cb].x, acc_i[g][cb]);
                }
#pragma unroll
            for (int cb = 0; cb < CB; ++cb)
#pragma unroll
                for (int g = 0; g < G; ++g) {
                    acc_r[g][cb] = mfma(-gi[g], v[cb].y, acc_r[g][cb]);
                    acc_i[g][cb] = mfma(gr[g], v[cb].y, acc_i[g][cb]);
                }
        }
    }

    // D layout of the 16x16x4 f64 MFMA: register i of a lane holds row (lane >> 4) + 4 i,
    // column lane & 15.
#pragma unroll
    for (int g = 0; g < G; ++g) {
        if (g0 + g >= p.L) break;
        double2 *Z = p.Z + (int64_t)(g0 + g) * p.zstride;
#pragma unroll
        for (int cb = 0; cb < CB; ++cb) {
            const int64_t col = col0 + cb * 16 + (lane & 15);
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int64_t row = row0 + kq + 4 * i;
                if (row < p.n && col < p.m) Z[row * p.ldz + col] = make_double2(acc_r[g][cb][i], acc_i[g][cb][i]);
            }
        }
    }
}

template <int G, int CB, Gen GEN, bool DECAY>
hipError_t launch_t(const SweepArgs &p, hipStream_t stream) {
    constexpr int NC = 16 * CB;
    dim3 grid((unsigned)(p.n_pad / kRowTile), (unsigned)((p.m + NC - 1) / NC), (unsigned)((p.L + G - 1) / G));
    hipLaunchKernelGGL((sweep_kernel<G, CB, GEN, DECAY>), grid, dim3(256), 0, stream, p);
    return hipGetLastError();
}

// Two operators per block: the 8 G CB accumulator doubles plus the generator must fit
// the 256 registers a wave gets when two waves share a SIMD.
template <Gen GEN, bool DECAY>
hipError_t launch_gen(const SweepArgs &p, hipStream_t stream) {
    if (p.m <= 16) return launch_t<2, 1, GEN, DECAY>(p, stream);
    if (p.m <= 32) return launch_t<2, 2, GEN, DECAY>(p, stream);
    return launch_t<2, 4, GEN, DECAY>(p, stream);
}

}  // namespace

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
