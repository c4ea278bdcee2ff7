// Reduced-precision sweep: Z_l = T_l V with the contraction on FP32, BF16 or FP16 matrix
// cores and FP32 accumulation.
//
// Same block and pipeline as the FP64 sweep (8 waves; producer waves 0-3 generate the
// entries of stage s + 1 while consumer waves 4-7 contract stage s through double-buffered
// LDS), with these differences:
// * The producer generates in FP64 (the shared generators; on gfx950 FP32 and FP64 vector
//   instructions issue at the same rate when packed FP32 is not used; for BF16 and FP16 the
//   sines and cosines come from the FP32 hardware after an FP64 reduction), with the entry
//   scale a_scale (which keeps them inside the FP16 range) folded into the point weights,
//   and rounds the real part, the imaginary part and their sum (Gauss's
//   three-multiplication product) to the contraction type.  The probe rows are scaled by 1 / max |V| (computed on the device by
//   absmax_kernel before the sweep, so any probe block stays inside the FP16 range) and
//   rounded the same way when staged; the epilogue undoes both scales.
// * Diagonal entries are stored as zero: the exact FP64 self terms are added afterwards by
//   add_diag_kernel (Z_l[a] += T_l[a,a] V[a]), so they never pass through low precision.
// * FP32: v_mfma_f32_16x16x4f32 per k-step of 4 triangles, entries stored [triangle][row].
//   BF16 / FP16: one v_mfma_f32_16x16x16{bf16,f16} per stage of 16 triangles; each lane
//   holds 4 consecutive triangles, so entries are stored [row][triangle] and probe rows
//   [column][triangle].
// * D layout of the FP32-accumulating 16x16 MFMAs (checked on the device): register i of a
//   lane holds row 4 (lane >> 4) + i, column lane & 15.
#include <algorithm>

#include "generators.h"

namespace bemrat {

namespace {

typedef float v4f __attribute__((ext_vector_type(4)));
typedef short v4s __attribute__((ext_vector_type(4)));
typedef _Float16 v4h __attribute__((ext_vector_type(4)));

// FP32 -> BF16 bits, round to nearest even (the hardware conversion on gfx950)
__device__ __forceinline__ short bf16_bits(float f) { return __builtin_bit_cast(short, (__bf16)f); }

template <Prec P>
struct Lp;

template <>
struct Lp<Prec::F32> {
    typedef float T;
    static constexpr bool k16 = false;
    __device__ static T cvt(float v) { return v; }
};

template <>
struct Lp<Prec::BF16> {
    typedef short T;
    typedef v4s V4;
    static constexpr bool k16 = true;
    __device__ static T cvt(float v) { return bf16_bits(v); }
    __device__ static v4f mma(V4 a, V4 b, v4f c) { return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0); }
};

template <>
struct Lp<Prec::F16> {
    typedef _Float16 T;
    typedef v4h V4;
    static constexpr bool k16 = true;
    __device__ static T cvt(float v) { return (_Float16)v; }
    __device__ static v4f mma(V4 a, V4 b, v4f c) { return __builtin_amdgcn_mfma_f32_16x16x16f16(a, b, c, 0, 0, 0); }
};

// Scale applied to the probe block: its largest modulus (the reduction result), or 1 for a
// zero block.
__device__ __forceinline__ double vscale_of(const unsigned long long *vmax) {
    const double m = __longlong_as_double((long long)*vmax);
    return m > 0.0 ? m : 1.0;
}

// LDS index of component c (0: real, 1: imaginary, 2: their sum) of the entry of operator j
// at (row, stage triangle), and of a staged probe value at (stage triangle, column).  The
// 16-bit layouts keep a row's 16 triangles together (the MFMA operand reads 4 of them as one
// 8-byte access) with a row stride of kRow16 = 20 halves (40 bytes): the 16 rows a producer
// wave stores at once then fall on 16 different LDS banks (a 32-byte stride put them on 8,
// measured: 11 bank-conflict cycles per LDS instruction), and the 8-byte reads stay aligned.
constexpr int kRow16 = 20;
template <bool K16>
__device__ __forceinline__ int a_index(int j, int c, int row, int tri) {
    return K16 ? ((j * 3 + c) * 16 + row) * kRow16 + tri : ((j * 3 + c) * kStage + tri) * 16 + row;
}
template <bool K16, int NC>
__device__ __forceinline__ int v_index(int c, int tri, int col) {
    return K16 ? (c * NC + col) * kRow16 + tri : (c * kStage + tri) * NC + col;
}

// LDS of one tile: double-buffered entries (3 components per operator), probe rows and
// quadrature points.
template <Prec P, int G, int CB>
struct LpLds {
    typedef typename Lp<P>::T T;
    static constexpr int R = Lp<P>::k16 ? kRow16 : kStage;  // elements per row of 16 triangles
    __attribute__((aligned(16))) T sA[2][4 * G * 3 * R * 16];
    __attribute__((aligned(16))) T sV[2][3 * R * 16 * CB];
    double4 sQ[2][kStage * kQuad];
};

// One tile: 16 target rows from row0, 16 CB columns from col0, operators L0 .. L0 + 4 G - 1,
// by the 512 threads of the block (per-call kernel: one tile per block; batched kernel: tiles
// of several meshes from a work queue, CAST = accesses through the global address space).
template <Prec P, int G, int CB, Gen GEN, bool DECAY, bool CAST>
__device__ __forceinline__ void sweep_lp_tile(const SweepArgs &p, int64_t row0, int64_t col0, int L0,
                                              LpLds<P, G, CB> &lds) {
    typedef Lp<P> LP;
    constexpr bool K16 = LP::k16;
    constexpr int NC = 16 * CB;
    constexpr int NOPS = 4 * G;
    constexpr int VPT = kStage * NC / 256;
    auto &sA = lds.sA;
    auto &sV = lds.sV;
    auto &sQ = lds.sQ;

    const int tid = threadIdx.x;
    const int64_t nstages = p.n_pad / kStage;

    if (tid < 256) {
        // ---- producer: thread t generates row t & 15, stage triangle t >> 4
        constexpr int QN = kStage * kQuad;
        const int brow = tid & 15, btri = tid >> 4;
        const int64_t grow = row0 + brow;
        const double4 xa = ld<CAST>(p.colloc, grow);
        const double scale = p.a_scale;
        const float vs = (float)(1.0 / vscale_of(p.vmax));
        Generator<NOPS, GEN, DECAY, P != Prec::F32> gen;
        gen.init(p, L0);
        // staged probe element i of this thread: stage triangle (tid + 256 i) / NC, column
        // tid % NC (256 is a multiple of NC); kept in FP32, as it is rounded anyway
        static_assert(256 % NC == 0, "a producer pass covers whole rows");
        const double2 *vbase = p.Vp2 + (int64_t)(tid / NC) * p.m_pad + col0 + tid % NC;
        const int64_t vstep = (int64_t)(256 / NC) * p.m_pad;
        const int64_t vstride = (int64_t)kStage * p.m_pad;
        float2 rv[VPT];
#pragma unroll
        for (int i = 0; i < VPT; ++i) {
            const double2 v = ld<CAST>(vbase, i * vstep);
            rv[i] = make_float2((float)v.x, (float)v.y);
        }
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
                for (int i = 0; i < VPT; ++i) {
                    const int idx = tid + 256 * i;
                    const int tri = idx / NC, col = idx % NC;
                    const float vr = rv[i].x * vs, vi = rv[i].y * vs;
                    sV[buf][v_index<K16, NC>(0, tri, col)] = LP::cvt(vr);
                    sV[buf][v_index<K16, NC>(1, tri, col)] = LP::cvt(vi);
                    sV[buf][v_index<K16, NC>(2, tri, col)] = LP::cvt(vr + vi);
                }
                if (tid < QN && it + 1 < nstages) sQ[buf ^ 1][tid] = rq;
                const bool diag = it * kStage + btri == grow;
                // the entry scale rides on the point weights (every generator is linear in
                // them); the diagonal gets weight 0 (it is added in FP64 afterwards)
                const double s = diag ? 0.0 : scale;
                double r[kQuad], wr[kQuad];
#pragma unroll
                for (int q = 0; q < kQuad; ++q) {
                    const double4 y = sQ[buf][btri * kQuad + q];
                    const double dx = xa.x - y.x, dy = xa.y - y.y, dz = xa.z - y.z;
                    double r2 = fma(dx, dx, fma(dy, dy, dz * dz));
                    r2 = diag ? 1.0 : r2;
                    const double rinv = rsqrt_pos(r2);
                    r[q] = r2 * rinv;
                    wr[q] = y.w * s * rinv;
                }
                if (it + 1 < nstages) {
#pragma unroll
                    for (int i = 0; i < VPT; ++i) {
                        const double2 v = ld<CAST>(vbase, i * vstep + (it + 1) * vstride);
                        rv[i] = make_float2((float)v.x, (float)v.y);
                    }
                }
                if (tid < QN && it + 2 < nstages) rq = ld<CAST>(p.quad, (it + 2) * QN + tid);
                double2 a[NOPS];
                gen.entries(r, wr, p, a);
#pragma unroll
                for (int j = 0; j < NOPS; ++j) {
                    const float ar = (float)a[j].x, ai = (float)a[j].y;
                    sA[buf][a_index<K16>(j, 0, brow, btri)] = LP::cvt(ar);
                    sA[buf][a_index<K16>(j, 1, brow, btri)] = LP::cvt(ai);
                    sA[buf][a_index<K16>(j, 2, brow, btri)] = LP::cvt(ar + ai);
                }
            }
            __syncthreads();
        }
    } else {
        // ---- consumer: wave w contracts operators L0 + G w ... of stage it - 1
        const int w = (tid >> 6) - 4;
        const int lane = tid & 63;
        const int ci = lane & 15, ck = lane >> 4;
        v4f P1[G][CB], P2[G][CB], P3[G][CB];
#pragma unroll
        for (int g = 0; g < G; ++g)
#pragma unroll
            for (int cb = 0; cb < CB; ++cb) {
                P1[g][cb] = v4f{0.f, 0.f, 0.f, 0.f};
                P2[g][cb] = v4f{0.f, 0.f, 0.f, 0.f};
                P3[g][cb] = v4f{0.f, 0.f, 0.f, 0.f};
            }
        __syncthreads();  // pairs with the producers' prologue barrier
        for (int64_t it = 0; it <= nstages; ++it) {
            if (it >= 1) {
                const int buf = (int)((it - 1) & 1);
                if constexpr (K16) {
                    typedef typename LP::V4 V4;
                    // lane (ci, ck) holds triangles 4 ck .. 4 ck + 3 of the stage
                    V4 ga[G][3];
#pragma unroll
                    for (int g = 0; g < G; ++g)
#pragma unroll
                        for (int c = 0; c < 3; ++c)
                            ga[g][c] = *reinterpret_cast<const V4 *>(&sA[buf][a_index<true>(w * G + g, c, ci, 4 * ck)]);
#pragma unroll
                    for (int cb = 0; cb < CB; ++cb) {
                        V4 vb[3];
#pragma unroll
                        for (int c = 0; c < 3; ++c)
                            vb[c] = *reinterpret_cast<const V4 *>(&sV[buf][v_index<true, NC>(c, 4 * ck, cb * 16 + ci)]);
#pragma unroll
                        for (int g = 0; g < G; ++g) {
                            P1[g][cb] = LP::mma(ga[g][0], vb[0], P1[g][cb]);
                            P2[g][cb] = LP::mma(ga[g][1], vb[1], P2[g][cb]);
                            P3[g][cb] = LP::mma(ga[g][2], vb[2], P3[g][cb]);
                        }
                    }
                } else {
#pragma unroll 2
                    for (int ks = 0; ks < kStageSteps; ++ks) {
                        const int tri = 4 * ks + ck;
                        float ga[G][3];
#pragma unroll
                        for (int g = 0; g < G; ++g)
#pragma unroll
                            for (int c = 0; c < 3; ++c) ga[g][c] = sA[buf][a_index<false>(w * G + g, c, ci, tri)];
#pragma unroll
                        for (int cb = 0; cb < CB; ++cb) {
                            float vb[3];
#pragma unroll
                            for (int c = 0; c < 3; ++c) vb[c] = sV[buf][v_index<false, NC>(c, tri, cb * 16 + ci)];
#pragma unroll
                            for (int g = 0; g < G; ++g) {
                                P1[g][cb] = __builtin_amdgcn_mfma_f32_16x16x4f32(ga[g][0], vb[0], P1[g][cb], 0, 0, 0);
                                P2[g][cb] = __builtin_amdgcn_mfma_f32_16x16x4f32(ga[g][1], vb[1], P2[g][cb], 0, 0, 0);
                                P3[g][cb] = __builtin_amdgcn_mfma_f32_16x16x4f32(ga[g][2], vb[2], P3[g][cb], 0, 0, 0);
                            }
                        }
                    }
                }
            }
            __syncthreads();
        }
        const double inv = vscale_of(p.vmax) / p.a_scale;
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
                    const int64_t row = row0 + 4 * ck + i;
                    const double p1 = P1[g][cb][i], p2 = P2[g][cb][i], p3 = P3[g][cb][i];
                    if (row < p.n && col < p.m)
                        st<CAST>(Z, row * p.ldz + col, make_double2((p1 - p2) * inv, (p3 - p1 - p2) * inv));
                }
            }
        }
    }
}

template <Prec P, int G, int CB, Gen GEN, bool DECAY>
__global__ __launch_bounds__(512, 1) void sweep_lp_kernel(SweepArgs p) {
    __shared__ LpLds<P, G, CB> lds;
    sweep_lp_tile<P, G, CB, GEN, DECAY, false>(p, (int64_t)blockIdx.x * 16, (int64_t)blockIdx.y * 16 * CB,
                                               (int)blockIdx.z * 4 * G, lds);
}

// Persistent batched form at reduced precision: as sweep_batch_kernel (work items
// (mesh, row block, column block, operator block) from a queue cleared by a kernel, one
// operator family per launch), with each mesh's entry scale and probe scale in its table
// entry.
template <Prec P, int G, int CB, Gen GEN, bool DECAY>
__global__ __launch_bounds__(512, 1) void sweep_lp_batch_kernel(const BatchEntry *__restrict__ table,
                                                                const int4 *__restrict__ items, int nitems,
                                                                unsigned *__restrict__ counter) {
    __shared__ LpLds<P, G, CB> lds;
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
        sweep_lp_tile<P, G, CB, GEN, DECAY, true>(p, (int64_t)__builtin_amdgcn_readfirstlane(item.y) * 16,
                                                  (int64_t)__builtin_amdgcn_readfirstlane(item.z) * 16 * CB,
                                                  __builtin_amdgcn_readfirstlane(item.w) * 4 * G, lds);
    }
}

__global__ void lp_batch_reset_kernel(unsigned *counter) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *counter = 0u;
}

// *out = max over the n x m block of max(|Re v|, |Im v|), as the bits of a non-negative
// double (which order like unsigned integers, so a device-wide atomicMax reduces them).
// *out must be zero beforehand (absmax_clear_kernel).
__global__ void absmax_clear_kernel(unsigned long long *out) { *out = 0ull; }

__global__ void absmax_kernel(const double2 *__restrict__ V, int64_t ldv, int64_t n, int64_t m,
                              unsigned long long *out) {
    __shared__ double red[256];
    double mx = 0.0;
    const int64_t total = n * m;
    for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
         idx += (int64_t)gridDim.x * blockDim.x) {
        const double2 v = V[(idx / m) * ldv + idx % m];
        mx = fmax(mx, fmax(fabs(v.x), fabs(v.y)));
    }
    red[threadIdx.x] = mx;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + s]);
        __syncthreads();
    }
    if (threadIdx.x == 0) atomicMax(out, (unsigned long long)__double_as_longlong(red[0]));
}

// Z_l[a][c] += S_l[a] V[a][c]: the FP64 diagonal (self-term) contribution.
__global__ void add_diag_kernel(const double2 *__restrict__ S, int64_t n_pad, const double2 *__restrict__ V,
                                int64_t ldv, double2 *__restrict__ Z, int64_t ldz, int64_t zstride, int64_t n,
                                int64_t m) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int l = blockIdx.y;
    if (idx >= n * m) return;
    const int64_t a = idx / m, c = idx % m;
    const double2 s = S[(int64_t)l * n_pad + a], v = V[a * ldv + c];
    double2 &z = Z[(int64_t)l * zstride + a * ldz + c];
    z.x += s.x * v.x - s.y * v.y;
    z.y += s.x * v.y + s.y * v.x;
}

template <Prec P, int G, int CB, Gen GEN, bool DECAY>
hipError_t launch_lp_t(const SweepArgs &p, hipStream_t stream) {
    constexpr int NC = 16 * CB;
    constexpr int NOPS = 4 * G;
    dim3 grid((unsigned)(p.n_pad / 16), (unsigned)((p.m + NC - 1) / NC), (unsigned)((p.L + NOPS - 1) / NOPS));
    hipLaunchKernelGGL((sweep_lp_kernel<P, G, CB, GEN, DECAY>), grid, dim3(512), 0, stream, p);
    return hipGetLastError();
}

// Block shape: 16 CB columns with CB = 1, 2, 4 or 8 by the column count (FP32 accumulators
// leave room for 8 column blocks of 2 operators per consumer wave), and 4 operators per
// consumer wave for the direct form up to 64 columns (its generation shares little across
// operators); otherwise 2.  The matrix work is cheap at these precisions, so each block
// amortises its generation (for the expansion forms, the per-point Bessel or power
// sequence) over as many operators and columns as the registers allow.
int lp_cb(int64_t m) { return m <= 16 ? 1 : m <= 32 ? 2 : m <= 64 ? 4 : 8; }
int lp_g(Gen gen, int64_t m) { return (gen == Gen::Direct || gen == Gen::DirectSym) && lp_cb(m) <= 4 ? 4 : 2; }

template <Prec P, Gen GEN, bool DECAY>
hipError_t launch_lp_gen(const SweepArgs &p, hipStream_t stream) {
    constexpr int G = GEN == Gen::Direct || GEN == Gen::DirectSym ? 4 : 2;  // lp_g up to 64 columns
    switch (lp_cb(p.m)) {
        case 1: return launch_lp_t<P, G, 1, GEN, DECAY>(p, stream);
        case 2: return launch_lp_t<P, G, 2, GEN, DECAY>(p, stream);
        case 4: return launch_lp_t<P, G, 4, GEN, DECAY>(p, stream);
        default: return launch_lp_t<P, 2, 8, GEN, DECAY>(p, stream);
    }
}

template <Prec P>
hipError_t launch_lp_prec(Gen gen, const SweepArgs &args, hipStream_t stream) {
    const bool decay = args.decay != 0;
    switch (gen) {
        case Gen::Direct:
            return decay ? launch_lp_gen<P, Gen::Direct, true>(args, stream)
                         : launch_lp_gen<P, Gen::Direct, false>(args, stream);
        case Gen::Taylor:
            return decay ? launch_lp_gen<P, Gen::Taylor, true>(args, stream)
                         : launch_lp_gen<P, Gen::Taylor, false>(args, stream);
        case Gen::Cheb:
            return decay ? hipErrorInvalidValue : launch_lp_gen<P, Gen::Cheb, false>(args, stream);
        case Gen::DirectSym:
            return decay ? launch_lp_gen<P, Gen::DirectSym, true>(args, stream) : hipErrorInvalidValue;
        default: return hipErrorInvalidValue;
    }
}

template <Prec P, int G, int CB, Gen GEN, bool DECAY>
hipError_t launch_lp_batch_t(const BatchEntry *table, const int4 *items, int nitems, unsigned *counter, int grid,
                             hipStream_t stream) {
    hipLaunchKernelGGL((sweep_lp_batch_kernel<P, G, CB, GEN, DECAY>), dim3(grid), dim3(512), 0, stream, table, items,
                       nitems, counter);
    return hipGetLastError();
}

// Direct (with decay: complex nodes) and Taylor families; the operator-per-wave count G
// follows lp_g: 4 for the direct form up to 64 columns, else 2.
template <Prec P>
hipError_t launch_lp_batch_prec(int variant, int cb, const BatchEntry *table, const int4 *items, int nitems,
                                unsigned *counter, int grid, hipStream_t stream) {
#define BEMRAT_LP_BATCH_CB(GEN, DECAY, G4)                                                                      \
    switch (cb) {                                                                                             \
        case 1: return launch_lp_batch_t<P, G4, 1, GEN, DECAY>(table, items, nitems, counter, grid, stream);  \
        case 2: return launch_lp_batch_t<P, G4, 2, GEN, DECAY>(table, items, nitems, counter, grid, stream);  \
        case 4: return launch_lp_batch_t<P, G4, 4, GEN, DECAY>(table, items, nitems, counter, grid, stream);  \
        case 8: return launch_lp_batch_t<P, 2, 8, GEN, DECAY>(table, items, nitems, counter, grid, stream);   \
        default: return hipErrorInvalidValue;                                                                 \
    }
    switch (variant) {
        case kBatchDirectDecay: BEMRAT_LP_BATCH_CB(Gen::Direct, true, 4)
        case kBatchDirect: BEMRAT_LP_BATCH_CB(Gen::Direct, false, 4)
        case kBatchTaylorDecay: BEMRAT_LP_BATCH_CB(Gen::Taylor, true, 2)
        case kBatchTaylor: BEMRAT_LP_BATCH_CB(Gen::Taylor, false, 2)
        case kBatchDirectSym: BEMRAT_LP_BATCH_CB(Gen::DirectSym, true, 4)
        default: return hipErrorInvalidValue;
    }
#undef BEMRAT_LP_BATCH_CB
}

}  // namespace

int sweep_lp_ops_per_block(Gen gen, int64_t m) { return 4 * lp_g(gen, m); }

int lp_batch_col_tile(int64_t m) { return lp_cb(m); }

int lp_batch_ops_per_block(Gen gen, int cb) { return (gen == Gen::Direct || gen == Gen::DirectSym) && cb <= 4 ? 16 : 8; }

hipError_t launch_sweep_lp_batch(Prec prec, int variant, int cb, const BatchEntry *table, const int4 *items,
                                 int nitems, unsigned *counter, int grid, hipStream_t stream) {
    if (grid < 1 || nitems < 0) return hipErrorInvalidValue;
    hipLaunchKernelGGL(lp_batch_reset_kernel, dim3(1), dim3(64), 0, stream, counter);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    switch (prec) {
        case Prec::F32: return launch_lp_batch_prec<Prec::F32>(variant, cb, table, items, nitems, counter, grid, stream);
        case Prec::BF16: return launch_lp_batch_prec<Prec::BF16>(variant, cb, table, items, nitems, counter, grid, stream);
        case Prec::F16: return launch_lp_batch_prec<Prec::F16>(variant, cb, table, items, nitems, counter, grid, stream);
        default: return hipErrorInvalidValue;
    }
}

int64_t sweep_lp_m_pad(int64_t m) {
    const int64_t nc = 16 * lp_cb(m);
    return (m + nc - 1) / nc * nc;
}

hipError_t launch_sweep_lp(Prec prec, Gen gen, const SweepArgs &args, hipStream_t stream) {
    switch (prec) {
        case Prec::F32: return launch_lp_prec<Prec::F32>(gen, args, stream);
        case Prec::BF16: return launch_lp_prec<Prec::BF16>(gen, args, stream);
        case Prec::F16: return launch_lp_prec<Prec::F16>(gen, args, stream);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_absmax(const double2 *V, int64_t ldv, int64_t n, int64_t m, unsigned long long *out,
                         hipStream_t stream) {
    hipLaunchKernelGGL(absmax_clear_kernel, dim3(1), dim3(1), 0, stream, out);
    const int64_t blocks = std::min<int64_t>(1024, (n * m + 255) / 256);
    hipLaunchKernelGGL(absmax_kernel, dim3((unsigned)std::max<int64_t>(blocks, 1)), dim3(256), 0, stream, V, ldv, n, m,
                       out);
    return hipGetLastError();
}

hipError_t launch_add_diag(const double2 *S, int64_t n_pad, const double2 *V, int64_t ldv, double2 *Z, int64_t ldz,
                           int64_t zstride, int64_t n, int64_t m, int L, hipStream_t stream) {
    const int bs = 256;
    dim3 grid((unsigned)((n * m + bs - 1) / bs), (unsigned)L);
    hipLaunchKernelGGL(add_diag_kernel, grid, dim3(bs), 0, stream, S, n_pad, V, ldv, Z, ldz, zstride, n, m);
    return hipGetLastError();
}

}  // namespace bemrat
