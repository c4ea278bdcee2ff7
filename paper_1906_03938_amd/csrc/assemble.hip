// Dense assembly of a node combination S = sum_j c_j T(z_j) (the Schur complement of the
// Cauchy linearisation, or the matrix G of the Chebyshev inverse iteration), for the
// factorisation the host driver's inverse iteration solves with.  Every entry is
// generated once, from the same generated operators T_l as the sweep, combined with the
// coefficients d_l = sum_j c_j Cf[j][l] of the node recombination:
//     S[a][b] = sum_l d_l T_l[a][b]   (a != b),   S[a][a] = sum_l d_l self_l[a].
// One thread per entry, 16 x 16 entries per block; generation-bound (no contraction), and
// the n^2 complex outputs are written once, coalesced along the row.
#include "generators.h"

namespace bemrat {

namespace {

constexpr int kAsmOps = 8;  // operators generated per pass (the sweep's block size)

template <Gen GEN, bool DECAY>
__global__ __launch_bounds__(256) void assemble_sum_kernel(SweepArgs p, const double2 *__restrict__ d,
                                                           double2 *__restrict__ S, int64_t lds) {
    const int64_t a = (int64_t)blockIdx.y * 16 + (threadIdx.x >> 4);
    const int64_t b = (int64_t)blockIdx.x * 16 + (threadIdx.x & 15);
    if (a >= p.n || b >= p.n) return;  // no barriers below
    double sr = 0.0, si = 0.0;
    if (a == b) {
        for (int l = 0; l < p.L; ++l) {
            const double2 s = p.self[(int64_t)l * p.n_pad + a], c = d[l];
            sr += c.x * s.x - c.y * s.y;
            si += c.x * s.y + c.y * s.x;
        }
    } else {
        const double4 xa = p.colloc[a];
        double r[kQuad], wr[kQuad];
#pragma unroll
        for (int q = 0; q < kQuad; ++q) {
            const double4 y = p.quad[b * kQuad + q];
            const double dx = xa.x - y.x, dy = xa.y - y.y, dz = xa.z - y.z;
            const double r2 = fma(dx, dx, fma(dy, dy, dz * dz));
            const double rinv = rsqrt_pos(r2);
            r[q] = r2 * rinv;
            wr[q] = y.w * rinv;
        }
        for (int L0 = 0; L0 < p.L; L0 += kAsmOps) {
            Generator<kAsmOps, GEN, DECAY> gen;
            gen.init(p, L0);
            double2 e[kAsmOps];
            gen.entries(r, wr, p, e);
#pragma unroll
            for (int j = 0; j < kAsmOps; ++j) {
                if (L0 + j < p.L) {
                    const double2 c = d[L0 + j];
                    sr += c.x * e[j].x - c.y * e[j].y;
                    si += c.x * e[j].y + c.y * e[j].x;
                }
            }
        }
    }
    S[a * lds + b] = make_double2(sr, si);
}

template <Gen GEN, bool DECAY>
hipError_t launch_asm(const SweepArgs &p, const double2 *d, double2 *S, int64_t lds, hipStream_t stream) {
    const int64_t blocks = (p.n + 15) / 16;
    dim3 grid((unsigned)blocks, (unsigned)blocks);
    hipLaunchKernelGGL((assemble_sum_kernel<GEN, DECAY>), grid, dim3(256), 0, stream, p, d, S, lds);
    return hipGetLastError();
}

}  // namespace

int assemble_ops_per_block() { return kAsmOps; }

hipError_t launch_assemble_sum(Gen gen, const SweepArgs &p, const double2 *d, double2 *S, int64_t lds,
                               hipStream_t stream) {
    if (p.n > (int64_t)65535 * 16) return hipErrorInvalidValue;  // grid.y limit
    const bool decay = p.decay != 0;
    switch (gen) {
        case Gen::Direct: return decay ? launch_asm<Gen::Direct, true>(p, d, S, lds, stream)
                                       : launch_asm<Gen::Direct, false>(p, d, S, lds, stream);
        case Gen::Taylor: return decay ? launch_asm<Gen::Taylor, true>(p, d, S, lds, stream)
                                       : launch_asm<Gen::Taylor, false>(p, d, S, lds, stream);
        case Gen::Cheb: return decay ? hipErrorInvalidValue : launch_asm<Gen::Cheb, false>(p, d, S, lds, stream);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace bemrat
