// Geometry staging and exact self terms on the device.
//
// prepare_mesh: per triangle, area, centroid (collocation point), the seven mapped points
// of Radon's degree-5 rule with physical weight A_b w_q / (4 pi) folded in.
//
// self_terms: T_aa(kappa) = int over triangle a of exp(i kappa |x_a - y|)/(4 pi |x_a - y|),
// written in polar coordinates around the centroid x_a.  Along direction theta the
// triangle extends to rho(theta) = d_e / cos(phi) (edge e at distance d_e, phi measured
// from the foot of the perpendicular), and int_0^rho exp(i kappa t) dt =
// (exp(i kappa rho) - 1)/(i kappa), so
//   T_aa = 1/(4 pi) sum_e int_{phi_e-}^{phi_e+} rho(phi) E(i kappa rho(phi)) dphi,
//   E(w) = (e^w - 1)/w,
// integrated with kSelfGL-point Gauss-Legendre per edge.  E is evaluated by its Taylor
// series for |w| < 1/4 and through expm1 otherwise, so no cancellation occurs at small
// kappa rho.
#include "devmath.h"
#include "internal.h"

namespace bemrat {

namespace {

__global__ void prepare_mesh_kernel(const double *__restrict__ xyz, const int32_t *__restrict__ tri,
                                    int64_t n, int64_t n_pad, DeviceMesh mesh,
                                    const double *__restrict__ rule) {
    const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= n_pad) return;
    const double inv4pi = 0.25 / 3.14159265358979323846;
    const int64_t src = b < n ? b : 0;  // pads reuse triangle 0's points with zero weight
    double P[3][3];
    for (int v = 0; v < 3; ++v) {
        const int64_t id = tri[3 * src + v];
        for (int c = 0; c < 3; ++c) P[v][c] = xyz[3 * id + c];
    }
    const double e1x = P[1][0] - P[0][0], e1y = P[1][1] - P[0][1], e1z = P[1][2] - P[0][2];
    const double e2x = P[2][0] - P[0][0], e2y = P[2][1] - P[0][1], e2z = P[2][2] - P[0][2];
    const double cx = e1y * e2z - e1z * e2y, cy = e1z * e2x - e1x * e2z, cz = e1x * e2y - e1y * e2x;
    const double A = 0.5 * sqrt(cx * cx + cy * cy + cz * cz);
    const double gx = (P[0][0] + P[1][0] + P[2][0]) / 3.0;
    const double gy = (P[0][1] + P[1][1] + P[2][1]) / 3.0;
    const double gz = (P[0][2] + P[1][2] + P[2][2]) / 3.0;
    mesh.colloc[b] = make_double4(gx, gy, gz, 0.0);
    for (int q = 0; q < kQuad; ++q) {
        // pads: every point is quadrature point 1 of triangle 0 (never a collocation point)
        const int qq = b < n ? q : 1;
        const double l0 = rule[3 * qq], l1 = rule[3 * qq + 1], l2 = rule[3 * qq + 2];
        const double px = l0 * P[0][0] + l1 * P[1][0] + l2 * P[2][0];
        const double py = l0 * P[0][1] + l1 * P[1][1] + l2 * P[2][1];
        const double pz = l0 * P[0][2] + l1 * P[1][2] + l2 * P[2][2];
        const double w = b < n ? A * rule[21 + q] * inv4pi : 0.0;
        mesh.quad[b * kQuad + q] = make_double4(px, py, pz, w);
    }
    for (int v = 0; v < 3; ++v)
        for (int c = 0; c < 3; ++c) mesh.vtx[9 * b + 3 * v + c] = b < n ? P[v][c] : 0.0;
    mesh.area[b] = b < n ? A : 0.0;
}

__global__ void self_terms_kernel(const double *__restrict__ vtx, const double *__restrict__ gl,
                                  int64_t n, int64_t n_pad, const double2 *__restrict__ kappa,
                                  int64_t nk, double2 *__restrict__ S, int64_t lds) {
    const int64_t a = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t k = blockIdx.y;
    if (a >= n_pad || k >= nk) return;
    if (a >= n) {
        S[k * lds + a] = make_double2(0.0, 0.0);
        return;
    }
    const double kr = kappa[k].x, ki = kappa[k].y;
    double P[3][3];
    for (int v = 0; v < 3; ++v)
        for (int c = 0; c < 3; ++c) P[v][c] = vtx[9 * a + 3 * v + c];
    double x[3];
    for (int c = 0; c < 3; ++c) x[c] = (P[0][c] + P[1][c] + P[2][c]) / 3.0;
    double tr = 0.0, ti = 0.0;
    for (int e = 0; e < 3; ++e) {
        const double *A = P[e], *B = P[(e + 1) % 3];
        double t[3], len2 = 0.0;
        for (int c = 0; c < 3; ++c) {
            t[c] = B[c] - A[c];
            len2 += t[c] * t[c];
        }
        const double len = sqrt(len2);
        for (int c = 0; c < 3; ++c) t[c] /= len;
        double s = 0.0;
        for (int c = 0; c < 3; ++c) s += (x[c] - A[c]) * t[c];
        double d2 = 0.0;
        for (int c = 0; c < 3; ++c) {
            const double f = A[c] + s * t[c] - x[c];
            d2 += f * f;
        }
        const double d = sqrt(d2);
        const double p0 = atan2(-s, d), p1 = atan2(len - s, d);
        const double half = 0.5 * (p1 - p0), mid = 0.5 * (p1 + p0);
        double er = 0.0, ei = 0.0;
        for (int i = 0; i < kSelfGL; ++i) {
            const double phi = mid + half * gl[i];
            const double rho = d / cos(phi);
            // w = i kappa rho
            const double2 E = exprel(-ki * rho, kr * rho);
            er += gl[kSelfGL + i] * rho * E.x;
            ei += gl[kSelfGL + i] * rho * E.y;
        }
        tr += half * er;
        ti += half * ei;
    }
    const double inv4pi = 0.25 / 3.14159265358979323846;
    S[k * lds + a] = make_double2(tr * inv4pi, ti * inv4pi);
}

// out[l][a] = sum_k F[k][l] * samples[k][a]  (rows of length n_pad)
__global__ void coef_dft_kernel(const double2 *__restrict__ samples, int64_t n_pad, int K,
                                const double2 *__restrict__ F, int L, double2 *__restrict__ out) {
    const int64_t a = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int l = blockIdx.y;
    if (a >= n_pad || l >= L) return;
    double sr = 0.0, si = 0.0;
    for (int k = 0; k < K; ++k) {
        const double2 f = F[(int64_t)k * L + l];
        const double2 v = samples[(int64_t)k * n_pad + a];
        sr += f.x * v.x - f.y * v.y;
        si += f.x * v.y + f.y * v.x;
    }
    out[(int64_t)l * n_pad + a] = make_double2(sr, si);
}

}  // namespace

hipError_t launch_prepare_mesh(const double *xyz, const int32_t *tri, int64_t n, int64_t n_pad,
                               DeviceMesh mesh, const double *rule, hipStream_t stream) {
    const int bs = 256;
    const unsigned grid = (unsigned)((n_pad + bs - 1) / bs);
    hipLaunchKernelGGL(prepare_mesh_kernel, dim3(grid), dim3(bs), 0, stream, xyz, tri, n, n_pad,
                       mesh, rule);
    return hipGetLastError();
}

hipError_t launch_self_terms(const DeviceMesh &mesh, const double2 *kappa, int64_t nk, double2 *S,
                             int64_t lds, hipStream_t stream) {
    const int bs = 128;
    dim3 grid((unsigned)((mesh.n_pad + bs - 1) / bs), (unsigned)nk);
    hipLaunchKernelGGL(self_terms_kernel, grid, dim3(bs), 0, stream, mesh.vtx, mesh.gl, mesh.n,
                       mesh.n_pad, kappa, nk, S, lds);
    return hipGetLastError();
}

hipError_t launch_coef_dft(const double2 *samples, int64_t n_pad, int K, const double2 *F, int L,
                           double2 *out, hipStream_t stream) {
    const int bs = 256;
    dim3 grid((unsigned)((n_pad + bs - 1) / bs), (unsigned)L);
    hipLaunchKernelGGL(coef_dft_kernel, grid, dim3(bs), 0, stream, samples, n_pad, K, F, L, out);
    return hipGetLastError();
}

}  // namespace bemrat
