// Near-field correction of the operator: for each near pair (a, b) of the mesh's list the
// 7-point entry T_ab(kappa) is replaced by the integral of the Green's function over
// triangle b (the boundary integral that the 7-point rule approximates, Section 1,
// eq. GreenFun), and the difference dT_ab = integral - 7-point value is applied to the probe
// block, folded with the node weights:
//     M[p][a, :] += sum_j W[j][p] sum_{b near a} dT_ab(z_j) V[b, :].
//
// Integral (polar form around the projection of x_a onto the plane of triangle b): with
// d the signed height of x_a over the plane, x' its foot, and for edge e its signed
// in-plane distance p_e from x' (positive on the interior side) and the tangential
// coordinates s_A < s_B of its end points,
//     int_b g dA = e^{i kappa |d|}/(4 pi) sum_e sign(p_e) int delta(rho) E(i kappa delta(rho)) dphi,
// where along direction phi the fan triangle (x', A, B) reaches rho = |p_e|/cos phi,
// delta(rho) = sqrt(rho^2 + d^2) - |d| = rho^2/(sqrt(rho^2 + d^2) + |d|), and
// E(w) = (e^w - 1)/w (the radial integral of g in closed form).  The angle is substituted
// by phi = atan(sinh u) (t = |p_e| sinh u along the edge, rho = |p_e| cosh u,
// dphi = du / cosh u), the sinh transformation of Johnston and Elliott (2005) that keeps the
// integrand smooth when x' is close to the edge line; the u-interval is split into panels
// of length <= 2 (the integrand's nearest singularities lie at Im u = +-pi/2), and into at
// least kappa_max rho_max / 2 of them (rho_max the distance to the farther end point, so that
// a panel spans about two radians of phase), each integrated with 16-point Gauss-Legendre;
// an interval that needs half of both (length <= 1, kappa_max rho_max <= 1) takes a single
// 10-point panel.
//
// One workgroup per target row; its pairs are taken 64 at a time, with 256 / (pairs in the
// chunk) node groups per pair, and every partial sum is reduced in a fixed order, so results
// are deterministic.  In the dense mode (S non-null, one weight set) the folded corrections
// are added to the matrix entries S[a][b] instead of being applied to a probe block.
#include "devmath.h"
#include "internal.h"

namespace bemrat {

namespace {

constexpr int kNfThreads = 256;
constexpr int kNfPairs = 64;
constexpr int kNfGL = 16;       // points per panel
constexpr int kNfGLShort = 10;  // points of the single panel of a short interval
constexpr int kNfMaxPanels = 64;
constexpr int kNfNodes = 4;  // nodes per thread evaluated together

struct NfArgs {
    const double4 *colloc;
    const double4 *quad;
    const double *vtx;
    const double *gl;  // on [-1, 1]: kNfGL nodes, their weights, kNfGLShort nodes, their weights
    const int64_t *rowptr;
    const int32_t *col;
    const double2 *kappa;  // N nodes
    const double2 *W;      // N x Pstride; this launch uses columns p0 .. p0 + P - 1
    int N, Pstride, p0, P;
    double kmax;           // max |kappa_j| (sets the panel count)
    const double2 *V;
    int64_t ldv, m;
    double2 *M;            // block p at M + p * mstride, row stride ldm
    int64_t ldm, mstride;
    double2 *S;            // dense mode (P = 1): S[a][b] += folded correction, row stride lds
    int64_t lds;
    // fold mode (Fout non-null): only the pairs k with flag[k] != 0 are integrated, and their
    // folded corrections are written to Fout[k * Fstride + p0 + p] instead of being applied
    double2 *Fout;
    const unsigned char *flag;
    int Fstride;
    // nodes with a nonzero weight among this launch's weight sets (all N when null): only these
    // are integrated
    const int *nodes;
    int nnodes;
};

// Geometry of the polar integral of one (target, source triangle) pair: the target's height
// |d| over the plane, and per edge the sign and size of its in-plane distance, the start and
// width of the sinh-transformed angle panels, their number and their rule (16 or 10 points).
struct NfGeom {
    double ad;
    double esg[3], eap[3], eu0[3], eh[3];
    int enp[3], enq[3];
};

__device__ __forceinline__ void nf_geometry(const double (&P)[3][3], const double (&x)[3], double kmax, NfGeom &o) {
    // unit normal, height and foot of x
    const double e1[3] = {P[1][0] - P[0][0], P[1][1] - P[0][1], P[1][2] - P[0][2]};
    const double e2[3] = {P[2][0] - P[0][0], P[2][1] - P[0][1], P[2][2] - P[0][2]};
    double nv[3] = {e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2], e1[0] * e2[1] - e1[1] * e2[0]};
    const double nn = sqrt(nv[0] * nv[0] + nv[1] * nv[1] + nv[2] * nv[2]);
    for (int c = 0; c < 3; ++c) nv[c] /= nn;
    const double d = (x[0] - P[0][0]) * nv[0] + (x[1] - P[0][1]) * nv[1] + (x[2] - P[0][2]) * nv[2];
    o.ad = fabs(d);
    const double xp[3] = {x[0] - d * nv[0], x[1] - d * nv[1], x[2] - d * nv[2]};
    // per edge: sign of p, |p|, start of the u-interval, panel width and count
    for (int e = 0; e < 3; ++e) {
        const double *A = P[e], *B = P[(e + 1) % 3];
        double tv[3] = {B[0] - A[0], B[1] - A[1], B[2] - A[2]};
        const double len = sqrt(tv[0] * tv[0] + tv[1] * tv[1] + tv[2] * tv[2]);
        for (int c = 0; c < 3; ++c) tv[c] /= len;
        // outward in-plane normal of the edge: t x n
        const double u[3] = {tv[1] * nv[2] - tv[2] * nv[1], tv[2] * nv[0] - tv[0] * nv[2],
                             tv[0] * nv[1] - tv[1] * nv[0]};
        const double ax = A[0] - xp[0], ay = A[1] - xp[1], az = A[2] - xp[2];
        const double bx = B[0] - xp[0], by = B[1] - xp[1], bz = B[2] - xp[2];
        const double pe = ax * u[0] + ay * u[1] + az * u[2];
        const double sA = ax * tv[0] + ay * tv[1] + az * tv[2];
        const double sB = bx * tv[0] + by * tv[1] + bz * tv[2];
        const double ap = fabs(pe);
        if (!(ap > 1e-30 * len)) {  // x' on the edge line: the fan triangle is empty
            o.esg[e] = 0.0;
            o.eap[e] = 0.0;
            o.eu0[e] = 0.0;
            o.eh[e] = 0.0;
            o.enp[e] = 0;
            o.enq[e] = 0;
            continue;
        }
        const double u0 = asinh(sA / ap), u1 = asinh(sB / ap);
        const double rmax = fmax(sqrt(ap * ap + sA * sA), sqrt(ap * ap + sB * sB));
        const double want = fmax(0.5 * (u1 - u0), 0.5 * kmax * rmax);
        const int np = want >= kNfMaxPanels ? kNfMaxPanels : (want <= 1.0 ? 1 : (int)ceil(want));
        o.esg[e] = pe > 0.0 ? 1.0 : -1.0;
        o.eap[e] = ap;
        o.eu0[e] = u0;
        o.eh[e] = (u1 - u0) / np;
        o.enp[e] = np;
        // an interval of at most 1 in u and 1 in phase: the nearest singularity lies pi/2
        // away, a Bernstein ellipse of parameter 6.4 (error ~ 6.4^-20 at 10 points)
        o.enq[e] = want <= 0.5 ? kNfGLShort : kNfGL;
    }
}

// The angular integrals s = sum_e sign(p_e) int delta E(i kappa delta) dphi of NN wavenumbers
// (kr + i ki) at once, over the panels of `o` (the integral over the triangle is then
// e^{i kappa |d|} s / (4 pi)).
template <int NN>
__device__ __forceinline__ void nf_radial(const NfGeom &o, const double *gl, const double (&kr)[NN],
                                          const double (&ki)[NN], double (&sr)[NN], double (&si)[NN]) {
    const double ad = o.ad;
    for (int e = 0; e < 3; ++e) {
        for (int pn = 0; pn < o.enp[e]; ++pn) {
            const double mid = o.eu0[e] + (pn + 0.5) * o.eh[e];
            const double scale = 0.5 * o.eh[e] * o.esg[e];
            const int nq = o.enq[e];
            const double *glx = nq == kNfGL ? gl : gl + 2 * kNfGL;
            for (int k = 0; k < nq; ++k) {
                const double uu = mid + 0.5 * o.eh[e] * glx[k];
                const double ch = cosh(uu);
                const double rho = o.eap[e] * ch;
                const double dl = rho * rho / (sqrt(rho * rho + ad * ad) + ad);
                const double wt = scale * glx[nq + k] * dl / ch;
#pragma unroll
                for (int s = 0; s < NN; ++s) {
                    const double2 E = exprel(-ki[s] * dl, kr[s] * dl);  // w = i kappa delta
                    sr[s] += wt * E.x;
                    si[s] += wt * E.y;
                }
            }
        }
    }
}

__global__ __launch_bounds__(kNfThreads) void nearfield_kernel(NfArgs g) {
    __shared__ double2 red[kNfThreads][kNfFold];
    __shared__ double2 fold[kNfPairs][kNfFold];
    __shared__ int32_t cols[kNfPairs];
    const int64_t a = blockIdx.x;
    const int t = threadIdx.x;
    const int64_t beg = g.rowptr[a], end = g.rowptr[a + 1];
    if (beg >= end) return;  // uniform over the workgroup
    const double4 xa = g.colloc[a];
    const double inv4pi = 0.25 / 3.14159265358979323846;
    for (int64_t base = beg; base < end; base += kNfPairs) {
        const int cnt = (int)(end - base < kNfPairs ? end - base : kNfPairs);
        // as many node groups per pair as the workgroup holds (at least 4), so rows with few
        // pairs still fill the lanes; thread t takes pair t / G and node group t % G, so the
        // G lanes of one pair follow the same panel loops
        const int G = kNfThreads / cnt;
        const int i = t / G, grp = t % G;
        // this thread's folded sums live in its own LDS slots (fewer live registers)
        double2 *acc = red[t];
#pragma unroll
        for (int p = 0; p < kNfFold; ++p) acc[p] = make_double2(0.0, 0.0);
        if (i < cnt && (!g.flag || g.flag[base + i])) {
            const int64_t b = g.col[base + i];
            if (grp == 0) cols[i] = (int32_t)b;
            double P[3][3];
#pragma unroll
            for (int v = 0; v < 3; ++v)
#pragma unroll
                for (int c = 0; c < 3; ++c) P[v][c] = g.vtx[9 * b + 3 * v + c];
            const double x[3] = {xa.x, xa.y, xa.z};
            NfGeom geo;
            nf_geometry(P, x, g.kmax, geo);
            const double ad = geo.ad;
            // this thread's nodes j = grp + G * s, s = 0, 1, ..., taken kNfNodes at a time: the
            // geometry of each quadrature point is computed once per chunk, and the chunk's
            // independent series evaluations overlap in the pipeline
            const int nn = g.nodes ? g.nnodes : g.N;
            for (int j0 = grp; j0 < nn; j0 += G * kNfNodes) {
                double kr[kNfNodes], ki[kNfNodes], sr[kNfNodes], si[kNfNodes];
#pragma unroll
                for (int s = 0; s < kNfNodes; ++s) {
                    const int jj = j0 + s * G;
                    const int j = jj < nn ? (g.nodes ? g.nodes[jj] : jj) : g.N;
                    const double2 kj = j < g.N ? g.kappa[j] : make_double2(0.0, 0.0);
                    kr[s] = kj.x;
                    ki[s] = kj.y;
                    sr[s] = 0.0;
                    si[s] = 0.0;
                }
                nf_radial<kNfNodes>(geo, g.gl, kr, ki, sr, si);
#pragma unroll
                for (int s = 0; s < kNfNodes; ++s) {
                    const int jj = j0 + s * G;
                    if (jj >= nn) break;
                    const int j = g.nodes ? g.nodes[jj] : jj;
                    // e^{i kappa |d|} / (4 pi)
                    double s0, c0;
                    sincos(kr[s] * ad, &s0, &c0);
                    const double m0 = exp(-ki[s] * ad) * inv4pi;
                    double dr = m0 * (c0 * sr[s] - s0 * si[s]), di = m0 * (c0 * si[s] + s0 * sr[s]);
                    // minus the 7-point value of the rule the sweep uses
#pragma unroll
                    for (int q = 0; q < kQuad; ++q) {
                        const double4 y = g.quad[b * kQuad + q];
                        const double qx = x[0] - y.x, qy = x[1] - y.y, qz = x[2] - y.z;
                        const double rq = sqrt(qx * qx + qy * qy + qz * qz);
                        double sq, cq;
                        sincos(kr[s] * rq, &sq, &cq);
                        const double mq = exp(-ki[s] * rq) * y.w / rq;  // y.w = A_b w_q / (4 pi)
                        dr -= mq * cq;
                        di -= mq * sq;
                    }
#pragma unroll
                    for (int p = 0; p < kNfFold; ++p) {
                        if (p < g.P) {
                            const double2 w = g.W[(int64_t)j * g.Pstride + g.p0 + p];
                            acc[p].x += w.x * dr - w.y * di;
                            acc[p].y += w.x * di + w.y * dr;
                        }
                    }
                }
            }
        }
        __syncthreads();
        // fold the node groups in a fixed order
        for (int idx = t; idx < cnt * g.P; idx += kNfThreads) {
            const int k = idx / g.P, p = idx % g.P;
            double2 s = red[k * G][p];
            for (int q = 1; q < G; ++q) {
                s.x += red[k * G + q][p].x;
                s.y += red[k * G + q][p].y;
            }
            fold[k][p] = s;
        }
        __syncthreads();
        if (g.Fout) {
            // fold mode: store the flagged pairs' folded corrections
            for (int idx = t; idx < cnt * g.P; idx += kNfThreads) {
                const int k = idx / g.P, p = idx % g.P;
                if (g.flag[base + k]) g.Fout[(base + k) * g.Fstride + g.p0 + p] = fold[k][p];
            }
            __syncthreads();
            continue;
        }
        if (g.S) {
            // dense mode: add the folded corrections to the matrix (one thread per pair)
            if (t < cnt) {
                double2 *out = g.S + a * g.lds + cols[t];
                const double2 o = *out;
                *out = make_double2(o.x + fold[t][0].x, o.y + fold[t][0].y);
            }
            __syncthreads();
            continue;
        }
        // apply to the probe block
        for (int64_t item = t; item < (int64_t)g.P * g.m; item += kNfThreads) {
            const int p = (int)(item / g.m);
            const int64_t c = item % g.m;
            double sr = 0.0, si = 0.0;
            for (int k = 0; k < cnt; ++k) {
                const double2 f = fold[k][p];
                const double2 v = g.V[(int64_t)cols[k] * g.ldv + c];
                // explicit fused steps: the pair-fold apply kernel rounds the same way
                sr = fma(-f.y, v.y, fma(f.x, v.x, sr));
                si = fma(f.y, v.x, fma(f.x, v.y, si));
            }
            double2 *out = g.M + p * g.mstride + a * g.ldm + c;
            const double2 o = *out;
            *out = make_double2(o.x + sr, o.y + si);
        }
        __syncthreads();
    }
}

// Series form of the folded correction.  While |kappa| R is small (R the distance from the
// target to the farthest point of triangle b) every part of dT_ab(kappa) is a short power series
// in kappa: the radial integral of the polar form,
//     e^{i kappa |d|} delta E(i kappa delta) = int_{|d|}^{R} e^{i kappa r} dr
//         = sum_n (i kappa)^n (R^{n+1} - |d|^{n+1}) / (n+1)!,
// and each 7-point term, e^{i kappa r_q} / r_q = sum_n (i kappa)^n r_q^{n-1} / n!.  Hence
//     dT_ab(kappa) = sum_{n<L} c_n (i kappa)^n,
//     c_n = sum_e sign(p_e) sum_points w_phi (R^{n+1} - |d|^{n+1}) / (4 pi (n+1)!)
//           - sum_q w_q r_q^{n-1} / n!,
// with w_phi a point's angular weight and w_q = A_b w_q / (4 pi) the 7-point weight, and the
// folded correction of weight set p is sum_n c_n mu[n][p], mu[n][p] = sum_j W[j][p] (i kappa_j)^n
// (formed on the host).  The angular points are those of the per-node kernel, so the two agree
// to rounding plus the truncation, which the host bounds through x = kappa_max R_max
// (x^L e^x / L! relative).  R^{n+1} - |d|^{n+1} is advanced as D_{n+1} = R D_n + |d|^n delta,
// free of cancellation when R is close to |d|.  One thread per pair; the pairs are taken in
// contiguous ranges per XCD (the L2 of an XCD then holds the triangles of neighbouring rows).
// 1/x for finite x > 0 away from the exponent limits: the hardware estimate and two Newton
// steps (the quadratic convergence takes it to the rounding of the last step).
__device__ __forceinline__ double rcp_nr(double x) {
    double t = __builtin_amdgcn_rcp(x);
    t = fma(fma(-x, t, 1.0), t, t);
    return fma(fma(-x, t, 1.0), t, t);
}

// sqrt(x) for normal x > 0 away from the exponent limits: the hardware reciprocal square root
// estimate refined by two coupled Newton steps for sqrt(x) and 1/(2 sqrt(x)) and a final
// residual correction.
__device__ __forceinline__ double sqrt_nr(double x) {
    const double y = __builtin_amdgcn_rsq(x);
    double g = x * y, h = 0.5 * y;
    const double r = fma(-g, h, 0.5);
    g = fma(g, r, g);
    h = fma(h, r, h);
    const double d = fma(-g, g, x);
    return fma(d, h, g);
}

struct NfSeriesArgs {
    const double4 *colloc;
    const double4 *quad;
    const double *vtx;
    const double *gl;
    const int32_t *row, *col;
    int64_t npairs, nblocks;
    double kmax;              // panel rule of the angular integral (as the per-node kernel)
    const double2 *mu;        // L x P, mu[n * P + p]
    int P;
    const unsigned char *flag;  // only the pairs with flag[k] != 0 when non-null
    double2 *F;               // F[k * Fstride + p0 + p]
    int Fstride, p0;
};

// Geometry of a workgroup's pairs kept between its two phases (structure of arrays).
struct NfGeomLds {
    double d[13][256];  // ad, esg[3], eap[3], eu0[3], eh[3]
    int i[6][256];      // enp[3], enq[3]
    int order[256];     // pair (thread) index by ascending angular point count
    int count[33], start[33];
};

template <int L>
__global__ __launch_bounds__(256) void nearfield_series_kernel(NfSeriesArgs g) {
    __shared__ NfGeomLds sg;
    // XCD-aware block order: the hardware deals workgroups to the 8 XCDs in turn, so block
    // i runs on XCD i % 8; give XCD x the contiguous blocks x * per .. x * per + per - 1
    const int64_t per = (g.nblocks + 7) / 8;
    const int64_t blk = (int64_t)(blockIdx.x % 8) * per + blockIdx.x / 8;
    if (blk >= g.nblocks) return;  // uniform over the workgroup
    const int t = threadIdx.x;
    // phase 1: every thread the geometry of pair t of the block, and its bucket by angular
    // point count (32: no work); the pairs are then handed to the lanes in bucket order, so
    // a wave's lanes run point loops of about the same length
    {
        const int64_t k = blk * 256 + t;
        int bucket = 32;
        if (k < g.npairs && (!g.flag || g.flag[k])) {
            const int64_t a = g.row[k], b = g.col[k];
            double P[3][3];
#pragma unroll
            for (int v = 0; v < 3; ++v)
#pragma unroll
                for (int c = 0; c < 3; ++c) P[v][c] = g.vtx[9 * b + 3 * v + c];
            const double4 xa = g.colloc[a];
            const double x[3] = {xa.x, xa.y, xa.z};
            NfGeom geo;
            nf_geometry(P, x, g.kmax, geo);
            sg.d[0][t] = geo.ad;
            int pts = 0;
#pragma unroll
            for (int e = 0; e < 3; ++e) {
                sg.d[1 + e][t] = geo.esg[e];
                sg.d[4 + e][t] = geo.eap[e];
                sg.d[7 + e][t] = geo.eu0[e];
                sg.d[10 + e][t] = geo.eh[e];
                sg.i[e][t] = geo.enp[e];
                sg.i[3 + e][t] = geo.enq[e];
                pts += geo.enp[e] * geo.enq[e];
            }
            bucket = pts <= 30 ? 0 : (pts - 30 + 5) / 6 < 31 ? (pts - 30 + 5) / 6 : 31;
        }
        if (t < 33) sg.count[t] = 0;
        __syncthreads();
        const int slot = atomicAdd(&sg.count[bucket], 1);
        __syncthreads();
        if (t == 0) {
            int s = 0;
            for (int q = 0; q < 33; ++q) {
                sg.start[q] = s;
                s += sg.count[q];
            }
        }
        __syncthreads();
        sg.order[sg.start[bucket] + slot] = t;
        __syncthreads();
    }
    // phase 2: lane t takes the pair of rank t (which lane takes which pair does not change
    // any result: each pair's sums run in its own registers)
    const int j = sg.order[t];
    const int64_t k = blk * 256 + j;
    if (k >= g.npairs || (g.flag && !g.flag[k])) return;
    const int64_t a = g.row[k], b = g.col[k];
    const double4 xa = g.colloc[a];
    const double x[3] = {xa.x, xa.y, xa.z};
    NfGeom geo;
    geo.ad = sg.d[0][j];
#pragma unroll
    for (int e = 0; e < 3; ++e) {
        geo.esg[e] = sg.d[1 + e][j];
        geo.eap[e] = sg.d[4 + e][j];
        geo.eu0[e] = sg.d[7 + e][j];
        geo.eh[e] = sg.d[10 + e][j];
        geo.enp[e] = sg.i[e][j];
        geo.enq[e] = sg.i[3 + e][j];
    }
    const double ad = geo.ad;
    double c[L];
#pragma unroll
    for (int n = 0; n < L; ++n) c[n] = 0.0;
    for (int e = 0; e < 3; ++e) {
        const int nq = geo.enq[e];
        const double *glx = nq == kNfGL ? g.gl : g.gl + 2 * kNfGL;
        const double half = 0.5 * geo.eh[e], scale = half * geo.esg[e];
        for (int pn = 0; pn < geo.enp[e]; ++pn) {
            const double mid = geo.eu0[e] + (pn + 0.5) * geo.eh[e];
            for (int q = 0; q < nq; ++q) {
                // cosh u = (e^u + e^-u)/2 (|u| < asinh(1e31) < 73 by the edge-line test), the
                // reciprocals by the hardware estimate and two Newton steps
                const double eu = exp_cw(mid + half * glx[q]);
                const double ch = 0.5 * (eu + rcp_nr(eu));
                const double rho = geo.eap[e] * ch;
                const double R = sqrt_nr(rho * rho + ad * ad);  // in [rho, 2 R_max]: normal
                const double dl = rho * rho * rcp_nr(R + ad);
                const double w = scale * glx[nq + q] * rcp_nr(ch);
                double D = dl, dp = dl;  // D_1 = R - |d|; dp = |d|^n delta
                c[0] += w * D;
#pragma unroll
                for (int n = 1; n < L; ++n) {
                    dp *= ad;
                    D = R * D + dp;
                    c[n] += w * D;
                }
            }
        }
    }
    {
        double f = 0.25 / 3.14159265358979323846;
#pragma unroll
        for (int n = 0; n < L; ++n) {
            f /= (double)(n + 1);
            c[n] *= f;
        }
    }
#pragma unroll
    for (int q = 0; q < kQuad; ++q) {
        const double4 y = g.quad[b * kQuad + q];
        const double qx = x[0] - y.x, qy = x[1] - y.y, qz = x[2] - y.z;
        const double r = sqrt(qx * qx + qy * qy + qz * qz);
        double s = y.w * rcp_nr(r);
        c[0] -= s;
#pragma unroll
        for (int n = 1; n < L; ++n) {
            s *= r * (1.0 / (double)n);
            c[n] -= s;
        }
    }
    double2 *out = g.F + k * g.Fstride + g.p0;
    for (int p = 0; p < g.P; ++p) {
        double fr = 0.0, fi = 0.0;
#pragma unroll
        for (int n = L - 1; n >= 0; --n) {  // smallest terms first
            const double2 m = g.mu[n * g.P + p];
            fr += c[n] * m.x;
            fi += c[n] * m.y;
        }
        out[p] = make_double2(fr, fi);
    }
}

// S[row[k]][col[k]] += F[k] for every pair (each entry appears once in the list).
__global__ __launch_bounds__(256) void pair_dense_add_kernel(const int32_t *__restrict__ row,
                                                             const int32_t *__restrict__ col,
                                                             const double2 *__restrict__ F, int64_t npairs,
                                                             double2 *__restrict__ S, int64_t lds) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= npairs) return;
    double2 *o = S + (int64_t)row[k] * lds + col[k];
    const double2 f = F[k], v = *o;
    *o = make_double2(v.x + f.x, v.y + f.y);
}

}  // namespace

hipError_t launch_nearfield(const DeviceMesh &mesh, const double *gl16, const int64_t *rowptr,
                            const int32_t *col, const double2 *kappa, int N, const double2 *W, int Pstride,
                            int p0, int P, double kmax, const double2 *V, int64_t ldv, int64_t m,
                            double2 *M, int64_t ldm, double2 *S, int64_t lds, const int *nodes, int nnodes,
                            hipStream_t stream) {
    NfArgs g;
    g.colloc = mesh.colloc;
    g.quad = mesh.quad;
    g.vtx = mesh.vtx;
    g.gl = gl16;
    g.rowptr = rowptr;
    g.col = col;
    g.kappa = kappa;
    g.W = W;
    g.N = N;
    g.Pstride = Pstride;
    g.p0 = p0;
    g.P = P;
    g.kmax = kmax;
    g.V = V;
    g.ldv = ldv;
    g.m = m;
    g.M = M ? M + (int64_t)p0 * mesh.n * ldm : nullptr;
    g.ldm = ldm;
    g.mstride = mesh.n * ldm;
    g.S = S;
    g.lds = lds;
    g.Fout = nullptr;
    g.flag = nullptr;
    g.Fstride = 0;
    g.nodes = nodes;
    g.nnodes = nnodes;
    hipLaunchKernelGGL(nearfield_kernel, dim3((unsigned)mesh.n), dim3(kNfThreads), 0, stream, g);
    return hipGetLastError();
}

hipError_t launch_nearfield_fold(const DeviceMesh &mesh, const double *gl16, const int64_t *rowptr,
                                 const int32_t *col, const unsigned char *flag, const double2 *kappa, int N,
                                 const double2 *W, int Pstride, int p0, int P, double kmax, double2 *F,
                                 const int *nodes, int nnodes, hipStream_t stream) {
    NfArgs g{};
    g.colloc = mesh.colloc;
    g.quad = mesh.quad;
    g.vtx = mesh.vtx;
    g.gl = gl16;
    g.rowptr = rowptr;
    g.col = col;
    g.kappa = kappa;
    g.W = W;
    g.N = N;
    g.Pstride = Pstride;
    g.p0 = p0;
    g.P = P;
    g.kmax = kmax;
    g.Fout = F;
    g.flag = flag;
    g.Fstride = Pstride;
    g.nodes = nodes;
    g.nnodes = nnodes;
    hipLaunchKernelGGL(nearfield_kernel, dim3((unsigned)mesh.n), dim3(kNfThreads), 0, stream, g);
    return hipGetLastError();
}

int nf_series_terms(double x) {
    // smallest L of the compiled lengths with x^L e^x / L! <= 1e-17, else 0
    if (!(x >= 0.0) || !(x < 64.0)) return 0;
    static const int lengths[] = {12, 16, 24, 32};
    double term = 1.0;  // x^n / n!
    const double ex = exp(x);
    int n = 0;
    for (int Lc : lengths) {
        while (n < Lc) {
            ++n;
            term *= x / n;
        }
        if (term * ex <= 1e-17) return Lc;
    }
    return 0;
}

hipError_t launch_nearfield_series(const DeviceMesh &mesh, const double *gl16, const int32_t *row, const int32_t *col,
                                   int64_t npairs, const unsigned char *flag, double kmax, const double2 *mu, int L,
                                   int P, double2 *F, int Fstride, int p0, hipStream_t stream) {
    if (npairs <= 0) return hipSuccess;
    NfSeriesArgs g;
    g.colloc = mesh.colloc;
    g.quad = mesh.quad;
    g.vtx = mesh.vtx;
    g.gl = gl16;
    g.row = row;
    g.col = col;
    g.npairs = npairs;
    g.nblocks = (npairs + 255) / 256;
    g.kmax = kmax;
    g.mu = mu;
    g.P = P;
    g.flag = flag;
    g.F = F;
    g.Fstride = Fstride;
    g.p0 = p0;
    const dim3 grid((unsigned)((g.nblocks + 7) / 8 * 8));
    switch (L) {
    case 12: hipLaunchKernelGGL(nearfield_series_kernel<12>, grid, dim3(256), 0, stream, g); break;
    case 16: hipLaunchKernelGGL(nearfield_series_kernel<16>, grid, dim3(256), 0, stream, g); break;
    case 24: hipLaunchKernelGGL(nearfield_series_kernel<24>, grid, dim3(256), 0, stream, g); break;
    case 32: hipLaunchKernelGGL(nearfield_series_kernel<32>, grid, dim3(256), 0, stream, g); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_pair_dense_add(const int32_t *row, const int32_t *col, const double2 *F, int64_t npairs, double2 *S,
                                 int64_t lds, hipStream_t stream) {
    if (npairs <= 0) return hipSuccess;
    hipLaunchKernelGGL(pair_dense_add_kernel, dim3((unsigned)((npairs + 255) / 256)), dim3(256), 0, stream, row, col, F,
                       npairs, S, lds);
    return hipGetLastError();
}

namespace {

// Labels for the learned correction: for sample s, the triangle P9[s] (3 vertices), the
// target x[s] and the wavenumber kappa[s], dT = (integral of g over the triangle, by the polar
// form above) - (Radon's 7-point value on the same triangle).  One thread per sample.
struct NfLabelArgs {
    const double *P9, *x;
    const double2 *kappa;
    double2 *out;
    int64_t S;
    double gl[2 * kNfGL + 2 * kNfGLShort];
    double rule[kQuad * 4];  // barycentric weights of P0, P1, P2 and the weight (sum 1) per point
};

__global__ __launch_bounds__(256) void nf_label_kernel(NfLabelArgs g) {
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= g.S) return;
    double P[3][3];
    for (int v = 0; v < 3; ++v)
        for (int c = 0; c < 3; ++c) P[v][c] = g.P9[9 * s + 3 * v + c];
    const double x[3] = {g.x[3 * s], g.x[3 * s + 1], g.x[3 * s + 2]};
    const double2 kap = g.kappa[s];
    const double kr[1] = {kap.x}, ki[1] = {kap.y};
    NfGeom geo;
    nf_geometry(P, x, sqrt(kap.x * kap.x + kap.y * kap.y), geo);
    double sr[1] = {0.0}, si[1] = {0.0};
    nf_radial<1>(geo, g.gl, kr, ki, sr, si);
    const double inv4pi = 0.25 / 3.14159265358979323846;
    double s0, c0;
    sincos(kap.x * geo.ad, &s0, &c0);
    const double m0 = exp(-kap.y * geo.ad) * inv4pi;
    double dr = m0 * (c0 * sr[0] - s0 * si[0]), di = m0 * (c0 * si[0] + s0 * sr[0]);
    const double e1[3] = {P[1][0] - P[0][0], P[1][1] - P[0][1], P[1][2] - P[0][2]};
    const double e2[3] = {P[2][0] - P[0][0], P[2][1] - P[0][1], P[2][2] - P[0][2]};
    const double cx = e1[1] * e2[2] - e1[2] * e2[1], cy = e1[2] * e2[0] - e1[0] * e2[2],
                 cz = e1[0] * e2[1] - e1[1] * e2[0];
    const double area = 0.5 * sqrt(cx * cx + cy * cy + cz * cz);
    for (int q = 0; q < kQuad; ++q) {
        const double *rq = g.rule + 4 * q;
        double y[3];
        for (int c = 0; c < 3; ++c) y[c] = rq[0] * P[0][c] + rq[1] * P[1][c] + rq[2] * P[2][c];
        const double qx = x[0] - y[0], qy = x[1] - y[1], qz = x[2] - y[2];
        const double r = sqrt(qx * qx + qy * qy + qz * qz);
        double sq, cq;
        sincos(kap.x * r, &sq, &cq);
        const double mq = exp(-kap.y * r) * area * rq[3] * inv4pi / r;
        dr -= mq * cq;
        di -= mq * sq;
    }
    g.out[s] = make_double2(dr, di);
}

}  // namespace

hipError_t launch_nf_labels(const double *P9, const double *x, const double2 *kappa, int64_t S, double2 *out,
                            const double *gl52, const double *rule28, hipStream_t stream) {
    NfLabelArgs g;
    g.P9 = P9;
    g.x = x;
    g.kappa = kappa;
    g.out = out;
    g.S = S;
    for (int i = 0; i < 2 * kNfGL + 2 * kNfGLShort; ++i) g.gl[i] = gl52[i];
    for (int i = 0; i < kQuad * 4; ++i) g.rule[i] = rule28[i];
    if (S <= 0) return hipSuccess;
    hipLaunchKernelGGL(nf_label_kernel, dim3((unsigned)((S + 255) / 256)), dim3(256), 0, stream, g);
    return hipGetLastError();
}

}  // namespace bemrat
