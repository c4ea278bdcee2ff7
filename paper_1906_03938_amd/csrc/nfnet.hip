// The learned near-field correction: a perceptron with three hidden layers of 128 tanh units
// that maps a (source triangle, target point, wavenumber) triple to the correction
// dT = (integral of g over the triangle) - (its 7-point value), g(r) = exp(i kappa r)/(4 pi r),
// trained on triples labelled by the library's own polar quadrature (nearfield.hip), which
// stays the fallback and the reference.  Not a step of the paper's method: a surrogate for the
// near-field refinement of the boundary integral of Section 1 (eq. GreenFun).
//
// Inputs.  In the unit frame of the source triangle (its longest edge A -> B on the x axis,
// the first longest of P0P1, P1P2, P2P0; lengths divided by h = |B - A|; the third vertex
// C = (p, q) with q > 0; mirrored across u = 1/2 when p > 1/2) the target has coordinates
// (u, v, w); the 19 inputs are
//   (p - 0.25)/0.25, (q - 0.5)/0.4, (u - 0.5)/1.5, (v - 0.3)/1.5, |w|, 2 Re(kappa h) - 1,
//   Im(kappa h)/0.3, r0 - 1, 0.5/r0, 0.3/r_k (k < 7), 0.5/s_k (k < 3),
// r0 the distance to the centroid, r_k to the points of Radon's rule (centroid; barycentric
// weight a1 on A, B, C; weight a2 on A, B, C) and s_k to A, B, C.  The two outputs y give
// dT = h (S_re y_0 + i S_im y_1) / (4 pi r0^4), S the output scales of the training set (r0^4
// takes out most of the decay with distance; dT depends on kappa only at second order, since
// the rule integrates the linear term of exp(i kappa r) exactly).
//
// Parameters (FP32, one array, row-major out x in): W1 [128 x 32] (input columns 19..31
// unused), b1 [128], W2 [128 x 128], b2, W3 [128 x 128], b3, W4 [2 x 128], b4 [2].
//
// Training (FP32 on the matrix cores, v_mfma_f32_16x16x4f32): one workgroup per tile of 32
// samples runs the forward pass (activations in LDS), the loss (1/B) sum (y - t)^2 and the
// back-propagation, and writes its share of the gradient to its own slot; a second kernel sums
// the slots in a fixed order and a third applies Adam, so training is deterministic.
#include <math.h>

#include "internal.h"

namespace bemrat {

namespace {

constexpr int H = kNetHidden;
constexpr int FP = kNetInPad;
constexpr int NO = kNetOut;
constexpr int64_t oW1 = 0, ob1 = (int64_t)H * FP, oW2 = ob1 + H, ob2 = oW2 + (int64_t)H * H, oW3 = ob2 + H,
                  ob3 = oW3 + (int64_t)H * H, oW4 = ob3 + H, ob4 = oW4 + (int64_t)NO * H;
static_assert(ob4 + NO == kNetParams, "parameter layout");

typedef float v4f __attribute__((ext_vector_type(4)));

__device__ __forceinline__ v4f mfma4(float a, float b, v4f c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// ---------------------------------------------------------------- input features

// Unit-frame coordinates of target x relative to source triangle P (see the file header).
__device__ __forceinline__ void net_frame(const double (&P)[3][3], const double (&x)[3], double &p, double &q,
                                          double &u, double &v, double &w, double &h) {
    double len[3];
#pragma unroll
    for (int e = 0; e < 3; ++e) {
        const double dx = P[(e + 1) % 3][0] - P[e][0], dy = P[(e + 1) % 3][1] - P[e][1],
                     dz = P[(e + 1) % 3][2] - P[e][2];
        len[e] = sqrt(dx * dx + dy * dy + dz * dz);
    }
    int e = 0;
    if (len[1] > len[e]) e = 1;
    if (len[2] > len[e]) e = 2;
    // A, B, C = P[e], P[e + 1], P[e + 2] (indices mod 3), picked by selects (no indexing by e)
    double A[3], B[3], C[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        A[c] = e == 0 ? P[0][c] : e == 1 ? P[1][c] : P[2][c];
        B[c] = e == 0 ? P[1][c] : e == 1 ? P[2][c] : P[0][c];
        C[c] = e == 0 ? P[2][c] : e == 1 ? P[0][c] : P[1][c];
    }
    h = e == 0 ? len[0] : e == 1 ? len[1] : len[2];
    const double ab[3] = {B[0] - A[0], B[1] - A[1], B[2] - A[2]};
    const double ac[3] = {C[0] - A[0], C[1] - A[1], C[2] - A[2]};
    const double ax[3] = {x[0] - A[0], x[1] - A[1], x[2] - A[2]};
    const double ex[3] = {ab[0] / h, ab[1] / h, ab[2] / h};
    double nv[3] = {ab[1] * ac[2] - ab[2] * ac[1], ab[2] * ac[0] - ab[0] * ac[2], ab[0] * ac[1] - ab[1] * ac[0]};
    const double nn = sqrt(nv[0] * nv[0] + nv[1] * nv[1] + nv[2] * nv[2]);
    nv[0] /= nn;
    nv[1] /= nn;
    nv[2] /= nn;
    const double ey[3] = {nv[1] * ex[2] - nv[2] * ex[1], nv[2] * ex[0] - nv[0] * ex[2], nv[0] * ex[1] - nv[1] * ex[0]};
    p = (ac[0] * ex[0] + ac[1] * ex[1] + ac[2] * ex[2]) / h;
    q = (ac[0] * ey[0] + ac[1] * ey[1] + ac[2] * ey[2]) / h;
    u = (ax[0] * ex[0] + ax[1] * ex[1] + ax[2] * ex[2]) / h;
    v = (ax[0] * ey[0] + ax[1] * ey[1] + ax[2] * ey[2]) / h;
    w = fabs(ax[0] * nv[0] + ax[1] * nv[1] + ax[2] * nv[2]) / h;
    if (p > 0.5) {
        p = 1.0 - p;
        u = 1.0 - u;
    }
}

// The 17 inputs that do not depend on the wavenumber (all but 5 and 6, which are left 0) and
// the centroid distance r0, from unit-frame coordinates.
__device__ __forceinline__ void net_geometry_inputs(double p, double q, double u, double v, double w, float (&f)[kNetIn],
                                                    double &r0) {
    const double cx = (1.0 + p) / 3.0, cy = q / 3.0;
    r0 = sqrt((u - cx) * (u - cx) + (v - cy) * (v - cy) + w * w);
    f[0] = (float)((p - 0.25) / 0.25);
    f[1] = (float)((q - 0.5) / 0.4);
    f[2] = (float)((u - 0.5) / 1.5);
    f[3] = (float)((v - 0.3) / 1.5);
    f[4] = (float)w;
    f[5] = 0.0f;
    f[6] = 0.0f;
    f[7] = (float)(r0 - 1.0);
    f[8] = (float)(0.5 / r0);
    // Radon's points: barycentric (la, lb, lc) on A = (0,0), B = (1,0), C = (p,q)
    const double s15 = sqrt(15.0);
    const double a1 = (9.0 - 2.0 * s15) / 21.0, b1 = (6.0 + s15) / 21.0;
    const double a2 = (9.0 + 2.0 * s15) / 21.0, b2 = (6.0 - s15) / 21.0;
    const double lam[7][3] = {{1.0 / 3.0, 1.0 / 3.0, 1.0 / 3.0}, {a1, b1, b1}, {b1, a1, b1}, {b1, b1, a1},
                              {a2, b2, b2}, {b2, a2, b2}, {b2, b2, a2}};
#pragma unroll
    for (int k = 0; k < 7; ++k) {
        const double yx = lam[k][1] + lam[k][2] * p, yy = lam[k][2] * q;
        const double rk = sqrt((u - yx) * (u - yx) + (v - yy) * (v - yy) + w * w);
        f[9 + k] = (float)(0.3 / rk);
    }
    const double vx[3] = {0.0, 1.0, p}, vy[3] = {0.0, 0.0, q};
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const double sk = sqrt((u - vx[k]) * (u - vx[k]) + (v - vy[k]) * (v - vy[k]) + w * w);
        f[16 + k] = (float)(0.5 / sk);
    }
}

// Inputs of (triangle P9[s], target x[s], wavenumber kappa[s]): X[s] (32 floats, columns
// 19..31 zero) and aux[s] = (h, r0, Re kappa h, Im kappa h).
__global__ __launch_bounds__(256) void net_features_kernel(const double *__restrict__ P9, const double *__restrict__ x,
                                                           const double2 *__restrict__ kappa, int64_t S,
                                                           float *__restrict__ X, double *__restrict__ aux) {
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= S) return;
    double P[3][3];
    for (int v = 0; v < 3; ++v)
        for (int c = 0; c < 3; ++c) P[v][c] = P9[9 * s + 3 * v + c];
    const double xs[3] = {x[3 * s], x[3 * s + 1], x[3 * s + 2]};
    double p, q, u, v, w, h, r0;
    net_frame(P, xs, p, q, u, v, w, h);
    float f[kNetIn];
    net_geometry_inputs(p, q, u, v, w, f, r0);
    const double2 k = kappa[s];
    const double khr = k.x * h, khi = k.y * h;
    f[5] = (float)(2.0 * khr - 1.0);
    f[6] = (float)(khi / 0.3);
    for (int i = 0; i < FP; ++i) X[s * FP + i] = i < kNetIn ? f[i] : 0.0f;
    aux[4 * s] = h;
    aux[4 * s + 1] = r0;
    aux[4 * s + 2] = khr;
    aux[4 * s + 3] = khi;
}

// ---------------------------------------------------------------- FP32 training

constexpr int TB = 32;       // samples per workgroup
constexpr int LDA = H + 4;   // LDS row stride of activations (conflict-free MFMA operand reads)
constexpr int LDX = FP + 4;  // LDS row stride of the inputs

struct TileArgs {
    const float *params;
    const float *X;   // B x 32
    const float *T;   // B x 2 targets (training) or NULL
    int64_t B;
    float inv_B;
    float *Y;         // B x 2 outputs or NULL
    float *partial;   // (training) gridDim.x x kNetParams gradient slots
    float *loss_part; // (training) gridDim.x loss slots
};

// out[r][n] = tanh(sum_k in[r][k] W[n][k] + b[n]) for the tile's 32 rows and the wave's 32
// columns n in [32 w, 32 w + 32); K a multiple of 4.
__device__ __forceinline__ void dense_tanh(const float *in, int ldin, int K, const float *W, const float *b, float *out,
                                           int w, int ci, int ck) {
#pragma unroll
    for (int rt = 0; rt < 2; ++rt)
#pragma unroll
        for (int nt = 0; nt < 2; ++nt) {
            const int r0 = 16 * rt, n0 = 32 * w + 16 * nt;
            v4f acc = {0.0f, 0.0f, 0.0f, 0.0f};
            for (int k0 = 0; k0 < K; k0 += 4)
                acc = mfma4(in[(r0 + ci) * ldin + k0 + ck], W[(int64_t)(n0 + ci) * K + k0 + ck], acc);
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int r = r0 + 4 * ck + i, n = n0 + ci;
                out[r * LDA + n] = tanhf(acc[i] + b[n]);
            }
        }
}

// Back-propagation through one hidden layer whose input is `ain` (32 x K, row stride ldin) and
// whose pre-activation gradient is dz (32 x 128): gW[n][k] = sum_r dz[r][n] ain[r][k],
// gb[n] = sum_r dz[r][n] (written to the slot), and, if dprev is non-null (K = 128),
// dprev[r][k] = (sum_n dz[r][n] W[n][k]) (1 - ain[r][k]^2).
__device__ __forceinline__ void dense_back(const float *dz, const float *ain, int ldin, int K, const float *W,
                                           float *gW, float *gb, float *dprev, int t, int w, int ci, int ck) {
    // weight gradient: rows n in [32 w, 32 w + 32), all K columns, reduction over the 32 rows r
    for (int nt = 0; nt < 2; ++nt)
        for (int k0 = 0; k0 < K; k0 += 16) {
            const int n0 = 32 * w + 16 * nt;
            v4f acc = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
            for (int r0 = 0; r0 < TB; r0 += 4) acc = mfma4(dz[(r0 + ck) * LDA + n0 + ci], ain[(r0 + ck) * ldin + k0 + ci], acc);
#pragma unroll
            for (int i = 0; i < 4; ++i) gW[(int64_t)(n0 + 4 * ck + i) * K + k0 + ci] = acc[i];
        }
    if (t < H) {
        float s = 0.0f;
        for (int r = 0; r < TB; ++r) s += dz[r * LDA + t];
        gb[t] = s;
    }
    if (!dprev) return;
    // input gradient: columns k in [32 w, 32 w + 32), all 32 rows, reduction over n
#pragma unroll
    for (int rt = 0; rt < 2; ++rt)
#pragma unroll
        for (int kt = 0; kt < 2; ++kt) {
            const int r0 = 16 * rt, k0 = 32 * w + 16 * kt;
            v4f acc = {0.0f, 0.0f, 0.0f, 0.0f};
            for (int n0 = 0; n0 < H; n0 += 4)
                acc = mfma4(dz[(r0 + ci) * LDA + n0 + ck], W[(int64_t)(n0 + ck) * K + k0 + ci], acc);
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int r = r0 + 4 * ck + i, k = k0 + ci;
                const float a = ain[r * ldin + k];
                dprev[r * LDA + k] = acc[i] * (1.0f - a * a);
            }
        }
}

template <bool TRAIN>
__global__ __launch_bounds__(256) void mlp_tile_kernel(TileArgs g) {
    __shared__ float sX[TB * LDX];
    __shared__ float sA[3][TB * LDA];
    __shared__ float sD[2][TB * LDA];
    __shared__ float sdY[TB][NO];
    __shared__ float sLoss[64];
    const int t = threadIdx.x, w = t >> 6, lane = t & 63, ci = lane & 15, ck = lane >> 4;
    const int64_t s0 = (int64_t)blockIdx.x * TB;
    const float *W1 = g.params + oW1, *b1 = g.params + ob1, *W2 = g.params + oW2, *b2 = g.params + ob2;
    const float *W3 = g.params + oW3, *b3 = g.params + ob3, *W4 = g.params + oW4, *b4 = g.params + ob4;
    for (int i = t; i < TB * FP; i += 256) {
        const int r = i / FP, k = i % FP;
        sX[r * LDX + k] = s0 + r < g.B ? g.X[(s0 + r) * FP + k] : 0.0f;
    }
    __syncthreads();
    dense_tanh(sX, LDX, FP, W1, b1, sA[0], w, ci, ck);
    __syncthreads();
    dense_tanh(sA[0], LDA, H, W2, b2, sA[1], w, ci, ck);
    __syncthreads();
    dense_tanh(sA[1], LDA, H, W3, b3, sA[2], w, ci, ck);
    __syncthreads();
    // outputs: thread t < 64 takes row t / 2, output t % 2
    if (t < 2 * TB) {
        const int r = t >> 1, o = t & 1;
        float y = b4[o];
        for (int k = 0; k < H; ++k) y = fmaf(sA[2][r * LDA + k], W4[o * H + k], y);
        const bool valid = s0 + r < g.B;
        if (g.Y && valid) g.Y[(s0 + r) * NO + o] = y;
        if (TRAIN) {
            const float d = valid ? y - g.T[(s0 + r) * NO + o] : 0.0f;
            sdY[r][o] = 2.0f * d * g.inv_B;
            sLoss[t] = d * d * g.inv_B;
        }
    }
    if (!TRAIN) return;
    __syncthreads();
    float *gp = g.partial + (int64_t)blockIdx.x * kNetParams;
    if (t == 0) {
        float s = 0.0f;
        for (int i = 0; i < 2 * TB; ++i) s += sLoss[i];
        g.loss_part[blockIdx.x] = s;
    }
    // output layer
    {
        const int o = t >> 7, k = t & (H - 1);
        float s = 0.0f;
        for (int r = 0; r < TB; ++r) s = fmaf(sdY[r][o], sA[2][r * LDA + k], s);
        gp[oW4 + o * H + k] = s;
        if (t < NO) {
            float sb = 0.0f;
            for (int r = 0; r < TB; ++r) sb += sdY[r][t];
            gp[ob4 + t] = sb;
        }
    }
    for (int i = t; i < TB * H; i += 256) {
        const int r = i / H, n = i % H;
        const float a = sA[2][r * LDA + n];
        sD[0][r * LDA + n] = (sdY[r][0] * W4[n] + sdY[r][1] * W4[H + n]) * (1.0f - a * a);
    }
    __syncthreads();
    dense_back(sD[0], sA[1], LDA, H, W3, gp + oW3, gp + ob3, sD[1], t, w, ci, ck);
    __syncthreads();
    dense_back(sD[1], sA[0], LDA, H, W2, gp + oW2, gp + ob2, sD[0], t, w, ci, ck);
    __syncthreads();
    dense_back(sD[0], sX, LDX, FP, W1, gp + oW1, gp + ob1, nullptr, t, w, ci, ck);
}

// grad[i] = sum over slots b = 0, 1, ... of partial[b][i]; loss = sum of the loss slots
// (thread 0 of block 0).
__global__ __launch_bounds__(256) void mlp_reduce_kernel(const float *__restrict__ partial, int slots,
                                                         const float *__restrict__ loss_part, float *__restrict__ grad,
                                                         float *__restrict__ loss) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < kNetParams) {
        float s = 0.0f;
        for (int b = 0; b < slots; ++b) s += partial[(int64_t)b * kNetParams + i];
        grad[i] = s;
    }
    if (i == 0 && loss) {
        float s = 0.0f;
        for (int b = 0; b < slots; ++b) s += loss_part[b];
        *loss = s;
    }
}

// Adam (Kingma and Ba, 2015), step counted from 1, bias corrections c1 = 1 - beta1^step,
// c2 = 1 - beta2^step computed on the host.
__global__ __launch_bounds__(256) void mlp_adam_kernel(float *__restrict__ params, const float *__restrict__ grad,
                                                       float *__restrict__ m, float *__restrict__ v, float lr,
                                                       float beta1, float beta2, float eps, float c1, float c2) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= kNetParams) return;
    const float gi = grad[i];
    const float mi = beta1 * m[i] + (1.0f - beta1) * gi;
    const float vi = beta2 * v[i] + (1.0f - beta2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    params[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// ---------------------------------------------------------------- FP16 inference

typedef _Float16 v4h __attribute__((ext_vector_type(4)));

// tanh x = 1 - 2 / (e^{2x} + 1) with the hardware exponential and reciprocal (relative error
// ~1e-6, far below the FP16 rounding of the activations that follows); saturates to +-1.
__device__ __forceinline__ float tanh_fast(float x) {
    const float e = __expf(2.0f * x);
    return 1.0f - 2.0f * __builtin_amdgcn_rcpf(e + 1.0f);
}

__device__ __forceinline__ v4f mfma16(v4h a, v4h b, v4f c) {
    return __builtin_amdgcn_mfma_f32_16x16x16f16(a, b, c, 0, 0, 0);
}

// FP16 weights in MFMA fragment order: tile (nb, kb) of a weight matrix W (16 rows 16 nb ..,
// 16 columns 16 kb ..) is 64 lanes x 4 halves, lane ci + 16 ck holding W[16 nb + ci][16 kb +
// 4 ck .. + 3]; tiles of W1 (8 x 2), W2 (8 x 8), W3 (8 x 8), then W4 padded to 16 rows (1 x 8).
constexpr int kFragW1 = 0, kFragW2 = 16, kFragW3 = 80, kFragW4 = 144, kFragTiles = 152;

__global__ __launch_bounds__(256) void net_pack_kernel(const float *__restrict__ params, v4h *__restrict__ frag) {
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;  // tile * 64 + lane
    if (idx >= kFragTiles * 64) return;
    const int tile = idx >> 6, lane = idx & 63, ci = lane & 15, ck = lane >> 4;
    const float *W;
    int K, nb, kb, rows;
    if (tile < kFragW2) {
        W = params + oW1, K = FP, nb = tile / 2, kb = tile % 2, rows = H;
    } else if (tile < kFragW3) {
        W = params + oW2, K = H, nb = (tile - kFragW2) / 8, kb = (tile - kFragW2) % 8, rows = H;
    } else if (tile < kFragW4) {
        W = params + oW3, K = H, nb = (tile - kFragW3) / 8, kb = (tile - kFragW3) % 8, rows = H;
    } else {
        W = params + oW4, K = H, nb = 0, kb = tile - kFragW4, rows = NO;
    }
    const int n = 16 * nb + ci;
    v4h v;
#pragma unroll
    for (int i = 0; i < 4; ++i) v[i] = (_Float16)(n < rows ? W[(int64_t)n * K + 16 * kb + 4 * ck + i] : 0.0f);
    frag[idx] = v;
}

// Distance from the unit-frame target (u, v, w) to the triangle (0,0), (1,0), (p,q).
__device__ __forceinline__ double unit_distance(double p, double q, double u, double v, double w) {
    // barycentric test of the projection
    const double d00 = 1.0, d01 = p, d11 = p * p + q * q, d20 = u, d21 = u * p + v * q;
    const double den = d00 * d11 - d01 * d01;
    const double lb = (d11 * d20 - d01 * d21) / den, lc = (d00 * d21 - d01 * d20) / den;
    if (lb >= 0.0 && lc >= 0.0 && lb + lc <= 1.0) return w;
    auto seg = [&](double ax, double ay, double bx, double by) {
        const double dx = bx - ax, dy = by - ay;
        double t = ((u - ax) * dx + (v - ay) * dy) / (dx * dx + dy * dy);
        t = fmin(fmax(t, 0.0), 1.0);
        const double ex = u - (ax + t * dx), ey = v - (ay + t * dy);
        return sqrt(ex * ex + ey * ey + w * w);
    };
    return fmin(fmin(seg(0.0, 0.0, 1.0, 0.0), seg(1.0, 0.0, p, q)), seg(p, q, 0.0, 0.0));
}

struct NetFoldArgs {
    const double4 *colloc;
    const double *vtx;
    const int64_t *rowptr;
    const int32_t *col;
    int64_t n, npairs;
    const double2 *kappa;  // N nodes
    int N;
    const double2 *W;      // N x Pstride moment weights; this launch folds columns p0 .. p0 + P - 1
    int Pstride, p0, P;
    const v4h *frag;       // packed FP16 weights
    const float *params;   // FP32 parameters (biases)
    double S_re, S_im;     // output scales
    // trust region: pairs outside use the quadrature
    double dmin, tan_min, kh_re_max, kh_im_max, kre_max, kim_max;
    double bin_edges[kNetBins + 1];
    int bin_ok[kNetBins];
    double2 *F;            // npairs x Pstride folded corrections
    unsigned char *flag;   // npairs: 1 = quadrature
    const int *nodes;      // nodes with a nonzero weight in this launch's columns (all N when null)
    int nnodes;
    const double2 *Wsum;   // frozen wavenumber: sum_j W[j][p0 + p], p < P
    double2 kc;
    double h2max;
};

constexpr int kNetWaves = 8;     // waves per workgroup (one LDS copy of the weights)
constexpr int64_t kPairChunk = 64;  // pairs per chunk of the quadrature kernel's apply phase

__global__ __launch_bounds__(64 * kNetWaves) __attribute__((amdgpu_waves_per_eu(4, 4))) void net_fold_kernel(NetFoldArgs g) {
    __shared__ v4h sW[kFragTiles * 64];
    __shared__ float sB[3 * H + NO];
    __shared__ float sF[kNetWaves][kNetInPad];  // each wave's pair inputs (5, 6 and 19.. zero)
    for (int i = threadIdx.x; i < kFragTiles * 64; i += blockDim.x) sW[i] = g.frag[i];
    for (int i = threadIdx.x; i < 3 * H + NO; i += blockDim.x)
        sB[i] = i < H ? g.params[ob1 + i] : i < 2 * H ? g.params[ob2 + i - H] : i < 3 * H ? g.params[ob3 + i - 2 * H]
                                                                                            : g.params[ob4 + i - 3 * H];
    __syncthreads();
    const int lane = threadIdx.x & 63, ci = lane & 15, ck = lane >> 4;
    const int64_t wave = (int64_t)blockIdx.x * kNetWaves + (threadIdx.x >> 6);
    const int64_t nwaves = (int64_t)gridDim.x * kNetWaves;
    const double inv4pi = 0.25 / 3.14159265358979323846;
    // each wave takes a contiguous range of pairs; its first row by bisection of rowptr, the
    // next ones by stepping (uniform over the wave)
    const int64_t per = (g.npairs + nwaves - 1) / nwaves;
    const int64_t k0 = wave * per, k1 = k0 + per < g.npairs ? k0 + per : g.npairs;
    int64_t a = 0;
    if (k0 < k1) {
        int64_t lo = 0, hi = g.n;  // rowptr[lo] <= k0 < rowptr[hi]
        while (hi - lo > 1) {
            const int64_t mid = (lo + hi) / 2;
            if (g.rowptr[mid] <= k0) lo = mid;
            else hi = mid;
        }
        a = lo;
    }
    for (int64_t k = k0; k < k1; ++k) {
        while (g.rowptr[a + 1] <= k) ++a;
        const int64_t b = g.col[k];
        double P[3][3];
        for (int v = 0; v < 3; ++v)
            for (int c = 0; c < 3; ++c) P[v][c] = g.vtx[9 * b + 3 * v + c];
        const double4 xa = g.colloc[a];
        const double x[3] = {xa.x, xa.y, xa.z};
        double p, q, u, v, w, h, r0;
        net_frame(P, x, p, q, u, v, w, h);
        float f[kNetIn];
        net_geometry_inputs(p, q, u, v, w, f, r0);
        // trust region (uniform over the wave)
        const double dist = unit_distance(p, q, u, v, w);
        bool ok = dist >= g.dmin && q >= (1.0 - p) * g.tan_min && q >= p * g.tan_min && g.kre_max * h <= g.kh_re_max &&
                  g.kim_max * h <= g.kh_im_max;
        if (ok) {
            int bin = -1;
            for (int i = 0; i < kNetBins; ++i)
                if (dist >= g.bin_edges[i] && dist < g.bin_edges[i + 1]) bin = i;
            ok = bin >= 0 && g.bin_ok[bin];
        }
        if (!ok) {
            if (lane == 0) g.flag[k] = 1;
            if (lane < g.P) g.F[k * g.Pstride + g.p0 + lane] = make_double2(0.0, 0.0);
            continue;
        }
        // stage the 17 geometric inputs in the wave's slot: lanes read their 8 by index
        float *fw = sF[threadIdx.x >> 6];
#pragma unroll
        for (int i = 0; i < kNetIn; ++i)
            if (lane == i) fw[i] = f[i];
        if (lane >= kNetIn && lane < kNetInPad) fw[lane] = 0.0f;
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        double accr[kNetMaxP], acci[kNetMaxP];
#pragma unroll
        for (int i = 0; i < kNetMaxP; ++i) accr[i] = acci[i] = 0.0;
        const double scale = h * inv4pi / (r0 * r0 * r0 * r0);
        const int nn = g.nodes ? g.nnodes : g.N;
        for (int j0 = 0; j0 < nn; j0 += 16) {
            // one sample block: the (j0 + ci)-th node of the list in the lanes of column ci
            const int jj = j0 + ci;
            const int j = jj < nn ? (g.nodes ? g.nodes[jj] : jj) : g.N;
            const double2 kj = j < g.N ? g.kappa[j] : make_double2(0.0, 0.0);
            v4h xin[2];
#pragma unroll
            for (int kb = 0; kb < 2; ++kb)
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int kk = 16 * kb + 4 * ck + i;
                    const float fv = kk == 5 ? (float)(2.0 * kj.x * h - 1.0)
                                   : kk == 6 ? (float)(kj.y * h / 0.3)
                                   : fw[kk];
                    xin[kb][i] = (_Float16)fv;
                }
            // layer 1 (K = 32), then the two hidden layers (K = 128): activations stay in the
            // B-operand layout (lane ci + 16 ck holds rows 4 ck .. 4 ck + 3 of each 16-row block)
            v4h act[8];
#pragma unroll
            for (int nb = 0; nb < 8; ++nb) {
                v4f d = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
                for (int kb = 0; kb < 2; ++kb) d = mfma16(sW[(kFragW1 + nb * 2 + kb) * 64 + lane], xin[kb], d);
#pragma unroll
                for (int i = 0; i < 4; ++i) act[nb][i] = (_Float16)tanh_fast(d[i] + sB[16 * nb + 4 * ck + i]);
            }
#pragma unroll
            for (int layer = 0; layer < 2; ++layer) {
                const int base = layer == 0 ? kFragW2 : kFragW3;
                const float *bias = sB + H * (layer + 1);
                v4f d[8];
#pragma unroll
                for (int nb = 0; nb < 8; ++nb) {
                    d[nb] = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
                    for (int kb = 0; kb < 8; ++kb) d[nb] = mfma16(sW[(base + nb * 8 + kb) * 64 + lane], act[kb], d[nb]);
                    __builtin_amdgcn_sched_barrier(0);  // keep each block's fragment loads with its MFMAs
                }
#pragma unroll
                for (int nb = 0; nb < 8; ++nb)
#pragma unroll
                    for (int i = 0; i < 4; ++i) act[nb][i] = (_Float16)tanh_fast(d[nb][i] + bias[16 * nb + 4 * ck + i]);
            }
            // outputs: rows 0 and 1 of the padded output tile, in lanes ck = 0 (registers 0, 1)
            v4f y = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int kb = 0; kb < 8; ++kb) y = mfma16(sW[(kFragW4 + kb) * 64 + lane], act[kb], y);
            // dT of node j (lanes ck == 0), folded with the weights; other lanes add nothing
            if (ck == 0 && j < g.N) {
                const double tr = scale * g.S_re * (double)(y[0] + sB[3 * H]);
                const double ti = scale * g.S_im * (double)(y[1] + sB[3 * H + 1]);
#pragma unroll
                for (int pp = 0; pp < kNetMaxP; ++pp) {
                    if (pp < g.P) {
                        const double2 wj = g.W[(int64_t)j * g.Pstride + g.p0 + pp];
                        accr[pp] += wj.x * tr - wj.y * ti;
                        acci[pp] += wj.x * ti + wj.y * tr;
                    }
                }
            }
        }
        // sum over the 16 sample lanes (fixed order: butterfly within lanes 0..15)
#pragma unroll
        for (int pp = 0; pp < kNetMaxP; ++pp) {
#pragma unroll
            for (int off = 8; off >= 1; off >>= 1) {
                accr[pp] += __shfl_xor(accr[pp], off, 16);
                acci[pp] += __shfl_xor(acci[pp], off, 16);
            }
        }
        if (lane == 0) {
            g.flag[k] = 0;
#pragma unroll
            for (int pp = 0; pp < kNetMaxP; ++pp)
                if (pp < g.P) g.F[k * g.Pstride + g.p0 + pp] = make_double2(accr[pp], acci[pp]);
        }
    }
}

// Frozen-wavenumber inference: the correction of a pair is taken as its value at the centre kc
// of the node set for every node (dT depends on kappa only through the rule's error on the
// smooth part of the kernel, so it changes over the nodes by about max_j |z_j - kc| |kappa|
// h^2 relative; the host turns the caller's bound on that into h2max).  A wave evaluates 16
// pairs per pass, one per MFMA column (the four lanes of a column form its pair's inputs),
// and F[k][p0 + p] = dT_k(kc) Wsum[p] for every p < P.
__global__ __launch_bounds__(64 * kNetWaves) __attribute__((amdgpu_waves_per_eu(4, 4))) void net_fold_frozen_kernel(
    NetFoldArgs g) {
    __shared__ v4h sW[kFragTiles * 64];
    __shared__ float sB[3 * H + NO];
    __shared__ float sF[kNetWaves][16][kNetInPad + 1];  // each wave's 16 pairs' inputs
    for (int i = threadIdx.x; i < kFragTiles * 64; i += blockDim.x) sW[i] = g.frag[i];
    for (int i = threadIdx.x; i < 3 * H + NO; i += blockDim.x)
        sB[i] = i < H ? g.params[ob1 + i] : i < 2 * H ? g.params[ob2 + i - H] : i < 3 * H ? g.params[ob3 + i - 2 * H]
                                                                                            : g.params[ob4 + i - 3 * H];
    __syncthreads();
    const int lane = threadIdx.x & 63, ci = lane & 15, ck = lane >> 4, wv = threadIdx.x >> 6;
    const int64_t wave = (int64_t)blockIdx.x * kNetWaves + wv;
    const int64_t nwaves = (int64_t)gridDim.x * kNetWaves;
    const double inv4pi = 0.25 / 3.14159265358979323846;
    // contiguous ranges of whole 16-pair passes per wave
    const int64_t passes = (g.npairs + 15) / 16;
    const int64_t per = (passes + nwaves - 1) / nwaves;
    const int64_t k0 = wave * per * 16;
    const int64_t k1 = k0 + per * 16 < g.npairs ? k0 + per * 16 : g.npairs;
    int64_t a = 0;  // row of the wave's current pass start (uniform)
    if (k0 < k1) {
        int64_t lo = 0, hi = g.n;  // rowptr[lo] <= k0 < rowptr[hi]
        while (hi - lo > 1) {
            const int64_t mid = (lo + hi) / 2;
            if (g.rowptr[mid] <= k0) lo = mid;
            else hi = mid;
        }
        a = lo;
    }
    float(*fw)[kNetInPad + 1] = sF[wv];
    for (int64_t kb = k0; kb < k1; kb += 16) {
        const int64_t k = kb + ci;
        const bool have = k < k1;
        int64_t ak = a;
        if (have)
            while (g.rowptr[ak + 1] <= k) ++ak;
        // the pass's last pair's row starts the next pass
        a = __shfl(ak, 15);
        bool ok = false;
        double scale = 0.0;
        if (have) {
            const int64_t b = g.col[k];
            double P[3][3];
            for (int v = 0; v < 3; ++v)
                for (int c = 0; c < 3; ++c) P[v][c] = g.vtx[9 * b + 3 * v + c];
            const double4 xa = g.colloc[ak];
            const double x[3] = {xa.x, xa.y, xa.z};
            double p, q, u, v, w, h, r0;
            net_frame(P, x, p, q, u, v, w, h);
            float f[kNetIn];
            net_geometry_inputs(p, q, u, v, w, f, r0);
            const double dist = unit_distance(p, q, u, v, w);
            ok = dist >= g.dmin && q >= (1.0 - p) * g.tan_min && q >= p * g.tan_min && g.kre_max * h <= g.kh_re_max &&
                 g.kim_max * h <= g.kh_im_max && h * h <= g.h2max;
            if (ok) {
                int bin = -1;
                for (int i = 0; i < kNetBins; ++i)
                    if (dist >= g.bin_edges[i] && dist < g.bin_edges[i + 1]) bin = i;
                ok = bin >= 0 && g.bin_ok[bin];
            }
            f[5] = (float)(2.0 * g.kc.x * h - 1.0);
            f[6] = (float)(g.kc.y * h / 0.3);
            scale = h * inv4pi / (r0 * r0 * r0 * r0);
            if (ck == 0) {
#pragma unroll
                for (int i = 0; i < kNetIn; ++i) fw[ci][i] = f[i];
#pragma unroll
                for (int i = kNetIn; i < kNetInPad; ++i) fw[ci][i] = 0.0f;
            }
        } else if (ck == 0) {
#pragma unroll
            for (int i = 0; i < kNetInPad; ++i) fw[ci][i] = 0.0f;
        }
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        v4h xin[2];
#pragma unroll
        for (int kbk = 0; kbk < 2; ++kbk)
#pragma unroll
            for (int i = 0; i < 4; ++i) xin[kbk][i] = (_Float16)fw[ci][16 * kbk + 4 * ck + i];
        v4h act[8];
#pragma unroll
        for (int nb = 0; nb < 8; ++nb) {
            v4f d = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int kbk = 0; kbk < 2; ++kbk) d = mfma16(sW[(kFragW1 + nb * 2 + kbk) * 64 + lane], xin[kbk], d);
#pragma unroll
            for (int i = 0; i < 4; ++i) act[nb][i] = (_Float16)tanh_fast(d[i] + sB[16 * nb + 4 * ck + i]);
        }
#pragma unroll
        for (int layer = 0; layer < 2; ++layer) {
            const int base = layer == 0 ? kFragW2 : kFragW3;
            const float *bias = sB + H * (layer + 1);
            v4f d[8];
#pragma unroll
            for (int nb = 0; nb < 8; ++nb) {
                d[nb] = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
                for (int kbk = 0; kbk < 8; ++kbk) d[nb] = mfma16(sW[(base + nb * 8 + kbk) * 64 + lane], act[kbk], d[nb]);
                __builtin_amdgcn_sched_barrier(0);
            }
#pragma unroll
            for (int nb = 0; nb < 8; ++nb)
#pragma unroll
                for (int i = 0; i < 4; ++i) act[nb][i] = (_Float16)tanh_fast(d[nb][i] + bias[16 * nb + 4 * ck + i]);
        }
        v4f y = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int kbk = 0; kbk < 8; ++kbk) y = mfma16(sW[(kFragW4 + kbk) * 64 + lane], act[kbk], y);
        // column ci's outputs sit in lane ci (ck == 0), registers 0 and 1
        if (have && ck == 0) {
            g.flag[k] = ok ? 0 : 1;
            const double tr = ok ? scale * g.S_re * (double)(y[0] + sB[3 * H]) : 0.0;
            const double ti = ok ? scale * g.S_im * (double)(y[1] + sB[3 * H + 1]) : 0.0;
            for (int pp = 0; pp < g.P; ++pp) {
                const double2 ws = g.Wsum[pp];
                g.F[k * g.Pstride + g.p0 + pp] = make_double2(ws.x * tr - ws.y * ti, ws.x * ti + ws.y * tr);
            }
        }
        __builtin_amdgcn_wave_barrier();  // the inputs of this pass are read before the next is staged
    }
}

// M[p][a, :] += sum over the pairs k of row a of F[k * Fstride + p] V[col[k], :], p < P <= kNfFold,
// added in chunks of 64 pairs in the order of the list, as the per-node quadrature kernel applies
// its folds (so a model that trusts no pair reproduces the quadrature's moments bitwise).
template <int PC>
__global__ __launch_bounds__(256) void pair_apply_kernel(const int64_t *__restrict__ rowptr,
                                                         const int32_t *__restrict__ col,
                                                         const double2 *__restrict__ F, int Fstride,
                                                         const double2 *__restrict__ V, int64_t ldv, int64_t m,
                                                         double2 *__restrict__ M, int64_t ldm, int64_t mstride,
                                                         int64_t n, int64_t nblocks) {
    // one wave per row, its lanes over the columns, the PC weight sets of the launch per lane;
    // rows in contiguous ranges per XCD (block i runs on XCD i % 8), so neighbouring rows,
    // which share most of their near triangles' rows of V, meet in the same L2
    const int64_t per = (nblocks + 7) / 8;
    const int64_t blk = (int64_t)(blockIdx.x % 8) * per + blockIdx.x / 8;
    // the row is uniform over the wave: say so, so that the list and the folds are read
    // through the scalar cache
    const int64_t a = blk * 4 + __builtin_amdgcn_readfirstlane((int)(threadIdx.x / 64));
    if (blk >= nblocks || a >= n) return;
    const int lane = threadIdx.x % 64;
    const int64_t beg = rowptr[a], end = rowptr[a + 1];
    if (beg == end) return;
    for (int64_t c = lane; c < m; c += 64) {
        double2 o[PC];
#pragma unroll
        for (int p = 0; p < PC; ++p) o[p] = M[p * mstride + a * ldm + c];
        // pairs in chunks of kPairChunk, each chunk's sum added to the running value (the
        // order of the per-node kernel's own apply phase)
        for (int64_t base = beg; base < end; base += kPairChunk) {
            const int64_t stop = end - base < kPairChunk ? end : base + kPairChunk;
            double sr[PC], si[PC];
#pragma unroll
            for (int p = 0; p < PC; ++p) sr[p] = si[p] = 0.0;
#pragma unroll 8
            for (int64_t k = base; k < stop; ++k) {
                const double2 v = V[(int64_t)col[k] * ldv + c];
#pragma unroll
                for (int p = 0; p < PC; ++p) {
                    const double2 f = F[k * Fstride + p];
                    // the per-node kernel's fused steps, for bitwise equal results
                    sr[p] = fma(-f.y, v.y, fma(f.x, v.x, sr[p]));
                    si[p] = fma(f.y, v.x, fma(f.x, v.y, si[p]));
                }
            }
#pragma unroll
            for (int p = 0; p < PC; ++p) o[p] = make_double2(o[p].x + sr[p], o[p].y + si[p]);
        }
#pragma unroll
        for (int p = 0; p < PC; ++p) M[p * mstride + a * ldm + c] = o[p];
    }
}

}  // namespace

hipError_t launch_net_features(const double *P9, const double *x, const double2 *kappa, int64_t S, float *X, double *aux,
                               hipStream_t stream) {
    if (S <= 0) return hipSuccess;
    hipLaunchKernelGGL(net_features_kernel, dim3((unsigned)((S + 255) / 256)), dim3(256), 0, stream, P9, x, kappa, S, X,
                       aux);
    return hipGetLastError();
}

int64_t net_slots(int64_t B) { return (B + TB - 1) / TB; }

hipError_t launch_net_forward(const float *params, const float *X, int64_t B, float *Y, hipStream_t stream) {
    if (B <= 0) return hipSuccess;
    TileArgs g{};
    g.params = params;
    g.X = X;
    g.B = B;
    g.Y = Y;
    hipLaunchKernelGGL(mlp_tile_kernel<false>, dim3((unsigned)net_slots(B)), dim3(256), 0, stream, g);
    return hipGetLastError();
}

hipError_t launch_net_gradient(const float *params, const float *X, const float *T, int64_t B, float *partial,
                               float *loss_part, float *grad, float *loss, hipStream_t stream) {
    if (B <= 0) return hipErrorInvalidValue;
    TileArgs g{};
    g.params = params;
    g.X = X;
    g.T = T;
    g.B = B;
    g.inv_B = 1.0f / (float)B;
    g.partial = partial;
    g.loss_part = loss_part;
    const int slots = (int)net_slots(B);
    hipLaunchKernelGGL(mlp_tile_kernel<true>, dim3((unsigned)slots), dim3(256), 0, stream, g);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(mlp_reduce_kernel, dim3((unsigned)((kNetParams + 255) / 256)), dim3(256), 0, stream, partial,
                       slots, loss_part, grad, loss);
    return hipGetLastError();
}

hipError_t launch_net_adam(float *params, const float *grad, float *m, float *v, float lr, float beta1, float beta2,
                           float eps, float c1, float c2, hipStream_t stream) {
    hipLaunchKernelGGL(mlp_adam_kernel, dim3((unsigned)((kNetParams + 255) / 256)), dim3(256), 0, stream, params, grad, m,
                       v, lr, beta1, beta2, eps, c1, c2);
    return hipGetLastError();
}

int64_t net_frag_bytes() { return (int64_t)kFragTiles * 64 * sizeof(v4h); }

hipError_t launch_net_pack(const float *params, void *frag, hipStream_t stream) {
    hipLaunchKernelGGL(net_pack_kernel, dim3((kFragTiles * 64 + 255) / 256), dim3(256), 0, stream, params,
                       static_cast<v4h *>(frag));
    return hipGetLastError();
}

hipError_t launch_net_fold(const NetFoldParams &q, hipStream_t stream) {
    if (q.npairs <= 0) return hipSuccess;
    if (q.P < 1 || (!q.Wsum && q.P > kNetMaxP)) return hipErrorInvalidValue;
    NetFoldArgs g;
    g.colloc = q.mesh->colloc;
    g.vtx = q.mesh->vtx;
    g.rowptr = q.rowptr;
    g.col = q.col;
    g.n = q.mesh->n;
    g.npairs = q.npairs;
    g.kappa = q.kappa;
    g.N = q.N;
    g.W = q.W;
    g.Pstride = q.Pstride;
    g.p0 = q.p0;
    g.P = q.P;
    g.frag = static_cast<const v4h *>(q.frag);
    g.params = q.params;
    g.S_re = q.S_re;
    g.S_im = q.S_im;
    g.dmin = q.dmin;
    g.tan_min = q.tan_min;
    g.kh_re_max = q.kh_re_max;
    g.kh_im_max = q.kh_im_max;
    g.kre_max = q.kre_max;
    g.kim_max = q.kim_max;
    for (int i = 0; i <= kNetBins; ++i) g.bin_edges[i] = q.bin_edges[i];
    for (int i = 0; i < kNetBins; ++i) g.bin_ok[i] = q.bin_ok[i];
    g.F = q.F;
    g.flag = q.flag;
    g.nodes = q.nodes;
    g.nnodes = q.nnodes;
    g.Wsum = q.Wsum;
    g.kc = q.kc;
    g.h2max = q.h2max;
    int cus = 256, dev = 0;
    if (hipGetDevice(&dev) == hipSuccess) (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (q.Wsum) {
        const int64_t passes = (q.npairs + 15) / 16;
        const int64_t want = (passes + kNetWaves - 1) / kNetWaves;
        const unsigned grid = (unsigned)(want < 2 * cus ? want : 2 * cus);
        hipLaunchKernelGGL(net_fold_frozen_kernel, dim3(grid), dim3(64 * kNetWaves), 0, stream, g);
        return hipGetLastError();
    }
    const int64_t want = (q.npairs + kNetWaves - 1) / kNetWaves;
    const unsigned grid = (unsigned)(want < 2 * cus ? want : 2 * cus);
    hipLaunchKernelGGL(net_fold_kernel, dim3(grid), dim3(64 * kNetWaves), 0, stream, g);
    return hipGetLastError();
}

hipError_t launch_pair_apply(const DeviceMesh &mesh, const int64_t *rowptr, const int32_t *col, const double2 *F, int P,
                             const double2 *V, int64_t ldv, int64_t m, double2 *M, int64_t ldm, hipStream_t stream) {
    const int64_t nblocks = (mesh.n + 3) / 4;
    const dim3 grid((unsigned)((nblocks + 7) / 8 * 8));
    // the sets in launches of 8, then 4, 2 and 1 (each set's sums are the same whichever
    // launch carries it)
    for (int p0 = 0; p0 < P;) {
        const int left = P - p0;
        const int pc = left >= 8 ? 8 : left >= 4 ? 4 : left >= 2 ? 2 : 1;
        const double2 *Fp = F + p0;
        double2 *Mp = M + (int64_t)p0 * mesh.n * ldm;
        switch (pc) {
        case 8:
            hipLaunchKernelGGL(pair_apply_kernel<8>, grid, dim3(256), 0, stream, rowptr, col, Fp, P, V, ldv, m, Mp, ldm,
                               mesh.n * ldm, mesh.n, nblocks);
            break;
        case 4:
            hipLaunchKernelGGL(pair_apply_kernel<4>, grid, dim3(256), 0, stream, rowptr, col, Fp, P, V, ldv, m, Mp, ldm,
                               mesh.n * ldm, mesh.n, nblocks);
            break;
        case 2:
            hipLaunchKernelGGL(pair_apply_kernel<2>, grid, dim3(256), 0, stream, rowptr, col, Fp, P, V, ldv, m, Mp, ldm,
                               mesh.n * ldm, mesh.n, nblocks);
            break;
        default:
            hipLaunchKernelGGL(pair_apply_kernel<1>, grid, dim3(256), 0, stream, rowptr, col, Fp, P, V, ldv, m, Mp, ldm,
                               mesh.n * ldm, mesh.n, nblocks);
            break;
        }
        p0 += pc;
    }
    return hipGetLastError();
}

}  // namespace bemrat

