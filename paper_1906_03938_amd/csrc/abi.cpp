// C ABI of libbemrat.so (declared in include/bemrat.h): argument checks, handle and
// workspace management, choice of sweep form, host-side node/weight construction, and
// the launch sequence of each call.  All numerical work on the operator runs in the HIP
// kernels of mesh.hip, sweep.hip and combine.hip.
#include "bemrat.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <complex>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "internal.h"
#include "block_combine.h"

using bemrat::DeviceMesh;
using cplx = std::complex<double>;

namespace {

thread_local std::string g_error;

bem_status fail(bem_status s, const std::string &msg) {
    g_error = msg;
    return s;
}

bem_status hip_fail(hipError_t e, const char *what) {
    g_error = std::string(what) + ": " + hipGetErrorString(e);
    return e == hipErrorOutOfMemory ? BEM_ENOMEM : BEM_EDEVICE;
}

#define HIP_TRY(expr, what)                          \
    do {                                             \
        hipError_t e_ = (expr);                      \
        if (e_ != hipSuccess) return hip_fail(e_, what); \
    } while (0)

// Device buffer that only grows.
struct Buffer {
    void *ptr = nullptr;
    size_t bytes = 0;
    hipError_t ensure(size_t need) {
        if (need <= bytes) return hipSuccess;
        if (ptr) {
            hipError_t e = hipFree(ptr);
            ptr = nullptr;
            bytes = 0;
            if (e != hipSuccess) return e;
        }
        hipError_t e = hipMalloc(&ptr, need);
        if (e != hipSuccess) {
            ptr = nullptr;
            return e;
        }
        bytes = need;
        return hipSuccess;
    }
    void release() {
        if (ptr) (void)hipFree(ptr);
        ptr = nullptr;
        bytes = 0;
    }
    template <class T>
    T *as() const { return static_cast<T *>(ptr); }
};

// Capacity of a handle's pinned parameter staging from its creation on (the allocation-free
// entry point takes parameter blocks up to this size).
constexpr size_t kStagingBytes = size_t(1) << 20;

// Pinned host staging for per-call parameters; reused once its last upload completed.
struct Staging {
    void *host = nullptr;
    size_t bytes = 0;
    hipEvent_t done = nullptr;
    bool pending = false;
    hipError_t ensure(size_t need) {
        if (pending) {
            hipError_t e = hipEventSynchronize(done);
            if (e != hipSuccess) return e;
            pending = false;
        }
        if (need <= bytes) return hipSuccess;
        if (host) (void)hipHostFree(host);
        host = nullptr;
        bytes = 0;
        hipError_t e = hipHostMalloc(&host, need, hipHostMallocDefault);
        if (e != hipSuccess) {
            host = nullptr;
            return e;
        }
        bytes = need;
        return hipSuccess;
    }
};

}  // namespace

struct bem_mesh {
    int device = 0;
    DeviceMesh dm;
    double diameter = 0.0;  // upper bound on every distance in the operator
    double mean_area = 0.0; // mean triangle area (sets the scale of reduced-precision entries)
    Buffer geom, gl, self, aux, Z, params, partial, probe, vmax, fself;
    // near field: host centroids and squared longest edges (the list's test), device list
    std::vector<double> nf_cen, nf_h2;
    Buffer nf_rowptr, nf_col, nf_gl;
    Buffer nf_row, nf_F;  // row of each pair; the series form's folded corrections of a chunk
    Buffer net_frag, net_F, net_flag;  // learned correction: packed weights, folds, fallback flags
    int64_t nf_pairs = 0;
    double nf_eta = 0.0;
    double nf_rmax = 0.0;    // bound on the distance from a pair's target to its triangle
    int nf_mode = BEM_NF_AUTO;
    int nf_last_terms = 0;   // series terms of the last near-field call (0: per node)
    Staging staging;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    bool timing = false, timed = false;
    uint32_t last_form = 0;
    int64_t last_ops = 0;
};

namespace {

struct DeviceGuard {
    int prev = -1;
    explicit DeviceGuard(int dev) {
        if (hipGetDevice(&prev) == hipSuccess && prev != dev) (void)hipSetDevice(dev);
        else prev = -1;
    }
    ~DeviceGuard() {
        if (prev >= 0) (void)hipSetDevice(prev);
    }
};

bool finite_c(const double *p, int64_t count) {
    for (int64_t i = 0; i < 2 * count; ++i)
        if (!std::isfinite(p[i])) return false;
    return true;
}

// True when `p` is device (or managed) memory usable by kernels of the current device.
bool is_device_ptr(const void *p) {
    if (!p) return false;
    hipPointerAttribute_t attr;
    hipError_t e = hipPointerGetAttributes(&attr, p);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    return attr.type == hipMemoryTypeDevice || attr.type == hipMemoryTypeManaged;
}

bem_status check_block(const void *p, int64_t m, int64_t ld, const char *name) {
    if (!p) return fail(BEM_EINVAL, std::string(name) + " is NULL");
    if (m <= 0) return fail(BEM_EINVAL, "m must be positive");
    if (ld < m) return fail(BEM_EINVAL, std::string("leading dimension of ") + name + " is smaller than m");
    if (!is_device_ptr(p)) return fail(BEM_EINVAL, std::string(name) + " is not device memory");
    return BEM_OK;
}

bem_status check_flags(uint32_t flags) {
    if (flags & ~(BEM_FORM_MASK | BEM_PREC_MASK)) return fail(BEM_EINVAL, "unknown flag bits");
    if ((flags & BEM_PREC_MASK) > BEM_PREC_F16) return fail(BEM_EUNSUPPORTED, "unknown arithmetic");
    return BEM_OK;
}

bem_status check_kappas(const bem_mesh *h, const double *k, int64_t nk, const char *name) {
    if (!k) return fail(BEM_EINVAL, std::string(name) + " is NULL");
    if (nk < 1) return fail(BEM_EINVAL, std::string("number of ") + name + " must be positive");
    if (!finite_c(k, nk)) return fail(BEM_EINVAL, std::string(name) + " has a non-finite value");
    for (int64_t i = 0; i < nk; ++i)
    {
        if (std::fabs(k[2 * i + 1]) * h->diameter > 700.0)
            return fail(BEM_EINVAL, std::string(name) + ": |Im kappa| x mesh diameter exceeds 700 (exp overflow)");
        if (std::fabs(k[2 * i]) * h->diameter > 1e6)
            return fail(BEM_EINVAL, std::string(name) + ": |Re kappa| x mesh diameter exceeds 1e6");
    }
    return BEM_OK;
}

// Radon's degree-5 seven-point rule: barycentric coordinates (7 x 3) then weights (7),
// weights summing to one.
void radon_rule(double *rule) {
    const double s = std::sqrt(15.0);
    const double p1 = (6.0 - s) / 21.0, q1 = (9.0 + 2.0 * s) / 21.0;  // orbit near vertices
    const double p2 = (6.0 + s) / 21.0, q2 = (9.0 - 2.0 * s) / 21.0;  // orbit near edges
    const double wv = (155.0 - s) / 1200.0, we = (155.0 + s) / 1200.0;
    const double pts[7][3] = {{1.0 / 3.0, 1.0 / 3.0, 1.0 / 3.0}, {q1, p1, p1}, {p1, q1, p1},
                              {p1, p1, q1}, {q2, p2, p2}, {p2, q2, p2}, {p2, p2, q2}};
    const double w[7] = {0.225, wv, wv, wv, we, we, we};
    for (int q = 0; q < 7; ++q) {
        for (int c = 0; c < 3; ++c) rule[3 * q + c] = pts[q][c];
        rule[21 + q] = w[q];
    }
}

// Gauss-Legendre rule of order n on [-1, 1]: Newton iteration on P_n from the
// asymptotic initial guesses, P_n and P_n' by the Bonnet recurrence.
void gauss_legendre(int n, double *x, double *w) {
    const double pi = 3.14159265358979323846;
    for (int i = 0; i < n; ++i) {
        double t = std::cos(pi * (4.0 * i + 3.0) / (4.0 * n + 2.0));
        double dp = 1.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = t;
            for (int k = 2; k <= n; ++k) {
                const double p2 = ((2.0 * k - 1.0) * t * p1 - (k - 1.0) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            dp = n * (t * p1 - p0) / (t * t - 1.0);
            const double dt = p1 / dp;
            t -= dt;
            if (std::fabs(dt) < 1e-16) break;
        }
        double p0 = 1.0, p1 = t;
        for (int k = 2; k <= n; ++k) {
            const double p2 = ((2.0 * k - 1.0) * t * p1 - (k - 1.0) * p0) / k;
            p0 = p1;
            p1 = p2;
        }
        dp = n * (t * p1 - p0) / (t * t - 1.0);
        x[i] = t;
        w[i] = 2.0 / ((1.0 - t * t) * dp * dp);
    }
}

// Parameter block assembled on the host, uploaded once per call.
struct Params {
    std::vector<double> d;
    size_t add(const double *p, size_t count) {
        const size_t off = d.size();
        d.insert(d.end(), p, p + count);
        // keep 16-byte alignment for double2 reads
        if (d.size() & 1) d.push_back(0.0);
        return off;
    }
};

// Copies the parameter block to `dst` (device) through the handle's pinned staging buffer.
// With `noalloc` the staging buffer is not grown (it holds kStagingBytes from the handle's
// creation on), and a larger block is an argument error.
bem_status upload_to(bem_mesh *h, const Params &p, double *dst, bool noalloc, hipStream_t s) {
    const size_t bytes = p.d.size() * sizeof(double);
    if (noalloc && bytes > h->staging.bytes)
        return fail(BEM_EINVAL, "parameter block of " + std::to_string(bytes) + " bytes exceeds the " +
                                    std::to_string(h->staging.bytes) + "-byte staging buffer of an allocation-free call");
    HIP_TRY(h->staging.ensure(bytes), "staging buffer");
    std::memcpy(h->staging.host, p.d.data(), bytes);
    HIP_TRY(hipMemcpyAsync(dst, h->staging.host, bytes, hipMemcpyHostToDevice, s), "parameter upload");
    HIP_TRY(hipEventRecord(h->staging.done, s), "event record");
    h->staging.pending = true;
    return BEM_OK;
}

bem_status upload(bem_mesh *h, const Params &p, hipStream_t s) {
    HIP_TRY(h->params.ensure(p.d.size() * sizeof(double)), "parameter buffer");
    return upload_to(h, p, h->params.as<double>(), false, s);
}

// Device workspace of one sweep call: the parameter block, the self-term table and samples,
// the zero-padded probe copy, the folded diagonal, the generated products Z and the probe
// scale.  Every entry point takes it from the handle's buffers (grown on demand), except
// contour_moments_noalloc, which carves the same pieces out of the library's static scratch
// array.
struct Work {
    double *params = nullptr;
    double2 *self = nullptr, *aux = nullptr, *probe = nullptr, *fself = nullptr, *Z = nullptr;
    unsigned long long *vmax = nullptr;
};
struct Need {
    size_t params = 0, self = 0, aux = 0, probe = 0, fself = 0, Z = 0, vmax = 0;
};

bem_status acquire_handle(bem_mesh *h, const Need &n, Work &w) {
    HIP_TRY(h->params.ensure(n.params), "parameter buffer");
    HIP_TRY(h->self.ensure(n.self), "self-term table");
    HIP_TRY(h->aux.ensure(n.aux), "self-term samples");
    HIP_TRY(h->probe.ensure(n.probe), "probe copy");
    HIP_TRY(h->fself.ensure(n.fself), "folded self terms");
    HIP_TRY(h->Z.ensure(n.Z), "sweep workspace");
    HIP_TRY(h->vmax.ensure(n.vmax), "probe scale");
    w.params = h->params.as<double>();
    w.self = h->self.as<double2>();
    w.aux = h->aux.as<double2>();
    w.probe = h->probe.as<double2>();
    w.fself = h->fself.as<double2>();
    w.Z = h->Z.as<double2>();
    w.vmax = h->vmax.as<unsigned long long>();
    return BEM_OK;
}

// The pieces laid out one after another in the current device's scratch array, each at a
// 256-byte boundary; BEM_EINVAL when they do not fit (nothing is launched).
bem_status acquire_scratch(const Need &n, Work &w) {
    void *base = nullptr;
    size_t cap = 0;
    HIP_TRY(bemrat::scratch_region(&base, &cap), "scratch array address");
    size_t off = 0;
    auto take = [&](size_t bytes) -> void * {
        void *p = static_cast<unsigned char *>(base) + off;
        off += (bytes + 255) / 256 * 256;
        return p;
    };
    w.params = static_cast<double *>(take(n.params));
    w.self = static_cast<double2 *>(take(n.self));
    w.aux = static_cast<double2 *>(take(n.aux));
    w.probe = static_cast<double2 *>(take(n.probe));
    w.fself = static_cast<double2 *>(take(n.fself));
    w.Z = static_cast<double2 *>(take(n.Z));
    w.vmax = static_cast<unsigned long long *>(take(n.vmax));
    if (off > cap)
        return fail(BEM_EINVAL, "the call needs " + std::to_string(off) + " bytes of workspace; the allocation-free "
                                "entry point has " + std::to_string(cap));
    return BEM_OK;
}

bemrat::Prec prec_of(uint32_t flags) { return static_cast<bemrat::Prec>((flags & BEM_PREC_MASK) >> 4); }

// Truncation tolerance of the expansion forms: 1e-14 in FP64; below the unit roundoff of
// the contraction type otherwise (FP32 6e-8, FP16 4.9e-4, BF16 3.9e-3).
double trunc_tol(bemrat::Prec p) {
    switch (p) {
        case bemrat::Prec::F32: return 1e-9;
        case bemrat::Prec::F16: return 1e-6;
        case bemrat::Prec::BF16: return 1e-5;
        default: return 1e-14;
    }
}

// The generated operators of one sweep and how each node combines them.
struct Plan {
    bemrat::Gen gen = bemrat::Gen::Direct;
    int L = 0;
    cplx c = 0.0;             // Taylor: centre; Cheb: alpha (real)
    double R = 0.0;           // Taylor: radius; Cheb: beta
    int miller_M = 0;         // Cheb: start index of the Bessel recurrence
    bool unsupported = false; // the requested form does not apply to these nodes
    bemrat::Prec prec = bemrat::Prec::F64;
    std::vector<cplx> kappa;  // Direct: L wavenumbers
    std::vector<cplx> Cf;     // N x L: T(z_j) = sum_l Cf[j][l] T_l
};

// Expansion length: smallest L with x^L/L! / (1 - x/(L+1)) <= 1e-14 e^{-x h}, where
// h = max_j max(Im t_j, 0) over the scaled nodes t_j = (z_j - c)/R: the truncated Taylor
// series of exp(i R r t) is then accurate to 1e-14 relative to its smallest value at the
// nodes (|exp(i R r t)| = e^{-R r Im t}; h = 1 on a circle, 0 for real nodes).  L is rounded
// up to a whole number of sweep blocks (the extra terms cost nothing and add accuracy).
int taylor_length(double x, double h, int block, double tol) {
    const double target = tol * std::exp(-x * h);
    double term = 1.0;
    for (int L = 1; L < bemrat::kMaxTaylor; ++L) {
        term *= x / L;
        if (L > x && term / (1.0 - x / (L + 1)) <= target) {
            const int r = (L + block - 1) / block * block;
            return std::min(r, bemrat::kMaxTaylor - 1);
        }
    }
    return bemrat::kMaxTaylor;
}

// Chebyshev (Jacobi-Anger) length for real nodes: smallest L > x/2 with
// 2 (x/2)^L / L! / (1 - (x/2)^2 / (L + 1)) <= 1e-14, x = beta diam (a bound on
// sum_{l >= L} |eps_l J_l(x)|, and |T_l| <= 1 on the interval), rounded up to whole blocks.
// Also returns the unrounded length in *need (the Bessel recurrence starts 10 above it,
// which is accurate to a few units of 1e-16 for these x).
int cheb_length(double x, int block, int *need, double tol) {
    double term = 2.0;
    for (int L = 1; L < bemrat::kMaxTaylor; ++L) {
        term *= 0.5 * x / L;
        const double q = 0.25 * x * x / (L + 1);
        if (L > 0.5 * x && q < 1.0 && term / (1.0 - q) <= tol) {
            *need = L;
            const int r = (L + block - 1) / block * block;
            return std::min(r, bemrat::kMaxTaylor - 1);
        }
    }
    *need = bemrat::kMaxTaylor;
    return bemrat::kMaxTaylor;
}

Plan make_plan(const bem_mesh *h, const double *z, int64_t N, int64_t m, uint32_t flags) {
    Plan plan;
    std::vector<cplx> zs(N);
    for (int64_t j = 0; j < N; ++j) zs[j] = cplx(z[2 * j], z[2 * j + 1]);
    double rmin = 1e300, rmax = -1e300, imin = 1e300, imax = -1e300;
    for (auto &v : zs) {
        rmin = std::min(rmin, v.real());
        rmax = std::max(rmax, v.real());
        imin = std::min(imin, v.imag());
        imax = std::max(imax, v.imag());
    }
    const cplx c(0.5 * (rmin + rmax), 0.5 * (imin + imax));
    double R = 0.0;
    for (auto &v : zs) R = std::max(R, std::abs(v - c));
    const uint32_t form = flags & BEM_FORM_MASK;
    double hmax = 0.0;
    if (R > 0.0)
        for (auto &v : zs) hmax = std::max(hmax, (v - c).imag() / R);
    const bemrat::Prec prec = prec_of(flags);
    // expansion lengths are whole multiples of the sweep's length unit
    const int block = bemrat::sweep_ops_per_block(bemrat::Gen::Taylor, m);
    const int cblock = bemrat::sweep_ops_per_block(bemrat::Gen::Cheb, m);
    plan.prec = prec;
    const double tol = trunc_tol(prec);
    int L = R > 0.0 ? taylor_length(R * h->diameter, hmax, block, tol) : bemrat::kMaxTaylor;
    const bool expand_ok = R > 0.0 && L < bemrat::kMaxTaylor;
    // Chebyshev form: every node real (then c is real and R is the half-width)
    const bool real_nodes = imin == 0.0 && imax == 0.0;
    int need = 0;
    const int Lc = real_nodes && R > 0.0 ? cheb_length(R * h->diameter, cblock, &need, tol) : bemrat::kMaxTaylor;
    const bool cheb_ok = real_nodes && R > 0.0 && Lc + 10 < bemrat::kMaxTaylor;
    if (form == BEM_FORM_CHEB && !cheb_ok) {
        plan.unsupported = true;
        return plan;
    }
    // FP64: the Chebyshev form only on request (each block reruns the whole Bessel
    // recurrence, so it generates fewer operators than EXPAND but costs more at these sizes).
    // Reduced precision: AUTO takes it for real nodes (the recombination does not amplify
    // rounding errors) and DIRECT for complex ones; EXPAND only on request.
    const bool lp = prec != bemrat::Prec::F64;
    if (form == BEM_FORM_CHEB || (lp && form == BEM_FORM_AUTO && cheb_ok && Lc < N)) {
        plan.gen = bemrat::Gen::Cheb;
        plan.L = Lc;
        plan.c = c;
        plan.R = R;
        // a multiple of 8 (the recurrence runs 8 steps per trip) at least need + 10 (FP64
        // and FP32: Bessel values to a few units of 1e-16) or need (BF16 and FP16: to 2e-10,
        // against the 1e-5 / 1e-6 truncation) and at least the block's top index
        const bool lp16 = prec == bemrat::Prec::BF16 || prec == bemrat::Prec::F16;
        plan.miller_M = std::max((need + (lp16 ? 0 : 10) + 7) / 8 * 8, Lc);
        plan.Cf.resize((size_t)N * Lc);
        const cplx ipow[4] = {cplx(1, 0), cplx(0, 1), cplx(-1, 0), cplx(0, -1)};
        for (int64_t j = 0; j < N; ++j) {
            const double xi = std::max(-1.0, std::min(1.0, (zs[j].real() - c.real()) / R));
            double tp = 1.0, tc = xi;  // T_0, T_1
            for (int l = 0; l < Lc; ++l) {
                const double tl = l == 0 ? 1.0 : (l == 1 ? xi : 0.0);
                double T = tl;
                if (l >= 2) {
                    const double tn = 2.0 * xi * tc - tp;
                    tp = tc;
                    tc = tn;
                    T = tn;
                }
                plan.Cf[j * Lc + l] = (l == 0 ? 1.0 : 2.0) * ipow[l & 3] * T;
            }
        }
        return plan;
    }
    const bool expand = form == BEM_FORM_EXPAND ? expand_ok : (!lp && form == BEM_FORM_AUTO && expand_ok && L < N);
    if (!expand) {
        plan.gen = bemrat::Gen::Direct;
        plan.L = (int)N;
        plan.kappa = zs;
        plan.Cf.assign((size_t)N * N, 0.0);
        for (int64_t j = 0; j < N; ++j) plan.Cf[j * N + j] = 1.0;
        return plan;
    }
    plan.gen = bemrat::Gen::Taylor;
    plan.L = L;
    plan.c = c;
    plan.R = R;
    plan.Cf.resize((size_t)N * L);
    for (int64_t j = 0; j < N; ++j) {
        const cplx t = (zs[j] - c) / R;
        cplx p = 1.0;
        for (int l = 0; l < L; ++l) {
            plan.Cf[j * L + l] = p;
            p *= t;
        }
    }
    return plan;
}

// A direct plan on a node set made of quadruples {x + iy, x - iy, x' + iy, x' - iy}, y != 0 (a
// circle centred on the real axis with N a multiple of 4 and the half-step offset is one), is
// turned into Gen::DirectSym: the operators are reordered so that every quadruple is
// consecutive in that order (Cf becomes the matching permutation), and the sweep shares one
// exp(-y r) and its reciprocal between the four nodes and one sincos between each conjugate
// pair.  Members are matched to 4 units in the last place of the largest node; the kernel
// evaluates them at the first member's y and at their own real parts, which moves no entry by
// more than about 1e-14 relative.  The generated operators stay one per node.  Returns whether
// the plan was changed.
bool symmetrize(Plan &plan) {
    if (plan.gen != bemrat::Gen::Direct) return false;
    const int N = plan.L;
    if (N < 4 || N % 4 != 0 || N > 4096) return false;
    double zmax = 0.0;
    for (const cplx &k : plan.kappa) zmax = std::max(zmax, std::abs(k));
    const double tol = 4.0 * 2.220446049250313e-16 * zmax;
    std::vector<int> up, lo;
    for (int j = 0; j < N; ++j) {
        const double y = plan.kappa[j].imag();
        if (y > tol) up.push_back(j);
        else if (y < -tol) lo.push_back(j);
        else return false;
    }
    if (up.size() != lo.size() || up.size() % 2 != 0) return false;
    std::vector<int> conj(N, -1);
    std::vector<char> taken(N, 0);
    for (int u : up) {
        const cplx zu = plan.kappa[u];
        for (int l : lo) {
            const cplx zl = plan.kappa[l];
            if (!taken[l] && std::abs(zl.real() - zu.real()) <= tol && std::abs(zl.imag() + zu.imag()) <= tol) {
                conj[u] = l;
                taken[l] = 1;
                break;
            }
        }
        if (conj[u] < 0) return false;
    }
    std::stable_sort(up.begin(), up.end(),
                     [&](int a, int b) { return plan.kappa[a].imag() < plan.kappa[b].imag(); });
    std::vector<int> perm;
    perm.reserve(N);
    for (size_t i = 0; i < up.size(); i += 2) {
        const int a = up[i], b = up[i + 1];
        if (std::abs(plan.kappa[a].imag() - plan.kappa[b].imag()) > tol) return false;
        if (std::abs(plan.kappa[a].real() - plan.kappa[b].real()) <= tol) return false;
        perm.push_back(a);
        perm.push_back(conj[a]);
        perm.push_back(b);
        perm.push_back(conj[b]);
    }
    // every quadruple's real parts must be mirror images about one centre c (the generator
    // forms exp(i x' r) as exp(2icr) conj(exp(i x r))), to 4 units of rounding of |z| (a phase
    // error of at most 8 eps |z|_max r)
    const double c0 = 0.5 * (plan.kappa[perm[0]].real() + plan.kappa[perm[2]].real());
    for (int g = 0; g < N; g += 4) {
        const double mid = 0.5 * (plan.kappa[perm[g]].real() + plan.kappa[perm[g + 2]].real());
        if (std::abs(mid - c0) > tol) return false;
    }
    std::vector<cplx> kap(N);
    for (int l = 0; l < N; ++l) kap[l] = plan.kappa[perm[l]];
    plan.kappa = kap;
    plan.Cf.assign((size_t)N * N, 0.0);
    for (int l = 0; l < N; ++l) plan.Cf[(size_t)perm[l] * N + l] = 1.0;
    plan.gen = bemrat::Gen::DirectSym;
    plan.c = cplx(c0, 0.0);
    return true;
}

bool is_direct(bemrat::Gen g) { return g == bemrat::Gen::Direct || g == bemrat::Gen::DirectSym; }

// Host part of the self terms of the plan's operators: the wavenumbers the self-term kernel
// evaluates (the nodes for DIRECT; K sample points for the expansion forms, with the DFT
// weights that turn the samples into expansion coefficients).
void self_params(const Plan &plan, Params &prm, size_t &off_self_kappa, size_t &off_dft, int &K) {
    if (is_direct(plan.gen)) {
        std::vector<double> k(2 * plan.L);
        for (int l = 0; l < plan.L; ++l) {
            k[2 * l] = plan.kappa[l].real();
            k[2 * l + 1] = plan.kappa[l].imag();
        }
        off_self_kappa = prm.add(k.data(), k.size());
        K = 0;
        return;
    }
    if (plan.gen == bemrat::Gen::Cheb) {
        // Chebyshev coefficients of T_aa(alpha + beta xi) from K first-kind points (DCT-II),
        // divided by eps_l i^l (which the recombination applies):
        // S_l = (1 / (K i^l)) sum_k cos(pi l (k + 1/2) / K) T_aa(kappa_k)
        K = plan.L < 48 ? 64 : 128;
        const double pi = 3.14159265358979323846;
        const cplx ipow_inv[4] = {cplx(1, 0), cplx(0, -1), cplx(-1, 0), cplx(0, 1)};
        std::vector<double> k(2 * K), F(2 * (size_t)K * plan.L);
        for (int q = 0; q < K; ++q) {
            const double th = pi * (q + 0.5) / K;
            k[2 * q] = plan.c.real() + plan.R * std::cos(th);
            k[2 * q + 1] = 0.0;
            for (int l = 0; l < plan.L; ++l) {
                const cplx f = ipow_inv[l & 3] * (std::cos(th * l) / K);
                F[2 * ((size_t)q * plan.L + l)] = f.real();
                F[2 * ((size_t)q * plan.L + l) + 1] = f.imag();
            }
        }
        off_self_kappa = prm.add(k.data(), k.size());
        off_dft = prm.add(F.data(), F.size());
        return;
    }
    // Expansion: sample T_aa on K points of the circle |kappa - c| = R and take the
    // Taylor coefficients by the trapezoidal (DFT) rule: S_l = (1/K) sum_k T_aa(c + R e^{i phi_k}) e^{-i l phi_k}.
    K = plan.L < 64 ? 64 : 128;
    const double pi = 3.14159265358979323846;
    std::vector<double> k(2 * K), F(2 * (size_t)K * plan.L);
    for (int q = 0; q < K; ++q) {
        const double phi = 2.0 * pi * q / K;
        const cplx kap = plan.c + plan.R * std::polar(1.0, phi);
        k[2 * q] = kap.real();
        k[2 * q + 1] = kap.imag();
        for (int l = 0; l < plan.L; ++l) {
            const cplx f = std::polar(1.0 / K, -phi * l);
            F[2 * ((size_t)q * plan.L + l)] = f.real();
            F[2 * ((size_t)q * plan.L + l) + 1] = f.imag();
        }
    }
    off_self_kappa = prm.add(k.data(), k.size());
    off_dft = prm.add(F.data(), F.size());
}

// Self terms for the plan's operators into h->self (L x n_pad).
bem_status build_self(bem_mesh *h, const Plan &plan, Params &prm, size_t &off_self_kappa,
                      size_t &off_dft, int &K, hipStream_t) {
    const int64_t n_pad = h->dm.n_pad;
    HIP_TRY(h->self.ensure(sizeof(double2) * (size_t)plan.L * n_pad), "self-term table");
    self_params(plan, prm, off_self_kappa, off_dft, K);
    if (K > 0) HIP_TRY(h->aux.ensure(sizeof(double2) * (size_t)K * n_pad), "self-term samples");
    return BEM_OK;
}

// Launches the self-term kernels of a plan (parameters at pbase, see self_params): the
// L x n_pad table `self`, through the K x n_pad samples `aux` for the expansion forms.
hipError_t launch_self(const DeviceMesh &dm, const Plan &plan, const double *pbase, size_t off_self_kappa,
                       size_t off_dft, int K, double2 *aux, double2 *self, hipStream_t s) {
    const double2 *kap = reinterpret_cast<const double2 *>(pbase + off_self_kappa);
    if (is_direct(plan.gen)) return bemrat::launch_self_terms(dm, kap, plan.L, self, dm.n_pad, s);
    hipError_t e = bemrat::launch_self_terms(dm, kap, K, aux, dm.n_pad, s);
    if (e != hipSuccess) return e;
    return bemrat::launch_coef_dft(aux, dm.n_pad, K, reinterpret_cast<const double2 *>(pbase + off_dft), plan.L, self,
                                   s);
}

// Sweep arguments of a plan on one mesh (probe copy, output and precision fields are
// filled by the caller).
bemrat::SweepArgs sweep_args(const DeviceMesh &dm, const Plan &plan, const double *pbase, size_t off_self_kappa,
                             size_t off_tables, const double2 *self) {
    bemrat::SweepArgs a{};
    a.colloc = dm.colloc;
    a.quad = dm.quad;
    a.self = self;
    a.n = dm.n;
    a.n_pad = dm.n_pad;
    a.L = plan.L;
    a.kappa = reinterpret_cast<const double2 *>(pbase + off_self_kappa);
    a.c_re = plan.c.real();
    a.c_im = plan.c.imag();
    a.R = plan.R;
    a.decay = 0;
    if (plan.gen == bemrat::Gen::Taylor) a.decay = plan.c.imag() != 0.0;
    for (const cplx &k : plan.kappa) a.decay |= k.imag() != 0.0;
    a.inv_fact = pbase + off_tables;
    a.inv_int = pbase + off_tables + bemrat::kMaxTaylor;
    a.miller_M = plan.miller_M;
    return a;
}

// Workspace of a sweep of `plan` (self terms through K samples) on probe blocks of m columns;
// the parameter block, Z and the folded diagonal are added by the caller.
Need sweep_need(const bem_mesh *h, const Plan &plan, int K, int64_t m) {
    Need n;
    const size_t n_pad = (size_t)h->dm.n_pad;
    n.self = sizeof(double2) * (size_t)plan.L * n_pad;
    n.aux = sizeof(double2) * (size_t)K * n_pad;
    const int64_t m_pad = plan.prec == bemrat::Prec::F64 ? bemrat::sweep_m_pad(m) : bemrat::sweep_lp_m_pad(m);
    n.probe = sizeof(double2) * n_pad * (size_t)m_pad;
    n.vmax = plan.prec == bemrat::Prec::F64 ? 0 : sizeof(unsigned long long);
    return n;
}

// Runs self terms + sweep for `plan` on probe block V; Z receives L blocks (zstride, ldz).
// The parameter block is at w.params already.
bem_status run_sweep(bem_mesh *h, const Plan &plan, const Work &w, const double *V, int64_t m, int64_t ldv,
                     double2 *Z, int64_t ldz, int64_t zstride, size_t off_self_kappa, size_t off_dft, int K,
                     size_t off_tables, hipStream_t s) {
    const DeviceMesh &dm = h->dm;
    const double *pbase = w.params;
    HIP_TRY(launch_self(dm, plan, pbase, off_self_kappa, off_dft, K, w.aux, w.self, s), "self-term kernel");
    // zero-padded copy of the probe block read by the sweep
    const int64_t m_pad = plan.prec == bemrat::Prec::F64 ? bemrat::sweep_m_pad(m) : bemrat::sweep_lp_m_pad(m);
    double2 *Vp2 = w.probe;
    HIP_TRY(bemrat::launch_prep_probe(reinterpret_cast<const double2 *>(V), ldv, dm.n, m, dm.n_pad, m_pad, Vp2, s),
            "probe copy kernel");
    bemrat::SweepArgs a = sweep_args(dm, plan, pbase, off_self_kappa, off_tables, w.self);
    a.Vp2 = Vp2;
    a.m_pad = m_pad;
    a.V = reinterpret_cast<const double2 *>(V);
    a.ldv = ldv;
    a.Z = Z;
    a.ldz = ldz;
    a.zstride = zstride;
    a.m = m;
    if (h->timing) HIP_TRY(hipEventRecord(h->ev0, s), "event record");
    if (plan.prec == bemrat::Prec::F64) {
        HIP_TRY(bemrat::launch_sweep(plan.gen, a, s), "sweep kernel");
    } else {
        // entries ~ A_b w_q / (4 pi r): scaled to ~ w_q / r, well inside the FP16 range;
        // the probe block by 1 / max |V| (a device reduction into the workspace)
        a.a_scale = 4.0 * 3.14159265358979323846 / h->mean_area;
        HIP_TRY(bemrat::launch_absmax(a.V, ldv, dm.n, m, w.vmax, s), "probe scale kernel");
        a.vmax = w.vmax;
        HIP_TRY(bemrat::launch_sweep_lp(plan.prec, plan.gen, a, s), "reduced-precision sweep kernel");
        HIP_TRY(bemrat::launch_add_diag(w.self, dm.n_pad, a.V, ldv, Z, ldz, zstride, dm.n, m, plan.L, s),
                "diagonal kernel");
    }
    if (h->timing) {
        HIP_TRY(hipEventRecord(h->ev1, s), "event record");
        h->timed = true;
    }
    h->last_form = is_direct(plan.gen) ? BEM_FORM_DIRECT
                   : plan.gen == bemrat::Gen::Taylor ? BEM_FORM_EXPAND
                                                     : BEM_FORM_CHEB;
    h->last_ops = plan.L;
    return BEM_OK;
}

size_t add_tables(Params &prm) {
    std::vector<double> t(2 * bemrat::kMaxTaylor);
    double f = 1.0;
    for (int l = 0; l < bemrat::kMaxTaylor; ++l) {
        if (l > 0) f /= l;
        t[l] = f;                                            // 1/l!
        t[bemrat::kMaxTaylor + l] = l > 0 ? 1.0 / l : 0.0;  // 1/l
    }
    return prm.add(t.data(), t.size());
}

size_t add_complex(Params &prm, const std::vector<cplx> &v) {
    return prm.add(reinterpret_cast<const double *>(v.data()), 2 * v.size());
}

// Centroids ((P0 + P1) + P2)/3 and squared longest edges, each formed in exactly this order
// (no contraction into fused multiply-adds), so that the near-pair test below gives the same
// answer as any other evaluation written the same way.
bool near_geometry(const double *xyz, const int32_t *tri, int64_t n, std::vector<double> &cen,
                   std::vector<double> &h2) {
#pragma clang fp contract(off)
    try {
        cen.assign(3 * (size_t)n, 0.0);
        h2.assign((size_t)n, 0.0);
    } catch (...) {
        return false;
    }
    for (int64_t b = 0; b < n; ++b) {
        const double *P[3];
        for (int v = 0; v < 3; ++v) P[v] = xyz + 3 * (int64_t)tri[3 * b + v];
        for (int c = 0; c < 3; ++c) cen[3 * b + c] = ((P[0][c] + P[1][c]) + P[2][c]) / 3.0;
        double best = 0.0;
        for (int e = 0; e < 3; ++e) {
            const double *A = P[e], *B = P[(e + 1) % 3];
            const double dx = B[0] - A[0], dy = B[1] - A[1], dz = B[2] - A[2];
            const double l2 = dx * dx + dy * dy + dz * dz;
            if (l2 > best) best = l2;
        }
        h2[b] = best;
    }
    return true;
}

// Near pairs (a, b), a != b, with |x_a - x_b|^2 < (eta*eta) h_b^2, row a listing its b in
// increasing order.  A uniform grid of cells no smaller than eta max_b h_b only prunes the
// candidates; the test itself is the one above.
bool near_list(const std::vector<double> &cen, const std::vector<double> &h2, int64_t n, double eta,
               std::vector<int64_t> &rowptr, std::vector<int32_t> &col) {
#pragma clang fp contract(off)
    double hmax2 = 0.0, lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
    for (int64_t b = 0; b < n; ++b) {
        hmax2 = std::max(hmax2, h2[b]);
        for (int c = 0; c < 3; ++c) {
            lo[c] = std::min(lo[c], cen[3 * b + c]);
            hi[c] = std::max(hi[c], cen[3 * b + c]);
        }
    }
    double cs = eta * std::sqrt(hmax2) * (1.0 + 1e-9);
    int64_t dims[3];
    for (;;) {
        int64_t cells = 1;
        for (int c = 0; c < 3; ++c) {
            dims[c] = (int64_t)((hi[c] - lo[c]) / cs) + 1;
            cells *= dims[c];
        }
        if (cells <= 8 * n + 64) break;
        cs *= 1.5;  // coarser cells: fewer, each holding more candidates
    }
    auto cell_of = [&](int64_t b, int c) {
        const int64_t k = (int64_t)((cen[3 * b + c] - lo[c]) / cs);
        return std::min(std::max(k, (int64_t)0), dims[c] - 1);
    };
    const int64_t ncell = dims[0] * dims[1] * dims[2];
    try {
        std::vector<int64_t> start(ncell + 1, 0);
        std::vector<int32_t> items(n);
        std::vector<int64_t> cell(n);
        for (int64_t b = 0; b < n; ++b) {
            cell[b] = (cell_of(b, 2) * dims[1] + cell_of(b, 1)) * dims[0] + cell_of(b, 0);
            ++start[cell[b] + 1];
        }
        for (int64_t k = 0; k < ncell; ++k) start[k + 1] += start[k];
        std::vector<int64_t> fill(start.begin(), start.end() - 1);
        for (int64_t b = 0; b < n; ++b) items[fill[cell[b]]++] = (int32_t)b;
        const double eta2 = eta * eta;
        rowptr.assign(n + 1, 0);
        col.clear();
        std::vector<int32_t> cand;
        for (int64_t a = 0; a < n; ++a) {
            cand.clear();
            const int64_t ia[3] = {cell_of(a, 0), cell_of(a, 1), cell_of(a, 2)};
            for (int64_t z = std::max<int64_t>(ia[2] - 1, 0); z <= std::min(ia[2] + 1, dims[2] - 1); ++z)
                for (int64_t y = std::max<int64_t>(ia[1] - 1, 0); y <= std::min(ia[1] + 1, dims[1] - 1); ++y)
                    for (int64_t x = std::max<int64_t>(ia[0] - 1, 0); x <= std::min(ia[0] + 1, dims[0] - 1); ++x) {
                        const int64_t k = (z * dims[1] + y) * dims[0] + x;
                        for (int64_t it = start[k]; it < start[k + 1]; ++it) {
                            const int64_t b = items[it];
                            if (b == a) continue;
                            const double dx = cen[3 * a] - cen[3 * b], dy = cen[3 * a + 1] - cen[3 * b + 1],
                                         dz = cen[3 * a + 2] - cen[3 * b + 2];
                            const double d2 = dx * dx + dy * dy + dz * dz;
                            if (d2 < eta2 * h2[b]) cand.push_back((int32_t)b);
                        }
                    }
            std::sort(cand.begin(), cand.end());
            col.insert(col.end(), cand.begin(), cand.end());
            rowptr[a + 1] = (int64_t)col.size();
        }
    } catch (...) {
        return false;
    }
    return true;
}

bem_status sync_status(hipStream_t s) {
    hipError_t e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "stream synchronize");
    e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "device error");
    return BEM_OK;
}

}  // namespace

namespace {

// Nodes j with a nonzero weight W[j][p] for some p in [p0, p0 + P) (W is N x Pstride, host).
std::vector<int> active_nodes(const double *W, int64_t N, int64_t Pstride, int64_t p0, int64_t P) {
    std::vector<int> out;
    for (int64_t j = 0; j < N; ++j)
        for (int64_t p = p0; p < p0 + P; ++p)
            if (W[2 * (j * Pstride + p)] != 0.0 || W[2 * (j * Pstride + p) + 1] != 0.0) {
                out.push_back((int)j);
                break;
            }
    return out;
}

// Appends int32 values to the parameter block (packed into its doubles); returns the offset.
size_t add_ints(Params &prm, const std::vector<int> &v) {
    std::vector<double> d((v.size() + 1) / 2 + 1, 0.0);
    std::memcpy(d.data(), v.data(), sizeof(int) * v.size());
    return prm.add(d.data(), d.size());
}

// The weights' moments the series form folds with: mu[n][p] = sum_j W[j][p0 + p] (i z_j)^n,
// n < L, p < Pc (row-major L x Pc complex).
size_t add_series_moments(Params &prm, const double *z, int64_t N, const double *W, int64_t Pstride, int64_t p0,
                          int64_t Pc, int L) {
    std::vector<double> mu(2 * (size_t)L * Pc, 0.0);
    for (int64_t j = 0; j < N; ++j) {
        const double kr = -z[2 * j + 1], ki = z[2 * j];  // i z_j
        for (int64_t p = 0; p < Pc; ++p) {
            double tr = W[2 * (j * Pstride + p0 + p)], ti = W[2 * (j * Pstride + p0 + p) + 1];
            if (tr == 0.0 && ti == 0.0) continue;
            for (int n = 0; n < L; ++n) {
                mu[2 * (n * Pc + p)] += tr;
                mu[2 * (n * Pc + p) + 1] += ti;
                const double ur = tr * kr - ti * ki, ui = tr * ki + ti * kr;
                tr = ur;
                ti = ui;
            }
        }
    }
    return prm.add(mu.data(), mu.size());
}

// Near-field corrections of moments, M[p] += sum_j W[j][p] dT(z_j) V: by the quadrature
// (model NULL) or by the model's network inside its trust region and the quadrature outside.
// Each launch integrates only the nodes with a nonzero weight among its weight sets.
bem_status nearfield_moments_impl(bem_mesh *h, const bem_net_model *model, const double *z, int64_t N,
                                  const double *W, int64_t P, const double *V, int64_t m, int64_t ldv, double *M,
                                  int64_t ldm, int64_t *fallback_pairs, hipStream_t stream) {
    if (!h) return fail(BEM_EINVAL, "mesh is NULL");
    DeviceGuard guard(h->device);
    bem_status st = check_kappas(h, z, N, "z");
    if (st != BEM_OK) return st;
    if (N > (int64_t)1 << 20) return fail(BEM_EINVAL, "too many nodes");
    if (!W || P < 1 || P > (int64_t)1 << 20) return fail(BEM_EINVAL, "need W and 1 <= P <= 2^20");
    if (!finite_c(W, N * P)) return fail(BEM_EINVAL, "W has a non-finite value");
    if ((st = check_block(V, m, ldv, "V")) != BEM_OK) return st;
    if ((st = check_block(M, m, ldm, "M")) != BEM_OK) return st;
    if (model) {
        if (!model->params || !is_device_ptr(model->params))
            return fail(BEM_EINVAL, "model parameters are NULL or not device memory");
        for (int i = 0; i < BEM_NET_BINS; ++i)
            if (!(model->bin_edges[i] <= model->bin_edges[i + 1])) return fail(BEM_EINVAL, "bin edges must increase");
        if (!(model->freeze_tol >= 0.0) || !std::isfinite(model->freeze_tol))
            return fail(BEM_EINVAL, "freeze_tol must be finite and >= 0");
    }
    if (fallback_pairs) *fallback_pairs = 0;
    if (h->nf_pairs == 0) return BEM_OK;  // no near pairs: nothing to add
    Params prm;
    const size_t off_z = prm.add(z, 2 * (size_t)N);
    const size_t off_w = prm.add(W, 2 * (size_t)(N * P));
    double kmax = 0.0, kre_max = 0.0, kim_max = 0.0, kre_min = 1e300;
    for (int64_t j = 0; j < N; ++j) {
        const cplx k(z[2 * j], z[2 * j + 1]);
        kmax = std::max(kmax, std::abs(k));
        kre_max = std::max(kre_max, std::abs(k.real()));
        kim_max = std::max(kim_max, std::abs(k.imag()));
        kre_min = std::min(kre_min, k.real());
    }
    // node lists per launch: network chunks of kNetMaxP and quadrature chunks of kNfFold sets
    struct Chunk {
        int64_t p0, P;
        size_t off;
        int nn;
    };
    std::vector<Chunk> net_chunks, quad_chunks;
    auto plan_chunks = [&](int64_t width, std::vector<Chunk> &out) {
        for (int64_t p0 = 0; p0 < P; p0 += width) {
            const int64_t Pc = std::min<int64_t>(width, P - p0);
            const std::vector<int> nodes = active_nodes(W, N, P, p0, Pc);
            out.push_back({p0, Pc, add_ints(prm, nodes), (int)nodes.size()});
        }
    };
    // frozen wavenumber: the centre of the nodes' bounding box, the nodes' spread about it and
    // the sums of the weights of every set
    const bool frozen = model && model->freeze_tol > 0.0;
    cplx kc = 0.0;
    double h2max = 0.0;
    size_t off_ws = 0;
    if (frozen) {
        double rmin = 1e300, rmax = -1e300, imin = 1e300, imax = -1e300;
        for (int64_t j = 0; j < N; ++j) {
            rmin = std::min(rmin, z[2 * j]);
            rmax = std::max(rmax, z[2 * j]);
            imin = std::min(imin, z[2 * j + 1]);
            imax = std::max(imax, z[2 * j + 1]);
        }
        kc = cplx(0.5 * (rmin + rmax), 0.5 * (imin + imax));
        double spread = 0.0;
        for (int64_t j = 0; j < N; ++j) spread = std::max(spread, std::abs(cplx(z[2 * j], z[2 * j + 1]) - kc));
        h2max = spread > 0.0 && kmax > 0.0 ? model->freeze_tol / (spread * kmax) : 1e300;
        std::vector<double> ws(2 * (size_t)P, 0.0);
        for (int64_t p = 0; p < P; ++p)
            for (int64_t j = 0; j < N; ++j) {
                ws[2 * p] += W[2 * (j * P + p)];
                ws[2 * p + 1] += W[2 * (j * P + p) + 1];
            }
        off_ws = prm.add(ws.data(), ws.size());
    }
    if (model && !frozen) plan_chunks(bemrat::kNetMaxP, net_chunks);
    plan_chunks(bemrat::kNfFold, quad_chunks);
    const int64_t pairs = h->nf_pairs;
    // series form: one moments table per quadrature chunk
    const int L = h->nf_mode == BEM_NF_AUTO ? bemrat::nf_series_terms(kmax * h->nf_rmax) : 0;
    h->nf_last_terms = L;
    std::vector<size_t> mu_off;
    if (L)
        for (const Chunk &c : quad_chunks) mu_off.push_back(add_series_moments(prm, z, N, W, P, c.p0, c.P, L));
    if (L && !model)
        HIP_TRY(h->nf_F.ensure(sizeof(double2) * (size_t)pairs * std::min<int64_t>(P, bemrat::kNfFold)),
                "near-field folds");
    if (model) {
        HIP_TRY(h->net_frag.ensure((size_t)bemrat::net_frag_bytes()), "packed network");
        HIP_TRY(h->net_F.ensure(sizeof(double2) * (size_t)pairs * P), "pair folds");
        HIP_TRY(h->net_flag.ensure((size_t)pairs), "fallback flags");
    }
    if ((st = upload(h, prm, stream)) != BEM_OK) return st;
    const double *base = h->params.as<double>();
    const double2 *kap = reinterpret_cast<const double2 *>(base + off_z);
    const double2 *Wd = reinterpret_cast<const double2 *>(base + off_w);
    const int64_t *rowptr = h->nf_rowptr.as<int64_t>();
    const int32_t *col = h->nf_col.as<int32_t>();
    if (!model && L) {
        double2 *F = h->nf_F.as<double2>();
        for (size_t i = 0; i < quad_chunks.size(); ++i) {
            const Chunk &c = quad_chunks[i];
            if (c.nn == 0) continue;
            HIP_TRY(bemrat::launch_nearfield_series(h->dm, h->nf_gl.as<double>(), h->nf_row.as<int32_t>(), col, pairs,
                                                    nullptr, kmax, reinterpret_cast<const double2 *>(base + mu_off[i]),
                                                    L, (int)c.P, F, (int)c.P, 0, stream),
                    "near-field series kernel");
            HIP_TRY(bemrat::launch_pair_apply(h->dm, rowptr, col, F, (int)c.P, reinterpret_cast<const double2 *>(V), ldv,
                                              m, reinterpret_cast<double2 *>(M) + c.p0 * h->dm.n * ldm, ldm, stream),
                    "pair apply kernel");
        }
        return BEM_OK;
    }
    if (!model) {
        for (const Chunk &c : quad_chunks) {
            if (c.nn == 0) continue;
            HIP_TRY(bemrat::launch_nearfield(h->dm, h->nf_gl.as<double>(), rowptr, col, kap, (int)N, Wd, (int)P,
                                             (int)c.p0, (int)c.P, kmax, reinterpret_cast<const double2 *>(V), ldv, m,
                                             reinterpret_cast<double2 *>(M), ldm, nullptr, 0,
                                             reinterpret_cast<const int *>(base + c.off), c.nn, stream),
                    "near-field kernel");
        }
        return BEM_OK;
    }
    double2 *F = h->net_F.as<double2>();
    unsigned char *flag = h->net_flag.as<unsigned char>();
    HIP_TRY(bemrat::launch_net_pack(model->params, h->net_frag.ptr, stream), "network packing kernel");
    bemrat::NetFoldParams q{};
    q.mesh = &h->dm;
    q.rowptr = rowptr;
    q.col = col;
    q.npairs = pairs;
    q.kappa = kap;
    q.N = (int)N;
    q.W = Wd;
    q.Pstride = (int)P;
    q.frag = h->net_frag.ptr;
    q.params = model->params;
    q.S_re = model->out_scale[0];
    q.S_im = model->out_scale[1];
    q.dmin = model->dmin;
    q.tan_min = std::tan(model->min_angle_deg * 3.14159265358979323846 / 180.0);
    q.kh_re_max = model->kh_re_max;
    q.kh_im_max = model->kh_im_max;
    q.kre_max = kre_max;
    q.kim_max = kim_max;
    // wavenumbers with a negative real part lie outside the trained range: quadrature for all
    if (kre_min < 0.0) q.kh_re_max = -1.0;
    for (int i = 0; i <= BEM_NET_BINS; ++i) q.bin_edges[i] = model->bin_edges[i];
    for (int i = 0; i < BEM_NET_BINS; ++i) q.bin_ok[i] = model->bin_trusted[i] != 0;
    q.F = F;
    q.flag = flag;
    q.Wsum = nullptr;
    if (frozen) {
        // one launch for every weight set: one evaluation per pair at kc
        q.Wsum = reinterpret_cast<const double2 *>(base + off_ws);
        q.kc = make_double2(kc.real(), kc.imag());
        q.h2max = h2max;
        q.p0 = 0;
        q.P = (int)P;
        q.nodes = nullptr;
        q.nnodes = 0;
        HIP_TRY(bemrat::launch_net_fold(q, stream), "network fold kernel (frozen wavenumber)");
    }
    for (const Chunk &c : net_chunks) {
        q.p0 = (int)c.p0;
        q.P = (int)c.P;
        q.nodes = reinterpret_cast<const int *>(base + c.off);
        q.nnodes = c.nn;
        HIP_TRY(bemrat::launch_net_fold(q, stream), "network fold kernel");
    }
    // the pairs outside the trust region: the quadrature, folded into the same array
    for (size_t i = 0; L && i < quad_chunks.size(); ++i)
        HIP_TRY(bemrat::launch_nearfield_series(h->dm, h->nf_gl.as<double>(), h->nf_row.as<int32_t>(), col, pairs, flag,
                                                kmax, reinterpret_cast<const double2 *>(base + mu_off[i]), L,
                                                (int)quad_chunks[i].P, F, (int)P, (int)quad_chunks[i].p0, stream),
                "near-field series kernel");
    for (const Chunk &c : L ? std::vector<Chunk>() : quad_chunks)
        HIP_TRY(bemrat::launch_nearfield_fold(h->dm, h->nf_gl.as<double>(), rowptr, col, flag, kap, (int)N, Wd, (int)P,
                                              (int)c.p0, (int)c.P, kmax, F, reinterpret_cast<const int *>(base + c.off),
                                              c.nn, stream),
                "near-field fold kernel");
    HIP_TRY(bemrat::launch_pair_apply(h->dm, rowptr, col, F, (int)P, reinterpret_cast<const double2 *>(V), ldv, m,
                                      reinterpret_cast<double2 *>(M), ldm, stream),
            "pair apply kernel");
    if (fallback_pairs) {
        std::vector<unsigned char> fl((size_t)pairs);
        HIP_TRY(hipMemcpyAsync(fl.data(), flag, (size_t)pairs, hipMemcpyDeviceToHost, stream), "flag download");
        HIP_TRY(hipStreamSynchronize(stream), "stream synchronize");
        int64_t c = 0;
        for (unsigned char f : fl) c += f != 0;
        *fallback_pairs = c;
    }
    return BEM_OK;
}

}  // namespace

extern "C" {

const char *bem_last_error(void) { return g_error.c_str(); }

bem_status bem_stream_status(hipStream_t stream) { return sync_status(stream); }

bem_status bem_mesh_create(const double *xyz, int64_t nv, const int32_t *tri, int64_t n, hipStream_t stream,
                           bem_mesh_t *out) {
    if (!out) return fail(BEM_EINVAL, "out is NULL");
    *out = nullptr;
    if (!xyz || !tri) return fail(BEM_EINVAL, "xyz or tri is NULL");
    if (nv < 3 || n < 1) return fail(BEM_EINVAL, "need nv >= 3 and n >= 1");
    if (n > (int64_t)1 << 31) return fail(BEM_EINVAL, "too many triangles");
    for (int64_t i = 0; i < 3 * nv; ++i)
        if (!std::isfinite(xyz[i])) return fail(BEM_EINVAL, "non-finite vertex coordinate");
    for (int64_t i = 0; i < 3 * n; ++i)
        if (tri[i] < 0 || tri[i] >= nv) return fail(BEM_EMESH, "triangle vertex index out of range");
    double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
    for (int64_t i = 0; i < nv; ++i)
        for (int c = 0; c < 3; ++c) {
            lo[c] = std::min(lo[c], xyz[3 * i + c]);
            hi[c] = std::max(hi[c], xyz[3 * i + c]);
        }
    auto *h = new (std::nothrow) bem_mesh;
    if (!h) return fail(BEM_ENOMEM, "host allocation failed");
    if (hipGetDevice(&h->device) != hipSuccess) {
        delete h;
        return fail(BEM_EDEVICE, "no HIP device");
    }
    // twice the radius of a ball around the box centre holding every vertex: an upper
    // bound on the distance between any two points of the surface
    double rad2 = 0.0;
    for (int64_t i = 0; i < nv; ++i) {
        double d2 = 0.0;
        for (int c = 0; c < 3; ++c) {
            const double d = xyz[3 * i + c] - 0.5 * (lo[c] + hi[c]);
            d2 += d * d;
        }
        rad2 = std::max(rad2, d2);
    }
    h->diameter = 2.0 * std::sqrt(rad2) * (1.0 + 1e-12);
    double area_sum = 0.0;
    for (int64_t t = 0; t < n; ++t) {
        const double *P0 = xyz + 3 * (int64_t)tri[3 * t], *P1 = xyz + 3 * (int64_t)tri[3 * t + 1],
                     *P2 = xyz + 3 * (int64_t)tri[3 * t + 2];
        const double u[3] = {P1[0] - P0[0], P1[1] - P0[1], P1[2] - P0[2]};
        const double v[3] = {P2[0] - P0[0], P2[1] - P0[1], P2[2] - P0[2]};
        const double c[3] = {u[1] * v[2] - u[2] * v[1], u[2] * v[0] - u[0] * v[2], u[0] * v[1] - u[1] * v[0]};
        area_sum += 0.5 * std::sqrt(c[0] * c[0] + c[1] * c[1] + c[2] * c[2]);
    }
    h->mean_area = area_sum / (double)n;
    if (!near_geometry(xyz, tri, n, h->nf_cen, h->nf_h2)) {
        delete h;
        return fail(BEM_ENOMEM, "host allocation failed");
    }
    const int64_t n_pad = (n + bemrat::kPad - 1) / bemrat::kPad * bemrat::kPad;
    h->dm.n = n;
    h->dm.n_pad = n_pad;
    // geometry: colloc (n_pad double4) | quad (7 n_pad double4) | vtx (9 n_pad) | area (n_pad)
    const size_t geom_bytes = sizeof(double4) * 8 * (size_t)n_pad + sizeof(double) * 10 * (size_t)n_pad;
    bem_status st = BEM_OK;
    hipError_t e = h->geom.ensure(geom_bytes);
    double *staging = nullptr;
    std::vector<double> area_host(n);
    if (e == hipSuccess) e = h->gl.ensure(sizeof(double) * (2 * bemrat::kSelfGL + 28));
    if (e == hipSuccess) e = hipEventCreate(&h->ev0);
    if (e == hipSuccess) e = hipEventCreate(&h->ev1);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&h->staging.done, hipEventDisableTiming);
    // pinned staging of the per-call parameter block, sized once here so that the
    // allocation-free entry point never has to grow it
    if (e == hipSuccess) e = h->staging.ensure(kStagingBytes);
    if (e == hipSuccess) e = hipMalloc(&staging, sizeof(double) * 3 * nv + sizeof(int32_t) * 3 * n);
    if (e != hipSuccess) {
        st = hip_fail(e, "mesh allocation");
    } else {
        char *g = h->geom.as<char>();
        h->dm.colloc = reinterpret_cast<double4 *>(g);
        h->dm.quad = reinterpret_cast<double4 *>(g + sizeof(double4) * n_pad);
        h->dm.vtx = reinterpret_cast<double *>(g + sizeof(double4) * 8 * n_pad);
        h->dm.area = h->dm.vtx + 9 * n_pad;
        h->dm.gl = h->gl.as<double>();
        std::vector<double> glh(2 * bemrat::kSelfGL + 28);
        gauss_legendre(bemrat::kSelfGL, glh.data(), glh.data() + bemrat::kSelfGL);
        radon_rule(glh.data() + 2 * bemrat::kSelfGL);
        double *d_xyz = staging;
        int32_t *d_tri = reinterpret_cast<int32_t *>(staging + 3 * nv);
        e = hipMemcpy(d_xyz, xyz, sizeof(double) * 3 * nv, hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipMemcpy(d_tri, tri, sizeof(int32_t) * 3 * n, hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipMemcpy(h->dm.gl, glh.data(), sizeof(double) * glh.size(), hipMemcpyHostToDevice);
        if (e == hipSuccess)
            e = bemrat::launch_prepare_mesh(d_xyz, d_tri, n, n_pad, h->dm, h->dm.gl + 2 * bemrat::kSelfGL, stream);
        if (e == hipSuccess) e = hipStreamSynchronize(stream);
        if (e == hipSuccess) e = hipMemcpy(area_host.data(), h->dm.area, sizeof(double) * n, hipMemcpyDeviceToHost);
        if (e != hipSuccess) st = hip_fail(e, "mesh preparation");
        (void)hipFree(staging);
    }
    if (st == BEM_OK) {
        for (int64_t b = 0; b < n; ++b)
            if (!(area_host[b] > 0.0) || !std::isfinite(area_host[b])) {
                char msg[96];
                std::snprintf(msg, sizeof msg, "degenerate triangle %lld (zero area)", (long long)b);
                st = fail(BEM_EMESH, msg);
                break;
            }
    }
    if (st != BEM_OK) {
        bem_mesh_destroy(h);
        return st;
    }
    *out = h;
    return BEM_OK;
}

void bem_mesh_destroy(bem_mesh_t h) {
    if (!h) return;
    DeviceGuard guard(h->device);
    (void)hipDeviceSynchronize();
    h->geom.release();
    h->gl.release();
    h->self.release();
    h->aux.release();
    h->Z.release();
    h->params.release();
    h->partial.release();
    h->probe.release();
    h->vmax.release();
    h->fself.release();
    h->net_frag.release();
    h->net_F.release();
    h->net_flag.release();
    h->nf_rowptr.release();
    h->nf_col.release();
    h->nf_gl.release();
    h->nf_row.release();
    h->nf_F.release();
    if (h->staging.host) (void)hipHostFree(h->staging.host);
    if (h->staging.done) (void)hipEventDestroy(h->staging.done);
    if (h->ev0) (void)hipEventDestroy(h->ev0);
    if (h->ev1) (void)hipEventDestroy(h->ev1);
    delete h;
}

int64_t bem_mesh_size(bem_mesh_t h) { return h ? h->dm.n : -1; }

bem_status bem_mesh_geometry(bem_mesh_t h, double *area, double *centroid, double *quad_xyz, double *quad_w,
                             hipStream_t stream) {
    if (!h) return fail(BEM_EINVAL, "mesh is NULL");
    DeviceGuard guard(h->device);
    bem_status st = sync_status(stream);
    if (st != BEM_OK) return st;
    const int64_t n = h->dm.n;
    if (area) HIP_TRY(hipMemcpy(area, h->dm.area, sizeof(double) * n, hipMemcpyDeviceToHost), "copy");
    if (centroid || quad_xyz || quad_w) {
        std::vector<double4> c(n), q(7 * n);
        HIP_TRY(hipMemcpy(c.data(), h->dm.colloc, sizeof(double4) * n, hipMemcpyDeviceToHost), "copy");
        HIP_TRY(hipMemcpy(q.data(), h->dm.quad, sizeof(double4) * 7 * n, hipMemcpyDeviceToHost), "copy");
        const double fourpi = 4.0 * 3.14159265358979323846;
        for (int64_t b = 0; b < n; ++b) {
            if (centroid) {
                centroid[3 * b] = c[b].x;
                centroid[3 * b + 1] = c[b].y;
                centroid[3 * b + 2] = c[b].z;
            }
            for (int k = 0; k < 7; ++k) {
                const double4 p = q[7 * b + k];
                if (quad_xyz) {
                    quad_xyz[21 * b + 3 * k] = p.x;
                    quad_xyz[21 * b + 3 * k + 1] = p.y;
                    quad_xyz[21 * b + 3 * k + 2] = p.z;
                }
                if (quad_w) quad_w[7 * b + k] = p.w * fourpi;
            }
        }
    }
    return BEM_OK;
}

bem_status bem_contour_nodes(double c_re, double c_im, double radius, int64_t N, double shift_re,
                             double shift_im, int64_t P, double *z, double *w, double *W) {
    if (N < 1) return fail(BEM_EINVAL, "N must be positive");
    if (!(radius > 0.0) || !std::isfinite(radius)) return fail(BEM_EINVAL, "radius must be positive");
    if (!std::isfinite(c_re) || !std::isfinite(c_im) || !std::isfinite(shift_re) || !std::isfinite(shift_im))
        return fail(BEM_EINVAL, "non-finite centre or shift");
    if (P < 0) return fail(BEM_EINVAL, "P must be >= 0");
    if (!z || !w || (P > 0 && !W)) return fail(BEM_EINVAL, "output is NULL");
    const double pi = 3.14159265358979323846;
    const cplx c(c_re, c_im), sh(shift_re, shift_im);
    for (int64_t j = 0; j < N; ++j) {
        const cplx e = std::polar(1.0, 2.0 * pi * (j + 0.5) / N);
        const cplx zj = c + radius * e;
        const cplx wj = -radius * e / (double)N;
        z[2 * j] = zj.real();
        z[2 * j + 1] = zj.imag();
        w[2 * j] = wj.real();
        w[2 * j + 1] = wj.imag();
        if (P > 0) {
            const cplx d = zj - sh;
            if (d == cplx(0.0, 0.0)) return fail(BEM_EINVAL, "a node coincides with the shift");
            const cplx inv = 1.0 / d;
            cplx acc = wj;
            for (int64_t p = 0; p < P; ++p) {
                acc *= inv;
                W[2 * (j * P + p)] = acc.real();
                W[2 * (j * P + p) + 1] = acc.imag();
            }
        }
    }
    return BEM_OK;
}

bem_status bem_cheb_nodes(double a, double b, int64_t N, double *kappa, double *coef) {
    if (N < 1) return fail(BEM_EINVAL, "N must be positive");
    if (!std::isfinite(a) || !std::isfinite(b) || !(a < b)) return fail(BEM_EINVAL, "need finite a < b");
    if (!kappa) return fail(BEM_EINVAL, "kappa is NULL");
    const double pi = 3.14159265358979323846;
    const double alpha = 0.5 * (a + b), beta = 0.5 * (b - a);
    for (int64_t k = 0; k < N; ++k) kappa[k] = alpha + beta * std::cos(pi * (k + 0.5) / N);
    if (coef)
        for (int64_t l = 0; l < N; ++l)
            for (int64_t k = 0; k < N; ++k)
                coef[l * N + k] = (l == 0 ? 1.0 : 2.0) / N * std::cos(pi * l * (k + 0.5) / N);
    return BEM_OK;
}

bem_status bem_self_terms(bem_mesh_t h, const double *kappa, int64_t nk, double *S, hipStream_t stream) {
    if (!h) return fail(BEM_EINVAL, "mesh is NULL");
    DeviceGuard guard(h->device);
    bem_status st = check_kappas(h, kappa, nk, "kappa");
    if (st != BEM_OK) return st;
    if (!S || !is_device_ptr(S)) return fail(BEM_EINVAL, "S is not device memory");
    if (nk > 65535) return fail(BEM_EINVAL, "at most 65535 wavenumbers per call");
    Params prm;
    const size_t off = prm.add(kappa, 2 * nk);
    st = upload(h, prm, stream);
    if (st != BEM_OK) return st;
    // the kernel writes n_pad entries per wavenumber; stage through the workspace
    HIP_TRY(h->aux.ensure(sizeof(double2) * (size_t)nk * h->dm.n_pad), "self-term buffer");
    HIP_TRY(bemrat::launch_self_terms(h->dm, reinterpret_cast<const double2 *>(h->params.as<double>() + off), nk,
                                      h->aux.as<double2>(), h->dm.n_pad, stream),
            "self-term kernel");
    HIP_TRY(hipMemcpy2DAsync(S, sizeof(double2) * h->dm.n, h->aux.ptr, sizeof(double2) * h->dm.n_pad,
                             sizeof(double2) * h->dm.n, nk, hipMemcpyDeviceToDevice, stream),
            "copy");
    return BEM_OK;
}

bem_status bem_assemble_apply(bem_mesh_t h, const double *kappa, int64_t nk, const double *V, int64_t m,
                              int64_t ldv, double *Y, int64_t ldy, uint32_t flags, hipStream_t stream) {
    if (!h) return fail(BEM_EINVAL, "mesh is NULL");
    DeviceGuard guard(h->device);
    bem_status st = check_flags(flags);
    if (st != BEM_OK) return st;
    if ((flags & BEM_FORM_MASK) == BEM_FORM_EXPAND || (flags & BEM_FORM_MASK) == BEM_FORM_CHEB)
        return fail(BEM_EUNSUPPORTED, "bem_assemble_apply evaluates each wavenumber directly");
    if ((st = check_kappas(h, kappa, nk, "kappa")) != BEM_OK) return st;
    if (nk > 65535) return fail(BEM_EINVAL, "at most 65535 wavenumbers per call");
    if ((st = check_block(V, m, ldv, "V")) != BEM_OK) return st;
    if ((st = check_block(Y, m, ldy, "Y")) != BEM_OK) return st;
    Plan plan = make_plan(h, kappa, nk, m, BEM_FORM_DIRECT | (flags & BEM_PREC_MASK));
    Params prm;
    const size_t off_tables = add_tables(prm);
    size_t off_k = 0, off_dft = 0;
    int K = 0;
    self_params(plan, prm, off_k, off_dft, K);
    Need need = sweep_need(h, plan, K, m);
    need.params = prm.d.size() * sizeof(double);
    Work w;
    if ((st = acquire_handle(h, need, w)) != BEM_OK) return st;
    if ((st = upload_to(h, prm, w.params, false, stream)) != BEM_OK) return st;
    return run_sweep(h, plan, w, V, m, ldv, reinterpret_cast<double2 *>(Y), ldy, h->dm.n * ldy, off_k, off_dft, K,
                     off_tables, stream);
}


}  // extern "C"

namespace {

// Combination coefficients of the weight sets: coef[l][p] = sum_j Cf[j][l] W[j][p].
std::vector<cplx> combination(const Plan &plan, const double *W, int64_t N, int64_t P) {
    std::vector<cplx> coef((size_t)plan.L * P, 0.0);
    for (int64_t j = 0; j < N; ++j)
        for (int l = 0; l < plan.L; ++l) {
            const cplx cf = plan.Cf[j * plan.L + l];
            if (cf == cplx(0.0, 0.0)) continue;
            for (int64_t p = 0; p < P; ++p) coef[l * P + p] += cf * cplx(W[2 * (j * P + p)], W[2 * (j * P + p) + 1]);
        }
    return coef;
}

// Taylor plans: the number of operators the weight sets reach.  Operator l's entries are
// bounded by g_l = x^l / l! (x = R times the mesh diameter) times the weight, so weight set
// p's term l is at most |coef[l][p]| g_l; the operators up to the highest l whose term exceeds
// the truncation tolerance times the largest term of its set are reached (rounded up to the
// length unit).  Moment weights of a circle whose centre is the expansion centre reach one
// operator each (the trapezoidal rule integrates t^k exactly: moment p is the coefficient of
// t^(p-1), T_(p-1) / R^(p-1)); their other coefficients are rounding noise, about sqrt(N)
// units in the last place of the largest.  Other plans: L.
int taylor_reach(const Plan &plan, const std::vector<cplx> &coef, int64_t P, double diameter, int64_t m) {
    if (plan.gen != bemrat::Gen::Taylor || P < 1) return plan.L;
    const int L = plan.L;
    const double x = plan.R * diameter, tol = trunc_tol(plan.prec);
    std::vector<double> g(L, 1.0);
    for (int l = 1; l < L; ++l) g[l] = g[l - 1] * x / l;
    std::vector<double> big(P, 0.0);
    for (int l = 0; l < L; ++l)
        for (int64_t p = 0; p < P; ++p) big[p] = std::max(big[p], std::abs(coef[l * P + p]) * g[l]);
    int last = 0;
    for (int l = 0; l < L; ++l)
        for (int64_t p = 0; p < P; ++p)
            if (std::abs(coef[l * P + p]) * g[l] > tol * big[p]) last = l;
    const int unit = bemrat::sweep_ops_per_block(bemrat::Gen::Taylor, m);
    return std::min(L, (last + unit) / unit * unit);
}

// Cuts a Taylor plan (Cf and coef) to the operators its weight sets reach; returns whether it
// was shortened.
bool trim_taylor(Plan &plan, std::vector<cplx> &coef, int64_t P, double diameter, int64_t m) {
    const int L = plan.L, Lt = taylor_reach(plan, coef, P, diameter, m);
    if (Lt >= L) return false;
    const size_t N = plan.Cf.size() / L;
    std::vector<cplx> Cf(N * Lt);
    for (size_t j = 0; j < N; ++j)
        for (int l = 0; l < Lt; ++l) Cf[j * Lt + l] = plan.Cf[j * L + l];
    plan.Cf.swap(Cf);
    coef.resize((size_t)Lt * P);
    plan.L = Lt;
    return true;
}

// The folded generator's coefficients: coef[l][p] (P columns) in rows of the fold width
// KL = fold_width(P), zero from column P on; for Taylor plans times each operator's own
// factor i^l / l! (the generator folds the plain power sums).
std::vector<cplx> fold_coefficients(const Plan &plan, const std::vector<cplx> &coef, int P) {
    const int KL = bemrat::fold_width(P);
    std::vector<cplx> fc((size_t)plan.L * KL, 0.0);
    cplx f = 1.0;
    for (int l = 0; l < plan.L; ++l) {
        if (plan.gen == bemrat::Gen::Taylor && l > 0) f *= cplx(0.0, 1.0 / l);
        for (int p = 0; p < P; ++p) fc[(size_t)l * KL + p] = coef[(size_t)l * P + p] * f;
    }
    return fc;
}

// Whether contour_moments folds its P weight sets into the sweep: the folded sweep generates
// every operator of an entry and folds it KL = fold_width(P) times, the unfolded one generates
// the operators in blocks and contracts each.  Measured at n = 81920 (kernel times): with 32
// Taylor operators and m = 32 the unfolded sweep takes 1015 ms, the folded one 311, 406 and
// 613-623 ms for P = 1, 2 and 3-4; at m = 64 1551 against 387, 490 and 686-700 ms; in the
// direct form (64 nodes, m = 32) 3320 against 1946 (P = 2) and 2460 ms (P = 4).  A fold of
// width 8 took 1136-1144 ms at m = 32 and 3400 ms in the direct form, slower than the
// unfolded sweep: there the folding outweighs the saved contractions.
bool fold_pays(const Plan &plan, int64_t P) {
    if (P > bemrat::kFoldMax) return false;
    const int KL = bemrat::fold_width((int)P);
    return (int64_t)plan.L * KL <= bemrat::kFoldCoef;
}

// Folded moments (FP64, direct or expansion plans, P <= kFoldMax): the sweep generates every
// operator of each entry and contracts only the P combinations sum_l coef[l][p] T_l, written
// straight to M; the diagonal is the same combination of the self terms.  The parameter
// block is at w.params already.
bem_status folded_moments(bem_mesh *h, const Plan &plan, const Work &w, size_t off_k, size_t off_dft, int K,
                          size_t off_tables, size_t off_coef, size_t off_fcoef, int P, const double *V, int64_t m,
                          int64_t ldv, double *M, int64_t ldm, hipStream_t s) {
    const DeviceMesh &dm = h->dm;
    const double *pbase = w.params;
    const double2 *coef = reinterpret_cast<const double2 *>(pbase + off_coef);
    HIP_TRY(launch_self(dm, plan, pbase, off_k, off_dft, K, w.aux, w.self, s), "self-term kernel");
    // fself[p][a] = sum_l coef[l][p] self_l[a]: the recombination kernel with one column
    HIP_TRY(bemrat::launch_combine(w.self, dm.n_pad, 1, plan.L, coef, P, dm.n_pad, 1, w.fself, 1, s),
            "folded self-term kernel");
    const int64_t m_pad = bemrat::sweep_m_pad(m);
    double2 *Vp2 = w.probe;
    HIP_TRY(bemrat::launch_prep_probe(reinterpret_cast<const double2 *>(V), ldv, dm.n, m, dm.n_pad, m_pad, Vp2, s),
            "probe copy kernel");
    bemrat::SweepArgs a = sweep_args(dm, plan, pbase, off_k, off_tables, w.fself);
    a.L = P;
    a.Lgen = plan.L;
    a.fcoef = reinterpret_cast<const double2 *>(pbase + off_fcoef);
    a.Vp2 = Vp2;
    a.m_pad = m_pad;
    a.V = reinterpret_cast<const double2 *>(V);
    a.ldv = ldv;
    a.Z = reinterpret_cast<double2 *>(M);
    a.ldz = ldm;
    a.zstride = dm.n * ldm;
    a.m = m;
    if (h->timing) HIP_TRY(hipEventRecord(h->ev0, s), "event record");
    HIP_TRY(bemrat::launch_sweep_fold(plan.gen, a, s), "folded sweep kernel");
    if (h->timing) {
        HIP_TRY(hipEventRecord(h->ev1, s), "event record");
        h->timed = true;
    }
    h->last_form = is_direct(plan.gen) ? BEM_FORM_DIRECT : BEM_FORM_EXPAND;
    h->last_ops = plan.L;
    return BEM_OK;
}

// contour_moments with its workspace from the handle (noalloc = false) or from the static
// scratch array (noalloc = true: nothing is allocated, sizes beyond the array are rejected).
bem_status contour_moments_impl(bem_mesh_t h, const double *z, int64_t N, const double *W, int64_t P,
                                const double *V, int64_t m, int64_t ldv, double *M, int64_t ldm, uint32_t flags,
                                bool noalloc, hipStream_t stream) {
    if (!h) return fail(BEM_EINVAL, "mesh is NULL");
    DeviceGuard guard(h->device);
    bem_status st = check_flags(flags);
    if (st != BEM_OK) return st;
    if ((st = check_kappas(h, z, N, "z")) != BEM_OK) return st;
    if (!W || P < 1) return fail(BEM_EINVAL, "need W and P >= 1");
    if (!finite_c(W, N * P)) return fail(BEM_EINVAL, "W has a non-finite value");
    if ((st = check_block(V, m, ldv, "V")) != BEM_OK) return st;
    if ((st = check_block(M, m, ldm, "M")) != BEM_OK) return st;
    Plan plan = make_plan(h, z, N, m, flags);
    if (plan.unsupported) return fail(BEM_EUNSUPPORTED, "the Chebyshev form needs real nodes in a bounded interval");
    symmetrize(plan);
    std::vector<cplx> coef = combination(plan, W, N, P);
    trim_taylor(plan, coef, P, h->diameter, m);
    const bool fold = plan.prec == bemrat::Prec::F64 && plan.gen != bemrat::Gen::Cheb && fold_pays(plan, P);
    Params prm;
    const size_t off_tables = add_tables(prm);
    size_t off_k = 0, off_dft = 0;
    int K = 0;
    self_params(plan, prm, off_k, off_dft, K);
    const size_t off_coef = add_complex(prm, coef);
    const size_t off_fcoef = fold ? add_complex(prm, fold_coefficients(plan, coef, (int)P)) : off_coef;
    Need need = sweep_need(h, plan, K, m);
    need.params = prm.d.size() * sizeof(double);
    const size_t zstride = (size_t)h->dm.n * m;
    if (fold) need.fself = sizeof(double2) * (size_t)P * h->dm.n_pad;
    else need.Z = sizeof(double2) * zstride * plan.L;
    Work w;
    if ((st = noalloc ? acquire_scratch(need, w) : acquire_handle(h, need, w)) != BEM_OK) return st;
    if ((st = upload_to(h, prm, w.params, noalloc, stream)) != BEM_OK) return st;
    if (fold)
        return folded_moments(h, plan, w, off_k, off_dft, K, off_tables, off_coef, off_fcoef, (int)P, V, m, ldv, M,
                              ldm, stream);
    if ((st = run_sweep(h, plan, w, V, m, ldv, w.Z, m, zstride, off_k, off_dft, K, off_tables, stream)) != BEM_OK)
        return st;
    HIP_TRY(bemrat::launch_combine(w.Z, zstride, m, plan.L, reinterpret_cast<const double2 *>(w.params + off_coef),
                                   (int)P, h->dm.n, m, reinterpret_cast<double2 *>(M), ldm, stream),
            "combine kernel");
    return BEM_OK;
}

}  // namespace

extern "C" {

bem_status contour_moments(bem_mesh_t h, const double *z, int64_t N, const double *W, int64_t P, const double *V,
                           int64_t m, int64_t ldv, double *M, int64_t ldm, uint32_t flags, hipStream_t stream) {
    return contour_moments_impl(h, z, N, W, P, V, m, ldv, M, ldm, flags, false, stream);
}

bem_status contour_moments_noalloc(bem_mesh_t h, const double *z, int64_t N, const double *W, int64_t P,
                                   const double *V, int64_t m, int64_t ldv, double *M, int64_t ldm, uint32_t flags,
                                   hipStream_t stream) {
    return contour_moments_impl(h, z, N, W, P, V, m, ldv, M, ldm, flags, true, stream);
}

bem_status cheb_moments(bem_mesh_t h, double a, double b, int64_t N, int64_t L, const double *V, int64_t m,
                        int64_t ldv, double *C, int64_t ldc, uint32_t flags, hipStream_t stream) {
    if (!h) return fail(BEM_EINVAL, "mesh is NULL");
    DeviceGuard guard(h->device);
    bem_status st = check_flags(flags);
    if (st != BEM_OK) return st;
    if (N < 1 || L < 1 || L > N) return fail(BEM_EINVAL, "need 1 <= L <= N");
    if (!std::isfinite(a) || !std::isfinite(b) || !(a < b)) return fail(BEM_EINVAL, "need finite a < b");
    if ((st = check_block(V, m, ldv, "V")) != BEM_OK) return st;
    if ((st = check_block(C, m, ldc, "C")) != BEM_OK) return st;
    std::vector<double> kap(N), cf((size_t)N * N);
    bem_cheb_nodes(a, b, N, kap.data(), cf.data());
    std::vector<double> z(2 * N);
    for (int64_t k = 0; k < N; ++k) {
        z[2 * k] = kap[k];
        z[2 * k + 1] = 0.0;
    }
    Plan plan = make_plan(h, z.data(), N, m, flags);
    if (plan.unsupported) return fail(BEM_EUNSUPPORTED, "the Chebyshev form needs real nodes in a bounded interval");
    Params prm;
    const size_t off_tables = add_tables(prm);
    size_t off_k = 0, off_dft = 0;
    int K = 0;
    if ((st = build_self(h, plan, prm, off_k, off_dft, K, stream)) != BEM_OK) return st;
    // combine coefficients: C_l = sum_k cf[l][k] T(kappa_k) V = sum_j (sum_k cf[l][k] Cf[k][j]) Z_j
    std::vector<cplx> coef((size_t)plan.L * L, 0.0);
    for (int64_t k = 0; k < N; ++k)
        for (int j = 0; j < plan.L; ++j) {
            const cplx t = plan.Cf[k * plan.L + j];
            if (t == cplx(0.0, 0.0)) continue;
            for (int64_t l = 0; l < L; ++l) coef[j * L + l] += cf[l * N + k] * t;
        }
    const size_t off_coef = add_complex(prm, coef);
    const size_t zstride = (size_t)h->dm.n * m;
    Need need = sweep_need(h, plan, K, m);
    need.params = prm.d.size() * sizeof(double);
    need.Z = sizeof(double2) * zstride * plan.L;
    Work w;
    if ((st = acquire_handle(h, need, w)) != BEM_OK) return st;
    if ((st = upload_to(h, prm, w.params, false, stream)) != BEM_OK) return st;
    if ((st = run_sweep(h, plan, w, V, m, ldv, w.Z, m, zstride, off_k, off_dft, K, off_tables, stream)) != BEM_OK)
        return st;
    HIP_TRY(bemrat::launch_combine(w.Z, zstride, m, plan.L, reinterpret_cast<const double2 *>(w.params + off_coef),
                                   (int)L, h->dm.n, m, reinterpret_cast<double2 *>(C), ldc, stream),
            "combine kernel");
    return BEM_OK;
}

bem_status rr_project(bem_mesh_t h, const double *z, int64_t N, const double *U, int64_t m, int64_t ldu,
                      double *Pout, const double *W, int64_t Pw, double *M, int64_t ldm, uint32_t flags,
                      hipStream_t stream) {
    if (!h) return fail(BEM_EINVAL, "mesh is NULL");
    DeviceGuard guard(h->device);
    bem_status st = check_flags(flags);
    if (st != BEM_OK) return st;
    if ((st = check_kappas(h, z, N, "z")) != BEM_OK) return st;
    if ((st = check_block(U, m, ldu, "U")) != BEM_OK) return st;
    if (!Pout || !is_device_ptr(Pout)) return fail(BEM_EINVAL, "Pout is not device memory");
    if (Pw < 0) return fail(BEM_EINVAL, "Pw must be >= 0");
    if (Pw > 0) {
        if (!W) return fail(BEM_EINVAL, "W is NULL");
        if (!finite_c(W, N * Pw)) return fail(BEM_EINVAL, "W has a non-finite value");
        if ((st = check_block(M, m, ldm, "M")) != BEM_OK) return st;
    }
    Plan plan = make_plan(h, z, N, m, flags);
    if (plan.unsupported) return fail(BEM_EUNSUPPORTED, "the Chebyshev form needs real nodes in a bounded interval");
    symmetrize(plan);
    Params prm;
    const size_t off_tables = add_tables(prm);
    size_t off_k = 0, off_dft = 0;
    int K = 0;
    if ((st = build_self(h, plan, prm, off_k, off_dft, K, stream)) != BEM_OK) return st;
    const size_t off_cf = add_complex(prm, plan.Cf);  // N x L
    size_t off_coef = 0;
    if (Pw > 0) {
        // the projections need every operator; the moments combine those their weight sets
        // reach, as contour_moments does (the coefficients past them are zero)
        std::vector<cplx> coef = combination(plan, W, N, Pw);
        const int reach = taylor_reach(plan, coef, Pw, h->diameter, m);
        std::fill(coef.begin() + (size_t)reach * Pw, coef.end(), cplx(0.0, 0.0));
        off_coef = add_complex(prm, coef);
    }
    const int64_t n = h->dm.n;
    const size_t zstride = (size_t)n * m;
    const int64_t rows_per_chunk = 4096;
    const int nchunks = (int)((n + rows_per_chunk - 1) / rows_per_chunk);
    Need need = sweep_need(h, plan, K, m);
    need.params = prm.d.size() * sizeof(double);
    need.Z = sizeof(double2) * zstride * plan.L;
    Work w;
    if ((st = acquire_handle(h, need, w)) != BEM_OK) return st;
    HIP_TRY(h->partial.ensure(sizeof(double2) * (size_t)plan.L * nchunks * m * m), "projection workspace");
    if ((st = upload_to(h, prm, w.params, false, stream)) != BEM_OK) return st;
    double2 *Z = w.Z;
    if ((st = run_sweep(h, plan, w, U, m, ldu, Z, m, zstride, off_k, off_dft, K, off_tables, stream)) != BEM_OK)
        return st;
    const double *pbase = w.params;
    HIP_TRY(bemrat::launch_project_partial(reinterpret_cast<const double2 *>(U), ldu, Z, zstride, m, plan.L, n, m,
                                           rows_per_chunk, nchunks, h->partial.as<double2>(), stream),
            "projection kernel");
    HIP_TRY(bemrat::launch_project_finish(h->partial.as<double2>(), nchunks, plan.L, m,
                                          reinterpret_cast<const double2 *>(pbase + off_cf), (int)N,
                                          reinterpret_cast<double2 *>(Pout), stream),
            "projection reduction kernel");
    if (Pw > 0)
        HIP_TRY(bemrat::launch_combine(Z, zstride, m, plan.L, reinterpret_cast<const double2 *>(pbase + off_coef),
                                       (int)Pw, n, m, reinterpret_cast<double2 *>(M), ldm, stream),
                "combine kernel");
    return BEM_OK;
}

bem_status bem_assemble_sum(bem_mesh_t h, const double *z, int64_t N, const double *c, double *S, int64_t lds,
                            uint32_t flags, hipStream_t stream) {
    if (!h) return fail(BEM_EINVAL, "mesh is NULL");
    DeviceGuard guard(h->device);
    bem_status st = check_flags(flags);
    if (st != BEM_OK) return st;
    if (prec_of(flags) != bemrat::Prec::F64) return fail(BEM_EUNSUPPORTED, "dense assembly runs in FP64 only");
    if ((st = check_kappas(h, z, N, "z")) != BEM_OK) return st;
    if (!c) return fail(BEM_EINVAL, "c is NULL");
    if (!finite_c(c, N)) return fail(BEM_EINVAL, "c has a non-finite value");
    if ((st = check_block(S, h->dm.n, lds, "S")) != BEM_OK) return st;
    Plan plan = make_plan(h, z, N, 1, flags);
    if (plan.unsupported) return fail(BEM_EUNSUPPORTED, "the Chebyshev form needs real nodes in a bounded interval");
    Params prm;
    const size_t off_tables = add_tables(prm);
    size_t off_k = 0, off_dft = 0;
    int K = 0;
    if ((st = build_self(h, plan, prm, off_k, off_dft, K, stream)) != BEM_OK) return st;
    // d_l = sum_j c_j Cf[j][l]
    std::vector<cplx> d(plan.L, 0.0);
    for (int64_t j = 0; j < N; ++j)
        for (int l = 0; l < plan.L; ++l) d[l] += cplx(c[2 * j], c[2 * j + 1]) * plan.Cf[j * plan.L + l];
    const size_t off_d = add_complex(prm, d);
    if ((st = upload(h, prm, stream)) != BEM_OK) return st;
    const double *pbase = h->params.as<double>();
    HIP_TRY(launch_self(h->dm, plan, pbase, off_k, off_dft, K, h->aux.as<double2>(), h->self.as<double2>(), stream),
            "self-term kernel");
    bemrat::SweepArgs a = sweep_args(h->dm, plan, pbase, off_k, off_tables, h->self.as<double2>());
    if (h->timing) HIP_TRY(hipEventRecord(h->ev0, stream), "event record");
    HIP_TRY(bemrat::launch_assemble_sum(plan.gen, a, reinterpret_cast<const double2 *>(pbase + off_d),
                                        reinterpret_cast<double2 *>(S), lds, stream),
            "assembly kernel");
    if (h->timing) {
        HIP_TRY(hipEventRecord(h->ev1, stream), "event record");
        h->timed = true;
    }
    h->last_form = plan.gen == bemrat::Gen::Direct ? BEM_FORM_DIRECT
                   : plan.gen == bemrat::Gen::Taylor ? BEM_FORM_EXPAND
                                                     : BEM_FORM_CHEB;
    h->last_ops = plan.L;
    return BEM_OK;
}

bem_status bem_mesh_set_nearfield(bem_mesh_t h, double eta) {
    if (!h) return fail(BEM_EINVAL, "mesh is NULL");
    if (!std::isfinite(eta) || eta < 0.0 || eta > 16.0) return fail(BEM_EINVAL, "need 0 <= eta <= 16");
    DeviceGuard guard(h->device);
    h->nf_pairs = 0;
    h->nf_eta = 0.0;
    if (eta == 0.0) return BEM_OK;
    std::vector<int64_t> rowptr;
    std::vector<int32_t> col;
    if (!near_list(h->nf_cen, h->nf_h2, h->dm.n, eta, rowptr, col))
        return fail(BEM_ENOMEM, "host allocation failed (near-pair list)");
    const int64_t nnz = (int64_t)col.size();
    // the row of every pair, and a bound on the distance from a pair's target (centroid a) to
    // any point of triangle b: |x_a - x_b| plus the centroid-to-vertex distance of b, at most
    // two thirds of a median, itself at most the longest edge
    std::vector<int32_t> row;
    double rmax = 0.0;
    try {
        row.resize((size_t)nnz);
    } catch (...) {
        return fail(BEM_ENOMEM, "host allocation failed (near-pair rows)");
    }
    for (int64_t a = 0; a < h->dm.n; ++a)
        for (int64_t k = rowptr[a]; k < rowptr[a + 1]; ++k) {
            const int64_t b = col[k];
            row[k] = (int32_t)a;
            double d2 = 0.0;
            for (int c = 0; c < 3; ++c) {
                const double d = h->nf_cen[3 * a + c] - h->nf_cen[3 * b + c];
                d2 += d * d;
            }
            rmax = std::max(rmax, std::sqrt(d2) + (2.0 / 3.0) * std::sqrt(h->nf_h2[b]));
        }
    double glh[2 * 16 + 2 * 10];  // 16-point rule, then the 10-point rule (nodes, weights)
    gauss_legendre(16, glh, glh + 16);
    gauss_legendre(10, glh + 32, glh + 42);
    HIP_TRY(h->nf_rowptr.ensure(sizeof(int64_t) * rowptr.size()), "near-pair list");
    HIP_TRY(h->nf_col.ensure(sizeof(int32_t) * std::max<int64_t>(nnz, 1)), "near-pair list");
    HIP_TRY(h->nf_gl.ensure(sizeof glh), "near-field rule");
    HIP_TRY(h->nf_row.ensure(sizeof(int32_t) * std::max<int64_t>(nnz, 1)), "near-pair rows");
    // a set-up call: synchronous copies, the device may still run earlier work on any stream
    HIP_TRY(hipDeviceSynchronize(), "device synchronize");
    HIP_TRY(hipMemcpy(h->nf_rowptr.ptr, rowptr.data(), sizeof(int64_t) * rowptr.size(), hipMemcpyHostToDevice),
            "near-pair list upload");
    if (nnz)
        HIP_TRY(hipMemcpy(h->nf_col.ptr, col.data(), sizeof(int32_t) * nnz, hipMemcpyHostToDevice),
                "near-pair list upload");
    if (nnz)
        HIP_TRY(hipMemcpy(h->nf_row.ptr, row.data(), sizeof(int32_t) * nnz, hipMemcpyHostToDevice),
                "near-pair rows upload");
    HIP_TRY(hipMemcpy(h->nf_gl.ptr, glh, sizeof glh, hipMemcpyHostToDevice), "near-field rule upload");
    h->nf_pairs = nnz;
    h->nf_eta = eta;
    h->nf_rmax = rmax * (1.0 + 1e-12);
    return BEM_OK;
}

bem_status bem_mesh_nearfield(bem_mesh_t h, int64_t *pairs, int64_t *rowptr, int32_t *col) {
    if (!h) return fail(BEM_EINVAL, "mesh is NULL");
    if (!pairs) return fail(BEM_EINVAL, "pairs is NULL");
    DeviceGuard guard(h->device);
    *pairs = h->nf_pairs;
    if (h->nf_eta == 0.0) {
        if (rowptr)
            for (int64_t a = 0; a <= h->dm.n; ++a) rowptr[a] = 0;
        return BEM_OK;
    }
    if (rowptr)
        HIP_TRY(hipMemcpy(rowptr, h->nf_rowptr.ptr, sizeof(int64_t) * (h->dm.n + 1), hipMemcpyDeviceToHost),
                "near-pair list download");
    if (col && h->nf_pairs)
        HIP_TRY(hipMemcpy(col, h->nf_col.ptr, sizeof(int32_t) * h->nf_pairs, hipMemcpyDeviceToHost),
                "near-pair list download");
    return BEM_OK;
}

bem_status bem_mesh_set_nearfield_mode(bem_mesh_t h, int mode) {
    if (!h) return fail(BEM_EINVAL, "mesh is NULL");
    if (mode != BEM_NF_AUTO && mode != BEM_NF_NODES) return fail(BEM_EINVAL, "mode must be BEM_NF_AUTO or BEM_NF_NODES");
    h->nf_mode = mode;
    return BEM_OK;
}

bem_status bem_nearfield_last_terms(bem_mesh_t h, int *terms) {
    if (!h) return fail(BEM_EINVAL, "mesh is NULL");
    if (!terms) return fail(BEM_EINVAL, "terms is NULL");
    *terms = h->nf_last_terms;
    return BEM_OK;
}

bem_status bem_nearfield_moments(bem_mesh_t h, const double *z, int64_t N, const double *W, int64_t P,
                                 const double *V, int64_t m, int64_t ldv, double *M, int64_t ldm,
                                 hipStream_t stream) {
    return nearfield_moments_impl(h, nullptr, z, N, W, P, V, m, ldv, M, ldm, nullptr, stream);
}

bem_status bem_nearfield_sum(bem_mesh_t h, const double *z, int64_t N, const double *c, double *S, int64_t lds,
                             hipStream_t stream) {
    if (!h) return fail(BEM_EINVAL, "mesh is NULL");
    DeviceGuard guard(h->device);
    bem_status st = check_kappas(h, z, N, "z");
    if (st != BEM_OK) return st;
    if (N > (int64_t)1 << 20) return fail(BEM_EINVAL, "too many nodes");
    if (!c || !finite_c(c, N)) return fail(BEM_EINVAL, "c is NULL or has a non-finite value");
    if (!S || lds < h->dm.n) return fail(BEM_EINVAL, "need S and lds >= n");
    if (!is_device_ptr(S)) return fail(BEM_EINVAL, "S is not device memory");
    if (h->nf_pairs == 0) return BEM_OK;
    Params prm;
    const size_t off_z = prm.add(z, 2 * (size_t)N);
    const size_t off_c = prm.add(c, 2 * (size_t)N);
    double kmax = 0.0;
    for (int64_t j = 0; j < N; ++j) kmax = std::max(kmax, std::abs(cplx(z[2 * j], z[2 * j + 1])));
    const int L = h->nf_mode == BEM_NF_AUTO ? bemrat::nf_series_terms(kmax * h->nf_rmax) : 0;
    h->nf_last_terms = L;
    if (L) {
        const size_t off_mu = add_series_moments(prm, z, N, c, 1, 0, 1, L);
        HIP_TRY(h->nf_F.ensure(sizeof(double2) * (size_t)h->nf_pairs), "near-field folds");
        if ((st = upload(h, prm, stream)) != BEM_OK) return st;
        const double *base = h->params.as<double>();
        double2 *F = h->nf_F.as<double2>();
        HIP_TRY(bemrat::launch_nearfield_series(h->dm, h->nf_gl.as<double>(), h->nf_row.as<int32_t>(),
                                                h->nf_col.as<int32_t>(), h->nf_pairs, nullptr, kmax,
                                                reinterpret_cast<const double2 *>(base + off_mu), L, 1, F, 1, 0, stream),
                "near-field series kernel");
        HIP_TRY(bemrat::launch_pair_dense_add(h->nf_row.as<int32_t>(), h->nf_col.as<int32_t>(), F, h->nf_pairs,
                                              reinterpret_cast<double2 *>(S), lds, stream),
                "pair dense add kernel");
        return BEM_OK;
    }
    if ((st = upload(h, prm, stream)) != BEM_OK) return st;
    const double *base = h->params.as<double>();
    HIP_TRY(bemrat::launch_nearfield(h->dm, h->nf_gl.as<double>(), h->nf_rowptr.as<int64_t>(), h->nf_col.as<int32_t>(),
                                     reinterpret_cast<const double2 *>(base + off_z), (int)N,
                                     reinterpret_cast<const double2 *>(base + off_c), 1, 0, 1, kmax, nullptr, 0, 0,
                                     nullptr, 0, reinterpret_cast<double2 *>(S), lds, nullptr, 0, stream),
            "near-field kernel");
    return BEM_OK;
}

bem_status bem_last_form(bem_mesh_t h, uint32_t *form, int64_t *operators) {
    if (!h) return fail(BEM_EINVAL, "mesh is NULL");
    if (form) *form = h->last_form;
    if (operators) *operators = h->last_ops;
    return BEM_OK;
}

bem_status bem_set_timing(bem_mesh_t h, int on) {
    if (!h) return fail(BEM_EINVAL, "mesh is NULL");
    h->timing = on != 0;
    return BEM_OK;
}

bem_status bem_last_kernel_ms(bem_mesh_t h, float *ms) {
    if (!h || !ms) return fail(BEM_EINVAL, "mesh or ms is NULL");
    if (!h->timed) return fail(BEM_EINVAL, "no timed sweep yet");
    DeviceGuard guard(h->device);
    HIP_TRY(hipEventSynchronize(h->ev1), "event synchronize");
    HIP_TRY(hipEventElapsedTime(ms, h->ev0, h->ev1), "event elapsed time");
    return BEM_OK;
}

}  // extern "C"

// ------------------------------------------------------------------ batched form ---

struct bem_batch {
    int device = 0;
    int64_t count = 0, N = 0, P = 0, m = 0, m_pad = 0;
    int variant = 0;   // bemrat::BatchVariant shared by every mesh
    bemrat::Prec prec = bemrat::Prec::F64;
    int cb = 0;        // 16-column groups per tile
    int grid = 0;      // persistent blocks (one per compute unit)
    uint32_t form = 0; // BEM_FORM_DIRECT or BEM_FORM_EXPAND
    std::vector<bem_mesh *> meshes;
    std::vector<int64_t> rows;   // count + 1: first packed row of each mesh
    std::vector<int64_t> ops;    // generated operators per mesh
    std::vector<size_t> off_coef, off_probe, off_Z;
    int64_t nitems = 0;
    std::vector<size_t> off_self;
    // folded (FP64, at most kFoldBatchMax = 4 weight sets): each mesh's fold coefficients, folded diagonal,
    // and the P x P identity that copies its folds out of Z
    bool fold = false;
    std::vector<size_t> off_fcoef, off_fself;
    size_t off_eye = 0;
    Buffer params, self, probe, Z, table, items, counter, vmax, fself;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    bool timing = false, timed = false;
};

namespace {

// Operators one work item generates (FP64: 16 for the expansion form up to 32 columns, else 8;
// reduced precision: 16 for the direct form up to 64 columns, else 8).
int batch_ops_per_item(const bem_batch *b, int cb) {
    if (b->prec == bemrat::Prec::F64) {
        const bool taylor = b->variant == bemrat::kBatchTaylor || b->variant == bemrat::kBatchTaylorDecay;
        return bemrat::batch_ops_per_item_f64(taylor ? bemrat::Gen::Taylor : bemrat::Gen::Direct, cb);
    }
    const bool direct = b->variant == bemrat::kBatchDirect || b->variant == bemrat::kBatchDirectDecay ||
                        b->variant == bemrat::kBatchDirectSym;
    return bemrat::lp_batch_ops_per_block(direct ? bemrat::Gen::Direct : bemrat::Gen::Taylor, cb);
}

int batch_max_col_tile(const bem_batch *b) {
    return b->prec == bemrat::Prec::F64 ? bemrat::batch_col_tile(b->m) : bemrat::lp_batch_col_tile(b->m);
}

hipError_t batch_launch(const bem_batch *b, int cb, int nitems, hipStream_t s) {
    if (b->fold)
        return bemrat::launch_sweep_fold_batch(b->variant, cb, (int)b->P, b->table.as<bemrat::BatchEntry>(),
                                               b->items.as<int4>(), nitems, b->counter.as<unsigned>(), b->grid, s);
    if (b->prec == bemrat::Prec::F64)
        return bemrat::launch_sweep_batch(b->variant, cb, b->table.as<bemrat::BatchEntry>(), b->items.as<int4>(),
                                          nitems, b->counter.as<unsigned>(), b->grid, s);
    return bemrat::launch_sweep_lp_batch(b->prec, b->variant, cb, b->table.as<bemrat::BatchEntry>(),
                                         b->items.as<int4>(), nitems, b->counter.as<unsigned>(), b->grid, s);
}

// Work items (mesh, row block, column block, operator block) of a batch for a column tile of
// cb 16-column groups: meshes with the most source triangles first (their tiles run longest),
// and within a mesh the row block varies fastest, as in the per-call grid.
std::vector<int4> batch_items(const bem_batch *b, int cb) {
    std::vector<int64_t> order(b->count);
    for (int64_t i = 0; i < b->count; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](int64_t x, int64_t y) {
        return b->meshes[x]->dm.n_pad > b->meshes[y]->dm.n_pad;
    });
    const int64_t cblocks = (b->m + 16 * cb - 1) / (16 * cb);
    std::vector<int4> items;
    for (int64_t i : order) {
        const int64_t rblocks = b->meshes[i]->dm.n_pad / 16;
        const int ops = batch_ops_per_item(b, cb);
        const int64_t oblocks = b->fold ? 1 : (b->ops[i] + ops - 1) / ops;
        for (int64_t ob = 0; ob < oblocks; ++ob)
            for (int64_t c = 0; c < cblocks; ++c)
                for (int64_t r = 0; r < rblocks; ++r) items.push_back(make_int4((int)i, (int)r, (int)c, (int)ob));
    }
    return items;
}

bem_status batch_upload_items(bem_batch *b, const std::vector<int4> &items, hipStream_t s) {
    HIP_TRY(b->items.ensure(sizeof(int4) * std::max<size_t>(items.size(), 1)), "work items");
    HIP_TRY(hipMemcpyAsync(b->items.ptr, items.data(), sizeof(int4) * items.size(), hipMemcpyHostToDevice, s),
            "work item upload");
    HIP_TRY(hipStreamSynchronize(s), "work item upload");
    b->nitems = (int64_t)items.size();
    return BEM_OK;
}

// Tile autotuner: times the persistent sweep for every admissible column tile on an even
// sample of the batch's own work (whole (mesh, row block, operator block) groups, so every
// candidate does the same arithmetic), after one untimed pass, and keeps the fastest.
bem_status batch_tune(bem_batch *b, hipStream_t s) {
    const int max_cb = batch_max_col_tile(b);
    int best_cb = max_cb;
    float best = 0.0f;
    for (int cb = 1; cb <= max_cb; cb *= 2) {
        const std::vector<int4> all = batch_items(b, cb);
        const int64_t cblocks = (b->m + 16 * cb - 1) / (16 * cb);
        // items come in runs of rblocks per (mesh, operator block, column block); take every
        // stride-th row of the cb-independent (mesh, operator block, row block) groups
        const int64_t groups = (int64_t)all.size() / cblocks;
        const int64_t want = 4 * (int64_t)b->grid;
        const int64_t stride = std::max<int64_t>(1, groups / want);
        std::vector<int4> sample;
        for (const int4 &it : all) {
            const int64_t key = (int64_t)it.y + 1000003LL * ((int64_t)it.x * 64 + it.w);
            if (key % stride == 0) sample.push_back(it);
        }
        bem_status st = batch_upload_items(b, sample, s);
        if (st != BEM_OK) return st;
        float ms = 0.0f;
        for (int rep = 0; rep < 2; ++rep) {
            HIP_TRY(hipEventRecord(b->ev0, s), "event record");
            HIP_TRY(batch_launch(b, cb, (int)b->nitems, s), "batched sweep kernel");
            HIP_TRY(hipEventRecord(b->ev1, s), "event record");
            HIP_TRY(hipEventSynchronize(b->ev1), "event synchronize");
            HIP_TRY(hipEventElapsedTime(&ms, b->ev0, b->ev1), "event elapsed time");
        }
        if (cb == 1 || ms < best) {
            best = ms;
            best_cb = cb;
        }
    }
    b->cb = best_cb;
    return BEM_OK;
}

}  // namespace

extern "C" {

void bem_batch_destroy(bem_batch_t b) {
    if (!b) return;
    DeviceGuard guard(b->device);
    (void)hipDeviceSynchronize();
    b->params.release();
    b->self.release();
    b->probe.release();
    b->Z.release();
    b->table.release();
    b->items.release();
    b->counter.release();
    b->vmax.release();
    b->fself.release();
    if (b->ev0) (void)hipEventDestroy(b->ev0);
    if (b->ev1) (void)hipEventDestroy(b->ev1);
    delete b;
}

bem_status bem_batch_create(const bem_mesh_t *meshes, int64_t count, const double *z, int64_t N, const double *W,
                            int64_t P, int64_t m, uint32_t flags, int tune, hipStream_t stream, bem_batch_t *out) {
    if (!out) return fail(BEM_EINVAL, "out is NULL");
    *out = nullptr;
    if (!meshes || count < 1) return fail(BEM_EINVAL, "need count >= 1 meshes");
    if (count > (1 << 20)) return fail(BEM_EINVAL, "too many meshes");
    bem_status st = check_flags(flags);
    if (st != BEM_OK) return st;
    const uint32_t form = flags & BEM_FORM_MASK;
    const bemrat::Prec prec = prec_of(flags);
    const bool lp = prec != bemrat::Prec::F64;
    if (form == BEM_FORM_CHEB) return fail(BEM_EUNSUPPORTED, "the batched form takes the DIRECT or EXPAND form");
    if (!z || N < 1) return fail(BEM_EINVAL, "need z and N >= 1");
    if (!W || P < 1) return fail(BEM_EINVAL, "need W and P >= 1");
    if (m < 1) return fail(BEM_EINVAL, "m must be positive");
    if (!finite_c(W, count * N * P)) return fail(BEM_EINVAL, "W has a non-finite value");
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev), "current device");
    for (int64_t i = 0; i < count; ++i) {
        if (!meshes[i]) return fail(BEM_EINVAL, "a mesh is NULL");
        if (meshes[i]->device != dev) return fail(BEM_EINVAL, "every mesh must live on the current device");
        if ((st = check_kappas(meshes[i], z + 2 * i * N, N, "z")) != BEM_OK) return st;
    }
    // one operator family for the launch: EXPAND for every mesh when every mesh admits it
    // (and, for AUTO in FP64, when it generates fewer operator entries than DIRECT), else
    // DIRECT; at reduced precision AUTO means DIRECT (the expansion's recombination amplifies
    // rounding errors)
    const uint32_t pbits = flags & BEM_PREC_MASK;
    std::vector<Plan> plans(count);
    bool all_expand = form == BEM_FORM_EXPAND || (form == BEM_FORM_AUTO && !lp);
    double cost_e = 0.0, cost_d = 0.0;
    for (int64_t i = 0; i < count && all_expand; ++i) {
        plans[i] = make_plan(meshes[i], z + 2 * i * N, N, m, BEM_FORM_EXPAND | pbits);
        const double n = (double)meshes[i]->dm.n;
        all_expand = plans[i].gen == bemrat::Gen::Taylor;
        cost_e += plans[i].L * n * n;
        cost_d += (double)N * n * n;
    }
    if (form == BEM_FORM_AUTO && all_expand && !(cost_e < cost_d)) all_expand = false;
    bool sym = false;
    if (!all_expand) {
        // the direct form shares transcendentals over node quadruples when every mesh's node
        // set is made of them (one family for the launch), as the per-mesh calls do
        sym = true;
        for (int64_t i = 0; i < count; ++i) {
            plans[i] = make_plan(meshes[i], z + 2 * i * N, N, m, BEM_FORM_DIRECT | pbits);
            sym = sym && symmetrize(plans[i]);
        }
        if (!sym)
            for (int64_t i = 0; i < count; ++i) plans[i] = make_plan(meshes[i], z + 2 * i * N, N, m, BEM_FORM_DIRECT | pbits);
    }
    // Taylor plans stop at the last operator the mesh's weight sets reach, as contour_moments'
    for (int64_t i = 0; i < count; ++i) {
        std::vector<cplx> coef = combination(plans[i], W + 2 * i * N * P, N, P);
        trim_taylor(plans[i], coef, P, meshes[i]->diameter, m);
    }
    bool decay = false;
    for (const Plan &p : plans) {
        if (p.gen == bemrat::Gen::Taylor) decay |= p.c.imag() != 0.0;
        for (const cplx &k : p.kappa) decay |= k.imag() != 0.0;
    }

    auto *b = new (std::nothrow) bem_batch;
    if (!b) return fail(BEM_ENOMEM, "host allocation failed");
    b->device = dev;
    b->count = count;
    b->N = N;
    b->P = P;
    b->m = m;
    b->form = all_expand ? BEM_FORM_EXPAND : BEM_FORM_DIRECT;
    b->variant = bemrat::batch_variant(all_expand ? bemrat::Gen::Taylor
                                       : sym      ? bemrat::Gen::DirectSym
                                                  : bemrat::Gen::Direct,
                                       decay);
    b->prec = prec;
    b->meshes.assign(meshes, meshes + count);
    // FP64 with up to four weight sets folds them into the sweep, as contour_moments does
    b->fold = !lp && P <= bemrat::kFoldBatchMax;
    for (const Plan &p : plans)
        b->fold = b->fold && (int64_t)p.L * bemrat::fold_width((int)P) <= bemrat::kFoldCoef;
    const int max_cb = batch_max_col_tile(b);
    b->cb = max_cb;
    b->m_pad = (m + 16 * max_cb - 1) / (16 * max_cb) * (16 * max_cb);
    int cus = 0;
    hipError_t e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    b->grid = e == hipSuccess && cus > 0 ? cus : 256;

    // parameters: tables, then per mesh the self-term wavenumbers and combine coefficients
    Params prm;
    const size_t off_tables = add_tables(prm);
    std::vector<size_t> off_k(count), off_dft(count);
    std::vector<size_t> &off_self = b->off_self;
    off_self.resize(count);
    std::vector<int> K(count);
    b->rows.assign(count + 1, 0);
    b->ops.resize(count);
    b->off_coef.resize(count);
    b->off_probe.resize(count);
    b->off_Z.resize(count);
    b->off_fcoef.assign(count, 0);
    b->off_fself.assign(count, 0);
    size_t self_total = 0, probe_total = 0, z_total = 0, aux_need = 0, fself_total = 0;
    for (int64_t i = 0; i < count; ++i) {
        const Plan &plan = plans[i];
        const DeviceMesh &dm = meshes[i]->dm;
        self_params(plan, prm, off_k[i], off_dft[i], K[i]);
        const std::vector<cplx> coef = combination(plan, W + 2 * i * N * P, N, P);
        b->off_coef[i] = add_complex(prm, coef);
        if (b->fold) {
            b->off_fcoef[i] = add_complex(prm, fold_coefficients(plan, coef, (int)P));
            b->off_fself[i] = fself_total;
            fself_total += (size_t)P * dm.n_pad;
        }
        b->ops[i] = plan.L;
        b->rows[i + 1] = b->rows[i] + dm.n;
        off_self[i] = self_total;
        self_total += (size_t)plan.L * dm.n_pad;
        b->off_probe[i] = probe_total;
        probe_total += (size_t)dm.n_pad * b->m_pad;
        b->off_Z[i] = z_total;
        z_total += (size_t)(b->fold ? P : plan.L) * dm.n * m;
        aux_need = std::max(aux_need, (size_t)K[i] * dm.n_pad);
    }
    if (b->fold) {
        std::vector<cplx> eye((size_t)P * P, 0.0);
        for (int64_t p = 0; p < P; ++p) eye[p * P + p] = 1.0;
        b->off_eye = add_complex(prm, eye);
    }
    Buffer aux;
    st = BEM_OK;
    auto step = [&](hipError_t err, const char *what) {
        if (st == BEM_OK && err != hipSuccess) st = hip_fail(err, what);
        return st == BEM_OK;
    };
    const size_t pbytes = prm.d.size() * sizeof(double);
    if (step(b->params.ensure(pbytes), "batch parameters") &&
        step(hipMemcpy(b->params.ptr, prm.d.data(), pbytes, hipMemcpyHostToDevice), "parameter upload") &&
        step(b->self.ensure(sizeof(double2) * self_total), "batch self terms") &&
        step(b->probe.ensure(sizeof(double2) * probe_total), "batch probe copy") &&
        step(b->Z.ensure(sizeof(double2) * z_total), "batch sweep workspace") &&
        step(b->table.ensure(sizeof(bemrat::BatchEntry) * count), "batch table") &&
        step(b->counter.ensure(sizeof(unsigned)), "work counter") &&
        step(b->vmax.ensure(sizeof(unsigned long long) * count), "probe scales") &&
        step(b->fself.ensure(sizeof(double2) * std::max<size_t>(fself_total, 1)), "folded self terms") &&
        step(aux.ensure(sizeof(double2) * std::max<size_t>(aux_need, 1)), "self-term samples") &&
        step(hipEventCreate(&b->ev0), "event") && step(hipEventCreate(&b->ev1), "event")) {
        const double *pbase = b->params.as<double>();
        std::vector<bemrat::BatchEntry> table(count);
        for (int64_t i = 0; i < count && st == BEM_OK; ++i) {
            const DeviceMesh &dm = meshes[i]->dm;
            double2 *self = b->self.as<double2>() + off_self[i];
            if (!step(launch_self(dm, plans[i], pbase, off_k[i], off_dft[i], K[i], aux.as<double2>(), self, stream),
                      "self-term kernel"))
                break;
            double2 *fself = b->fself.as<double2>() + b->off_fself[i];
            // folded: the diagonal is the same fold of the self terms (fself[p] = sum_l coef[l][p] self_l)
            if (b->fold &&
                !step(bemrat::launch_combine(self, dm.n_pad, 1, plans[i].L,
                                             reinterpret_cast<const double2 *>(pbase + b->off_coef[i]), (int)P,
                                             dm.n_pad, 1, fself, 1, stream),
                      "folded self-term kernel"))
                break;
            bemrat::SweepArgs a = sweep_args(dm, plans[i], pbase, off_k[i], off_tables, b->fold ? fself : self);
            if (b->fold) {
                a.L = (int)P;
                a.Lgen = plans[i].L;
                a.fcoef = reinterpret_cast<const double2 *>(pbase + b->off_fcoef[i]);
            }
            a.Vp2 = b->probe.as<double2>() + b->off_probe[i];
            a.m_pad = b->m_pad;
            a.Z = b->Z.as<double2>() + b->off_Z[i];
            a.ldz = m;
            a.zstride = dm.n * m;
            a.m = m;
            // reduced precision: entries ~ A_b w_q / (4 pi r) scaled to ~ w_q / r; the probe
            // block by 1 / max |V_i| (reduced per call into the mesh's slot)
            a.a_scale = 4.0 * 3.14159265358979323846 / meshes[i]->mean_area;
            a.vmax = b->vmax.as<unsigned long long>() + i;
            table[i].args = a;
            table[i].variant = b->variant;
        }
        if (st == BEM_OK &&
            step(hipMemcpyAsync(b->table.ptr, table.data(), sizeof(bemrat::BatchEntry) * count, hipMemcpyHostToDevice,
                                stream),
                 "batch table upload") &&
            step(hipStreamSynchronize(stream), "batch set-up")) {
            if (tune) {
                // the sample runs read the probe copy and the probe scales: give them defined
                // contents (zeros; a zero scale reads as 1)
                if (step(hipMemsetAsync(b->probe.ptr, 0, sizeof(double2) * probe_total, stream), "probe clear") &&
                    step(hipMemsetAsync(b->vmax.ptr, 0, sizeof(unsigned long long) * count, stream), "scale clear"))
                    st = batch_tune(b, stream);
            }
            if (st == BEM_OK) st = batch_upload_items(b, batch_items(b, b->cb), stream);
        }
    }
    (void)hipStreamSynchronize(stream);
    aux.release();
    if (st != BEM_OK) {
        bem_batch_destroy(b);
        return st;
    }
    if (b->nitems > INT32_MAX) {
        bem_batch_destroy(b);
        return fail(BEM_EINVAL, "too many work items");
    }
    *out = b;
    return BEM_OK;
}

bem_status bem_batch_layout(bem_batch_t b, int64_t *rows, int64_t *operators, uint32_t *form, int *col_tile) {
    if (!b) return fail(BEM_EINVAL, "batch is NULL");
    if (rows) std::copy(b->rows.begin(), b->rows.end(), rows);
    if (operators) std::copy(b->ops.begin(), b->ops.end(), operators);
    if (form) *form = b->form;
    if (col_tile) *col_tile = 16 * b->cb;
    return BEM_OK;
}

bem_status bem_batch_moments(bem_batch_t b, const double *V, double *M, hipStream_t stream) {
    if (!b) return fail(BEM_EINVAL, "batch is NULL");
    DeviceGuard guard(b->device);
    if (!V || !is_device_ptr(V)) return fail(BEM_EINVAL, "V is not device memory");
    if (!M || !is_device_ptr(M)) return fail(BEM_EINVAL, "M is not device memory");
    const int64_t m = b->m;
    const bool lp = b->prec != bemrat::Prec::F64;
    const double2 *V2 = reinterpret_cast<const double2 *>(V);
    for (int64_t i = 0; i < b->count; ++i) {
        const DeviceMesh &dm = b->meshes[i]->dm;
        HIP_TRY(bemrat::launch_prep_probe(V2 + b->rows[i] * m, m, dm.n, m, dm.n_pad, b->m_pad,
                                          b->probe.as<double2>() + b->off_probe[i], stream),
                "probe copy kernel");
        if (lp)
            HIP_TRY(bemrat::launch_absmax(V2 + b->rows[i] * m, m, dm.n, m, b->vmax.as<unsigned long long>() + i, stream),
                    "probe scale kernel");
    }
    if (b->timing) HIP_TRY(hipEventRecord(b->ev0, stream), "event record");
    HIP_TRY(batch_launch(b, b->cb, (int)b->nitems, stream), "batched sweep kernel");
    if (b->timing) {
        HIP_TRY(hipEventRecord(b->ev1, stream), "event record");
        b->timed = true;
    }
    const double *pbase = b->params.as<double>();
    for (int64_t i = 0; i < b->count; ++i) {
        const int64_t n = b->meshes[i]->dm.n;
        if (lp)
            HIP_TRY(bemrat::launch_add_diag(b->self.as<double2>() + b->off_self[i], b->meshes[i]->dm.n_pad,
                                            V2 + b->rows[i] * m, m, b->Z.as<double2>() + b->off_Z[i], m, n * m, n, m,
                                            (int)b->ops[i], stream),
                    "diagonal kernel");
        // the moments from Z: the recombination of the operators, or (folded) a copy of the folds
        HIP_TRY(bemrat::launch_combine(b->Z.as<double2>() + b->off_Z[i], n * m, m, b->fold ? (int)b->P : (int)b->ops[i],
                                       reinterpret_cast<const double2 *>(pbase + (b->fold ? b->off_eye : b->off_coef[i])),
                                       (int)b->P, n, m, reinterpret_cast<double2 *>(M) + b->P * b->rows[i] * m, m, stream),
                "combine kernel");
    }
    return BEM_OK;
}

bem_status bem_batch_set_timing(bem_batch_t b, int on) {
    if (!b) return fail(BEM_EINVAL, "batch is NULL");
    b->timing = on != 0;
    return BEM_OK;
}

bem_status bem_batch_last_kernel_ms(bem_batch_t b, float *ms) {
    if (!b || !ms) return fail(BEM_EINVAL, "batch or ms is NULL");
    if (!b->timed) return fail(BEM_EINVAL, "no timed batch call yet");
    DeviceGuard guard(b->device);
    HIP_TRY(hipEventSynchronize(b->ev1), "event synchronize");
    HIP_TRY(hipEventElapsedTime(ms, b->ev0, b->ev1), "event elapsed time");
    return BEM_OK;
}

}  // extern "C"

// ---------------------------------------------------------------- learned near field

namespace {

bool device_ptrs(std::initializer_list<const void *> ps) {
    for (const void *p : ps)
        if (!is_device_ptr(p)) return false;
    return true;
}

}  // namespace

extern "C" {

int64_t bem_net_params(void) { return bemrat::kNetParams; }

bem_status bem_nf_labels(const double *P9, const double *x, const double *kappa, int64_t S, double *out,
                         hipStream_t stream) {
    if (S < 1) return fail(BEM_EINVAL, "need S >= 1");
    if (!device_ptrs({P9, x, kappa, out})) return fail(BEM_EINVAL, "P9, x, kappa and out must be device memory");
    double gl[2 * 16 + 2 * 10];
    gauss_legendre(16, gl, gl + 16);
    gauss_legendre(10, gl + 32, gl + 42);
    double r[28], rule[28];
    radon_rule(r);  // 7 x 3 barycentric weights, then the 7 weights
    for (int q = 0; q < 7; ++q) {
        for (int c = 0; c < 3; ++c) rule[4 * q + c] = r[3 * q + c];
        rule[4 * q + 3] = r[21 + q];
    }
    HIP_TRY(bemrat::launch_nf_labels(P9, x, reinterpret_cast<const double2 *>(kappa), S,
                                     reinterpret_cast<double2 *>(out), gl, rule, stream),
            "label kernel");
    return BEM_OK;
}

bem_status bem_net_features(const double *P9, const double *x, const double *kappa, int64_t S, float *X, double *aux,
                            hipStream_t stream) {
    if (S < 1) return fail(BEM_EINVAL, "need S >= 1");
    if (!device_ptrs({P9, x, kappa, X, aux})) return fail(BEM_EINVAL, "all arrays must be device memory");
    HIP_TRY(bemrat::launch_net_features(P9, x, reinterpret_cast<const double2 *>(kappa), S, X, aux, stream),
            "feature kernel");
    return BEM_OK;
}

bem_status bem_net_forward(const float *params, const float *X, int64_t B, float *Y, hipStream_t stream) {
    if (B < 1) return fail(BEM_EINVAL, "need B >= 1");
    if (!device_ptrs({params, X, Y})) return fail(BEM_EINVAL, "params, X and Y must be device memory");
    HIP_TRY(bemrat::launch_net_forward(params, X, B, Y, stream), "forward kernel");
    return BEM_OK;
}

int64_t bem_net_work_floats(int64_t B) {
    if (B < 1) return -1;
    const int64_t slots = bemrat::net_slots(B);
    return slots * (bemrat::kNetParams + 1);
}

bem_status bem_net_gradient(const float *params, const float *X, const float *T, int64_t B, float *work, float *grad,
                            float *loss, hipStream_t stream) {
    if (B < 1) return fail(BEM_EINVAL, "need B >= 1");
    if (!device_ptrs({params, X, T, work, grad, loss}))
        return fail(BEM_EINVAL, "params, X, T, work, grad and loss must be device memory");
    const int64_t slots = bemrat::net_slots(B);
    HIP_TRY(bemrat::launch_net_gradient(params, X, T, B, work, work + slots * bemrat::kNetParams, grad, loss, stream),
            "gradient kernels");
    return BEM_OK;
}

bem_status bem_net_adam(float *params, const float *grad, float *m, float *v, int64_t step, double lr,
                        hipStream_t stream) {
    if (step < 1 || !(lr > 0.0) || !std::isfinite(lr)) return fail(BEM_EINVAL, "need step >= 1 and lr > 0");
    if (!device_ptrs({params, grad, m, v})) return fail(BEM_EINVAL, "params, grad, m and v must be device memory");
    const double b1 = 0.9, b2 = 0.999;
    const double c1 = 1.0 - std::pow(b1, (double)step), c2 = 1.0 - std::pow(b2, (double)step);
    HIP_TRY(bemrat::launch_net_adam(params, grad, m, v, (float)lr, (float)b1, (float)b2, 1e-8f, (float)c1, (float)c2,
                                    stream),
            "Adam kernel");
    return BEM_OK;
}

int64_t bem_lu_work_bytes(int64_t n, int64_t m) {
    if (n < 1 || m < 0) return -1;
    return m == 0 ? bemrat::lu_factor_work_bytes() : bemrat::lu_solve_work_bytes(n, m);
}

bem_status bem_lu_factor(double *A, int64_t n, int64_t lda, int64_t *ipiv, int64_t *perm, int64_t *info, void *work,
                         int64_t work_bytes, hipStream_t stream) {
    if (n < 1 || lda < n) return fail(BEM_EINVAL, "need n >= 1 and lda >= n");
    if (!device_ptrs({A, ipiv, perm, info, work})) return fail(BEM_EINVAL, "A, ipiv, perm, info and work must be device memory");
    if (work_bytes < bemrat::lu_factor_work_bytes()) return fail(BEM_EINVAL, "work is smaller than bem_lu_work_bytes(n, 0)");
    HIP_TRY(bemrat::lu_factor(reinterpret_cast<double2 *>(A), n, lda, ipiv, perm, info, work, stream), "LU kernels");
    return BEM_OK;
}

bem_status bem_lu_solve(const double *LU, int64_t n, int64_t lda, const int64_t *perm, const double *B, int64_t ldb,
                        double *X, int64_t ldx, int64_t m, void *work, int64_t work_bytes, hipStream_t stream) {
    if (n < 1 || m < 1 || lda < n || ldb < m || ldx < m) return fail(BEM_EINVAL, "need n, m >= 1, lda >= n, ldb and ldx >= m");
    if (!device_ptrs({LU, perm, B, X, work})) return fail(BEM_EINVAL, "LU, perm, B, X and work must be device memory");
    if (work_bytes < bemrat::lu_solve_work_bytes(n, m)) return fail(BEM_EINVAL, "work is smaller than bem_lu_work_bytes(n, m)");
    const char *b0 = reinterpret_cast<const char *>(B), *x0 = reinterpret_cast<const char *>(X);
    const int64_t bb = ((n - 1) * ldb + m) * 16, xb = ((n - 1) * ldx + m) * 16;
    if (b0 < x0 + xb && x0 < b0 + bb) return fail(BEM_EINVAL, "X overlaps B");
    HIP_TRY(bemrat::lu_solve(reinterpret_cast<const double2 *>(LU), n, lda, perm, reinterpret_cast<const double2 *>(B),
                             ldb, reinterpret_cast<double2 *>(X), ldx, m, work, stream),
            "LU solve kernels");
    return BEM_OK;
}

bem_status bem_block_combine(const double *const *blocks, int64_t nb, const double *coef, int64_t n, int64_t m,
                             int64_t ldx, double *out, int64_t ldo, hipStream_t stream) {
    if (!blocks || nb < 1 || nb > bemrat::kBlockCombineMax)
        return fail(BEM_EINVAL, "need 1 <= nb <= 64 block pointers");
    if (n < 1 || m < 1 || ldx < m || ldo < m) return fail(BEM_EINVAL, "need n, m >= 1, ldx and ldo >= m");
    if (!device_ptrs({coef, out})) return fail(BEM_EINVAL, "coef and out must be device memory");
    const int64_t xb = ((n - 1) * ldx + m) * 16, ob = ((n - 1) * ldo + m) * 16;
    const char *o0 = reinterpret_cast<const char *>(out);
    for (int64_t b = 0; b < nb; ++b) {
        if (!is_device_ptr(blocks[b])) return fail(BEM_EINVAL, "every block must be device memory");
        const char *b0 = reinterpret_cast<const char *>(blocks[b]);
        // out may be one of the blocks (each element is read and written by one thread), not
        // overlap one otherwise
        if (b0 < o0 + ob && o0 < b0 + xb && !(b0 == o0 && ldo == ldx)) return fail(BEM_EINVAL, "out overlaps a block");
    }
    HIP_TRY(bemrat::launch_block_combine(reinterpret_cast<const double2 *const *>(blocks), (int)nb,
                                         reinterpret_cast<const double2 *>(coef), n, m, ldx,
                                         reinterpret_cast<double2 *>(out), ldo, stream),
            "block combine kernel");
    return BEM_OK;
}

bem_status bem_nearfield_moments_net(bem_mesh_t h, const bem_net_model *model, const double *z, int64_t N,
                                     const double *W, int64_t P, const double *V, int64_t m, int64_t ldv, double *M,
                                     int64_t ldm, int64_t *fallback_pairs, hipStream_t stream) {
    if (!model) return fail(BEM_EINVAL, "model is NULL");
    return nearfield_moments_impl(h, model, z, N, W, P, V, m, ldv, M, ldm, fallback_pairs, stream);
}

bem_status bem_nearfield_project(bem_mesh_t h, const bem_net_model *model, const double *z, int64_t N, const double *U,
                                 int64_t m, int64_t ldu, double *Pout, hipStream_t stream) {
    if (!h) return fail(BEM_EINVAL, "mesh is NULL");
    DeviceGuard guard(h->device);
    bem_status st = check_kappas(h, z, N, "z");
    if (st != BEM_OK) return st;
    if (N > 4096) return fail(BEM_EINVAL, "at most 4096 nodes");
    if ((st = check_block(U, m, ldu, "U")) != BEM_OK) return st;
    if (!Pout || !is_device_ptr(Pout)) return fail(BEM_EINVAL, "Pout is not device memory");
    if (h->nf_pairs == 0) return BEM_OK;
    const int64_t n = h->dm.n;
    const size_t zstride = (size_t)n * m;
    // per-node corrections Y_j = dT(z_j) U, then Pout[j] += U^H Y_j
    std::vector<double> eye(2 * (size_t)N * N, 0.0);
    for (int64_t j = 0; j < N; ++j) eye[2 * (j * N + j)] = 1.0;
    const int64_t rows_per_chunk = 4096;
    const int nchunks = (int)((n + rows_per_chunk - 1) / rows_per_chunk);
    HIP_TRY(h->Z.ensure(sizeof(double2) * zstride * N), "correction workspace");
    HIP_TRY(h->partial.ensure(sizeof(double2) * (size_t)N * nchunks * m * m), "projection workspace");
    double2 *Y = h->Z.as<double2>();
    HIP_TRY(hipMemsetAsync(Y, 0, sizeof(double2) * zstride * N, stream), "workspace clear");
    if ((st = nearfield_moments_impl(h, model, z, N, eye.data(), N, U, m, ldu, reinterpret_cast<double *>(Y), m,
                                     nullptr, stream)) != BEM_OK)
        return st;
    HIP_TRY(bemrat::launch_project_partial(reinterpret_cast<const double2 *>(U), ldu, Y, zstride, m, (int)N, n, m,
                                           rows_per_chunk, nchunks, h->partial.as<double2>(), stream),
            "projection kernel");
    HIP_TRY(bemrat::launch_project_add(h->partial.as<double2>(), nchunks, (int)N, m, reinterpret_cast<double2 *>(Pout),
                                       stream),
            "projection reduction kernel");
    return BEM_OK;
}

}  // extern "C"

