"""ctypes binding of libbemrat.so (C ABI in include/bemrat.h).

Argument marshalling only: tensors are passed as device pointers with their row
strides, the stream is torch's current stream, and every numerical step runs in the
library's HIP kernels.  There is no fallback: if the library is missing or no HIP device
is present the calls raise.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libbemrat.so")

BEM_OK, BEM_EINVAL, BEM_EMESH, BEM_ENOMEM, BEM_EDEVICE, BEM_EUNSUPPORTED = range(6)
FORM_AUTO, FORM_DIRECT, FORM_EXPAND, FORM_CHEB = 0, 1, 2, 3
PREC_F64, PREC_F32, PREC_BF16, PREC_F16 = 0x00, 0x10, 0x20, 0x30
FORM_MASK, PREC_MASK = 0x03, 0xF0
NF_AUTO, NF_NODES = 0, 1
STATUS_NAMES = {0: "BEM_OK", 1: "BEM_EINVAL", 2: "BEM_EMESH", 3: "BEM_ENOMEM", 4: "BEM_EDEVICE",
                5: "BEM_EUNSUPPORTED"}

# every symbol declared in include/bemrat.h
EXPORTS = [
    "bem_mesh_create", "bem_mesh_destroy", "bem_mesh_size", "bem_mesh_geometry",
    "bem_contour_nodes", "bem_cheb_nodes", "bem_self_terms", "bem_assemble_apply",
    "contour_moments", "cheb_moments", "rr_project", "bem_last_form", "bem_set_timing",
    "bem_last_kernel_ms", "bem_stream_status", "bem_last_error",
    "bem_assemble_sum", "bem_batch_create", "bem_batch_destroy", "bem_batch_layout", "bem_batch_moments",
    "bem_batch_set_timing", "bem_batch_last_kernel_ms",
    "bem_mesh_set_nearfield", "bem_mesh_nearfield", "bem_nearfield_moments", "bem_nearfield_sum",
    "bem_mesh_set_nearfield_mode", "bem_nearfield_last_terms",
    "contour_moments_noalloc",
    "bem_net_params", "bem_nf_labels", "bem_net_features", "bem_net_forward", "bem_net_work_floats",
    "bem_net_gradient", "bem_net_adam", "bem_nearfield_moments_net", "bem_nearfield_project",
    "bem_lu_work_bytes", "bem_lu_factor", "bem_lu_solve", "bem_block_combine",
]

NET_PARAMS = 37506
NET_INPUTS = 32
NET_BINS = 8


class NetModelC(ctypes.Structure):
    """The C struct bem_net_model (include/bemrat.h)."""
    _fields_ = [("params", ctypes.c_void_p), ("out_scale", ctypes.c_double * 2), ("dmin", ctypes.c_double),
                ("min_angle_deg", ctypes.c_double), ("kh_re_max", ctypes.c_double), ("kh_im_max", ctypes.c_double),
                ("bin_edges", ctypes.c_double * (NET_BINS + 1)), ("bin_trusted", ctypes.c_int * NET_BINS),
                ("freeze_tol", ctypes.c_double)]


class BemError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


_dp = ctypes.POINTER(ctypes.c_double)
_vp = ctypes.c_void_p
_i64 = ctypes.c_int64
_u32 = ctypes.c_uint32
_lib = None


def lib():
    """Loads libbemrat.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_1906_03938_amd.build`")
    L = ctypes.CDLL(LIB_PATH)
    L.bem_mesh_create.argtypes = [_dp, _i64, ctypes.POINTER(ctypes.c_int32), _i64, _vp, ctypes.POINTER(_vp)]
    L.bem_mesh_destroy.argtypes = [_vp]
    L.bem_mesh_destroy.restype = None
    L.bem_mesh_size.argtypes = [_vp]
    L.bem_mesh_size.restype = _i64
    L.bem_mesh_geometry.argtypes = [_vp, _dp, _dp, _dp, _dp, _vp]
    L.bem_contour_nodes.argtypes = [ctypes.c_double, ctypes.c_double, ctypes.c_double, _i64, ctypes.c_double,
                                    ctypes.c_double, _i64, _dp, _dp, _dp]
    L.bem_cheb_nodes.argtypes = [ctypes.c_double, ctypes.c_double, _i64, _dp, _dp]
    L.bem_self_terms.argtypes = [_vp, _dp, _i64, _vp, _vp]
    L.bem_assemble_apply.argtypes = [_vp, _dp, _i64, _vp, _i64, _i64, _vp, _i64, _u32, _vp]
    L.contour_moments.argtypes = [_vp, _dp, _i64, _dp, _i64, _vp, _i64, _i64, _vp, _i64, _u32, _vp]
    L.contour_moments_noalloc.argtypes = [_vp, _dp, _i64, _dp, _i64, _vp, _i64, _i64, _vp, _i64, _u32, _vp]
    L.cheb_moments.argtypes = [_vp, ctypes.c_double, ctypes.c_double, _i64, _i64, _vp, _i64, _i64, _vp, _i64,
                               _u32, _vp]
    L.rr_project.argtypes = [_vp, _dp, _i64, _vp, _i64, _i64, _vp, _dp, _i64, _vp, _i64, _u32, _vp]
    L.bem_last_form.argtypes = [_vp, ctypes.POINTER(_u32), ctypes.POINTER(_i64)]
    L.bem_set_timing.argtypes = [_vp, ctypes.c_int]
    L.bem_last_kernel_ms.argtypes = [_vp, ctypes.POINTER(ctypes.c_float)]
    L.bem_stream_status.argtypes = [_vp]
    L.bem_last_error.argtypes = []
    L.bem_last_error.restype = ctypes.c_char_p
    L.bem_assemble_sum.argtypes = [_vp, _dp, _i64, _dp, _vp, _i64, _u32, _vp]
    L.bem_batch_create.argtypes = [ctypes.POINTER(_vp), _i64, _dp, _i64, _dp, _i64, _i64, _u32, ctypes.c_int, _vp,
                                   ctypes.POINTER(_vp)]
    L.bem_batch_destroy.argtypes = [_vp]
    L.bem_batch_destroy.restype = None
    L.bem_batch_layout.argtypes = [_vp, ctypes.POINTER(_i64), ctypes.POINTER(_i64), ctypes.POINTER(_u32),
                                   ctypes.POINTER(ctypes.c_int)]
    L.bem_batch_moments.argtypes = [_vp, _vp, _vp, _vp]
    L.bem_batch_set_timing.argtypes = [_vp, ctypes.c_int]
    L.bem_batch_last_kernel_ms.argtypes = [_vp, ctypes.POINTER(ctypes.c_float)]
    L.bem_mesh_set_nearfield.argtypes = [_vp, ctypes.c_double]
    L.bem_mesh_nearfield.argtypes = [_vp, ctypes.POINTER(_i64), _vp, _vp]
    L.bem_mesh_set_nearfield_mode.argtypes = [_vp, ctypes.c_int]
    L.bem_nearfield_last_terms.argtypes = [_vp, ctypes.POINTER(ctypes.c_int)]
    L.bem_nearfield_moments.argtypes = [_vp, _dp, _i64, _dp, _i64, _vp, _i64, _i64, _vp, _i64, _vp]
    L.bem_nearfield_sum.argtypes = [_vp, _dp, _i64, _dp, _vp, _i64, _vp]
    L.bem_net_params.argtypes = []
    L.bem_nf_labels.argtypes = [_vp, _vp, _vp, _i64, _vp, _vp]
    L.bem_net_features.argtypes = [_vp, _vp, _vp, _i64, _vp, _vp, _vp]
    L.bem_net_forward.argtypes = [_vp, _vp, _i64, _vp, _vp]
    L.bem_net_work_floats.argtypes = [_i64]
    L.bem_net_gradient.argtypes = [_vp, _vp, _vp, _i64, _vp, _vp, _vp, _vp]
    L.bem_net_adam.argtypes = [_vp, _vp, _vp, _vp, _i64, ctypes.c_double, _vp]
    L.bem_nearfield_moments_net.argtypes = [_vp, ctypes.POINTER(NetModelC), _dp, _i64, _dp, _i64, _vp, _i64, _i64, _vp,
                                            _i64, ctypes.POINTER(_i64), _vp]
    L.bem_nearfield_project.argtypes = [_vp, ctypes.POINTER(NetModelC), _dp, _i64, _vp, _i64, _i64, _vp, _vp]
    L.bem_lu_work_bytes.argtypes = [_i64, _i64]
    L.bem_lu_factor.argtypes = [_vp, _i64, _i64, _vp, _vp, _vp, _vp, _i64, _vp]
    L.bem_lu_solve.argtypes = [_vp, _i64, _i64, _vp, _vp, _i64, _vp, _i64, _i64, _vp, _i64, _vp]
    L.bem_block_combine.argtypes = [ctypes.POINTER(_vp), _i64, _vp, _i64, _i64, _i64, _vp, _i64, _vp]
    for name in EXPORTS:
        f = getattr(L, name)
        if name not in ("bem_mesh_destroy", "bem_mesh_size", "bem_last_error", "bem_batch_destroy", "bem_net_params",
                        "bem_net_work_floats", "bem_lu_work_bytes"):
            f.restype = ctypes.c_int
    L.bem_net_params.restype = _i64
    L.bem_net_work_floats.restype = _i64
    L.bem_lu_work_bytes.restype = _i64
    if L.bem_net_params() != NET_PARAMS:
        raise ImportError("libbemrat.so was built with a different network layout")
    _lib = L
    return L


def _check(status: int):
    if status != BEM_OK:
        raise BemError(status, lib().bem_last_error().decode())


def _host_complex(values) -> np.ndarray:
    return np.ascontiguousarray(np.atleast_1d(np.asarray(values, dtype=np.complex128)))


def _hp(a: np.ndarray):
    return a.view(np.float64).ctypes.data_as(_dp) if a.dtype == np.complex128 else a.ctypes.data_as(_dp)


def _torch():
    import torch

    return torch


def _stream():
    torch = _torch()
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _block(t, name):
    """(pointer, m, ld) of a complex128 CUDA matrix whose rows may be strided."""
    torch = _torch()
    if not isinstance(t, torch.Tensor) or t.dtype != torch.complex128 or not t.is_cuda:
        raise TypeError(f"{name} must be a complex128 CUDA tensor")
    if t.dim() != 2 or t.stride(1) != 1:
        raise ValueError(f"{name} must be 2-D with unit column stride")
    return ctypes.c_void_p(t.data_ptr()), t.shape[1], t.stride(0)


def _out_blocks(t, blocks, n, m, name):
    """Checks a caller-supplied output of `blocks` blocks of n x m complex128 on the device,
    laid out as the C ABI expects (block p at 2*p*n*ld doubles, row stride ld >= m)."""
    torch = _torch()
    if not isinstance(t, torch.Tensor) or t.dtype != torch.complex128 or not t.is_cuda:
        raise TypeError(f"{name} must be a complex128 CUDA tensor")
    if t.dim() != 3 or t.shape[0] < blocks or t.shape[1] != n or t.shape[2] != m:
        raise ValueError(f"{name} must have shape ({blocks}, {n}, {m}), got {tuple(t.shape)}")
    if t.stride(2) != 1 or t.stride(0) != n * t.stride(1):
        raise ValueError(f"{name} must have unit column stride and blocks of n rows back to back")
    return t


def _dense_out(t, n, name):
    """Checks an n x n (row stride >= n) complex128 device matrix."""
    torch = _torch()
    if not isinstance(t, torch.Tensor) or t.dtype != torch.complex128 or not t.is_cuda:
        raise TypeError(f"{name} must be a complex128 CUDA tensor")
    if t.dim() != 2 or t.shape[0] != n or t.shape[1] < n or t.stride(1) != 1 or t.stride(0) < n:
        raise ValueError(f"{name} must be an n x n (row stride >= n) complex128 device matrix")
    return t


# ------------------------------------------------------------------- host routines


def contour_nodes(c, radius, N, shift=None, P=0):
    """Trapezoidal nodes/weights on |z - c| = radius and moment weights (host, in C)."""
    c = complex(c)
    shift = c if shift is None else complex(shift)
    z = np.zeros(N, dtype=np.complex128)
    w = np.zeros(N, dtype=np.complex128)
    W = np.zeros((N, max(P, 1)), dtype=np.complex128)
    _check(lib().bem_contour_nodes(c.real, c.imag, float(radius), N, shift.real, shift.imag, P, _hp(z), _hp(w),
                                   _hp(W)))
    return z, w, (W[:, :P] if P else None)


def cheb_nodes(a, b, N):
    kappa = np.zeros(N)
    coef = np.zeros((N, N))
    _check(lib().bem_cheb_nodes(float(a), float(b), N, kappa.ctypes.data_as(_dp), coef.ctypes.data_as(_dp)))
    return kappa, coef


# ------------------------------------------------------------------------- the mesh


class Mesh:
    """A triangle mesh resident on the current HIP device."""

    def __init__(self, xyz, tri):
        xyz = np.ascontiguousarray(xyz, dtype=np.float64)
        tri = np.ascontiguousarray(tri, dtype=np.int32)
        if xyz.ndim != 2 or xyz.shape[1] != 3 or tri.ndim != 2 or tri.shape[1] != 3:
            raise ValueError("xyz must be (nv, 3) and tri (n, 3)")
        h = ctypes.c_void_p()
        _check(lib().bem_mesh_create(xyz.ctypes.data_as(_dp), xyz.shape[0],
                                     tri.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), tri.shape[0], _stream(),
                                     ctypes.byref(h)))
        self._h = h
        self.n = tri.shape[0]

    def close(self):
        if getattr(self, "_h", None):
            lib().bem_mesh_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # -- helpers
    def _out(self, blocks, m):
        torch = _torch()
        return torch.empty((blocks, self.n, m), dtype=torch.complex128, device="cuda")

    def geometry(self):
        n = self.n
        area = np.zeros(n)
        cen = np.zeros((n, 3))
        qp = np.zeros((n, 7, 3))
        qw = np.zeros((n, 7))
        _check(lib().bem_mesh_geometry(self._h, area.ctypes.data_as(_dp), cen.ctypes.data_as(_dp),
                                       qp.ctypes.data_as(_dp), qw.ctypes.data_as(_dp), _stream()))
        return area, cen, qp, qw

    def self_terms(self, kappas):
        torch = _torch()
        k = _host_complex(kappas)
        S = torch.empty((k.size, self.n), dtype=torch.complex128, device="cuda")
        _check(lib().bem_self_terms(self._h, _hp(k), k.size, ctypes.c_void_p(S.data_ptr()), _stream()))
        return S

    def assemble_apply(self, kappas, V, out=None, form=FORM_DIRECT):
        k = _host_complex(kappas)
        pv, m, ldv = _block(V, "V")
        Y = self._out(k.size, m) if out is None else _out_blocks(out, k.size, self.n, m, "out")
        _check(lib().bem_assemble_apply(self._h, _hp(k), k.size, pv, m, ldv, ctypes.c_void_p(Y.data_ptr()),
                                        Y.stride(1), form, _stream()))
        return Y

    def contour_moments(self, z, W, V, out=None, form=FORM_AUTO):
        z = _host_complex(z)
        W = np.ascontiguousarray(np.asarray(W, dtype=np.complex128).reshape(z.size, -1))
        pv, m, ldv = _block(V, "V")
        M = self._out(W.shape[1], m) if out is None else _out_blocks(out, W.shape[1], self.n, m, "out")
        _check(lib().contour_moments(self._h, _hp(z), z.size, _hp(W), W.shape[1], pv, m, ldv,
                                     ctypes.c_void_p(M.data_ptr()), M.stride(1), form, _stream()))
        return M

    def contour_moments_noalloc(self, z, W, V, out, form=FORM_AUTO):
        """contour_moments with the library's static scratch as workspace (no device
        allocation); `out` (P, n, m) complex128 must be given."""
        z = _host_complex(z)
        W = np.ascontiguousarray(np.asarray(W, dtype=np.complex128).reshape(z.size, -1))
        pv, m, ldv = _block(V, "V")
        M = _out_blocks(out, W.shape[1], self.n, m, "out")
        _check(lib().contour_moments_noalloc(self._h, _hp(z), z.size, _hp(W), W.shape[1], pv, m, ldv,
                                             ctypes.c_void_p(M.data_ptr()), M.stride(1), form, _stream()))
        return M

    def nearfield_moments_net(self, model, z, W, V, out=None, count_fallback=False):
        """Adds the near-field correction sum_j W[j, p] dT(z_j) V to out (zeros if None), with
        the network of `model` (a bem_net_model, see nfnet.NearFieldNet.c_model) inside its
        trust region and the quadrature elsewhere.  Returns out, or (out, number of pairs the
        quadrature handled) with count_fallback."""
        z = _host_complex(z)
        W = np.ascontiguousarray(np.asarray(W, dtype=np.complex128).reshape(z.size, -1))
        pv, m, ldv = _block(V, "V")
        M = self._out(W.shape[1], m) if out is None else _out_blocks(out, W.shape[1], self.n, m, "out")
        if out is None:
            M.zero_()
        cnt = _i64(0)
        _check(lib().bem_nearfield_moments_net(self._h, ctypes.byref(model), _hp(z), z.size, _hp(W), W.shape[1], pv, m,
                                               ldv, ctypes.c_void_p(M.data_ptr()), M.stride(1),
                                               ctypes.byref(cnt) if count_fallback else None, _stream()))
        return (M, int(cnt.value)) if count_fallback else M

    def nearfield_project(self, z, U, P, model=None):
        """Adds U^H dT(z_j) U to the projections P (N x m x m complex128, device) in place: the
        quadrature's correction, or the network's inside the trust region of `model` (a
        bem_net_model)."""
        torch = _torch()
        z = _host_complex(z)
        pu, m, ldu = _block(U, "U")
        if not isinstance(P, torch.Tensor) or P.dtype != torch.complex128 or not P.is_cuda or not P.is_contiguous() \
                or tuple(P.shape) != (z.size, m, m):
            raise ValueError(f"P must be a contiguous ({z.size}, {m}, {m}) complex128 CUDA tensor")
        _check(lib().bem_nearfield_project(self._h, ctypes.byref(model) if model is not None else None, _hp(z), z.size,
                                           pu, m, ldu, ctypes.c_void_p(P.data_ptr()), _stream()))
        return P

    def set_nearfield(self, eta: float):
        """Builds (eta > 0) or removes (eta = 0) the mesh's near-pair list."""
        _check(lib().bem_mesh_set_nearfield(self._h, float(eta)))

    def set_nearfield_mode(self, mode: int):
        """NF_AUTO (series form where it converges, the default) or NF_NODES (every node)."""
        _check(lib().bem_mesh_set_nearfield_mode(self._h, int(mode)))

    def nearfield_last_terms(self) -> int:
        """Series length of the last near-field call (0: evaluated per node)."""
        L = ctypes.c_int(0)
        _check(lib().bem_nearfield_last_terms(self._h, ctypes.byref(L)))
        return L.value

    def nearfield_list(self):
        """(rowptr[n + 1], col[pairs]) of the near-pair list as NumPy arrays."""
        cnt = _i64(0)
        _check(lib().bem_mesh_nearfield(self._h, ctypes.byref(cnt), None, None))
        rowptr = np.zeros(self.n + 1, dtype=np.int64)
        col = np.zeros(max(cnt.value, 1), dtype=np.int32)
        _check(lib().bem_mesh_nearfield(self._h, ctypes.byref(cnt), rowptr.ctypes.data_as(_vp),
                                        col.ctypes.data_as(_vp)))
        return rowptr, col[:cnt.value]

    def nearfield_moments(self, z, W, V, out=None):
        """Adds sum_j W[j, p] dT(z_j) V to out (zeros if None) and returns it."""
        z = _host_complex(z)
        W = np.ascontiguousarray(np.asarray(W, dtype=np.complex128).reshape(z.size, -1))
        pv, m, ldv = _block(V, "V")
        M = self._out(W.shape[1], m) if out is None else _out_blocks(out, W.shape[1], self.n, m, "out")
        if out is None:
            M.zero_()
        _check(lib().bem_nearfield_moments(self._h, _hp(z), z.size, _hp(W), W.shape[1], pv, m, ldv,
                                           ctypes.c_void_p(M.data_ptr()), M.stride(1), _stream()))
        return M

    def nearfield_sum(self, z, c, S):
        """Adds sum_j c_j dT(z_j) to the dense n x n matrix S (device, complex128) in place."""
        z = _host_complex(z)
        c = _host_complex(c)
        if c.size != z.size:
            raise ValueError("need one coefficient per node")
        _dense_out(S, self.n, "S")
        _check(lib().bem_nearfield_sum(self._h, _hp(z), z.size, _hp(c), ctypes.c_void_p(S.data_ptr()), S.stride(0),
                                       _stream()))
        return S

    def cheb_moments(self, a, b, N, L, V, out=None, form=FORM_AUTO):
        pv, m, ldv = _block(V, "V")
        C = self._out(L, m) if out is None else _out_blocks(out, L, self.n, m, "out")
        _check(lib().cheb_moments(self._h, float(a), float(b), N, L, pv, m, ldv, ctypes.c_void_p(C.data_ptr()),
                                  C.stride(1), form, _stream()))
        return C

    def rr_project(self, z, U, W=None, out=None, moments_out=None, form=FORM_AUTO):
        torch = _torch()
        z = _host_complex(z)
        pu, m, ldu = _block(U, "U")
        Pout = torch.empty((z.size, m, m), dtype=torch.complex128, device="cuda") if out is None else out
        if out is not None:
            _out_blocks(out, z.size, m, m, "out")
            if not out.is_contiguous():
                raise ValueError("out must be a contiguous (N, m, m) tensor")
        M = None
        if W is not None:
            W = np.ascontiguousarray(np.asarray(W, dtype=np.complex128).reshape(z.size, -1))
            M = self._out(W.shape[1], m) if moments_out is None else \
                _out_blocks(moments_out, W.shape[1], self.n, m, "moments_out")
            _check(lib().rr_project(self._h, _hp(z), z.size, pu, m, ldu, ctypes.c_void_p(Pout.data_ptr()), _hp(W),
                                    W.shape[1], ctypes.c_void_p(M.data_ptr()), M.stride(1), form, _stream()))
        else:
            _check(lib().rr_project(self._h, _hp(z), z.size, pu, m, ldu, ctypes.c_void_p(Pout.data_ptr()), None, 0,
                                    None, m, form, _stream()))
        return (Pout, M) if W is not None else Pout

    def assemble_sum(self, z, c, out=None, form=FORM_AUTO):
        """Dense S = sum_j c_j T(z_j) (n x n complex128 on the device)."""
        torch = _torch()
        z = _host_complex(z)
        c = _host_complex(c)
        if c.size != z.size:
            raise ValueError("z and c must have the same length")
        S = torch.empty((self.n, self.n), dtype=torch.complex128, device="cuda") if out is None else \
            _dense_out(out, self.n, "out")
        _check(lib().bem_assemble_sum(self._h, _hp(z), z.size, _hp(c), ctypes.c_void_p(S.data_ptr()), S.stride(0),
                                      form, _stream()))
        return S

    def last_form(self):
        f = _u32()
        ops = _i64()
        _check(lib().bem_last_form(self._h, ctypes.byref(f), ctypes.byref(ops)))
        return int(f.value), int(ops.value)

    def set_timing(self, on=True):
        _check(lib().bem_set_timing(self._h, 1 if on else 0))

    def last_kernel_ms(self):
        ms = ctypes.c_float()
        _check(lib().bem_last_kernel_ms(self._h, ctypes.byref(ms)))
        return float(ms.value)


class Batch:
    """Several meshes, each with its own nodes z[i] (N complex) and moment weights W[i]
    (N x P), whose contour moments run as one persistent launch (bem_batch_create).  The
    probe blocks are packed: mesh i owns rows rows[i]:rows[i+1] of V (rows[-1] x m); the
    moments come back packed the same way, P blocks per mesh (see split)."""

    def __init__(self, meshes, z, W, m, form=FORM_AUTO, tune=False):
        meshes = list(meshes)
        count = len(meshes)
        z = np.ascontiguousarray(np.asarray(z, dtype=np.complex128).reshape(count, -1))
        N = z.shape[1]
        W = np.ascontiguousarray(np.asarray(W, dtype=np.complex128).reshape(count, N, -1))
        handles = (_vp * count)(*[mm._h for mm in meshes])
        h = ctypes.c_void_p()
        _check(lib().bem_batch_create(handles, count, _hp(z), N, _hp(W), W.shape[2], int(m), form, 1 if tune else 0,
                                      _stream(), ctypes.byref(h)))
        self._h = h
        self._meshes = meshes  # the batch reads their geometry
        self.count, self.N, self.P, self.m = count, N, W.shape[2], int(m)
        rows = np.zeros(count + 1, dtype=np.int64)
        ops = np.zeros(count, dtype=np.int64)
        f = _u32()
        ct = ctypes.c_int()
        _check(lib().bem_batch_layout(h, rows.ctypes.data_as(ctypes.POINTER(_i64)),
                                      ops.ctypes.data_as(ctypes.POINTER(_i64)), ctypes.byref(f), ctypes.byref(ct)))
        self.rows, self.operators, self.form, self.col_tile = rows, ops, int(f.value), int(ct.value)

    def close(self):
        if getattr(self, "_h", None):
            lib().bem_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def moments(self, V, out=None):
        """Packed moments of the packed probe block V (rows[-1] x m complex128, contiguous)."""
        torch = _torch()
        if not isinstance(V, torch.Tensor) or V.dtype != torch.complex128 or not V.is_cuda:
            raise TypeError("V must be a complex128 CUDA tensor")
        if tuple(V.shape) != (int(self.rows[-1]), self.m) or not V.is_contiguous():
            raise ValueError(f"V must be a contiguous ({int(self.rows[-1])}, {self.m}) tensor")
        M = torch.empty(self.P * int(self.rows[-1]) * self.m, dtype=torch.complex128, device="cuda") \
            if out is None else out
        if not isinstance(M, torch.Tensor) or M.dtype != torch.complex128 or not M.is_cuda:
            raise TypeError("out must be a complex128 CUDA tensor")
        if M.numel() != self.P * int(self.rows[-1]) * self.m or not M.is_contiguous():
            raise ValueError("out has the wrong size or layout")
        _check(lib().bem_batch_moments(self._h, ctypes.c_void_p(V.data_ptr()), ctypes.c_void_p(M.data_ptr()),
                                       _stream()))
        return M

    def split(self, M):
        """Views of the packed moments: a list of (P, n_i, m) blocks, one per mesh."""
        out = []
        for i in range(self.count):
            a, b = int(self.rows[i]), int(self.rows[i + 1])
            out.append(M[self.P * a * self.m:self.P * b * self.m].view(self.P, b - a, self.m))
        return out

    def set_timing(self, on=True):
        _check(lib().bem_batch_set_timing(self._h, 1 if on else 0))

    def last_kernel_ms(self):
        ms = ctypes.c_float()
        _check(lib().bem_batch_last_kernel_ms(self._h, ctypes.byref(ms)))
        return float(ms.value)


def stream_status():
    _check(lib().bem_stream_status(_stream()))


# ------------------------------------------------------------- learned near field


def _dev_tensor(t, dtype, shape, name):
    torch = _torch()
    if not isinstance(t, torch.Tensor) or t.dtype != dtype or not t.is_cuda or not t.is_contiguous():
        raise TypeError(f"{name} must be a contiguous {dtype} CUDA tensor")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")
    return ctypes.c_void_p(t.data_ptr())


def nf_labels(P9, x, kappa):
    """dT = integral - 7-point value for each (triangle P9[s] (S x 9 or S x 3 x 3 float64),
    target x[s] (S x 3), wavenumber kappa[s] (complex128)), by the library's quadrature."""
    torch = _torch()
    S = kappa.shape[0]
    out = torch.empty(S, dtype=torch.complex128, device="cuda")
    _check(lib().bem_nf_labels(_dev_tensor(P9.reshape(S, 9), torch.float64, (S, 9), "P9"),
                               _dev_tensor(x, torch.float64, (S, 3), "x"),
                               _dev_tensor(kappa, torch.complex128, (S,), "kappa"), S, ctypes.c_void_p(out.data_ptr()),
                               _stream()))
    return out


def net_features(P9, x, kappa):
    """(X (S x 32 float32 network inputs), aux (S x 4 float64: h, r0, Re kappa h, Im kappa h))."""
    torch = _torch()
    S = kappa.shape[0]
    X = torch.empty((S, NET_INPUTS), dtype=torch.float32, device="cuda")
    aux = torch.empty((S, 4), dtype=torch.float64, device="cuda")
    _check(lib().bem_net_features(_dev_tensor(P9.reshape(S, 9), torch.float64, (S, 9), "P9"),
                                  _dev_tensor(x, torch.float64, (S, 3), "x"),
                                  _dev_tensor(kappa, torch.complex128, (S,), "kappa"), S, ctypes.c_void_p(X.data_ptr()),
                                  ctypes.c_void_p(aux.data_ptr()), _stream()))
    return X, aux


def net_forward(params, X, out=None):
    """FP32 forward pass: Y (B x 2) of inputs X (B x 32)."""
    torch = _torch()
    B = X.shape[0]
    Y = torch.empty((B, 2), dtype=torch.float32, device="cuda") if out is None else out
    _check(lib().bem_net_forward(_dev_tensor(params, torch.float32, (NET_PARAMS,), "params"),
                                 _dev_tensor(X, torch.float32, (B, NET_INPUTS), "X"), B,
                                 _dev_tensor(Y, torch.float32, (B, 2), "out"), _stream()))
    return Y


def net_work(B):
    torch = _torch()
    return torch.empty(int(lib().bem_net_work_floats(int(B))), dtype=torch.float32, device="cuda")


def net_gradient(params, X, T, work=None, grad=None, loss=None):
    """(grad, loss) of the mean squared error (1/B) sum (Y - T)^2 on the batch (X, T)."""
    torch = _torch()
    B = X.shape[0]
    work = net_work(B) if work is None else work
    grad = torch.empty(NET_PARAMS, dtype=torch.float32, device="cuda") if grad is None else grad
    loss = torch.empty(1, dtype=torch.float32, device="cuda") if loss is None else loss
    if work.numel() < lib().bem_net_work_floats(B):
        raise ValueError("work is too small")
    _check(lib().bem_net_gradient(_dev_tensor(params, torch.float32, (NET_PARAMS,), "params"),
                                  _dev_tensor(X, torch.float32, (B, NET_INPUTS), "X"),
                                  _dev_tensor(T, torch.float32, (B, 2), "T"), B, ctypes.c_void_p(work.data_ptr()),
                                  _dev_tensor(grad, torch.float32, (NET_PARAMS,), "grad"),
                                  _dev_tensor(loss, torch.float32, (1,), "loss"), _stream()))
    return grad, loss


def net_adam(params, grad, m, v, step, lr):
    """One Adam update of params (in place) with moment estimates m, v (in place)."""
    torch = _torch()
    args = [_dev_tensor(t, torch.float32, (NET_PARAMS,), n) for t, n in ((params, "params"), (grad, "grad"), (m, "m"),
                                                                          (v, "v"))]
    _check(lib().bem_net_adam(*args, int(step), float(lr), _stream()))


def block_combine(blocks, coef, out=None):
    """out[r, c] = sum_b coef[b, c] blocks[b][r, c] on the device (bem_block_combine): blocks
    are n x m complex128 CUDA tensors with one row stride, coef an nb x m complex array
    (host; copied to the device), out a new n x m tensor unless given."""
    torch = _torch()
    blocks = list(blocks)
    if not blocks:
        raise ValueError("need at least one block")
    ptrs, ldx = [], None
    n, m = blocks[0].shape
    for k, b in enumerate(blocks):
        p, mb, ld = _block(b, f"blocks[{k}]")
        if b.shape[0] != n or mb != m or (ldx is not None and ld != ldx):
            raise ValueError("blocks must share shape and row stride")
        ldx = ld
        ptrs.append(p.value)
    coef = np.ascontiguousarray(np.asarray(coef, dtype=np.complex128).reshape(len(blocks), m))
    cd = torch.from_numpy(coef).to(blocks[0].device)
    X = torch.empty((n, m), dtype=torch.complex128, device=blocks[0].device) if out is None else out
    xp, mx, ldo = _block(X, "out")
    if X.shape[0] != n or mx != m:
        raise ValueError("out must have the blocks' shape")
    arr = (_vp * len(ptrs))(*ptrs)
    _check(lib().bem_block_combine(arr, len(ptrs), ctypes.c_void_p(cd.data_ptr()), n, m, ldx, xp, ldo, _stream()))
    return X


class LU:
    """The library's dense LU (bem_lu_factor) of a complex128 CUDA matrix A, in place: A is
    overwritten by its factors.  solve(B) returns A^-1 B for a complex128 CUDA tensor B (n x m)."""

    def __init__(self, A):
        torch = _torch()
        ptr, n, lda = _block(A, "A")
        if A.shape[0] != n:
            raise ValueError("A must be square")
        self.A, self.n = A, n
        self.ipiv = torch.empty(n, dtype=torch.int64, device=A.device)
        self.perm = torch.empty(n, dtype=torch.int64, device=A.device)
        self._info = torch.empty(1, dtype=torch.int64, device=A.device)
        wb = lib().bem_lu_work_bytes(n, 0)
        work = torch.empty(wb, dtype=torch.uint8, device=A.device)
        _check(lib().bem_lu_factor(ptr, n, lda, ctypes.c_void_p(self.ipiv.data_ptr()),
                                   ctypes.c_void_p(self.perm.data_ptr()), ctypes.c_void_p(self._info.data_ptr()),
                                   ctypes.c_void_p(work.data_ptr()), wb, _stream()))
        self._work = work

    @property
    def info(self) -> int:
        """0, or j + 1 for the first column j without a nonzero finite pivot (synchronises)."""
        return int(self._info.item())

    def solve(self, B, out=None):
        torch = _torch()
        bp, m, ldb = _block(B, "B")
        if B.shape[0] != self.n:
            raise ValueError(f"B must have {self.n} rows")
        X = torch.empty((self.n, m), dtype=torch.complex128, device=B.device) if out is None else out
        xp, mx, ldx = _block(X, "out")
        if X.shape[0] != self.n or mx != m:
            raise ValueError("out must have the shape of B")
        wb = lib().bem_lu_work_bytes(self.n, m)
        work = torch.empty(wb, dtype=torch.uint8, device=B.device)
        _check(lib().bem_lu_solve(ctypes.c_void_p(self.A.data_ptr()), self.n, self.A.stride(0),
                                  ctypes.c_void_p(self.perm.data_ptr()), bp, ldb, xp, ldx, m,
                                  ctypes.c_void_p(work.data_ptr()), wb, _stream()))
        return X
