"""Thin ctypes binding of libacopf.so (include/acopf.h).

Argument marshalling only: every evaluation step runs in the library's HIP
kernels.  Functions keep the C names; device buffers are torch tensors
(float64, contiguous, on the net's GPU) and streams default to torch's
current stream.  If the library is missing this module raises: there is no
CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional, Sequence

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libacopf.so")

ACOPF_OK, ACOPF_EINVAL, ACOPF_ENOMEM, ACOPF_EHIP, ACOPF_EBUDGET, ACOPF_ESTATE = 0, -1, -2, -3, -4, -5
ACOPF_F, ACOPF_GRADF, ACOPF_C, ACOPF_J, ACOPF_H, ACOPF_ALL = 1, 2, 4, 8, 16, 31
ACOPF_POLAR, ACOPF_CARTESIAN = 0, 1
ACOPF_SLACK_IMBALANCE, ACOPF_SLACK_LOADLOSS = 1, 2

_i32p = C.POINTER(C.c_int32)
_i64p = C.POINTER(C.c_int64)
_f64p = C.POINTER(C.c_double)


class AcopfError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"acopf error {code}: {msg}")
        self.code = code


class acopf_net_desc(C.Structure):
    _fields_ = [("nbus", C.c_int32), ("nbranch", C.c_int32), ("ngen", C.c_int32),
                ("base_mva", C.c_double),
                ("br_from", _i32p), ("br_to", _i32p), ("br_r", _f64p), ("br_x", _f64p),
                ("br_b", _f64p), ("br_tap", _f64p), ("br_shift", _f64p), ("br_rate", _f64p),
                ("bus_pd", _f64p), ("bus_qd", _f64p), ("bus_gs", _f64p), ("bus_bs", _f64p),
                ("gen_bus", _i32p), ("gen_c2", _f64p), ("gen_c1", _f64p), ("gen_c0", _f64p)]


class acopf_dims(C.Structure):
    _fields_ = [("n", C.c_int64), ("m", C.c_int64), ("m_eq", C.c_int64), ("nnz_jac", C.c_int64),
                ("nnz_hess", C.c_int64), ("nbus", C.c_int32), ("nbranch", C.c_int32),
                ("ngen", C.c_int32), ("outage", C.c_int32)]


class acopf_net_opts(C.Structure):
    _fields_ = [("form", C.c_int32), ("slacks", C.c_uint32), ("imb_c2", C.c_double),
                ("imb_c1", C.c_double), ("loss_c2", C.c_double), ("loss_c1", C.c_double)]


def net_opts(form: int = ACOPF_POLAR, slacks: int = 0, imb_cost=(0.0, 0.0),
             loss_cost=(0.0, 0.0)) -> acopf_net_opts:
    """acopf_net_opts from Python values; costs are (c2, c1) per MW."""
    return acopf_net_opts(int(form), int(slacks), float(imb_cost[0]), float(imb_cost[1]),
                          float(loss_cost[0]), float(loss_cost[1]))


class acopf_sched(C.Structure):
    _fields_ = [("tile_be", C.c_int32), ("grid_mult", C.c_int32), ("xcd_group", C.c_int32),
                ("no_graph", C.c_int32)]


_lib = None

# name -> (restype, argtypes)
_SIGS = {
    "acopf_last_error": (C.c_char_p, []),
    "acopf_version": (C.c_int, []),
    "acopf_net_create": (C.c_int, [C.POINTER(acopf_net_desc), C.POINTER(C.c_void_p)]),
    "acopf_net_create_form": (C.c_int, [C.POINTER(acopf_net_desc), C.c_int32,
                                        C.POINTER(C.c_void_p)]),
    "acopf_net_form": (C.c_int, [C.c_void_p, _i32p]),
    "acopf_net_create_opts": (C.c_int, [C.POINTER(acopf_net_desc), C.POINTER(acopf_net_opts),
                                        C.POINTER(C.c_void_p)]),
    "acopf_pattern_host_opts": (C.c_int, [C.POINTER(acopf_net_desc), C.POINTER(acopf_net_opts),
                                          C.c_int32, C.POINTER(acopf_dims), _i32p, _i32p, _i32p,
                                          _i32p]),
    "acopf_net_create_outage": (C.c_int, [C.c_void_p, C.c_int32, C.POINTER(C.c_void_p)]),
    "acopf_net_destroy": (C.c_int, [C.c_void_p]),
    "acopf_dims_get": (C.c_int, [C.c_void_p, C.POINTER(acopf_dims)]),
    "acopf_pattern": (C.c_int, [C.c_void_p, _i32p, _i32p, _i32p, _i32p]),
    "acopf_pattern_host": (C.c_int, [C.POINTER(acopf_net_desc), C.c_int32, C.POINTER(acopf_dims),
                                     _i32p, _i32p, _i32p, _i32p]),
    "acopf_flow_limits": (C.c_int, [C.c_void_p, _f64p]),
    "acopf_flow_limits_host": (C.c_int, [C.POINTER(acopf_net_desc), C.c_int32, _f64p]),
    "acopf_pattern_host_form": (C.c_int, [C.POINTER(acopf_net_desc), C.c_int32, C.c_int32,
                                          C.POINTER(acopf_dims), _i32p, _i32p, _i32p, _i32p]),
    "acopf_eval_f_g": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                 C.c_void_p]),
    "acopf_eval_jac": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "acopf_eval_hess": (C.c_int, [C.c_void_p, C.c_void_p, C.c_double, C.c_void_p, C.c_void_p,
                                  C.c_void_p]),
    "acopf_vjp": (C.c_int, [C.c_void_p, C.c_void_p, C.c_double, C.c_void_p, C.c_void_p,
                            C.c_void_p]),
    "acopf_hvp": (C.c_int, [C.c_void_p, C.c_void_p, C.c_double, C.c_void_p, C.c_void_p, C.c_void_p,
                            C.c_void_p]),
    "acopf_jvp": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "acopf_batch_hvp": (C.c_int, [C.c_void_p] + [C.c_void_p] * 5 + [C.c_void_p]),
    "acopf_batch_jvp": (C.c_int, [C.c_void_p] + [C.c_void_p] * 3 + [C.c_void_p]),
    "acopf_eval_all": (C.c_int, [C.c_void_p, C.c_void_p, C.c_double, C.c_void_p, C.c_void_p,
                                 C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_uint,
                                 C.c_void_p]),
    "acopf_batch_create": (C.c_int, [C.POINTER(C.c_void_p), C.c_int32, C.POINTER(acopf_sched),
                                     C.POINTER(C.c_void_p)]),
    "acopf_batch_destroy": (C.c_int, [C.c_void_p]),
    "acopf_batch_offsets": (C.c_int, [C.c_void_p, _i64p, _i64p, _i64p, _i64p]),
    "acopf_batch_eval": (C.c_int, [C.c_void_p] + [C.c_void_p] * 8 + [C.c_uint, C.c_void_p]),
    "acopf_batch_eval_noalloc": (C.c_int, [C.c_void_p] + [C.c_void_p] * 8
                                 + [C.c_uint, C.c_void_p]),
    "acopf_batch_vjp": (C.c_int, [C.c_void_p] + [C.c_void_p] * 4 + [C.c_void_p]),
    "acopf_batch_xdot": (C.c_int, [C.c_void_p] * 5),
    "acopf_batch_eval_range": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32] + [C.c_void_p] * 8
                               + [C.c_uint, C.c_void_p]),
    "acopf_batch_serve_window": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32, C.c_void_p]
                                 + [C.c_double] * 4 + [C.c_void_p] * 9),
    "acopf_batch_draw_iterates": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32, C.c_void_p]
                                  + [C.c_double] * 4 + [C.c_void_p, C.c_void_p, C.c_void_p]),
    "acopf_couple_create": (C.c_int, [C.c_void_p, _i32p, _i32p, C.c_int32, C.POINTER(C.c_void_p)]),
    "acopf_couple_destroy": (C.c_int, [C.c_void_p]),
    "acopf_couple_dims": (C.c_int, [C.c_void_p, _i64p, _i64p]),
    "acopf_couple_pattern": (C.c_int, [C.c_void_p, _i64p, _i64p]),
    "acopf_couple_eval": (C.c_int, [C.c_void_p] * 5),
    "acopf_couple_vjp": (C.c_int, [C.c_void_p] * 4),
    "acopf_couple_jvp": (C.c_int, [C.c_void_p] * 4),
}


def lib():
    """Load libacopf.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_2203_10587_amd.build` (no CPU fallback exists)")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _check(rc):
    if rc != ACOPF_OK:
        raise AcopfError(rc, lib().acopf_last_error().decode())


# ---------------------------------------------------------------------------
# argument marshalling


class _Desc:
    """acopf_net_desc over contiguous copies of a grid's arrays (kept alive)."""

    def __init__(self, g):
        i32 = lambda a: np.ascontiguousarray(a, dtype=np.int32)
        f64 = lambda a: np.ascontiguousarray(a, dtype=np.float64)
        self.arrs = dict(
            br_from=i32(g.br_from), br_to=i32(g.br_to), br_r=f64(g.br_r), br_x=f64(g.br_x),
            br_b=f64(g.br_b), br_tap=f64(g.br_tap), br_shift=f64(g.br_shift),
            br_rate=f64(g.br_rate),
            bus_pd=f64(g.bus_pd), bus_qd=f64(g.bus_qd), bus_gs=f64(g.bus_gs), bus_bs=f64(g.bus_bs),
            gen_bus=i32(g.gen_bus), gen_c2=f64(g.gen_c2), gen_c1=f64(g.gen_c1),
            gen_c0=f64(g.gen_c0))
        d = acopf_net_desc()
        d.nbus = int(g.nbus)
        d.nbranch = len(self.arrs["br_from"])
        d.ngen = len(self.arrs["gen_bus"])
        d.base_mva = float(getattr(g, "base_mva", 100.0))
        for k, a in self.arrs.items():
            setattr(d, k, a.ctypes.data_as(_i32p if a.dtype == np.int32 else _f64p))
        self.desc = d


def _ptr(t, n: Optional[int] = None, name: str = "buffer"):
    """Device pointer of a float64 CUDA tensor (None -> NULL), size-checked."""
    if t is None:
        return None
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != torch.float64:
        raise TypeError(f"{name}: expected a float64 CUDA tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name}: tensor must be contiguous")
    if n is not None and t.numel() != n:
        raise ValueError(f"{name}: expected {n} elements, got {t.numel()}")
    return C.c_void_p(t.data_ptr())


def _stream(stream):
    if stream is None:
        import torch
        return C.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return C.c_void_p(stream)
    return C.c_void_p(stream.cuda_stream)


class Net:
    """Owner of an acopf_net handle."""

    def __init__(self, handle, dims: acopf_dims, parent: Optional["Net"] = None):
        self.handle = handle
        self.dims = dims
        self.parent = parent
        self.children = 0

    @property
    def n(self):
        return int(self.dims.n)

    @property
    def m(self):
        return int(self.dims.m)

    @property
    def nnz_jac(self):
        return int(self.dims.nnz_jac)

    @property
    def nnz_hess(self):
        return int(self.dims.nnz_hess)

    def close(self):
        b = self.__dict__.pop("_vjp_batch", None)
        if b is not None:
            b.close()
        if self.handle:
            _check(lib().acopf_net_destroy(self.handle))
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _dims(handle) -> acopf_dims:
    d = acopf_dims()
    _check(lib().acopf_dims_get(handle, C.byref(d)))
    return d


def acopf_net_create(grid) -> Net:
    d = _Desc(grid)
    h = C.c_void_p()
    _check(lib().acopf_net_create(C.byref(d.desc), C.byref(h)))
    return Net(h, _dims(h))


def acopf_net_create_form(grid, form: int) -> Net:
    """A net in the representation `form` (ACOPF_POLAR or ACOPF_CARTESIAN)."""
    d = _Desc(grid)
    h = C.c_void_p()
    _check(lib().acopf_net_create_form(C.byref(d.desc), int(form), C.byref(h)))
    return Net(h, _dims(h))


def acopf_net_create_opts(grid, opts: Optional[acopf_net_opts] = None) -> Net:
    """A net with options (representation, slack blocks and their penalties);
    None gives the polar model without slacks."""
    d = _Desc(grid)
    h = C.c_void_p()
    _check(lib().acopf_net_create_opts(C.byref(d.desc), C.byref(opts) if opts is not None else None,
                                       C.byref(h)))
    return Net(h, _dims(h))


def acopf_net_form(net: Net) -> int:
    out = C.c_int32()
    _check(lib().acopf_net_form(net.handle, C.byref(out)))
    return int(out.value)


def acopf_net_create_outage(base: Net, branch: int) -> Net:
    h = C.c_void_p()
    _check(lib().acopf_net_create_outage(base.handle, int(branch), C.byref(h)))
    return Net(h, _dims(h), parent=base)


def acopf_net_destroy(net: Net):
    net.close()


def acopf_pattern(net: Net):
    d = net.dims
    jp = np.empty(d.m + 1, np.int32)
    jc = np.empty(d.nnz_jac, np.int32)
    hp = np.empty(d.n + 1, np.int32)
    hc = np.empty(d.nnz_hess, np.int32)
    _check(lib().acopf_pattern(net.handle, jp.ctypes.data_as(_i32p), jc.ctypes.data_as(_i32p),
                               hp.ctypes.data_as(_i32p), hc.ctypes.data_as(_i32p)))
    return jp, jc, hp, hc


def acopf_flow_limits(net: Net) -> np.ndarray:
    """h+ of the net's flow rows (host float64 array of 2 live branches)."""
    out = np.empty(2 * int(net.dims.nbranch), np.float64)
    _check(lib().acopf_flow_limits(net.handle, out.ctypes.data_as(_f64p)))
    return out


def acopf_flow_limits_host(grid, outage: int = -1) -> np.ndarray:
    d = _Desc(grid)
    live = len(d.arrs["br_from"]) - (1 if outage >= 0 else 0)
    out = np.empty(2 * live, np.float64)
    _check(lib().acopf_flow_limits_host(C.byref(d.desc), int(outage), out.ctypes.data_as(_f64p)))
    return out


def acopf_pattern_host(grid, outage: int = -1):
    return acopf_pattern_host_form(grid, ACOPF_POLAR, outage)


def acopf_pattern_host_opts(grid, opts: Optional[acopf_net_opts] = None, outage: int = -1):
    d = _Desc(grid)
    o = C.byref(opts) if opts is not None else None
    dims = acopf_dims()
    _check(lib().acopf_pattern_host_opts(C.byref(d.desc), o, int(outage), C.byref(dims),
                                         None, None, None, None))
    jp = np.empty(dims.m + 1, np.int32)
    jc = np.empty(dims.nnz_jac, np.int32)
    hp = np.empty(dims.n + 1, np.int32)
    hc = np.empty(dims.nnz_hess, np.int32)
    _check(lib().acopf_pattern_host_opts(C.byref(d.desc), o, int(outage), None,
                                         jp.ctypes.data_as(_i32p), jc.ctypes.data_as(_i32p),
                                         hp.ctypes.data_as(_i32p), hc.ctypes.data_as(_i32p)))
    return dims, jp, jc, hp, hc


def acopf_pattern_host_form(grid, form: int, outage: int = -1):
    d = _Desc(grid)
    dims = acopf_dims()
    _check(lib().acopf_pattern_host_form(C.byref(d.desc), int(form), int(outage), C.byref(dims),
                                         None, None, None, None))
    jp = np.empty(dims.m + 1, np.int32)
    jc = np.empty(dims.nnz_jac, np.int32)
    hp = np.empty(dims.n + 1, np.int32)
    hc = np.empty(dims.nnz_hess, np.int32)
    _check(lib().acopf_pattern_host_form(C.byref(d.desc), int(form), int(outage), None,
                                         jp.ctypes.data_as(_i32p), jc.ctypes.data_as(_i32p),
                                         hp.ctypes.data_as(_i32p), hc.ctypes.data_as(_i32p)))
    return dims, jp, jc, hp, hc


def acopf_eval_f_g(net: Net, x, f=None, grad_f=None, c=None, stream=None):
    _check(lib().acopf_eval_f_g(net.handle, _ptr(x, net.n, "x"), _ptr(f, 1, "f"),
                                _ptr(grad_f, net.n, "grad_f"), _ptr(c, net.m, "c"),
                                _stream(stream)))


def acopf_eval_jac(net: Net, x, jac_val, stream=None):
    _check(lib().acopf_eval_jac(net.handle, _ptr(x, net.n, "x"),
                                _ptr(jac_val, net.nnz_jac, "jac_val"), _stream(stream)))


def acopf_eval_hess(net: Net, x, sigma: float, lam, hess_val, stream=None):
    _check(lib().acopf_eval_hess(net.handle, _ptr(x, net.n, "x"), float(sigma),
                                 _ptr(lam, net.m, "lambda"),
                                 _ptr(hess_val, net.nnz_hess, "hess_val"), _stream(stream)))


def acopf_vjp(net: Net, x, w_f: float, w_c, u, stream=None):
    _check(lib().acopf_vjp(net.handle, _ptr(x, net.n, "x"), float(w_f), _ptr(w_c, net.m, "w_c"),
                           _ptr(u, net.n, "u"), _stream(stream)))


def acopf_hvp(net: Net, x, sigma: float, lam, d, out, stream=None):
    _check(lib().acopf_hvp(net.handle, _ptr(x, net.n, "x"), float(sigma), _ptr(lam, net.m, "lambda"),
                           _ptr(d, net.n, "d"), _ptr(out, net.n, "out"), _stream(stream)))


def acopf_jvp(net: Net, x, d, out, stream=None):
    _check(lib().acopf_jvp(net.handle, _ptr(x, net.n, "x"), _ptr(d, net.n, "d"),
                           _ptr(out, net.m, "out"), _stream(stream)))


def acopf_eval_all(net: Net, x, sigma: float, lam, f, grad_f, c, jac_val, hess_val,
                   what: int = ACOPF_ALL, stream=None):
    _check(lib().acopf_eval_all(
        net.handle, _ptr(x, net.n, "x"), float(sigma), _ptr(lam, net.m, "lambda"),
        _ptr(f, 1, "f"), _ptr(grad_f, net.n, "grad_f"), _ptr(c, net.m, "c"),
        _ptr(jac_val, net.nnz_jac, "jac_val"), _ptr(hess_val, net.nnz_hess, "hess_val"),
        C.c_uint(what), _stream(stream)))


# ---------------------------------------------------------------------------
# batches


class Batch:
    """Owner of an acopf_batch handle plus its offsets (numpy int64, count+1)."""

    def __init__(self, handle, nets: Sequence[Net]):
        self.handle = handle
        self.nets = list(nets)
        k = len(nets)
        self.x_off = np.empty(k + 1, np.int64)
        self.c_off = np.empty(k + 1, np.int64)
        self.j_off = np.empty(k + 1, np.int64)
        self.h_off = np.empty(k + 1, np.int64)
        _check(lib().acopf_batch_offsets(handle, self.x_off.ctypes.data_as(_i64p),
                                         self.c_off.ctypes.data_as(_i64p),
                                         self.j_off.ctypes.data_as(_i64p),
                                         self.h_off.ctypes.data_as(_i64p)))

    @property
    def count(self):
        return len(self.nets)

    def close(self):
        if self.handle:
            _check(lib().acopf_batch_destroy(self.handle))
            self.handle = None

    def __del__(self):
        try:
            if self.handle:
                lib().acopf_batch_destroy(self.handle)
        except Exception:
            pass


def acopf_batch_create(nets: Sequence[Net], tile_be: int = 256, grid_mult: int = 4,
                       xcd_group: int = 1, no_graph: int = 0) -> Batch:
    arr = (C.c_void_p * len(nets))(*[n.handle.value if isinstance(n.handle, C.c_void_p)
                                     else n.handle for n in nets])
    s = acopf_sched(tile_be, grid_mult, xcd_group, no_graph)
    h = C.c_void_p()
    _check(lib().acopf_batch_create(arr, len(nets), C.byref(s), C.byref(h)))
    return Batch(h, nets)


def acopf_batch_destroy(b: Batch):
    b.close()


def acopf_batch_eval(b: Batch, x, sigma, lam, f, grad_f, c, jac_val, hess_val,
                     what: int = ACOPF_ALL, stream=None):
    k = b.count
    _check(lib().acopf_batch_eval(
        b.handle, _ptr(x, int(b.x_off[-1]), "x"), _ptr(sigma, k, "sigma"),
        _ptr(lam, int(b.c_off[-1]), "lambda"), _ptr(f, k, "f"),
        _ptr(grad_f, int(b.x_off[-1]), "grad_f"), _ptr(c, int(b.c_off[-1]), "c"),
        _ptr(jac_val, int(b.j_off[-1]), "jac_val"), _ptr(hess_val, int(b.h_off[-1]), "hess_val"),
        C.c_uint(what), _stream(stream)))


def acopf_batch_eval_noalloc(b: Batch, x, sigma, lam, f, grad_f, c, jac_val, hess_val,
                             what: int = ACOPF_ALL, stream=None):
    k = b.count
    _check(lib().acopf_batch_eval_noalloc(
        b.handle, _ptr(x, int(b.x_off[-1]), "x"), _ptr(sigma, k, "sigma"),
        _ptr(lam, int(b.c_off[-1]), "lambda"), _ptr(f, k, "f"),
        _ptr(grad_f, int(b.x_off[-1]), "grad_f"), _ptr(c, int(b.c_off[-1]), "c"),
        _ptr(jac_val, int(b.j_off[-1]), "jac_val"), _ptr(hess_val, int(b.h_off[-1]), "hess_val"),
        C.c_uint(what), _stream(stream)))


def acopf_batch_xdot(b: Batch, a, v, out, stream=None):
    nx = int(b.x_off[-1])
    _check(lib().acopf_batch_xdot(b.handle, _ptr(a, nx, "a"), _ptr(v, nx, "v"),
                                  _ptr(out, b.count, "out"), _stream(stream)))


def acopf_batch_vjp(b: Batch, x, w_f, w_c, u, stream=None):
    k = b.count
    _check(lib().acopf_batch_vjp(
        b.handle, _ptr(x, int(b.x_off[-1]), "x"), _ptr(w_f, k, "w_f"),
        _ptr(w_c, int(b.c_off[-1]), "w_c"), _ptr(u, int(b.x_off[-1]), "u"), _stream(stream)))


def acopf_batch_eval_range(b: Batch, first: int, count: int, x, sigma, lam, f, grad_f, c,
                           jac_val, hess_val, what: int = ACOPF_ALL, stream=None):
    k = b.count
    _check(lib().acopf_batch_eval_range(
        b.handle, int(first), int(count), _ptr(x, int(b.x_off[-1]), "x"), _ptr(sigma, k, "sigma"),
        _ptr(lam, int(b.c_off[-1]), "lambda"), _ptr(f, k, "f"),
        _ptr(grad_f, int(b.x_off[-1]), "grad_f"), _ptr(c, int(b.c_off[-1]), "c"),
        _ptr(jac_val, int(b.j_off[-1]), "jac_val"), _ptr(hess_val, int(b.h_off[-1]), "hess_val"),
        C.c_uint(what), _stream(stream)))


def acopf_batch_draw_iterates(b: Batch, first: int, count: int, seeds, bounds, x, lam,
                              stream=None):
    """seeds: int64/uint64 CUDA tensor of b.count entries (bit pattern used);
    bounds: (pmin, pmax, qmin, qmax)."""
    import torch
    if not (isinstance(seeds, torch.Tensor) and seeds.is_cuda and seeds.dtype in (torch.int64,)
            and seeds.is_contiguous() and seeds.numel() == b.count):
        raise TypeError("seeds: expected a contiguous int64 CUDA tensor of batch-count entries")
    pmin, pmax, qmin, qmax = (float(v) for v in bounds)
    _check(lib().acopf_batch_draw_iterates(
        b.handle, int(first), int(count), C.c_void_p(seeds.data_ptr()), pmin, pmax, qmin, qmax,
        _ptr(x, int(b.x_off[-1]), "x"), _ptr(lam, int(b.c_off[-1]), "lambda"), _stream(stream)))


def acopf_batch_serve_window(b: Batch, first: int, count: int, seeds, bounds, x, lam, sigma,
                             f, grad_f, c, jac_val, hess_val, stream=None):
    """seeds: host sequence of count request seeds (bit patterns, unsigned
    64-bit); bounds: (pmin, pmax, qmin, qmax)."""
    k = b.count
    arr = (C.c_uint64 * int(count))(*[int(v) & 0xFFFFFFFFFFFFFFFF for v in seeds])
    pmin, pmax, qmin, qmax = (float(v) for v in bounds)
    _check(lib().acopf_batch_serve_window(
        b.handle, int(first), int(count), C.cast(arr, C.c_void_p), pmin, pmax, qmin, qmax,
        _ptr(x, int(b.x_off[-1]), "x"), _ptr(lam, int(b.c_off[-1]), "lambda"),
        _ptr(sigma, k, "sigma"), _ptr(f, k, "f"), _ptr(grad_f, int(b.x_off[-1]), "grad_f"),
        _ptr(c, int(b.c_off[-1]), "c"), _ptr(jac_val, int(b.j_off[-1]), "jac_val"),
        _ptr(hess_val, int(b.h_off[-1]), "hess_val"), _stream(stream)))


def acopf_batch_hvp(b: Batch, x, sigma, lam, d, out, stream=None):
    nx, nc = int(b.x_off[-1]), int(b.c_off[-1])
    _check(lib().acopf_batch_hvp(b.handle, _ptr(x, nx, "x"), _ptr(sigma, b.count, "sigma"),
                                 _ptr(lam, nc, "lambda"), _ptr(d, nx, "d"), _ptr(out, nx, "out"),
                                 _stream(stream)))


def acopf_batch_jvp(b: Batch, x, d, out, stream=None):
    nx, nc = int(b.x_off[-1]), int(b.c_off[-1])
    _check(lib().acopf_batch_jvp(b.handle, _ptr(x, nx, "x"), _ptr(d, nx, "d"), _ptr(out, nc, "out"),
                                 _stream(stream)))


class Couple:
    """Owner of an acopf_couple handle; keeps its batch alive."""

    def __init__(self, handle, batch: Batch, child, parent):
        self.handle = handle
        self.batch = batch
        self.child = np.asarray(child, np.int32)
        self.parent = np.asarray(parent, np.int32)
        rows, nnz = C.c_int64(), C.c_int64()
        _check(lib().acopf_couple_dims(handle, C.byref(rows), C.byref(nnz)))
        self.rows, self.nnz = int(rows.value), int(nnz.value)

    def close(self):
        if self.handle:
            _check(lib().acopf_couple_destroy(self.handle))
            self.handle = None

    def __del__(self):
        try:
            if self.handle:
                lib().acopf_couple_destroy(self.handle)
        except Exception:
            pass


def acopf_couple_create(batch: Batch, child: Sequence[int], parent: Sequence[int]) -> Couple:
    ch = np.ascontiguousarray(child, dtype=np.int32)
    pa = np.ascontiguousarray(parent, dtype=np.int32)
    if ch.shape != pa.shape or ch.ndim != 1:
        raise ValueError("child and parent must be 1-D arrays of equal length")
    h = C.c_void_p()
    _check(lib().acopf_couple_create(batch.handle, ch.ctypes.data_as(_i32p),
                                     pa.ctypes.data_as(_i32p), len(ch), C.byref(h)))
    return Couple(h, batch, ch, pa)


def acopf_couple_destroy(cp: Couple):
    cp.close()


def acopf_couple_pattern(cp: Couple):
    """(rowptr, col) of the coupling rows over the packed x, int64 numpy."""
    rp = np.empty(cp.rows + 1, np.int64)
    col = np.empty(max(cp.nnz, 1), np.int64)
    _check(lib().acopf_couple_pattern(cp.handle, rp.ctypes.data_as(_i64p), col.ctypes.data_as(_i64p)))
    return rp, col[:cp.nnz]


def acopf_couple_eval(cp: Couple, x, c, jac_val, stream=None):
    nx = int(cp.batch.x_off[-1])
    _check(lib().acopf_couple_eval(cp.handle, _ptr(x, nx, "x"), _ptr(c, cp.rows, "c"),
                                   _ptr(jac_val, cp.nnz, "jac_val"), _stream(stream)))


def acopf_couple_vjp(cp: Couple, w, u, stream=None):
    nx = int(cp.batch.x_off[-1])
    _check(lib().acopf_couple_vjp(cp.handle, _ptr(w, cp.rows, "w"), _ptr(u, nx, "u"),
                                  _stream(stream)))


def acopf_couple_jvp(cp: Couple, d, out, stream=None):
    nx = int(cp.batch.x_off[-1])
    _check(lib().acopf_couple_jvp(cp.handle, _ptr(d, nx, "d"), _ptr(out, cp.rows, "out"),
                                  _stream(stream)))
