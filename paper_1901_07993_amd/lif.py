"""ctypes binding of the C ABI in include/lif.h (argument marshalling only).

Every computation runs in the HIP library ``liblif.so``; if it is missing or
cannot be loaded, ``load()`` raises -- there is no other code path.

Matrices are passed as block lists: any object with attributes ``n``, ``b``,
``brow``, ``bcol``, ``vals`` (numpy arrays: host; torch CUDA tensors: device).
"""
from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, byref, c_char_p, c_double, c_int32, c_int64, c_uint64, c_void_p
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblif.so")

OK, ERR_INVALID, ERR_NOT_PD, ERR_NO_CONVERGENCE, ERR_OUT_OF_MEMORY, ERR_HIP, ERR_STATE = range(7)
FP64, MIXED_FP32, MIXED_BF16 = 0, 1, 2
STOP_PAPER, STOP_TOL = 0, 1
START_SQRT2_OVER_GERSH, START_INV_SQRT_GERSH, START_INV_SQRT_LMAX, START_GIVEN = 0, 1, 2, 3
REFINE_LOCAL, REFINE_NONLOCAL = 0, 1
PRODUCT_UPPER = 2

_STATUS_NAMES = {1: "LIF_ERR_INVALID", 2: "LIF_ERR_NOT_PD", 3: "LIF_ERR_NO_CONVERGENCE",
                 4: "LIF_ERR_OUT_OF_MEMORY", 5: "LIF_ERR_HIP", 6: "LIF_ERR_STATE"}

EXPORTED = ("lif_opts_default", "lif_create", "lif_refine", "lif_localized", "lif_rinch", "lif_get_Z", "lif_residual",
            "lif_multiply", "lif_multiply_add", "lif_multiply_noalloc", "lif_backward", "lif_destroy",
            "lif_last_error", "lif_residual_against", "lif_set_opts")


class LifError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{_STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


class Blocks(ctypes.Structure):
    _fields_ = [("n", c_int64), ("b", c_int32), ("nnzb", c_int64), ("brow", c_void_p), ("bcol", c_void_p),
                ("vals", c_void_p), ("on_device", c_int32)]


class Opts(ctypes.Structure):
    _fields_ = [("m", c_int32), ("tau", c_double), ("prec", c_int32), ("stop", c_int32), ("tol", c_double),
                ("max_iter", c_int32), ("base_rows", c_int64), ("start", c_int32), ("start_value", c_double),
                ("checkpoint", c_int32), ("mem_cap_bytes", c_uint64), ("stream", c_void_p), ("timing", c_int32),
                ("presize", c_int32), ("refinement", c_int32), ("prec_switch", c_double),
                ("sym_delta", c_int32), ("residual_panel_rows", c_int32), ("update_panel_rows", c_int32),
                ("update_prec", c_int32)]


class Info(ctypes.Structure):
    _fields_ = [("iterations_top", c_int32), ("levels", c_int32), ("iterations_total", c_int32),
                ("stagnated", c_int32), ("start_scale", c_double), ("delta_tracked", c_double),
                ("flops_leaf_gemm", c_double), ("seconds_total", c_double), ("seconds_leaf_gemm", c_double),
                ("leaf_gemm_launches", c_int64), ("products_total", c_int64), ("nnzb_Z", c_int64),
                ("n_norms", c_int32), ("norms", c_double * 64), ("iterations_redone", c_int32),
                ("cpl_tasks", c_int32), ("cpl_products", c_int32), ("iterations_reduced", c_int32),
                ("mem_peak_bytes", c_uint64), ("mem_reserved_bytes", c_uint64), ("products_compacted", c_int32),
                ("pair_panels", c_int32), ("flops_leaf_gemm_reduced", c_double),
                ("seconds_leaf_gemm_reduced", c_double), ("leaf_gemm_launches_reduced", c_int64),
                ("seconds_leaf_factorization", c_double), ("flops_leaf_factorization", c_double),
                ("seconds_symbolic", c_double), ("bytes_symbolic", c_double), ("symbolic_launches", c_int64),
                ("flops_leaf_gemm_fp32", c_double), ("seconds_leaf_gemm_fp32", c_double),
                ("leaf_gemm_launches_fp32", c_int64)]

    def as_dict(self) -> dict:
        d = {k: getattr(self, k) for k, _ in self._fields_ if k != "norms"}
        d["norms"] = [self.norms[i] for i in range(self.n_norms)]
        return d


_lib = None


def load() -> ctypes.CDLL:
    """Loads liblif.so (built by ``paper_1901_07993_amd.build``); raises if absent."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -c 'import __graft_entry__ as g; g.build()'`")
    lib = ctypes.CDLL(LIB_PATH)
    lib.lif_opts_default.argtypes = [POINTER(Opts)]
    lib.lif_create.argtypes = [POINTER(Blocks), POINTER(Opts), POINTER(c_void_p)]
    lib.lif_refine.argtypes = [c_void_p, POINTER(Blocks), POINTER(Info)]
    lib.lif_localized.argtypes = [c_void_p, POINTER(Info)]
    lib.lif_rinch.argtypes = [c_void_p, POINTER(Info)]
    lib.lif_get_Z.argtypes = [c_void_p, POINTER(c_int64), c_void_p, c_void_p, c_void_p, c_int32]
    lib.lif_residual.argtypes = [c_void_p, POINTER(c_double)]
    lib.lif_residual_against.argtypes = [c_void_p, POINTER(Blocks), POINTER(c_double)]
    lib.lif_set_opts.argtypes = [c_void_p, POINTER(Opts)]
    lib.lif_multiply.argtypes = [c_void_p, POINTER(Blocks), c_int32, POINTER(Blocks), c_int32, c_double,
                                 POINTER(c_int64), c_void_p, c_void_p, c_void_p, c_int32, POINTER(c_int64)]
    lib.lif_multiply_add.argtypes = [c_void_p, POINTER(Blocks), c_int32, POINTER(Blocks), c_int32, c_double,
                                     POINTER(Blocks), c_double, c_double, POINTER(c_int64), c_void_p, c_void_p,
                                     c_void_p, c_int32, POINTER(c_int64)]
    lib.lif_multiply_noalloc.argtypes = [POINTER(Blocks), c_int32, POINTER(Blocks), c_int32, c_double,
                                         POINTER(Blocks), c_double, c_double, c_int32, c_void_p, c_int64,
                                         POINTER(c_int64), c_void_p, c_void_p, c_void_p, POINTER(c_int64)]
    lib.lif_backward.argtypes = [c_void_p, POINTER(Blocks), POINTER(c_int64), c_void_p, c_void_p, c_void_p, c_int32]
    lib.lif_destroy.argtypes = [c_void_p]
    lib.lif_destroy.restype = None
    lib.lif_last_error.argtypes = [c_void_p]
    lib.lif_last_error.restype = c_char_p
    for name in EXPORTED:
        if name not in ("lif_destroy", "lif_last_error"):
            getattr(lib, name).restype = c_int32
    _lib = lib
    return lib


@dataclass
class HostBlocks:
    n: int
    b: int
    brow: np.ndarray
    bcol: np.ndarray
    vals: np.ndarray

    @property
    def nnzb(self) -> int:
        return int(self.brow.shape[0])

    @property
    def nb(self) -> int:
        return (self.n + self.b - 1) // self.b


@dataclass
class DeviceBlocks:
    """A block list whose arrays are torch tensors on the GPU."""
    n: int
    b: int
    brow: object
    bcol: object
    vals: object

    @property
    def nnzb(self) -> int:
        return int(self.brow.shape[0])


def _is_torch(x) -> bool:
    return type(x).__module__.startswith("torch")


def _marshal(M):
    """(Blocks struct, keep-alive list) for a block list on host or device."""
    keep = []
    if _is_torch(M.vals):
        import torch
        assert M.vals.is_cuda, "torch block lists must live on the GPU"
        brow = M.brow.to(torch.int32).contiguous()
        bcol = M.bcol.to(torch.int32).contiguous()
        vals = M.vals.to(torch.float64).contiguous()
        keep += [brow, bcol, vals]
        st = Blocks(int(M.n), int(M.b), int(brow.shape[0]), brow.data_ptr(), bcol.data_ptr(), vals.data_ptr(), 1)
    else:
        brow = np.ascontiguousarray(M.brow, dtype=np.int32)
        bcol = np.ascontiguousarray(M.bcol, dtype=np.int32)
        vals = np.ascontiguousarray(M.vals, dtype=np.float64)
        keep += [brow, bcol, vals]
        st = Blocks(int(M.n), int(M.b), int(brow.shape[0]), brow.ctypes.data, bcol.ctypes.data, vals.ctypes.data, 0)
    return st, keep


def _current_stream():
    try:
        import torch
        if torch.cuda.is_available():
            return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    except Exception:  # noqa: BLE001 - no torch GPU: the null stream
        pass
    return ctypes.c_void_p(0)


def default_opts(**kw) -> Opts:
    o = Opts()
    load().lif_opts_default(byref(o))
    for k, v in kw.items():
        if k == "stream":
            o.stream = v
        else:
            setattr(o, k, v)
    return o


class Factorization:
    """One inverse-factorization problem: S (block list) and options.

    Keyword options mirror ``lif_opts``: m, tau, prec, stop, tol, max_iter,
    base_rows, start, start_value, checkpoint, mem_cap_bytes, timing, presize,
    refinement, prec_switch, sym_delta, residual_panel_rows, update_panel_rows,
    update_prec.
    """

    def __init__(self, S, **opts):
        lib = load()
        if "stream" not in opts:
            opts["stream"] = _current_stream()
        self._opts = default_opts(**opts)
        st, keep = _marshal(S)
        h = c_void_p()
        rc = lib.lif_create(byref(st), byref(self._opts), byref(h))
        del keep
        if rc != OK:
            raise LifError(rc, lib.lif_last_error(None).decode())
        self._h = h
        self.n, self.b = int(S.n), int(S.b)

    def _check(self, rc):
        if rc != OK:
            raise LifError(rc, load().lif_last_error(self._h).decode())

    def refine(self, Z0=None) -> dict:
        info = Info()
        if Z0 is None:
            self._check(load().lif_refine(self._h, None, byref(info)))
        else:
            st, keep = _marshal(Z0)
            self._check(load().lif_refine(self._h, byref(st), byref(info)))
            del keep
        return info.as_dict()

    def localized(self) -> dict:
        info = Info()
        self._check(load().lif_localized(self._h, byref(info)))
        return info.as_dict()

    def rinch(self) -> dict:
        """Recursive inverse Cholesky (lif_rinch)."""
        info = Info()
        self._check(load().lif_rinch(self._h, byref(info)))
        return info.as_dict()

    def _out_arrays(self, k: int, on_device: bool):
        if on_device:
            import torch
            brow = torch.empty(k, dtype=torch.int32, device="cuda")
            bcol = torch.empty(k, dtype=torch.int32, device="cuda")
            vals = torch.empty((k, self.b, self.b), dtype=torch.float64, device="cuda")
            return (brow, bcol, vals), (brow.data_ptr(), bcol.data_ptr(), vals.data_ptr())
        brow = np.empty(k, np.int32)
        bcol = np.empty(k, np.int32)
        vals = np.empty((k, self.b, self.b), np.float64)
        return (brow, bcol, vals), (brow.ctypes.data, bcol.ctypes.data, vals.ctypes.data)

    def _blocks(self, arrs, on_device: bool):
        return (DeviceBlocks if on_device else HostBlocks)(self.n, self.b, *arrs)

    def get_Z(self, on_device: bool = False):
        """The factor as a block list (HostBlocks, or DeviceBlocks of torch
        tensors on the GPU with ``on_device``)."""
        lib = load()
        nnzb = c_int64(0)
        self._check(lib.lif_get_Z(self._h, byref(nnzb), None, None, None, int(on_device)))
        arrs, ptrs = self._out_arrays(nnzb.value, on_device)
        self._check(lib.lif_get_Z(self._h, byref(nnzb), *ptrs, int(on_device)))
        return self._blocks(arrs, on_device)

    def residual(self) -> float:
        out = c_double(0.0)
        self._check(load().lif_residual(self._h, byref(out)))
        return out.value

    def residual_against(self, S) -> float:
        """||I - Z^T S Z||_F of the handle's Z against another S (for example
        the matrix before the block truncation applied at creation)."""
        out = c_double(0.0)
        st, keep = _marshal(S)
        self._check(load().lif_residual_against(self._h, byref(st), byref(out)))
        del keep
        return out.value

    def set_opts(self, **opts):
        """Changes options of the handle (not tau or mem_cap_bytes): the same
        S and warm memory pool serve the next factorization."""
        o = Opts()
        ctypes.memmove(byref(o), byref(self._opts), ctypes.sizeof(Opts))
        for k, v in opts.items():
            setattr(o, k, v)
        self._check(load().lif_set_opts(self._h, byref(o)))
        self._opts = o

    def multiply(self, A, transA: bool, B, transB: bool, tau: float = 0.0, upper: bool = False,
                 alpha: float = 1.0, D=None, gamma: float = 0.0):
        """C = trunc_tau(alpha op(A) op(B) [+ gamma D]) (only its upper block
        triangle when ``upper``); returns (HostBlocks, products).  Without D
        and with alpha = 1 this is lif_multiply, otherwise lif_multiply_add."""
        transA = int(transA) | (PRODUCT_UPPER if upper else 0)
        lib = load()
        sa, ka = _marshal(A)
        sb, kb = _marshal(B)
        sd, kd = _marshal(D) if D is not None else (None, None)
        nnzb = c_int64(0)
        prods = c_int64(0)

        def call(brow, bcol, vals):
            if D is None and alpha == 1.0:
                return lib.lif_multiply(self._h, byref(sa), int(transA), byref(sb), int(transB), float(tau),
                                        byref(nnzb), brow, bcol, vals, 0, byref(prods))
            return lib.lif_multiply_add(self._h, byref(sa), int(transA), byref(sb), int(transB), float(alpha),
                                        byref(sd) if sd is not None else None, float(gamma), float(tau),
                                        byref(nnzb), brow, bcol, vals, 0, byref(prods))

        self._check(call(None, None, None))
        k = nnzb.value
        brow = np.empty(k, np.int32)
        bcol = np.empty(k, np.int32)
        vals = np.empty((k, self.b, self.b), np.float64)
        self._check(call(brow.ctypes.data, bcol.ctypes.data, vals.ctypes.data))
        del ka, kb, kd
        return HostBlocks(self.n, self.b, brow, bcol, vals), prods.value

    def backward(self, G, on_device: bool = False):
        """sym(dL/dS) on S's block pattern for L = tr(G^T Z) (needs checkpoint=1);
        HostBlocks, or DeviceBlocks with ``on_device``."""
        lib = load()
        st, keep = _marshal(G)
        nnzb = c_int64(0)
        self._check(lib.lif_backward(self._h, byref(st), byref(nnzb), None, None, None, int(on_device)))
        arrs, ptrs = self._out_arrays(nnzb.value, on_device)
        self._check(lib.lif_backward(self._h, None, byref(nnzb), *ptrs, int(on_device)))
        del keep
        return self._blocks(arrs, on_device)

    def close(self):
        if getattr(self, "_h", None):
            load().lif_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:  # noqa: BLE001
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


def multiply_noalloc(A, transA: bool, B, transB: bool, tau: float = 0.0, prec: int = FP64, alpha: float = 1.0,
                     D=None, gamma: float = 0.0, capacity: int | None = None, upper: bool = False):
    """lif_multiply_noalloc on device block lists (torch CUDA tensors): the
    product trunc_tau(alpha op(A) op(B) [+ gamma D]) with no allocation in
    the library.  The output arrays are allocated here, by the caller, with
    ``capacity`` blocks (default: every block of the n x n block grid).
    Returns (DeviceBlocks, products); raises LifError (status
    ERR_INVALID with the needed count when the capacity is short)."""
    import torch
    lib = load()
    sa, ka = _marshal(A)
    sb, kb = _marshal(B)
    sd, kd = _marshal(D) if D is not None else (None, None)
    nb = (int(A.n) + int(A.b) - 1) // int(A.b)
    cap = nb * nb if capacity is None else int(capacity)
    brow = torch.empty(max(cap, 1), dtype=torch.int32, device="cuda")
    bcol = torch.empty(max(cap, 1), dtype=torch.int32, device="cuda")
    vals = torch.empty((max(cap, 1), int(A.b), int(A.b)), dtype=torch.float64, device="cuda")
    nnzb = c_int64(0)
    prods = c_int64(0)
    trans_a = int(transA) | (PRODUCT_UPPER if upper else 0)
    rc = lib.lif_multiply_noalloc(byref(sa), trans_a, byref(sb), int(transB), float(alpha),
                                  byref(sd) if sd is not None else None, float(gamma), float(tau), int(prec),
                                  _current_stream(), cap, byref(nnzb), brow.data_ptr(), bcol.data_ptr(),
                                  vals.data_ptr(), byref(prods))
    del ka, kb, kd
    if rc != OK:
        err = LifError(rc, lib.lif_last_error(None).decode())
        err.nnzb = nnzb.value
        raise err
    k = nnzb.value
    return DeviceBlocks(int(A.n), int(A.b), brow[:k], bcol[:k], vals[:k]), prods.value


def factorize(S, method: str = "lif", **opts):
    """Z with S^{-1} = Z Z^T for a block list S: ``method`` "lif" (lif_localized),
    "irsi" (lif_refine from a scaled identity) or "rinch" (lif_rinch); opts as
    for Factorization.  Returns (Z, info): Z as DeviceBlocks when S's arrays
    are torch GPU tensors, else HostBlocks."""
    on_device = _is_torch(S.vals)
    with Factorization(S, **opts) as f:
        info = {"lif": f.localized, "irsi": f.refine, "rinch": f.rinch}[method]()
        return f.get_Z(on_device=on_device), info


def _scatter_to_pattern(brow_from, bcol_from, vals_from, brow_to, bcol_to, nb):
    """Blocks of one sorted block list placed at the positions of another
    (zeros where the second has a block the first lacks), on the GPU."""
    import torch
    key_to = brow_to.to(torch.int64) * nb + bcol_to.to(torch.int64)
    key_from = brow_from.to(torch.int64) * nb + bcol_from.to(torch.int64)
    out = torch.zeros((key_to.shape[0],) + tuple(vals_from.shape[1:]), dtype=vals_from.dtype,
                      device=vals_from.device)
    if key_from.numel():
        pos = torch.searchsorted(key_to, key_from)
        out[pos] = vals_from
    return out


try:
    import torch as _torch

    class LIFFunction(_torch.autograd.Function):
        """Z = the inverse factor of S as a differentiable torch operation.

        apply(S_vals, pattern, method="lif", opts=None) -> (Z_vals, Z_brow, Z_bcol)
          S_vals  [nnzb, b, b] float64 CUDA tensor, the blocks of S listed in
                  ``pattern`` (an object with n, b, brow, bcol; int32 CUDA
                  tensors sorted by (row, col), both (i, j) and (j, i) of the
                  symmetric pattern);
          method  "lif" or "irsi"; opts: keyword options of Factorization.
        The backward pass calls lif_backward with G = dL/dZ on Z's pattern
        and returns sym(dL/dS) on S's pattern: for a symmetric perturbation E
        of S, dL = <grad, E>.  Blocks of S dropped by the truncation at tau
        get a zero gradient.  The handle (and its per-iteration checkpoints)
        lives until the backward pass has run.
        """

        @staticmethod
        def forward(ctx, S_vals, pattern, method="lif", opts=None):
            S = DeviceBlocks(int(pattern.n), int(pattern.b), pattern.brow, pattern.bcol, S_vals.detach())
            f = Factorization(S, checkpoint=1, **(opts or {}))
            {"lif": f.localized, "irsi": f.refine}[method]()
            Z = f.get_Z(on_device=True)
            ctx.f = f
            ctx.pattern = pattern
            ctx.zpat = (Z.brow, Z.bcol)
            ctx.mark_non_differentiable(Z.brow, Z.bcol)
            return Z.vals, Z.brow, Z.bcol

        @staticmethod
        def backward(ctx, g_vals, g_brow=None, g_bcol=None):
            p = ctx.pattern
            n, b = int(p.n), int(p.b)
            nb = (n + b - 1) // b
            g = g_vals.contiguous()
            tail = n - (nb - 1) * b
            if tail < b:
                # Z's entries beyond n are constant zeros: their gradient is dropped
                g = g.clone()
                g[ctx.zpat[0] == nb - 1, tail:, :] = 0.0
                g[ctx.zpat[1] == nb - 1, :, tail:] = 0.0
            G = DeviceBlocks(n, b, ctx.zpat[0], ctx.zpat[1], g)
            dS = ctx.f.backward(G, on_device=True)
            ctx.f.close()
            grad = _scatter_to_pattern(dS.brow, dS.bcol, dS.vals, p.brow, p.bcol, nb)
            return grad, None, None, None
except ImportError:  # torch absent: the ctypes binding still works with host arrays
    pass
