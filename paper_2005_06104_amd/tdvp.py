"""Thin ctypes binding of the C-ABI in include/tdvp.h (argument marshalling only).

Every numerical step runs in the HIP library ``lib/libtdvp_gfx950.so``; this
module only converts Python/NumPy/PyTorch arguments to plain pointers and
sizes.  Loading fails loudly when the library has not been built.  PyTorch
provides device memory (its caching allocator is handed to the library) and
the stream.
"""
from __future__ import annotations

import ctypes as C
import weakref
import os
import re
import sys
from typing import List, Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "lib", "libtdvp_gfx950.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "tdvp.h")

TDVP_OK, TDVP_ERR_ARG, TDVP_ERR_ALLOC, TDVP_ERR_DEVICE, TDVP_ERR_NOCONV, TDVP_ERR_NUMERIC, TDVP_ERR_STATE = range(7)
STATUS_NAMES = ["OK", "ERR_ARG", "ERR_ALLOC", "ERR_DEVICE", "ERR_NOCONV", "ERR_NUMERIC", "ERR_STATE"]
TDVP_FP64, TDVP_FP32, TDVP_BF16_FP32ACC, TDVP_BF16X3_FP32ACC = 0, 1, 2, 3
OP_N, OP_T, OP_C, OP_R = 0, 1, 2, 3
PREC = {"fp64": TDVP_FP64, "fp32": TDVP_FP32, "bf16": TDVP_BF16_FP32ACC, "bf16x3": TDVP_BF16X3_FP32ACC}


class TdvpError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES[status] if 0 <= status < 7 else status}: {msg}")
        self.status = status


class tdvp_term(C.Structure):
    _fields_ = [("site_i", C.c_int32), ("site_j", C.c_int32), ("op_i", C.c_int32), ("op_j", C.c_int32),
                ("re", C.c_double), ("im", C.c_double)]


class tdvp_expand_params(C.Structure):
    _fields_ = [("k", C.c_int), ("eps_K", C.c_double), ("eps_M", C.c_double), ("chi_max", C.c_int),
                ("prec", C.c_int), ("skip_if_full", C.c_int), ("apply_method", C.c_int), ("fit_passes", C.c_int)]


class tdvp_expand_stats(C.Structure):
    _fields_ = [("ms_krylov", C.c_double), ("ms_extend", C.c_double), ("n_added", C.c_int),
                ("max_bond", C.c_int), ("krylov_max_bond", C.c_int), ("skipped", C.c_int),
                ("discarded_K", C.c_double)]


class tdvp_sweep_params(C.Structure):
    _fields_ = [("dt_re", C.c_double), ("dt_im", C.c_double), ("eps", C.c_double), ("chi_max", C.c_int),
                ("krylov_tol", C.c_double), ("krylov_max", C.c_int), ("prec", C.c_int),
                ("normalize", C.c_int), ("strict", C.c_int)]


class tdvp_sweep_stats(C.Structure):
    _fields_ = [("ms", C.c_double), ("ms_matvec", C.c_double), ("flops_matvec", C.c_double),
                ("n_matvec", C.c_longlong), ("n_keff", C.c_longlong), ("max_lanczos", C.c_int),
                ("n_unconverged", C.c_int), ("discarded", C.c_double), ("energy", C.c_double),
                ("ms_heff_gemm", C.c_double), ("flops_heff_gemm", C.c_double), ("n_heff_gemm", C.c_longlong)]


class tdvp_observables(C.Structure):
    _fields_ = [("energy", C.c_double), ("norm", C.c_double), ("overlap_re", C.c_double),
                ("overlap_im", C.c_double), ("sz", C.POINTER(C.c_double)), ("bond_dims", C.POINTER(C.c_int))]


ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)

_lib = None


def header_functions() -> List[str]:
    """Names of the functions declared in include/tdvp.h."""
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[\w\s\*]*?\b(tdvp_\w+)\s*\(", txt, flags=re.M)
    return sorted(set(n for n in names if not n.endswith("_fn")))


def load():
    """Load the HIP library (raises if it is missing)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"HIP library not built: {LIB_PATH} (run __graft_entry__.build())")
    lib = C.CDLL(LIB_PATH)
    vp, i, d, ll = C.c_void_p, C.c_int, C.c_double, C.c_longlong
    sig = {
        "tdvp_version": (C.c_char_p, []),
        "tdvp_ctx_create": (i, [i, vp, ALLOC_FN, FREE_FN, vp, C.POINTER(vp)]),
        "tdvp_ctx_destroy": (None, [vp]),
        "tdvp_last_error": (C.c_char_p, [vp]),
        "tdvp_synchronize": (i, [vp]),
        "tdvp_create_mpo": (i, [vp, i, C.POINTER(tdvp_term), i, d, d, d, d, C.POINTER(vp), C.POINTER(i)]),
        "tdvp_mpo_to_host": (i, [vp, C.POINTER(d), C.c_size_t]),
        "tdvp_build_mpo_host": (i, [i, C.POINTER(tdvp_term), i, d, d, d, d, C.POINTER(i), C.POINTER(d), C.c_size_t]),
        "tdvp_mpo_destroy": (None, [vp]),
        "tdvp_mps_from_host": (i, [vp, i, C.POINTER(i), C.POINTER(d), C.POINTER(i), C.POINTER(vp)]),
        "tdvp_mps_charges": (i, [vp, C.POINTER(i), C.POINTER(i), C.c_size_t]),
        "tdvp_mpo_charges_host": (i, [i, C.POINTER(tdvp_term), i, d, d, d, d, C.POINTER(i), C.POINTER(i),
                                      C.c_size_t]),
        "tdvp_mps_bond_dims": (i, [vp, C.POINTER(i), C.POINTER(i), i]),
        "tdvp_mps_to_host": (i, [vp, C.POINTER(d), C.c_size_t]),
        "tdvp_mps_destroy": (None, [vp]),
        "tdvp_apply_mpo": (i, [vp, vp, vp, i, d, i, i, C.POINTER(vp), C.POINTER(d)]),
        "tdvp_expand_basis": (i, [vp, i, C.POINTER(vp), C.POINTER(vp), C.POINTER(tdvp_expand_params),
                                  C.POINTER(tdvp_expand_stats)]),
        "tdvp_sweep": (i, [vp, i, C.POINTER(vp), C.POINTER(vp), C.POINTER(tdvp_sweep_params),
                           C.POINTER(tdvp_sweep_stats)]),
        "tdvp_measure": (i, [vp, i, C.POINTER(vp), C.POINTER(vp), C.POINTER(vp), C.POINTER(tdvp_observables)]),
        "tdvp_sweep2": (i, [vp, i, C.POINTER(vp), C.POINTER(vp), C.POINTER(tdvp_sweep_params),
                            C.POINTER(tdvp_sweep_stats)]),
        "tdvp_gemm": (i, [vp, i, i, i, i, i, i, d, d, vp, ll, ll, vp, ll, ll, d, d, vp, ll, ll, i]),
        "tdvp_heff_apply": (i, [vp, i, i, i, i, i, C.POINTER(d), vp, vp, vp, vp, vp]),
        "tdvp_keff_apply": (i, [vp, i, i, i, i, vp, vp, vp, vp, vp]),
        "tdvp_env_left": (i, [vp, i, i, i, i, i, C.POINTER(d), vp, vp, vp, vp]),
        "tdvp_env_right": (i, [vp, i, i, i, i, i, C.POINTER(d), vp, vp, vp, vp]),
        "tdvp_eigh": (i, [vp, i, i, vp, vp, C.POINTER(d)]),
        "tdvp_eigh_sectors": (i, [vp, i, vp, C.POINTER(C.c_int32), vp, C.POINTER(d), C.POINTER(C.c_int32)]),
        "tdvp_cholesky": (i, [vp, i, vp, vp, vp, C.POINTER(C.c_int)]),
        "tdvp_squeezing_xi2": (i, [i, d, d, d, d, d, d, C.POINTER(d)]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _iptr(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_int))


def terms_array(terms) -> "C.Array":
    arr = (tdvp_term * max(1, len(terms)))()
    for k, (i, j, oi, oj, cf) in enumerate(terms):
        cf = complex(cf)
        arr[k] = tdvp_term(int(i), int(j), int(oi), int(oj), cf.real, cf.imag)
    return arr


# ------------------------------------------------------------------ context
_live_contexts = weakref.WeakSet()
_atexit_registered = False


def _close_all_contexts():
    """Destroy every live context (and its MPO/MPS handles) while torch and the
    HIP runtime are still fully alive: the contexts free device memory through
    torch's caching allocator, which must not be called back during
    interpreter shutdown."""
    for c in list(_live_contexts):
        try:
            c.close()
        except Exception:
            pass


class Context:
    """tdvp_ctx bound to the current torch device and stream, allocating
    through torch's caching allocator."""

    def __init__(self, device: Optional[int] = None, use_torch_allocator: bool = True):
        import torch
        self.lib = load()
        self.device = torch.cuda.current_device() if device is None else int(device)
        self.stream = torch.cuda.current_stream(self.device)
        self._torch = torch
        if use_torch_allocator:
            dev, st = self.device, self.stream

            def _alloc(nbytes, user):
                try:
                    return torch.cuda.caching_allocator_alloc(int(nbytes), dev, st)
                except Exception:
                    return None

            def _free(ptr, user):
                torch.cuda.caching_allocator_delete(ptr)

            self._alloc = ALLOC_FN(_alloc)
            self._free = FREE_FN(_free)
        else:
            self._alloc = ALLOC_FN()
            self._free = FREE_FN()
        h = C.c_void_p()
        st = self.lib.tdvp_ctx_create(self.device, C.c_void_p(self.stream.cuda_stream), self._alloc, self._free,
                                      None, C.byref(h))
        if st != TDVP_OK:
            raise TdvpError(st, "tdvp_ctx_create failed")
        self.h = h
        # MPO / MPS handles free their device memory through this context:
        # they are destroyed before it
        self._children = weakref.WeakSet()
        # atexit handlers run last-registered first: registered after torch
        # was imported, the contexts are closed before torch's own handlers
        global _atexit_registered
        _live_contexts.add(self)
        if not _atexit_registered:
            import atexit
            atexit.register(_close_all_contexts)
            _atexit_registered = True

    def check(self, st: int, what: str):
        if st != TDVP_OK:
            raise TdvpError(st, f"{what}: {self.lib.tdvp_last_error(self.h).decode()}")

    def close(self):
        if getattr(self, "h", None):
            for child in list(getattr(self, "_children", ())):
                child._destroy()
            self.lib.tdvp_ctx_destroy(self.h)
            self.h = None

    def __del__(self, _finalizing=sys.is_finalizing):
        try:
            if _finalizing():   # torch may be gone: leave the memory to the process exit
                return
            self.close()
        except Exception:
            pass


def tdvp_ctx_create(device: Optional[int] = None) -> Context:
    return Context(device)


def tdvp_version() -> str:
    return load().tdvp_version().decode()


def tdvp_synchronize(ctx: Context):
    ctx.check(ctx.lib.tdvp_synchronize(ctx.h), "tdvp_synchronize")


# ---------------------------------------------------------------------- MPO
class MPO:
    def __init__(self, ctx: Context, h, dims):
        self.ctx, self.h, self.dims = ctx, h, list(dims)
        ctx._children.add(self)

    @property
    def n_sites(self):
        return len(self.dims) - 1

    def to_host(self) -> List[np.ndarray]:
        n = sum(self.dims[i] * self.dims[i + 1] * 4 for i in range(self.n_sites))
        buf = np.zeros(2 * n, dtype=np.float64)
        self.ctx.check(self.ctx.lib.tdvp_mpo_to_host(self.h, _dptr(buf), buf.size), "tdvp_mpo_to_host")
        z = buf.view(np.complex128)
        out, off = [], 0
        for i in range(self.n_sites):
            sz = self.dims[i] * self.dims[i + 1] * 4
            out.append(z[off:off + sz].reshape(self.dims[i], self.dims[i + 1], 2, 2).copy())
            off += sz
        return out

    def _destroy(self):
        if self.h and self.ctx.h:
            self.ctx.lib.tdvp_mpo_destroy(self.h)
        self.h = None

    def __del__(self, _finalizing=sys.is_finalizing):
        try:
            if _finalizing():
                return
            self._destroy()
        except Exception:
            pass


def tdvp_create_mpo(ctx: Context, n_sites: int, terms, c0: complex = 0.0, c1: complex = 1.0) -> MPO:
    arr = terms_array(terms)
    dims = np.zeros(n_sites + 1, dtype=np.int32)
    h = C.c_void_p()
    c0, c1 = complex(c0), complex(c1)
    ctx.check(ctx.lib.tdvp_create_mpo(ctx.h, n_sites, arr, len(terms), c0.real, c0.imag, c1.real, c1.imag,
                                      C.byref(h), _iptr(dims)), "tdvp_create_mpo")
    return MPO(ctx, h, dims)


def tdvp_build_mpo_host(n_sites: int, terms, c0: complex = 0.0, c1: complex = 1.0) -> List[np.ndarray]:
    """Host-only MPO construction (no device needed)."""
    lib = load()
    arr = terms_array(terms)
    dims = np.zeros(n_sites + 1, dtype=np.int32)
    c0, c1 = complex(c0), complex(c1)
    st = lib.tdvp_build_mpo_host(n_sites, arr, len(terms), c0.real, c0.imag, c1.real, c1.imag, _iptr(dims),
                                 None, 0)
    if st != TDVP_OK:
        raise TdvpError(st, "tdvp_build_mpo_host")
    n = sum(int(dims[i]) * int(dims[i + 1]) * 4 for i in range(n_sites))
    buf = np.zeros(2 * n, dtype=np.float64)
    st = lib.tdvp_build_mpo_host(n_sites, arr, len(terms), c0.real, c0.imag, c1.real, c1.imag, _iptr(dims),
                                 _dptr(buf), buf.size)
    if st != TDVP_OK:
        raise TdvpError(st, "tdvp_build_mpo_host")
    z = buf.view(np.complex128)
    out, off = [], 0
    for i in range(n_sites):
        sz = int(dims[i] * dims[i + 1] * 4)
        out.append(z[off:off + sz].reshape(int(dims[i]), int(dims[i + 1]), 2, 2).copy())
        off += sz
    return out


# ---------------------------------------------------------------------- MPS
class MPS:
    def __init__(self, ctx: Context, h, n_sites: int):
        self.ctx, self.h, self.n_sites = ctx, h, n_sites
        ctx._children.add(self)

    def bond_dims(self) -> List[int]:
        dims = np.zeros(self.n_sites + 1, dtype=np.int32)
        n = C.c_int()
        self.ctx.check(self.ctx.lib.tdvp_mps_bond_dims(self.h, C.byref(n), _iptr(dims), dims.size),
                       "tdvp_mps_bond_dims")
        return [int(x) for x in dims]

    def to_host(self) -> List[np.ndarray]:
        return tdvp_mps_to_host(self)

    def _destroy(self):
        if self.h and self.ctx.h:
            self.ctx.lib.tdvp_mps_destroy(self.h)
        self.h = None

    def __del__(self, _finalizing=sys.is_finalizing):
        try:
            if _finalizing():
                return
            self._destroy()
        except Exception:
            pass


def tdvp_mps_from_host(ctx: Context, tensors: Sequence[np.ndarray], charges=None) -> MPS:
    """charges: None, or one integer array per bond (n_sites + 1), ascending."""
    N = len(tensors)
    dims = np.array([tensors[0].shape[0]] + [t.shape[2] for t in tensors], dtype=np.int32)
    flat = np.concatenate([np.ascontiguousarray(t, dtype=np.complex128).ravel() for t in tensors])
    buf = flat.view(np.float64)
    qp = None
    if charges is not None:
        q = np.concatenate([np.asarray(c, dtype=np.int32).ravel() for c in charges]).astype(np.int32)
        if len(charges) != N + 1 or q.size != int(dims.sum()):
            raise ValueError("one charge per bond index needed")
        qp = _iptr(q)
    h = C.c_void_p()
    ctx.check(ctx.lib.tdvp_mps_from_host(ctx.h, N, _iptr(dims), _dptr(buf), qp, C.byref(h)), "tdvp_mps_from_host")
    return MPS(ctx, h, N)


def tdvp_mps_charges(mps: MPS):
    """The bond charges (list of n_sites + 1 arrays) or None for a state without them."""
    has = C.c_int()
    mps.ctx.check(mps.ctx.lib.tdvp_mps_charges(mps.h, C.byref(has), None, 0), "tdvp_mps_charges")
    if not has.value:
        return None
    dims = mps.bond_dims()
    q = np.zeros(sum(dims), dtype=np.int32)
    mps.ctx.check(mps.ctx.lib.tdvp_mps_charges(mps.h, C.byref(has), _iptr(q), q.size), "tdvp_mps_charges")
    out, off = [], 0
    for m in dims:
        out.append(q[off:off + m].copy())
        off += m
    return out


def tdvp_mpo_charges_host(n_sites: int, terms, c0: complex = 0.0, c1: complex = 1.0):
    """Channel charges of the MPO of c0 + c1 H (list per bond), or None when it does not conserve S^z."""
    lib = load()
    arr = terms_array(terms)
    c0, c1 = complex(c0), complex(c1)
    dims = np.zeros(n_sites + 1, dtype=np.int32)
    st = lib.tdvp_build_mpo_host(n_sites, arr, len(terms), c0.real, c0.imag, c1.real, c1.imag, _iptr(dims), None, 0)
    if st != TDVP_OK:
        raise TdvpError(st, "tdvp_build_mpo_host")
    cons = C.c_int()
    q = np.zeros(int(dims.sum()), dtype=np.int32)
    st = lib.tdvp_mpo_charges_host(n_sites, arr, len(terms), c0.real, c0.imag, c1.real, c1.imag, C.byref(cons),
                                   _iptr(q), q.size)
    if st != TDVP_OK:
        raise TdvpError(st, "tdvp_mpo_charges_host")
    if not cons.value:
        return None
    out, off = [], 0
    for m in dims:
        out.append(q[off:off + m].copy())
        off += m
    return out


def tdvp_mps_to_host(mps: MPS) -> List[np.ndarray]:
    dims = mps.bond_dims()
    n = sum(dims[i] * 2 * dims[i + 1] for i in range(mps.n_sites))
    buf = np.zeros(2 * n, dtype=np.float64)
    mps.ctx.check(mps.ctx.lib.tdvp_mps_to_host(mps.h, _dptr(buf), buf.size), "tdvp_mps_to_host")
    z = buf.view(np.complex128)
    out, off = [], 0
    for i in range(mps.n_sites):
        sz = dims[i] * 2 * dims[i + 1]
        out.append(z[off:off + sz].reshape(dims[i], 2, dims[i + 1]).copy())
        off += sz
    return out


# ------------------------------------------------------------ GSE-TDVP1 step
def _handles(objs):
    arr = (C.c_void_p * len(objs))()
    for k, o in enumerate(objs):
        arr[k] = o.h
    return arr


APPLY = {"denmat": 0, "fit": 1}


def tdvp_apply_mpo(ctx: Context, psi: MPS, op: MPO, method: str = "fit", eps: float = 0.0,
                   chi_max: int = 1 << 30, passes: int = 3):
    """(new MPS = op|psi>, normalised and truncated; discarded weight)."""
    h = C.c_void_p()
    disc = C.c_double()
    ctx.check(ctx.lib.tdvp_apply_mpo(ctx.h, psi.h, op.h, APPLY[method], float(eps), int(chi_max), int(passes),
                                     C.byref(h), C.byref(disc)), "tdvp_apply_mpo")
    return MPS(ctx, h, psi.n_sites), disc.value


def tdvp_expand_basis(ctx: Context, psi: Sequence[MPS], op: Sequence[MPO], k: int, eps_K: float, eps_M: float,
                      chi_max: int, prec: str = "fp64", skip_if_full: bool = True, apply: str = "denmat",
                      fit_passes: int = 3) -> List[dict]:
    p = tdvp_expand_params(int(k), float(eps_K), float(eps_M), int(chi_max), PREC[prec], int(bool(skip_if_full)),
                           APPLY[apply], int(fit_passes))
    stats = (tdvp_expand_stats * len(psi))()
    ctx.check(ctx.lib.tdvp_expand_basis(ctx.h, len(psi), _handles(psi), _handles(op), C.byref(p), stats),
              "tdvp_expand_basis")
    return [{f: getattr(s, f) for f, _ in tdvp_expand_stats._fields_} for s in stats]


def tdvp_sweep(ctx: Context, psi: Sequence[MPS], H: Sequence[MPO], dt: complex, eps: float = 0.0,
               chi_max: int = 1 << 30, krylov_tol: float = 1e-12, krylov_max: int = 30, prec: str = "fp64",
               normalize: bool = False, strict: bool = False) -> List[dict]:
    dt = complex(dt)
    p = tdvp_sweep_params(dt.real, dt.imag, float(eps), int(min(chi_max, 2 ** 31 - 1)), float(krylov_tol),
                          int(krylov_max), PREC[prec], int(bool(normalize)), int(bool(strict)))
    stats = (tdvp_sweep_stats * len(psi))()
    st = ctx.lib.tdvp_sweep(ctx.h, len(psi), _handles(psi), _handles(H), C.byref(p), stats)
    out = [{f: getattr(s, f) for f, _ in tdvp_sweep_stats._fields_} for s in stats]
    if st == TDVP_ERR_NOCONV:   # strict mode: the sweep completed; the statistics travel with the error
        err = TdvpError(st, f"tdvp_sweep: {ctx.lib.tdvp_last_error(ctx.h).decode()}")
        err.stats = out
        raise err
    ctx.check(st, "tdvp_sweep")
    return out


def tdvp_sweep2(ctx: Context, psi: Sequence[MPS], H: Sequence[MPO], dt: complex, eps: float = 0.0,
                chi_max: int = 1 << 30, krylov_tol: float = 1e-12, krylov_max: int = 30, prec: str = "fp64",
                normalize: bool = False, strict: bool = False) -> List[dict]:
    """One two-site TDVP sweep (the comparison method); arguments as tdvp_sweep."""
    dt = complex(dt)
    p = tdvp_sweep_params(dt.real, dt.imag, float(eps), int(min(chi_max, 2 ** 31 - 1)), float(krylov_tol),
                          int(krylov_max), PREC[prec], int(bool(normalize)), int(bool(strict)))
    stats = (tdvp_sweep_stats * len(psi))()
    st = ctx.lib.tdvp_sweep2(ctx.h, len(psi), _handles(psi), _handles(H), C.byref(p), stats)
    out = [{f: getattr(s, f) for f, _ in tdvp_sweep_stats._fields_} for s in stats]
    if st == TDVP_ERR_NOCONV:   # strict mode: the sweep completed; the statistics travel with the error
        err = TdvpError(st, f"tdvp_sweep2: {ctx.lib.tdvp_last_error(ctx.h).decode()}")
        err.stats = out
        raise err
    ctx.check(st, "tdvp_sweep2")
    return out


def tdvp_measure(ctx: Context, psi: Sequence[MPS], H: Optional[Sequence[MPO]] = None,
                 other: Optional[Sequence[MPS]] = None) -> List[dict]:
    n = len(psi)
    obs = (tdvp_observables * n)()
    keep = []
    for j, m in enumerate(psi):
        sz = np.zeros(m.n_sites, dtype=np.float64)
        bd = np.zeros(m.n_sites + 1, dtype=np.int32)
        keep.append((sz, bd))
        obs[j].sz = _dptr(sz)
        obs[j].bond_dims = _iptr(bd)
    ctx.check(ctx.lib.tdvp_measure(ctx.h, n, _handles(psi), _handles(H) if H else None,
                                   _handles(other) if other else None, obs), "tdvp_measure")
    out = []
    for j in range(n):
        out.append({"energy": obs[j].energy, "norm": obs[j].norm,
                    "overlap": complex(obs[j].overlap_re, obs[j].overlap_im),
                    "sz": keep[j][0].copy(), "bond_dims": [int(x) for x in keep[j][1]]})
    return out


def tdvp_squeezing_xi2(n_spins: int, sx: float, syy: float, szz: float, syz_sym: float, sy: float = 0.0,
                       sz: float = 0.0) -> float:
    """Squeezing parameter of eqs. (14)-(15) from measured total-spin moments."""
    out = C.c_double()
    st = load().tdvp_squeezing_xi2(int(n_spins), float(sx), float(sy), float(sz), float(syy), float(szz),
                                   float(syz_sym), C.byref(out))
    if st != TDVP_OK:
        raise TdvpError(st, "tdvp_squeezing_xi2: bad moments")
    return out.value


# -------------------------------------------------------- kernel-level calls
def _tp(t) -> C.c_void_p:
    return C.c_void_p(t.data_ptr()) if t is not None else None


def _prec_of(t, prec: Optional[str] = None) -> int:
    """complex128 tensors run in FP64; complex64 tensors in FP32 or, when
    prec is "bf16" or "bf16x3", with BF16 matrix-core inputs."""
    import torch
    if t.dtype == torch.complex128:
        if prec not in (None, "fp64"):
            raise TypeError(f"precision {prec} needs complex64 operands")
        return TDVP_FP64
    if t.dtype == torch.complex64:
        if prec == "fp64":
            raise TypeError("precision fp64 needs complex128 operands")
        return PREC[prec or "fp32"]
    raise TypeError(f"unsupported dtype {t.dtype}")


def tdvp_gemm(ctx: Context, op_a: int, op_b: int, M: int, N: int, K: int, alpha, A, lda, stride_a, B, ldb, stride_b,
              beta, Cout, ldc, stride_c, batch: int = 1, prec: Optional[str] = None):
    alpha, beta = complex(alpha), complex(beta)
    ctx.check(ctx.lib.tdvp_gemm(ctx.h, _prec_of(A, prec), op_a, op_b, M, N, K, alpha.real, alpha.imag, _tp(A), lda,
                                stride_a, _tp(B), ldb, stride_b, beta.real, beta.imag, _tp(Cout), ldc, stride_c,
                                batch), "tdvp_gemm")


def tdvp_eigh(ctx: Context, H, rows, method: int = 0) -> np.ndarray:
    """Eigendecomposition of the Hermitian complex128 device matrix H:
    fills rows (row j = v_j^dagger) and returns the eigenvalues, descending."""
    n = H.shape[0]
    lam = np.zeros(n)
    ctx.check(ctx.lib.tdvp_eigh(ctx.h, int(method), n, _tp(H), _tp(rows), _dptr(lam)), "tdvp_eigh")
    return lam


def tdvp_eigh_sectors(ctx: Context, H, charges, rows):
    """Eigendecomposition of the complex128 device matrix H, block diagonal
    under the index charges: fills rows (row j = v_j^dagger, zero outside its
    block) and returns (eigenvalues descending, charge of each eigenvector)."""
    n = H.shape[0]
    q = np.ascontiguousarray(charges, dtype=np.int32)
    if q.shape != (n,):
        raise ValueError("one charge per index")
    lam = np.zeros(n)
    qo = np.zeros(n, dtype=np.int32)
    ctx.check(ctx.lib.tdvp_eigh_sectors(ctx.h, n, _tp(H), q.ctypes.data_as(C.POINTER(C.c_int32)), _tp(rows),
                                        _dptr(lam), qo.ctypes.data_as(C.POINTER(C.c_int32))), "tdvp_eigh_sectors")
    return lam, qo


def tdvp_cholesky(ctx: Context, G, L, Linv) -> int:
    """Cholesky factor L (lower) and L^-1 of the Hermitian positive definite
    complex128 device matrix G (n x n, n <= 512); returns the info code (0 ok,
    1 not positive definite)."""
    n = G.shape[0]
    info = C.c_int(-1)
    ctx.check(ctx.lib.tdvp_cholesky(ctx.h, n, _tp(G), _tp(L), _tp(Linv), C.byref(info)), "tdvp_cholesky")
    return int(info.value)


def _w_host(W: np.ndarray):
    Wc = np.ascontiguousarray(W, dtype=np.complex128)
    return Wc, Wc.view(np.float64).ctypes.data_as(C.POINTER(C.c_double))


def tdvp_heff_apply(ctx: Context, W: np.ndarray, L, Rt, Cin, Y, workspace=None, prec: Optional[str] = None):
    ml, wl, _ = L.shape
    wr, mr, _ = Rt.shape
    Wc, wp = _w_host(W)
    ctx.check(ctx.lib.tdvp_heff_apply(ctx.h, _prec_of(L, prec), ml, wl, wr, mr, wp, _tp(L), _tp(Rt), _tp(Cin), _tp(Y),
                                      _tp(workspace)), "tdvp_heff_apply")


def tdvp_heff_apply_u1(ctx: Context, W: np.ndarray, L, Rt, Cin, Y, ql, qr, qwl, qwr, prec: Optional[str] = None):
    """tdvp_heff_apply on charged tensors: bond charges ql (of a, a'), qr (of
    b, b'), MPO channel charges qwl, qwr; the products walk the nonzero
    blocks only."""
    ml, wl, _ = L.shape
    wr, mr, _ = Rt.shape
    Wc, wp = _w_host(W)
    arrs = [np.ascontiguousarray(x, dtype=np.int32) for x in (ql, qr, qwl, qwr)]
    if [a.shape for a in arrs] != [(ml,), (mr,), (wl,), (wr,)]:
        raise ValueError("charge arrays do not match the tensor shapes")
    ip = [a.ctypes.data_as(C.POINTER(C.c_int32)) for a in arrs]
    fn = ctx.lib.tdvp_heff_apply_u1
    fn.restype = C.c_int
    fn.argtypes = [C.c_void_p, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, C.POINTER(C.c_double)] + \
        [C.POINTER(C.c_int32)] * 4 + [C.c_void_p] * 4
    ctx.check(fn(ctx.h, _prec_of(L, prec), ml, wl, wr, mr, wp, *ip, _tp(L), _tp(Rt), _tp(Cin), _tp(Y)),
              "tdvp_heff_apply_u1")


def tdvp_heff_apply_noalloc(ctx: Context, W: np.ndarray, L, Rt, Cin, Y, prec: Optional[str] = None):
    ml, wl, _ = L.shape
    wr, mr, _ = Rt.shape
    Wc, wp = _w_host(W)
    fn = ctx.lib.tdvp_heff_apply_noalloc
    fn.restype = C.c_int
    fn.argtypes = [C.c_void_p, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, C.POINTER(C.c_double), C.c_void_p,
                   C.c_void_p, C.c_void_p, C.c_void_p]
    ctx.check(fn(ctx.h, _prec_of(L, prec), ml, wl, wr, mr, wp, _tp(L), _tp(Rt), _tp(Cin), _tp(Y)),
              "tdvp_heff_apply_noalloc")


def tdvp_keff_apply(ctx: Context, L, Rt, X, Y, workspace=None, prec: Optional[str] = None):
    ml, w, _ = L.shape
    _, mr, _ = Rt.shape
    ctx.check(ctx.lib.tdvp_keff_apply(ctx.h, _prec_of(L, prec), ml, w, mr, _tp(L), _tp(Rt), _tp(X), _tp(Y),
                                      _tp(workspace)), "tdvp_keff_apply")


def tdvp_env_left(ctx: Context, W: np.ndarray, L, A, Lout, workspace=None, prec: Optional[str] = None):
    ml, wl, _ = L.shape
    mr = A.shape[2]
    wr = W.shape[1]
    Wc, wp = _w_host(W)
    ctx.check(ctx.lib.tdvp_env_left(ctx.h, _prec_of(L, prec), ml, wl, wr, mr, wp, _tp(L), _tp(A), _tp(Lout),
                                    _tp(workspace)), "tdvp_env_left")


def tdvp_env_right(ctx: Context, W: np.ndarray, Rt, B, Rout, workspace=None, prec: Optional[str] = None):
    wr, mr, _ = Rt.shape
    ml = B.shape[0]
    wl = W.shape[0]
    Wc, wp = _w_host(W)
    ctx.check(ctx.lib.tdvp_env_right(ctx.h, _prec_of(Rt, prec), ml, wl, wr, mr, wp, _tp(Rt), _tp(B), _tp(Rout),
                                     _tp(workspace)), "tdvp_env_right")
