"""h2x: H^2-matrix x block-of-vectors products and block CG on AMD MI355X.

Thin Python binding of the C ABI in ``include/h2x.h`` (library ``libh2x.so``
next to this file).  Every step of the computation runs in the library's HIP
kernels; this module only marshals arguments.  PyTorch provides device memory
(workspaces, inputs, outputs) and the current stream.  There is no CPU
fallback: if the library is missing, every call raises.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

__all__ = ["Plan", "H2Matrix", "Batch", "h2_matmul", "h2_matmul_noalloc", "h2_matmul_adjoint", "h2_grad", "block_cg_solve",
           "block_cg_refine", "block_cg_mixed", "batch_matmul", "batch_block_cg_solve", "library_path", "load_library", "F64", "F32",
           "BF16", "TREE_ORDER"]

F64, F32, BF16 = 0, 1, 2
_PREC = {"f64": F64, "f32": F32, "bf16": BF16, F64: F64, F32: F32, BF16: BF16}
_KERNEL = {"exp": 0, "poly": 1, "const": 2, "helmholtz": 3}
TREE_ORDER = 1

_HERE = os.path.dirname(os.path.abspath(__file__))
_lib = None


def library_path() -> str:
    return os.path.join(_HERE, "libh2x.so")


class H2xError(RuntimeError):
    pass


class _Params(C.Structure):
    _fields_ = [("kernel", C.c_int), ("ell", C.c_double), ("shift", C.c_double), ("eta", C.c_double),
                ("leaf_size", C.c_int32), ("cheb_order", C.c_int32)]


class _Stats(C.Structure):
    _fields_ = [("n", C.c_int64), ("clusters", C.c_int64), ("leaves", C.c_int64), ("n_adm", C.c_int64),
                ("n_near", C.c_int64), ("near_entries", C.c_int64), ("depth", C.c_int32), ("k", C.c_int32),
                ("bytes_operator", C.c_int64 * 3), ("bytes_near", C.c_int64), ("adm_depth", C.c_int32),
                ("split_depth", C.c_int32), ("deep_blocks", C.c_int64)]


class _CgParams(C.Structure):
    _fields_ = [("rtol", C.c_double), ("max_iter", C.c_int32), ("freeze_converged", C.c_int32),
                ("check_every", C.c_int32), ("variant", C.c_int32), ("graph", C.c_int32)]


CG_INDEPENDENT, CG_SHARED = 0, 1
_VARIANT = {"independent": CG_INDEPENDENT, "shared": CG_SHARED, CG_INDEPENDENT: CG_INDEPENDENT, CG_SHARED: CG_SHARED}


class _GmresParams(C.Structure):
    _fields_ = [("rtol", C.c_double), ("restart", C.c_int32), ("max_iter", C.c_int32),
                ("check_every", C.c_int32), ("reserved", C.c_int32)]


class _GmresInfo(C.Structure):
    _fields_ = [("iters", C.c_int32), ("cycles", C.c_int32), ("status", C.c_int32), ("reserved", C.c_int32),
                ("col_res", C.POINTER(C.c_double)), ("col_iters", C.POINTER(C.c_int32)),
                ("col_status", C.POINTER(C.c_int32))]


class _TuneInfo(C.Structure):
    _fields_ = [("nj_transfer", C.c_int32), ("nj_coupling", C.c_int32), ("np_leaf", C.c_int32),
                ("overlap", C.c_int32), ("fuse_up", C.c_int32), ("leaf_kind", C.c_int32), ("split", C.c_int32),
                ("ms_default", C.c_double), ("ms_tuned", C.c_double)]


class _CgInfo(C.Structure):
    _fields_ = [("iters", C.c_int32), ("status", C.c_int32), ("outer_iters", C.c_int32),
                ("col_relres", C.POINTER(C.c_double)),
                ("col_iters", C.POINTER(C.c_int32)), ("col_status", C.POINTER(C.c_int32)),
                ("sys_iters", C.POINTER(C.c_int32))]


def load_library():
    """Load libh2x.so (built by ``paper_2509_17257_amd.build``); raises if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    path = library_path()
    if not os.path.exists(path):
        raise H2xError(f"{path} is not built; run paper_2509_17257_amd/build.py (no CPU fallback exists)")
    lib = C.CDLL(path)
    P, I64, D, I32, SZ = C.c_void_p, C.c_int64, C.c_double, C.c_int32, C.c_size_t
    sig = {
        "h2x_plan_create": (C.c_int, [P, I64, C.POINTER(_Params), C.POINTER(P)]),
        "h2x_plan_destroy": (None, [P]),
        "h2x_plan_stats": (C.c_int, [P, C.POINTER(_Stats)]),
        "h2x_plan_perm": (C.c_int, [P, P]),
        "h2x_plan_clusters": (C.c_int, [P, P, P, P, P, P, P]),
        "h2x_plan_blocks": (C.c_int, [P, P, P, P, P]),
        "h2x_plan_merge": (C.c_int, [P, I32, C.POINTER(P)]),
        "h2x_plan_systems": (C.c_int, [P, C.POINTER(I32), P]),
        "h2x_batch_create": (C.c_int, [P, I32, C.POINTER(P)]),
        "h2x_batch_destroy": (None, [P]),
        "h2x_batch_matmul_workspace_bytes": (SZ, [P, I64]),
        "h2x_batch_matmul": (C.c_int, [P, I64, D, P, I64, D, P, I64, I32, P, SZ, P]),
        "h2x_batch_block_cg_workspace_bytes": (SZ, [P, I64]),
        "h2x_batch_block_cg": (C.c_int, [P, C.POINTER(_CgParams), I64, P, I64, P, I64, P, SZ, C.POINTER(_CgInfo),
                                         P]),
        "h2x_mat_workspace_bytes": (SZ, [P, C.c_int]),
        "h2x_mat_create": (C.c_int, [P, C.c_int, P, SZ, P, C.POINTER(P)]),
        "h2x_mat_destroy": (None, [P]),
        "h2x_matmul_workspace_bytes": (SZ, [P, I64]),
        "h2x_matmul": (C.c_int, [P, I64, D, P, I64, D, P, I64, I32, P, SZ, P]),
        "h2x_matmul_timed": (C.c_int, [P, I64, D, P, I64, D, P, I64, I32, P, SZ, P, P]),
        "h2x_matmul_noalloc": (C.c_int, [P, I64, D, P, I64, D, P, I64, I32, P]),
        "h2x_timer_create": (C.c_int, [I32, C.POINTER(P)]),
        "h2x_timer_destroy": (None, [P]),
        "h2x_matmul_marked": (C.c_int, [P, I64, D, P, I64, D, P, I64, I32, P, SZ, P, P, I32]),
        "h2x_timer_read": (C.c_int, [P, I32, P]),
        "h2x_block_cg_workspace_bytes": (SZ, [P, I64]),
        "h2x_block_cg": (C.c_int, [P, C.POINTER(_CgParams), I64, P, I64, P, I64, P, SZ, C.POINTER(_CgInfo), P]),
        "h2x_block_cg_refine_workspace_bytes": (SZ, [P, P, I64]),
        "h2x_block_cg_refine": (C.c_int, [P, P, C.POINTER(_CgParams), D, I32, I64, P, I64, P, I64, P, SZ,
                                          C.POINTER(_CgInfo), P]),
        "h2x_matmul_adjoint_workspace_bytes": (SZ, [P, I64]),
        "h2x_matmul_adjoint": (C.c_int, [P, I64, D, P, I64, D, P, I64, P, SZ, P]),
        "h2x_grad_workspace_bytes": (SZ, [P, I64]),
        "h2x_grad": (C.c_int, [P, I64, P, I64, P, I64, P, P, P, D, I32, P, SZ, P]),
        "h2x_mat_set_ell": (C.c_int, [P, D, P]),
        "h2x_mat_coupling": (C.c_int, [P, P, P]),
        "h2x_mat_set_coupling": (C.c_int, [P, P, P]),
        "h2x_block_cg_mixed_workspace_bytes": (SZ, [P, P, I64]),
        "h2x_block_cg_mixed": (C.c_int, [P, P, C.POINTER(_CgParams), D, I64, P, I64, P, I64, P, SZ,
                                         C.POINTER(_CgInfo), P]),
        "h2x_block_gmres_workspace_bytes": (SZ, [P, I64, I32]),
        "h2x_block_gmres": (C.c_int, [P, C.POINTER(_GmresParams), I64, P, I64, P, I64, P, SZ,
                                      C.POINTER(_GmresInfo), P]),
        "h2x_solve_workspace_bytes": (SZ, [P, I32, I32, I64, I32]),
        "h2x_choose_chunk": (C.c_int, [P, I32, I32, I32, I64, SZ, I32, P, P, P]),
        "h2x_product_times_workspace_bytes": (SZ, [P, I32, P]),
        "h2x_product_times": (C.c_int, [P, I32, P, I32, P, SZ, P, P]),
        "h2x_block_cg_chunked": (C.c_int, [P, C.POINTER(_CgParams), I64, I64, P, I64, P, I64, P, SZ,
                                           C.POINTER(_CgInfo), P]),
        "h2x_block_gmres_chunked": (C.c_int, [P, C.POINTER(_GmresParams), I64, I64, P, I64, P, I64, P, SZ,
                                              C.POINTER(_GmresInfo), P]),
        "h2x_mat_autotune_workspace_bytes": (SZ, [P, I64]),
        "h2x_mat_autotune": (C.c_int, [P, I64, P, SZ, P, C.POINTER(_TuneInfo)]),
        "h2x_mat_set_tune": (C.c_int, [P, I64, C.POINTER(_TuneInfo)]),
        "h2x_mat_get_tune": (C.c_int, [P, I64, C.POINTER(_TuneInfo)]),
        "h2x_last_error": (C.c_char_p, []),
        "h2x_version": (C.c_char_p, []),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def _check(status: int, what: str):
    if status != 0:
        msg = load_library().h2x_last_error().decode()
        raise H2xError(f"{what} failed with status {status}: {msg}")


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


class Plan:
    """Host topology: cluster tree, block tree, lists (h2x_plan_create)."""

    def __init__(self, points, *, kernel="exp", ell=0.5, shift=1.0, eta=1.0, leaf=32, p=3, _handle=None,
                 _parts=None):
        lib = load_library()
        if _handle is None:
            pts = np.ascontiguousarray(points, dtype=np.float64)
            if pts.ndim != 2 or pts.shape[1] != 3:
                raise ValueError("points must be n x 3")
            prm = _Params(_KERNEL[kernel] if isinstance(kernel, str) else int(kernel), float(ell), float(shift),
                          float(eta), int(leaf), int(p))
            h = C.c_void_p()
            _check(lib.h2x_plan_create(_ptr(pts), pts.shape[0], C.byref(prm), C.byref(h)), "h2x_plan_create")
        else:
            h = _handle
        self._h = h
        self._parts = _parts
        self.params = dict(kernel=kernel, ell=ell, shift=shift, eta=eta, leaf=leaf, p=p)
        st = _Stats()
        _check(lib.h2x_plan_stats(h, C.byref(st)), "h2x_plan_stats")
        self.n, self.C, self.leaves = st.n, st.clusters, st.leaves
        self.n_adm, self.n_near, self.near_entries = st.n_adm, st.n_near, st.near_entries
        self.depth, self.k = st.depth, st.k
        self.bytes_operator = list(st.bytes_operator)
        self.bytes_near = st.bytes_near
        self.adm_depth, self.split_depth, self.deep_blocks = st.adm_depth, st.split_depth, st.deep_blocks

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.h2x_plan_destroy(self._h)
            self._h = None

    @classmethod
    def merge(cls, plans):
        """Block-diagonal union of plans with one Chebyshev order (h2x_plan_merge)."""
        plans = list(plans)
        arr = (C.c_void_p * len(plans))(*[p._h for p in plans])
        h = C.c_void_p()
        _check(load_library().h2x_plan_merge(arr, len(plans), C.byref(h)), "h2x_plan_merge")
        p0 = plans[0].params
        return cls(None, _handle=h, _parts=plans, **dict(p0, ell=float("nan"), shift=float("nan")))

    def systems(self) -> np.ndarray:
        """First row of every system plus the total (h2x_plan_systems)."""
        cnt = C.c_int32()
        _check(load_library().h2x_plan_systems(self._h, C.byref(cnt), None), "h2x_plan_systems")
        off = np.zeros(cnt.value + 1, np.int64)
        _check(load_library().h2x_plan_systems(self._h, C.byref(cnt), _ptr(off)), "h2x_plan_systems")
        return off

    def perm(self) -> np.ndarray:
        a = np.zeros(self.n, np.int64)
        _check(load_library().h2x_plan_perm(self._h, _ptr(a)), "h2x_plan_perm")
        return a

    def clusters(self) -> dict:
        out = {nm: np.zeros(self.C, np.int64) for nm in ("first", "size", "parent", "son0", "son1", "depth")}
        _check(load_library().h2x_plan_clusters(self._h, *[_ptr(out[nm]) for nm in
                                                          ("first", "size", "parent", "son0", "son1", "depth")]),
               "h2x_plan_clusters")
        return out

    def blocks(self) -> dict:
        at, as_ = np.zeros(self.n_adm, np.int64), np.zeros(self.n_adm, np.int64)
        nt, ns = np.zeros(self.n_near, np.int64), np.zeros(self.n_near, np.int64)
        _check(load_library().h2x_plan_blocks(self._h, _ptr(at), _ptr(as_), _ptr(nt), _ptr(ns)), "h2x_plan_blocks")
        return dict(adm_t=at, adm_s=as_, near_t=nt, near_s=ns)


def _stream(torch, device):
    return C.c_void_p(torch.cuda.current_stream(device).cuda_stream)


class H2Matrix:
    """An H^2 operator filled on the GPU (h2x_mat_create) inside a torch-owned workspace."""

    def __init__(self, points_or_plan, *, storage="f64", device="cuda", **params):
        import torch
        lib = load_library()
        self.plan = points_or_plan if isinstance(points_or_plan, Plan) else Plan(points_or_plan, **params)
        self.storage = _PREC[storage]
        self.device = torch.device(device)
        nbytes = lib.h2x_mat_workspace_bytes(self.plan._h, self.storage)
        if nbytes == 0:
            raise H2xError("h2x_mat_workspace_bytes returned 0")
        self._ws = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        h = C.c_void_p()
        _check(lib.h2x_mat_create(self.plan._h, self.storage, C.c_void_p(self._ws.data_ptr()), nbytes,
                                  _stream(torch, self.device), C.byref(h)), "h2x_mat_create")
        self._h = h
        self.n, self.k = self.plan.n, self.plan.k
        self.ell = float(self.plan.params["ell"])
        kern = self.plan.params.get("kernel", "exp")
        self.complex = kern in ("helmholtz", 3)  # complex operator: column pairs (real, imaginary)
        self._mm_ws = {}

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.h2x_mat_destroy(self._h)
            self._h = None

    _WS = {"matmul": "h2x_matmul_workspace_bytes", "cg": "h2x_block_cg_workspace_bytes",
           "adjoint": "h2x_matmul_adjoint_workspace_bytes", "grad": "h2x_grad_workspace_bytes"}

    def workspace(self, m: int, kind: str = "matmul"):
        import torch
        key = (kind, m)
        ws = self._mm_ws.get(key)
        if ws is None:
            nb = getattr(load_library(), self._WS[kind])(self._h, m)
            ws = torch.empty(max(nb, 256), dtype=torch.uint8, device=self.device)
            self._mm_ws[key] = ws
        return ws

    def autotune(self, m: int) -> dict:
        """Choose the matrix-core tile shapes for m columns by timing (h2x_mat_autotune);
        later products and solves with a similar column count use them."""
        import torch
        lib = load_library()
        nb = lib.h2x_mat_autotune_workspace_bytes(self._h, int(m))
        ws = torch.empty(max(nb, 256), dtype=torch.uint8, device=self.device)
        info = _TuneInfo()
        _check(lib.h2x_mat_autotune(self._h, int(m), C.c_void_p(ws.data_ptr()), ws.numel(),
                                    _stream(torch, self.device), C.byref(info)), "h2x_mat_autotune")
        return dict(nj_transfer=info.nj_transfer, nj_coupling=info.nj_coupling, np_leaf=info.np_leaf,
                    overlap=info.overlap, fuse_up=info.fuse_up, leaf_kind=info.leaf_kind, split=info.split,
                    ms_default=info.ms_default, ms_tuned=info.ms_tuned)

    _SHAPES = ("nj_transfer", "nj_coupling", "np_leaf", "overlap", "fuse_up", "leaf_kind", "split")

    def set_tune(self, m: int, **shapes) -> None:
        """Store tile shapes for m's column-count entry without timing (h2x_mat_set_tune);
        fields not given are 0 (the built-in rule)."""
        bad = set(shapes) - set(self._SHAPES)
        if bad:
            raise ValueError(f"unknown shape fields {sorted(bad)}")
        info = _TuneInfo(**{k: int(v) for k, v in shapes.items()})
        _check(load_library().h2x_mat_set_tune(self._h, int(m), C.byref(info)), "h2x_mat_set_tune")

    def get_tune(self, m: int) -> dict:
        """The tile shapes stored for m's column-count entry (h2x_mat_get_tune)."""
        info = _TuneInfo()
        _check(load_library().h2x_mat_get_tune(self._h, int(m), C.byref(info)), "h2x_mat_get_tune")
        return {k: getattr(info, k) for k in self._SHAPES}

    def product_times(self, cands, reps: int = 5) -> list:
        """Mean time (ms) of one product for each column count in cands (h2x_product_times):
        the throughput curve of the chunk policy."""
        import torch
        c = np.ascontiguousarray(cands, dtype=np.int64)
        lib = load_library()
        nb = lib.h2x_product_times_workspace_bytes(self._h, len(c), _ptr(c))
        ws = torch.empty(max(nb, 256), dtype=torch.uint8, device=self.device)
        ms = np.zeros(len(c))
        _check(lib.h2x_product_times(self._h, len(c), _ptr(c), int(reps), C.c_void_p(ws.data_ptr()), ws.numel(),
                                     _stream(torch, self.device), _ptr(ms)), "h2x_product_times")
        return [float(v) for v in ms]

    def set_ell(self, ell: float) -> None:
        """Refill S and the near field for a new kernel length scale (h2x_mat_set_ell)."""
        import torch
        _check(load_library().h2x_mat_set_ell(self._h, float(ell), _stream(torch, self.device)), "h2x_mat_set_ell")
        self.ell = float(ell)

    def coupling(self):
        """The coupling matrices as an (n_adm, k, k) float64 CUDA tensor (h2x_mat_coupling)."""
        import torch
        out = torch.empty((self.plan.n_adm, self.k, self.k), dtype=torch.float64, device=self.device)
        if self.plan.n_adm:
            _check(load_library().h2x_mat_coupling(self._h, C.c_void_p(out.data_ptr()), _stream(torch, self.device)),
                   "h2x_mat_coupling")
        return out

    def set_coupling(self, S) -> None:
        """Overwrite the coupling matrices with an (n_adm, k, k) float64 CUDA tensor
        (h2x_mat_set_coupling)."""
        import torch
        if S.dtype != torch.float64 or S.device.type != "cuda" or tuple(S.shape) != (self.plan.n_adm, self.k, self.k):
            raise ValueError("S must be an (n_adm, k, k) float64 CUDA tensor")
        S = S.contiguous()
        if self.plan.n_adm:
            _check(load_library().h2x_mat_set_coupling(self._h, C.c_void_p(S.data_ptr()), _stream(torch, self.device)),
                   "h2x_mat_set_coupling")
            torch.cuda.current_stream(self.device).synchronize()


STAGES = ("forward_leaf", "forward_transfer", "coupling", "backward_transfer", "leaf_near")


class Timer:
    """Stage events for `slots` products (h2x_timer_create): h2_matmul(..., timer=T, slot=i)
    records product i's stage boundaries without waiting; T.read(i) waits for them and
    returns the stage durations (ms, STAGES order)."""

    def __init__(self, slots: int):
        h = C.c_void_p()
        _check(load_library().h2x_timer_create(int(slots), C.byref(h)), "h2x_timer_create")
        self._h, self.slots = h, int(slots)

    def read(self, slot: int) -> np.ndarray:
        out = np.zeros(len(STAGES))
        _check(load_library().h2x_timer_read(self._h, int(slot), _ptr(out)), "h2x_timer_read")
        return out

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.h2x_timer_destroy(self._h)
            self._h = None


def h2_matmul(A: H2Matrix, X, *, alpha=1.0, beta=0.0, out=None, tree_order=False, stage_ms=None, timer=None,
              slot=0):
    """Y <- beta Y + alpha A X on the GPU (h2x_matmul).  X: (n, m) float64 CUDA tensor, or
    complex128 for a complex (Helmholtz) operator (its memory is 2m real columns).

    With ``stage_ms`` (a float64 numpy array of len(STAGES)) the product runs through
    h2x_matmul_timed and the per-stage durations in ms are written into it (blocking); with
    ``timer`` (a Timer) through h2x_matmul_marked into ``slot`` (not blocking)."""
    import torch
    if X.is_complex():
        Xr = _as_real(torch, X)
        Yr = None if out is None else _as_real(torch, out)
        Yr = h2_matmul(A, Xr, alpha=alpha, beta=beta, out=Yr, tree_order=tree_order, stage_ms=stage_ms, timer=timer,
                       slot=slot)
        return torch.view_as_complex(Yr.reshape(Yr.shape[0], -1, 2)) if out is None else out
    squeeze = X.dim() == 1
    X2 = X.reshape(-1, 1) if squeeze else X
    if X2.dtype != torch.float64 or X2.device.type != "cuda" or X2.stride(1) != 1:
        raise ValueError("X must be a row-major float64 CUDA tensor")
    n, m = X2.shape
    if n != A.n:
        raise ValueError("X has the wrong number of rows")
    if out is None:
        if beta != 0.0:
            raise ValueError("beta != 0 needs out")
        out = torch.empty((n, m), dtype=torch.float64, device=X2.device)
    Y = out.reshape(-1, 1) if out.dim() == 1 else out
    if Y.stride(1) != 1:
        raise ValueError("out must be row-major")
    ws = A.workspace(m)
    args = (A._h, m, float(alpha), C.c_void_p(X2.data_ptr()), X2.stride(0), float(beta), C.c_void_p(Y.data_ptr()),
            Y.stride(0), TREE_ORDER if tree_order else 0, C.c_void_p(ws.data_ptr()), ws.numel(),
            _stream(torch, X2.device))
    if timer is not None:
        _check(load_library().h2x_matmul_marked(*args, timer._h, int(slot)), "h2x_matmul_marked")
    elif stage_ms is None:
        _check(load_library().h2x_matmul(*args), "h2x_matmul")
    else:
        assert stage_ms.dtype == np.float64 and stage_ms.size >= len(STAGES)
        _check(load_library().h2x_matmul_timed(*args, _ptr(stage_ms)), "h2x_matmul_timed")
    return out


def _as_real(torch, Z):
    """A row-major complex128 (n, m) tensor as its (n, 2m) float64 view (pairs real, imaginary)."""
    Z2 = Z.reshape(-1, 1) if Z.dim() == 1 else Z
    if Z2.dtype != torch.complex128 or Z2.device.type != "cuda" or not Z2.is_contiguous():
        raise ValueError("complex input must be a contiguous complex128 CUDA tensor")
    return torch.view_as_real(Z2).reshape(Z2.shape[0], -1)


def _rowmajor(T, n, what):
    import torch
    if T.dtype != torch.float64 or T.device.type != "cuda" or T.dim() != 2 or T.stride(1) != 1 or T.shape[0] != n:
        raise ValueError(f"{what} must be a row-major (n, m) float64 CUDA tensor")


NOALLOC_MAX_BYTES = 128 << 20  # H2X_NOALLOC_MAX_BYTES


def h2_matmul_noalloc(A: H2Matrix, X, *, alpha=1.0, beta=0.0, out=None, tree_order=False):
    """Y <- beta Y + alpha A X through h2x_matmul_noalloc: the library's static scratch array
    instead of a workspace (the call allocates nothing on the device; ``out`` must be given
    when the caller cannot allocate).  X, out: (n, m) row-major float64 CUDA tensors."""
    import torch
    _rowmajor(X, A.n, "X")
    n, m = X.shape
    if out is None:
        if beta != 0.0:
            raise ValueError("beta != 0 needs out")
        out = torch.empty((n, m), dtype=torch.float64, device=X.device)
    _rowmajor(out, n, "out")
    _check(load_library().h2x_matmul_noalloc(A._h, m, float(alpha), C.c_void_p(X.data_ptr()), X.stride(0),
                                             float(beta), C.c_void_p(out.data_ptr()), out.stride(0),
                                             TREE_ORDER if tree_order else 0, _stream(torch, X.device)),
           "h2x_matmul_noalloc")
    return out


def h2_matmul_adjoint(A: H2Matrix, X, *, alpha=1.0, beta=0.0, out=None):
    """Y <- beta Y + alpha A^T X through the column lists (h2x_matmul_adjoint)."""
    import torch
    _rowmajor(X, A.n, "X")
    n, m = X.shape
    if out is None:
        if beta != 0.0:
            raise ValueError("beta != 0 needs out")
        out = torch.empty((n, m), dtype=torch.float64, device=X.device)
    _rowmajor(out, n, "out")
    ws = A.workspace(m, "adjoint")
    _check(load_library().h2x_matmul_adjoint(A._h, m, float(alpha), C.c_void_p(X.data_ptr()), X.stride(0),
                                             float(beta), C.c_void_p(out.data_ptr()), out.stride(0),
                                             C.c_void_p(ws.data_ptr()), ws.numel(), _stream(torch, X.device)),
           "h2x_matmul_adjoint")
    return out


DELL_TERMS = {"all": 3, "coupling": 1, "near": 2}


def h2_grad(A: H2Matrix, X, dY, *, want_dS=True, want_dN=False, want_dell=True, scale=1.0, dell_terms="all"):
    """Gradients of scale * <dY, A X> (h2x_grad): returns (dS, dN, dell) as CUDA tensors,
    None where not requested.  dS: (n_adm, k, k) in the order of Plan.blocks(); dN: the
    near-field blocks, each |t| x |s| row-major in tree order, concatenated; dell: 0-d,
    summed over the terms named by dell_terms ("all", "coupling" or "near")."""
    import torch
    _rowmajor(X, A.n, "X")
    _rowmajor(dY, A.n, "dY")
    if dY.shape != X.shape:
        raise ValueError("X and dY must have the same shape")
    m = X.shape[1]
    dev = X.device
    dS = torch.empty((A.plan.n_adm, A.k, A.k), dtype=torch.float64, device=dev) if want_dS else None
    dN = torch.empty(A.plan.near_entries, dtype=torch.float64, device=dev) if want_dN else None
    dl = torch.empty((), dtype=torch.float64, device=dev) if want_dell else None
    ws = A.workspace(m, "grad")
    vp = lambda t: C.c_void_p(t.data_ptr()) if t is not None and t.numel() else None
    _check(load_library().h2x_grad(A._h, m, vp(X), X.stride(0), vp(dY), dY.stride(0), vp(dS), vp(dN), vp(dl),
                                   float(scale), DELL_TERMS[dell_terms], C.c_void_p(ws.data_ptr()), ws.numel(),
                                   _stream(torch, dev)), "h2x_grad")
    return dS, dN, dl


@dataclass
class CgInfo:
    iters: int
    status: int
    col_relres: np.ndarray
    col_iters: np.ndarray
    col_status: np.ndarray
    outer_iters: int = 0
    sys_iters: np.ndarray = None


def _new_info(m, nsys=1):
    rel = np.zeros(nsys * m)
    its = np.zeros(nsys * m, np.int32)
    sts = np.zeros(nsys * m, np.int32)
    sys = np.zeros(nsys, np.int32)
    i32 = lambda a: a.ctypes.data_as(C.POINTER(C.c_int32))
    info = _CgInfo(0, 0, 0, rel.ctypes.data_as(C.POINTER(C.c_double)), i32(its), i32(sts), i32(sys))
    return info, rel, its, sts, sys


def _info(info, rel, its, sts, sys, nsys, m):
    shp = (nsys, m) if nsys > 1 else (m,)
    return CgInfo(info.iters, info.status, rel.reshape(shp), its.reshape(shp), sts.reshape(shp), info.outer_iters,
                  sys)


def block_cg_solve(A: H2Matrix, B, X0=None, *, rtol=1e-8, max_iter=10000, freeze_converged=False,
                   check_every=4, variant="independent", graph=False):
    """Solve A X = B (block CG, h2x_block_cg).  variant "independent": the paper's m
    independent CG iterations sharing the product; "shared": one shared block Krylov
    space with m x m Gram matrices.  graph: replay check_every captured iterations as
    one HIP graph.  On a merged plan every system is solved on its own (info arrays
    are systems x m).  Returns (X, CgInfo)."""
    import torch
    if B.dtype != torch.float64 or B.device.type != "cuda" or B.dim() != 2 or B.stride(1) != 1:
        raise ValueError("B must be a row-major (n, m) float64 CUDA tensor")
    n, m = B.shape
    X = torch.zeros_like(B) if X0 is None else X0.clone()
    ws = A.workspace(m, "cg")
    nsys = len(A.plan.systems()) - 1
    info, rel, its, sts, sys = _new_info(m, nsys)
    prm = _CgParams(float(rtol), int(max_iter), int(bool(freeze_converged)), int(check_every), _VARIANT[variant],
                    int(bool(graph)))
    _check(load_library().h2x_block_cg(A._h, C.byref(prm), m, C.c_void_p(B.data_ptr()), B.stride(0),
                                       C.c_void_p(X.data_ptr()), X.stride(0), C.c_void_p(ws.data_ptr()), ws.numel(),
                                       C.byref(info), _stream(torch, B.device)), "h2x_block_cg")
    return X, _info(info, rel, its, sts, sys, nsys, m)


@dataclass
class GmresInfo:
    iters: int
    cycles: int
    status: int
    col_res: np.ndarray
    col_iters: np.ndarray
    col_status: np.ndarray


def block_gmres_solve(A: H2Matrix, B, X0=None, *, rtol=1e-8, restart=30, max_iter=10000, check_every=4):
    """Solve A X = B with block GMRES(restart) (h2x_block_gmres): m independent GMRES
    processes sharing one product per Arnoldi step, restarted from the improved
    iterate until every column's true residual is within rtol.  Returns (X, GmresInfo)."""
    import torch
    if B.is_complex():  # complex operator: m complex columns as 2m real ones
        Br = _as_real(torch, B)
        X0r = None if X0 is None else _as_real(torch, X0.contiguous())
        Xr, info = block_gmres_solve(A, Br, X0r, rtol=rtol, restart=restart, max_iter=max_iter,
                                     check_every=check_every)
        return torch.view_as_complex(Xr.reshape(Xr.shape[0], -1, 2)), info
    if B.dtype != torch.float64 or B.device.type != "cuda" or B.dim() != 2 or B.stride(1) != 1:
        raise ValueError("B must be a row-major (n, m) float64 CUDA tensor")
    n, m = B.shape
    X = torch.zeros_like(B) if X0 is None else X0.clone()
    lib = load_library()
    nb = lib.h2x_block_gmres_workspace_bytes(A._h, m, int(restart))
    if nb == 0:
        raise ValueError("block_gmres_solve: need m >= 1 and restart >= 1")
    ws = torch.empty(nb, dtype=torch.uint8, device=B.device)
    mi = m // 2 if A.complex else m  # info entries per complex column
    res = np.zeros(mi)
    its = np.zeros(mi, np.int32)
    sts = np.zeros(mi, np.int32)
    i32 = lambda a: a.ctypes.data_as(C.POINTER(C.c_int32))
    info = _GmresInfo(0, 0, 0, 0, res.ctypes.data_as(C.POINTER(C.c_double)), i32(its), i32(sts))
    prm = _GmresParams(float(rtol), int(restart), int(max_iter), int(check_every), 0)
    _check(lib.h2x_block_gmres(A._h, C.byref(prm), m, C.c_void_p(B.data_ptr()), B.stride(0),
                               C.c_void_p(X.data_ptr()), X.stride(0), C.c_void_p(ws.data_ptr()), ws.numel(),
                               C.byref(info), _stream(torch, B.device)), "h2x_block_gmres")
    return X, GmresInfo(info.iters, info.cycles, info.status, res, its, sts)


_SOLVER = {"cg": 0, "gmres": 1}


def solve_workspace_bytes(plan: Plan, m: int, *, storage="f64", solver="cg", restart=30) -> int:
    """Device workspace of one solve of m right-hand sides (h2x_solve_workspace_bytes)."""
    return load_library().h2x_solve_workspace_bytes(plan._h, _PREC[storage], _SOLVER[solver], int(m), int(restart))


def choose_chunk(plan: Plan, m: int, mem_bytes: int, *, storage="f64", solver="cg", restart=30, curve=None) -> int:
    """m_chunk for m right-hand sides under a workspace budget (h2x_choose_chunk); curve:
    optional {column count: ms per product} throughput curve."""
    out = np.zeros(1, np.int64)
    if curve:
        cm = np.ascontiguousarray(list(curve.keys()), dtype=np.int64)
        ms = np.ascontiguousarray(list(curve.values()), dtype=np.float64)
        args = (len(cm), _ptr(cm), _ptr(ms))
    else:
        args = (0, None, None)
    _check(load_library().h2x_choose_chunk(plan._h, _PREC[storage], _SOLVER[solver], int(restart), int(m),
                                           int(mem_bytes), *args, _ptr(out)), "h2x_choose_chunk")
    return int(out[0])


def block_cg_solve_chunked(A: H2Matrix, B, m_chunk: int, X0=None, *, rtol=1e-8, max_iter=10000,
                           freeze_converged=False, check_every=4, variant="independent"):
    """Block CG over the columns of B in chunks of m_chunk (h2x_block_cg_chunked)."""
    import torch
    if B.dtype != torch.float64 or B.device.type != "cuda" or B.dim() != 2 or B.stride(1) != 1:
        raise ValueError("B must be a row-major (n, m) float64 CUDA tensor")
    n, m = B.shape
    X = torch.zeros_like(B) if X0 is None else X0.clone()
    lib = load_library()
    mc = min(int(m_chunk), m)
    nb = solve_workspace_bytes(A.plan, mc, storage=A.storage, solver="cg")
    ws = torch.empty(max(nb, 256), dtype=torch.uint8, device=B.device)
    info, rel, its, sts, sys = _new_info(m, 1)
    prm = _CgParams(float(rtol), int(max_iter), int(bool(freeze_converged)), int(check_every), _VARIANT[variant], 0)
    _check(lib.h2x_block_cg_chunked(A._h, C.byref(prm), m, mc, C.c_void_p(B.data_ptr()), B.stride(0),
                                    C.c_void_p(X.data_ptr()), X.stride(0), C.c_void_p(ws.data_ptr()), ws.numel(),
                                    C.byref(info), _stream(torch, B.device)), "h2x_block_cg_chunked")
    return X, _info(info, rel, its, sts, sys, 1, m)


def block_gmres_solve_chunked(A: H2Matrix, B, m_chunk: int, X0=None, *, rtol=1e-8, restart=30, max_iter=10000,
                              check_every=4):
    """Block GMRES over the columns of B in chunks of m_chunk (h2x_block_gmres_chunked)."""
    import torch
    if B.dtype != torch.float64 or B.device.type != "cuda" or B.dim() != 2 or B.stride(1) != 1:
        raise ValueError("B must be a row-major (n, m) float64 CUDA tensor")
    n, m = B.shape
    X = torch.zeros_like(B) if X0 is None else X0.clone()
    lib = load_library()
    mc = min(int(m_chunk), m)
    nb = solve_workspace_bytes(A.plan, mc, storage=A.storage, solver="gmres", restart=restart)
    ws = torch.empty(max(nb, 256), dtype=torch.uint8, device=B.device)
    res = np.zeros(m)
    its = np.zeros(m, np.int32)
    sts = np.zeros(m, np.int32)
    i32 = lambda a: a.ctypes.data_as(C.POINTER(C.c_int32))
    info = _GmresInfo(0, 0, 0, 0, res.ctypes.data_as(C.POINTER(C.c_double)), i32(its), i32(sts))
    prm = _GmresParams(float(rtol), int(restart), int(max_iter), int(check_every), 0)
    _check(lib.h2x_block_gmres_chunked(A._h, C.byref(prm), m, mc, C.c_void_p(B.data_ptr()), B.stride(0),
                                       C.c_void_p(X.data_ptr()), X.stride(0), C.c_void_p(ws.data_ptr()), ws.numel(),
                                       C.byref(info), _stream(torch, B.device)), "h2x_block_gmres_chunked")
    return X, GmresInfo(info.iters, info.cycles, info.status, res, its, sts)


def solve_chunked(A: H2Matrix, B, mem_bytes: int, *, solver="cg", candidates=(8, 16, 32, 64, 128), restart=30,
                  **kw):
    """Solve A X = B in right-hand-side chunks sized by the chunk policy: the throughput
    curve of the candidate column counts (h2x_product_times), then h2x_choose_chunk under
    the workspace budget mem_bytes, then the chunked solver.  Returns (X, info, m_chunk)."""
    m = B.shape[1]
    cands = sorted({min(int(c), m) for c in candidates})
    curve = dict(zip(cands, A.product_times(cands)))
    mc = choose_chunk(A.plan, m, mem_bytes, storage=A.storage, solver=solver, restart=restart, curve=curve)
    if solver == "cg":
        X, info = block_cg_solve_chunked(A, B, mc, **kw)
    else:
        X, info = block_gmres_solve_chunked(A, B, mc, restart=restart, **kw)
    return X, info, mc


def block_cg_refine(A: H2Matrix, A_lo: H2Matrix, B, *, rtol=1e-10, inner_rtol=1e-4, max_outer=50,
                    max_inner=10000, check_every=4):
    """Mixed precision: FP64 refinement around block CG with the low-precision A_lo
    (h2x_block_cg_refine).  A and A_lo must share one Plan.  Returns (X, CgInfo)."""
    import torch
    if B.dtype != torch.float64 or B.device.type != "cuda" or B.dim() != 2 or B.stride(1) != 1:
        raise ValueError("B must be a row-major (n, m) float64 CUDA tensor")
    n, m = B.shape
    X = torch.zeros_like(B)
    lib = load_library()
    nb = lib.h2x_block_cg_refine_workspace_bytes(A._h, A_lo._h, m)
    ws = torch.empty(max(nb, 256), dtype=torch.uint8, device=B.device)
    info, rel, its, sts, sys = _new_info(m)
    prm = _CgParams(float(inner_rtol), int(max_inner), 0, int(check_every), CG_INDEPENDENT, 0)
    _check(lib.h2x_block_cg_refine(A._h, A_lo._h, C.byref(prm), float(rtol), int(max_outer), m,
                                   C.c_void_p(B.data_ptr()), B.stride(0), C.c_void_p(X.data_ptr()), X.stride(0),
                                   C.c_void_p(ws.data_ptr()), ws.numel(), C.byref(info), _stream(torch, B.device)),
           "h2x_block_cg_refine")
    return X, _info(info, rel, its, sts, sys, 1, m)


def block_cg_mixed(A: H2Matrix, A_lo: H2Matrix, B, *, rtol=1e-10, delta=0.1, max_iter=10000, check_every=4,
                   graph=False):
    """Mixed precision in one CG run (h2x_block_cg_mixed): iterations with the
    low-precision A_lo, the residual recomputed with the FP64 A whenever it has
    dropped by delta since the last recomputation and before stopping.  A and A_lo
    share one Plan.  Returns (X, CgInfo); info.outer_iters counts recomputations."""
    import torch
    if B.dtype != torch.float64 or B.device.type != "cuda" or B.dim() != 2 or B.stride(1) != 1:
        raise ValueError("B must be a row-major (n, m) float64 CUDA tensor")
    n, m = B.shape
    X = torch.zeros_like(B)
    lib = load_library()
    nb = lib.h2x_block_cg_mixed_workspace_bytes(A._h, A_lo._h, m)
    ws = torch.empty(max(nb, 256), dtype=torch.uint8, device=B.device)
    info, rel, its, sts, sys = _new_info(m)
    prm = _CgParams(float(rtol), int(max_iter), 0, int(check_every), CG_INDEPENDENT, int(bool(graph)))
    _check(lib.h2x_block_cg_mixed(A._h, A_lo._h, C.byref(prm), float(delta), m, C.c_void_p(B.data_ptr()),
                                  B.stride(0), C.c_void_p(X.data_ptr()), X.stride(0), C.c_void_p(ws.data_ptr()),
                                  ws.numel(), C.byref(info), _stream(torch, B.device)), "h2x_block_cg_mixed")
    return X, _info(info, rel, its, sts, sys, 1, m)


class Batch:
    """Many independent systems (h2x_batch): systems with one Chebyshev order and
    storage share one merged plan and operator, so every product stage is one launch
    over all of them.  Rows of every batch-wide block are the systems' rows
    concatenated in ``order`` (the operators' order; ``order[i]`` lists the system
    indices, in the caller's numbering, of operator i)."""

    def __init__(self, systems, *, storage="f64", device="cuda"):
        """systems: list of (points, params dict) pairs."""
        import torch
        groups = {}
        for i, (pts, prm) in enumerate(systems):
            groups.setdefault(int(prm.get("p", 3)), []).append(i)
        self.device = torch.device(device)
        self.order, self.plans, self.mats = [], [], []
        self._parts = []
        for p in sorted(groups):
            idx = groups[p]
            parts = [Plan(systems[i][0], **systems[i][1]) for i in idx]
            merged = Plan.merge(parts)
            self._parts.append(parts)
            self.plans.append(merged)
            self.mats.append(H2Matrix(merged, storage=storage, device=self.device))
            self.order.append(idx)
        self.sizes = np.array([len(systems[i][0]) for i in range(len(systems))], np.int64)
        perm = [i for idx in self.order for i in idx]
        self.system_order = np.array(perm, np.int64)
        self.row_offsets = np.zeros(len(perm) + 1, np.int64)
        self.row_offsets[1:] = np.cumsum(self.sizes[self.system_order])
        self.n = int(self.row_offsets[-1])
        arr = (C.c_void_p * len(self.mats))(*[a._h for a in self.mats])
        h = C.c_void_p()
        _check(load_library().h2x_batch_create(arr, len(self.mats), C.byref(h)), "h2x_batch_create")
        self._h = h
        self._ws = {}

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.h2x_batch_destroy(self._h)
            self._h = None

    def autotune(self, m: int) -> list:
        """Autotune every operator of the batch for m columns."""
        return [A.autotune(m) for A in self.mats]

    def rows(self, i: int):
        """Row range of system i (caller's numbering) in batch-wide blocks."""
        pos = int(np.nonzero(self.system_order == i)[0][0])
        return int(self.row_offsets[pos]), int(self.row_offsets[pos + 1])

    def workspace(self, m, kind):
        import torch
        ws = self._ws.get((kind, m))
        if ws is None:
            f = {"matmul": "h2x_batch_matmul_workspace_bytes", "cg": "h2x_batch_block_cg_workspace_bytes"}[kind]
            nb = getattr(load_library(), f)(self._h, m)
            ws = torch.empty(max(nb, 256), dtype=torch.uint8, device=self.device)
            self._ws[(kind, m)] = ws
        return ws


def batch_matmul(batch: Batch, X, *, alpha=1.0, beta=0.0, out=None):
    """Y <- beta Y + alpha diag(A_1, ...) X over the batch (h2x_batch_matmul)."""
    import torch
    _rowmajor(X, batch.n, "X")
    m = X.shape[1]
    if out is None:
        if beta != 0.0:
            raise ValueError("beta != 0 needs out")
        out = torch.empty_like(X)
    _rowmajor(out, batch.n, "out")
    ws = batch.workspace(m, "matmul")
    _check(load_library().h2x_batch_matmul(batch._h, m, float(alpha), C.c_void_p(X.data_ptr()), X.stride(0),
                                           float(beta), C.c_void_p(out.data_ptr()), out.stride(0), 0,
                                           C.c_void_p(ws.data_ptr()), ws.numel(), _stream(torch, X.device)),
           "h2x_batch_matmul")
    return out


def batch_block_cg_solve(batch: Batch, B, *, rtol=1e-8, max_iter=10000, check_every=4, graph=True):
    """Block CG on every system of the batch at once (h2x_batch_block_cg).  Systems with
    fewer right-hand sides pad B with zero columns.  Returns (X, CgInfo) with info arrays
    in the batch's system order (batch.system_order)."""
    import torch
    _rowmajor(B, batch.n, "B")
    m = B.shape[1]
    X = torch.zeros_like(B)
    ws = batch.workspace(m, "cg")
    nsys = len(batch.system_order)
    info, rel, its, sts, sys = _new_info(m, nsys)
    prm = _CgParams(float(rtol), int(max_iter), 0, int(check_every), CG_INDEPENDENT, int(bool(graph)))
    _check(load_library().h2x_batch_block_cg(batch._h, C.byref(prm), m, C.c_void_p(B.data_ptr()), B.stride(0),
                                             C.c_void_p(X.data_ptr()), X.stride(0), C.c_void_p(ws.data_ptr()),
                                             ws.numel(), C.byref(info), _stream(torch, B.device)),
           "h2x_batch_block_cg")
    return X, _info(info, rel, its, sts, sys, nsys, m)
