"""Independent FP64 CPU oracle for the H^2 x X product and block CG.

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the benchmark's CPU
baseline leg may import this package; the product path never does.  It shares no
code with the HIP library (``paper_2509_17257_amd``) and imports nothing from it.

Everything that follows the paper lives in ``h2_oracle.c`` (cluster tree, block
tree, Chebyshev H^2 representation, forward / list-wise multiplication /
backward product, block CG).  This module marshals numpy arrays in and out and
adds the few dense checks that are plain linear algebra (dense kernel matrix,
dense Cholesky solve).

Pins: every function here is checked by ``tests/test_oracle_*.py`` against facts
fixed by the paper's definitions or by mathematics (partition of unity,
polynomial reproduction, nestedness, exactness for a polynomial kernel,
dense-assembly identity, closed-form solves).  The absolute interpolation error
for the exponential kernel is "parity unpinned": the paper gives no value for
it; only its geometric decay in the interpolation order is checked.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

from . import build as _build

KERNEL_EXP, KERNEL_POLY, KERNEL_CONST, KERNEL_HELMHOLTZ = 0, 1, 2, 3
_KERNELS = {"exp": KERNEL_EXP, "poly": KERNEL_POLY, "const": KERNEL_CONST, "helmholtz": KERNEL_HELMHOLTZ}

_lib = None

# rounding points of the emulated low-precision product that matmul_lowp(omit=...) can
# switch off one at a time (planted slips for the tests)
LOWP_OMIT = {"x_leaf": 1, "xhat_transfer": 2, "xhat_coupling": 4, "yhat_transfer": 8, "yhat_leaf": 16,
             "x_near_to_storage": 32, "fp64_sums": 64}


def _load():
    global _lib
    if _lib is not None:
        return _lib
    path = _build.build(force=False)
    lib = C.CDLL(path)
    P = C.c_void_p
    I64 = C.c_int64
    D = C.c_double
    lib.orc_build.restype = P
    lib.orc_build.argtypes = [P, I64, C.c_int, D, D, D, C.c_int, C.c_int]
    lib.orc_free.argtypes = [P]
    lib.orc_info.argtypes = [P, P]
    lib.orc_get_tree.argtypes = [P] * 12
    lib.orc_get_blocks.argtypes = [P] * 5
    lib.orc_get_lists.argtypes = [P] * 3
    for nm in ("orc_get_nodes", "orc_get_V", "orc_get_E", "orc_get_S", "orc_get_N",
               "orc_set_S", "orc_set_N", "orc_set_E"):
        getattr(lib, nm).argtypes = [P, P]
    lib.orc_basis_direct.argtypes = [P, I64, P]
    lib.orc_set_ell.argtypes = [P, D]
    lib.orc_matmul.argtypes = [P, I64, D, P, D, P]
    lib.orc_matmul_recursive.argtypes = [P, I64, D, P, D, P]
    lib.orc_forward_transform.argtypes = [P, I64, P, P]
    lib.orc_dense.argtypes = [P, P]
    lib.orc_dense_dell.argtypes = [P, P]
    lib.orc_block_cg.restype = I64
    lib.orc_block_cg.argtypes = [P, I64, P, P, D, I64, C.c_int, P, P]
    lib.orc_cg1.restype = I64
    lib.orc_cg1.argtypes = [P, P, P, D, I64]
    lib.orc_matmul_lowp.argtypes = [P, C.c_int, I64, D, P, D, P]
    lib.orc_matmul_lowp_planted.argtypes = [P, C.c_int, I64, D, P, D, P, C.c_int]
    lib.orc_block_cg_lowp.restype = I64
    lib.orc_block_cg_lowp.argtypes = [P, C.c_int, I64, P, P, D, I64, P, P]
    lib.orc_refine_cg.restype = I64
    lib.orc_refine_cg.argtypes = [P, C.c_int, I64, P, P, D, D, I64, I64, P, P, P]
    lib.orc_block_cg_mixed.restype = I64
    lib.orc_block_cg_mixed.argtypes = [P, C.c_int, I64, P, P, D, D, I64, I64, P, P, P]
    lib.orc_round_bf16_array.argtypes = [P, P, I64]
    lib.orc_matmul_adjoint.argtypes = [P, I64, D, P, D, P]
    lib.orc_grad.argtypes = [P, I64, P, P, P, P, P]
    lib.orc_block_cg_shared.restype = I64
    lib.orc_block_cg_shared.argtypes = [P, I64, P, P, D, I64, D, P, P]
    lib.orc_block_gmres.restype = I64
    lib.orc_block_gmres.argtypes = [P, I64, P, P, D, I64, I64, P, P, P, P]
    lib.orc_block_gmres_c.restype = I64
    lib.orc_block_gmres_c.argtypes = [P, I64, P, P, D, I64, I64, P, P, P, P]
    lib.orc_dense_complex.argtypes = [P, P]
    lib.orc_is_complex.restype = C.c_int
    lib.orc_is_complex.argtypes = [P]
    lib.orc_num_threads.restype = C.c_int
    lib.orc_set_threads.argtypes = [C.c_int]
    _lib = lib
    return lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


def num_threads() -> int:
    return int(_load().orc_num_threads())


def set_threads(t: int) -> None:
    _load().orc_set_threads(int(t))


class OracleH2:
    """H^2 approximation of g(x_i, x_j) + shift * delta_ij built from the paper's definitions."""

    def __init__(self, points, *, kernel="exp", ell=0.5, shift=1.0, eta=1.0, leaf=32, p=3):
        lib = _load()
        pts = np.ascontiguousarray(points, dtype=np.float64)
        if pts.ndim != 2 or pts.shape[1] != 3:
            raise ValueError("points must be n x 3")
        self.n = pts.shape[0]
        self.kernel = _KERNELS[kernel] if isinstance(kernel, str) else int(kernel)
        self.ell, self.shift, self.eta, self.leaf, self.p = float(ell), float(shift), float(eta), int(leaf), int(p)
        self.k = self.p ** 3
        self._h = lib.orc_build(_ptr(pts), self.n, self.kernel, self.ell, self.shift, self.eta, self.leaf, self.p)
        if not self._h:
            raise ValueError("oracle build failed")
        self.points = pts
        info = np.zeros(16, dtype=np.int64)
        lib.orc_info(self._h, _ptr(info))
        (self.n, self.C, self.leaves, self.n_adm, self.n_near, self.near_entries,
         self.depth, self.k, self.p, self.nb) = [int(v) for v in info[:10]]

    def __del__(self):
        if getattr(self, "_h", None):
            _load().orc_free(self._h)
            self._h = None

    # -- structure ---------------------------------------------------------
    def tree(self) -> dict:
        C_ = self.C
        out = dict(perm=np.zeros(self.n, np.int64))
        for nm in ("first", "size", "son0", "son1", "parent", "depth"):
            out[nm] = np.zeros(C_, np.int64)
        for nm in ("blo", "bhi", "ilo", "ihi"):
            out[nm] = np.zeros((C_, 3), np.float64)
        _load().orc_get_tree(self._h, *[_ptr(out[nm]) for nm in
                                        ("perm", "first", "size", "son0", "son1", "parent", "depth",
                                         "blo", "bhi", "ilo", "ihi")])
        return out

    def blocks(self) -> dict:
        nb = self.nb
        bt, bs, boff = np.zeros(nb, np.int64), np.zeros(nb, np.int64), np.zeros(nb, np.int64)
        badm = np.zeros(nb, np.int32)
        _load().orc_get_blocks(self._h, _ptr(bt), _ptr(bs), _ptr(badm), _ptr(boff))
        lp = np.zeros(self.C + 1, np.int64)
        lb = np.zeros(nb, np.int64)
        _load().orc_get_lists(self._h, _ptr(lp), _ptr(lb))
        return dict(t=bt, s=bs, adm=badm.astype(bool), off=boff, list_ptr=lp, list_blk=lb)

    def nodes(self) -> np.ndarray:
        a = np.zeros((self.C, self.k, 3))
        _load().orc_get_nodes(self._h, _ptr(a))
        return a

    def V(self) -> np.ndarray:
        a = np.zeros((self.n, self.k))
        _load().orc_get_V(self._h, _ptr(a))
        return a

    def E(self) -> np.ndarray:
        a = np.zeros((self.C, self.k, self.k))
        _load().orc_get_E(self._h, _ptr(a))
        return a

    def S(self) -> np.ndarray:
        a = np.zeros((self.n_adm, self.k, self.k))
        _load().orc_get_S(self._h, _ptr(a))
        return a

    def N(self) -> np.ndarray:
        a = np.zeros(self.near_entries)
        _load().orc_get_N(self._h, _ptr(a))
        return a

    def set_S(self, S: np.ndarray) -> None:
        S = np.ascontiguousarray(S, dtype=np.float64)
        assert S.size == self.n_adm * self.k * self.k
        _load().orc_set_S(self._h, _ptr(S))

    def set_N(self, N: np.ndarray) -> None:
        N = np.ascontiguousarray(N, dtype=np.float64)
        assert N.size == self.near_entries
        _load().orc_set_N(self._h, _ptr(N))

    def set_E(self, E: np.ndarray) -> None:
        E = np.ascontiguousarray(E, dtype=np.float64)
        assert E.size == self.C * self.k * self.k
        _load().orc_set_E(self._h, _ptr(E))

    def set_ell(self, ell: float) -> None:
        self.ell = float(ell)
        _load().orc_set_ell(self._h, self.ell)

    def basis_direct(self, c: int) -> np.ndarray:
        sz = int(self.tree()["size"][c])
        a = np.zeros((sz, self.k))
        _load().orc_basis_direct(self._h, int(c), _ptr(a))
        return a

    # -- products ----------------------------------------------------------
    def matmul(self, X, alpha=1.0, beta=0.0, Y=None, recursive=False) -> np.ndarray:
        """Y <- beta Y + alpha A_H2 X (X, Y: n x m, original point order)."""
        X = np.ascontiguousarray(X, dtype=np.float64)
        squeeze = X.ndim == 1
        if squeeze:
            X = X[:, None].copy()
        m = X.shape[1]
        out = np.zeros((self.n, m)) if Y is None else np.ascontiguousarray(Y, dtype=np.float64).reshape(self.n, m).copy()
        fn = _load().orc_matmul_recursive if recursive else _load().orc_matmul
        fn(self._h, m, float(alpha), _ptr(X), float(beta), _ptr(out))
        return out[:, 0] if squeeze else out

    def matmul_lowp(self, X, prec, alpha=1.0, beta=0.0, Y=None, omit=0) -> np.ndarray:
        """Emulated low-precision operator (prec "f32" or "bf16"): V, E, S rounded to the
        storage type, near field to FP32, FP32 accumulation.  omit != 0 switches rounding
        points off (planted slips for the tests; see LOWP_OMIT)."""
        pr = {"f32": 1, "bf16": 2}[prec]
        X = np.ascontiguousarray(X, dtype=np.float64)
        m = X.shape[1]
        out = np.zeros((self.n, m)) if Y is None else np.ascontiguousarray(Y, dtype=np.float64).copy()
        if omit:
            _load().orc_matmul_lowp_planted(self._h, pr, m, float(alpha), _ptr(X), float(beta), _ptr(out), int(omit))
        else:
            _load().orc_matmul_lowp(self._h, pr, m, float(alpha), _ptr(X), float(beta), _ptr(out))
        return out

    def refine_cg(self, B, prec, rtol=1e-10, inner_rtol=1e-4, max_outer=50, max_inner=10000):
        """FP64 iterative refinement around block CG with the low-precision operator.  Each
        column returns its outer iterate with the smallest FP64 true residual."""
        pr = {"f32": 1, "bf16": 2}[prec]
        B = np.ascontiguousarray(B, dtype=np.float64)
        X = np.zeros_like(B)
        tot = np.zeros(1, np.int64)
        rel = np.zeros(B.shape[1])
        st = np.zeros(1, np.int32)
        outer = _load().orc_refine_cg(self._h, pr, B.shape[1], _ptr(B), _ptr(X), float(rtol), float(inner_rtol),
                                      int(max_outer), int(max_inner), _ptr(tot), _ptr(rel), _ptr(st))
        return X, dict(outer=int(outer), inner=int(tot[0]), col_relres=rel, status=int(st[0]))

    def block_cg_mixed(self, B, prec, rtol=1e-10, delta=0.1, max_iter=10000, check=4):
        """Mixed precision in one CG run: iterations with the emulated low-precision
        operator, the residual recomputed with the FP64 operator (residual replacement).
        Each column returns the recomputed iterate with the smallest true residual."""
        pr = {"f32": 1, "bf16": 2}[prec]
        B = np.ascontiguousarray(B, dtype=np.float64)
        X = np.zeros_like(B)
        rep = np.zeros(1, np.int64)
        rel = np.zeros(B.shape[1])
        st = np.zeros(1, np.int32)
        it = _load().orc_block_cg_mixed(self._h, pr, B.shape[1], _ptr(B), _ptr(X), float(rtol), float(delta),
                                        int(max_iter), int(check), _ptr(rep), _ptr(rel), _ptr(st))
        return X, dict(iters=int(it), replacements=int(rep[0]), col_relres=rel, status=int(st[0]))

    def matmul_adjoint(self, X, alpha=1.0, beta=0.0, Y=None) -> np.ndarray:
        """Y <- beta Y + alpha A^T X through the column lists (transposed blocks)."""
        X = np.ascontiguousarray(X, dtype=np.float64)
        m = X.shape[1]
        out = np.zeros((self.n, m)) if Y is None else np.ascontiguousarray(Y, dtype=np.float64).copy()
        _load().orc_matmul_adjoint(self._h, m, float(alpha), _ptr(X), float(beta), _ptr(out))
        return out

    def grad(self, X, dY, want_dS=True, want_dN=True):
        """Gradients of <dY, A X>: dS (n_adm x k x k, block-tree order), dN (near entries,
        row-major per block), dell (scalar)."""
        X = np.ascontiguousarray(X, dtype=np.float64)
        dY = np.ascontiguousarray(dY, dtype=np.float64)
        dS = np.zeros((self.n_adm, self.k, self.k)) if want_dS else None
        dN = np.zeros(self.near_entries) if want_dN else None
        dl = np.zeros(1)
        _load().orc_grad(self._h, X.shape[1], _ptr(X), _ptr(dY), _ptr(dS) if want_dS else None,
                         _ptr(dN) if want_dN else None, _ptr(dl))
        return dS, dN, float(dl[0])

    def forward_transform(self, X) -> np.ndarray:
        X = np.ascontiguousarray(X, dtype=np.float64)
        m = X.shape[1]
        xh = np.zeros((self.C, self.k, m))
        _load().orc_forward_transform(self._h, m, _ptr(X), _ptr(xh))
        return xh

    def dense(self) -> np.ndarray:
        if self.n > 8192:
            raise ValueError("dense assembly only for n <= 8192")
        A = np.zeros((self.n, self.n))
        _load().orc_dense(self._h, _ptr(A))
        return A

    def dense_dell(self) -> np.ndarray:
        if self.n > 8192:
            raise ValueError("dense assembly only for n <= 8192")
        A = np.zeros((self.n, self.n))
        _load().orc_dense_dell(self._h, _ptr(A))
        return A

    # -- solvers -----------------------------------------------------------
    def block_cg(self, B, X0=None, rtol=1e-8, max_iter=10000, freeze_converged=False):
        B = np.ascontiguousarray(B, dtype=np.float64)
        m = B.shape[1]
        X = np.zeros_like(B) if X0 is None else np.ascontiguousarray(X0, dtype=np.float64).copy()
        ci = np.zeros(m, np.int64)
        st = np.zeros(m, np.int32)
        it = _load().orc_block_cg(self._h, m, _ptr(B), _ptr(X), float(rtol), int(max_iter),
                                  int(bool(freeze_converged)), _ptr(ci), _ptr(st))
        return X, dict(iters=int(it), col_iters=ci, status=st)

    def block_cg_shared(self, B, X0=None, rtol=1e-8, max_iter=10000, drop=1e-6):
        """Block CG over one shared block Krylov space (m x m Gram matrices, Cholesky,
        Cholesky-QR orthonormalisation with deflation of dependent directions)."""
        B = np.ascontiguousarray(B, dtype=np.float64)
        m = B.shape[1]
        X = np.zeros_like(B) if X0 is None else np.ascontiguousarray(X0, dtype=np.float64).copy()
        rk = np.zeros(1, np.int64)
        st = np.zeros(m, np.int32)
        it = _load().orc_block_cg_shared(self._h, m, _ptr(B), _ptr(X), float(rtol), int(max_iter), float(drop),
                                         _ptr(rk), _ptr(st))
        return X, dict(iters=int(it), rank_min=int(rk[0]), status=st)

    def block_gmres(self, B, X0=None, rtol=1e-8, restart=30, max_iter=10000):
        """Block GMRES(restart) without a preconditioner: m independent GMRES processes
        sharing one product per Arnoldi step (classical Gram-Schmidt, Givens rotations,
        restart with the improved iterate)."""
        B = np.ascontiguousarray(B, dtype=np.float64)
        m = B.shape[1]
        X = np.zeros_like(B) if X0 is None else np.ascontiguousarray(X0, dtype=np.float64).copy()
        ci = np.zeros(m, np.int64)
        st = np.zeros(m, np.int32)
        est = np.zeros(m, np.float64)
        cyc = np.zeros(1, np.int64)
        it = _load().orc_block_gmres(self._h, m, _ptr(B), _ptr(X), float(rtol), int(restart), int(max_iter),
                                     _ptr(ci), _ptr(st), _ptr(est), _ptr(cyc))
        return X, dict(iters=int(it), cycles=int(cyc[0]), col_iters=ci, status=st, res_est=est)

    def matmul_complex(self, X, alpha=1.0) -> np.ndarray:
        """Y = alpha A X for the complex (Helmholtz) operator, X complex n x m."""
        X = np.ascontiguousarray(X, dtype=np.complex128)
        Xr = np.ascontiguousarray(X.view(np.float64).reshape(X.shape[0], -1))
        Y = np.zeros_like(Xr)
        _load().orc_matmul(self._h, Xr.shape[1], float(alpha), _ptr(Xr), 0.0, _ptr(Y))
        return Y.view(np.complex128)

    def dense_complex(self) -> np.ndarray:
        """The complex H^2 matrix assembled densely (small n only)."""
        A = np.zeros((self.n, 2 * self.n))
        _load().orc_dense_complex(self._h, _ptr(A))
        return A.view(np.complex128)

    def block_gmres_complex(self, B, X0=None, rtol=1e-8, restart=30, max_iter=10000):
        """Block GMRES(restart) over the complex numbers (conjugate inner product, complex
        Givens rotations) for the complex operator; B complex n x m."""
        B = np.ascontiguousarray(B, dtype=np.complex128)
        m = B.shape[1]
        Br = np.ascontiguousarray(B.view(np.float64).reshape(B.shape[0], -1))
        X = np.zeros_like(Br) if X0 is None else np.ascontiguousarray(
            np.ascontiguousarray(X0, dtype=np.complex128).view(np.float64).reshape(B.shape[0], -1)).copy()
        ci = np.zeros(m, np.int64)
        st = np.zeros(m, np.int32)
        est = np.zeros(m, np.float64)
        cyc = np.zeros(1, np.int64)
        it = _load().orc_block_gmres_c(self._h, m, _ptr(Br), _ptr(X), float(rtol), int(restart), int(max_iter),
                                       _ptr(ci), _ptr(st), _ptr(est), _ptr(cyc))
        return X.view(np.complex128), dict(iters=int(it), cycles=int(cyc[0]), col_iters=ci, status=st, res_est=est)

    def cg1(self, b, x0=None, rtol=1e-8, max_iter=10000):
        b = np.ascontiguousarray(b, dtype=np.float64).reshape(-1)
        x = np.zeros_like(b) if x0 is None else np.ascontiguousarray(x0, dtype=np.float64).reshape(-1).copy()
        it = _load().orc_cg1(self._h, _ptr(b), _ptr(x), float(rtol), int(max_iter))
        return x, int(it)


def round_bf16(values) -> np.ndarray:
    """The oracle's bfloat16 rounding of FP32 values (returned as FP32)."""
    a = np.ascontiguousarray(values, dtype=np.float32)
    out = np.empty_like(a)
    _load().orc_round_bf16_array(_ptr(a), _ptr(out), a.size)
    return out


def kernel_matrix(points, *, kernel="exp", ell=0.5, shift=1.0) -> np.ndarray:
    """The exact dense matrix g(x_i, x_j) + shift * delta_ij (no H^2 approximation); complex
    for the Helmholtz kernel."""
    P = np.asarray(points, dtype=np.float64)
    kern = _KERNELS[kernel] if isinstance(kernel, str) else int(kernel)
    if kern == KERNEL_EXP:
        D = np.sqrt(((P[:, None, :] - P[None, :, :]) ** 2).sum(-1))
        A = np.exp(-D / ell)
    elif kern == KERNEL_HELMHOLTZ:  # (4 pi / n) exp(i kappa r) / (4 pi r), kappa = ell; no self-interaction
        D = np.sqrt(((P[:, None, :] - P[None, :, :]) ** 2).sum(-1))
        with np.errstate(divide="ignore", invalid="ignore"):
            A = np.where(D > 0, np.exp(1j * ell * D) / (P.shape[0] * D), 0.0)
    elif kern == KERNEL_POLY:
        A = (1.0 + P @ P.T) ** 2
    else:
        A = np.ones((P.shape[0], P.shape[0]))
    A[np.diag_indices_from(A)] += shift
    return A
