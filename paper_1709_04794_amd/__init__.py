"""MI355X-native multi-shift solver for fast semi-supervised discriminant analysis.

Thin Python binding of ``libfsda.so`` (the C ABI declared in ``include/fsda.h``).
It only marshals arguments: every step of the solve runs in the library's HIP
kernels.  PyTorch provides device memory and the current stream.

    op = Operator.from_problem(problem)              # fsda_build_operator
    W, iters, relres, status = op.solve(betas, rtol)  # fsda_multishift_solve
    S = op.project(W)                                 # fsda_project

The library must have been built (``python -m paper_1709_04794_amd.build``);
importing the binding without it raises immediately.
"""
from __future__ import annotations

import ctypes
import os
import re
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfsda.so")
HEADER = os.path.join(os.path.dirname(_HERE), "include", "fsda.h")

OK, NOT_CONVERGED = 0, 1
E_ARG, E_CSR, E_LABELS, E_RANGE, E_BREAKDOWN, E_WORKSPACE, E_HIP, E_OVERFLOW = -1, -2, -3, -4, -5, -6, -7, -8
FP64, MIXED = 0, 1
MAX_SHIFTS, MAX_CHUNK, MAX_TARGETS, MAX_BATCH_CHUNK, MAX_COLUMNS = 64, 256, 4096, 128, 64
STATIC_SCRATCH_BYTES = 64 << 20  # FSDA_STATIC_SCRATCH_BYTES
# kernel classes for fsda_time_kernel
K_X, K_S, K_XT, K_XTL, K_RESID, K_PUPD, K_FOLD = 0, 1, 2, 3, 4, 5, 6
# ... and of the batched FP32 correction solves of the mixed path
K_BX, K_BS, K_BXT, K_BRESID, K_BPUPD = 7, 8, 9, 10, 11
# ... and the shift-state fold of fsda_multishift_solve_batch
K_TFOLD = 12
# ... and the assembly of the X^T rows cut into XCD slices (sample ranges per XCD)
K_ASM = 13


class FsdaError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__("fsda status %d: %s" % (code, msg))
        self.code = code


class Problem(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("d", ctypes.c_int64),
                ("x_rowptr", ctypes.c_void_p), ("x_col", ctypes.c_void_p), ("x_nnz", ctypes.c_int64),
                ("s_rowptr", ctypes.c_void_p), ("s_col", ctypes.c_void_p), ("s_nnz", ctypes.c_int64),
                ("lab_idx", ctypes.c_void_p), ("lab_y", ctypes.c_void_p), ("n_lab", ctypes.c_int64),
                ("alpha", ctypes.c_double), ("precision", ctypes.c_int)]


_lib = None


def lib():
    """The loaded libfsda.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libfsda.so is not built: run `python -m paper_1709_04794_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        P, I, D = ctypes.c_void_p, ctypes.c_int, ctypes.c_double
        pp = ctypes.POINTER(Problem)
        L.fsda_workspace_size.argtypes = [pp, I, I, ctypes.POINTER(ctypes.c_size_t)]
        L.fsda_build_operator.argtypes = [pp, I, I, P, ctypes.c_size_t, P, ctypes.POINTER(P)]
        L.fsda_rhs.argtypes = [P, P, P, P]
        L.fsda_apply.argtypes = [P, D, P, P, P]
        L.fsda_multishift_solve.argtypes = [P, P, P, I, D, I, I, P, P, P, P]
        L.fsda_project.argtypes = [P, P, I, P, P]
        L.fsda_time_kernel.argtypes = [P, I, I]
        L.fsda_kernel_time.argtypes = [P, ctypes.POINTER(D), ctypes.POINTER(ctypes.c_int64)]
        L.fsda_sa_rhs.argtypes = [P, P, P, P]
        L.fsda_sa_solve.argtypes = [P, P, P, I, D, I, I, P, P, P, P]
        L.fsda_regression_solve.argtypes = [P, P, P, I, D, I, I, I, P, P, P, P]
        L.fsda_columns_workspace_size.argtypes = [P, I, ctypes.POINTER(ctypes.c_size_t)]
        L.fsda_solve_columns.argtypes = [P, P, P, I, D, I, P, ctypes.c_size_t, P, P, P, P]
        L.fsda_holdout.argtypes = [P, P, I, P, P, ctypes.c_int64, P, P, P]
        L.fsda_hypergradient.argtypes = [P, P, P, P, I, P, P, P]
        L.fsda_batch_workspace_size.argtypes = [P, I, I, I, ctypes.POINTER(ctypes.c_size_t)]
        L.fsda_multishift_solve_batch.argtypes = [P, I, P, P, P, P, I, D, I, I, P, ctypes.c_size_t, P, P, P, P]
        L.fsda_solve_columns_static.argtypes = [P, P, P, I, D, I, P, P, P, P]
        L.fsda_solve_report.argtypes = [P, I, P, P, P]
        L.fsda_holdout_batch.argtypes = [P, I, P, I, P, P, P, P, P, P]
        L.fsda_columns_batch_workspace_size.argtypes = [P, I, I, ctypes.POINTER(ctypes.c_size_t)]
        L.fsda_solve_columns_batch.argtypes = [P, I, P, P, P, P, I, P, D, I, P, ctypes.c_size_t, P, P, P, P]
        L.fsda_hypergradient_batch.argtypes = [P, I, P, P, P, P, P, P, I, P, P, P]
        L.fsda_gather_sum.argtypes = [P, P, ctypes.c_int64, P, I, P]
        L.fsda_set_batch_tile.argtypes = [P, I]
        L.fsda_get_batch_tile.argtypes = [P, ctypes.POINTER(ctypes.c_int)]
        L.fsda_batch_autotune.argtypes = [P, I, P, P, P, P, I, I, P, ctypes.c_size_t, P, P,
                                          ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int), P]
        L.fsda_set_batch_groups.argtypes = [P, I]
        L.fsda_get_batch_groups.argtypes = [P, ctypes.POINTER(ctypes.c_int)]
        L.fsda_destroy_operator.argtypes = [P]
        L.fsda_destroy_operator.restype = None
        L.fsda_last_error.argtypes = []
        L.fsda_last_error.restype = ctypes.c_char_p
        for f in (L.fsda_workspace_size, L.fsda_build_operator, L.fsda_rhs, L.fsda_apply, L.fsda_multishift_solve,
                  L.fsda_project, L.fsda_time_kernel, L.fsda_kernel_time, L.fsda_batch_workspace_size,
                  L.fsda_multishift_solve_batch, L.fsda_sa_rhs, L.fsda_sa_solve, L.fsda_regression_solve,
                  L.fsda_columns_workspace_size, L.fsda_solve_columns, L.fsda_holdout, L.fsda_hypergradient,
                  L.fsda_gather_sum, L.fsda_set_batch_tile, L.fsda_get_batch_tile, L.fsda_batch_autotune,
                  L.fsda_holdout_batch, L.fsda_columns_batch_workspace_size, L.fsda_solve_columns_batch,
                  L.fsda_hypergradient_batch, L.fsda_solve_columns_static, L.fsda_solve_report,
                  L.fsda_set_batch_groups, L.fsda_get_batch_groups):
            f.restype = ctypes.c_int
        _lib = L
    return _lib


def declared_functions() -> list:
    """Names of the functions declared in include/fsda.h."""
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(fsda_\w+)\s*\(", txt, re.M)))


def _check(rc: int) -> int:
    if rc < 0:
        raise FsdaError(rc, lib().fsda_last_error().decode())
    return rc


def _stream(stream=None):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _ptr(t) -> Optional[ctypes.c_void_p]:
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def gather_sum(src, idx, grid: int = 2048, stream=None, part=None, checked: bool = False):
    """Per-block sums of src[idx] (fsda_gather_sum): a measurement aid for the
    rate of random 8-byte gathers.  src: contiguous CUDA float64, idx:
    contiguous CUDA int32 with every entry in [0, len(src)), checked here before
    the kernel reads them unless the caller has checked them (checked=True, so
    that a timed call enqueues the kernel alone).  part: optional CUDA float64
    output of `grid` entries."""
    import torch
    if src.dtype != torch.float64 or idx.dtype != torch.int32 or not (src.is_cuda and idx.is_cuda):
        raise TypeError("src must be CUDA float64 and idx CUDA int32")
    if not (src.is_contiguous() and idx.is_contiguous()):
        raise ValueError("src and idx must be contiguous")
    if not checked and idx.numel() and (int(idx.min()) < 0 or int(idx.max()) >= src.numel()):
        raise ValueError("idx entries outside [0, len(src))")
    if part is None:
        part = torch.empty(grid, dtype=torch.float64, device=src.device)
    elif part.dtype != torch.float64 or not part.is_cuda or part.numel() < grid:
        raise ValueError("part must be CUDA float64 with at least grid entries")
    _check(lib().fsda_gather_sum(_ptr(src), _ptr(idx), idx.numel(), _ptr(part), int(grid), _stream(stream)))
    return part


class Operator:
    """A built SDA operator on one GPU (fsda_build_operator).

    The CSR arrays (int32), labeled indices (int32) and labels (int8, +-1) are
    torch tensors on the GPU; the handle keeps references to them and owns a
    workspace tensor.
    """

    def __init__(self, n: int, d: int, x_rowptr, x_col, s_rowptr, s_col, lab_idx, lab_y, alpha: float,
                 precision: int = FP64, max_shifts: int = 32, max_chunk: int = 128, stream=None):
        import torch
        self.n, self.d = int(n), int(d)
        self.alpha = float(alpha)
        self.precision = precision
        self.max_shifts, self.max_chunk = int(max_shifts), int(max_chunk)
        self._keep = [x_rowptr, x_col, s_rowptr, s_col, lab_idx, lab_y]
        for t, dt in ((x_rowptr, torch.int32), (x_col, torch.int32), (s_rowptr, torch.int32), (s_col, torch.int32),
                      (lab_idx, torch.int32), (lab_y, torch.int8)):
            if t.dtype != dt or not t.is_cuda or not t.is_contiguous():
                raise TypeError("CSR and label arrays must be contiguous CUDA tensors of the documented dtypes")
        self.pb = Problem(self.n, self.d, x_rowptr.data_ptr(), x_col.data_ptr(), x_col.numel(),
                          s_rowptr.data_ptr(), s_col.data_ptr(), s_col.numel(),
                          lab_idx.data_ptr(), lab_y.data_ptr(), lab_idx.numel(), self.alpha, int(precision))
        size = ctypes.c_size_t(0)
        _check(lib().fsda_workspace_size(ctypes.byref(self.pb), self.max_shifts, self.max_chunk, ctypes.byref(size)))
        self.ws_bytes = int(size.value)
        self.ws = torch.empty(self.ws_bytes + 256, dtype=torch.uint8, device=x_col.device)
        base = self.ws.data_ptr()
        self._ws_ptr = (base + 255) // 256 * 256
        h = ctypes.c_void_p()
        _check(lib().fsda_build_operator(ctypes.byref(self.pb), self.max_shifts, self.max_chunk,
                                         ctypes.c_void_p(self._ws_ptr), ctypes.c_size_t(self.ws_bytes),
                                         _stream(stream), ctypes.byref(h)))
        self.handle = h
        self.device = x_col.device

    @classmethod
    def from_problem(cls, pb, precision: int = FP64, max_shifts: Optional[int] = None, max_chunk: int = 128,
                     device: str = "cuda", alpha: Optional[float] = None, **kw):
        """Uploads a ``synth.Problem``-like object (numpy arrays) and builds."""
        import torch

        def up(a, dt):
            return torch.from_numpy(np.ascontiguousarray(a)).to(device=device, dtype=dt)
        s_col = pb.s_col if pb.s_col.size else np.zeros(1, dtype=np.int32)
        x_col = pb.x_col if pb.x_col.size else np.zeros(1, dtype=np.int32)
        op = cls(pb.n, pb.d, up(pb.x_rowptr, torch.int32), up(x_col, torch.int32)[:pb.x_col.size],
                 up(pb.s_rowptr, torch.int32), up(s_col, torch.int32)[:pb.s_col.size],
                 up(pb.lab_idx, torch.int32), up(pb.lab_y, torch.int8), pb.alpha if alpha is None else alpha,
                 precision=precision,
                 max_shifts=max_shifts if max_shifts is not None else max(1, len(pb.betas)), max_chunk=max_chunk,
                 **kw)
        return op

    # -- calls -------------------------------------------------------------
    def rhs(self, r=None, stream=None):
        import torch
        b = torch.empty(self.d, dtype=torch.float64, device=self.device)
        _check(lib().fsda_rhs(self.handle, _ptr(r), _ptr(b), _stream(stream)))
        return b

    def apply(self, sigma: float, p, stream=None):
        import torch
        q = torch.empty(self.d, dtype=torch.float64, device=self.device)
        _check(lib().fsda_apply(self.handle, float(sigma), _ptr(p), _ptr(q), _stream(stream)))
        return q

    def solve(self, betas: Sequence[float], rtol: float, maxit: int = 100000, chunk: int = 0, b=None, out=None,
              stream=None):
        """Returns (W [S, d] float64 tensor, iters [S] int32, relres [S] float64, status)."""
        import torch
        betas = np.ascontiguousarray(betas, dtype=np.float64)
        S = betas.size
        W = out if out is not None else torch.empty((S, self.d), dtype=torch.float64, device=self.device)
        iters = np.zeros(S, dtype=np.int32)
        relres = np.zeros(S, dtype=np.float64)
        rc = _check(lib().fsda_multishift_solve(self.handle, _ptr(b), betas.ctypes.data_as(ctypes.c_void_p), S,
                                                float(rtol), int(maxit), int(chunk), _ptr(W),
                                                iters.ctypes.data_as(ctypes.c_void_p),
                                                relres.ctypes.data_as(ctypes.c_void_p), _stream(stream)))
        return W, iters, relres, rc

    def solve_report(self, nshift: int):
        """Per shift of the last solve: iterations of the shared recurrence, of the
        correction solve (mixed path), refinement steps taken (fsda_solve_report)."""
        out = [np.zeros(int(nshift), dtype=np.int32) for _ in range(3)]
        _check(lib().fsda_solve_report(self.handle, int(nshift), *[o.ctypes.data_as(ctypes.c_void_p) for o in out]))
        return {"main_iters": out[0], "refine_iters": out[1], "steps": out[2]}

    def sa_rhs(self, r=None, stream=None):
        """Right-hand side of the sample-space solve (Alg. sasda): y_c, or the printed one for start vector r."""
        import torch
        g = torch.empty(self.n, dtype=torch.float64, device=self.device)
        _check(lib().fsda_sa_rhs(self.handle, _ptr(r), _ptr(g), _stream(stream)))
        return g

    def sa_solve(self, betas: Sequence[float], rtol: float, maxit: int = 100000, chunk: int = 0, g=None,
                 stream=None):
        """Ratings of the samples by the sample-space solve (Alg. sasda).

        Returns (Z [S, n] float64 tensor, iters [S] int32, relres [S] float64, status)."""
        import torch
        betas = np.ascontiguousarray(betas, dtype=np.float64)
        S = betas.size
        Z = torch.empty((S, self.n), dtype=torch.float64, device=self.device)
        iters = np.zeros(S, dtype=np.int32)
        relres = np.zeros(S, dtype=np.float64)
        rc = _check(lib().fsda_sa_solve(self.handle, _ptr(g), betas.ctypes.data_as(ctypes.c_void_p), S, float(rtol),
                                        int(maxit), int(chunk), _ptr(Z), iters.ctypes.data_as(ctypes.c_void_p),
                                        relres.ctypes.data_as(ctypes.c_void_p), _stream(stream)))
        return Z, iters, relres, rc

    def regression_solve(self, z, betas: Sequence[float], rtol: float, maxit: int = 100000, chunk: int = 0,
                         shared_basis: bool = True, stream=None):
        """(X^T X + beta I) w = X^T z for every beta (fsda_regression_solve).

        Returns (W [S, d] float64 tensor, iters [S] int32, relres [S] float64, status)."""
        import torch
        betas = np.ascontiguousarray(betas, dtype=np.float64)
        S = betas.size
        W = torch.empty((S, self.d), dtype=torch.float64, device=self.device)
        iters = np.zeros(S, dtype=np.int32)
        relres = np.zeros(S, dtype=np.float64)
        rc = _check(lib().fsda_regression_solve(self.handle, _ptr(z), betas.ctypes.data_as(ctypes.c_void_p), S,
                                                float(rtol), int(maxit), int(chunk), int(bool(shared_basis)), _ptr(W),
                                                iters.ctypes.data_as(ctypes.c_void_p),
                                                relres.ctypes.data_as(ctypes.c_void_p), _stream(stream)))
        return W, iters, relres, rc

    def solve_columns(self, B, sigmas: Sequence[float], rtol: float, maxit: int = 100000, stream=None):
        """A(sigma_c) x_c = b_c for the rows b_c of B [ncol, d] (fsda_solve_columns).

        Returns (X [ncol, d] float64 tensor, iters [ncol] int32, relres [ncol] float64, status)."""
        import torch
        B = B.contiguous()
        sig = np.ascontiguousarray(sigmas, dtype=np.float64)
        K = sig.size
        size = ctypes.c_size_t(0)
        _check(lib().fsda_columns_workspace_size(self.handle, K, ctypes.byref(size)))
        need = int(size.value) + 256
        if getattr(self, "_cws", None) is None or self._cws.numel() < need:
            self._cws = None
            self._cws = torch.empty(need, dtype=torch.uint8, device=self.device)
        ws = (self._cws.data_ptr() + 255) // 256 * 256
        X = torch.empty((K, self.d), dtype=torch.float64, device=self.device)
        iters = np.zeros(K, dtype=np.int32)
        relres = np.zeros(K, dtype=np.float64)
        rc = _check(lib().fsda_solve_columns(self.handle, _ptr(B), sig.ctypes.data_as(ctypes.c_void_p), K, float(rtol),
                                             int(maxit), ctypes.c_void_p(ws), ctypes.c_size_t(int(size.value)),
                                             _ptr(X), iters.ctypes.data_as(ctypes.c_void_p),
                                             relres.ctypes.data_as(ctypes.c_void_p), _stream(stream)))
        return X, iters, relres, rc

    def solve_columns_static(self, B, sigmas: Sequence[float], rtol: float, maxit: int = 100000, stream=None):
        """solve_columns with the library's static scratch instead of a workspace
        (fsda_solve_columns_static; allocates nothing but the outputs made here)."""
        import torch
        B = B.contiguous()
        sig = np.ascontiguousarray(sigmas, dtype=np.float64)
        K = sig.size
        X = torch.empty((K, self.d), dtype=torch.float64, device=self.device)
        iters = np.zeros(K, dtype=np.int32)
        relres = np.zeros(K, dtype=np.float64)
        rc = _check(lib().fsda_solve_columns_static(self.handle, _ptr(B), sig.ctypes.data_as(ctypes.c_void_p), K,
                                                    float(rtol), int(maxit), _ptr(X),
                                                    iters.ctypes.data_as(ctypes.c_void_p),
                                                    relres.ctypes.data_as(ctypes.c_void_p), _stream(stream)))
        return X, iters, relres, rc

    def holdout(self, W, ho_idx, ho_y, gradient: bool = True, stream=None):
        """Hold-out loss per row of W and (optionally) its gradient in w (fsda_holdout)."""
        import torch
        W = W.contiguous()
        S = W.shape[0]
        loss = np.zeros(S, dtype=np.float64)
        G = torch.empty((S, self.d), dtype=torch.float64, device=self.device) if gradient else None
        _check(lib().fsda_holdout(self.handle, _ptr(W), S, _ptr(ho_idx), _ptr(ho_y), int(ho_idx.numel()),
                                  loss.ctypes.data_as(ctypes.c_void_p), _ptr(G), _stream(stream)))
        return loss, G

    def hypergradient(self, W, Lam, betas: Sequence[float], stream=None):
        """(dH/dlog beta [S], dH/dalpha [S]) from solutions and adjoint solutions (fsda_hypergradient)."""
        betas = np.ascontiguousarray(betas, dtype=np.float64)
        S = betas.size
        dlb = np.zeros(S, dtype=np.float64)
        da = np.zeros(S, dtype=np.float64)
        _check(lib().fsda_hypergradient(self.handle, _ptr(W.contiguous()), _ptr(Lam.contiguous()),
                                        betas.ctypes.data_as(ctypes.c_void_p), S, dlb.ctypes.data_as(ctypes.c_void_p),
                                        da.ctypes.data_as(ctypes.c_void_p), _stream(stream)))
        return dlb, da

    def solve_batch(self, labels, betas: Sequence[float], rtol: float, maxit: int = 100000, chunk: int = 0,
                    stream=None):
        """Several targets over this operator's X and S (fsda_multishift_solve_batch).

        ``labels`` is a list of (lab_idx, lab_y) pairs (numpy arrays or tensors;
        int32 indices, +-1 labels), one per target, at most MAX_TARGETS.
        Returns (W [ntarget, S, d] float64 tensor, iters [ntarget, S] int32,
        relres [ntarget, S] float64, status).
        """
        import torch
        lab_idx, lab_y, off = self._labels(labels)
        betas = np.ascontiguousarray(betas, dtype=np.float64)
        S, K = betas.size, len(labels)
        ws, size = self._batch_workspace(K, S, chunk)
        W = torch.empty((K, S, self.d), dtype=torch.float64, device=self.device)
        iters = np.zeros(K * S, dtype=np.int32)
        relres = np.zeros(K * S, dtype=np.float64)
        rc = _check(lib().fsda_multishift_solve_batch(
            self.handle, K, _ptr(lab_idx), _ptr(lab_y), off.ctypes.data_as(ctypes.c_void_p),
            betas.ctypes.data_as(ctypes.c_void_p), S, float(rtol), int(maxit), int(chunk), ctypes.c_void_p(ws),
            ctypes.c_size_t(size), _ptr(W), iters.ctypes.data_as(ctypes.c_void_p),
            relres.ctypes.data_as(ctypes.c_void_p), _stream(stream)))
        return W, iters.reshape(K, S), relres.reshape(K, S), rc

    def holdout_batch(self, W, heldout, gradient: bool = True, stream=None):
        """Hold-out loss of every (target, shift) (fsda_holdout_batch).

        W [ntarget, S, d] from solve_batch; ``heldout`` a list of (ho_idx, ho_y)
        pairs, one per target (int32 rows, float64 targets).  Returns (loss
        [ntarget, S] numpy, G [ntarget, S, d] tensor or None)."""
        import torch
        W = W.contiguous()
        K, S = W.shape[0], W.shape[1]
        if len(heldout) != K:
            raise ValueError("one held-out set per target")
        idx = [torch.as_tensor(np.asarray(i.cpu() if hasattr(i, "cpu") else i), dtype=torch.int32) for i, _ in heldout]
        ys = [torch.as_tensor(np.asarray(y.cpu() if hasattr(y, "cpu") else y), dtype=torch.float64) for _, y in heldout]
        off = np.zeros(K + 1, dtype=np.int64)
        off[1:] = np.cumsum([i.numel() for i in idx])
        hi, hy = torch.cat(idx).to(self.device), torch.cat(ys).to(self.device)
        loss = np.zeros(K * S, dtype=np.float64)
        G = torch.empty((K, S, self.d), dtype=torch.float64, device=self.device) if gradient else None
        _check(lib().fsda_holdout_batch(self.handle, K, _ptr(W), S, _ptr(hi), _ptr(hy),
                                        off.ctypes.data_as(ctypes.c_void_p), loss.ctypes.data_as(ctypes.c_void_p),
                                        _ptr(G), _stream(stream)))
        return loss.reshape(K, S), G

    def solve_columns_batch(self, labels, betas: Sequence[float], B, rtol: float, maxit: int = 100000, stream=None):
        """A_c(beta_s) x_cs = B_cs for every (target c, shift s) (fsda_solve_columns_batch):
        ``labels`` as in solve_batch, B [ntarget, S, d].  Returns (X [ntarget, S, d],
        iters [ntarget, S], relres [ntarget, S], status)."""
        import torch
        lab_idx, lab_y, off = self._labels(labels)
        betas = np.ascontiguousarray(betas, dtype=np.float64)
        S, K = betas.size, len(labels)
        B = B.contiguous()
        if tuple(B.shape) != (K, S, self.d):
            raise ValueError("B must be [ntarget, nshift, d]")
        size = ctypes.c_size_t(0)
        _check(lib().fsda_columns_batch_workspace_size(self.handle, K, S, ctypes.byref(size)))
        need = int(size.value) + 256
        if getattr(self, "_cbws", None) is None or self._cbws.numel() < need:
            self._cbws = None
            self._cbws = torch.empty(need, dtype=torch.uint8, device=self.device)
        ws = (self._cbws.data_ptr() + 255) // 256 * 256
        X = torch.empty((K, S, self.d), dtype=torch.float64, device=self.device)
        iters = np.zeros(K * S, dtype=np.int32)
        relres = np.zeros(K * S, dtype=np.float64)
        rc = _check(lib().fsda_solve_columns_batch(
            self.handle, K, _ptr(lab_idx), _ptr(lab_y), off.ctypes.data_as(ctypes.c_void_p),
            betas.ctypes.data_as(ctypes.c_void_p), S, _ptr(B), float(rtol), int(maxit), ctypes.c_void_p(ws),
            ctypes.c_size_t(int(size.value)), _ptr(X), iters.ctypes.data_as(ctypes.c_void_p),
            relres.ctypes.data_as(ctypes.c_void_p), _stream(stream)))
        return X, iters.reshape(K, S), relres.reshape(K, S), rc

    def hypergradient_batch(self, labels, W, Lam, betas: Sequence[float], stream=None):
        """(dH/dlog beta [ntarget, S], dH/dalpha [ntarget, S]) per target (fsda_hypergradient_batch)."""
        lab_idx, lab_y, off = self._labels(labels)
        betas = np.ascontiguousarray(betas, dtype=np.float64)
        S, K = betas.size, len(labels)
        dlb = np.zeros(K * S, dtype=np.float64)
        da = np.zeros(K * S, dtype=np.float64)
        _check(lib().fsda_hypergradient_batch(self.handle, K, _ptr(lab_idx), _ptr(lab_y),
                                              off.ctypes.data_as(ctypes.c_void_p), _ptr(W.contiguous()),
                                              _ptr(Lam.contiguous()), betas.ctypes.data_as(ctypes.c_void_p), S,
                                              dlb.ctypes.data_as(ctypes.c_void_p), da.ctypes.data_as(ctypes.c_void_p),
                                              _stream(stream)))
        return dlb.reshape(K, S), da.reshape(K, S)

    def _labels(self, labels):
        """(lab_idx, lab_y) pairs of several targets -> concatenated device arrays and host offsets."""
        import torch
        if not 1 <= len(labels) <= MAX_TARGETS:
            raise ValueError("between 1 and %d targets per call" % MAX_TARGETS)
        idx = [torch.as_tensor(np.asarray(i.cpu() if hasattr(i, "cpu") else i), dtype=torch.int32) for i, _ in labels]
        ys = [torch.as_tensor(np.asarray(y.cpu() if hasattr(y, "cpu") else y), dtype=torch.int8) for _, y in labels]
        off = np.zeros(len(labels) + 1, dtype=np.int64)
        off[1:] = np.cumsum([i.numel() for i in idx])
        return torch.cat(idx).to(self.device), torch.cat(ys).to(self.device), off

    def _batch_workspace(self, K: int, S: int, chunk: int):
        """Device address (256-byte aligned) and size of the batch workspace for the tile in use."""
        import torch
        size = ctypes.c_size_t(0)
        _check(lib().fsda_batch_workspace_size(self.handle, K, S, int(chunk), ctypes.byref(size)))
        need = int(size.value) + 256
        if getattr(self, "_bws", None) is None or self._bws.numel() < need:
            self._bws = None
            self._bws = torch.empty(need, dtype=torch.uint8, device=self.device)
        return (self._bws.data_ptr() + 255) // 256 * 256, int(size.value)

    def set_batch_tile(self, tile: int) -> None:
        """Targets per tile of solve_batch: 4, 8 or 16, or 0 for the default (fsda_set_batch_tile)."""
        _check(lib().fsda_set_batch_tile(self.handle, int(tile)))

    @property
    def batch_tile(self) -> int:
        t = ctypes.c_int(0)
        _check(lib().fsda_get_batch_tile(self.handle, ctypes.byref(t)))
        return int(t.value)

    def set_batch_groups(self, groups: int) -> None:
        """Groups of tile lanes per row of solve_batch's row products: 1, 2 or 4, or 0 for
        the default (fsda_set_batch_groups)."""
        _check(lib().fsda_set_batch_groups(self.handle, int(groups)))

    @property
    def batch_groups(self) -> int:
        g = ctypes.c_int(0)
        _check(lib().fsda_get_batch_groups(self.handle, ctypes.byref(g)))
        return int(g.value)

    def autotune_batch(self, labels, betas: Sequence[float], trial_iters: int = 32, stream=None):
        """Times tiles of 4, 8 and 16 targets with 1, 2 and 4 groups of lanes per row on these
        targets (fsda_batch_autotune) and keeps the fastest shape for solve_batch.  Returns
        (tile, groups, {(tile, groups): shifted target-iterations per s})."""
        import torch
        lab_idx, lab_y, off = self._labels(labels)
        betas = np.ascontiguousarray(betas, dtype=np.float64)
        S, K = betas.size, len(labels)
        self.set_batch_tile(0)  # the workspace of the largest tile tried
        ws, size = self._batch_workspace(K, S, 0)
        W = torch.empty((min(K, 16), S, self.d), dtype=torch.float64, device=self.device)
        tile, groups = ctypes.c_int(0), ctypes.c_int(0)
        rates = np.zeros(9, dtype=np.float64)
        _check(lib().fsda_batch_autotune(self.handle, K, _ptr(lab_idx), _ptr(lab_y), off.ctypes.data_as(ctypes.c_void_p),
                                         betas.ctypes.data_as(ctypes.c_void_p), S, int(trial_iters),
                                         ctypes.c_void_p(ws), ctypes.c_size_t(size), _ptr(W), _stream(stream),
                                         ctypes.byref(tile), ctypes.byref(groups),
                                         rates.ctypes.data_as(ctypes.c_void_p)))
        shapes = [(t, g) for t in (4, 8, 16) for g in (1, 2, 4)]
        return int(tile.value), int(groups.value), {sh: float(r) for sh, r in zip(shapes, rates) if r > 0}

    def project(self, W, stream=None):
        import torch
        W = W.contiguous()
        S = W.shape[0]
        out = torch.empty((S, self.n), dtype=torch.float64, device=self.device)
        _check(lib().fsda_project(self.handle, _ptr(W), S, _ptr(out), _stream(stream)))
        return out

    def time_kernel(self, kernel: int, enable: bool = True, every: int = 1):
        """Events around every `every`-th launch of kernel class `kernel` (off when not enable)."""
        _check(lib().fsda_time_kernel(self.handle, int(kernel), int(every) if enable else 0))

    def kernel_time(self):
        ms = ctypes.c_double(0)
        n = ctypes.c_int64(0)
        _check(lib().fsda_kernel_time(self.handle, ctypes.byref(ms), ctypes.byref(n)))
        return ms.value, n.value

    def close(self):
        if getattr(self, "handle", None):
            lib().fsda_destroy_operator(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
