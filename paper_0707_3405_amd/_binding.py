"""ctypes binding of libpwlobpcg.so (include/pwlobpcg.h).

Argument marshalling only: every step of the computation runs in the library's
HIP kernels.  PyTorch supplies device memory and the HIP stream.

Block vectors are complex128 CUDA tensors of shape (nb, ld): row j is band j,
which is the library's column-major [ld x nb] layout with leading dimension ld
(>= npw).  Small matrices passed to the building-block calls follow the same
rule: a (q, ldc) tensor is a column-major [ldc x q] matrix.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libpwlobpcg.so")

PW_OK, PW_ERR_ARG, PW_ERR_STATE, PW_ERR_NOMEM, PW_ERR_DEVICE, PW_ERR_NOT_CONVERGED, PW_ERR_NUMERIC = range(7)
STATUS_NAMES = {0: "PW_OK", 1: "PW_ERR_ARG", 2: "PW_ERR_STATE", 3: "PW_ERR_NOMEM",
                4: "PW_ERR_DEVICE", 5: "PW_ERR_NOT_CONVERGED", 6: "PW_ERR_NUMERIC"}
PW_PREC_FP64, PW_PREC_MIXED, PW_PREC_MIXED_BF16, PW_PREC_MIXED_BF16_GRAM, PW_PREC_MIXED_FP32_RR = 0, 1, 2, 3, 4

EXPORTS = ("pw_create", "pw_destroy", "pw_last_error", "pw_init_basis", "pw_fft_sizes",
           "pw_get_miller", "pw_get_kinetic", "pw_set_local_potential", "pw_set_projectors",
           "pw_workspace_size", "pw_set_workspace", "pw_apply_H", "pw_lobpcg_solve",
           "pw_get_residuals", "pw_get_stats", "pw_gram", "pw_block_update", "pw_small_eigh",
           "pw_residuals", "pw_gram_mixed", "pw_block_update_mixed", "pw_lobpcg_solve_batch",
           "pw_density", "pw_set_overlap", "pw_apply_O", "pw_chol_inv", "pw_autotune",
           "pw_set_tuning", "pw_small_eigh_noalloc", "pw_apply_H_batch", "pw_set_phase_timing")


class PWError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")
        self.status = status
        self.message = message


class PWTuning(ctypes.Structure):
    _fields_ = [("fft_sticks_per_block", ctypes.c_int32), ("fft_plane_rows", ctypes.c_int32),
                ("gemm_split_workgroups", ctypes.c_int32), ("apply_ms_default", ctypes.c_double),
                ("apply_ms_tuned", ctypes.c_double), ("gemm_ms_default", ctypes.c_double),
                ("gemm_ms_tuned", ctypes.c_double), ("fft_radix2", ctypes.c_int32)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class PWStats(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int32), ("blocks", ctypes.c_int32),
                ("h_applies", ctypes.c_int32), ("p_restarts", ctypes.c_int32),
                ("ms_total", ctypes.c_double), ("ms_apply", ctypes.c_double),
                ("ms_gemm", ctypes.c_double), ("ms_dense", ctypes.c_double),
                ("ms_vec", ctypes.c_double), ("ms_final_rr", ctypes.c_double),
                ("mixed_iterations", ctypes.c_int32)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


_lib = None


def library_path() -> str:
    return _LIB_PATH


def load_library():
    """Load libpwlobpcg.so; raises ImportError if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        raise ImportError(f"{_LIB_PATH} is missing: run __graft_entry__.build() first")
    lib = ctypes.CDLL(_LIB_PATH)
    P, I32, I64, D, SZ = (ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double,
                          ctypes.c_size_t)
    sig = {
        "pw_create": (ctypes.c_int, [ctypes.c_int, P, ctypes.POINTER(P)]),
        "pw_destroy": (None, [P]),
        "pw_last_error": (ctypes.c_char_p, [P]),
        "pw_init_basis": (ctypes.c_int, [P, P, P, D, P, ctypes.POINTER(I64)]),
        "pw_fft_sizes": (ctypes.c_int, [P, I32, ctypes.POINTER(I32)]),
        "pw_get_miller": (ctypes.c_int, [P, P]),
        "pw_get_kinetic": (ctypes.c_int, [P, P]),
        "pw_set_local_potential": (ctypes.c_int, [P, P, ctypes.c_int]),
        "pw_set_projectors": (ctypes.c_int, [P, I32, P, I32, P, P]),
        "pw_workspace_size": (ctypes.c_int, [P, I32, I32, ctypes.c_int, ctypes.POINTER(SZ)]),
        "pw_set_workspace": (ctypes.c_int, [P, P, SZ]),
        "pw_apply_H": (ctypes.c_int, [P, P, I64, P, I64, I32, ctypes.c_int]),
        "pw_apply_O": (ctypes.c_int, [P, P, I64, P, I64, I32, ctypes.c_int]),
        "pw_apply_H_batch": (ctypes.c_int, [P, I32, P, P, P, P, I32, ctypes.c_int]),
        "pw_set_overlap": (ctypes.c_int, [P, P]),
        "pw_chol_inv": (ctypes.c_int, [P, P, I64, I32, P, I64]),
        "pw_autotune": (ctypes.c_int, [P, I32, ctypes.POINTER(PWTuning)]),
        "pw_set_tuning": (ctypes.c_int, [P, ctypes.POINTER(PWTuning)]),
        "pw_lobpcg_solve": (ctypes.c_int, [P, I32, I32, D, I32, ctypes.c_int, P, I64, I32, P]),
        "pw_get_residuals": (ctypes.c_int, [P, P]),
        "pw_get_stats": (ctypes.c_int, [P, ctypes.POINTER(PWStats)]),
        "pw_set_phase_timing": (ctypes.c_int, [P, I32]),
        "pw_gram": (ctypes.c_int, [P, P, I64, P, I64, I64, I32, I32, P, I64]),
        "pw_block_update": (ctypes.c_int, [P, P, I64, P, I64, I64, I32, I32, D, D, P, I64]),
        "pw_gram_mixed": (ctypes.c_int, [P, P, I64, P, I64, I64, I32, I32, P, I64]),
        "pw_lobpcg_solve_batch": (ctypes.c_int, [P, I32, I32, I32, D, I32, ctypes.c_int, P, P, I32, P, P]),
        "pw_density": (ctypes.c_int, [P, P, I64, I32, P, P]),
        "pw_block_update_mixed": (ctypes.c_int, [P, P, I64, P, I64, I64, I32, I32, D, D, P, I64]),
        "pw_small_eigh": (ctypes.c_int, [P, P, I64, I32, I32, P, P, I64]),
        "pw_small_eigh_noalloc": (ctypes.c_int, [P, P, I64, I32, I32, P, P, I64]),
        "pw_residuals": (ctypes.c_int, [P, P, I64, P, I64, I32, P, P, P, I64]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def apply_H_batch(ctxs, Xs, Ys, nb=None, prec=PW_PREC_FP64):
    """Y_k = H_k X_k for the contexts of one cell's k-points in one call
    (pw_apply_H_batch): X_k, Y_k are [nb, npw_k] tensors as for Context.apply_H;
    the contexts share a device, a stream and an FFT grid."""
    if not (len(ctxs) == len(Xs) == len(Ys)) or not ctxs:
        raise ValueError("need one X and one Y per context")
    nb = Xs[0].shape[0] if nb is None else nb
    dt = _block_dtype_name(prec)
    for c, X, Y in zip(ctxs, Xs, Ys):
        c._check_tensors([("X", X, dt, nb, c.npw, None), ("Y", Y, dt, nb, c.npw, None)])
    n = len(ctxs)
    hs = (ctypes.c_void_p * n)(*[c.h.value for c in ctxs])
    xp = (ctypes.c_void_p * n)(*[_ptr(X).value for X in Xs])
    yp = (ctypes.c_void_p * n)(*[_ptr(Y).value for Y in Ys])
    lx = (ctypes.c_int64 * n)(*[_ld(X) for X in Xs])
    ly = (ctypes.c_int64 * n)(*[_ld(Y) for Y in Ys])
    ctxs[0]._check(ctxs[0].lib.pw_apply_H_batch(hs, n, xp, lx, yp, ly, nb, prec))
    return Ys


def fft_sizes():
    lib = load_library()
    cnt = ctypes.c_int32(0)
    buf = (ctypes.c_int32 * 64)()
    lib.pw_fft_sizes(buf, 64, ctypes.byref(cnt))
    return [buf[i] for i in range(cnt.value)]


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


def _ld(t):
    """Leading dimension of a (ncol, ld) tensor with unit stride in ld."""
    if t.dim() == 1:
        return t.shape[0]
    if t.shape[1] > 1 and t.stride(1) != 1:
        raise ValueError("block tensors must have unit stride along the row")
    if t.shape[0] <= 1:          # a single column: any leading dimension >= rows
        return max(t.shape[1], 1)
    return t.stride(0)


def _block_dtype_name(prec):
    return "complex128" if prec == PW_PREC_FP64 else "complex64"


class Context:
    """One pw_ctx bound to a device and a HIP stream (default: torch's current)."""

    def __init__(self, device: int = 0, stream=None):
        """device < 0 makes a host-only context (basis tables only, no kernels)."""
        self.lib = load_library()
        if device >= 0:
            import torch
            self._torch = torch
            if stream is None:
                stream = torch.cuda.current_stream(device)
            handle = stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream)
        else:
            self._torch = None
            handle = 0
        self.stream = stream
        h = ctypes.c_void_p()
        self._check(self.lib.pw_create(device, ctypes.c_void_p(handle), ctypes.byref(h)), ctx=False)
        self.h = h
        self.device = device
        self.npw = 0
        self._ws = None
        self._keep = []

    def _check_tensors(self, specs):
        """Refuse, before any library call, tensors the library would read or write
        out of bounds or in the wrong element type.  specs: (name, tensor, dtype,
        ncols, nrows, numel) -- wrong dtype, fewer than `ncols` columns (bands) or
        `nrows` rows per column, fewer than `numel` elements (contiguous), then
        memory that is not on this context's device."""
        import torch
        for name, t, dtype, ncols, nrows, numel in specs:
            if not isinstance(t, torch.Tensor):
                raise ValueError(f"{name} must be a torch tensor")
            if t.dtype != getattr(torch, dtype):
                raise ValueError(f"{name} must be {dtype}, got {t.dtype}")
            if numel is not None:
                if t.numel() < numel or not t.is_contiguous():
                    raise ValueError(f"{name} must be contiguous with {numel} elements, "
                                     f"got {tuple(t.shape)}")
                continue
            if t.dim() not in (1, 2):
                raise ValueError(f"{name} must be a (columns, rows) tensor, got {tuple(t.shape)}")
            cols = 1 if t.dim() == 1 else t.shape[0]
            rows = t.shape[-1]
            if ncols is not None and cols < ncols:
                raise ValueError(f"{name} has {cols} columns, the call needs {ncols}")
            if nrows is not None and ncols != 0 and rows < nrows:
                raise ValueError(f"{name} has {rows} rows per column, the call needs {nrows}")
        for name, t, *_ in specs:
            if not t.is_cuda or t.device.index != self.device:
                raise ValueError(f"{name} must be on cuda:{self.device}, got {t.device}")

    def _check(self, status, ctx=True, allow=()):
        if status == PW_OK or status in allow:
            return status
        msg = self.lib.pw_last_error(self.h).decode() if ctx and getattr(self, "h", None) else ""
        raise PWError(status, msg)

    def close(self):
        if getattr(self, "h", None):
            self.lib.pw_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---- setup ---------------------------------------------------------------
    def init_basis(self, cell, kfrac, ecut, fft_n):
        cell = np.ascontiguousarray(np.asarray(cell, np.float64).reshape(9))
        kf = np.ascontiguousarray(np.asarray(kfrac, np.float64).reshape(3))
        n = np.ascontiguousarray(np.asarray(fft_n, np.int32).reshape(3))
        npw = ctypes.c_int64(0)
        self._check(self.lib.pw_init_basis(self.h, cell.ctypes.data, kf.ctypes.data, float(ecut),
                                           n.ctypes.data, ctypes.byref(npw)))
        self.npw = npw.value
        self.fft_n = tuple(int(x) for x in n)
        self._ws = None
        return self.npw

    def grid_n(self):
        """FFT grid (n0, n1, n2) of the current basis ((0, 0, 0) before init_basis)."""
        return getattr(self, "fft_n", (0, 0, 0))

    def get_miller(self):
        out = np.zeros((self.npw, 3), np.int32)
        self._check(self.lib.pw_get_miller(self.h, out.ctypes.data))
        return out

    def get_kinetic(self):
        out = np.zeros(self.npw, np.float64)
        self._check(self.lib.pw_get_kinetic(self.h, out.ctypes.data))
        return out

    def set_local_potential(self, v):
        torch = self._torch
        if torch is not None and isinstance(v, torch.Tensor) and v.is_cuda:
            v = v.contiguous()
            self._check(self.lib.pw_set_local_potential(self.h, _ptr(v), 1))
        else:
            arr = np.ascontiguousarray(np.asarray(v, np.float64))
            self._check(self.lib.pw_set_local_potential(self.h, arr.ctypes.data, 0))

    def set_projectors(self, pos, lm, D):
        if pos is None or len(lm) == 0:
            self._check(self.lib.pw_set_projectors(self.h, 0, None, 0, None, None))
            return
        pos = np.ascontiguousarray(np.asarray(pos, np.float64))
        lm = np.ascontiguousarray(np.asarray(lm, np.int32))
        D = np.ascontiguousarray(np.asarray(D, np.float64))
        self._check(self.lib.pw_set_projectors(self.h, pos.shape[0], pos.ctypes.data, lm.shape[0],
                                               lm.ctypes.data, D.ctypes.data))

    def set_overlap(self, q):
        """O = I + sum_p q_p |beta_p><beta_p| (None: O = I); size the workspace afterwards."""
        if q is None:
            self._check(self.lib.pw_set_overlap(self.h, None))
            return
        q = np.ascontiguousarray(np.asarray(q, np.float64))
        self._check(self.lib.pw_set_overlap(self.h, q.ctypes.data))

    def workspace_size(self, nbands, block, prec=PW_PREC_FP64):
        out = ctypes.c_size_t(0)
        self._check(self.lib.pw_workspace_size(self.h, nbands, block, prec, ctypes.byref(out)))
        return out.value

    def set_workspace(self, tensor):
        self._check(self.lib.pw_set_workspace(self.h, _ptr(tensor), tensor.numel() * tensor.element_size()))
        self._ws = tensor

    def alloc_workspace(self, nbands, block, prec=PW_PREC_FP64):
        torch = self._torch
        nbytes = self.workspace_size(nbands, block, prec)
        ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=f"cuda:{self.device}")
        off = (-ws.data_ptr()) % 256
        ws = ws[off:off + nbytes]
        self.set_workspace(ws)
        return ws

    # ---- hot path --------------------------------------------------------------
    def apply_H(self, X, Y, nb=None, prec=PW_PREC_FP64):
        nb = X.shape[0] if nb is None else nb
        dt = _block_dtype_name(prec)
        self._check_tensors([("X", X, dt, nb, self.npw, None), ("Y", Y, dt, nb, self.npw, None)])
        self._check(self.lib.pw_apply_H(self.h, _ptr(X), _ld(X), _ptr(Y), _ld(Y), nb, prec))
        return Y

    def apply_O(self, X, Y, nb=None, prec=PW_PREC_FP64):
        nb = X.shape[0] if nb is None else nb
        dt = _block_dtype_name(prec)
        self._check_tensors([("X", X, dt, nb, self.npw, None), ("Y", Y, dt, nb, self.npw, None)])
        self._check(self.lib.pw_apply_O(self.h, _ptr(X), _ld(X), _ptr(Y), _ld(Y), nb, prec))
        return Y

    def lobpcg_solve(self, nbands, block, tol, max_iter, X, use_guess=False, prec=PW_PREC_FP64,
                     allow_not_converged=False):
        self._check_tensors([("X", X, "complex128", max(int(nbands), 0), self.npw, None)])
        eig = np.zeros(max(int(nbands), 0), np.float64)
        allow = (PW_ERR_NOT_CONVERGED,) if allow_not_converged else ()
        st = self._check(self.lib.pw_lobpcg_solve(self.h, nbands, block, float(tol), max_iter, prec,
                                                  _ptr(X), _ld(X), int(bool(use_guess)),
                                                  eig.ctypes.data), allow=allow)
        return eig, st

    def density(self, X, occ, rho, nb=None):
        """rho (device float64 [N, N, N]) = sum_n occ[n] |psi_n(r)|^2 of the columns of X."""
        nb = X.shape[0] if nb is None else nb
        occ = np.ascontiguousarray(np.asarray(occ, np.float64)).reshape(-1)
        if occ.size < nb:
            raise ValueError(f"occ has {occ.size} entries, the call needs {nb}")
        n = self.grid_n()
        self._check_tensors([("X", X, "complex128", nb, self.npw, None),
                             ("rho", rho, "float64", None, None, n[0] * n[1] * n[2])])
        self._check(self.lib.pw_density(self.h, _ptr(X), _ld(X), nb, occ.ctypes.data, _ptr(rho)))
        return rho

    def get_residuals(self, nbands):
        out = np.zeros(nbands, np.float64)
        self._check(self.lib.pw_get_residuals(self.h, out.ctypes.data))
        return out

    def set_phase_timing(self, on=True):
        """Per-phase HIP events in later solves (pw_stats phase times; ~5 % slower)."""
        self._check(self.lib.pw_set_phase_timing(self.h, 1 if on else 0))

    def get_stats(self):
        s = PWStats()
        self._check(self.lib.pw_get_stats(self.h, ctypes.byref(s)))
        return s.as_dict()

    # ---- building blocks ---------------------------------------------------------
    def gram(self, A, B, C, K=None, p=None, q=None):
        """C = A^H B; A, B complex128 (pw_gram) or complex64 (pw_gram_mixed), C complex128."""
        K = A.shape[1] if K is None else K
        p = A.shape[0] if p is None else p
        q = B.shape[0] if q is None else q
        fn = self.lib.pw_gram_mixed if A.dtype == self._torch.complex64 else self.lib.pw_gram
        self._check(fn(self.h, _ptr(A), _ld(A), _ptr(B), _ld(B), K, p, q, _ptr(C), _ld(C)))
        return C

    def block_update(self, A, Cm, Y, alpha=1.0, beta=0.0, K=None, p=None, q=None):
        """Y = alpha A C + beta Y; A, Y complex128 or complex64, C complex128."""
        K = A.shape[1] if K is None else K
        p = A.shape[0] if p is None else p
        q = Cm.shape[0] if q is None else q
        fn = (self.lib.pw_block_update_mixed if A.dtype == self._torch.complex64
              else self.lib.pw_block_update)
        self._check(fn(self.h, _ptr(A), _ld(A), _ptr(Cm), _ld(Cm), K, p, q,
                       float(alpha), float(beta), _ptr(Y), _ld(Y)))
        return Y

    def small_eigh(self, A, n, k, w, V):
        self._check(self.lib.pw_small_eigh(self.h, _ptr(A), _ld(A), n, k, _ptr(w), _ptr(V), _ld(V)))

    def small_eigh_noalloc(self, A, n, k, w, V):
        """pw_small_eigh on the library's static scratch (no workspace, allocates nothing)."""
        self._check(self.lib.pw_small_eigh_noalloc(self.h, _ptr(A), _ld(A), n, k, _ptr(w), _ptr(V),
                                                   _ld(V)))

    def autotune(self, nb):
        """Time the FFT tile and split-K candidates on this context; keep and return the choice."""
        out = PWTuning()
        self._check(self.lib.pw_autotune(self.h, nb, ctypes.byref(out)))
        return out.as_dict()

    def set_tuning(self, fft_sticks_per_block=0, fft_plane_rows=0, gemm_split_workgroups=0, reset=False,
                   fft_radix2=0):
        if reset:
            self._check(self.lib.pw_set_tuning(self.h, None))
            return
        t = PWTuning(fft_sticks_per_block, fft_plane_rows, gemm_split_workgroups, 0.0, 0.0, 0.0, 0.0,
                     fft_radix2)
        self._check(self.lib.pw_set_tuning(self.h, ctypes.byref(t)))

    def chol_inv(self, G, n, Rinv):
        """Rinv = R^-1 for G = R^H R (device complex128 tensors, [col][row] storage)."""
        self._check(self.lib.pw_chol_inv(self.h, _ptr(G), _ld(G), n, _ptr(Rinv), _ld(Rinv)))

    def residuals(self, X, HX, nb, theta, res, W=None):
        self._check(self.lib.pw_residuals(self.h, _ptr(X), _ld(X), _ptr(HX), _ld(HX), nb, _ptr(theta),
                                          _ptr(res), _ptr(W) if W is not None else None,
                                          _ld(W) if W is not None else 0))
