"""ctypes binding of liblsh (include/lsh.h, include/lsh_dev.h).

Argument marshalling only: every step of the method runs in the HIP library.
Device arrays are torch tensors on the current HIP device (complex128 fields,
float64 b); the current torch stream is passed to every call.  The binding
raises if the library is missing or a call fails -- there is no fallback.
"""
from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, c_double, c_int, c_long, c_void_p

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblsh.so")

LSH_OK, LSH_NOT_CONVERGED = 0, 1
(LSH_ERR_INVALID_ARG, LSH_ERR_INPUT_NONFINITE, LSH_ERR_SINGULAR, LSH_ERR_HIP, LSH_ERR_NOMEM,
 LSH_ERR_UNSUPPORTED, LSH_ERR_WORKSPACE_TOO_SMALL) = -1, -2, -3, -4, -5, -6, -7
LSH_FACTOR_TRANSPOSE = 1
LSH_FP64, LSH_FP32 = 0, 1
MAX_ITERS = 200
MAX_LEVELS = 32

EXPORTED = [
    "lsh_plan_workspace", "lsh_plan_create", "lsh_plan_destroy", "lsh_plan_workspace_used", "lsh_plan_ranks",
    "lsh_plan_level", "lsh_plan_block", "lsh_plan_table", "lsh_factor_workspace", "lsh_factor_create",
    "lsh_factor_workspace_used", "lsh_factor_destroy", "lsh_apply_precond", "lsh_apply_operator",
    "lsh_solve_workspace", "lsh_solve", "lsh_solve_adjoint", "lsh_eval_points", "lsh_correction_weights",
    "lsh_last_error", "lsh_dev_gemm", "lsh_dev_gemm_split", "lsh_dev_inverse_workspace", "lsh_dev_inverse",
    "lsh_profile_enable", "lsh_profile_query", "lsh_profile_names", "lsh_eval_points_adjoint", "lsh_grad_b",
    "lsh_build_workspace", "lsh_build", "lsh_batch_factor_workspace", "lsh_batch_factor", "lsh_profile_only",
    "lsh_plan_lowrank", "lsh_plan_cache_info", "lsh_plan_cache_clear", "lsh_plan_cache_save",
    "lsh_plan_cache_load", "lsh_gemm_variants", "lsh_gemm_tune_workspace", "lsh_gemm_tune", "lsh_gemm_table_save",
    "lsh_gemm_table_load", "lsh_gemm_table_clear", "lsh_gemm_record", "lsh_gemm_recorded",
    "lsh_gemm_force_variant", "lsh_dev_inverse_static", "lsh_fused_levels", "lsh_profile_bytes",
    "lsh_apply_fused_levels",
]

# tuned GEMM variant choices (written by tune_gemm.py on an MI355X); LSH_GEMM_TABLE overrides the path,
# LSH_GEMM_TABLE=none loads nothing (the library's model then chooses)
GEMM_TABLE = os.path.join(HERE, "tune", "gemm_table.txt")


class LshDesc(ctypes.Structure):
    _fields_ = [("n", c_int), ("h", c_double), ("x0", c_double), ("y0", c_double), ("kappa", c_double),
                ("op_order", c_int), ("leaf", c_int), ("tol", c_double), ("proxy_width", c_int),
                ("hbs_prec", c_int), ("merge", c_int), ("hbs_order", c_int), ("plan_cache", c_int),
                ("full_levels", c_int)]


MERGE = {"auto": 0, "schur": 1, "lowrank": 2}


class LshSolveOpts(ctypes.Structure):
    _fields_ = [("tol", c_double), ("maxit", c_int), ("precondition", c_int)]


class LshInfo(ctypes.Structure):
    _fields_ = [("iterations", c_int), ("residual", c_double), ("true_residual", c_double),
                ("history", c_double * (MAX_ITERS + 1)), ("ms_precond", c_double), ("ms_operator", c_double),
                ("ms_ortho", c_double)]


class LshError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"liblsh error {code}: {msg}")
        self.code = code


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built (run __graft_entry__.build())")
        # torch ships its own HIP runtime; load it first so that liblsh's
        # libamdhip64 dependency resolves to that same copy (one runtime per
        # process, shared device memory and streams).
        import torch  # noqa: F401
        L = ctypes.CDLL(LIB_PATH)
        L.lsh_last_error.restype = ctypes.c_char_p
        L.lsh_plan_workspace.argtypes = [POINTER(LshDesc), POINTER(ctypes.c_size_t)]
        L.lsh_plan_create.argtypes = [POINTER(LshDesc), c_void_p, ctypes.c_size_t, c_void_p, POINTER(c_void_p)]
        L.lsh_plan_workspace_used.argtypes = [c_void_p, POINTER(ctypes.c_size_t), POINTER(ctypes.c_size_t)]
        L.lsh_plan_destroy.argtypes = [c_void_p]
        L.lsh_plan_ranks.argtypes = [c_void_p, POINTER(c_int), POINTER(c_int)]
        L.lsh_plan_level.argtypes = [c_void_p, c_int, POINTER(c_int), POINTER(c_int), POINTER(c_int),
                                     POINTER(c_int), c_void_p, c_void_p]
        L.lsh_plan_block.argtypes = [c_void_p, c_int, POINTER(c_int), c_void_p, c_void_p]
        L.lsh_plan_table.argtypes = [c_void_p, POINTER(c_int), c_void_p, c_void_p]
        L.lsh_factor_workspace.argtypes = [c_void_p, c_int, POINTER(ctypes.c_size_t)]
        L.lsh_factor_create.argtypes = [c_void_p, c_void_p, c_int, c_void_p, ctypes.c_size_t, c_void_p,
                                        POINTER(c_void_p)]
        L.lsh_factor_workspace_used.argtypes = [c_void_p, POINTER(ctypes.c_size_t), POINTER(ctypes.c_size_t)]
        L.lsh_factor_destroy.argtypes = [c_void_p]
        L.lsh_build_workspace.argtypes = [POINTER(LshDesc), c_int, POINTER(ctypes.c_size_t),
                                          POINTER(ctypes.c_size_t)]
        L.lsh_build.argtypes = [POINTER(LshDesc), c_void_p, c_int, c_void_p, ctypes.c_size_t, c_void_p,
                                ctypes.c_size_t, c_void_p, POINTER(c_void_p), POINTER(c_void_p)]
        L.lsh_batch_factor_workspace.argtypes = [c_int, POINTER(c_void_p), c_int, POINTER(ctypes.c_size_t),
                                                 POINTER(ctypes.c_size_t)]
        L.lsh_batch_factor.argtypes = [c_int, POINTER(c_void_p), POINTER(c_void_p), c_int, POINTER(c_void_p),
                                       POINTER(ctypes.c_size_t), c_void_p, ctypes.c_size_t, c_void_p,
                                       POINTER(c_void_p)]
        L.lsh_apply_precond.argtypes = [c_void_p, c_int, c_void_p, c_void_p, c_int, c_void_p]
        L.lsh_apply_operator.argtypes = [c_void_p, c_void_p, c_void_p, c_void_p, c_int, c_void_p]
        L.lsh_solve_workspace.argtypes = [c_void_p, c_int, c_int, POINTER(ctypes.c_size_t)]
        L.lsh_solve.argtypes = [c_void_p, c_void_p, c_int, c_void_p, c_void_p, POINTER(LshSolveOpts),
                                POINTER(LshInfo), c_void_p, ctypes.c_size_t, c_void_p]
        L.lsh_solve_adjoint.argtypes = [c_void_p, c_void_p, c_int, c_void_p, POINTER(LshSolveOpts),
                                        POINTER(LshInfo), c_void_p, ctypes.c_size_t, c_void_p]
        L.lsh_eval_points.argtypes = [c_void_p, c_void_p, c_void_p, c_int, c_void_p, c_int, c_void_p]
        L.lsh_correction_weights.argtypes = [c_int, c_double, POINTER(c_int), POINTER(c_int), POINTER(c_double)]
        L.lsh_dev_gemm.argtypes = [c_int, c_int, c_int, c_int, POINTER(c_double), c_void_p, c_long, c_long, c_int,
                                   c_void_p, c_long, c_long, c_int, POINTER(c_double), c_void_p, c_long, c_long,
                                   c_void_p, c_long, c_long, c_int, c_void_p]
        L.lsh_dev_gemm_split.argtypes = [c_int, c_int, c_int, c_int, POINTER(c_double), c_void_p, c_long, c_long,
                                         c_int, c_void_p, c_long, c_long, c_int, POINTER(c_double), c_void_p, c_long,
                                         c_long, c_void_p, c_long, c_long, c_int, c_void_p, ctypes.c_size_t, c_void_p]
        L.lsh_dev_inverse_workspace.argtypes = [c_int, c_int, c_int, POINTER(ctypes.c_size_t)]
        L.lsh_dev_inverse.argtypes = [c_int, c_void_p, c_int, c_long, c_long, c_int, c_void_p, c_void_p,
                                      ctypes.c_size_t, c_void_p]
        L.lsh_eval_points_adjoint.argtypes = [c_void_p, c_void_p, c_void_p, c_int, c_void_p, c_int, c_void_p]
        L.lsh_grad_b.argtypes = [c_void_p, c_void_p, c_void_p, c_void_p, c_int, c_void_p, c_void_p]
        L.lsh_profile_enable.argtypes = [c_int]
        L.lsh_profile_query.argtypes = [ctypes.c_char_p, POINTER(c_int), POINTER(c_double), POINTER(c_double)]
        L.lsh_profile_names.argtypes = [ctypes.c_char_p, c_int]
        L.lsh_profile_only.argtypes = [ctypes.c_char_p]
        L.lsh_profile_bytes.argtypes = [ctypes.c_char_p, POINTER(c_double)]
        L.lsh_plan_lowrank.argtypes = [c_void_p, c_int, POINTER(c_int), POINTER(c_int), c_void_p, c_void_p,
                                       c_void_p]
        L.lsh_plan_cache_info.argtypes = [POINTER(c_int), POINTER(ctypes.c_size_t)]
        L.lsh_plan_cache_clear.argtypes = []
        L.lsh_plan_cache_save.argtypes = [ctypes.c_char_p]
        L.lsh_plan_cache_load.argtypes = [ctypes.c_char_p]
        L.lsh_gemm_variants.argtypes = [c_int, POINTER(c_int), ctypes.c_char_p, c_int]
        L.lsh_gemm_tune_workspace.argtypes = [c_int, c_int, c_int, c_int, c_int, POINTER(ctypes.c_size_t)]
        L.lsh_gemm_tune.argtypes = [c_int, c_int, c_int, c_int, c_int, c_int, c_void_p, ctypes.c_size_t, c_void_p,
                                    POINTER(c_int), POINTER(c_double)]
        L.lsh_gemm_table_save.argtypes = [ctypes.c_char_p]
        L.lsh_gemm_table_load.argtypes = [ctypes.c_char_p, POINTER(c_int)]
        L.lsh_gemm_table_clear.argtypes = []
        L.lsh_gemm_record.argtypes = [c_int]
        L.lsh_gemm_recorded.argtypes = [POINTER(c_int), POINTER(c_int), c_int]
        L.lsh_gemm_force_variant.argtypes = [c_int]
        L.lsh_fused_levels.argtypes = [c_int]
        L.lsh_apply_fused_levels.argtypes = [c_int]
        L.lsh_dev_inverse_static.argtypes = [c_int, c_void_p, c_int, c_long, c_long, c_int, c_void_p, c_void_p]
        table = os.environ.get("LSH_GEMM_TABLE", GEMM_TABLE)
        if table != "none" and os.path.exists(table):
            n = c_int(0)
            if L.lsh_gemm_table_load(table.encode(), ctypes.byref(n)) != LSH_OK:
                raise RuntimeError(f"cannot load the GEMM table {table}: {L.lsh_last_error().decode()}")
        _lib = L
    return _lib


def _check(rc, allow_not_converged=False):
    if rc == LSH_OK or (allow_not_converged and rc == LSH_NOT_CONVERGED):
        return rc
    raise LshError(rc, lib().lsh_last_error().decode())


def _stream():
    import torch
    return c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t, dtype=None, numel=None):
    import torch
    if not t.is_cuda:
        raise ValueError("expected a device tensor")
    if not t.is_contiguous():
        raise ValueError("expected a contiguous tensor")
    if dtype is not None and t.dtype != dtype:
        raise TypeError(f"expected {dtype}, got {t.dtype}")
    if numel is not None and t.numel() < numel:
        raise ValueError(f"tensor too small: {t.numel()} < {numel}")
    return c_void_p(t.data_ptr())


def workspace(nbytes):
    """A caller-owned device workspace of nbytes (torch's allocator aligns it to 512 bytes)."""
    import torch
    return torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device="cuda")


def _size():
    return ctypes.c_size_t(0)


def lsh_correction_weights(order: int, kh: float):
    """Host call: stencil offsets (count, 2) and tau (count,) complex."""
    cnt = c_int(0)
    off = (c_int * 50)()
    tau = (c_double * 50)()
    _check(lib().lsh_correction_weights(order, kh, ctypes.byref(cnt), off, tau))
    k = cnt.value
    o = np.array(off[: 2 * k]).reshape(k, 2)
    t = np.array(tau[: 2 * k]).reshape(k, 2)
    return o, t[:, 0] + 1j * t[:, 1]


class Plan:
    """lsh_plan_create: tree, weights, kernel table, per-level row IDs, FFT spectrum."""

    def __init__(self, n, kappa, op_order=10, leaf=8, tol=1e-4, proxy_width=2, prec="fp32",
                 h=None, x0=-0.5, y0=-0.5, merge="auto", hbs_order=4, plan_cache=False, ws=None, _create=True,
                 full_levels=0):
        self.desc = LshDesc(n=n, h=(1.0 / n if h is None else h), x0=x0, y0=y0, kappa=kappa,
                            op_order=op_order, leaf=leaf, tol=tol, proxy_width=proxy_width,
                            hbs_prec=LSH_FP32 if prec == "fp32" else LSH_FP64, merge=MERGE[merge],
                            hbs_order=hbs_order, plan_cache=int(bool(plan_cache)), full_levels=full_levels)
        self.n = n
        self.h = self.desc.h
        self.kappa = kappa
        self.handle = c_void_p()
        self.ws = None  # the plan's device workspace (caller-owned; lives as long as the plan)
        if _create:
            nb = _size()
            _check(lib().lsh_plan_workspace(ctypes.byref(self.desc), ctypes.byref(nb)))
            self.ws = workspace(nb.value) if ws is None else ws
            _check(lib().lsh_plan_create(ctypes.byref(self.desc), _ptr(self.ws), self.ws.numel(), _stream(),
                                         ctypes.byref(self.handle)))

    def workspace_used(self):
        """(bytes of the workspace used at most, workspace size)."""
        u, z = _size(), _size()
        _check(lib().lsh_plan_workspace_used(self.handle, ctypes.byref(u), ctypes.byref(z)))
        return u.value, z.value

    def close(self):
        if self.handle:
            lib().lsh_plan_destroy(self.handle)
            self.handle = c_void_p()
        self.ws = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def ranks(self):
        L = c_int(0)
        r = (c_int * (MAX_LEVELS + 1))()
        _check(lib().lsh_plan_ranks(self.handle, ctypes.byref(L), r))
        return L.value, list(r[: L.value + 1])

    def level(self, level):
        """(J, cand, U) of a level: pivots, candidate coords (m, 2), U (m, k) complex128 on device."""
        import torch
        m, k = c_int(0), c_int(0)
        _check(lib().lsh_plan_level(self.handle, level, ctypes.byref(m), ctypes.byref(k), None, None, None,
                                    _stream()))
        J = (c_int * k.value)()
        cand = (c_int * (2 * m.value))()
        U = torch.empty((m.value, k.value), dtype=torch.complex128, device="cuda")
        _check(lib().lsh_plan_level(self.handle, level, None, None, J, cand, _ptr(U), _stream()))
        return np.array(J[:]), np.array(cand[:]).reshape(-1, 2), U

    def block(self, level):
        import torch
        c = c_int(0)
        _check(lib().lsh_plan_block(self.handle, level, ctypes.byref(c), None, _stream()))
        out = torch.empty((c.value, c.value), dtype=torch.complex128, device="cuda")
        _check(lib().lsh_plan_block(self.handle, level, None, _ptr(out), _stream()))
        return out

    def lowrank_ranks(self):
        """Rank r of each parent level's low-rank sibling block (0: Schur-form merges there)."""
        out = []
        for l in range(self.ranks()[0]):
            c, r = c_int(0), c_int(0)
            _check(lib().lsh_plan_lowrank(self.handle, l, ctypes.byref(c), ctypes.byref(r), None, None, _stream()))
            out.append(r.value)
        return out

    def lowrank(self, level):
        """(L, Rt) of parent level `level` (G_ab ~= L Rt, complex128 on device), or None
        where that level's merges use the Schur form."""
        import torch
        c, r = c_int(0), c_int(0)
        _check(lib().lsh_plan_lowrank(self.handle, level, ctypes.byref(c), ctypes.byref(r), None, None, _stream()))
        if r.value == 0:
            return None
        L = torch.empty((c.value, r.value), dtype=torch.complex128, device="cuda")
        Rt = torch.empty((r.value, c.value), dtype=torch.complex128, device="cuda")
        _check(lib().lsh_plan_lowrank(self.handle, level, None, None, _ptr(L), _ptr(Rt), _stream()))
        return L, Rt

    def table(self):
        import torch
        D = c_int(0)
        _check(lib().lsh_plan_table(self.handle, ctypes.byref(D), None, _stream()))
        out = torch.empty((D.value + 1, D.value + 1), dtype=torch.complex128, device="cuda")
        _check(lib().lsh_plan_table(self.handle, None, _ptr(out), _stream()))
        return out

    def apply_operator(self, b, x, out=None):
        """y = x + kappa^2 b (K * x); b=None gives K * x.  x: (nrhs, n, n) complex128."""
        import torch
        x = x.reshape(-1, self.n, self.n)
        y = torch.empty_like(x) if out is None else out
        bp = _ptr(b, torch.float64, self.n * self.n) if b is not None else None
        _check(lib().lsh_apply_operator(self.handle, bp, _ptr(x, torch.complex128), _ptr(y, torch.complex128),
                                        x.shape[0], _stream()))
        return y

    def eval_points(self, sigma, xy):
        import torch
        sigma = sigma.reshape(-1, self.n, self.n)
        xy = xy.reshape(-1, 2).contiguous()
        out = torch.empty((sigma.shape[0], xy.shape[0]), dtype=torch.complex128, device="cuda")
        _check(lib().lsh_eval_points(self.handle, _ptr(sigma, torch.complex128), _ptr(xy, torch.float64),
                                     xy.shape[0], _ptr(out), sigma.shape[0], _stream()))
        return out


    def eval_points_adjoint(self, g, xy):
        """out[m] = E^H g[m] on the grid (adjoint of eval_points)."""
        import torch
        g = g.reshape(-1, xy.reshape(-1, 2).shape[0]).contiguous()
        xy = xy.reshape(-1, 2).contiguous()
        out = torch.empty((g.shape[0], self.n, self.n), dtype=torch.complex128, device="cuda")
        _check(lib().lsh_eval_points_adjoint(self.handle, _ptr(g, torch.complex128), _ptr(xy, torch.float64),
                                             xy.shape[0], _ptr(out), g.shape[0], _stream()))
        return out

    def grad_b(self, lam, u_inc, u):
        """-kappa^2 Re sum_m conj(lam_m) (u_inc_m + u_m), shape (n, n) float64."""
        import torch
        n = self.n
        lam = lam.reshape(-1, n, n).contiguous()
        u_inc = u_inc.reshape(-1, n, n).contiguous()
        u = u.reshape(-1, n, n).contiguous()
        out = torch.empty((n, n), dtype=torch.float64, device="cuda")
        _check(lib().lsh_grad_b(self.handle, _ptr(lam, torch.complex128), _ptr(u_inc, torch.complex128),
                                _ptr(u, torch.complex128), lam.shape[0], _ptr(out), _stream()))
        return out


class Factor:
    """lsh_factor_create: Algorithm 1 for the potential b (float64, (n, n), device).
    transpose=True reserves room for M^T (apply_precond(transpose=True), solve_adjoint)."""

    def __init__(self, plan: Plan, b, transpose=False, ws=None, _handle=None, _ws=None):
        import torch
        self.plan = plan
        self.handle = c_void_p()
        self.ws = _ws  # the factor's device workspace (caller-owned)
        if _handle is not None:
            self.handle = _handle
            return
        b = b.reshape(plan.n, plan.n).contiguous()
        flags = LSH_FACTOR_TRANSPOSE if transpose else 0
        nb = _size()
        _check(lib().lsh_factor_workspace(plan.handle, flags, ctypes.byref(nb)))
        self.ws = workspace(nb.value) if ws is None else ws
        _check(lib().lsh_factor_create(plan.handle, _ptr(b, torch.float64), flags, _ptr(self.ws), self.ws.numel(),
                                       _stream(), ctypes.byref(self.handle)))

    def workspace_used(self):
        u, z = _size(), _size()
        _check(lib().lsh_factor_workspace_used(self.handle, ctypes.byref(u), ctypes.byref(z)))
        return u.value, z.value

    def solve_workspace_bytes(self, nrhs, maxit):
        nb = _size()
        _check(lib().lsh_solve_workspace(self.handle, nrhs, maxit, ctypes.byref(nb)))
        return nb.value

    def _solve_ws(self, nrhs, maxit, ws=None):
        if ws is None:
            ws = workspace(self.solve_workspace_bytes(nrhs, maxit))
        return ws, ws.numel()

    def close(self):
        if self.handle:
            lib().lsh_factor_destroy(self.handle)
            self.handle = c_void_p()
        self.ws = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def apply_precond(self, x, transpose=False):
        import torch
        n = self.plan.n
        x = x.reshape(-1, n, n).contiguous()
        y = torch.empty_like(x)
        _check(lib().lsh_apply_precond(self.handle, int(transpose), _ptr(x, torch.complex128),
                                       _ptr(y, torch.complex128), x.shape[0], _stream()))
        return y

    def solve(self, u_inc, tol=1e-10, maxit=100, precondition=True, want_u=True, ws=None):
        """sigma, u, info for incident fields u_inc (nrhs, n, n) complex128.
        ws: a solve workspace (uint8 device tensor) to reuse, else a new one."""
        import torch
        n = self.plan.n
        u_inc = u_inc.reshape(-1, n, n).contiguous()
        sig = torch.empty_like(u_inc)
        u = torch.empty_like(u_inc) if want_u else None
        opts = LshSolveOpts(tol=tol, maxit=maxit, precondition=int(precondition))
        info = LshInfo()
        ws, nb = self._solve_ws(u_inc.shape[0], maxit, ws)
        rc = _check(lib().lsh_solve(self.handle, _ptr(u_inc, torch.complex128), u_inc.shape[0], _ptr(sig),
                                    _ptr(u) if u is not None else None, ctypes.byref(opts), ctypes.byref(info),
                                    _ptr(ws), nb, _stream()), allow_not_converged=True)
        return sig, u, info, rc

    def solve_adjoint(self, g, tol=1e-10, maxit=100, ws=None):
        import torch
        n = self.plan.n
        g = g.reshape(-1, n, n).contiguous()
        lam = torch.empty_like(g)
        opts = LshSolveOpts(tol=tol, maxit=maxit, precondition=1)
        info = LshInfo()
        ws, nb = self._solve_ws(g.shape[0], maxit, ws)
        rc = _check(lib().lsh_solve_adjoint(self.handle, _ptr(g, torch.complex128), g.shape[0], _ptr(lam),
                                            ctypes.byref(opts), ctypes.byref(info), _ptr(ws), nb, _stream()),
                    allow_not_converged=True)
        return lam, info, rc


def build_workspaces(n, kappa, op_order=10, leaf=8, tol=1e-4, proxy_width=2, prec="fp32", h=None, x0=-0.5,
                     y0=-0.5, merge="auto", hbs_order=4, plan_cache=False, transpose=False, full_levels=0):
    """(plan_ws, factor_ws): device workspaces sized for lsh_build (allocate once, reuse across builds)."""
    d = LshDesc(n=n, h=(1.0 / n if h is None else h), x0=x0, y0=y0, kappa=kappa, op_order=op_order, leaf=leaf,
                tol=tol, proxy_width=proxy_width, hbs_prec=LSH_FP32 if prec == "fp32" else LSH_FP64,
                merge=MERGE[merge], hbs_order=hbs_order, plan_cache=int(bool(plan_cache)),
                full_levels=full_levels)
    pb, fb = _size(), _size()
    _check(lib().lsh_build_workspace(ctypes.byref(d), LSH_FACTOR_TRANSPOSE if transpose else 0, ctypes.byref(pb),
                                     ctypes.byref(fb)))
    return workspace(pb.value), workspace(fb.value)


def build(n, kappa, b, op_order=10, leaf=8, tol=1e-4, proxy_width=2, prec="fp32", h=None, x0=-0.5, y0=-0.5,
          merge="auto", hbs_order=4, plan_cache=False, transpose=False, workspaces=None, full_levels=0):
    """lsh_build: plan and factor pipelined by level; returns (Plan, Factor).
    workspaces: (plan_ws, factor_ws) from build_workspaces, reused (else new ones)."""
    import torch
    P = Plan(n, kappa, op_order, leaf, tol, proxy_width, prec, h, x0, y0, merge=merge, hbs_order=hbs_order,
             plan_cache=plan_cache, _create=False, full_levels=full_levels)
    if workspaces is None:
        workspaces = build_workspaces(n, kappa, op_order, leaf, tol, proxy_width, prec, h, x0, y0, merge,
                                      hbs_order, plan_cache, transpose, full_levels)
    pw, fw = workspaces
    fh = c_void_p()
    b = b.reshape(n, n).contiguous()
    _check(lib().lsh_build(ctypes.byref(P.desc), _ptr(b, torch.float64), LSH_FACTOR_TRANSPOSE if transpose else 0,
                           _ptr(pw), pw.numel(), _ptr(fw), fw.numel(), _stream(), ctypes.byref(P.handle),
                           ctypes.byref(fh)))
    P.ws = pw
    return P, Factor(P, None, _handle=fh, _ws=fw)


def batch_factor(plans, bs, transpose=False):
    """lsh_batch_factor: Algorithm 1 for many instances at once (each level's
    products and inverses grouped over all instances); returns one Factor per
    plan."""
    import torch
    n = len(plans)
    flags = LSH_FACTOR_TRANSPOSE if transpose else 0
    bs = [b.reshape(p.n, p.n).contiguous() for p, b in zip(plans, bs)]
    ph = (c_void_p * n)(*[p.handle.value for p in plans])
    bp = (c_void_p * n)(*[_ptr(b, torch.float64).value for b in bs])
    fb = (ctypes.c_size_t * n)()
    sb = _size()
    _check(lib().lsh_batch_factor_workspace(n, ph, flags, fb, ctypes.byref(sb)))
    wss = [workspace(fb[i]) for i in range(n)]
    shared = workspace(sb.value)
    wp = (c_void_p * n)(*[w.data_ptr() for w in wss])
    fh = (c_void_p * n)()
    _check(lib().lsh_batch_factor(n, ph, bp, flags, wp, fb, _ptr(shared), sb.value, _stream(), fh))
    return [Factor(p, None, _handle=c_void_p(fh[i]), _ws=wss[i]) for i, p in enumerate(plans)]


def dev_gemm(A, B, opA=0, opB=0, alpha=1.0, beta=0.0, D=None, out=None, ws=None):
    """Batched complex GEMM through lsh_dev_gemm.  A, B: (batch, r, c) complex tensors.
    ws: a device tensor of scratch bytes for lsh_dev_gemm_split (split K)."""
    import torch
    prec = LSH_FP64 if A.dtype == torch.complex128 else LSH_FP32
    bA, ra, ca = A.shape
    bB, rb, cb = B.shape
    M, K = (ra, ca) if opA in (0, 3) else (ca, ra)
    N = cb if opB in (0, 3) else rb
    batch = max(bA, bB)
    C = torch.empty((batch, M, N), dtype=A.dtype, device=A.device) if out is None else out
    al = (c_double * 2)(complex(alpha).real, complex(alpha).imag)
    be = (c_double * 2)(complex(beta).real, complex(beta).imag)
    Dp = _ptr(D) if D is not None else None
    args = (prec, M, N, K, al, _ptr(A), ca, ra * ca if bA > 1 else 0, opA, _ptr(B), cb, rb * cb if bB > 1 else 0,
            opB, be, Dp, N, M * N if D is not None else 0, _ptr(C), N, M * N, batch)
    if ws is None:
        _check(lib().lsh_dev_gemm(*args, _stream()))
    else:
        _check(lib().lsh_dev_gemm_split(*args, _ptr(ws), ws.numel() * ws.element_size(), _stream()))
    return C


def dev_inverse(A):
    """In-place batched inverse; returns (A, info)."""
    import torch
    prec = LSH_FP64 if A.dtype == torch.complex128 else LSH_FP32
    b, c, _ = A.shape
    info = torch.zeros(b, dtype=torch.int32, device=A.device)
    nb = ctypes.c_size_t(0)
    _check(lib().lsh_dev_inverse_workspace(prec, c, b, ctypes.byref(nb)))
    ws = workspace(nb.value)
    _check(lib().lsh_dev_inverse(prec, _ptr(A), c, c, c * c, b, _ptr(info), _ptr(ws), nb.value, _stream()))
    return A, info


def gemm_variants(prec="fp32"):
    n = c_int(0)
    buf = ctypes.create_string_buffer(1024)
    _check(lib().lsh_gemm_variants(LSH_FP32 if prec == "fp32" else LSH_FP64, ctypes.byref(n), buf, 1024))
    return buf.value.decode().split(";")


def gemm_tune(prec, M, N, K, batch, reps=5):
    """Time every GEMM variant on one shape (lsh_gemm_tune); returns (best, ms per variant)."""
    p = LSH_FP32 if prec == "fp32" else LSH_FP64
    nb = _size()
    _check(lib().lsh_gemm_tune_workspace(p, M, N, K, batch, ctypes.byref(nb)))
    ws = workspace(nb.value)
    count = len(gemm_variants(prec))
    ms = (c_double * count)()
    best = c_int(0)
    _check(lib().lsh_gemm_tune(p, M, N, K, batch, reps, _ptr(ws), nb.value, _stream(), ctypes.byref(best), ms))
    return best.value, list(ms)


def fused_levels(min_boxes=1):
    """Persistent one-launch levels for later FP32 factors: levels with at least
    min_boxes boxes (0 or False: none; True: every eligible level)."""
    _check(lib().lsh_fused_levels(int(min_boxes)))


def apply_fused_levels(min_vectors=-1):
    """One-launch-per-pass apply levels: Woodbury levels with at least
    min_vectors box vectors (0: none; 1: every eligible level; -1: the
    default)."""
    _check(lib().lsh_apply_fused_levels(int(min_vectors)))


def gemm_force_variant(v=-1):
    _check(lib().lsh_gemm_force_variant(int(v)))


def gemm_record(on=True):
    _check(lib().lsh_gemm_record(int(on)))


def gemm_recorded():
    """{(prec, M, N, K, batch): number of products} since gemm_record(True) (prec 1 = FP32, 0 = FP64)."""
    n = c_int(0)
    _check(lib().lsh_gemm_recorded(ctypes.byref(n), None, 0))
    buf = (c_int * (6 * max(n.value, 1)))()
    _check(lib().lsh_gemm_recorded(ctypes.byref(n), buf, n.value))
    return {tuple(buf[6 * i:6 * i + 5]): buf[6 * i + 5] for i in range(n.value)}


def gemm_table_save(path):
    _check(lib().lsh_gemm_table_save(str(path).encode()))


def gemm_table_load(path):
    n = c_int(0)
    _check(lib().lsh_gemm_table_load(str(path).encode(), ctypes.byref(n)))
    return n.value


def gemm_table_clear():
    _check(lib().lsh_gemm_table_clear())


def lsh_profile_enable(on=True):
    _check(lib().lsh_profile_enable(int(on)))


def lsh_profile_only(prefix=None):
    """Record only the kernels whose name starts with prefix (None: all)."""
    _check(lib().lsh_profile_only(prefix.encode() if prefix else None))


def plan_cache_info():
    """(entries, host bytes) of the process-wide plan cache."""
    n, b = c_int(0), ctypes.c_size_t(0)
    _check(lib().lsh_plan_cache_info(ctypes.byref(n), ctypes.byref(b)))
    return n.value, b.value


def plan_cache_clear():
    _check(lib().lsh_plan_cache_clear())


def plan_cache_save(path):
    _check(lib().lsh_plan_cache_save(str(path).encode()))


def plan_cache_load(path):
    _check(lib().lsh_plan_cache_load(str(path).encode()))


def lsh_profile_query(name):
    """(launches, total ms, total algorithmic work) of one kernel name."""
    n, ms, w = c_int(0), c_double(0), c_double(0)
    _check(lib().lsh_profile_query(name.encode(), ctypes.byref(n), ctypes.byref(ms), ctypes.byref(w)))
    return n.value, ms.value, w.value


def lsh_profile_bytes(name):
    """Summed algorithmic bytes recorded for one kernel name (GEMMs: operands and result once)."""
    b = c_double(0)
    _check(lib().lsh_profile_bytes(name.encode(), ctypes.byref(b)))
    return b.value


def lsh_profile_names():
    buf = ctypes.create_string_buffer(4096)
    _check(lib().lsh_profile_names(buf, 4096))
    return [x for x in buf.value.decode().split(";") if x]


def receiver_field(b, u_inc, xy, plan: Plan, tol=1e-10, maxit=100):
    """Scattered field at off-grid receivers, differentiable in b.

    Forward: Algorithm 1 for b, preconditioned FGMRES for sigma, then
    u(x_r) = h^2 sum_j G(x_r - x_j) sigma_j.  Backward (the adjoint method):
    g = E^H dL/du*, lambda = A^{-H} g by the transposed-HBS-preconditioned
    solve, dL/db = -kappa^2 Re sum_m conj(lambda_m) u_tot_m.  All steps run in
    liblsh; this function only routes the tensors.
    """
    return _ReceiverField.apply(b, u_inc, xy, plan, tol, maxit)


def _autograd_function():
    import torch

    class ReceiverField(torch.autograd.Function):
        @staticmethod
        def forward(ctx, b, u_inc, xy, plan, tol, maxit):
            F = Factor(plan, b.detach(), transpose=True)
            sig, u, info, rc = F.solve(u_inc.detach(), tol=tol, maxit=maxit)
            if rc != LSH_OK:
                raise LshError(rc, "forward solve did not converge")
            ur = plan.eval_points(sig, xy)
            ctx.F, ctx.plan, ctx.tol, ctx.maxit = F, plan, tol, maxit
            ctx.save_for_backward(u_inc.detach(), u, xy)
            return ur

        @staticmethod
        def backward(ctx, grad_ur):
            u_inc, u, xy = ctx.saved_tensors
            g = ctx.plan.eval_points_adjoint(grad_ur.contiguous(), xy)
            lam, info, rc = ctx.F.solve_adjoint(g, tol=ctx.tol, maxit=ctx.maxit)
            if rc != LSH_OK:
                raise LshError(rc, "adjoint solve did not converge")
            gb = ctx.plan.grad_b(lam, u_inc, u)
            return gb, None, None, None, None, None

    return ReceiverField


class _Lazy:
    fn = None

    @classmethod
    def apply(cls, *args):
        if cls.fn is None:
            cls.fn = _autograd_function()
        return cls.fn.apply(*args)


_ReceiverField = _Lazy
