"""Python binding of libhelm (include/helm.h): argument marshalling only.

Every call forwards device pointers of torch tensors to the C ABI; all the
arithmetic of the solver runs in the HIP kernels of libhelm.so.  PyTorch
provides device memory and the stream (torch's current stream at the time a
Solver is built).  If libhelm.so is missing, loading fails with an error
that says how to build it: there is no fallback path.
"""

import ctypes
import math
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhelm.so")

HELM_OK, HELM_EINVAL, HELM_ENOMEM, HELM_EDEVICE, HELM_ENOCONV, HELM_ENOTSUP = 0, -1, -2, -3, -4, -5
HELM_P1_TRI_RIGHT, HELM_Q1_HEX, HELM_MIXED_DG0_P1 = 1, 2, 3
HELM_FP64, HELM_FP32_MG = 0, 1
HELM_OUTER_FGMRES, HELM_OUTER_RICHARDSON = 0, 1
HELM_CYCLE_V_JACOBI, HELM_CYCLE_W_GMRES = 0, 1
OPS = {"B0": 0, "BDELTA": 1, "BSHIFT": 2, "L": 3, "N": 4, "H": 5, "M": 6, "MIXED": 7,
       "MIXED_SHIFT": 8}

# every symbol include/helm.h declares
EXPORTS = ("helm_opts_default", "helm_strerror", "helm_create", "helm_destroy", "helm_nodes",
           "helm_vector_length",
           "helm_workspace_bytes", "helm_solve", "helm_load_nodal", "helm_apply",
           "helm_hss_residual", "helm_jacobi", "helm_restrict_residual", "helm_prolong_correct",
           "helm_coarse_solve", "helm_vcycle", "helm_vcycle_noalloc", "helm_precondition", "helm_hss_history",
           "helm_last_error",
           "helm_server_create", "helm_server_submit", "helm_server_step", "helm_server_query",
           "helm_server_load", "helm_server_destroy")


class HelmError(RuntimeError):
    def __init__(self, status, what):
        self.status = status
        msg = "%s failed: %s (%d)" % (what, strerror(status), status)
        detail = last_error()
        if detail:
            msg += " [%s]" % detail
        super().__init__(msg)


class helm_mesh(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int), ("elem", ctypes.c_int), ("n", ctypes.c_int),
                ("levels", ctypes.c_int)]


class helm_bc(ctypes.Structure):
    _fields_ = [("dirichlet_faces", ctypes.c_uint)]


class helm_opts(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int), ("nu1", ctypes.c_int), ("nu2", ctypes.c_int),
                ("omega", ctypes.c_double), ("hss_m", ctypes.c_int), ("hss_steps", ctypes.c_int),
                ("restart", ctypes.c_int), ("max_outer", ctypes.c_int), ("x0_given", ctypes.c_int),
                ("profile", ctypes.c_int), ("mg_cycles", ctypes.c_int),
                ("no_graphs", ctypes.c_int), ("no_small", ctypes.c_int),
                ("verbose", ctypes.c_int), ("no_stream", ctypes.c_int),
                ("full_reorth", ctypes.c_int), ("split", ctypes.c_int),
                ("outer", ctypes.c_int), ("cycle", ctypes.c_int),
                ("smooth_its", ctypes.c_int)]


class helm_stats(ctypes.Structure):
    _fields_ = [("outer_its", ctypes.c_int), ("restarts", ctypes.c_int),
                ("hss_steps", ctypes.c_int), ("vcycles", ctypes.c_longlong),
                ("converged", ctypes.c_int), ("arnoldi_rel_residual", ctypes.c_double),
                ("true_rel_residual", ctypes.c_double), ("solve_ms", ctypes.c_double),
                ("precond_ms", ctypes.c_double), ("sweep_ms", ctypes.c_double),
                ("sweep_launches", ctypes.c_longlong), ("sweep_bytes", ctypes.c_double),
                ("mg_cycles", ctypes.c_int), ("vcycle_rate", ctypes.c_double),
                ("reorth_passes", ctypes.c_longlong), ("outer_rate", ctypes.c_double)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


class helm_server_opts(ctypes.Structure):
    _fields_ = [("hbm_budget_bytes", ctypes.c_double), ("max_cols", ctypes.c_int),
                ("precision", ctypes.c_int), ("restart", ctypes.c_int),
                ("max_outer", ctypes.c_int)]


class helm_request_info(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int), ("converged", ctypes.c_int), ("outer_its", ctypes.c_int),
                ("true_rel_residual", ctypes.c_double), ("t_submit", ctypes.c_double),
                ("t_admit", ctypes.c_double), ("t_done", ctypes.c_double)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


_lib = None


def lib():
    """Load libhelm.so (once).  Raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError("libhelm.so not found at %s; build it with "
                          "`python -m paper_2506_18694_amd.build`" % LIB_PATH)
    L = ctypes.CDLL(LIB_PATH)
    P, I, D = ctypes.c_void_p, ctypes.c_int, ctypes.c_double
    sig = {
        "helm_opts_default": (None, [ctypes.POINTER(helm_opts)]),
        "helm_strerror": (ctypes.c_char_p, [I]),
        "helm_last_error": (ctypes.c_char_p, []),
        "helm_create": (I, [ctypes.POINTER(helm_mesh), D, D, D, ctypes.POINTER(helm_bc),
                            ctypes.POINTER(helm_opts), P, ctypes.POINTER(P)]),
        "helm_destroy": (I, [P]),
        "helm_nodes": (ctypes.c_longlong, [P, I]),
        "helm_vector_length": (ctypes.c_longlong, [P]),
        "helm_workspace_bytes": (I, [P, I, ctypes.POINTER(ctypes.c_size_t)]),
        "helm_solve": (I, [P, P, P, I, D, P, ctypes.POINTER(helm_stats)]),
        "helm_load_nodal": (I, [P, P, P, I]),
        "helm_apply": (I, [P, I, I, I, P, P, I]),
        "helm_hss_residual": (I, [P, I, P, P, P, I]),
        "helm_jacobi": (I, [P, I, I, P, P, P, I]),
        "helm_restrict_residual": (I, [P, I, I, P, P, P, I]),
        "helm_prolong_correct": (I, [P, I, I, P, P, I]),
        "helm_coarse_solve": (I, [P, I, P, P, I]),
        "helm_vcycle": (I, [P, I, P, P, I, P]),
        "helm_vcycle_noalloc": (I, [P, I, P, P, I]),
        "helm_precondition": (I, [P, P, P, I, P]),
        "helm_hss_history": (I, [P, P, P, I, P, ctypes.POINTER(D)]),
        "helm_server_create": (I, [ctypes.POINTER(helm_server_opts), ctypes.POINTER(P)]),
        "helm_server_submit": (I, [P, I, I, I, D, D, P, P, I, D, ctypes.POINTER(ctypes.c_longlong)]),
        "helm_server_step": (I, [P, ctypes.POINTER(I)]),
        "helm_server_query": (I, [P, ctypes.c_longlong, ctypes.POINTER(helm_request_info)]),
        "helm_server_load": (I, [P, ctypes.POINTER(I), ctypes.POINTER(I), ctypes.POINTER(D)]),
        "helm_server_destroy": (I, [P]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    _lib = L
    return L


def strerror(status):
    return lib().helm_strerror(status).decode()


def last_error():
    try:
        return lib().helm_last_error().decode()
    except Exception:
        return ""


def _check(status, what):
    if status != HELM_OK:
        raise HelmError(status, what)
    return status


def _ptr(t):
    return ctypes.c_void_p(0 if t is None else t.data_ptr())


class Solver:
    """A helm_t handle for one mesh and parameter set.

    Vectors are torch tensors on the current CUDA (HIP) device: complex128
    for FP64 arguments, complex64 for FP32 ones, shape (nrhs, N) or (N,).
    """

    def __init__(self, dim, n, levels, k, delta=0.0, delta_hat=None, precision="fp64",
                 restart=0, max_outer=0, hss_steps=0, hss_m=1, omega=2.0 / 3.0,
                 dirichlet_faces=0, profile=False, mg_cycles=0, graphs=True, small_kernel=True,
                 verbose=0, stream=None, streaming=True, split=False,
                 full_reorth=False, outer="fgmres", x0_given=False, cycle="v",
                 smooth_its=0, mixed=False):
        import torch
        self.torch = torch
        L = lib()
        elem = HELM_Q1_HEX if dim == 3 else (HELM_MIXED_DG0_P1 if mixed else HELM_P1_TRI_RIGHT)
        mesh = helm_mesh(dim, elem, n, levels)
        opts = helm_opts()
        L.helm_opts_default(ctypes.byref(opts))
        opts.precision = HELM_FP64 if precision == "fp64" else HELM_FP32_MG
        opts.restart, opts.max_outer = restart, max_outer
        opts.hss_steps, opts.hss_m, opts.omega = hss_steps, hss_m, omega
        opts.profile = 1 if profile else 0
        opts.mg_cycles = mg_cycles
        opts.no_graphs = 0 if graphs else 1
        opts.no_small = 0 if small_kernel else 1
        opts.verbose = int(verbose)
        opts.no_stream = 0 if streaming else 1
        opts.split = 1 if split else 0
        opts.full_reorth = 1 if full_reorth else 0
        opts.outer = {"fgmres": HELM_OUTER_FGMRES, "richardson": HELM_OUTER_RICHARDSON}[outer]
        opts.x0_given = 1 if x0_given else 0
        opts.cycle = {"v": HELM_CYCLE_V_JACOBI, "w": HELM_CYCLE_W_GMRES}[cycle]
        opts.smooth_its = int(smooth_its)
        self.x0_given = bool(x0_given)
        # the library's step count: hss_steps, else m * ceil(k)
        self.n_hss = int(hss_steps) if hss_steps > 0 else int(hss_m * math.ceil(float(k)))
        bc = helm_bc(dirichlet_faces)
        if stream is None:
            stream = torch.cuda.current_stream()
        self.stream = stream
        handle = ctypes.c_void_p()
        dh = float(k) if delta_hat is None else float(delta_hat)
        _check(L.helm_create(ctypes.byref(mesh), float(k), float(delta), dh, ctypes.byref(bc),
                             ctypes.byref(opts), ctypes.c_void_p(stream.cuda_stream),
                             ctypes.byref(handle)), "helm_create")
        self.h = handle
        self.dim, self.n, self.levels, self.k = dim, n, levels, float(k)
        self.delta, self.delta_hat = float(delta), dh
        self.precision = precision
        self.prec_code = opts.precision
        self.N = self.nodes(0)
        self.mixed = bool(mixed)
        self.NV = int(L.helm_vector_length(self.h))  # column length of rhs / x
        self._ws = {}

    # -- lifetime -----------------------------------------------------------
    def close(self):
        if getattr(self, "h", None):
            _check(lib().helm_destroy(self.h), "helm_destroy")
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- sizes ----------------------------------------------------------------
    def nodes(self, level=0):
        return int(lib().helm_nodes(self.h, level))

    def workspace_bytes(self, nrhs):
        b = ctypes.c_size_t()
        _check(lib().helm_workspace_bytes(self.h, nrhs, ctypes.byref(b)), "helm_workspace_bytes")
        return b.value

    def workspace(self, nrhs):
        """A cached device workspace for nrhs columns (torch uint8 buffer)."""
        ws = self._ws.get(nrhs)
        if ws is None:
            self._ws.clear()
            ws = self.torch.empty(self.workspace_bytes(nrhs), dtype=self.torch.uint8, device="cuda")
            self._ws[nrhs] = ws
        return ws

    # -- helpers ----------------------------------------------------------------
    def _vec_dtype(self, prec):
        return self.torch.complex128 if prec == HELM_FP64 else self.torch.complex64

    def _prec(self, prec):
        if prec is None:
            return self.prec_code
        return {"fp64": HELM_FP64, "fp32": HELM_FP32_MG, HELM_FP64: HELM_FP64,
                HELM_FP32_MG: HELM_FP32_MG}[prec]

    @staticmethod
    def _cols(t):
        return 1 if t.dim() == 1 else t.shape[0]

    def _check_vec(self, t, n_nodes, dtype, what):
        if t.device.type != "cuda" or t.dtype != dtype or not t.is_contiguous():
            raise ValueError("%s must be a contiguous %s CUDA tensor" % (what, dtype))
        if t.shape[-1] != n_nodes:
            raise ValueError("%s has %d nodes, expected %d" % (what, t.shape[-1], n_nodes))

    # -- the solve ------------------------------------------------------------------
    def solve(self, rhs, x=None, tol=1e-8, workspace=None, x0=None):
        """x = B^{-1} rhs (FP64 outer FGMRES or Richardson, as built); returns
        (x, stats dict).  x0: initial guess (copied into x; needs a solver
        built with x0_given=True, which otherwise starts from 0)."""
        torch = self.torch
        self._check_vec(rhs, self.NV, torch.complex128, "rhs")
        nrhs = self._cols(rhs)
        if x is None:
            x = torch.empty_like(rhs)
        self._check_vec(x, self.NV, torch.complex128, "x")
        if x0 is not None:
            if not self.x0_given:
                raise ValueError("x0 needs a Solver built with x0_given=True")
            x.copy_(x0)
        elif self.x0_given:
            raise ValueError("this Solver was built with x0_given=True: pass x0")
        ws = self.workspace(nrhs) if workspace is None else workspace
        st = helm_stats()
        rc = lib().helm_solve(self.h, _ptr(rhs), _ptr(x), nrhs, float(tol), _ptr(ws),
                              ctypes.byref(st))
        if rc not in (HELM_OK, HELM_ENOCONV):
            raise HelmError(rc, "helm_solve")
        d = st.as_dict()
        d["status"] = rc
        return x, d

    def load_nodal(self, f):
        """b = M f for real FP64 nodal values f (nrhs, N) on the device; on a
        mixed handle the mixed right-hand side [M f / (delta - ik) | 0]."""
        torch = self.torch
        if f.dtype != torch.float64 or f.device.type != "cuda" or not f.is_contiguous():
            raise ValueError("f must be a contiguous float64 CUDA tensor")
        nrhs = self._cols(f)
        shape = f.shape[:-1] + (self.NV,)
        b = torch.empty(shape, dtype=torch.complex128, device=f.device)
        _check(lib().helm_load_nodal(self.h, _ptr(f), _ptr(b), nrhs), "helm_load_nodal")
        return b

    # -- the individual steps ------------------------------------------------------
    def apply(self, op, x, level=0, prec=None):
        p = self._prec(prec)
        n_len = self.NV if op.startswith("MIXED") else self.nodes(level)
        self._check_vec(x, n_len, self._vec_dtype(p), "x")
        y = self.torch.empty_like(x)
        _check(lib().helm_apply(self.h, OPS[op], level, p, _ptr(x), _ptr(y), self._cols(x)),
               "helm_apply")
        return y

    def hss_residual(self, R, u=None, prec=None):
        p = self._prec(prec)
        self._check_vec(R, self.N, self._vec_dtype(p), "R")
        if u is not None:
            self._check_vec(u, self.N, self._vec_dtype(p), "u")
        rho = self.torch.empty_like(R)
        _check(lib().helm_hss_residual(self.h, p, _ptr(R), _ptr(u), _ptr(rho), self._cols(R)),
               "helm_hss_residual")
        return rho

    def jacobi(self, b, x_in=None, level=0, prec=None):
        p = self._prec(prec)
        self._check_vec(b, self.nodes(level), self._vec_dtype(p), "b")
        out = self.torch.empty_like(b)
        _check(lib().helm_jacobi(self.h, level, p, _ptr(x_in), _ptr(b), _ptr(out), self._cols(b)),
               "helm_jacobi")
        return out

    def restrict_residual(self, x, b, level=0, prec=None):
        p = self._prec(prec)
        nrhs = self._cols(b)
        shape = (self.nodes(level + 1),) if b.dim() == 1 else (nrhs, self.nodes(level + 1))
        bc = self.torch.empty(shape, dtype=b.dtype, device=b.device)
        _check(lib().helm_restrict_residual(self.h, level, p, _ptr(x), _ptr(b), _ptr(bc), nrhs),
               "helm_restrict_residual")
        return bc

    def prolong_correct(self, e, x, level=0, prec=None):
        """x += P e in place; returns x."""
        p = self._prec(prec)
        _check(lib().helm_prolong_correct(self.h, level, p, _ptr(e), _ptr(x), self._cols(x)),
               "helm_prolong_correct")
        return x

    def coarse_solve(self, b, prec=None):
        p = self._prec(prec)
        x = self.torch.empty_like(b)
        _check(lib().helm_coarse_solve(self.h, p, _ptr(b), _ptr(x), self._cols(b)),
               "helm_coarse_solve")
        return x

    def vcycle(self, b):
        x = self.torch.empty_like(b)
        nrhs = self._cols(b)
        _check(lib().helm_vcycle(self.h, self.prec_code, _ptr(b), _ptr(x), nrhs,
                                 _ptr(self.workspace(nrhs))), "helm_vcycle")
        return x

    def vcycle_noalloc(self, b, x=None):
        """The cycle of vcycle() through helm_vcycle_noalloc: the level
        vectors live in the library's per-device scratch (no workspace)."""
        if x is None:
            x = self.torch.empty_like(b)
        _check(lib().helm_vcycle_noalloc(self.h, self.prec_code, _ptr(b), _ptr(x), self._cols(b)),
               "helm_vcycle_noalloc")
        return x

    def hss_history(self, v):
        """(z, res): the preconditioner applied to v, and res[c, s] =
        ||v_c - B_shift u_s|| after HSS step s (res[c, 0] = ||v_c||), a
        float64 numpy array (nrhs, hss_steps + 1)."""
        import numpy as np
        self._check_vec(v, self.NV, self.torch.complex128, "v")
        z = self.torch.empty_like(v)
        nrhs = self._cols(v)
        steps = self.n_hss
        res = np.zeros((nrhs, steps + 1), dtype=np.float64)
        _check(lib().helm_hss_history(self.h, _ptr(v), _ptr(z), nrhs, _ptr(self.workspace(nrhs)),
                                      res.ctypes.data_as(ctypes.POINTER(ctypes.c_double))),
               "helm_hss_history")
        return z, res

    def precondition(self, v):
        self._check_vec(v, self.NV, self.torch.complex128, "v")
        z = self.torch.empty_like(v)
        nrhs = self._cols(v)
        _check(lib().helm_precondition(self.h, _ptr(v), _ptr(z), nrhs,
                                       _ptr(self.workspace(nrhs))), "helm_precondition")
        return z


class Server:
    """helm_server_t: continuous batching of independent solves (marshalling
    only; admission, batching and the solves run in libhelm)."""

    def __init__(self, hbm_budget_bytes, max_cols=8, precision="fp32", restart=0, max_outer=0):
        import torch
        self.torch = torch
        o = helm_server_opts(float(hbm_budget_bytes), int(max_cols),
                             HELM_FP64 if precision == "fp64" else HELM_FP32_MG,
                             int(restart), int(max_outer))
        handle = ctypes.c_void_p()
        _check(lib().helm_server_create(ctypes.byref(o), ctypes.byref(handle)), "helm_server_create")
        self.s = handle
        self._keep = {}  # request id -> (rhs, x) tensors kept alive until done

    def submit(self, rhs, n, levels, k, delta_hat=None, dim=2, tol=1e-8):
        """Queue rhs (complex128 CUDA tensor, (nrhs, N)); returns (id, x)."""
        if rhs.dtype != self.torch.complex128 or rhs.device.type != "cuda" or not rhs.is_contiguous():
            raise ValueError("rhs must be a contiguous complex128 CUDA tensor")
        rhs2 = rhs if rhs.dim() == 2 else rhs[None]
        x = self.torch.empty_like(rhs2)
        rid = ctypes.c_longlong()
        dh = float(k) if delta_hat is None else float(delta_hat)
        _check(lib().helm_server_submit(self.s, dim, n, levels, float(k), dh, _ptr(rhs2), _ptr(x),
                                        rhs2.shape[0], float(tol), ctypes.byref(rid)),
               "helm_server_submit")
        self._keep[rid.value] = (rhs2, x)
        return rid.value, x

    def step(self):
        done = ctypes.c_int()
        _check(lib().helm_server_step(self.s, ctypes.byref(done)), "helm_server_step")
        return done.value

    def query(self, rid):
        info = helm_request_info()
        _check(lib().helm_server_query(self.s, rid, ctypes.byref(info)), "helm_server_query")
        d = info.as_dict()
        if d["status"] == 2:
            self._keep.pop(rid, None)
        return d

    def load(self):
        q, r, b = ctypes.c_int(), ctypes.c_int(), ctypes.c_double()
        _check(lib().helm_server_load(self.s, ctypes.byref(q), ctypes.byref(r), ctypes.byref(b)),
               "helm_server_load")
        return q.value, r.value, b.value

    def close(self):
        if getattr(self, "s", None):
            lib().helm_server_destroy(self.s)
            self.s = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
