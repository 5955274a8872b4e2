"""ctypes binding of include/nc.h (argument marshalling only).

Every computation runs in the HIP library libnc.so; PyTorch supplies device memory
(the workspace and the caller's arrays) and the HIP stream.  Importing this module
does not need a GPU, but creating a Solver does, and a missing library raises.
"""

import ctypes
import os

import torch

from .build import lib_path

NC_OK, NC_NOT_CONVERGED = 0, 1
NC_EINVAL, NC_ENOMEM, NC_EHIP, NC_ENAN = -1, -2, -3, -4
NC_FP64, NC_MIXED = 0, 1
NC_DENSE_MAX = 2000   # largest coarsest-grid system inverted densely
NC_HIST_MAX = 32      # Newton steps / refinement sweeps recorded per solve
NC_FILTER_CONE, NC_FILTER_PDE = 0, 1
NC_MMA_ROWS = 10

EXPORTED = [
    "nc_problem_default", "nc_workspace_bytes", "nc_create", "nc_destroy", "nc_status_string",
    "nc_set_design", "nc_get_gamma", "nc_filter_apply", "nc_residual", "nc_linearize", "nc_jac_apply", "nc_jacT_apply",
    "nc_jac_apply_f32", "nc_jacT_apply_f32", "nc_solve_state", "nc_objective", "nc_objective_grad",
    "nc_solve_adjoint", "nc_sensitivity", "nc_objective_sensitivity", "nc_volume", "nc_set_problem", "nc_mma_update", "nc_precondition", "nc_cone_filter", "nc_dense_inverse",
    "nc_dense_inverse_noalloc", "nc_set_timing", "nc_get_timing",
    "nc_ns_workspace_bytes", "nc_ns_create", "nc_ns_destroy", "nc_ns_set_problem", "nc_ns_set_design", "nc_ns_get_gamma", "nc_ns_residual",
    "nc_ns_linearize", "nc_ns_jac_apply", "nc_ns_jacT_apply", "nc_ns_precondition", "nc_ns_solve_state",
    "nc_ns_objective", "nc_ns_objective_grad", "nc_ns_solve_adjoint", "nc_ns_sensitivity",
]

TIMER_CLASSES = ["residual", "jv", "jtw", "smooth", "smooth_T", "pt_residual", "diag", "uproj", "transfer",
                 "coarse", "mdot", "maxpy", "vector", "setup", "smooth_coarse", "pt_residual_coarse"]


class NCProblem(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int), ("ny", ctypes.c_int), ("nz", ctypes.c_int),
        ("h", ctypes.c_double),
        ("rho0", ctypes.c_double), ("mu", ctypes.c_double), ("cp", ctypes.c_double), ("g0", ctypes.c_double),
        ("alpha", ctypes.c_double),
        ("k_f", ctypes.c_double), ("k_s", ctypes.c_double),
        ("kappa_f", ctypes.c_double), ("kappa_s", ctypes.c_double),
        ("q_c", ctypes.c_double), ("q_p", ctypes.c_double),
        ("q_h", ctypes.c_double),
        ("patch_x0", ctypes.c_double), ("patch_x1", ctypes.c_double),
        ("patch_y0", ctypes.c_double), ("patch_y1", ctypes.c_double),
        ("Q", ctypes.c_double),
        ("filter_radius", ctypes.c_double),
        ("precision", ctypes.c_int), ("levels", ctypes.c_int),
        ("newton_step_rtol", ctypes.c_double), ("krylov_rtol", ctypes.c_double), ("adjoint_rtol", ctypes.c_double),
        ("newton_maxit", ctypes.c_int), ("krylov_restart", ctypes.c_int), ("krylov_maxit", ctypes.c_int),
        ("smooth_pre", ctypes.c_int), ("smooth_post", ctypes.c_int),
        ("smooth_omega", ctypes.c_double),
        ("smooth_pre_coarse", ctypes.c_int), ("smooth_post_coarse", ctypes.c_int),
        ("krylov_rtol_mixed", ctypes.c_double), ("gs_passes", ctypes.c_int),
        ("coarse_tail", ctypes.c_int), ("newton_eta0", ctypes.c_double),
        ("filter_kind", ctypes.c_int),
        ("sym_x", ctypes.c_int), ("sym_y", ctypes.c_int),
        ("q_box", ctypes.c_double * 6), ("solid_box", ctypes.c_double * 6), ("design_box", ctypes.c_double * 6),
        ("smooth_omega_fallback", ctypes.c_double), ("f64_krylov_fallback", ctypes.c_int),
    ]


class NCInfo(ctypes.Structure):
    _fields_ = [
        ("newton_its", ctypes.c_int), ("krylov_its", ctypes.c_int), ("refine_its", ctypes.c_int),
        ("levels", ctypes.c_int),
        ("res0", ctypes.c_double * 5), ("res", ctypes.c_double * 5), ("rel_res", ctypes.c_double),
        ("t_setup", ctypes.c_double), ("t_solve", ctypes.c_double), ("t_total", ctypes.c_double),
        ("hist_len", ctypes.c_int), ("hist_krylov", ctypes.c_int * NC_HIST_MAX),
        ("hist_res", (ctypes.c_double * 5) * NC_HIST_MAX), ("krylov_f64", ctypes.c_int),
    ]

    def as_dict(self):
        n = self.hist_len
        return {"newton_its": self.newton_its, "krylov_its": self.krylov_its, "refine_its": self.refine_its,
                "levels": self.levels, "res0": list(self.res0), "res": list(self.res), "rel_res": self.rel_res,
                "t_setup": self.t_setup, "t_solve": self.t_solve, "t_total": self.t_total,
                "hist_krylov": list(self.hist_krylov[:n]), "hist_res": [list(self.hist_res[k]) for k in range(n)],
                "krylov_f64": self.krylov_f64}


_LIB = None


def load():
    """Load libnc.so from the package's lib/ directory (raises if it was not built)."""
    global _LIB
    if _LIB is None:
        path = lib_path()
        if not os.path.exists(path):
            raise RuntimeError(f"HIP library not built: {path} missing (run paper_1904_00182_amd/build.py)")
        lib = ctypes.CDLL(path)
        P, I, D, V, S = ctypes.POINTER(NCProblem), ctypes.c_int, ctypes.c_double, ctypes.c_void_p, ctypes.c_size_t
        sig = {
            "nc_problem_default": (None, [P, I, I, I]),
            "nc_workspace_bytes": (S, [P]),
            "nc_create": (I, [P, V, S, V, ctypes.POINTER(V)]),
            "nc_destroy": (I, [V]),
            "nc_status_string": (ctypes.c_char_p, [I]),
            "nc_set_design": (I, [V, V]),
            "nc_get_gamma": (I, [V, V]),
            "nc_filter_apply": (I, [V, I, V, V]),
            "nc_residual": (I, [V, V, V]),
            "nc_linearize": (I, [V, V]),
            "nc_jac_apply": (I, [V, V, V]),
            "nc_precondition": (I, [V, I, V, V, V]),
            "nc_jacT_apply": (I, [V, V, V]),
            "nc_jac_apply_f32": (I, [V, V, V]),
            "nc_jacT_apply_f32": (I, [V, V, V]),
            "nc_solve_state": (I, [V, V, ctypes.POINTER(NCInfo)]),
            "nc_objective": (I, [V, V, ctypes.POINTER(D)]),
            "nc_objective_grad": (I, [V, V, V]),
            "nc_objective_sensitivity": (I, [V, V, V, V, V]),
            "nc_volume": (I, [V, ctypes.POINTER(D), V]),
            "nc_set_problem": (I, [V, P]),
            "nc_mma_update": (I, [V, I, V, V, D, V, D, V, ctypes.POINTER(D)]),
            "nc_solve_adjoint": (I, [V, V, V, V, ctypes.POINTER(NCInfo)]),
            "nc_sensitivity": (I, [V, V, V, V, V]),
            "nc_cone_filter": (I, [I, I, I, D, V, V, I, V]),
            "nc_dense_inverse": (I, [V, I, V, V, V]),
            "nc_dense_inverse_noalloc": (I, [V, I, V]),
            "nc_set_timing": (I, [V, I]),
            "nc_get_timing": (I, [V, ctypes.POINTER(D), ctypes.POINTER(ctypes.c_long), ctypes.POINTER(D), I]),
            "nc_ns_workspace_bytes": (S, [P]),
            "nc_ns_create": (I, [P, V, S, V, ctypes.POINTER(V)]),
            "nc_ns_destroy": (I, [V]),
            "nc_ns_set_problem": (I, [V, P]),
            "nc_ns_set_design": (I, [V, V]),
            "nc_ns_get_gamma": (I, [V, V]),
            "nc_ns_residual": (I, [V, V, V]),
            "nc_ns_linearize": (I, [V, V]),
            "nc_ns_jac_apply": (I, [V, V, V]),
            "nc_ns_jacT_apply": (I, [V, V, V]),
            "nc_ns_precondition": (I, [V, I, V, V]),
            "nc_ns_solve_state": (I, [V, V, ctypes.POINTER(NCInfo)]),
            "nc_ns_objective": (I, [V, V, ctypes.POINTER(D)]),
            "nc_ns_objective_grad": (I, [V, V, V]),
            "nc_ns_solve_adjoint": (I, [V, V, V, V, ctypes.POINTER(NCInfo)]),
            "nc_ns_sensitivity": (I, [V, V, V, V, V]),
        }
        for name, (res, argt) in sig.items():
            f = getattr(lib, name)
            f.restype = res
            f.argtypes = argt
        _LIB = lib
    return _LIB


def default_problem(nx, ny, nz, **overrides):
    p = NCProblem()
    load().nc_problem_default(ctypes.byref(p), nx, ny, nz)
    for k, v in overrides.items():
        if not hasattr(p, k):
            raise KeyError(k)
        if k in ("q_box", "solid_box", "design_box"):
            v = (ctypes.c_double * 6)(*v)
        setattr(p, k, v)
    return p


def copy_problem(problem, **overrides):
    """A copy of an NCProblem with some fields replaced."""
    p = NCProblem()
    ctypes.memmove(ctypes.byref(p), ctypes.byref(problem), ctypes.sizeof(NCProblem))
    for k, v in overrides.items():
        if not hasattr(p, k):
            raise KeyError(k)
        if k in ("q_box", "solid_box", "design_box"):
            v = (ctypes.c_double * 6)(*v)
        setattr(p, k, v)
    return p


def workspace_bytes(problem):
    return int(load().nc_workspace_bytes(ctypes.byref(problem)))


class NCError(RuntimeError):
    def __init__(self, status, what):
        self.status = status
        super().__init__(f"{what}: {load().nc_status_string(status).decode()} ({status})")


def _check(status, what, allow_not_converged=False):
    if status == NC_OK or (allow_not_converged and status == NC_NOT_CONVERGED):
        return status
    raise NCError(status, what)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


def _stream_handle(stream):
    return ctypes.c_void_p(stream.cuda_stream if stream is not None else 0)


class Solver:
    """One solver context: a caller-owned workspace tensor on `device` and one stream."""

    def __init__(self, problem, device="cuda:0", stream=None):
        self.lib = load()
        self.p = problem
        self.device = torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.nbytes = workspace_bytes(problem)
        if self.nbytes == 0:
            raise NCError(NC_EINVAL, "nc_workspace_bytes")
        self.workspace = torch.empty(self.nbytes + 256, dtype=torch.uint8, device=self.device)
        self.ctx = ctypes.c_void_p()
        _check(self.lib.nc_create(ctypes.byref(problem), _ptr(self.workspace), self.nbytes + 256,
                                  _stream_handle(self.stream), ctypes.byref(self.ctx)), "nc_create")
        self.N = (problem.nx + 1) * (problem.ny + 1) * (problem.nz + 1)
        self.E = problem.nx * problem.ny * problem.nz
        self.last_info = None

    def close(self):
        if self.ctx:
            self.lib.nc_destroy(self.ctx)
            self.ctx = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- helpers
    def _vec(self, dtype=torch.float64):
        return torch.zeros((self.N, 5), dtype=dtype, device=self.device)

    def _in(self, t, shape, dtype=torch.float64):
        t = torch.as_tensor(t).to(device=self.device, dtype=dtype).contiguous()
        if tuple(t.shape) != tuple(shape) and t.numel() != int(torch.tensor(shape).prod()):
            raise ValueError(f"expected shape {shape}, got {tuple(t.shape)}")
        return t.reshape(shape)

    # -- C ABI, one method per entry point
    def set_design(self, x):
        self._x = self._in(x, (self.E,))
        _check(self.lib.nc_set_design(self.ctx, _ptr(self._x)), "nc_set_design")

    def gamma(self):
        g = torch.empty(self.E, dtype=torch.float64, device=self.device)
        _check(self.lib.nc_get_gamma(self.ctx, _ptr(g)), "nc_get_gamma")
        return g

    def filter_apply(self, x, transpose=False):
        """y = F x (F^T x) with the context's density filter, via nc_filter_apply."""
        x = self._in(x, (self.E,))
        y = torch.empty(self.E, dtype=torch.float64, device=self.device)
        _check(self.lib.nc_filter_apply(self.ctx, 1 if transpose else 0, _ptr(x), _ptr(y)), "nc_filter_apply")
        return y

    def residual(self, s):
        s = self._in(s, (self.N, 5))
        r = self._vec()
        _check(self.lib.nc_residual(self.ctx, _ptr(s), _ptr(r)), "nc_residual")
        return r

    def linearize(self, s):
        self._lin = self._in(s, (self.N, 5))
        _check(self.lib.nc_linearize(self.ctx, _ptr(self._lin)), "nc_linearize")

    def jac_apply(self, v, transpose=False):
        dt = v.dtype if v.dtype in (torch.float32, torch.float64) else torch.float64
        v = self._in(v, (self.N, 5), dt)
        y = self._vec(dt)
        if dt == torch.float64:
            f = self.lib.nc_jacT_apply if transpose else self.lib.nc_jac_apply
        else:
            f = self.lib.nc_jacT_apply_f32 if transpose else self.lib.nc_jac_apply_f32
        _check(f(self.ctx, _ptr(v), _ptr(y)), "nc_jac_apply")
        return y

    def precondition(self, s, v, transpose=False):
        """z = M^-1 v (M^-T v) for the (P, T) pairs v [N][2]: one multigrid V-cycle of the
        Krylov preconditioner, with the hierarchy rebuilt at the state s [N][5]."""
        s = self._in(s, (self.N, 5), torch.float64)
        v = self._in(v, (self.N, 2), torch.float64)
        z = torch.empty((self.N, 2), dtype=torch.float64, device=self.device)
        _check(self.lib.nc_precondition(self.ctx, 1 if transpose else 0, _ptr(s), _ptr(v), _ptr(z)),
               "nc_precondition")
        return z

    def solve_state(self, s0=None, out=None):
        s = out if out is not None else self._vec()
        if s0 is not None:
            s.copy_(self._in(s0, (self.N, 5)))
        elif out is None:
            s.zero_()
        info = NCInfo()
        st = _check(self.lib.nc_solve_state(self.ctx, _ptr(s), ctypes.byref(info)), "nc_solve_state",
                    allow_not_converged=True)
        self.last_info = info.as_dict()
        self.last_info["status"] = st
        return s

    def objective(self, s):
        s = self._in(s, (self.N, 5))
        f = ctypes.c_double()
        _check(self.lib.nc_objective(self.ctx, _ptr(s), ctypes.byref(f)), "nc_objective")
        return f.value

    def objective_grad(self, s=None):
        """d f / d s of the compliance; s is required when the problem has a volumetric
        source (its SUPG-weighted load depends on the state)."""
        g = self._vec()
        sp = _ptr(self._in(s, (self.N, 5))) if s is not None else None
        _check(self.lib.nc_objective_grad(self.ctx, sp, _ptr(g)), "nc_objective_grad")
        return g

    def objective_sensitivity(self, s, lam, with_gamma=False):
        """d f / d x of nc_objective (adjoint term plus the explicit design term)."""
        s = self._in(s, (self.N, 5))
        lam = self._in(lam, (self.N, 5))
        dfdx = torch.empty(self.E, dtype=torch.float64, device=self.device)
        dfdg = torch.empty(self.E, dtype=torch.float64, device=self.device) if with_gamma else None
        _check(self.lib.nc_objective_sensitivity(self.ctx, _ptr(s), _ptr(lam), _ptr(dfdx),
                                                 _ptr(dfdg) if dfdg is not None else None), "nc_objective_sensitivity")
        return (dfdx, dfdg) if with_gamma else dfdx

    def volume(self, with_grad=True):
        """(solid fraction of the design domain, its gradient w.r.t. x or None)."""
        frac = ctypes.c_double()
        dg = torch.empty(self.E, dtype=torch.float64, device=self.device) if with_grad else None
        _check(self.lib.nc_volume(self.ctx, ctypes.byref(frac), _ptr(dg) if dg is not None else None), "nc_volume")
        return frac.value, dg

    def solve_adjoint(self, s, rhs, out=None):
        s = self._in(s, (self.N, 5))
        rhs = self._in(rhs, (self.N, 5))
        lam = out if out is not None else self._vec()
        info = NCInfo()
        st = _check(self.lib.nc_solve_adjoint(self.ctx, _ptr(s), _ptr(rhs), _ptr(lam), ctypes.byref(info)),
                    "nc_solve_adjoint", allow_not_converged=True)
        self.last_info = info.as_dict()
        self.last_info["status"] = st
        return lam

    def set_problem(self, problem):
        """Replace the context's parameters (same grid and layout) via nc_set_problem; the
        design must be set again afterwards."""
        _check(self.lib.nc_set_problem(self.ctx, ctypes.byref(problem)), "nc_set_problem")
        self.p = problem

    def mma_state(self):
        """A zeroed MMA state array (NC_MMA_ROWS x E) for mma_update."""
        return torch.zeros((NC_MMA_ROWS, self.E), dtype=torch.float64, device=self.device)

    def mma_update(self, it, x, dfdx, g, dgdx, move, state):
        """One MMA iteration on the design elements (x updated in place); returns lambda."""
        lam = ctypes.c_double()
        for t in (x, dfdx, dgdx, state):
            if t.dtype != torch.float64 or not t.is_contiguous() or t.device != self.device:
                raise ValueError("mma_update needs contiguous float64 tensors on the solver's device")
        _check(self.lib.nc_mma_update(self.ctx, int(it), _ptr(x), _ptr(dfdx), float(g), _ptr(dgdx), float(move),
                                      _ptr(state), ctypes.byref(lam)), "nc_mma_update")
        return lam.value

    def set_timing(self, enable=True):
        _check(self.lib.nc_set_timing(self.ctx, 1 if enable else 0), "nc_set_timing")

    def timing(self, with_bytes=False):
        """{class: (total ms, launches)} of the kernels timed since set_timing(True); with
        `with_bytes`, {class: (total ms, launches, algorithmic bytes)}."""
        n = len(TIMER_CLASSES)
        ms = (ctypes.c_double * n)()
        cnt = (ctypes.c_long * n)()
        by = (ctypes.c_double * n)()
        r = self.lib.nc_get_timing(self.ctx, ms, cnt, by, n)
        if r < 0:
            raise NCError(r, "nc_get_timing")
        if with_bytes:
            return {TIMER_CLASSES[k]: (ms[k], cnt[k], by[k]) for k in range(n)}
        return {TIMER_CLASSES[k]: (ms[k], cnt[k]) for k in range(n)}

    def sensitivity(self, s, lam, with_gamma=False):
        s = self._in(s, (self.N, 5))
        lam = self._in(lam, (self.N, 5))
        dfdx = torch.empty(self.E, dtype=torch.float64, device=self.device)
        dfdg = torch.empty(self.E, dtype=torch.float64, device=self.device) if with_gamma else None
        _check(self.lib.nc_sensitivity(self.ctx, _ptr(s), _ptr(lam), _ptr(dfdx),
                                       _ptr(dfdg) if dfdg is not None else None), "nc_sensitivity")
        return (dfdx, dfdg) if with_gamma else dfdx


def ns_workspace_bytes(problem):
    return int(load().nc_ns_workspace_bytes(ctypes.byref(problem)))


class NSSolver:
    """One context of the Navier-Stokes / Brinkman flow model (nc_ns_* entry points): a
    caller-owned workspace tensor on `device` and one stream."""

    def __init__(self, problem, device="cuda:0", stream=None):
        self.lib = load()
        self.p = problem
        self.device = torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.nbytes = ns_workspace_bytes(problem)
        if self.nbytes == 0:
            raise NCError(NC_EINVAL, "nc_ns_workspace_bytes")
        self.workspace = torch.empty(self.nbytes + 256, dtype=torch.uint8, device=self.device)
        self.ctx = ctypes.c_void_p()
        _check(self.lib.nc_ns_create(ctypes.byref(problem), _ptr(self.workspace), self.nbytes + 256,
                                     _stream_handle(self.stream), ctypes.byref(self.ctx)), "nc_ns_create")
        self.N = (problem.nx + 1) * (problem.ny + 1) * (problem.nz + 1)
        self.E = problem.nx * problem.ny * problem.nz
        self.last_info = None

    def close(self):
        if self.ctx:
            self.lib.nc_ns_destroy(self.ctx)
            self.ctx = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _vec(self):
        return torch.zeros((self.N, 5), dtype=torch.float64, device=self.device)

    _in = Solver._in

    def set_problem(self, problem):
        """Replace the context's parameters (same grid and layout) via nc_ns_set_problem; the
        design must be set again afterwards."""
        _check(self.lib.nc_ns_set_problem(self.ctx, ctypes.byref(problem)), "nc_ns_set_problem")
        self.p = problem

    def set_design(self, x):
        self._x = self._in(x, (self.E,))
        _check(self.lib.nc_ns_set_design(self.ctx, _ptr(self._x)), "nc_ns_set_design")

    def gamma(self):
        g = torch.empty(self.E, dtype=torch.float64, device=self.device)
        _check(self.lib.nc_ns_get_gamma(self.ctx, _ptr(g)), "nc_ns_get_gamma")
        return g

    def residual(self, s):
        s = self._in(s, (self.N, 5))
        r = self._vec()
        _check(self.lib.nc_ns_residual(self.ctx, _ptr(s), _ptr(r)), "nc_ns_residual")
        return r

    def linearize(self, s):
        self._lin = self._in(s, (self.N, 5))
        _check(self.lib.nc_ns_linearize(self.ctx, _ptr(self._lin)), "nc_ns_linearize")

    def jac_apply(self, v, transpose=False):
        v = self._in(v, (self.N, 5))
        y = self._vec()
        f = self.lib.nc_ns_jacT_apply if transpose else self.lib.nc_ns_jac_apply
        _check(f(self.ctx, _ptr(v), _ptr(y)), "nc_ns_jac_apply")
        return y

    def precondition(self, v, transpose=False):
        v = self._in(v, (self.N, 5))
        z = self._vec()
        _check(self.lib.nc_ns_precondition(self.ctx, 1 if transpose else 0, _ptr(v), _ptr(z)), "nc_ns_precondition")
        return z

    def solve_state(self, s0=None, out=None):
        s = out if out is not None else self._vec()
        if s0 is not None:
            s.copy_(self._in(s0, (self.N, 5)))
        elif out is None:
            s.zero_()
        info = NCInfo()
        st = _check(self.lib.nc_ns_solve_state(self.ctx, _ptr(s), ctypes.byref(info)), "nc_ns_solve_state",
                    allow_not_converged=True)
        self.last_info = info.as_dict()
        self.last_info["status"] = st
        return s

    def objective(self, s):
        s = self._in(s, (self.N, 5))
        f = ctypes.c_double()
        _check(self.lib.nc_ns_objective(self.ctx, _ptr(s), ctypes.byref(f)), "nc_ns_objective")
        return f.value

    def objective_grad(self, s):
        s = self._in(s, (self.N, 5))
        g = self._vec()
        _check(self.lib.nc_ns_objective_grad(self.ctx, _ptr(s), _ptr(g)), "nc_ns_objective_grad")
        return g

    def solve_adjoint(self, s, rhs, out=None):
        s = self._in(s, (self.N, 5))
        rhs = self._in(rhs, (self.N, 5))
        lam = out if out is not None else self._vec()
        info = NCInfo()
        st = _check(self.lib.nc_ns_solve_adjoint(self.ctx, _ptr(s), _ptr(rhs), _ptr(lam), ctypes.byref(info)),
                    "nc_ns_solve_adjoint", allow_not_converged=True)
        self.last_info = info.as_dict()
        self.last_info["status"] = st
        return lam

    def sensitivity(self, s, lam, with_gamma=False):
        s = self._in(s, (self.N, 5))
        lam = self._in(lam, (self.N, 5))
        dfdx = torch.empty(self.E, dtype=torch.float64, device=self.device)
        dfdg = torch.empty(self.E, dtype=torch.float64, device=self.device) if with_gamma else None
        _check(self.lib.nc_ns_sensitivity(self.ctx, _ptr(s), _ptr(lam), _ptr(dfdx),
                                          _ptr(dfdg) if dfdg is not None else None), "nc_ns_sensitivity")
        return (dfdx, dfdg) if with_gamma else dfdx


def cone_filter(x, nx, ny, nz, radius, stream=None):
    """y = F_R x on an nx*ny*nz element grid (device tensors), via nc_cone_filter."""
    x = x.contiguous().to(torch.float64)
    y = torch.empty_like(x)
    st = stream if stream is not None else torch.cuda.current_stream(x.device)
    _check(load().nc_cone_filter(nx, ny, nz, float(radius), _ptr(x), _ptr(y), 0, _stream_handle(st)),
           "nc_cone_filter")
    return y


def dense_inverse(a, stream=None):
    """(A^-1, (A^-1)^T) of a square float64 device tensor via nc_dense_inverse, the
    multigrid's coarsest-grid inverse."""
    n = a.shape[0]
    if a.dim() != 2 or a.shape[1] != n:
        raise ValueError("dense_inverse needs a square matrix")
    buf = torch.empty(2 * n * n, dtype=torch.float64, device=a.device)
    buf[: n * n].copy_(a.reshape(-1))
    iwork = torch.empty(2 * max(n, 1), dtype=torch.int32, device=a.device)
    dwork = torch.empty(2 * max(n, 1), dtype=torch.float64, device=a.device)
    st = stream if stream is not None else torch.cuda.current_stream(a.device)
    _check(load().nc_dense_inverse(_ptr(buf), n, _ptr(iwork), _ptr(dwork), _stream_handle(st)), "nc_dense_inverse")
    return buf[: n * n].view(n, n), buf[n * n:].view(n, n)


def dense_inverse_noalloc(buf, n, stream=None):
    """In-place nc_dense_inverse_noalloc on a float64 device buffer of 2 n^2 entries whose
    first n^2 hold A: afterwards they hold A^-1 and the next n^2 (A^-1)^T.  No device
    memory is allocated (the library's static scratch is used)."""
    if buf.dtype != torch.float64 or buf.numel() < 2 * n * n or not buf.is_contiguous():
        raise ValueError("dense_inverse_noalloc needs a contiguous float64 buffer of 2 n^2 entries")
    st = stream if stream is not None else torch.cuda.current_stream(buf.device)
    _check(load().nc_dense_inverse_noalloc(_ptr(buf), n, _stream_handle(st)), "nc_dense_inverse_noalloc")
    return buf
