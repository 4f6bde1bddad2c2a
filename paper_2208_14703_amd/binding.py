"""Thin ctypes binding over libm1mg.so (include/m1.h).

The binding only marshals arguments. Every step of the solver runs in the HIP
library. PyTorch supplies device memory (float64 tensors) and the current HIP
stream.

State tensors are float64 of shape (4, ny, nx) holding E, Fx, Fy, T. In 1-D the
shape is (4, 1, nx) and the Fy plane is not passed to the library (NULL).
Opacity tensors are float64 of shape (2, ny, nx) holding sigma_a, sigma_s.

Importing this module does not load the library. The first call that needs it
loads it and raises RuntimeError when it is missing: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "_lib", "libm1mg.so")

BC = {"periodic": 0, "reflective": 1, "neumann": 2, "dirichlet": 3, "inflow": 4}
PRECISION = {"fp64": 0, "mixed": 1}
DTAU_RULE = {"signed": 0, "literal": 1}
SMOOTHER = {"jacobi": 0, "rbgs": 1}
CYCLE = {"V": 0, "W": 1, "F": 2}
TRANSFER = {"full": 0, "mean": 1}
STATUS = {0: "M1_OK", 1: "M1_ERR_ARG", 2: "M1_ERR_NOT_ADMISSIBLE", 3: "M1_ERR_NO_CONVERGENCE", 4: "M1_ERR_WORKSPACE",
          5: "M1_ERR_DEVICE", 6: "M1_ERR_BUSY", 7: "M1_ERR_BUDGET"}


class M1Error(RuntimeError):
    def __init__(self, status: int, what: str):
        super().__init__(f"{what}: {STATUS.get(status, status)}")
        self.status = status


class m1_bc(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("pad_", ctypes.c_int32), ("E", ctypes.c_double), ("Fx", ctypes.c_double),
                ("Fy", ctypes.c_double), ("lo", ctypes.c_double), ("hi", ctypes.c_double), ("Eo", ctypes.c_double)]


class m1_grid(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int32), ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("pad_", ctypes.c_int32),
                ("hx", ctypes.c_double), ("hy", ctypes.c_double), ("dt", ctypes.c_double), ("c", ctypes.c_double),
                ("a_r", ctypes.c_double), ("c_v", ctypes.c_double), ("bc", m1_bc * 4)]


class m1_params(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int32) for n in ("levels", "nu0", "nu_l", "pseudo_steps", "sub_steps", "max_cycles",
                                              "dtau_rule", "pseudo_local", "precision", "smoother", "cycle",
                                              "transfer", "dtau_carry", "pad_")] + \
               [(n, ctypes.c_double) for n in ("dtau_im0", "eps_inc", "eps_dec", "eta", "rtol", "dtau_min",
                                               "dtau_max", "omega")]


class m1_state(ctypes.Structure):
    _fields_ = [("E", ctypes.c_void_p), ("Fx", ctypes.c_void_p), ("Fy", ctypes.c_void_p), ("T", ctypes.c_void_p)]


class m1_bc3(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("pad_", ctypes.c_int32), ("E", ctypes.c_double), ("Fx", ctypes.c_double),
                ("Fy", ctypes.c_double), ("Fz", ctypes.c_double)]


class m1_grid3(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32), ("pad_", ctypes.c_int32),
                ("hx", ctypes.c_double), ("hy", ctypes.c_double), ("hz", ctypes.c_double), ("dt", ctypes.c_double),
                ("c", ctypes.c_double), ("a_r", ctypes.c_double), ("c_v", ctypes.c_double), ("bc", m1_bc3 * 6)]


class m1_state3(ctypes.Structure):
    _fields_ = [(n, ctypes.c_void_p) for n in ("E", "Fx", "Fy", "Fz", "T")]


class m1_opacity(ctypes.Structure):
    _fields_ = [("sigma_a", ctypes.c_void_p), ("sigma_s", ctypes.c_void_p)]


class m1_info(ctypes.Structure):
    _fields_ = [("cycles", ctypes.c_int32), ("status", ctypes.c_int32), ("levels", ctypes.c_int32),
                ("steps_done", ctypes.c_int32), ("r0", ctypes.c_double), ("rel_residual", ctypes.c_double),
                ("dtau", ctypes.c_double), ("first_bad_cell", ctypes.c_int64), ("stalled_cells", ctypes.c_int64)]


_lib = None


def lib():
    """Load libm1mg.so (raises when it has not been built)."""
    global _lib
    if _lib is None:
        # The library must bind to the HIP runtime that torch uses (torch ships its own
        # copy): load torch's first, or the process ends up with two runtimes and the
        # library sees no device.
        import torch  # noqa: F401
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_2208_14703_amd.build.build() "
                               "(there is no CPU fallback)")
        L = ctypes.CDLL(LIB_PATH)
        P = ctypes.POINTER
        vp = ctypes.c_void_p
        L.m1_strerror.restype = ctypes.c_char_p
        L.m1_strerror.argtypes = [ctypes.c_int]
        L.m1_default_params.argtypes = [P(m1_params)]
        L.m1_workspace_bytes.restype = ctypes.c_size_t
        L.m1_workspace_bytes.argtypes = [P(m1_grid), P(m1_params)]
        L.m1_plan_create.argtypes = [P(m1_grid), P(m1_params), P(m1_opacity), vp, ctypes.c_size_t, vp, P(vp)]
        L.m1_plan_destroy.argtypes = [vp]
        L.m1_plan_levels.restype = ctypes.c_int32
        L.m1_plan_levels.argtypes = [vp]
        L.m1_level_dims.argtypes = [vp, ctypes.c_int32, P(ctypes.c_int32), P(ctypes.c_int32)]
        L.m1_residual.argtypes = [vp, P(m1_state), P(m1_state), P(ctypes.c_double), P(m1_state)]
        L.m1_vcycle.argtypes = [vp, P(m1_state), P(m1_state), ctypes.c_double, P(m1_info)]
        L.m1_step.argtypes = [vp, P(m1_state), ctypes.c_int32, P(m1_info)]
        L.m1_apply_A.argtypes = [vp, ctypes.c_int32, P(m1_state), P(m1_state)]
        L.m1_sweep.argtypes = [vp, P(m1_state), P(m1_state), P(m1_state)]
        L.m1_sweeps.argtypes = [vp, P(m1_state), P(m1_state), P(m1_state), ctypes.c_int32]
        L.m1_pseudo_step.argtypes = [vp, ctypes.c_int32, ctypes.c_double, P(m1_state), P(m1_state), P(m1_state)]
        L.m1_restrict.argtypes = [vp, ctypes.c_int32, P(m1_state), P(m1_state)]
        L.m1_prolong_project.argtypes = [vp, ctypes.c_int32, P(m1_state), P(m1_state), P(m1_state), P(m1_state)]
        L.m1_residual_restrict.argtypes = [vp, ctypes.c_int32, P(m1_state), P(m1_state), P(m1_state), P(m1_state)]
        L.m1_sync.argtypes = [vp]
        L.m1_stalls.argtypes = [vp, P(ctypes.c_int64), ctypes.c_int32]
        L.m1_stalls.restype = ctypes.c_int
        L.m1_step_static.argtypes = [P(m1_grid), P(m1_params), P(m1_opacity), P(m1_state), ctypes.c_int32, vp,
                                     P(m1_info)]
        L.m1_engine_request_bytes.restype = ctypes.c_size_t
        L.m1_engine_request_bytes.argtypes = [P(m1_grid), P(m1_params)]
        L.m1_engine_create.argtypes = [P(m1_params), vp, ctypes.c_size_t, ctypes.c_int32, vp, P(vp)]
        L.m1_engine_destroy.argtypes = [vp]
        L.m1_batch_submit.argtypes = [vp, P(m1_grid), P(m1_params), P(m1_opacity), P(m1_state), ctypes.c_int32,
                                      P(ctypes.c_uint64)]
        L.m1_batch_run.argtypes = [vp, ctypes.c_int32, P(ctypes.c_int32), P(ctypes.c_int32)]
        L.m1_batch_poll.argtypes = [vp, ctypes.c_uint64, P(m1_info)]
        L.m1_batch_wait.argtypes = [vp, ctypes.c_uint64, P(m1_info)]
        L.m1_batch_cancel.argtypes = [vp, ctypes.c_uint64]
        L.m1_batch_times.argtypes = [vp, ctypes.c_uint64, P(ctypes.c_double), P(ctypes.c_double),
                                     P(ctypes.c_double)]
        L.m1_batch_release.argtypes = [vp, ctypes.c_uint64]
        L.m1_engine_memory.argtypes = [vp, P(ctypes.c_size_t), P(ctypes.c_size_t), P(ctypes.c_int32),
                                       P(ctypes.c_int32)]
        L.m1_engine_memory.restype = ctypes.c_int
        L.m1_serve_start.argtypes = [vp, ctypes.c_int32]
        L.m1_serve_stop.argtypes = [vp]
        L.m1_tune_set.argtypes = [ctypes.c_char_p, ctypes.c_int64]
        L.m1_tune_set.restype = ctypes.c_int
        L.m1_tune_get.argtypes = [ctypes.c_char_p]
        L.m1_tune_get.restype = ctypes.c_int64
        L.m1_workspace3_bytes.restype = ctypes.c_size_t
        L.m1_workspace3_bytes.argtypes = [P(m1_grid3), P(m1_params)]
        L.m1_plan3_create.argtypes = [P(m1_grid3), P(m1_params), P(m1_opacity), vp, ctypes.c_size_t, vp, P(vp)]
        L.m1_plan3_destroy.argtypes = [vp]
        L.m1_plan3_levels.restype = ctypes.c_int32
        L.m1_plan3_levels.argtypes = [vp]
        L.m1_level3_dims.argtypes = [vp, ctypes.c_int32] + [P(ctypes.c_int32)] * 3
        L.m1_apply3.argtypes = [vp, ctypes.c_int32, P(m1_state3), P(m1_state3)]
        L.m1_sweep3.argtypes = [vp, P(m1_state3), P(m1_state3), P(m1_state3)]
        L.m1_pseudo_step3.argtypes = [vp, ctypes.c_int32, ctypes.c_double, P(m1_state3), P(m1_state3), P(m1_state3)]
        L.m1_restrict3.argtypes = [vp, ctypes.c_int32, P(m1_state3), P(m1_state3)]
        L.m1_prolong_project3.argtypes = [vp, ctypes.c_int32, P(m1_state3), P(m1_state3), P(m1_state3),
                                          P(m1_state3)]
        L.m1_residual3.argtypes = [vp, P(m1_state3), P(m1_state3), P(ctypes.c_double), P(m1_state3)]
        L.m1_vcycle3.argtypes = [vp, P(m1_state3), P(m1_state3), ctypes.c_double]
        L.m1_step3.argtypes = [vp, P(m1_state3), ctypes.c_int32, P(m1_info)]
        for name in ("m1_plan3_create", "m1_level3_dims", "m1_apply3", "m1_sweep3", "m1_pseudo_step3", "m1_restrict3",
                     "m1_prolong_project3", "m1_residual3", "m1_vcycle3", "m1_step3"):
            getattr(L, name).restype = ctypes.c_int
        for name in ("m1_plan_create", "m1_residual", "m1_vcycle", "m1_step", "m1_apply_A", "m1_sweep",
                     "m1_sweeps", "m1_pseudo_step", "m1_restrict", "m1_prolong_project", "m1_sync", "m1_level_dims",
                     "m1_engine_create", "m1_batch_submit", "m1_batch_run", "m1_batch_poll", "m1_batch_wait",
                     "m1_batch_cancel", "m1_batch_times", "m1_batch_release", "m1_serve_start", "m1_serve_stop",
                     "m1_step_static", "m1_residual_restrict"):
            getattr(L, name).restype = ctypes.c_int
        _lib = L
        _apply_stored_tuning(L)
    return _lib


TUNE_ENV = {"sweep_rows": "M1_SWEEP_ROWS", "pair_rows": "M1_PAIR_ROWS", "mx_sweep_rows": "M1_MX_SWEEP_ROWS",
            "residual_restrict": "M1_RESIDUAL_RESTRICT", "tail_cells": "M1_TAIL_CELLS",
            "tiled_max_cells": "M1_TILED_MAX_CELLS", "graphs": "M1_GRAPHS", "batch_grid": "M1_BATCH_GRID"}


def _apply_stored_tuning(L):
    """Launch-shape settings the autotuner stored for this device (environment variables take precedence)."""
    import torch
    if not torch.cuda.is_available():
        return
    from . import autotune
    settings = autotune.load(autotune.device_key()) or {}
    for key, value in settings.items():
        if key in TUNE_ENV and os.environ.get(TUNE_ENV[key]) is None:
            L.m1_tune_set(key.encode(), int(value))


def tune_set(key: str, value: int):
    """Set a launch-shape setting (m1_tune_set); applies to plans and engines created afterwards."""
    _check(lib().m1_tune_set(key.encode(), int(value)), "m1_tune_set")


def tune_get(key: str) -> int:
    return int(lib().m1_tune_get(key.encode()))


def _check(status: int, what: str):
    if status != 0:
        raise M1Error(status, what)


def make_grid(problem: dict) -> m1_grid:
    g = m1_grid()
    g.dim, g.nx, g.ny = problem["dim"], problem["nx"], problem["ny"]
    g.hx, g.hy, g.dt = problem["hx"], problem["hy"], problem["dt"]
    g.c, g.a_r, g.c_v = problem["c"], problem["a_r"], problem["c_v"]
    for s, bc in enumerate(problem["bc"]):
        g.bc[s].kind = BC[bc["kind"]]
        g.bc[s].E, g.bc[s].Fx, g.bc[s].Fy = bc.get("E", 0.0), bc.get("Fx", 0.0), bc.get("Fy", 0.0)
        g.bc[s].lo, g.bc[s].hi, g.bc[s].Eo = bc.get("lo", 0.0), bc.get("hi", 1.0), bc.get("Eo", 0.0)
    return g


def default_params(**kw) -> dict:
    """The paper's solver parameters (see m1_params in include/m1.h), updated with kw."""
    p = m1_params()
    lib().m1_default_params(ctypes.byref(p))
    d = {name: getattr(p, name) for name, _ in m1_params._fields_}
    d["dtau_rule"] = "signed"
    d["precision"] = "fp64"
    d["smoother"] = "jacobi"
    d["cycle"] = "V"
    d["transfer"] = "full"
    d.update(kw)
    return d


def make_params(d: dict) -> m1_params:
    p = m1_params()
    for k, v in d.items():
        if k == "precision":
            v = PRECISION[v] if isinstance(v, str) else v
        elif k == "dtau_rule":
            v = DTAU_RULE[v] if isinstance(v, str) else v
        elif k == "smoother":
            v = SMOOTHER[v] if isinstance(v, str) else v
        elif k == "cycle":
            v = CYCLE[v] if isinstance(v, str) else v
        elif k == "transfer":
            v = TRANSFER[v] if isinstance(v, str) else v
        setattr(p, k, v)
    return p


def _stream_handle(stream) -> int:
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream


class Plan:
    """A solver plan for one grid: level hierarchy in a torch-allocated workspace."""

    def __init__(self, problem: dict, sigma, params: dict | None = None, stream=None):
        import torch
        self.torch = torch
        self.problem = problem
        self.dim = problem["dim"]
        self.grid = make_grid(problem)
        self.params_d = default_params(**(params or {}))
        self.params = make_params(self.params_d)
        L = lib()
        self.sigma = sigma.contiguous()
        assert self.sigma.dtype == torch.float64 and self.sigma.is_cuda
        assert tuple(self.sigma.shape) == (2, problem["ny"], problem["nx"])
        nbytes = L.m1_workspace_bytes(ctypes.byref(self.grid), ctypes.byref(self.params))
        if nbytes == 0:
            raise M1Error(1, "m1_workspace_bytes")
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.sigma.device)
        base = self.workspace.data_ptr()
        off = (-base) % 256
        self.ws_ptr, self.ws_bytes = base + off, nbytes
        op = m1_opacity(self.sigma[0].data_ptr(), self.sigma[1].data_ptr())
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.sigma.device)
        h = ctypes.c_void_p()
        _check(L.m1_plan_create(ctypes.byref(self.grid), ctypes.byref(self.params), ctypes.byref(op),
                                ctypes.c_void_p(self.ws_ptr), self.ws_bytes, ctypes.c_void_p(self.stream.cuda_stream),
                                ctypes.byref(h)), "m1_plan_create")
        self.handle = h
        self.levels = L.m1_plan_levels(h)

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and _lib is not None:
            _lib.m1_plan_destroy(h)
            self.handle = None

    # ---- helpers
    def level_dims(self, level: int):
        nx, ny = ctypes.c_int32(), ctypes.c_int32()
        _check(lib().m1_level_dims(self.handle, level, ctypes.byref(nx), ctypes.byref(ny)), "m1_level_dims")
        return nx.value, ny.value

    def new_state(self, level: int = 0):
        nx, ny = self.level_dims(level)
        return self.torch.zeros((4, ny, nx), dtype=self.torch.float64, device=self.sigma.device)

    def _st(self, t) -> m1_state:
        assert t.dtype == self.torch.float64 and t.is_cuda and t.is_contiguous() and t.shape[0] == 4
        return m1_state(t[0].data_ptr(), t[1].data_ptr(), t[2].data_ptr() if self.dim == 2 else None,
                        t[3].data_ptr())

    # ---- the C ABI
    def step(self, v, nsteps: int = 1) -> dict:
        info = m1_info()
        st = lib().m1_step(self.handle, ctypes.byref(self._st(v)), nsteps, ctypes.byref(info))
        out = {"status": st, "cycles": info.cycles, "levels": info.levels, "steps_done": info.steps_done,
               "r0": info.r0, "rel_residual": info.rel_residual, "dtau": info.dtau,
               "first_bad_cell": info.first_bad_cell, "stalled_cells": info.stalled_cells}
        if st not in (0, 3):
            raise M1Error(st, f"m1_step {out}")
        return out

    def vcycle(self, v, vn, dtau: float, want_info: bool = False):
        info = m1_info() if want_info else None
        _check(lib().m1_vcycle(self.handle, ctypes.byref(self._st(v)), ctypes.byref(self._st(vn)), dtau,
                               ctypes.byref(info) if want_info else None), "m1_vcycle")
        return _info_dict(info) if want_info else None

    def stalls(self, reset: bool = False) -> int:
        """Pseudo-time stalls counted on this plan since its creation, its last step or the last reset."""
        n = ctypes.c_int64()
        _check(lib().m1_stalls(self.handle, ctypes.byref(n), 1 if reset else 0), "m1_stalls")
        return n.value

    def residual(self, v, vn, want_r: bool = False):
        r = self.torch.zeros_like(v) if want_r else None
        norm = ctypes.c_double()
        _check(lib().m1_residual(self.handle, ctypes.byref(self._st(v)), ctypes.byref(self._st(vn)),
                                 ctypes.byref(norm), ctypes.byref(self._st(r)) if want_r else None), "m1_residual")
        return (norm.value, r) if want_r else norm.value

    def apply_A(self, level: int, v):
        out = self.new_state(level)
        _check(lib().m1_apply_A(self.handle, level, ctypes.byref(self._st(v)), ctypes.byref(self._st(out))),
               "m1_apply_A")
        return out

    def sweep(self, b, v):
        out = self.torch.zeros_like(v)
        _check(lib().m1_sweep(self.handle, ctypes.byref(self._st(b)), ctypes.byref(self._st(v)),
                              ctypes.byref(self._st(out))), "m1_sweep")
        return out

    def sweeps(self, b, v, n: int):
        out = self.torch.zeros_like(v)
        _check(lib().m1_sweeps(self.handle, ctypes.byref(self._st(b)), ctypes.byref(self._st(v)),
                               ctypes.byref(self._st(out)), n), "m1_sweeps")
        return out

    def pseudo_step(self, level: int, dtau: float, f, u):
        out = self.new_state(level)
        _check(lib().m1_pseudo_step(self.handle, level, dtau, ctypes.byref(self._st(f)), ctypes.byref(self._st(u)),
                                    ctypes.byref(self._st(out))), "m1_pseudo_step")
        return out

    def restrict(self, level: int, x):
        out = self.new_state(level + 1)
        _check(lib().m1_restrict(self.handle, level, ctypes.byref(self._st(x)), ctypes.byref(self._st(out))),
               "m1_restrict")
        return out

    def residual_restrict(self, level: int, u, rhs, vc=None, rc=None):
        """R(u) and R(rhs - A_level(u)) on level + 1 (one launch in 2-D)."""
        vc = self.new_state(level + 1) if vc is None else vc
        rc = self.new_state(level + 1) if rc is None else rc
        _check(lib().m1_residual_restrict(self.handle, level, ctypes.byref(self._st(u)), ctypes.byref(self._st(rhs)),
                                          ctypes.byref(self._st(vc)), ctypes.byref(self._st(rc))),
               "m1_residual_restrict")
        return vc, rc

    def prolong_project(self, level: int, u, uc, vc, out=None):
        out = self.torch.zeros_like(u) if out is None else out
        _check(lib().m1_prolong_project(self.handle, level, ctypes.byref(self._st(u)), ctypes.byref(self._st(uc)),
                                        ctypes.byref(self._st(vc)), ctypes.byref(self._st(out))), "m1_prolong_project")
        return out

    def sync(self):
        _check(lib().m1_sync(self.handle), "m1_sync")


STATIC_SCRATCH_BYTES = 80 << 20  # M1_STATIC_SCRATCH_BYTES


def step_static(problem: dict, sigma, v, nsteps: int = 1, params: dict | None = None, stream=None) -> dict:
    """m1_step_static: nsteps implicit steps of state v (torch float64 (4, ny, nx) on the current
    device) on the library's static device workspace; no plan, no allocation."""
    import torch
    g = make_grid(problem)
    p = make_params(default_params(**(params or {})))
    sigma = sigma.contiguous()
    assert sigma.dtype == torch.float64 and sigma.is_cuda and v.dtype == torch.float64 and v.is_contiguous()
    op = m1_opacity(sigma[0].data_ptr(), sigma[1].data_ptr())
    st = m1_state(v[0].data_ptr(), v[1].data_ptr(), v[2].data_ptr() if problem["dim"] == 2 else None,
                  v[3].data_ptr())
    s = stream if stream is not None else torch.cuda.current_stream()
    info = m1_info()
    rc = lib().m1_step_static(ctypes.byref(g), ctypes.byref(p), ctypes.byref(op), ctypes.byref(st), nsteps,
                              ctypes.c_void_p(s.cuda_stream), ctypes.byref(info))
    out = dict(_info_dict(info), first_bad_cell=info.first_bad_cell)
    if rc not in (0, 3):
        raise M1Error(rc, f"m1_step_static {out}")
    out["status"] = rc
    return out


def _info_dict(info: m1_info) -> dict:
    return {"status": info.status, "cycles": info.cycles, "levels": info.levels, "steps_done": info.steps_done,
            "r0": info.r0, "rel_residual": info.rel_residual, "dtau": info.dtau, "stalled_cells": info.stalled_cells}


class Engine:
    """Batched / continuously batched solves of many 2-D problems (m1_engine).

    The arena (a torch uint8 tensor) is allocated once; each request's plan is
    carved from it when the request is admitted.  Requests keep references to
    their state and opacity tensors until they are released.
    """

    def __init__(self, arena_bytes: int, params: dict | None = None, max_requests: int = 1024, device="cuda",
                 stream=None):
        import torch
        self.torch = torch
        self.params_d = default_params(**(params or {}))
        self.params = make_params(self.params_d)
        self.arena = torch.empty(int(arena_bytes) + 256, dtype=torch.uint8, device=device)
        base = self.arena.data_ptr()
        off = (-base) % 256
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.arena.device)
        h = ctypes.c_void_p()
        _check(lib().m1_engine_create(ctypes.byref(self.params), ctypes.c_void_p(base + off), int(arena_bytes),
                                      max_requests, ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h)),
               "m1_engine_create")
        self.handle = h
        self.keep = {}

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and _lib is not None:
            _lib.m1_engine_destroy(h)
            self.handle = None

    def memory(self) -> dict:
        """HBM of the request pool in use and in total, resident and waiting requests (m1_engine_memory)."""
        used, total = ctypes.c_size_t(), ctypes.c_size_t()
        res, pend = ctypes.c_int32(), ctypes.c_int32()
        _check(lib().m1_engine_memory(self.handle, ctypes.byref(used), ctypes.byref(total), ctypes.byref(res),
                                      ctypes.byref(pend)), "m1_engine_memory")
        return {"pool_in_use": used.value, "pool_bytes": total.value, "resident": res.value, "pending": pend.value}

    @staticmethod
    def request_bytes(problem: dict, params: dict | None = None) -> int:
        return lib().m1_engine_request_bytes(ctypes.byref(make_grid(problem)),
                                             ctypes.byref(make_params(default_params(**(params or {})))))

    def submit(self, problem: dict, sigma, v, nsteps: int, params: dict | None = None) -> int:
        assert v.dtype == self.torch.float64 and v.is_cuda and v.is_contiguous() and tuple(v.shape)[0] == 4
        sigma = sigma.contiguous()
        g = make_grid(problem)
        p = make_params(default_params(**{**self.params_d, **(params or {})})) if params else None
        op = m1_opacity(sigma[0].data_ptr(), sigma[1].data_ptr())
        st = m1_state(v[0].data_ptr(), v[1].data_ptr(), v[2].data_ptr(), v[3].data_ptr())
        t = ctypes.c_uint64()
        _check(lib().m1_batch_submit(self.handle, ctypes.byref(g), ctypes.byref(p) if p else None, ctypes.byref(op),
                                     ctypes.byref(st), nsteps, ctypes.byref(t)), "m1_batch_submit")
        self.keep[t.value] = (sigma, v)
        return t.value

    def run(self, cycles: int = 4):
        nr, npd = ctypes.c_int32(), ctypes.c_int32()
        _check(lib().m1_batch_run(self.handle, cycles, ctypes.byref(nr), ctypes.byref(npd)), "m1_batch_run")
        return nr.value, npd.value

    def poll(self, ticket: int):
        info = m1_info()
        st = lib().m1_batch_poll(self.handle, ticket, ctypes.byref(info))
        if st == 6:
            return None
        _check(st, "m1_batch_poll")
        return _info_dict(info)

    def wait(self, ticket: int) -> dict:
        """Block until the request is done (the request's own status is in the result)."""
        info = m1_info()
        st = lib().m1_batch_wait(self.handle, ticket, ctypes.byref(info))
        if self.poll(ticket) is None:  # not done: the engine or the serving loop failed
            raise M1Error(st, "m1_batch_wait")
        return _info_dict(info)

    def serve_start(self, cycles: int = 4):
        """Start the library's serving thread (rounds of `cycles` V-cycles)."""
        _check(lib().m1_serve_start(self.handle, cycles), "m1_serve_start")

    def serve_stop(self):
        """Stop and join the serving thread; raises the first error it met."""
        _check(lib().m1_serve_stop(self.handle), "m1_serve_stop")

    def cancel(self, ticket: int):
        _check(lib().m1_batch_cancel(self.handle, ticket), "m1_batch_cancel")

    def times(self, ticket: int):
        a, b, c = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
        _check(lib().m1_batch_times(self.handle, ticket, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)),
               "m1_batch_times")
        return a.value, b.value, c.value

    def release(self, ticket: int):
        _check(lib().m1_batch_release(self.handle, ticket), "m1_batch_release")
        self.keep.pop(ticket, None)


def to_device(a: np.ndarray, device="cuda"):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to(device)


# ---------------------------------------------------------------------------- three dimensions
def make_grid3(problem: dict) -> m1_grid3:
    g = m1_grid3()
    for k in ("nx", "ny", "nz", "hx", "hy", "hz", "dt", "c", "a_r", "c_v"):
        setattr(g, k, problem[k])
    for s, bc in enumerate(problem["bc"]):
        g.bc[s].kind = BC[bc["kind"]]
        g.bc[s].E = bc.get("E", 0.0)
        g.bc[s].Fx = bc.get("Fx", 0.0)
        g.bc[s].Fy = bc.get("Fy", 0.0)
        g.bc[s].Fz = bc.get("Fz", 0.0)
    return g


class Plan3:
    """A 3-D solver plan (m1_plan3_*): states are (5, nz, ny, nx) float64 tensors holding E, Fx, Fy, Fz, T."""

    def __init__(self, problem: dict, sigma, params: dict | None = None, stream=None):
        import torch
        self.torch = torch
        self.problem = problem
        self.grid = make_grid3(problem)
        self.params = make_params(default_params(**(params or {})))
        L = lib()
        self.sigma = sigma.contiguous()
        assert self.sigma.dtype == torch.float64 and self.sigma.is_cuda
        assert tuple(self.sigma.shape) == (2, problem["nz"], problem["ny"], problem["nx"])
        nbytes = L.m1_workspace3_bytes(ctypes.byref(self.grid), ctypes.byref(self.params))
        if nbytes == 0:
            raise M1Error(1, "m1_workspace3_bytes")
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.sigma.device)
        base = self.workspace.data_ptr()
        self.ws_ptr, self.ws_bytes = base + (-base) % 256, nbytes
        op = m1_opacity(self.sigma[0].data_ptr(), self.sigma[1].data_ptr())
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.sigma.device)
        h = ctypes.c_void_p()
        _check(L.m1_plan3_create(ctypes.byref(self.grid), ctypes.byref(self.params), ctypes.byref(op),
                                 ctypes.c_void_p(self.ws_ptr), self.ws_bytes, ctypes.c_void_p(self.stream.cuda_stream),
                                 ctypes.byref(h)), "m1_plan3_create")
        self.handle = h
        self.levels = L.m1_plan3_levels(h)

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and _lib is not None:
            _lib.m1_plan3_destroy(h)
            self.handle = None

    def level_dims(self, level: int):
        d = [ctypes.c_int32() for _ in range(3)]
        _check(lib().m1_level3_dims(self.handle, level, *[ctypes.byref(x) for x in d]), "m1_level3_dims")
        return tuple(x.value for x in d)

    def new_state(self, level: int = 0):
        nx, ny, nz = self.level_dims(level)
        return self.torch.zeros((5, nz, ny, nx), dtype=self.torch.float64, device=self.sigma.device)

    def _st(self, t) -> m1_state3:
        assert t.dtype == self.torch.float64 and t.is_cuda and t.is_contiguous() and t.shape[0] == 5
        return m1_state3(*[t[q].data_ptr() for q in range(5)])

    def step(self, v, nsteps: int = 1) -> dict:
        info = m1_info()
        st = lib().m1_step3(self.handle, ctypes.byref(self._st(v)), nsteps, ctypes.byref(info))
        out = _info_dict(info)
        out["status"] = st
        out["first_bad_cell"] = info.first_bad_cell
        if st not in (0, 3):
            raise M1Error(st, f"m1_step3 {out}")
        return out

    def vcycle(self, v, vn, dtau: float):
        _check(lib().m1_vcycle3(self.handle, ctypes.byref(self._st(v)), ctypes.byref(self._st(vn)), dtau),
               "m1_vcycle3")

    def residual(self, v, vn, want_r: bool = False):
        r = self.torch.zeros_like(v) if want_r else None
        norm = ctypes.c_double()
        _check(lib().m1_residual3(self.handle, ctypes.byref(self._st(v)), ctypes.byref(self._st(vn)),
                                  ctypes.byref(norm), ctypes.byref(self._st(r)) if want_r else None), "m1_residual3")
        return (norm.value, r) if want_r else norm.value

    def apply_A(self, level: int, v):
        out = self.new_state(level)
        _check(lib().m1_apply3(self.handle, level, ctypes.byref(self._st(v)), ctypes.byref(self._st(out))),
               "m1_apply3")
        return out

    def sweep(self, b, v):
        out = self.torch.zeros_like(v)
        _check(lib().m1_sweep3(self.handle, ctypes.byref(self._st(b)), ctypes.byref(self._st(v)),
                               ctypes.byref(self._st(out))), "m1_sweep3")
        return out

    def pseudo_step(self, level: int, dtau: float, f, u):
        out = self.new_state(level)
        _check(lib().m1_pseudo_step3(self.handle, level, dtau, ctypes.byref(self._st(f)), ctypes.byref(self._st(u)),
                                     ctypes.byref(self._st(out))), "m1_pseudo_step3")
        return out

    def restrict(self, level: int, x):
        out = self.new_state(level + 1)
        _check(lib().m1_restrict3(self.handle, level, ctypes.byref(self._st(x)), ctypes.byref(self._st(out))),
               "m1_restrict3")
        return out

    def prolong_project(self, level: int, u, uc, vc, out=None):
        out = self.torch.zeros_like(u) if out is None else out
        _check(lib().m1_prolong_project3(self.handle, level, ctypes.byref(self._st(u)), ctypes.byref(self._st(uc)),
                                         ctypes.byref(self._st(vc)), ctypes.byref(self._st(out))),
               "m1_prolong_project3")
        return out
