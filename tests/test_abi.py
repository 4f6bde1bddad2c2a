"""C-ABI checks that need no GPU: the library loads, exports every declared
symbol, and host-side argument validation works (nothing is enqueued)."""
import ctypes
import os
import re

import pytest

from paper_2208_14703_amd import binding, inputs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            src = open(os.path.join(ROOT, "include", fn)).read()
            src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
            names |= set(re.findall(r"\b(m1_[a-z_0-9]+)\s*\(", src))
    return sorted(names)


def test_library_exports_every_declared_symbol():
    if not os.path.exists(binding.LIB_PATH):
        pytest.skip("libm1mg.so not built")
    L = binding.lib()
    names = declared_functions()
    assert len(names) >= 15
    for n in names:
        assert hasattr(L, n), n


def test_default_params_are_the_papers():
    p = binding.default_params()
    assert (p["nu0"], p["pseudo_steps"], p["nu_l"], p["dtau_im0"]) == (3, 3, 1, 1e-3)
    assert p["omega"] == 1.0 and p["levels"] == 0


def test_workspace_size_and_host_validation():
    L = binding.lib()
    prob, _, _, _ = inputs.hot_wall_2d(n=1024)
    g = binding.make_grid(prob)
    p = binding.make_params(binding.default_params())
    nbytes = L.m1_workspace_bytes(ctypes.byref(g), ctypes.byref(p))
    # finest: b, tmp, rbar (12 fields); coarse levels: 22 fields on a third of the cells
    assert 12 * 8 * 1024 ** 2 < nbytes < 24 * 8 * 1024 ** 2
    bad = binding.make_grid(prob)
    bad.dt = -1.0
    assert L.m1_workspace_bytes(ctypes.byref(bad), ctypes.byref(p)) == 0
    bad = binding.make_grid(prob)
    bad.bc[0].kind = 0   # periodic on one side only
    assert L.m1_workspace_bytes(ctypes.byref(bad), ctypes.byref(p)) == 0
    p2 = binding.make_params(binding.default_params(omega=1.5))
    assert L.m1_workspace_bytes(ctypes.byref(g), ctypes.byref(p2)) == 0
    p3 = binding.make_params(binding.default_params(levels=12))   # 1024 has only 9 levels down to side 4
    assert L.m1_workspace_bytes(ctypes.byref(g), ctypes.byref(p3)) == 0
    p4 = binding.make_params(binding.default_params(precision="mixed", nu_l=2))  # mixed fuses one sweep per step
    assert L.m1_workspace_bytes(ctypes.byref(g), ctypes.byref(p4)) == 0
    p5 = binding.make_params(binding.default_params(precision="mixed"))
    assert L.m1_workspace_bytes(ctypes.byref(g), ctypes.byref(p5)) > 0
    # plan creation rejects a too-small or misaligned workspace before touching it
    op = binding.m1_opacity(0x10000, 0x20000)
    h = ctypes.c_void_p()
    st = L.m1_plan_create(ctypes.byref(g), ctypes.byref(p), ctypes.byref(op), ctypes.c_void_p(0x100000), 1024,
                          None, ctypes.byref(h))
    assert st == 4 and not h.value
    st = L.m1_plan_create(ctypes.byref(g), ctypes.byref(p), ctypes.byref(op), ctypes.c_void_p(0x100008), nbytes,
                          None, ctypes.byref(h))
    assert st == 4
    st = L.m1_plan_create(ctypes.byref(bad), ctypes.byref(p), ctypes.byref(op), ctypes.c_void_p(0x100000), nbytes,
                          None, ctypes.byref(h))
    assert st == 1
    assert L.m1_strerror(2).decode().startswith("state not admissible")
    # operations on a null plan are argument errors, checked before anything is enqueued
    assert L.m1_sweep(None, None, None, None) == 1
    assert L.m1_sweeps(None, None, None, None, 2) == 1


def test_one_dimensional_grid_validation():
    L = binding.lib()
    prob, _, _, _ = inputs.gaussian_1d()
    g = binding.make_grid(prob)
    p = binding.make_params(binding.default_params())
    assert L.m1_workspace_bytes(ctypes.byref(g), ctypes.byref(p)) > 0
    g.ny = 2
    assert L.m1_workspace_bytes(ctypes.byref(g), ctypes.byref(p)) == 0


def test_tuning_settings_round_trip():
    """Launch-shape settings: known keys round-trip, unknown keys and bad values are rejected (host only)."""
    from paper_2208_14703_amd import binding
    L = binding.lib()
    for key in ("tail_cells", "tiled_max_cells", "batch_grid"):
        old = binding.tune_get(key)
        assert old > 0
        binding.tune_set(key, old + 1)
        assert binding.tune_get(key) == old + 1
        binding.tune_set(key, old)
        assert binding.tune_get(key) == old
    g = binding.tune_get("graphs")
    assert g in (0, 1)
    binding.tune_set("graphs", 1 - g)
    assert binding.tune_get("graphs") == 1 - g
    binding.tune_set("graphs", g)
    assert L.m1_tune_set(b"graphs", 2) == 1
    r = binding.tune_get("sweep_rows")
    for rows in (0, 4, 8, 16):
        binding.tune_set("sweep_rows", rows)
        assert binding.tune_get("sweep_rows") == rows
    binding.tune_set("sweep_rows", r)
    assert L.m1_tune_set(b"sweep_rows", 5) == 1 and binding.tune_get("sweep_rows") == r
    assert L.m1_tune_set(b"no_such_key", 5) == 1
    assert L.m1_tune_get(b"no_such_key") == -1
    assert L.m1_tune_set(b"tail_cells", -1) == 1
    assert L.m1_tune_set(b"batch_grid", 0) == 1


def test_autotuner_builtin_values_match_the_library():
    """The autotuner starts from the library's built-in launch shapes (no GPU:
    nothing stored is applied, and no M1_* variable is set in the test run)."""
    import os
    from paper_2208_14703_amd import autotune, binding
    binding.lib()
    for key, val in autotune.BUILTIN.items():
        if os.environ.get(binding.TUNE_ENV[key]) is None:
            assert binding.tune_get(key) == val, key
    assert set(autotune.BUILTIN) == set(binding.TUNE_ENV) == set(autotune.CANDIDATES)


def test_workspace3_size_and_host_validation():
    """The 3-D plans' host checks: workspace bytes of the level hierarchy, and 0 for the grids and parameter
    choices they reject (nothing is enqueued)."""
    L = binding.lib()
    prob, _, _, _ = inputs.hot_wall_3d(n=64)
    g = binding.make_grid3(prob)
    p = binding.make_params(binding.default_params())
    nbytes = L.m1_workspace3_bytes(ctypes.byref(g), ctypes.byref(p))
    # finest: b, tmp, residual (15 fields); coarse levels (1/7 of the cells): 27 fields
    assert 15 * 8 * 64 ** 3 < nbytes < 20 * 8 * 64 ** 3
    pl = binding.make_params(binding.default_params(levels=4))  # 64 -> 32 -> 16 -> 8
    assert 0 < L.m1_workspace3_bytes(ctypes.byref(g), ctypes.byref(pl)) < nbytes
    pl = binding.make_params(binding.default_params(levels=5))  # side 4 is the coarsest level: 64 .. 4 is 5 levels
    assert L.m1_workspace3_bytes(ctypes.byref(g), ctypes.byref(pl)) == nbytes
    pl = binding.make_params(binding.default_params(levels=6))
    assert L.m1_workspace3_bytes(ctypes.byref(g), ctypes.byref(pl)) == 0
    for extra in (dict(precision="mixed"), dict(cycle=3), dict(transfer="mean"), dict(nu_l=2),
                  dict(smoother="rbgs"), dict(omega=1.5)):
        q = binding.make_params(binding.default_params(**extra))
        assert L.m1_workspace3_bytes(ctypes.byref(g), ctypes.byref(q)) == 0, extra
    for kind in ("W", "F"):  # the cycle shapes use the V-cycle's buffers
        q = binding.make_params(binding.default_params(cycle=kind))
        assert L.m1_workspace3_bytes(ctypes.byref(g), ctypes.byref(q)) == nbytes
    bad = binding.make_grid3(prob)
    bad.bc[4].kind = 0  # periodic on one z side only
    assert L.m1_workspace3_bytes(ctypes.byref(bad), ctypes.byref(p)) == 0
    bad = binding.make_grid3(prob)
    bad.bc[2].kind = 4  # inflow sides are 2-D only
    assert L.m1_workspace3_bytes(ctypes.byref(bad), ctypes.byref(p)) == 0
    bad = binding.make_grid3(prob)
    bad.bc[0].Fx = 2.0 * bad.c * bad.bc[0].E  # a non-admissible wall state
    assert L.m1_workspace3_bytes(ctypes.byref(bad), ctypes.byref(p)) == 0
    bad = binding.make_grid3(prob)
    bad.hz = 0.0
    assert L.m1_workspace3_bytes(ctypes.byref(bad), ctypes.byref(p)) == 0
