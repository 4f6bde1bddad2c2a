"""Batched solves (m1_engine): many problems of uneven sizes advance together,
one launch per level operation.  Each request must give exactly the result of
solving it alone (same kernels, same per-request norms and controls), also
when the arena is so small that requests queue and are admitted as others
finish (continuous batching).

Every batched and served run also carries an anchor request solved to a tight
tolerance (its own rtol; the engine lets tolerances differ per request), whose
result is compared with the oracle's converged solution: relative 1e-10 in
FP64, and the stated mixed-precision bound (5e-10 at rtol 1e-12).
"""
import time

import numpy as np
import pytest

import oracle
from paper_2208_14703_amd import binding, inputs
from tests.gpu_util import announce, rel_err, to_dev, to_host

pytestmark = pytest.mark.gpu

PARAMS = dict(omega=0.8, rtol=1e-8)
ANCHOR_RTOL = {"fp64": 1e-13, "mixed": 1e-12}
ANCHOR_BOUND = {"fp64": 1e-10, "mixed": 5e-10}
_anchor_ref = {}


def anchor(precision, params=None):
    """A 96 x 64 hot-wall problem of two steps with a tight per-request rtol."""
    prob, v, sig = inputs.random_problem(77, 2, 96, 64, bc_kinds=("dirichlet", "reflective", "periodic", "periodic"),
                                         cfl=100.0, log10_sa=(-3, 3), fmax=0.95, block=8)
    p = dict(params or PARAMS, precision=precision, rtol=ANCHOR_RTOL[precision], max_cycles=20000)
    return prob, v, sig, 2, p


def check_anchor(prob, v, sig, ns, precision, got, info):
    """The anchor request's result against the oracle's converged solution."""
    assert info["status"] == 0 and info["steps_done"] == ns, info
    if ns not in _anchor_ref:
        o = oracle.Oracle(prob, sig)
        _anchor_ref[ns], _ = o.step(v, ns, oracle.make_params(omega=PARAMS["omega"], rtol=1e-13, max_cycles=50000))
    err = rel_err(got, _anchor_ref[ns], prob["c"])
    print(f"anchor {precision}: cycles {info['cycles']} rel {info['rel_residual']:.3e} error vs oracle {err:.3e}",
          flush=True)
    assert err <= ANCHOR_BOUND[precision], (precision, err)


def problems(n, sides=(64, 128, 256)):
    out = []
    rng = np.random.default_rng(5)
    for k in range(n):
        side = int(sides[k % len(sides)])
        prob, v, sig = inputs.random_problem(300 + k, 2, side, side, cfl=100.0, log10_sa=(-3, 3), fmax=0.95,
                                             block=32 if side >= 64 else 8)
        if k % 3 == 2:   # a hot wall on some of them
            prob["bc"] = [dict(kind="dirichlet", E=30.0, Fx=0.0, Fy=0.0)] + [dict(kind="reflective")] * 3
        out.append((prob, v, sig, 1 + int(rng.integers(0, 3))))
    return out


def alone(prob, v, sig, nsteps, params=PARAMS):
    P = binding.Plan(prob, to_dev(sig), params)
    vd = to_dev(v)
    info = P.step(vd, nsteps)
    return to_host(vd), info


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("arena", ["large", "tight"])
def test_batch_matches_alone(precision, arena):
    announce("batch vs alone", precision, arena)
    params = dict(PARAMS, precision=precision)
    cases = problems(9)
    need = max(binding.Engine.request_bytes(p, params) for p, _, _, _ in cases)
    # tight: room for two of the largest requests at once, so the others queue
    arena_bytes = (4096 << 20) if arena == "large" else int(2.5 * need) + (2 << 20)
    E = binding.Engine(arena_bytes, params, max_requests=64)
    states, tickets = [], []
    for prob, v, sig, ns in cases:
        vd = to_dev(v)
        states.append(vd)
        tickets.append(E.submit(prob, to_dev(sig), vd, ns))
    ap, av, asg, ans, apar = anchor(precision)
    avd = to_dev(av)
    at = E.submit(ap, to_dev(asg), avd, ans, apar)
    tickets.append(at)
    done = set()
    rounds = 0
    while len(done) < len(tickets):
        E.run(3)
        rounds += 1
        for t in tickets:
            if t not in done and E.poll(t) is not None:
                done.add(t)
        assert rounds < 5000
    ainfo = E.poll(at)
    check_anchor(ap, av, asg, ans, precision, to_host(avd), ainfo)
    np.testing.assert_array_equal(to_host(avd), alone(ap, av, asg, ans, apar)[0])
    for (prob, v, sig, ns), vd, t in zip(cases, states, tickets):
        info = E.poll(t)
        ref, info_a = alone(prob, v, sig, ns, params)
        assert info["status"] == 0 and info["steps_done"] == ns
        assert info["cycles"] == info_a["cycles"], (info["cycles"], info_a["cycles"])
        np.testing.assert_array_equal(to_host(vd), ref)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("nu0,m", [(1, 3), (2, 3), (4, 3), (3, 1), (3, 5)])
def test_batch_sweep_counts_match_alone(precision, nu0, m):
    """Odd and even finest-level sweep counts (the default is 3) and other odd
    pseudo-time step counts (the engine requires odd ones): the engine's cycles
    move the iterate (FP64), the pending correction (mixed) and the coarse
    iterates between their buffers once per sweep or step, and every request
    still equals its solo solve, bitwise, with the same cycle counts."""
    announce("batch sweep counts", precision, nu0, m)
    params = dict(PARAMS, precision=precision, nu0=nu0, pseudo_steps=m)
    cases = problems(4)
    ap, av, asg, ans, apar = anchor(precision, params)
    need = sum(binding.Engine.request_bytes(p, params) for p, _, _, _ in cases + [(ap, 0, 0, 0)])
    E = binding.Engine(need + (16 << 20), params, max_requests=8)
    states, tickets = [], []
    for prob, v, sig, ns in cases:
        vd = to_dev(v)
        states.append(vd)
        tickets.append(E.submit(prob, to_dev(sig), vd, ns))
    avd = to_dev(av)
    at = E.submit(ap, to_dev(asg), avd, ans, apar)
    infos = [E.wait(t) for t in tickets]
    ainfo = E.wait(at)  # the anchor takes more cycles than the others: wait before reading its state
    check_anchor(ap, av, asg, ans, precision, to_host(avd), ainfo)
    np.testing.assert_array_equal(to_host(avd), alone(ap, av, asg, ans, apar)[0])
    for (prob, v, sig, ns), vd, info in zip(cases, states, infos):
        ref, info_a = alone(prob, v, sig, ns, params)
        assert info["status"] == 0 and info_a["status"] == 0
        assert info["cycles"] == info_a["cycles"], (info["cycles"], info_a["cycles"])
        np.testing.assert_array_equal(to_host(vd), ref)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_batch_ragged_shapes_match_alone(precision):
    """Sides that are not multiples of the tile shapes (64 x rows for the
    staged sweeps, 32 x 4 coarse cells for the fused residual-restriction),
    odd coarse levels and every kind of side, batched together: each request
    equals its solo solve to the bit."""
    announce("batch ragged shapes", precision)
    params = dict(PARAMS, precision=precision)
    shapes = [(100, 36), (66, 10), (130, 70), (96, 80), (200, 28), (36, 132)]
    kinds = [("periodic",) * 4, ("dirichlet", "reflective", "neumann", "reflective"),
             ("dirichlet", "neumann", "periodic", "periodic"), ("reflective",) * 4]
    cases = []
    for k, (nx, ny) in enumerate(shapes):
        prob, v, sig = inputs.random_problem(700 + k, 2, nx, ny, bc_kinds=kinds[k % len(kinds)], cfl=80.0,
                                             log10_sa=(-3, 3), fmax=0.9, block=4)
        cases.append((prob, v, sig, 1 + k % 2))
    need = sum(binding.Engine.request_bytes(p, params) for p, _, _, _ in cases)
    E = binding.Engine(need + (16 << 20), params, max_requests=16)
    states, tickets = [], []
    for prob, v, sig, ns in cases:
        vd = to_dev(v)
        states.append(vd)
        tickets.append(E.submit(prob, to_dev(sig), vd, ns))
    infos = [E.wait(t) for t in tickets]
    for (prob, v, sig, ns), vd, info in zip(cases, states, infos):
        ref, info_a = alone(prob, v, sig, ns, params)
        assert info["status"] == 0 and info_a["status"] == 0
        assert info["cycles"] == info_a["cycles"]
        np.testing.assert_array_equal(to_host(vd), ref)


def test_batch_budget_cancel_and_arguments():
    announce("batch: budget / cancel / args")
    E = binding.Engine(32 << 20, PARAMS, max_requests=8)
    prob, v, sig = inputs.random_problem(1, 2, 512, 512, cfl=100.0)
    with pytest.raises(binding.M1Error) as ei:
        E.submit(prob, to_dev(sig), to_dev(v), 1)
    assert ei.value.status == 7   # can never fit
    p1 = inputs.gaussian_1d(n=64)
    with pytest.raises(binding.M1Error) as ei:
        E.submit(p1[0], to_dev(p1[2]), to_dev(p1[1]), 1)
    assert ei.value.status == 1   # batches are 2-D
    prob, v, sig = inputs.random_problem(2, 2, 64, 64, cfl=100.0)
    vd = to_dev(v)
    t = E.submit(prob, to_dev(sig), vd, 20)
    E.run(1)
    E.cancel(t)
    E.run(1)
    info = E.poll(t)
    assert info is not None and info["status"] == 6
    got = to_host(vd)
    assert np.all(got[0] > 0) and np.all(got[3] > 0)
    # a request with an invalid opacity leaves with M1_ERR_ARG before any cycle touches its state,
    # while a valid one admitted in the same round runs normally
    bad_sig = sig.copy()
    bad_sig[0, 3, 5] = -1.0
    vb = to_dev(v)
    vg = to_dev(v)
    tb = E.submit(prob, to_dev(bad_sig), vb, 2)
    tg = E.submit(prob, to_dev(sig), vg, 1)
    assert E.wait(tb)["status"] == 1
    assert E.wait(tg)["status"] == 0
    np.testing.assert_array_equal(to_host(vb), v)
    assert not np.array_equal(to_host(vg), v)
    # mixed precision: a cancelled request's FP64 state may sit in the partner
    # buffer; it must come back to the caller's arrays, finite and admissible
    params = dict(PARAMS, precision="mixed")
    E2 = binding.Engine(64 << 20, params, max_requests=8)
    v0 = v.copy()
    vd = to_dev(v0)
    t = E2.submit(prob, to_dev(sig), vd, 20)
    E2.run(3)
    E2.run(2)
    E2.cancel(t)
    E2.run(1)
    info = E2.poll(t)
    assert info is not None and info["status"] == 6 and info["cycles"] > 0
    got = to_host(vd)
    assert np.all(np.isfinite(got)) and np.all(got[0] > 0) and np.all(got[3] > 0)
    assert np.all(np.hypot(got[1], got[2]) <= prob["c"] * got[0] * (1 + 1e-12))
    assert not np.array_equal(got, v0)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_serving_loop_matches_alone(precision):
    """Requests submitted while others are on the GPU (the library's serving
    thread drives the rounds) are admitted as memory frees up, overlap on the
    device, and each result equals solving it alone, bitwise."""
    announce("serving loop vs alone", precision)
    params = dict(PARAMS, precision=precision)
    cases = problems(7)
    need = max(binding.Engine.request_bytes(p, params) for p, _, _, _ in cases)
    E = binding.Engine(int(2.5 * need) + (2 << 20), params, max_requests=64)
    E.serve_start(2)
    states, tickets = [], []
    ap, av, asg, ans, apar = anchor(precision)
    avd = to_dev(av)
    for k, (prob, v, sig, ns) in enumerate(cases):
        vd = to_dev(v)
        sd = to_dev(sig)
        states.append(vd)
        tickets.append(E.submit(prob, sd, vd, ns))
        if k == 2:
            at = E.submit(ap, to_dev(asg), avd, ans, apar)
        time.sleep(0.01)
    infos = [E.wait(t) for t in tickets]
    ainfo = E.wait(at)
    check_anchor(ap, av, asg, ans, precision, to_host(avd), ainfo)
    E.serve_stop()
    tm = [E.times(t) for t in tickets]
    # some request was admitted while an earlier one was still running
    assert any(tm[k][1] < max(tm[j][2] for j in range(k)) for k in range(1, len(tm)))
    for (prob, v, sig, ns), vd, info in zip(cases, states, infos):
        ref, info_a = alone(prob, v, sig, ns, params)
        assert info["status"] == 0 and info["steps_done"] == ns
        assert info["cycles"] == info_a["cycles"]
        np.testing.assert_array_equal(to_host(vd), ref)
    # the loop sleeps when empty and serves again after a restart
    E.serve_start(3)
    prob, v, sig, ns = cases[0]
    vd = to_dev(v)
    t = E.submit(prob, to_dev(sig), vd, ns)
    assert E.wait(t)["status"] == 0
    E.serve_stop()
    np.testing.assert_array_equal(to_host(vd), alone(prob, v, sig, ns, params)[0])


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_serving_concurrent_clients(precision):
    """Four client threads submit and wait at the same time while the
    library's serving thread runs rounds (submit, poll and wait enter the
    library from several threads at once; ctypes releases the GIL).  Every
    request finishes and equals its solo solve, bitwise."""
    import threading
    announce("serving, concurrent clients", precision)
    params = dict(PARAMS, precision=precision)
    cases = problems(12)
    need = max(binding.Engine.request_bytes(p, params) for p, _, _, _ in cases)
    E = binding.Engine(int(3.5 * need) + (2 << 20), params, max_requests=64)
    devs = [(to_dev(sig), to_dev(v)) for _, v, sig, _ in cases]
    results, errors = [None] * len(cases), []

    def client(idx):
        try:
            for k in idx:
                prob, _, _, ns = cases[k]
                t = E.submit(prob, devs[k][0], devs[k][1], ns)
                time.sleep(0.002)
                results[k] = E.wait(t)
        except Exception as exc:  # reported by the main thread
            errors.append(exc)

    ap, av, asg, ans, apar = anchor(precision)
    avd = to_dev(av)
    E.serve_start(2)
    threads = [threading.Thread(target=client, args=(list(range(c, len(cases), 4)),), daemon=True) for c in range(4)]
    for th in threads:
        th.start()
    at = E.submit(ap, to_dev(asg), avd, ans, apar)
    ainfo = E.wait(at)
    for th in threads:
        th.join(timeout=120)
    alive = [th.is_alive() for th in threads]
    E.serve_stop()
    assert not errors, errors
    assert not any(alive)
    check_anchor(ap, av, asg, ans, precision, to_host(avd), ainfo)
    for k, (prob, v, sig, ns) in enumerate(cases):
        ref, info_a = alone(prob, v, sig, ns, params)
        assert results[k]["status"] == 0 and results[k]["steps_done"] == ns
        assert results[k]["cycles"] == info_a["cycles"]
        np.testing.assert_array_equal(to_host(devs[k][1]), ref)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_launch_shape_settings_do_not_change_results(precision):
    """The autotuner's settings (m1_tune_set) only move work between launches:
    a plain solve with the tail and tiled bounds moved across its levels, and a
    batched run whose grid cap makes every block loop over many tiles, give
    the default settings' results to the bit."""
    announce("launch shapes", precision)
    params = dict(PARAMS, precision=precision)
    keys = ("sweep_rows", "pair_rows", "mx_sweep_rows", "residual_restrict", "tail_cells", "tiled_max_cells",
            "batch_grid")
    saved = {key: binding.tune_get(key) for key in keys}
    # wide enough for tiles inside the grid (their fused correction sweep stages the coarse corrections once)
    prob, v, sig = inputs.random_problem(41, 2, 260, 136, cfl=100.0, block=8)
    cases = problems(4)
    need = sum(binding.Engine.request_bytes(p, params) for p, _, _, _ in cases)
    settings = [dict(saved),
                dict(sweep_rows=0, pair_rows=0, mx_sweep_rows=0, residual_restrict=0, tail_cells=64,
                     tiled_max_cells=0, batch_grid=7),
                dict(sweep_rows=16, pair_rows=16, mx_sweep_rows=8, residual_restrict=1, tail_cells=1024,
                     tiled_max_cells=262144, batch_grid=64),
                dict(saved, sweep_rows=4, pair_rows=4, mx_sweep_rows=16, residual_restrict=0)]
    outs = []
    try:
        for st in settings:
            for key in keys:
                binding.tune_set(key, st[key])
            one, info = alone(prob, v, sig, 2, params)
            assert info["status"] == 0
            E = binding.Engine(need + (16 << 20), params, max_requests=8)
            states, tickets = [], []
            for p, bv, bs, ns in cases:
                vd = to_dev(bv)
                states.append(vd)
                tickets.append(E.submit(p, to_dev(bs), vd, ns))
            infos = [E.wait(t) for t in tickets]
            assert all(i["status"] == 0 for i in infos)
            outs.append((one, info["cycles"], [to_host(x) for x in states], [i["cycles"] for i in infos]))
    finally:
        for key in keys:
            binding.tune_set(key, saved[key])
    for one, cyc, batch, bcyc in outs[1:]:
        np.testing.assert_array_equal(one, outs[0][0])
        assert cyc == outs[0][1] and bcyc == outs[0][3]
        for a, b in zip(batch, outs[0][2]):
            np.testing.assert_array_equal(a, b)
