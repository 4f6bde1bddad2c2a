"""V-cycles replayed from hipGraph recordings (launch-shape setting "graphs")
give the results of the same cycles enqueued launch by launch, to the bit.

Each recording is replayed many times, with the library's own eager work
(right-hand side, norms, host synchronisation) between replays, and every
step's result is compared; a second state buffer makes the plan record new
cycles while the first buffer's recordings stay cached.  Engine rounds record
their V-cycle once the resident set has been the same for a round; requests
submitted between rounds force a rebuild and a new recording.
"""
import contextlib

import numpy as np
import pytest

from paper_2208_14703_amd import binding, inputs
from tests.gpu_util import announce, to_dev, to_host

pytestmark = pytest.mark.gpu

PARAMS = dict(omega=0.8, rtol=1e-8)


@contextlib.contextmanager
def graphs(on: int):
    old = binding.tune_get("graphs")
    binding.tune_set("graphs", on)
    try:
        yield
    finally:
        binding.tune_set("graphs", old)


def case(name):
    if name == "hot128":
        prob, v, sig, _ = inputs.hot_wall_2d(n=128)
        return prob, v, sig, {}
    if name == "gauss1d":
        prob, v, sig, _ = inputs.gaussian_1d(n=256)
        return prob, v, sig, {}
    if name == "one_level_odd":  # one level and an odd sweep count: the iterate changes buffer every cycle
        prob, v, sig = inputs.random_problem(7, 2, 48, 40, cfl=20.0, block=8)
        return prob, v, sig, dict(levels=1, nu0=3, max_cycles=20000)
    prob, v, sig = inputs.random_problem(17, 2, 96, 80, cfl=100.0, block=8,
                                         bc_kinds=("dirichlet", "neumann", "periodic", "periodic"))
    return prob, v, sig, {}


def run_sequence(prob, v, sig, params):
    """Three calls on one buffer, then two steps on a second buffer, then the first again."""
    P = binding.Plan(prob, to_dev(sig), params)
    a, b = to_dev(v), to_dev(v)
    out = []
    for vd, ns in ((a, 1), (a, 1), (a, 1), (b, 2), (a, 1)):
        info = P.step(vd, ns)
        b.mul_(1.0)  # other work on the stream between replays
        out.append((to_host(vd), info["cycles"], info["status"]))
    return out


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("name", ["hot128", "gauss1d", "one_level_odd", "bcs96x80"])
def test_plan_replays_match_enqueued_cycles(name, precision):
    announce("graphs: plan", name, precision)
    prob, v, sig, extra = case(name)
    params = dict(PARAMS, precision=precision, **extra)
    with graphs(0):
        ref = run_sequence(prob, v, sig, params)
    with graphs(1):
        got = run_sequence(prob, v, sig, params)
    for (x, cx, sx), (y, cy, sy) in zip(got, ref):
        assert sx == sy == 0
        assert cx == cy
        np.testing.assert_array_equal(x, y)


def batch_cases(n, seed0):
    out = []
    for k in range(n):
        side = (64, 128, 96)[k % 3]
        prob, v, sig = inputs.random_problem(seed0 + k, 2, side, side, cfl=100.0, log10_sa=(-3, 3), fmax=0.95,
                                             block=32 if side % 32 == 0 else 8)
        out.append((prob, v, sig, 1 + k % 3))
    return out


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_engine_replays_match_alone(precision):
    announce("graphs: engine", precision)
    params = dict(PARAMS, precision=precision)
    first, later = batch_cases(3, 500), batch_cases(3, 600)
    need = sum(binding.Engine.request_bytes(p, params) for p, _, _, _ in first + later)
    with graphs(1):
        E = binding.Engine(need + (16 << 20), params, max_requests=16)
        states, tickets = [], []

        def submit(cases):
            for prob, v, sig, ns in cases:
                vd = to_dev(v)
                states.append(vd)
                tickets.append(E.submit(prob, to_dev(sig), vd, ns))

        submit(first)
        for _ in range(4):  # rounds 2.. replay the recording of this resident set
            E.run(2)
        submit(later)  # rebuild, then a new recording
        rounds = 0
        while any(E.poll(t) is None for t in tickets):
            E.run(2)
            rounds += 1
            assert rounds < 5000
        infos = [E.poll(t) for t in tickets]
    with graphs(0):
        for (prob, v, sig, ns), vd, info in zip(first + later, states, infos):
            P = binding.Plan(prob, to_dev(sig), params)
            ref = to_dev(v)
            info_a = P.step(ref, ns)
            assert info["status"] == 0 and info["steps_done"] == ns
            assert info["cycles"] == info_a["cycles"]
            np.testing.assert_array_equal(to_host(vd), to_host(ref))
