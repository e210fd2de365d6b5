"""The persistent step kernel (tuning field `persist`): several steps of every
member in one launch, work items of step t starting as soon as their own
lattice has finished step t - 1.  It must give the same bits as one launch
per step of the same shape, inside and outside HIP graphs, and report a
dependency wait that runs past its bound as an error (forced from the host
with a bound of zero polls, so every kernel still exits normally)."""
import os
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

from paper_0904_0939_amd import fdtd as F  # noqa: E402
from paper_0904_0939_amd import workloads as W  # noqa: E402
from paper_0904_0939_amd.solver import Batch, Solver  # noqa: E402


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def make_batch(dtype="f32"):
    rng = np.random.default_rng(9)
    lats = [W.Lattice(N, 12.0, W.POT_WELLS, W.random_wells(rng), seed=6) for N in (40, 64, 96, 48, 72)]
    b = Batch(lats, dtype=dtype)
    for m, l in enumerate(lats):
        b.set_potential(l.pot_kind, l.pot_params, member=m)
    b.set_initial(6)
    return b, lats


@pytest.mark.parametrize("persist,graph", [(7, False), (64, True), (3, True), (200, False)])
def test_batch_persistent_equals_per_step_launches(persist, graph):
    say(f"case: persistent batch persist={persist} graph={graph}")
    ref, lats = make_batch()
    t = ref.tuning()
    assert t["persist"] == 64  # the batch default
    ref.set_tuning(t["vz"], t["ry"], t["xchunk"], t["grid"], t["xcd_remap"], t["depth"], 0, 0)
    ref.evolve(150, use_graph=graph)
    b, _ = make_batch()
    b.set_tuning(t["vz"], t["ry"], t["xchunk"], t["grid"], t["xcd_remap"], t["depth"], 0, persist)
    b.evolve(150, use_graph=graph)
    for m in range(len(lats)):
        assert np.array_equal(b.state(m), ref.state(m)), m
        assert b.history(m, 150) == ref.history(m, 150), m
    assert b.observables() == ref.observables()


@pytest.mark.parametrize("dtype", ["f64", "bf16"])
def test_single_lattice_persistent_equals_per_step(dtype):
    say(f"case: persistent single {dtype}")
    out = []
    for persist in (0, 16):
        s = Solver(64, 10.0, dtype=dtype)
        s.set_potential(F.POT_CORNELL, W.CORNELL_PARAMS)
        s.set_initial(2, parity=W.parity_word(z=2))
        t = s.tuning()
        s.set_tuning(t["vz"], t["ry"], 0, 0, 1, t["depth"], 0, persist)
        s.evolve(101)
        out.append((s.state(), s.observables()[0]))
        s.close()
    assert np.array_equal(out[0][0], out[1][0])
    assert out[0][1] == out[1][1]


def test_persistent_convergence_stop_matches():
    say("case: persistent convergence")
    done = []
    for persist in (0, 10):
        s = Solver(24, 8.0, dtype="f64")
        s.set_potential(F.POT_HO, [1, 1, 1])
        s.set_initial(2)
        t = s.tuning()
        s.set_tuning(t["vz"], t["ry"], 0, 0, 1, 1, 0, persist)
        done.append(s.evolve(20000, check_every=50, rel_tol=1e-9))
        s.close()
    assert done[0] == done[1] and done[0][1]


def test_bounded_wait_reports_an_error():
    """A bound of zero polls makes the first unmet wait give up: 256
    work-groups against 16 work items per step, so work items of step 1 are
    taken while step 0 runs.  The launch drains and evolve reports EHIP; a
    handle made without the bound works as before."""
    say("case: persistent wait bound")
    os.environ["FDTD_PERSIST_SPIN_LIMIT"] = "0"
    try:
        s = Solver(64, 10.0, dtype="f32")
    finally:
        del os.environ["FDTD_PERSIST_SPIN_LIMIT"]
    s.set_potential(F.POT_HO, [1, 1, 1])
    s.set_initial(1)
    t = s.tuning()
    s.set_tuning(t["vz"], t["ry"], 0, 0, 1, 1, 0, 8)
    with pytest.raises(F.FdtdError) as ei:
        s.evolve(8, use_graph=False)
    assert ei.value.status == F.EHIP and "dependency wait" in str(ei.value)
    s.close()
    s = Solver(64, 10.0, dtype="f32")
    s.set_potential(F.POT_HO, [1, 1, 1])
    s.set_initial(1)
    s.set_tuning(t["vz"], t["ry"], 0, 0, 1, 1, 0, 8)
    s.evolve(16)
    assert s.observables()[0]["step"] == 16


@pytest.mark.parametrize("passes,steps,graph,depth", [(5, 150, True, 2), (64, 151, False, 2),
                                                     (1, 40, True, 2), (8, 97, True, 4),
                                                     (8, 97, True, 5)])
def test_batch_persistent_two_step_passes_equal_per_pass_launches(passes, steps, graph, depth):
    """Persistent two-step passes (tblock 2 with persist = passes per launch):
    the same bits, histories and observables as one launch per pass of the
    same tiles, odd step counts included (the last step runs alone)."""
    say(f"case: persistent two-step batch passes={passes} steps={steps} graph={graph} depth={depth}")
    out = []
    for persist in (0, passes):
        b, lats = make_batch()
        b.set_tuning(4, 1, 0, 0, 1, depth, 0, persist, 1, 2)
        b.evolve(steps, use_graph=graph)
        out.append(([b.state(m) for m in range(len(lats))],
                    [b.history(m, steps) for m in range(len(lats))], b.observables()))
        b.close()
    for m in range(len(out[0][0])):
        assert np.array_equal(out[0][0][m], out[1][0][m]), m
        assert out[0][1][m] == out[1][1][m], m
    assert out[0][2] == out[1][2]


@pytest.mark.parametrize("dtype,depth,tile", [("f64", 2, 0), ("bf16", 2, 0), ("f32", 4, 0),
                                              ("f32", 4, 1), ("bf16", 3, 1), ("f32", 5, 1)])
def test_single_lattice_persistent_two_step_equals_per_pass(dtype, depth, tile):
    say(f"case: persistent two-step single {dtype} depth={depth} tile={tile}")
    vz = {"f64": 2, "bf16": 8, "f32": 4}[dtype]
    out = []
    for persist in (0, 8):
        s = Solver(72, 10.0, dtype=dtype)
        s.set_potential(F.POT_CORNELL, W.CORNELL_PARAMS)
        s.set_initial(2, parity=W.parity_word(z=2))
        s.set_tuning(vz, 1, 0, 0, 1, depth, 0, persist, 1, 2, tile)
        s.evolve(61)
        out.append((s.state(), s.observables()[0]))
        s.close()
    assert np.array_equal(out[0][0], out[1][0])
    assert out[0][1] == out[1][1]


def test_persistent_two_step_bounded_wait_reports_an_error():
    say("case: persistent two-step wait bound")
    os.environ["FDTD_PERSIST_SPIN_LIMIT"] = "0"
    try:
        s = Solver(64, 10.0, dtype="f32")
    finally:
        del os.environ["FDTD_PERSIST_SPIN_LIMIT"]
    s.set_potential(F.POT_HO, [1, 1, 1])
    s.set_initial(1)
    s.set_tuning(4, 1, 0, 0, 1, 2, 0, 4, 0, 2)
    with pytest.raises(F.FdtdError) as ei:
        s.evolve(8, use_graph=False)
    assert ei.value.status == F.EHIP and "dependency wait" in str(ei.value)
    s.close()
