"""Temporal blocking (tuning field `tblock` = 2): one pass over HBM advances a
lattice two steps, on tiles of the (y, z) plane.  With the rescale off it
must give the same bits as one launch per step (the per-site arithmetic and,
for BF16, the rounding bits are shared; only the FP64 summation order of the
reductions differs, tiles instead of flattened chunks); with a rescale every
second step the states agree to the rounding of that order (BF16: to its
stochastic rounding, which then draws other roundings); with a rescale every
step, or passes that start at an odd step, it must follow the FP64 oracle to
the parity tolerances (FP64 1e-10, FP32 1e-5)."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

import oracle as orc  # noqa: E402
from paper_0904_0939_amd import fdtd as F  # noqa: E402
from paper_0904_0939_amd import workloads as W  # noqa: E402
from paper_0904_0939_amd.solver import Batch, Solver  # noqa: E402


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def rel_l2(a, b):
    a = np.asarray(a, dtype=np.float64).ravel()
    b = np.asarray(b, dtype=np.float64).ravel()
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


VW = {"f32": 4, "f64": 2, "bf16": 8}
POT = {"ho": (F.POT_HO, [1.0, 1.2, 0.8]), "cornell": (F.POT_CORNELL, W.CORNELL_PARAMS)}


def run(dtype, N, pot, xchunk, depth, vfuse, tblock, steps, renorm, graph, L=10.0, seed=5,
        tile=0):
    s = Solver(N, L, dtype=dtype)
    s.set_potential(*POT[pot])
    s.set_initial(seed)
    # one-step launches prefetch at most 3 planes (depth 4 is the two-step
    # pass's) and have no tile shape
    s.set_tuning(VW[dtype], 1, xchunk, 0, 1, depth if tblock == 2 else min(depth, 3), 0, 0,
                 vfuse, tblock, tile if tblock == 2 else 0)
    s.evolve(steps, renorm_every=renorm, use_graph=graph)
    out = (s.state(), s.observables()[0], s.history(0, steps))
    s.close()
    return out


# (dtype, N, potential, xchunk, depth, vfuse, tile): tiles ragged in y and z,
# several x-ranges per lattice, the in-kernel potential, and sides beyond
# 256 vz (F32 and BF16 tiles are 32 x 64 sites, or 16 x 128 with tile 1; F64
# 16 x 32)
CASES = [
    ("f32", 40, "cornell", 0, 1, 0, 0),
    ("f32", 64, "ho", 8, 2, 0, 0),
    ("f32", 96, "cornell", 24, 1, 1, 0),
    ("f32", 516, "cornell", 0, 2, 1, 0),
    ("f64", 48, "ho", 0, 1, 0, 0),
    ("f64", 300, "cornell", 32, 1, 0, 0),
    ("bf16", 64, "cornell", 0, 2, 0, 0),
    ("bf16", 96, "ho", 24, 3, 1, 0),
    # prefetch depths 4 and 5 (an 8-slot ring): whole trips, every tail length
    ("f32", 72, "cornell", 0, 4, 0, 0),
    ("f32", 100, "ho", 30, 4, 1, 0),
    ("bf16", 64, "cornell", 0, 4, 1, 0),
    ("f32", 72, "ho", 9, 5, 1, 0),
    ("f32", 100, "cornell", 0, 5, 0, 0),
    ("bf16", 96, "cornell", 24, 5, 1, 0),
    # 16 x 128 tiles: a lattice narrower than one tile, sides ragged in y and
    # z (136 = 128 + 8, 8.5 tiles of 16 rows), side 516, BF16
    ("f32", 40, "ho", 0, 2, 0, 1),
    ("f32", 136, "cornell", 24, 4, 0, 1),
    ("f32", 516, "cornell", 0, 5, 1, 1),
    ("bf16", 136, "ho", 40, 3, 1, 1),
]


def same_records(h1, h2, rel):
    assert [r["step"] for r in h1] == [r["step"] for r in h2]
    for a, b in zip(h1, h2):
        for k in ("norm2", "energy", "kinetic", "potential", "r_rms"):
            assert a[k] == pytest.approx(b[k], rel=rel, abs=1e-300), (a["step"], k)


@pytest.mark.parametrize("dtype,N,pot,xchunk,depth,vfuse,tile", CASES)
def test_two_step_passes_equal_one_step_launches(dtype, N, pot, xchunk, depth, vfuse, tile):
    # graph-captured chunks of 64 + 54 (N < 256) or 50 steps: odd numbers of
    # passes, so the buffer holding the result flips differently from the
    # step count
    steps = 50 if N >= 256 else 118
    for graph in (True, False):
        say(f"case: tblock {dtype} N={N} {pot} xchunk={xchunk} depth={depth} vfuse={vfuse} "
            f"tile={tile} graph={graph}")
        # rescale off: the states are the same bits
        ref = run(dtype, N, pot, xchunk, depth, vfuse, 0, steps, 0, graph)
        got = run(dtype, N, pot, xchunk, depth, vfuse, 2, steps, 0, graph, tile=tile)
        assert np.array_equal(got[0], ref[0])
        assert ref[1]["step"] == got[1]["step"] == steps
        # BF16 lanes hold 8 sites in one-step launches and 4 here: their FP32
        # partial sums round differently
        same_records(got[2], ref[2], 1e-6 if dtype == "bf16" else 1e-12)
    # a rescale every second step: the scale comes from sums taken in another
    # order, so the states agree to that rounding
    ref = run(dtype, N, pot, xchunk, depth, vfuse, 0, steps, 2, True)
    got = run(dtype, N, pot, xchunk, depth, vfuse, 2, steps, 2, True, tile=tile)
    tol = {"f32": 1e-6, "f64": 1e-13, "bf16": 1e-2}[dtype]
    got_s, ref_s = got[0], ref[0]
    if dtype == "bf16":
        got_s = (got_s.astype(np.uint32) << 16).view(np.float32)
        ref_s = (ref_s.astype(np.uint32) << 16).view(np.float32)
    assert rel_l2(got_s, ref_s) < tol
    same_records(got[2], ref[2], {"f32": 1e-6, "f64": 1e-12, "bf16": 1e-3}[dtype])


@pytest.mark.parametrize("dtype,N,grid,tile", [("f32", 8, 0, 0), ("f64", 6, 0, 0), ("f32", 44, 7, 0),
                                              ("f64", 34, 3, 0), ("f32", 8, 0, 1), ("f32", 140, 5, 1),
                                              ("bf16", 24, 2, 1)])
def test_small_lattices_and_fewer_work_groups_than_tiles(dtype, N, grid, tile):
    """Lattices smaller than one tile (most lanes and the whole halo frame
    outside the lattice), and a grid of fewer work-groups than tiles (each
    work-group takes several tiles in turn), on both tile shapes."""
    say(f"case: tblock {dtype} N={N} grid={grid} tile={tile}")
    out = []
    for tblock in (0, 2):
        s = Solver(N, 6.0, dtype=dtype)
        s.set_potential(*POT["ho"])
        s.set_initial(3)
        s.set_tuning(VW[dtype], 1, 0, grid, 1, 1, 0, 0, 0, tblock, tile if tblock == 2 else 0)
        s.evolve(50, renorm_every=0)
        out.append((s.state(), s.history(0, 50)))
        s.close()
    assert np.array_equal(out[0][0], out[1][0])
    # BF16 lanes hold 8 sites in one-step launches and 4 here (FP32 partial
    # sums rounded differently)
    same_records(out[1][1], out[0][1], 1e-6 if dtype == "bf16" else 1e-12)


def test_odd_step_count_runs_a_single_step_at_the_end():
    say("case: tblock odd count f32 40^3")
    ref = run("f32", 40, "ho", 0, 1, 0, 0, 61, 0, True)
    got = run("f32", 40, "ho", 0, 1, 0, 2, 61, 0, True)
    assert np.array_equal(got[0], ref[0])
    same_records(got[2], ref[2], 1e-12)


@pytest.mark.parametrize("dtype,N,pot,tol", [("f64", 32, "ho", 1e-10), ("f32", 40, "cornell", 1e-5)])
def test_rescale_every_step_and_odd_starts_follow_the_oracle(dtype, N, pot, tol):
    """renorm_every = 1 defers each pass's first rescale to its second step;
    after 3 steps the passes start at odd steps.  The oracle rescales every
    step: the normalised states and energies agree to the dtype's tolerance."""
    say(f"case: tblock vs oracle {dtype} N={N}")
    L, seed = 10.0, 7
    s = Solver(N, L, dtype=dtype)
    s.set_potential(*POT[pot])
    s.set_initial(seed)
    s.set_tuning(VW[dtype], 1, 0, 0, 1, 1, 0, 0, 0, 2)
    s.evolve(3)
    s.evolve(300)
    kind, params = POT[pot]
    V = orc.potential(kind, params, N, L)
    psi = orc.initial(N, seed)
    orc.evolve(psi, V, L, (L / N) ** 2 / 8, 303)
    e_gpu = s.observables()[0]["energy"]
    e_orc = orc.observables(psi, V, L)["energy"]
    say(f"energy {e_gpu:.12f} oracle {e_orc:.12f}")
    assert e_gpu == pytest.approx(e_orc, rel=tol)
    assert rel_l2(s.psi(), orc.normalized(psi, L)) < tol
    hist = s.history(0, 303)
    assert [r["step"] for r in hist] == list(range(303))


def test_batch_two_step_passes_equal_one_step_launches():
    """Lattices of several sides in one handle: tiles of every member in one
    launch (both tile shapes), each member's sums finalised by its own last
    work-group."""
    say("case: tblock batch f32")
    rng = np.random.default_rng(4)
    lats = [W.Lattice(N, 12.0, W.POT_WELLS, W.random_wells(rng), seed=2) for N in (40, 64, 96, 48, 72)]
    out = []
    for tblock, tile in ((0, 0), (2, 0), (2, 1)):
        b = Batch(lats, dtype="f32")
        for m, l in enumerate(lats):
            b.set_potential(l.pot_kind, l.pot_params, member=m)
        b.set_initial(2)
        b.set_tuning(4, 1, 0, 0, 1, 2, 0, 0, 0, tblock, tile)
        b.evolve(60, renorm_every=0)
        out.append(([b.state(m) for m in range(len(lats))], [b.history(m, 60) for m in range(len(lats))]))
        b.close()
    for got in out[1:]:
        for m in range(len(lats)):
            assert np.array_equal(out[0][0][m], got[0][m]), m
            same_records(got[1][m], out[0][1][m], 1e-12)
