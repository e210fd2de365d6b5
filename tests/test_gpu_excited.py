"""Excited states (Sec. III) and the dodecahedron well (Sec. VII.E) on the
GPU against the FP64 oracle: the well's membership test site by site (odd
N puts sites exactly on faces), the one-shot projection of the snapshot
method, and relaxation with the lower states projected out every k steps."""
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
    if a @ b < 0:
        b = -b
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.mark.parametrize("N", [40, 41, 33])
def test_dodecahedron_well_matches_oracle_site_by_site(N):
    """FP64: 40 steps from the same noise.  A single site on the wrong side
    of a face would change V there by 100 and show far above 1e-10."""
    say(f"case: dodecahedron N={N}")
    L = 0.1 * N
    s = Solver(N, L, dtype="f64", dt_over_a2=0.1)
    s.set_potential(F.POT_DODECA, [-100.0])
    s.set_initial(3)
    s.evolve(40)
    V = orc.potential(orc.POT_DODECA, [-100.0], N, L)
    psi = orc.initial(N, 3)
    orc.evolve(psi, V, L, 0.1 * (L / N) ** 2, 40)
    np.testing.assert_allclose(s.psi(), psi, rtol=0, atol=1e-11 * np.abs(psi).max())
    ob, oo = s.observables()[0], orc.observables(psi, V, L)
    assert ob["potential"] == pytest.approx(oo["potential"], rel=1e-11)


@pytest.mark.parametrize("dtype,tol", [("f64", 1e-12), ("f32", 2e-6)])
def test_projection_matches_oracle(dtype, tol):
    """Two non-orthogonal numpy states projected out of a numpy state, one
    after the other: coefficients and result against the oracle."""
    say(f"case: projection {dtype}")
    N, L = 24, 8.0
    rng = np.random.default_rng(8)
    phi = [rng.standard_normal((N, N, N)) for _ in range(2)]
    phi[1] += 0.3 * phi[0]
    psi0 = rng.standard_normal((N, N, N)) + 0.7 * phi[0] - 0.4 * phi[1]
    if dtype == "f32":  # both sides see the values the GPU stores
        phi = [p.astype(np.float32).astype(np.float64) for p in phi]
        psi0 = psi0.astype(np.float32).astype(np.float64)
    s = Solver(N, L, dtype=dtype)
    s.set_potential(F.POT_HO, [1, 1, 1])
    s.set_initial_array(psi0)
    s.set_projection_states(phi)
    coef = s.project()
    ref, rc = orc.project_out(psi0, phi)
    np.testing.assert_allclose(coef, rc, rtol=tol)
    got = s.state().astype(np.float64)
    assert np.linalg.norm(got - ref) <= tol * np.linalg.norm(ref)
    # the pending scale was reset from the new norm
    assert s.observables()[0]["norm2"] == pytest.approx((L / N) ** 3 * np.sum(ref * ref), rel=tol)


@pytest.mark.parametrize("every,graph", [(1, False), (7, True), (64, True)])
def test_deflated_relaxation_matches_oracle_fp64(every, graph):
    """Anisotropic oscillator: converge the ground state (oracle), then relax
    a new start with it projected out every k steps, on both sides."""
    say(f"case: deflated fp64 every={every} graph={graph}")
    N, L = 16, 10.0
    dt = (L / N) ** 2 / 8
    w = [1.0, 1.6, 2.3]
    V = orc.potential(orc.POT_HO, w, N, L)
    psi0 = orc.initial(N, 5)  # each side converges its own ground state
    orc.evolve(psi0, V, L, dt, 4000)
    g = Solver(N, L, dtype="f64")
    g.set_potential(F.POT_HO, w)
    g.set_initial(5)
    g.evolve(4000)
    T = 640
    s = Solver(N, L, dtype="f64")
    s.set_potential(F.POT_HO, w)
    s.set_initial(6)
    s.set_projection_states([g.psi()])
    s.evolve(T, project_every=every, use_graph=graph)
    psi = orc.initial(N, 6)
    orc.evolve(psi, V, L, dt, T, deflate=[psi0], project_every=every)
    eo = orc.observables(psi, V, L)["energy"]
    assert s.observables()[0]["energy"] == pytest.approx(eo, rel=1e-10)
    assert rel_l2(s.psi(), psi) < 1e-9
    # the first excitation is the x one: E0 + 1 up to discretisation
    e0 = orc.observables(psi0, V, L)["energy"]
    assert abs(eo - e0 - 1.0) < 0.05


def test_snapshot_method_on_the_gpu():
    """The paper's one-shot estimate with GPU states: a snapshot at 240 steps
    minus its ground-state component has the first excited energy to the
    oracle's accuracy (and the oracle's own estimate)."""
    say("case: snapshot method")
    N, L = 16, 10.0
    w = [1.0, 1.6, 2.3]
    g = Solver(N, L, dtype="f64")
    g.set_potential(F.POT_HO, w)
    g.set_initial(5)
    g.evolve(4000)
    psi0 = g.psi()
    s = Solver(N, L, dtype="f64")
    s.set_potential(F.POT_HO, w)
    s.set_initial(5)
    s.evolve(240)
    s.set_projection_states([psi0])
    s.project()
    e_gpu = s.observables()[0]["energy"]
    V = orc.potential(orc.POT_HO, w, N, L)
    dt = (L / N) ** 2 / 8
    o0 = orc.initial(N, 5)
    orc.evolve(o0, V, L, dt, 4000)
    snap = orc.initial(N, 5)
    orc.evolve(snap, V, L, dt, 240)
    est, _ = orc.project_out(snap, [o0])
    assert e_gpu == pytest.approx(orc.observables(est, V, L)["energy"], rel=1e-10)


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_deflated_relaxation_reduced_precision(dtype):
    """FP32 against the oracle to 1e-5; BF16 storage (FP32 ground state kept)
    to the BF16 floor, then an FP32 finish to 1e-5."""
    say(f"case: deflated {dtype}")
    N, L = 24, 10.0
    dt = (L / N) ** 2 / 8
    w = [1.0, 1.4, 2.0]
    V = orc.potential(orc.POT_HO, w, N, L)
    psi0 = orc.initial(N, 2)
    orc.evolve(psi0, V, L, dt, 6000)
    T = 3000
    psi = orc.initial(N, 4)
    orc.evolve(psi, V, L, dt, T, deflate=[psi0], project_every=10)
    eo = orc.observables(psi, V, L)["energy"]
    g = Solver(N, L, dtype="f64")  # the GPU's own ground state, FP64
    g.set_potential(F.POT_HO, w)
    g.set_initial(2)
    g.evolve(6000)
    s = Solver(N, L, dtype=dtype)
    s.set_potential(F.POT_HO, w)
    s.set_initial(4)
    s.set_projection_states([g.psi()])
    s.evolve(T, project_every=10)
    e = s.observables()[0]["energy"]
    assert e == pytest.approx(eo, rel=1e-5 if dtype == "f32" else 2e-3)


def test_batch_member_projection():
    """Projection acts on the member that keeps states; others are untouched."""
    say("case: batch projection")
    lats = [W.Lattice(N, 10.0, W.POT_HO, [1.0, 1.5, 2.0], seed=3) for N in (16, 20)]
    b = Batch(lats, dtype="f64")
    for m, l in enumerate(lats):
        b.set_potential(l.pot_kind, l.pot_params, member=m)
    b.set_initial(3)
    start0 = b.state(0)
    dt = (10.0 / 20) ** 2 / 8
    V = orc.potential(orc.POT_HO, [1.0, 1.5, 2.0], 20, 10.0)
    psi0 = orc.initial(20, 7)  # each side converges its own ground state
    orc.evolve(psi0, V, 10.0, dt, 3000)
    g = Solver(20, 10.0, dtype="f64")
    g.set_potential(F.POT_HO, [1.0, 1.5, 2.0])
    g.set_initial(7)
    g.evolve(3000)
    b.set_projection_states([g.psi()], member=1)
    b.evolve(200, project_every=5)
    # member 0 as a plain single-lattice run from the same start
    s = Solver(16, 10.0, dtype="f64")
    s.set_potential(F.POT_HO, [1.0, 1.5, 2.0])
    s.set_initial_array(start0)
    psi = orc.initial(20, 3, member=1)
    orc.evolve(psi, V, 10.0, dt, 200, deflate=[psi0], project_every=5)
    assert b.observables()[1]["energy"] == pytest.approx(orc.observables(psi, V, 10.0)["energy"], rel=1e-10)
    s.evolve(200)
    assert b.observables()[0]["energy"] == pytest.approx(s.observables()[0]["energy"], rel=1e-12)
