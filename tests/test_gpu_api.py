"""GPU tests of the parts of the interface around the step: Gaussian starts,
workspace ownership, the autotuner leaving the state untouched, the history
ring, conversions on readout, the multi-resolution helper and the autograd
Function.  Every numerical check is against the FP64 oracle."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

import oracle as orc  # noqa: E402
from paper_0904_0939_amd import fdtd as F  # noqa: E402
from paper_0904_0939_amd import workloads as W  # noqa: E402
from paper_0904_0939_amd.solver import EnergyOfPotential, Solver, multires  # noqa: E402


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def rel_l2(a, b):
    a = np.asarray(a, dtype=np.float64).ravel()
    b = np.asarray(b, dtype=np.float64).ravel()
    if a @ b < 0:
        b = -b
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def test_gauss_start_with_parity_matches_oracle():
    """Unit normals by Box-Muller from the same SplitMix64 draws, made S_x and
    A_y; then 200 FP64 steps."""
    say("case: gauss start fp64 24^3")
    N, L, seed = 24, 8.0, 21
    par = W.parity_word(x=1, y=2)
    s = Solver(N, L, dtype="f64")
    s.set_potential(F.POT_HO, [1.0, 1.3, 0.7])
    s.set_initial(seed, kind=F.INIT_GAUSS, parity=par)
    g0 = s.state()
    o0 = orc.initial(N, seed, kind=orc.INIT_GAUSS, parity=orc.parity_word(x=1, y=2))
    # log / sin / cos of the two sides may differ in the last bits
    assert np.abs(g0 - o0).max() < 1e-13 * np.abs(o0).max()
    assert np.array_equal(g0[::-1], g0) and np.array_equal(g0[:, ::-1], -g0)
    s.evolve(200)
    V = orc.potential(orc.POT_HO, [1.0, 1.3, 0.7], N, L)
    orc.evolve(o0, V, L, (L / N) ** 2 / 8, 200)
    assert s.observables()[0]["energy"] == pytest.approx(orc.observables(o0, V, L)["energy"],
                                                         rel=1e-10)


def test_library_and_caller_workspace_give_identical_bits():
    say("case: workspace ownership fp32 40^3")
    out = []
    for bind in (True, False):
        s = Solver(40, 10.0, dtype="f32", bind_torch_workspace=bind)
        s.set_potential(F.POT_CORNELL, W.CORNELL_PARAMS)
        s.set_initial(4)
        s.evolve(77)
        out.append((s.state(), s.observables()[0]["energy"]))
        s.close()
    assert np.array_equal(out[0][0], out[1][0])
    assert out[0][1] == out[1][1]


def test_autotune_leaves_state_step_and_history_untouched():
    say("case: autotune restore fp32 48^3")
    s = Solver(48, 10.0, dtype="f32", history=64)
    s.set_potential(F.POT_HO, [1, 1, 1])
    s.set_initial(8)
    s.evolve(30)
    before = s.state()
    ob = s.observables()[0]
    hist = s.history(0, 64)
    t, ms = s.autotune(3)
    assert ms > 0 or ms == -1.0
    assert np.array_equal(s.state(), before)
    ob2 = s.observables()[0]
    assert ob2["step"] == ob["step"] == 30
    # the reduction pass now runs in the chosen shape, which groups the lanes'
    # FP32 partial sums differently
    assert ob2["energy"] == pytest.approx(ob["energy"], rel=1e-6)
    assert s.history(0, 64) == hist
    assert s.tuning() == t
    s.evolve(10)
    assert s.observables()[0]["step"] == 40


def test_autotune_cache_file_carries_shapes_to_a_new_cache(tmp_path):
    """Shapes timed by one autotune call, saved to a file, cleared from the
    cache and loaded back, are set by a later autotune call without timing;
    an entry the handle rejects is dropped and the shapes are timed anew."""
    say("case: autotune cache file fp32 40^3")
    empty = tmp_path / "empty.txt"
    empty.write_text("")

    def solver():
        s = Solver(40, 10.0, dtype="f32")
        s.set_potential(F.POT_HO, [1, 1, 1])
        s.set_initial(9)
        return s

    F.fdtd_tune_cache_load(str(empty))
    s = solver()
    t1, ms1 = s.autotune(3)
    assert ms1 > 0
    s.close()
    path = tmp_path / "shapes.txt"
    F.fdtd_tune_cache_save(str(path))
    lines = [line for line in path.read_text().splitlines() if not line.startswith("#")]
    # the HO potential is evaluated in the kernel (vfuse 1): the key says so
    assert len(lines) == 1 and lines[0].split()[0].endswith(f"cu:{F.F32}:40:fv")
    assert lines[0].startswith("gfx950/")
    F.fdtd_tune_cache_load(str(empty))
    F.fdtd_tune_cache_load(str(path))
    s = solver()
    t2, ms2 = s.autotune(3)
    assert ms2 == -1.0 and t2 == t1 and s.tuning() == t1
    s.close()
    # vz = 3 fits no dtype: the entry is dropped, the shapes timed again
    key = lines[0].split()[0]
    bad = tmp_path / "bad.txt"
    bad.write_text(f"{key} 3 1 0 0 1 1 0 0 1 0 0\n")
    F.fdtd_tune_cache_load(str(bad))
    s = solver()
    t3, ms3 = s.autotune(3)
    assert ms3 > 0
    s.evolve(20)
    assert s.observables()[0]["step"] == 20
    s.close()


def test_autotune_keys_the_potential_source(tmp_path):
    """A lattice whose step reads the V table and one whose step evaluates V
    itself are tuned apart: the second autotune call times its own shapes
    and keeps the in-kernel potential."""
    say("case: autotune key per potential source fp32 40^3")
    empty = tmp_path / "empty.txt"
    empty.write_text("")
    F.fdtd_tune_cache_load(str(empty))
    shapes = []
    for vfuse in (0, 1):
        s = Solver(40, 10.0, dtype="f32")
        s.set_potential(F.POT_HO, [1, 1, 1])
        s.set_initial(9)
        t = s.tuning()
        t["vfuse"] = vfuse
        s.set_tuning(**t)
        got, ms = s.autotune(3)
        assert ms > 0 and got["vfuse"] == vfuse and s.tuning()["vfuse"] == vfuse
        s.evolve(10)
        assert s.observables()[0]["step"] == 10
        s.close()
    path = tmp_path / "shapes.txt"
    F.fdtd_tune_cache_save(str(path))
    keys = sorted(line.split()[0] for line in path.read_text().splitlines() if not line.startswith("#"))
    assert len(keys) == 2 and keys[1] == keys[0] + ":fv"
    F.fdtd_tune_cache_load(str(empty))


def test_history_ring_keeps_the_last_records():
    """A 16-record ring after 50 FP64 steps holds steps 34..49, each the
    oracle's energy of the state entering that step."""
    say("case: history ring fp64 12^3")
    N, L, seed = 12, 6.0, 5
    s = Solver(N, L, dtype="f64", history=16)
    s.set_potential(F.POT_CORNELL, W.CORNELL_PARAMS)
    s.set_initial(seed)
    s.evolve(50)
    h = s.history(0, 100)
    assert [r["step"] for r in h] == list(range(34, 50))
    assert len(s.history(0, 5)) == 5 and s.history(0, 5)[-1]["step"] == 49
    V = orc.potential(orc.POT_CORNELL, W.CORNELL_PARAMS, N, L)
    psi = orc.initial(N, seed)
    a = L / N
    energies = []
    for t in range(50):
        energies.append(orc.observables(psi, V, L)["energy"])
        psi = orc.normalized(orc.step(psi, V, L, a * a / 8), L)
    for r in h:
        assert r["energy"] == pytest.approx(energies[r["step"]], rel=1e-11)


def test_readout_conversions():
    """FP64 state read as FP32 / BF16 on the device and FP32 on the host,
    normalised to a^3 sum psi^2 = 1."""
    import torch

    say("case: readout conversions")
    N, L = 20, 8.0
    s = Solver(N, L, dtype="f64")
    s.set_potential(F.POT_HO, [1, 1, 1])
    s.set_initial(2)
    s.evolve(20)
    ref = s.psi(dtype=np.float64)
    a3 = (L / N) ** 3
    assert a3 * np.sum(ref * ref) == pytest.approx(1.0, rel=1e-12)
    assert np.array_equal(s.psi(dtype=np.float32), ref.astype(np.float32))
    d32 = s.psi_tensor(dtype=torch.float32).cpu().numpy()
    assert np.array_equal(d32, ref.astype(np.float32))
    b16 = s.psi_tensor(dtype=torch.bfloat16).float().cpu().numpy().astype(np.float64)
    assert np.abs(b16 - ref).max() <= 2.0 ** -8 * np.abs(ref).max()


@pytest.mark.parametrize("two_step", [False, True])
def test_multires_chain_reaches_the_oracle_ground_state(two_step):
    """BF16 16^3 -> FP32 32^3 (HO, L = 10): the chain's converged energy equals
    the oracle's converged FP64 energy on 32^3 from noise, with one or two
    steps per pass."""
    say(f"case: multires 16 -> 32 two_step={two_step}")
    L = 10.0
    s, log = multires([16, 32], L, F.POT_HO, [1, 1, 1], ["bf16", "f32"], seed=3,
                      rel_tol=(1e-5, 1e-8), max_steps=(4000, 40000), check_every=50,
                      two_step=two_step)
    if two_step:
        assert s.tuning()["tblock"] == 2 and s.tuning()["depth"] == 5
    assert [n for n, _, _ in log] == [16, 32]
    assert log[-1][2], log  # the FP32 level converged
    e = s.observables()[0]["energy"]
    V = orc.potential(orc.POT_HO, [1, 1, 1], 32, L)
    psi = orc.initial(32, 3)
    orc.evolve(psi, V, L, (L / 32) ** 2 / 8, 40000, check_every=50, rel_tol=1e-11)
    eo = orc.observables(psi, V, L)["energy"]
    say(f"chain {e:.10f} oracle {eo:.10f} steps {log}")
    assert e == pytest.approx(eo, rel=2e-6)
    assert rel_l2(s.psi(), psi) < 1e-3


def test_multires_two_step_takes_wide_tiles_for_large_table_levels():
    """two_step on a chain whose potential is only a table (the dodecahedron
    well): the 512^3 FP32 level takes 16 x 128 tiles, and the chain ends where
    the same chain with one step per pass ends (the rescale follows every
    second step, so the energies agree to rounding)."""
    say("case: multires 256 -> 512 dodecahedron two_step tiles")
    out = []
    for two_step in (False, True):
        s, log = multires([256, 512], 25.6, F.POT_DODECA, [-100.0], ["f32", "f32"], seed=5,
                          rel_tol=(0.0, 0.0), max_steps=(200, 200), two_step=two_step)
        t = s.tuning()
        if two_step:
            assert t["tblock"] == 2 and t["tile"] == 1 and t["vfuse"] == 1
        out.append((s.observables()[0]["energy"], [n for _, n, _ in log]))
        s.close()
    assert out[0][1] == out[1][1] == [200, 200]
    assert out[1][0] == pytest.approx(out[0][0], rel=1e-6)


def test_energy_of_potential_autograd_matches_oracle():
    """E(theta) with V(theta) = V0 + theta_0 W0 + theta_1 W1 built in torch:
    backward through the adjoint equals sum G W_k of the oracle's reverse
    recurrence, and central differences of the oracle's energy."""
    import torch

    say("case: autograd 10^3")
    N, L, T, k = 10, 8.0, 40, 8
    # inputs from numpy, handed to both sides
    x = (np.arange(N) * 2 - (N - 1)) * (L / N) / 2
    X, Y, Z = np.meshgrid(x, x, x, indexing="ij")
    V0n = 0.5 * (X**2 + Y**2 + Z**2)
    W0 = np.exp(-(X**2 + Y**2 + Z**2))
    W1 = X * Z
    psi0n = np.random.default_rng(11).uniform(-1.0, 1.0, (N, N, N))
    V0 = torch.tensor(V0n, dtype=torch.float64, device="cuda")
    Wt = [torch.tensor(w, dtype=torch.float64, device="cuda") for w in (W0, W1)]
    theta = torch.tensor([-0.7, 0.2], dtype=torch.float64, device="cuda", requires_grad=True)
    psi0 = torch.tensor(psi0n, dtype=torch.float64, device="cuda")
    s = Solver(N, L, dtype="f64")
    V = V0 + theta[0] * Wt[0] + theta[1] * Wt[1]
    E = EnergyOfPotential.apply(V, s, psi0, T, k)
    E.backward()
    g = theta.grad.cpu().numpy()
    th = [-0.7, 0.2]
    Vn = V0n + th[0] * W0 + th[1] * W1
    dt = (L / N) ** 2 / 8
    Eo, Go = orc.energy_grad_v(psi0n.copy(), Vn, L, dt, T)
    assert float(E.detach()) == pytest.approx(Eo, rel=1e-12)
    go = np.array([np.sum(Go * W0), np.sum(Go * W1)])
    np.testing.assert_allclose(g, go, rtol=1e-9, atol=1e-12 * np.abs(go).max())
    h = 1e-5
    for j, Wj in enumerate((W0, W1)):
        e = []
        for sg in (1, -1):
            p = psi0n.copy()
            Vh = Vn + sg * h * Wj
            orc.evolve(p, Vh, L, dt, T)
            e.append(orc.observables(p, Vh, L)["energy"])
        assert g[j] == pytest.approx((e[0] - e[1]) / (2 * h), rel=1e-6, abs=1e-9)


def test_readme_python_example_runs(tmp_path, monkeypatch):
    """The Python example of the README runs as written (in a scratch
    directory, where it writes its launch-shape file)."""
    import os
    import re

    say("case: README example")
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    text = open(os.path.join(root, "README.md")).read()
    blocks = re.findall(r"```python\n(.*?)```", text, re.S)
    assert blocks
    monkeypatch.chdir(tmp_path)
    env = {}
    exec(compile(blocks[0], "README.md", "exec"), env)
    assert (tmp_path / "shapes.txt").exists()
    assert env["s"].observables()[0]["energy"] < 1.0
