"""GPU tests of the runtime around the kernels: the graph cache across launch
shapes, asynchronous evolve calls, checkpoint and resume, caller workspaces
poisoned with NaN, the gradient driver with a short history ring, and the
reimposition of the Sec. IV symmetry operators on a state that does not have
the symmetry (against the oracle's orc_reimpose, bit for bit)."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

import oracle as orc  # noqa: E402
from paper_0904_0939_amd import fdtd as F  # noqa: E402
from paper_0904_0939_amd import workloads as W  # noqa: E402
from paper_0904_0939_amd.solver import EnergyOfPotential, Solver  # noqa: E402


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def cornell(N, dtype, seed=4, **kw):
    s = Solver(N, 12.0, dtype=dtype, **kw)
    s.set_potential(F.POT_CORNELL, W.CORNELL_PARAMS)
    s.set_initial(seed)
    return s


# ------------------------------------------------------------ graph cache --
def test_graphs_survive_launch_shape_changes_on_one_handle():
    """Shape A, then a shape with more work items (the item and partial-sum
    buffers are reallocated), then A again, all through captured graphs: the
    state must equal a fresh handle's run of the same shapes bit for bit."""
    say("case: graph cache across shapes fp32 48^3")
    A = (4, 1, 0, 0, 1, 1, 0, 0, 0, 0)
    B = (4, 1, 8, 0, 1, 1, 0, 0, 0, 2)  # two-step tiles, x-ranges of 8 planes
    C = (1, 1, 4, 0, 1, 1, 0, 0, 0, 0)  # scalar lanes, more items still

    def run(handle, shapes):
        for t in shapes:
            handle.set_tuning(*t)
            handle.evolve(24, use_graph=True)
        return handle.state()

    one = cornell(48, "f32")
    got = run(one, [A, B, A, C, A])
    c = one.counters()
    assert c["graph_captures"] >= 3 and c["graph_replays"] >= 5
    ref = []
    for t in (A, B, A, C, A):
        fresh = cornell(48, "f32")
        if ref:
            fresh.restore(ref[-1])
        fresh.set_tuning(*t)
        fresh.evolve(24, use_graph=False)
        ref.append(fresh.checkpoint())
        last = fresh.state()
        fresh.close()
    assert np.array_equal(got, last)
    one.close()


# ---------------------------------------------------------- async evolve --
@pytest.mark.parametrize("steps", [20, 21, 400])
def test_async_evolve_equals_sync_and_captures_once(steps):
    say(f"case: async evolve {steps} steps fp32 64^3")
    a = cornell(64, "f32")
    b = cornell(64, "f32")
    a.evolve(steps, use_graph=True)
    b.evolve(steps, use_graph=True, async_launch=True)
    assert np.array_equal(a.state(), b.state())
    # every graph a call of this length replays exists after one call per
    # input buffer: later calls capture nothing
    b.evolve(steps, use_graph=True, async_launch=True)
    c0 = b.counters()
    for _ in range(3):
        b.evolve(steps, use_graph=True, async_launch=True)
    c1 = b.counters()
    assert c1["graph_captures"] == c0["graph_captures"]
    assert c1["graph_replays"] > c0["graph_replays"]
    assert c1["allocations"] == c0["allocations"]
    a.evolve(4 * steps, use_graph=True)  # one call of 4x the length: other graphs, same launches
    assert np.array_equal(a.state(), b.state())
    assert b.observables()[0]["step"] == 5 * steps


def test_async_evolve_reports_nonfinite_on_the_next_synchronous_call():
    say("case: async non-finite report")
    s = Solver(16, 8.0, dtype="f32")
    V = np.zeros((16, 16, 16))
    V[3, 4, 5] = np.nan
    s.set_potential_array(V)
    s.set_initial(1)
    s.evolve(10, async_launch=True)
    with pytest.raises(F.FdtdError) as e:
        s.evolve(1)
    assert e.value.status == F.ENONFINITE


# ------------------------------------------------------ checkpoint/resume --
@pytest.mark.parametrize("dtype", ["f64", "f32", "bf16"])
def test_split_run_takes_the_same_bits_as_an_unsplit_run(dtype):
    """A run stopped, saved, loaded into a fresh handle and continued ends in
    the same bits as the run carried through, BF16 stochastic rounding
    included (its bits depend on the step count the record carries)."""
    say(f"case: checkpoint resume {dtype} 40^3")
    k = 37
    whole = cornell(40, dtype, seed=6)
    whole.evolve(2 * k)
    part = cornell(40, dtype, seed=6)
    part.evolve(k)
    rec = part.checkpoint()
    part.close()
    resumed = Solver(40, 12.0, dtype=dtype)
    resumed.set_potential(F.POT_CORNELL, W.CORNELL_PARAMS)
    resumed.restore(rec)
    assert resumed.observables()[0]["step"] == k
    resumed.evolve(k)
    assert np.array_equal(whole.state(), resumed.state())
    ow, orr = whole.observables()[0], resumed.observables()[0]
    assert orr["step"] == ow["step"] == 2 * k
    assert orr["tau"] == ow["tau"]
    assert orr["energy"] == ow["energy"]
    # the resumed history starts at the record's step
    hist = resumed.history(0, 1000)
    assert len(hist) == k and hist[0]["step"] == k
    assert [h["energy"] for h in hist] == [h["energy"] for h in whole.history(0, k)]


def test_checkpoint_on_device_and_mismatch_errors():
    say("case: checkpoint device record")
    import torch

    s = cornell(32, "f32", seed=2)
    s.evolve(10)
    n = F.fdtd_checkpoint_size(s.h, 0)
    dev = torch.empty(n, dtype=torch.uint8, device="cuda")
    F.fdtd_checkpoint_save(s.h, 0, dev.data_ptr(), 1)
    host = s.checkpoint()
    assert np.array_equal(dev.cpu().numpy(), host)
    t = Solver(32, 12.0, dtype="f32")
    t.set_potential(F.POT_CORNELL, W.CORNELL_PARAMS)
    F.fdtd_checkpoint_load(t.h, 0, dev.data_ptr(), 1)
    assert np.array_equal(t.state(), s.state())
    for other in (Solver(32, 12.0, dtype="f64"), Solver(40, 12.0, dtype="f32"),
                  Solver(32, 13.0, dtype="f32")):
        with pytest.raises(F.FdtdError) as e:
            other.restore(host)
        assert e.value.status == F.EINVAL


# ------------------------------------------------------ poisoned workspace --
@pytest.mark.parametrize("dtype", ["f32", "bf16", "f64"])
def test_nan_filled_caller_workspace_gives_the_same_bits(dtype):
    """Every byte of a caller's workspace set to 0xFF (a NaN in every float
    type) before binding: padding, unused ring records and partial-sum slots
    must never reach a result."""
    say(f"case: poisoned workspace {dtype}")
    import torch

    out = []
    for poison in (False, True):
        s = Solver(36, 12.0, dtype=dtype, bind_torch_workspace=False)
        nbytes = F.fdtd_workspace_size(s.h)
        ws = torch.full((nbytes,), 255 if poison else 0, dtype=torch.uint8, device="cuda")
        F.fdtd_bind_workspace(s.h, ws.data_ptr(), nbytes)
        s._ws = ws
        s.set_potential(F.POT_CORNELL, W.CORNELL_PARAMS)
        s.set_initial(8)
        s.evolve(50)
        s.evolve(30, check_every=10, rel_tol=1e-30)
        out.append((s.state(), s.observables()[0], [h["energy"] for h in s.history(0, 80)]))
        s.close()
    assert np.array_equal(out[0][0], out[1][0])
    assert out[0][1] == out[1][1]
    assert out[0][2] == out[1][2] and all(np.isfinite(out[1][2]))


# ------------------------------------------------- gradient, short ring --
def test_gradient_with_history_shorter_than_a_segment():
    """checkpoint_every larger than the history ring: the forward's scales are
    read back before the ring wraps, so the gradient is the default ring's."""
    say("case: gradient history 16 < k 40")
    p = [1.0, 1.0, 1.0, 1.5, 0.3, 0.0, -0.2, 0.8]
    res = []
    for hist in (0, 16):
        s = Solver(16, 8.0, dtype="f32", history=hist)
        s.set_potential(F.POT_WELLS, p)
        s.set_initial(14)
        E, g, G = s.energy_grad(120, 40, theta=p, wrt=[3, 7], want_field=True)
        res.append((E, g, G.cpu().numpy()))
        s.close()
    assert res[0][0] == res[1][0]
    assert res[0][1] == res[1][1]
    assert np.array_equal(res[0][2], res[1][2])


def test_energy_of_potential_without_grad_runs_no_adjoint():
    """Under no_grad the Function only relaxes and reads E (no checkpoint
    buffers are allocated); with grad it gives the same E."""
    say("case: EnergyOfPotential no_grad")
    import torch

    N, L = 16, 8.0
    s = Solver(N, L, dtype="f32")
    s.set_potential(F.POT_HO, [1, 1, 1])
    s.set_initial(3)
    psi0 = s.psi_tensor()
    V = torch.tensor(orc.potential(orc.POT_HO, [1, 1, 1], N, L), device="cuda")
    with torch.no_grad():
        e_ng = EnergyOfPotential.apply(V, s, psi0, 60, 20)
    assert getattr(s, "_gws", None) is None  # no checkpoint workspace was needed
    Vg = V.clone().requires_grad_(True)
    e_g = EnergyOfPotential.apply(Vg, s, psi0, 60, 20)
    assert s._gws is not None
    assert float(e_ng) == pytest.approx(float(e_g.detach()), rel=1e-14)
    e_g.backward()
    assert Vg.grad is not None and torch.isfinite(Vg.grad).all()


def test_gradient_workspace_is_reused_and_a_small_bound_one_is_refused():
    """Library-owned checkpoint memory is allocated once and kept for later
    calls that fit; a caller-bound buffer below fdtd_grad_workspace_size is
    refused with ENOMEM; a large enough one gives the same gradient."""
    say("case: gradient workspace")
    import torch

    p = [1.0, 1.0, 1.0, 1.5, 0.3, 0.0, -0.2, 0.8]
    out = []
    for mode in ("library", "bound"):
        s = Solver(16, 8.0, dtype="f32")
        s.set_potential(F.POT_WELLS, p)
        s.set_initial(14)
        if mode == "library":
            a0 = s.counters()["allocations"]
            r = F.fdtd_energy_grad(s.h, 60, 20, p, [3, 7])
            a1 = s.counters()["allocations"]
            F.fdtd_energy_grad(s.h, 40, 20, p, [3, 7])  # fits: no new allocation
            assert s.counters()["allocations"] == a1 == a0 + 1
            s.set_initial(14)
            r = F.fdtd_energy_grad(s.h, 60, 20, p, [3, 7])
        else:
            need = F.fdtd_grad_workspace_size(s.h, 60, 20)
            small = torch.empty(need - 256, dtype=torch.uint8, device="cuda")
            F.fdtd_bind_grad_workspace(s.h, small.data_ptr(), need - 256)
            with pytest.raises(F.FdtdError) as e:
                F.fdtd_energy_grad(s.h, 60, 20, p, [3, 7])
            assert e.value.status == F.ENOMEM
            ws = torch.full((need,), 255, dtype=torch.uint8, device="cuda")  # NaN-filled
            F.fdtd_bind_grad_workspace(s.h, ws.data_ptr(), need)
            s.set_initial(14)
            r = F.fdtd_energy_grad(s.h, 60, 20, p, [3, 7])
        out.append(r)
        s.close()
    assert out[0] == out[1]


# ------------------------------------------------- Sec. IV reimposition --
@pytest.mark.parametrize("dtype,N,par", [
    ("f32", 24, dict(z=2)), ("f32", 25, dict(x=2, y=1)), ("f64", 19, dict(x=1, y=2, z=2)),
    ("bf16", 32, dict(y=2)), ("bf16", 27, dict(x=2, z=1)), ("f32", 33, dict(x=1, y=1, z=1))])
def test_reimposition_of_a_state_without_the_symmetry_matches_the_oracle(dtype, N, par):
    """A noise state with no symmetry, the parity word recorded with it: after
    k steps evolve reimposes the symmetry.  A second handle runs the same k
    steps without it; the oracle's orc_reimpose of that state must equal the
    first handle's state bit for bit (copies and sign flips are exact), and
    the state must not already have had the symmetry."""
    say(f"case: reimpose {dtype} N={N} {par}")
    word = W.parity_word(**par)
    rng = np.random.default_rng(N)
    user = rng.uniform(-1, 1, (N, N, N))
    k = 6
    runs = []
    for p in (word, 0):
        s = Solver(N, 10.0, dtype=dtype)
        s.set_potential(F.POT_HO, [1.0, 1.1, 0.9])
        F.fdtd_set_initial(s.h, 0, F.INIT_USER, 0, p, user.ctypes.data, F.F64, 0)
        s.evolve(k, reimpose_parity_every=k, use_graph=False)
        runs.append(s.state())
        s.close()
    got, plain = runs
    if dtype == "bf16":
        to64 = lambda u: (u.astype(np.uint32) << 16).view(np.float32).astype(np.float64)
        ref = orc.reimpose(to64(plain), word)
        assert np.array_equal(to64(got), ref)
    else:
        ref = orc.reimpose(plain.astype(np.float64), word)
        assert np.array_equal(got.astype(np.float64), ref)
    assert not np.array_equal(plain.astype(np.float64) if dtype != "bf16" else plain, got)
