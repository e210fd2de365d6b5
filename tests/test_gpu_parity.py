"""GPU parity: the HIP path through the C ABI against the FP64 CPU oracle on
the same seeded inputs.  Tolerances:
  * FP64 path: energies within 1e-10 relative, states within 1e-10 of max|psi|;
  * FP32 path: energies within 1e-5 relative, normalised states within 1e-5
    relative L2 (FP32 rounding of ~6e-8 per step, damped by the relaxation);
  * BF16 storage: the raw BF16 level is reported against the 2^-9 rounding
    floor (about 2e-3 relative L2 for a smooth state) and gated at 1e-3 L2
    only after an FP32 finish;
  * integer outputs (steps done, converged flags) exactly; parity and
    launch-shape invariance bit for bit.
"""
import math
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


def bf16_round(x):
    """Round float64 values to bfloat16 (nearest even) on the CPU, via float32."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    return (u.astype(np.uint32) << 16).view(np.float32).astype(np.float64)


def bf16_bits_to_f64(u16):
    return (np.asarray(u16, dtype=np.uint32) << 16).view(np.float32).astype(np.float64)


def gpu_run(N, L, dtype, kind, params, seed, steps, parity=0, renorm=1, tuning=None, graph=True,
            dt_over=0.125, check_every=0, rel_tol=0.0):
    s = Solver(N, L, dtype=dtype, dt_over_a2=dt_over)
    if tuning:
        s.set_tuning(*tuning)
    s.set_potential(kind, params)
    s.set_initial(seed, parity=parity)
    done, conv = s.evolve(steps, renorm_every=renorm, use_graph=graph, check_every=check_every,
                          rel_tol=rel_tol)
    return s, done, conv


def oracle_run(N, L, kind, params, seed, steps, parity=0, dt_over=0.125, renorm=1,
               check_every=0, rel_tol=0.0, psi0=None):
    a = L / N
    V = orc.potential(kind, params, N, L)
    psi = orc.initial(N, seed, parity=parity) if psi0 is None else psi0.copy()
    done, conv, hist = orc.evolve(psi, V, L, dt_over * a * a, steps, renorm_every=renorm,
                                  check_every=check_every, rel_tol=rel_tol)
    return psi, V, done, conv, hist


# --------------------------------------------------------------- FP64 path --
def test_fp64_ho_32cubed_3000_steps():
    """Oscillator r^2/2 on 32^3, L = 10, dt = a^2/8, uniform noise, 3000 steps,
    renormalised every step; expected ground state near 1.5."""
    say("case: fp64 ho 32^3 3000 steps")
    N, L, seed, T = 32, 10.0, 1, 3000
    s, done, _ = gpu_run(N, L, "f64", F.POT_HO, [1, 1, 1], seed, T)
    assert done == T
    ob = s.observables()[0]
    psi_o, V, *_ = oracle_run(N, L, orc.POT_HO, [1, 1, 1], seed, T)
    oo = orc.observables(psi_o, V, L)
    assert ob["energy"] == pytest.approx(oo["energy"], rel=1e-10)
    assert ob["r_rms"] == pytest.approx(oo["r_rms"], rel=1e-10)
    assert ob["kinetic"] == pytest.approx(oo["kinetic"], rel=1e-10)
    assert abs(ob["energy"] - 1.5) < 0.01
    g = s.psi()
    assert np.max(np.abs(g - psi_o)) < 1e-10 * np.max(np.abs(psi_o))
    assert ob["step"] == T


def test_fp64_history_matches_oracle_energies_step_by_step():
    say("case: fp64 history 20^3")
    N, L, seed = 20, 8.0, 3
    s, *_ = gpu_run(N, L, "f64", F.POT_CORNELL, W.CORNELL_PARAMS, seed, 60)
    hist = s.history(0, 100)
    assert [h["step"] for h in hist] == list(range(60))
    V = orc.potential(orc.POT_CORNELL, W.CORNELL_PARAMS, N, L)
    psi = orc.initial(N, seed)
    a = L / N
    for t in range(60):
        e = orc.observables(psi, V, L)["energy"]
        assert hist[t]["energy"] == pytest.approx(e, rel=1e-11), t
        psi = orc.normalized(orc.step(psi, V, L, a * a / 8), L)


def test_fp64_convergence_stop_matches_oracle_exactly():
    say("case: fp64 convergence 16^3")
    N, L, seed = 16, 8.0, 2
    s, done, conv = gpu_run(N, L, "f64", F.POT_HO, [1, 1, 1], seed, 20000, check_every=50,
                            rel_tol=1e-9)
    _, _, odone, oconv, _ = oracle_run(N, L, orc.POT_HO, [1, 1, 1], seed, 20000, check_every=50,
                                       rel_tol=1e-9)
    assert conv and oconv and done == odone


# --------------------------------------------------------------- FP32 path --
@pytest.mark.parametrize("N", [36, 100])
def test_fp32_cornell_several_tiles_and_ragged_tail(N):
    """N = 100: the (y, z) plane of 10^4 sites spans five work items of 2048
    with a ragged last one; N = 36 fits one.  Cornell -0.4/r + 0.2 r + 0.05 z^2."""
    say(f"case: fp32 cornell {N}^3")
    L, seed, T = 30.0 * N / 128, 7, 300
    s, *_ = gpu_run(N, L, "f32", F.POT_CORNELL, W.CORNELL_PARAMS, seed, T)
    ob = s.observables()[0]
    psi_o, V, *_ = oracle_run(N, L, orc.POT_CORNELL, W.CORNELL_PARAMS, seed, T)
    oo = orc.observables(psi_o, V, L)
    assert ob["energy"] == pytest.approx(oo["energy"], rel=1e-5)
    assert ob["r_rms"] == pytest.approx(oo["r_rms"], rel=1e-5)
    assert rel_l2(s.psi(), psi_o) < 1e-5


def test_fp32_coulomb_even_and_odd_starts():
    """Coulomb -1/r from the same noise made S_z (even) and A_z (odd)."""
    say("case: fp32 coulomb even/odd 40^3")
    N, L, T = 40, 12.5, 400
    for par in (W.parity_word(z=1), W.parity_word(z=2)):
        s, *_ = gpu_run(N, L, "f32", F.POT_COULOMB, [1.0], 2, T, parity=par)
        psi_o, V, *_ = oracle_run(N, L, orc.POT_COULOMB, [1.0], 2, T, parity=par)
        assert s.observables()[0]["energy"] == pytest.approx(orc.observables(psi_o, V, L)["energy"], rel=1e-5)
        assert rel_l2(s.psi(), psi_o) < 1e-5


@pytest.mark.parametrize("tuning", [(4, 1, 8, 0, 0, 1), (4, 2, 16, 0, 1, 2), (4, 2, 72, 0, 1, 3),
                                    (1, 1, 13, 0, 0, 1), (1, 4, 5, 37, 1, 1), (4, 2, 7, 64, 1, 3),
                                    (4, 1, 0, 0, 1, 2), (4, 2, 11, 0, 0, 1),
                                    (4, 1, 0, 0, 1, 1, 1), (4, 1, 7, 0, 1, 2, 1), (4, 1, 13, 3, 1, 3, 1),
                                    (4, 1, 9, 0, 1, 3, 2), (1, 1, 10, 0, 1, 1, 2),
                                    (4, 2, 0, 0, 1, 1, 3), (4, 1, 9, 0, 0, 2, 3)])
def test_fp32_state_is_independent_of_launch_shape(tuning):
    """Without renormalisation the update of a site does not depend on the
    tiling, so every launch shape yields the same bits."""
    say(f"case: fp32 tiling {tuning}")
    N, L = 72, 12.0
    ref, *_ = gpu_run(N, L, "f32", F.POT_WELLS, W.random_wells(np.random.default_rng(1)), 5, 25,
                      renorm=0, tuning=(4, 2, 32, 0, 1, 2))
    s, *_ = gpu_run(N, L, "f32", F.POT_WELLS, W.random_wells(np.random.default_rng(1)), 5, 25,
                    renorm=0, tuning=tuning)
    assert np.array_equal(s.state(), ref.state())


def test_reductions_agree_across_work_item_counts():
    """Each work item hands its partial sums to the member's last work-group
    inside the launch.  With a rescale every step the state depends on every
    step's sums, so a partial read before it landed would show at once: the
    histories of launch shapes with 18 to 1152 work items per step (and a grid
    smaller than the item count) must agree to FP32 grouping rounding, and
    the result must match the oracle."""
    say("case: reductions across work-item counts")
    N, L, T = 96, 12.0, 300
    params = W.random_wells(np.random.default_rng(2))
    runs, final = [], []
    for tun in [(4, 2, 0, 0, 1, 1), (4, 1, 4, 0, 1, 2), (4, 2, 8, 7, 0, 1), (4, 1, 2, 0, 1, 1, 3)]:
        s, *_ = gpu_run(N, L, "f32", F.POT_WELLS, params, 8, T, tuning=tun)
        runs.append(s.history(0, T))
        final.append(s.observables()[0]["energy"])
        s.close()
    for h in runs[1:]:
        for a, b in zip(h, runs[0]):
            assert a["step"] == b["step"]
            assert a["energy"] == pytest.approx(b["energy"], rel=1e-6), a["step"]
            assert a["norm2"] == pytest.approx(b["norm2"], rel=1e-6), a["step"]
    assert final[1:] == pytest.approx([final[0]] * 3, rel=1e-6)
    psi, V, *_ = oracle_run(N, L, orc.POT_WELLS, params, 8, T)
    assert final[0] == pytest.approx(orc.observables(psi, V, L)["energy"], rel=1e-5)


@pytest.mark.parametrize("N,tunings", [
    (40, [(8, 1, 0, 0, 1, 2), (8, 1, 5, 0, 0, 1), (8, 1, 3, 0, 1, 3), (1, 4, 9, 0, 1, 1),
          (1, 1, 0, 0, 1, 1), (8, 1, 0, 0, 1, 1, 1), (1, 1, 7, 0, 1, 1, 2), (8, 1, 0, 0, 1, 2, 3)]),
    (42, [(1, 1, 0, 0, 1, 1), (1, 4, 0, 0, 1, 1), (1, 2, 3, 0, 0, 1)]),
    (45, [(1, 1, 0, 0, 1, 1), (1, 2, 4, 0, 1, 1), (1, 4, 0, 11, 0, 1)])])
def test_bf16_state_is_independent_of_launch_shape_and_keeps_parity(N, tunings):
    """The stochastic rounding of a BF16 store draws its bits from the site's
    mirror-canonical index and the step only: without renormalisation (whose
    FP64 sums are grouped by the tiling) every launch shape stores the same
    bits, and an odd start stays odd bit for bit.  N = 42 puts a z-pair of
    the shared hash across the centre; N = 45 takes one hash per site."""
    say(f"case: bf16 tiling N={N}")
    L = 12.0
    par = W.parity_word(z=2, y=1)
    # odd N puts a site at r = 0, where the Cornell potential is infinite
    kind, params = (F.POT_CORNELL, W.CORNELL_PARAMS) if N % 2 == 0 else (F.POT_HO, [1, 1.2, 0.8])
    states = []
    for t in tunings:
        # the V table for every shape: the LDS-tile and 512-lane variants read it
        t = tuple(t) + (0,) * (7 - len(t)) + (0, 0)
        s, *_ = gpu_run(N, L, "bf16", kind, params, 9, 40, tuning=t, parity=par, renorm=0)
        states.append(s.state())
        s.close()
    v = bf16_bits_to_f64(states[0])
    assert np.abs(v).max() > 0
    assert np.array_equal(v[:, :, ::-1], -v)
    assert np.array_equal(v[:, ::-1, :], v)
    for t, st in zip(tunings[1:], states[1:]):
        assert np.array_equal(st, states[0]), t


@pytest.mark.parametrize("dtype,variant", [("f64", 1), ("f64", 2), ("bf16", 1), ("f32", 1), ("f64", 3)])
def test_large_group_variants_against_oracle(dtype, variant):
    """The LDS-tile, 512-lane and written-through-store variants of the fused
    step against the oracle (N = 104: several chunks, ragged tail, halo rows
    crossing chunks)."""
    say(f"case: variant {variant} {dtype}")
    N, L, T = 104, 20.0, 200
    vz = {"f64": 2, "f32": 4, "bf16": 8}[dtype]
    tun = (vz, 1, 0, 0, 1, 1, variant)
    s, *_ = gpu_run(N, L, dtype, F.POT_CORNELL, W.CORNELL_PARAMS, 5, T, tuning=tun,
                    parity=W.parity_word(z=2))
    psi_o, V, *_ = oracle_run(N, L, orc.POT_CORNELL, W.CORNELL_PARAMS, 5, T,
                              parity=orc.parity_word(z=2))
    e = orc.observables(psi_o, V, L)["energy"]
    tol = {"f64": 1e-10, "f32": 1e-5, "bf16": 5e-3}[dtype]
    assert s.observables()[0]["energy"] == pytest.approx(e, rel=tol)
    v = s.state()
    v = bf16_bits_to_f64(v) if dtype == "bf16" else v
    assert np.array_equal(v[:, :, ::-1], -v)


def test_graph_replay_equals_direct_launches():
    say("case: graph vs direct 48^3")
    N, L = 48, 10.0
    a, *_ = gpu_run(N, L, "f32", F.POT_HO, [1, 1.2, 0.8], 4, 256, graph=True, check_every=64, rel_tol=0)
    b, *_ = gpu_run(N, L, "f32", F.POT_HO, [1, 1.2, 0.8], 4, 256, graph=False, check_every=64, rel_tol=0)
    assert np.array_equal(a.state(), b.state())
    ha, hb = a.history(0, 256), b.history(0, 256)
    assert [h["energy"] for h in ha] == [h["energy"] for h in hb]


@pytest.mark.parametrize("dtype", ["f64", "f32", "bf16"])
def test_odd_parity_is_preserved_bit_for_bit(dtype):
    say(f"case: parity {dtype}")
    N, L = 48, 12.0
    s, *_ = gpu_run(N, L, dtype, F.POT_CORNELL, W.CORNELL_PARAMS, 6, 300,
                    parity=W.parity_word(z=2, x=1))
    st = s.state()
    if dtype == "bf16":
        v = bf16_bits_to_f64(st)
    else:
        v = st.astype(np.float64)
    assert np.array_equal(v[:, :, ::-1], -v)
    assert np.array_equal(v[::-1, :, :], v)
    assert np.abs(v).max() > 0


def test_odd_lattice_side_scalar_lanes_and_zero_midplane():
    say("case: odd N 45 A_x")
    N, L = 45, 9.0
    s, *_ = gpu_run(N, L, "f32", F.POT_HO, [1, 1, 1], 8, 200, parity=W.parity_word(x=2))
    assert s.tuning()["vz"] == 1
    v = s.state()
    assert not v[N // 2].any()
    assert np.array_equal(v[::-1], -v)
    psi_o, V, *_ = oracle_run(N, L, orc.POT_HO, [1, 1, 1], 8, 200, parity=orc.parity_word(x=2))
    assert rel_l2(s.psi(), psi_o) < 1e-5


def test_reimposed_parity_keeps_state_exact():
    N, L = 32, 10.0
    s, *_ = gpu_run(N, L, "f32", F.POT_HO, [1, 1, 1], 1, 64, parity=W.parity_word(y=2))
    s.evolve(100, reimpose_parity_every=10)
    v = s.state()
    assert np.array_equal(v[:, ::-1, :], -v)


# --------------------------------------------------------------- BF16 path --
def test_bf16_level_then_fp32_finish():
    """BF16 storage (FP32 math) on 64^3, then the state moves to an FP32
    lattice for a finish; the finished state meets 1e-3 L2 and 1e-5 energy."""
    say("case: bf16 64^3 then fp32 finish")
    N, L, seed = 64, 10.0, 9
    T1, T2 = 1500, 600
    b, *_ = gpu_run(N, L, "bf16", F.POT_HO, [1, 1, 1], seed, T1)
    psi_o, V, *_ = oracle_run(N, L, orc.POT_HO, [1, 1, 1], seed, T1)
    raw = rel_l2(b.psi(), psi_o)
    say(f"bf16 level: relative L2 vs oracle {raw:.3e}")
    assert raw < 1e-2
    f = Solver(N, L, dtype="f32")
    f.set_potential(F.POT_HO, [1, 1, 1])
    f.set_initial_array(b.psi_tensor(0, dtype=__import__("torch").float32))
    f.evolve(T2)
    psi_o2 = psi_o.copy()
    orc.evolve(psi_o2, V, L, (L / N) ** 2 / 8, T2)
    fin = rel_l2(f.psi(), psi_o2)
    say(f"after fp32 finish: relative L2 {fin:.3e}")
    assert fin < 1e-3
    assert f.observables()[0]["energy"] == pytest.approx(orc.observables(psi_o2, V, L)["energy"], rel=1e-5)


# ------------------------------------------------------------- upsample ----
def test_upsample_fp64_dyadic_and_general_ratio():
    say("case: upsample fp64")
    L = 9.0
    for Nc, Nf in ((16, 32), (24, 40)):
        c = Solver(Nc, L, dtype="f64")
        c.set_potential(F.POT_HO, [1, 1, 1])
        c.set_initial(11)
        f = Solver(Nf, L, dtype="f64")
        f.set_potential(F.POT_HO, [1, 1, 1])
        F.fdtd_upsample(c.h, 0, f.h, 0)
        ref = orc.upsample(orc.initial(Nc, 11), Nf, L)
        np.testing.assert_allclose(f.psi(), ref, rtol=0, atol=1e-12 * np.abs(ref).max())
        assert f.observables()[0]["step"] == 0


@pytest.mark.parametrize("Nc,cd,Nf,fd", [(33, "f64", 65, "f64"), (50, "f64", 77, "f64"),
                                         (40, "f64", 24, "f64"), (31, "bf16", 62, "f64"),
                                         (26, "f32", 45, "f32"), (40, "bf16", 90, "f64"),
                                         (34, "bf16", 100, "f32"), (2, "bf16", 9, "f64"),
                                         (26, "f32", 52, "f64"), (20, "bf16", 40, "bf16"),
                                         (2, "f64", 4, "f32"), (18, "f64", 36, "bf16"),
                                         (35, "f32", 70, "f32")])
def test_upsample_ragged_sides_and_coarser_targets(Nc, cd, Nf, fd):
    """Fine sides that are not a multiple of the kernel's 4-site vectors,
    non-integer ratios, a target coarser than the source (several coarse
    planes between two fine ones), BF16 sources of even side under fine
    sides of at least twice theirs (the coarse rows read as site pairs), and
    exact doublings of even sides (the dedicated 2x kernel, every storage
    type; 35 -> 70 is odd and takes the general kernel)."""
    say(f"case: upsample {Nc} {cd} -> {Nf} {fd}")
    L = 9.0
    c = Solver(Nc, L, dtype=cd)
    c.set_potential(F.POT_HO, [1, 1, 1])
    c.set_initial(13)
    f = Solver(Nf, L, dtype=fd)
    f.set_potential(F.POT_HO, [1, 1, 1])
    F.fdtd_upsample(c.h, 0, f.h, 0)
    coarse = orc.initial(Nc, 13)
    if cd == "bf16":
        coarse = bf16_round(coarse)
    elif cd == "f32":
        coarse = coarse.astype(np.float32).astype(np.float64)
    ref = orc.upsample(coarse, Nf, L)
    # BF16 fine storage: the interpolated values rounded once to 8 bits (2^-9)
    tol = {"f64": 1e-12, "f32": 1e-6, "bf16": 2.0 ** -8}[fd]
    np.testing.assert_allclose(f.psi(), ref, rtol=0, atol=tol * np.abs(ref).max())
    c.close()
    f.close()


@pytest.mark.parametrize("Nc,Nf,L,dtype", [(64, 128, 51.2, "f32"), (40, 90, 9.3, "f64"),
                                          (33, 66, 7.7, "f32"), (48, 96, 51.2, "bf16")])
def test_upsample_keeps_odd_states_odd_bit_for_bit_at_any_spacing(Nc, Nf, L, dtype):
    """Spacings that are not dyadic fractions (a = 0.8 -> 0.4, ...): the
    fine-to-coarse map is taken at the mirror-canonical index, so mirrored
    fine sites add the same two products and an odd state stays exactly
    odd (a last-bit asymmetry would seed the even ground state, which then
    grows during an odd-state relaxation)."""
    say(f"case: upsample antisymmetry {Nc}->{Nf} L={L} {dtype}")
    par = W.parity_word(z=2)
    c = Solver(Nc, L, dtype=dtype)
    c.set_potential(F.POT_HO, [1, 1, 1])
    c.set_initial(17, parity=par)
    c.evolve(20)
    f = Solver(Nf, L, dtype="f32" if dtype == "bf16" else dtype)
    f.set_potential(F.POT_HO, [1, 1, 1])
    F.fdtd_upsample(c.h, 0, f.h, 0)
    v = f.state()
    assert np.array_equal(v[:, :, ::-1], -v)
    c.close()
    f.close()


def test_upsample_from_bf16_and_parity():
    say("case: upsample bf16 -> f32")
    Nc, Nf, L = 32, 64, 10.0
    par = W.parity_word(z=2)
    c = Solver(Nc, L, dtype="bf16")
    c.set_potential(F.POT_HO, [1, 1, 1])
    c.set_initial(12, parity=par)
    f = Solver(Nf, L, dtype="f32")
    f.set_potential(F.POT_HO, [1, 1, 1])
    F.fdtd_upsample(c.h, 0, f.h, 0)
    coarse = bf16_round(orc.initial(Nc, 12, parity=orc.parity_word(z=2)))
    ref = orc.upsample(coarse, Nf, L)
    assert rel_l2(f.psi(), ref) < 1e-6
    v = f.state()
    assert np.array_equal(v[:, :, ::-1], -v)


# ---------------------------------------------------------------- batch ----
def test_batch_of_uneven_lattices_fp64():
    say("case: batch fp64")
    rng = np.random.default_rng(21)
    lats = [W.Lattice(N, 12.0, W.POT_WELLS, W.random_wells(rng), seed=3) for N in (8, 12, 20, 24, 16)]
    b = Batch(lats, dtype="f64")
    for m, l in enumerate(lats):
        b.set_potential(l.pot_kind, l.pot_params, member=m)
    b.set_initial(3)
    b.evolve(200)
    obs = b.observables()
    for m, l in enumerate(lats):
        V = orc.potential(orc.POT_WELLS, l.pot_params, l.N, l.L)
        psi = orc.initial(l.N, 3, member=m)
        orc.evolve(psi, V, l.L, l.dt, 200)
        assert obs[m]["energy"] == pytest.approx(orc.observables(psi, V, l.L)["energy"], rel=1e-10), m
        np.testing.assert_allclose(b.psi(m), psi, rtol=0, atol=1e-10 * np.abs(psi).max())


def test_batch_fp32_matches_single_lattice_runs_bitwise():
    """Members of a batch step exactly as they would alone (renorm off).  The
    batch's noise is the oracle's, member by member, bit for bit (FP32
    storage); each single run starts from a copy of its member's GPU start."""
    say("case: batch fp32 vs singles")
    rng = np.random.default_rng(5)
    lats = [W.Lattice(N, 12.0, W.POT_WELLS, W.random_wells(rng), seed=4) for N in (48, 64, 96, 32)]
    b = Batch(lats, dtype="f32")
    for m, l in enumerate(lats):
        b.set_potential(l.pot_kind, l.pot_params, member=m)
    b.set_initial(4)
    starts = [b.state(m) for m in range(len(lats))]
    for m, l in enumerate(lats):
        assert np.array_equal(starts[m], orc.initial(l.N, 4, member=m).astype(np.float32)), m
    b.evolve(40, renorm_every=0)
    obs = b.observables()
    for m, l in enumerate(lats):
        s = Solver(l.N, l.L, dtype="f32")
        s.set_potential(l.pot_kind, l.pot_params)
        s.set_initial_array(starts[m])
        s.evolve(40, renorm_every=0)
        assert np.array_equal(s.state(), b.state(m)), m
        V = orc.potential(orc.POT_WELLS, l.pot_params, l.N, l.L)
        psi = orc.initial(l.N, 4, member=m)
        orc.evolve(psi, V, l.L, l.dt, 40, renorm_every=0)
        assert obs[m]["energy"] == pytest.approx(orc.observables(psi, V, l.L)["energy"], rel=1e-5), m


# ------------------------------------------------------------- gradient ----
def test_gradient_fp64_matches_oracle_adjoint():
    say("case: gradient fp64 10^3")
    N, L, T, k = 10, 8.0, 30, 7
    p = [1.0, 1.0, 1.0, 1.5, 0.3, 0.0, -0.2, 0.8, 0.7, -1.0, 0.5, 0.2, 1.1]
    s = Solver(N, L, dtype="f64")
    s.set_potential(F.POT_WELLS, p)
    s.set_initial(13)
    wrt = [3, 7, 8, 12]
    E, g, G = s.energy_grad(T, k, theta=p, wrt=wrt, want_field=True)
    V = orc.potential(orc.POT_WELLS, p, N, L)
    Eo, Go = orc.energy_grad_v(orc.initial(N, 13), V, L, (L / N) ** 2 / 8, T)
    assert E == pytest.approx(Eo, rel=1e-12)
    Gg = G.cpu().numpy()
    np.testing.assert_allclose(Gg, Go, rtol=0, atol=1e-9 * np.abs(Go).max())
    for j, gj in zip(wrt, g):
        assert gj == pytest.approx(float(np.sum(Go * orc.wells_dv(p, N, L, j))), rel=1e-9)
    assert s.observables()[0]["step"] == T


def test_gradient_fp32_matches_oracle_adjoint():
    say("case: gradient fp32 16^3")
    N, L, T, k = 16, 8.0, 50, 10
    p = [1.0, 1.0, 1.0, 1.5, 0.3, 0.0, -0.2, 0.8]
    s = Solver(N, L, dtype="f32")
    s.set_potential(F.POT_WELLS, p)
    s.set_initial(14)
    E, g, _ = s.energy_grad(T, k, theta=p, wrt=[3, 7])
    V = orc.potential(orc.POT_WELLS, p, N, L)
    Eo, Go = orc.energy_grad_v(orc.initial(N, 14), V, L, (L / N) ** 2 / 8, T)
    assert E == pytest.approx(Eo, rel=1e-5)
    for j, gj in zip([3, 7], g):
        assert gj == pytest.approx(float(np.sum(Go * orc.wells_dv(p, N, L, j))), rel=1e-4)


WELLS2 = [1.0, 0.8, 1.2, 2.0, 0.5, -0.3, 0.2, 0.9, 1.1, -1.0, 0.4, 0.0, 0.6]


@pytest.mark.parametrize("kind,params,N", [
    (F.POT_CONST, [0.3], 10),
    (F.POT_HO, [1.0, 1.3, 0.7], 11),
    (F.POT_COULOMB, [1.2], 10),
    (F.POT_COULOMB_REG, [0.9], 10),
    (F.POT_CORNELL, [0.4, 0.2, 0.05], 10),
    (F.POT_WELLS, WELLS2, 11),
    (F.POT_DODECA, [-5.0], 12),
])
def test_gradient_wrt_every_parameter_of_every_kind(kind, params, N):
    """dE/dtheta for every parameter of every analytic kind (FP64), against
    the oracle's dE/dV contracted with its own dV/dtheta."""
    say(f"case: gradient kind {kind} N={N}")
    L, T, k = 8.0, 30, 7
    s = Solver(N, L, dtype="f64")
    s.set_potential(kind, params)
    s.set_initial(15)
    wrt = list(range(len(params)))
    E, g, _ = s.energy_grad(T, k, theta=params, wrt=wrt)
    V = orc.potential(kind, params, N, L)
    Eo, Go = orc.energy_grad_v(orc.initial(N, 15), V, L, (L / N) ** 2 / 8, T)
    assert E == pytest.approx(Eo, rel=1e-12)
    ref = [float(np.sum(Go * orc.potential_dv(kind, params, N, L, j))) for j in wrt]
    scale = max(abs(r) for r in ref)
    for j, gj, rj in zip(wrt, g, ref):
        assert gj == pytest.approx(rj, rel=1e-9, abs=1e-12 * scale), j
    s.close()


def test_gradient_parameter_checks():
    say("case: gradient parameter checks")
    s = Solver(10, 8.0, dtype="f64")
    s.set_potential(F.POT_CORNELL, [0.4, 0.2, 0.05])
    s.set_initial(1)
    for theta, wrt in (([0.4, 0.2, 0.06], [0]),      # not the parameters V was set from
                       ([0.4, 0.2], [0]),            # too few
                       ([0.4, 0.2, 0.05], [3]),      # not a Cornell parameter
                       ([0.4, 0.2, 0.05], [-1])):
        with pytest.raises(F.FdtdError) as ei:
            s.energy_grad(5, 5, theta=theta, wrt=wrt)
        assert ei.value.status == F.EINVAL
    V = orc.potential(orc.POT_CORNELL, [0.4, 0.2, 0.05], 10, 8.0)
    s.set_potential_array(V)  # a caller's array: no parameters to contract with
    with pytest.raises(F.FdtdError):
        s.energy_grad(5, 5, theta=[0.4, 0.2, 0.05], wrt=[0])
    E, g, G = s.energy_grad(5, 5, want_field=True)  # dE/dV alone still works
    assert np.isfinite(E) and G is not None
    s.close()


@pytest.mark.parametrize("dtype,N", [("f64", 9), ("f32", 18), ("f32", 40), ("f64", 24)])
def test_gradient_field_matches_oracle_across_launch_shapes(dtype, N):
    """dE/dV site by site: scalar lanes (N not a multiple of the vector
    width), several chunks of the flattened plane with a ragged last one, and
    one x-range per plane (N = 40: 2 chunks x 40 ranges)."""
    say(f"case: gradient field {dtype} {N}^3")
    L, T, k = 8.0, 40, 9
    p = [1.0, 1.2, 0.9, 1.5, 0.3, 0.0, -0.2, 0.8, 0.7, -1.0, 0.5, 0.2, 1.1]
    s = Solver(N, L, dtype=dtype)
    s.set_potential(F.POT_WELLS, p)
    s.set_initial(15)
    E, g, G = s.energy_grad(T, k, theta=p, wrt=[3, 7], want_field=True)
    V = orc.potential(orc.POT_WELLS, p, N, L)
    Eo, Go = orc.energy_grad_v(orc.initial(N, 15), V, L, (L / N) ** 2 / 8, T)
    tol = 1e-9 if dtype == "f64" else 1e-4
    assert E == pytest.approx(Eo, rel=1e-12 if dtype == "f64" else 1e-5)
    np.testing.assert_allclose(G.cpu().numpy(), Go, rtol=0, atol=tol * np.abs(Go).max())
    for j, gj in zip([3, 7], g):
        assert gj == pytest.approx(float(np.sum(Go * orc.wells_dv(p, N, L, j))), rel=tol)


# ----------------------------------------------------------- error paths ----
@pytest.mark.parametrize("dtype,N", [("f64", 2), ("f64", 3), ("f32", 2), ("f32", 5), ("f32", 4),
                                     ("bf16", 2), ("bf16", 7)])
def test_smallest_lattices_against_oracle(dtype, N):
    """Lattices of a few sites per side: most neighbours are the zero ghosts,
    a lane's vector is partly or wholly outside the lattice, an odd side has
    its midplane site at the centre."""
    say(f"case: smallest lattice {dtype} N={N}")
    L, T, p = 4.0, 40, [1.0, 1.2, 0.8]
    s = Solver(N, L, dtype=dtype)
    s.set_potential(F.POT_HO, p)
    s.set_initial(5)
    s.evolve(T)
    ob = s.observables()[0]
    V = orc.potential(orc.POT_HO, p, N, L)
    psi = orc.initial(N, 5)
    orc.evolve(psi, V, L, (L / N) ** 2 / 8, T)
    e = orc.observables(psi, V, L)["energy"]
    assert ob["step"] == T
    if dtype == "bf16":
        # stochastically rounded 8-bit significands: the relaxation agrees
        # to the storage precision
        assert ob["energy"] == pytest.approx(e, rel=2e-2)
        return
    tol = {"f64": 1e-10, "f32": 1e-5}[dtype]
    assert ob["energy"] == pytest.approx(e, rel=tol)
    ref = orc.normalized(psi, L)
    np.testing.assert_allclose(s.psi(), ref, rtol=0, atol=tol * np.abs(ref).max())
    s.close()


def test_nonfinite_initial_state_is_reported():
    s = Solver(16, 8.0, dtype="f32")
    s.set_potential(F.POT_HO, [1, 1, 1])
    bad = np.zeros((16, 16, 16))
    bad[3, 4, 5] = np.nan
    with pytest.raises(F.FdtdError) as ei:
        s.set_initial_array(bad)
    assert ei.value.status == F.ENONFINITE
    with pytest.raises(F.FdtdError) as ei:
        s.set_initial_array(np.zeros((16, 16, 16)))
    assert ei.value.status == F.ENONFINITE
    s.set_initial(1)
    s.evolve(10)


def test_evolve_reports_nonfinite_potential():
    s = Solver(16, 8.0, dtype="f32")
    V = np.zeros((16, 16, 16))
    V[2, 2, 2] = np.inf
    s.set_potential_array(V)
    s.set_initial(1)
    with pytest.raises(F.FdtdError) as ei:
        s.evolve(5)
    assert ei.value.status == F.ENONFINITE
