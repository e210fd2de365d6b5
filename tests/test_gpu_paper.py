"""The paper's own setups on one GPU (Sec. VII), reached by the multi-
resolution chain of Sec. VI in FP32 with FP64 reductions, against the
energies the paper prints (tests/golden/paper_values.json, each with its
section).  Where a printed value is not reproduced the test checks what the
lattice must give instead (the exact level it approximates) and says so:
  * regulated Coulomb 512^3: E0 matches the printed -0.499; the first
    excited level converges to -0.12466 (0.27% from -1/8, by the A_z start
    and by projection alike), the paper prints -0.122 (2.4%, its snapshot
    estimate);
  * A_z on 256^3: E1 matches all five printed digits (-0.12507); the next
    odd level converges to -0.055451 (0.19% from -1/18), the paper prints
    -0.055360;
  * dodecahedron (regular solid; the printed vertex list has one family with
    two coordinates exchanged): NOT reproduced.  The lattice levels are
    -99.857 / -99.710 on 128^3 and -99.991 on 512^3; the paper prints
    -99.78 / -99.55 / -99.97.  A run from noise stopped by the paper's own
    rule (binding energy changing by less than a part in 10^6 per 100
    steps) ends within a few thousandths of the converged level, so the
    stop rule does not account for the gap at 128^3.  The tests check what
    the lattice must satisfy instead: the stop rule's energy against the
    converged level, and the inverse-square scaling of the level above the
    well bottom between the 128^3 and 512^3 solids (same spacing, sides
    127 a and 511 a)."""
import json
import os
import sys

import pytest

pytestmark = pytest.mark.gpu

from paper_0904_0939_amd import fdtd as F  # noqa: E402
from paper_0904_0939_amd import workloads as W  # noqa: E402
from paper_0904_0939_amd.solver import multires  # noqa: E402

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")))


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def test_ho_512_ground_state():
    g = GOLD["ho_512"]
    s, log = multires((128, 256, 512), g["L"], F.POT_HO, [1, 1, 1], ["f32"] * 3, seed=13,
                      rel_tol=(1e-6, 1e-6, 1e-9), dt_over_a2=0.25)
    e = s.observables()[0]["energy"]
    say(f"HO 512^3: E0 = {e:.7f} (paper {g['E0']}) {log}")
    assert all(c for _, _, c in log)
    assert abs(e - g["E0"]) <= 5e-6  # the printed six digits


def test_coulomb_512_ground_and_first_excited():
    g = GOLD["coulomb_512"]
    L, a = g["L"], g["a"]
    args = dict(dt_over_a2=0.25, v_inf=1.0 / a, rel_tol=(1e-6, 1e-6, 1e-8))
    s0, log0, kept = multires((128, 256, 512), L, F.POT_COULOMB_REG, [1.0], ["f32"] * 3, seed=11,
                              keep=True, **args)
    e0 = s0.observables()[0]["binding"]
    s0.close()
    say(f"Coulomb 512^3: E0 = {e0:.6f} (paper {g['E0']}) {log0}")
    assert abs(e0 - g["E0"]) <= 5e-4  # the printed three decimals
    sz, logz = multires((128, 256, 512), L, F.POT_COULOMB_REG, [1.0], ["f32"] * 3, seed=11,
                        parity=W.parity_word(z=2), **args)
    e1z = sz.observables()[0]["binding"]
    sz.close()
    sp, logp = multires((128, 256, 512), L, F.POT_COULOMB_REG, [1.0], ["f32"] * 3, seed=21,
                        project={N: [kept[N]] for N in kept}, **args)
    e1p = sp.observables()[0]["binding"]
    sp.close()
    say(f"  E1 = {e1z:.6f} (A_z start), {e1p:.6f} (ground state projected out); paper {g['E1']}")
    assert abs(e1z + 0.125) < 0.005 * 0.125
    assert abs(e1p - e1z) < 1e-4 * abs(e1z)


def test_coulomb_az_256_first_and_second_odd_levels():
    g = GOLD["coulomb_az_256"]
    L = g["L"]
    args = dict(dt_over_a2=0.25, v_inf=1.0 / g["a"], rel_tol=(1e-6, 1e-6, 1e-8),
                parity=W.parity_word(z=2))
    s1, log1, kept = multires((64, 128, 256), L, F.POT_COULOMB_REG, [1.0], ["f32"] * 3, seed=12,
                              keep=True, **args)
    e1 = s1.observables()[0]["binding"]
    s1.close()
    s2, log2 = multires((64, 128, 256), L, F.POT_COULOMB_REG, [1.0], ["f32"] * 3, seed=22,
                        project={N: [kept[N]] for N in kept}, max_steps=(60000,), **args)
    e2 = s2.observables()[0]["binding"]
    s2.close()
    say(f"A_z 256^3: E1 = {e1:.7f} (paper {g['E1']}), E2 = {e2:.7f} (paper {g['E2']}) {log2}")
    assert abs(e1 - g["E1"]) <= 5e-6  # all five printed digits
    assert abs(e2 + 1.0 / 18.0) < 0.003 / 18.0


def test_coulomb_multires_to_1024():
    g = GOLD["coulomb_multires_1024"]
    s, log = multires((128, 256, 512, 1024), g["L"], F.POT_COULOMB_REG, [1.0], ["f32"] * 4,
                      seed=11, dt_over_a2=0.25, v_inf=1.0 / g["a"],
                      rel_tol=(1e-6,))
    e = s.observables()[0]["binding"]
    s.close()
    say(f"Coulomb 1024^3: E0 = {e:.7f} (paper {g['E0']}) {log}")
    assert abs(e - g["E0"]) < 1e-4


def _stop_rule_run(g, parity, seed=14):
    """128^3 from noise, no multi-resolution, FP32 with FP64 reductions:
    stopped by the paper's rule (check every 100 steps, binding energy
    changed by at most 1e-6 of itself), then carried on to a change below
    1e-9 of itself (the converged level, to about 1e-5)."""
    from paper_0904_0939_amd.solver import Solver

    s = Solver(g["N"], g["N"] * g["a"], dt=g["dt"], dtype="f32")
    s.set_potential(F.POT_DODECA, [-100.0])
    s.set_initial(seed, parity=parity)
    done, conv = s.evolve(400000, check_every=100, rel_tol=1e-6)
    e_stop = s.observables()[0]["binding"]
    more, conv2 = s.evolve(400000, check_every=100, rel_tol=1e-9)
    e_conv = s.observables()[0]["binding"]
    s.close()
    return done, conv, e_stop, done + more, conv2, e_conv


def test_dodecahedron_128_with_the_papers_stop_rule():
    """The paper's 128^3 run (a = 0.1, dt = 0.001) stopped by its own
    criterion.  Relaxation approaches a level from above, and the stop rule
    leaves E - E_level of about 1e-4 / (2 gap x 0.1) ~ 3e-3 for a gap of
    0.15: the stop energy lies above the converged level by less than 0.01.
    The printed -99.78 / -99.55 are not reproduced (logged)."""
    g = GOLD["dodecahedron_128"]
    conv = {}
    for name, par, printed in (("E0", 0, g["E0"]), ("E1", W.parity_word(z=2), g["E1"])):
        n1, c1, e_stop, n2, c2, e_conv = _stop_rule_run(g, par)
        say(f"dodecahedron 128^3 {name}: stop rule at step {n1}: {e_stop:.6f}; converged at "
            f"step {n2}: {e_conv:.6f}; paper {printed} (not reproduced)")
        assert c1 and c2
        assert -100.0 < e_conv <= e_stop + 1e-5
        assert e_stop - e_conv < 0.01
        conv[name] = e_conv
    # the odd start converges to a level above the ground state
    assert conv["E0"] < conv["E1"]


def test_dodecahedron_level_scales_with_the_inverse_square_of_the_size():
    """The solid spans the lattice (u = -1 at the first site, 1 at the last),
    so at one spacing a the 512^3 solid is (511/127) times the 128^3 one.
    For a well this deep (penetration 1/sqrt(200) ~ 0.07 against inradii of
    5.4 and 21.7) the level above the bottom, E + 100, scales as the inverse
    square of the size to within a few per cent.  Both lattices: FP32
    multi-resolution chains converged to 1e-9 per 100 steps."""
    out = {}
    for key, levels in (("dodecahedron_128", (32, 64, 128)), ("dodecahedron_512", (128, 256, 512))):
        g = GOLD[key]
        L = g["N"] * g["a"]
        s, log = multires(levels, L, F.POT_DODECA, [-100.0], ["f32"] * 3, seed=14,
                          dt_over_a2=g["dt"] / g["a"] ** 2, rel_tol=(1e-9,),
                          max_steps=(60000,))
        out[key] = s.observables()[0]["energy"]
        s.close()
        say(f"{key}: E0 = {out[key]:.6f} (paper {g['E0']}, not reproduced) {log}")
    ratio = (out["dodecahedron_512"] + 100.0) / (out["dodecahedron_128"] + 100.0)
    expect = (127.0 / 511.0) ** 2
    say(f"(E + 100) ratio 512 / 128: {ratio:.5f}; inverse square of the size {expect:.5f}")
    assert abs(ratio / expect - 1.0) < 0.05
