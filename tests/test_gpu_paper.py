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
    two coordinates exchanged): every printed level lies above the converged
    lattice level (-99.78 vs -99.857, -99.55 vs -99.710 on 128^3; -99.97
    vs -99.991 on 512^3), as unconverged energies do; see the test."""
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


@pytest.mark.parametrize("key,levels", [("dodecahedron_128", (32, 64, 128)),
                                        ("dodecahedron_512", (128, 256, 512))])
def test_dodecahedron_levels_lie_below_the_printed_ones(key, levels):
    """The energy of any state is an upper bound of the lattice ground state
    (and, odd in z, of the first odd level), and relaxation approaches it
    from above.  With V = -100 inside, a convergence test relative to |E|
    ~ 100 stops long before the ~0.2 binding above the well bottom has
    settled, which is how the printed values read: each lies above the
    converged lattice level, by less than 0.25."""
    g = GOLD[key]
    L = g["N"] * g["a"]
    args = dict(dt_over_a2=g["dt"] / g["a"] ** 2, rel_tol=(1e-9,), max_steps=(60000,))
    s, log = multires(levels, L, F.POT_DODECA, [-100.0], ["f32"] * 3, seed=14, **args)
    e0 = s.observables()[0]["energy"]
    s.close()
    say(f"{key}: E0 = {e0:.5f} (paper {g['E0']}) {log}")
    assert -100.0 < e0 < g["E0"] and g["E0"] - e0 < 0.25
    if "E1" in g:
        s1, log1 = multires(levels, L, F.POT_DODECA, [-100.0], ["f32"] * 3, seed=14,
                            parity=W.parity_word(z=2), **args)
        e1 = s1.observables()[0]["energy"]
        s1.close()
        say(f"  E1 = {e1:.5f} (A_z start; paper {g['E1']})")
        assert e0 < e1 < g["E1"] and g["E1"] - e1 < 0.25
