"""Pins of the oracle's potentials, noise draw and symmetry operators that the
first pin file leaves open: the three terms of the Cornell-type potential
(benchmark configuration 3), the regulated Coulomb potential of
Eq. (coulombpot) (Sec. VII.C), the Box-Muller draw of the Gaussian start and
the Sec. IV reimposition.

Each pin compares the oracle with something other than its own formula: a
continuum limit (hydrogenic -p0^2/2, the Airy ground state of a linear
potential), exact separable lattice levels from a tridiagonal eigensolver,
the published SplitMix64 outputs pushed through the textbook Box-Muller map,
and plain numpy mirror copies.
"""
import math

import numpy as np
import pytest
import scipy.linalg as sla

import oracle as orc

AIRY_A1 = 2.338107410459767  # first zero of Ai(-x)


def relax(kind, p, N, L, dt_over_a2=0.125, parity=0, v_inf=0.0, tol=1e-9, steps=60000):
    """The oracle's relaxation from seeded noise to a change below tol per 100
    steps; returns its observables."""
    a = L / N
    V = orc.potential(kind, p, N, L)
    psi = orc.initial(N, 7, parity=parity)
    done, conv, _ = orc.evolve(psi, V, L, dt_over_a2 * a * a, steps, check_every=100,
                               rel_tol=tol, v_inf=v_inf)
    assert conv, f"no convergence in {done} steps"
    return orc.observables(psi, V, L, v_inf=v_inf)


def richardson(a1, e1, a2, e2, p):
    """Limit a -> 0 of e(a) = e0 + c a^p through two points."""
    return (e2 * a1**p - e1 * a2**p) / (a1**p - a2**p)


def level_1d(N, L, v_of_x, k, mass=1.0):
    """k-th eigenvalue of -1/(2m) d^2/dx^2 + v(x) on the N cell-centred sites of
    [-L/2, L/2] with zero ghosts: the tridiagonal second-difference operator."""
    a = L / N
    x = (2.0 * np.arange(N) - (N - 1)) * (0.5 * a)
    d = 1.0 / (mass * a * a) + v_of_x(x)
    e = -0.5 / (mass * a * a) * np.ones(N - 1)
    return sla.eigh_tridiagonal(d, e, eigvals_only=True)[k]


# ------------------------------------------------ Cornell-type potential --
def test_cornell_inverse_r_term_reaches_the_hydrogenic_level():
    """p = (p0, 0, 0) is the attractive -p0/r: its ground level tends to
    -p0^2 / 2 as a -> 0 (second order on this lattice).  A sign slip, a
    dropped p0 or a wrong term fails it."""
    p0, L = 2.0, 8.0
    res = [(L / N, relax(orc.POT_CORNELL, [p0, 0.0, 0.0], N, L)["energy"]) for N in (32, 48)]
    (a1, e1), (a2, e2) = res
    exact = -0.5 * p0 * p0
    assert exact < e2 < e1  # variational on the lattice, approaching from above
    assert abs(richardson(a1, e1, a2, e2, 2) / exact - 1.0) < 1e-2


def test_cornell_linear_term_reaches_the_airy_level():
    """p = (0, p1, 0) is the confining p1 r: the s-wave ground level of
    -u''/2m + p1 r u = E u with u(0) = 0 is (p1^2 / 2m)^(1/3) a1, a1 the first
    zero of Ai(-x).  Second-order convergence on the lattice; the
    extrapolation lands within 2e-4."""
    p1, L = 1.0, 12.0
    res = [(L / N, relax(orc.POT_CORNELL, [0.0, p1, 0.0], N, L)["energy"]) for N in (32, 48)]
    (a1, e1), (a2, e2) = res
    exact = (p1 * p1 / 2.0) ** (1.0 / 3.0) * AIRY_A1
    assert e1 < e2 < exact  # this lattice approaches the level from below
    assert abs(richardson(a1, e1, a2, e2, 2) / exact - 1.0) < 2e-4


def test_cornell_z2_term_gives_the_separable_lattice_levels():
    """p = (0, 0, p2) is V = p2 z^2, separable: the lattice levels are sums of
    a free Dirichlet level along x and y and an oscillator level along z
    (tridiagonal eigenvalues).  The even start relaxes to box(0) + box(0) +
    osc(0); the start made odd in z (A_z) to box(0) + box(0) + osc(1).  The
    readout sits above these by the O(dt^2) gap of the update's fixed point
    (checked: it shrinks 16x from dt = a^2/8 to a^2/32).  With z^2 exchanged
    for x^2 the odd-z level would be osc(0) + box(0) + box(1), 48% lower."""
    p2, N, L = 0.5, 20, 8.0
    box0 = level_1d(N, L, lambda x: 0.0 * x, 0)
    for k, parity in ((0, 0), (1, orc.parity_word(z=orc.PAR_A))):
        osc = level_1d(N, L, lambda x: p2 * x * x, k)
        exact = 2.0 * box0 + osc
        gaps = []
        for dto in (1.0 / 8.0, 1.0 / 32.0):
            e = relax(orc.POT_CORNELL, [0.0, 0.0, p2], N, L, dt_over_a2=dto, parity=parity,
                      tol=1e-13, steps=200000)["energy"]
            gaps.append(e / exact - 1.0)
        assert 0.0 < gaps[1] < 5e-6
        assert gaps[0] / gaps[1] == pytest.approx(16.0, rel=0.05)
    # the odd-z level tells the z axis from the x axis
    swapped = level_1d(N, L, lambda x: p2 * x * x, 0) + box0 + level_1d(N, L, lambda x: 0.0 * x, 1)
    assert abs(swapped / (2.0 * box0 + level_1d(N, L, lambda x: p2 * x * x, 1)) - 1.0) > 0.3


def test_cornell_terms_superpose():
    """The Cornell potential is linear in its three parameters: with all three
    set it is the sum of the three single-term potentials pinned above (to
    rounding), so no term takes another's parameter."""
    N, L = 12, 9.0
    p = [0.4, 0.2, 0.05]
    full = orc.potential(orc.POT_CORNELL, p, N, L)
    parts = sum(orc.potential(orc.POT_CORNELL, [p[i] if j == i else 0.0 for j in range(3)], N, L)
                for i in range(3))
    assert np.allclose(full, parts, rtol=1e-14, atol=1e-14)


# ------------------------------------------- regulated Coulomb, Sec. VII.C --
def test_regulated_coulomb_is_zero_inside_a_and_continuous_at_a():
    """Eq. (coulombpot): V = 0 for r < a and -p0/r + p0/a for r >= a, which is
    0 again at r = a (continuous) and positive outside.  An odd lattice has a
    site at r = 0 (inside) and six at r = a."""
    p0, N, L = 1.5, 9, 9.0 * 0.7
    a = L / N
    V = orc.potential(orc.POT_COULOMB_REG, [p0], N, L)
    c = N // 2
    assert V[c, c, c] == 0.0
    for d in ((1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1)):
        assert abs(V[c + d[0], c + d[1], c + d[2]]) <= 1e-15 * p0 / a
    assert V.min() >= -1e-15 * p0 / a and V.max() < p0 / a
    assert np.isfinite(V).all()


def test_regulated_coulomb_binding_reaches_the_hydrogenic_level():
    """With v_inf = p0 / a the binding energy E - v_inf tends to -p0^2 / 2 as
    a -> 0 (Sec. VII.C: the shift does not change the binding energy).  The
    cut inside r < a makes the leading error of order between a and a^2 here
    (measured: the differences of three spacings 1/4, 1/6, 1/8 fall by 2.12,
    between 2.0 for order 1 and 2.86 for order 2), so the limit lies between
    the first- and second-order extrapolations of the two coarser spacings."""
    p0, L = 2.0, 8.0
    res = []
    for N in (32, 48):
        a = L / N
        res.append((a, relax(orc.POT_COULOMB_REG, [p0], N, L, v_inf=p0 / a)["binding"]))
    (a1, e1), (a2, e2) = res
    exact = -0.5 * p0 * p0
    assert exact < e2 < e1
    lo, hi = richardson(a1, e1, a2, e2, 1), richardson(a1, e1, a2, e2, 2)
    assert lo < exact < hi
    assert abs(lo / exact - 1) < 0.05 and abs(hi / exact - 1) < 0.05


# ----------------------------------------------------- Box-Muller draw --
def test_gaussian_start_is_box_muller_of_the_published_splitmix64_outputs():
    """GAUSS kind, seed 0, member 0: site 0 takes SplitMix64 outputs 1 and 2
    (published: 0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4) as u1 = (o1 >> 11)
    2^-53 + 2^-53 in (0, 1] and u2 = (o2 >> 11) 2^-53, and the Box-Muller
    normal sqrt(-2 ln u1) cos(2 pi u2)."""
    o1, o2 = 0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4
    u1 = (o1 >> 11) / 2.0**53 + 2.0**-53
    u2 = (o2 >> 11) / 2.0**53
    want = math.sqrt(-2.0 * math.log(u1)) * math.cos(2.0 * math.pi * u2)
    g = orc.initial(2, seed=0, kind=orc.INIT_GAUSS)
    assert g.reshape(-1)[0] == pytest.approx(want, rel=1e-15, abs=1e-15)
    # a swap of the two uniforms, or sin for cos, would be far off
    assert abs(want - math.sqrt(-2.0 * math.log(u2 + 2.0**-53)) * math.cos(2.0 * math.pi * u1)) > 0.1
    assert abs(want - math.sqrt(-2.0 * math.log(u1)) * math.sin(2.0 * math.pi * u2)) > 0.1


# -------------------------------------------------- reimposition, Sec. IV --
def numpy_mirror(psi, axis, mode):
    """The lower half of `axis` copied onto its mirror with numpy flips; the
    sign flipped under A (mode 2); the mid plane of odd N zeroed under A."""
    out = psi.copy()
    N = psi.shape[axis]
    h = N // 2
    lower = np.take(psi, np.arange(h), axis=axis)
    sign = -1.0 if mode == orc.PAR_A else 1.0
    idx = [slice(None)] * 3
    idx[axis] = slice(N - h, N)
    out[tuple(idx)] = sign * np.flip(lower, axis=axis)
    if N % 2 == 1 and mode == orc.PAR_A:
        idx[axis] = h
        out[tuple(idx)] = 0.0
    return out


@pytest.mark.parametrize("N", [6, 7])
@pytest.mark.parametrize("axis", [0, 1, 2])
@pytest.mark.parametrize("mode", [orc.PAR_S, orc.PAR_A])
def test_reimpose_is_the_mirror_copy_of_the_lower_half(N, axis, mode):
    rng = np.random.default_rng(11 + N)
    psi = rng.standard_normal((N, N, N))
    word = orc.parity_word(**{"xyz"[axis]: mode})
    got = orc.reimpose(psi, word)
    assert np.array_equal(got, numpy_mirror(psi, axis, mode))
    # idempotent, and the lower half is untouched
    assert np.array_equal(orc.reimpose(got, word), got)
    h = N // 2
    assert np.array_equal(np.take(got, np.arange(h), axis=axis), np.take(psi, np.arange(h), axis=axis))


def test_reimpose_on_several_axes_composes_the_single_axis_copies():
    N = 7
    psi = np.random.default_rng(3).standard_normal((N, N, N))
    word = orc.parity_word(x=orc.PAR_S, y=orc.PAR_A, z=orc.PAR_A)
    want = numpy_mirror(numpy_mirror(numpy_mirror(psi, 0, orc.PAR_S), 1, orc.PAR_A), 2, orc.PAR_A)
    assert np.array_equal(orc.reimpose(psi, word), want)
