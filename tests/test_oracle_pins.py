"""Pins of the FP64 oracle against things the paper and the mathematics fix.

None of these re-types the oracle's formula: each compares the oracle with an
independent construction (closed-form lattice modes, a dense matrix built from
Kronecker products, scipy eigensolvers, the paper's printed numbers, the
published SplitMix64 sequence, brute-force finite differences).
"""
import json
import math
import os

import numpy as np
import pytest
import scipy.linalg as sla

import oracle as orc

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------- helpers --
def dense_ops(V, L, dt, mass=1.0):
    """Dense H = -lap/(2m) + V and D = I + (dt/2) V on an N^3 Dirichlet lattice,
    built from the 1-d second-difference matrix by Kronecker sums."""
    N = V.shape[0]
    a = L / N
    T = (np.diag(-2.0 * np.ones(N)) + np.diag(np.ones(N - 1), 1) + np.diag(np.ones(N - 1), -1)) / a**2
    I = np.eye(N)
    lap = np.kron(T, np.kron(I, I)) + np.kron(I, np.kron(T, I)) + np.kron(I, np.kron(I, T))
    H = -lap / (2.0 * mass) + np.diag(V.reshape(-1))
    D = np.eye(N**3) + 0.5 * dt * np.diag(V.reshape(-1))
    return H, D


def box_mode(N, k):
    n = np.arange(1, N + 1)
    f = [np.sin(kk * math.pi * n / (N + 1)) for kk in k]
    return np.einsum("i,j,k->ijk", f[0], f[1], f[2])


def box_lambda(N, L, k, mass=1.0, v0=0.0):
    a = L / N
    return sum(2.0 / (mass * a * a) * math.sin(kk * math.pi / (2 * (N + 1))) ** 2 for kk in k) + v0


# ------------------------------------------------------- closed-form modes --
@pytest.mark.parametrize("k", [(1, 1, 1), (2, 1, 3), (5, 4, 6), (7, 7, 7)])
@pytest.mark.parametrize("v0", [0.0, 0.7, -1.3])
def test_step_multiplies_box_mode_by_closed_form_factor(k, v0):
    N, L, mass = 7, 3.5, 1.0
    a = L / N
    dt = a * a / 8
    psi = box_mode(N, k)
    V = orc.potential(orc.POT_CONST, [v0], N, L)
    out = orc.step(psi, V, L, dt, mass)
    lam = box_lambda(N, L, k, mass, v0)
    g = 1.0 - dt * lam / (1.0 + 0.5 * dt * v0)
    np.testing.assert_allclose(out, g * psi, rtol=0, atol=1e-13)
    ob = orc.observables(psi, V, L, mass)
    assert ob["energy"] == pytest.approx(lam, rel=1e-13)


def test_two_mode_energy_history_closed_form():
    N, L, mass, v0 = 9, 4.0, 1.3, 0.25
    a = L / N
    dt = mass * a * a / 5
    k0, k1 = (1, 1, 1), (2, 1, 1)
    p0, p1 = box_mode(N, k0), box_mode(N, k1)
    l0, l1 = box_lambda(N, L, k0, mass, v0), box_lambda(N, L, k1, mass, v0)
    g0 = 1 - dt * l0 / (1 + 0.5 * dt * v0)
    g1 = 1 - dt * l1 / (1 + 0.5 * dt * v0)
    n0, n1 = np.sum(p0 * p0), np.sum(p1 * p1)
    psi = p0 + 3.0 * p1
    V = orc.potential(orc.POT_CONST, [v0], N, L)
    for t in range(40):
        c0, c1 = g0**t, 3.0 * g1**t
        expect = (c0 * c0 * n0 * l0 + c1 * c1 * n1 * l1) / (c0 * c0 * n0 + c1 * c1 * n1)
        assert orc.observables(psi, V, L, mass)["energy"] == pytest.approx(expect, rel=1e-12)
        psi = orc.step(psi, V, L, dt, mass)


@pytest.mark.parametrize("mass", [1.0, 0.5, 2.0])
def test_stability_bound_on_checkerboard_mode(mass):
    """von Neumann bound dt < m a^2 / 3 (Sec. III).  On a finite lattice the
    highest mode has lambda_max = (6 / m a^2) sin^2(N pi / 2(N + 1)), so it
    grows once dt exceeds 2 / lambda_max, a bound that tends to m a^2 / 3."""
    N, L = 40, 20.0
    a = L / N
    V = orc.potential(orc.POT_CONST, [0.0], N, L)
    psi = box_mode(N, (N, N, N))
    lam_max = box_lambda(N, L, (N, N, N), mass)
    dt_crit = 2.0 / lam_max
    assert mass * a * a / 3 < dt_crit < 1.01 * mass * a * a / 3
    for dt, grows in ((1.02 * mass * a * a / 3, True), (0.98 * mass * a * a / 3, False)):
        p = psi.copy()
        for _ in range(60):
            p = orc.step(p, V, L, dt, mass)
        ratio = np.abs(p).max() / np.abs(psi).max()
        assert (ratio > 1.0) == grows
        g = 1.0 - dt * lam_max
        assert ratio == pytest.approx(abs(g) ** 60, rel=1e-9)


# ------------------------------------------------------------ dense checks --
def test_step_equals_dense_operator_random_potential():
    """psi' = (I - dt D^-1 H) psi: the update equation with A, B of Sec. III."""
    rng = np.random.default_rng(3)
    N, L, mass = 6, 5.0, 0.8
    a = L / N
    dt = mass * a * a / 4
    V = rng.uniform(-2, 3, size=(N, N, N))
    psi = rng.standard_normal((N, N, N))
    H, D = dense_ops(V, L, dt, mass)
    expect = psi.reshape(-1) - dt * np.linalg.solve(D, H @ psi.reshape(-1))
    np.testing.assert_allclose(orc.step(psi, V, L, dt, mass).reshape(-1), expect, rtol=0, atol=1e-12)
    np.testing.assert_allclose(orc.hpsi(psi, V, L, mass).reshape(-1), H @ psi.reshape(-1),
                               rtol=0, atol=1e-11)
    ob = orc.observables(psi, V, L, mass, v_inf=0.4)
    v = psi.reshape(-1)
    assert ob["energy"] == pytest.approx(v @ H @ v / (v @ v), rel=1e-13)
    assert ob["binding"] == pytest.approx(ob["energy"] - 0.4, rel=1e-13)
    assert ob["norm2"] == pytest.approx((v @ v) * a**3, rel=1e-14)


def test_converged_energy_is_generalised_eigenpair_8cubed():
    """The fixed point of the update is the lowest vector of H psi = mu D psi;
    the readout is <H> of that vector and lies above lambda_min(H)."""
    N, L = 8, 10.0
    a = L / N
    dt = a * a / 8
    V = orc.potential(orc.POT_HO, [1.0, 1.0, 1.0], N, L)
    H, D = dense_ops(V, L, dt)
    w, U = sla.eigh(H, D)
    u = U[:, 0]
    e_gen = u @ H @ u / (u @ u)
    lam_min = sla.eigh(H, eigvals_only=True)[0]
    psi = orc.initial(N, seed=11)
    done, conv, hist = orc.evolve(psi, V, L, dt, 4000, renorm_every=1, check_every=100,
                                  rel_tol=1e-15)
    e = orc.observables(psi, V, L)["energy"]
    assert e == pytest.approx(e_gen, rel=1e-11)
    assert e >= lam_min
    # state agrees with the generalised eigenvector up to sign
    v = orc.normalized(psi, L).reshape(-1)
    u = u / np.linalg.norm(u) * np.linalg.norm(v)
    assert min(np.linalg.norm(v - u), np.linalg.norm(v + u)) < 1e-8 * np.linalg.norm(v)


def test_fdtd_energy_gap_scales_as_dt_squared():
    N, L = 8, 10.0
    a = L / N
    V = orc.potential(orc.POT_HO, [1.0, 1.0, 1.0], N, L)
    lam_min = sla.eigh(dense_ops(V, L, 0.0)[0], eigvals_only=True)[0]
    gaps = []
    for dt in (a * a / 16, a * a / 32, a * a / 64):
        H, D = dense_ops(V, L, dt)
        psi = orc.initial(N, seed=5)
        orc.evolve(psi, V, L, dt, 40000, check_every=200, rel_tol=1e-15)
        gaps.append(orc.observables(psi, V, L)["energy"] - lam_min)
    assert all(g > 0 for g in gaps)
    assert gaps[0] / gaps[1] == pytest.approx(4.0, rel=0.05)
    assert gaps[1] / gaps[2] == pytest.approx(4.0, rel=0.05)


# ----------------------------------------------------- separable HO + paper --
def ho_lambda_1d(N, L):
    a = L / N
    x = orc.coords(N, L)
    d = 1.0 / a**2 + 0.5 * x * x
    e = -0.5 / a**2 * np.ones(N - 1)
    return sla.eigh_tridiagonal(d, e, eigvals_only=True, select="i", select_range=(0, 0))[0]


def test_paper_ho_energy_from_discrete_hamiltonian():
    """Sec. VII.D prints E0 = 1.49996 at 512^3, a = 0.02 for V = r^2/2; the
    lattice Hamiltonian on cell-centred sites is separable, so its lowest
    eigenvalue is three times the 1-d one."""
    g = json.load(open(os.path.join(GOLDEN, "paper_values.json")))["ho_512"]
    e = 3 * ho_lambda_1d(g["N"], g["L"])
    assert round(e, g["digits"]) == pytest.approx(g["E0"], abs=1e-12)


def test_ho_cfg_32cubed_converges_to_just_above_lambda_min():
    """32^3, L = 10, dt = a^2/8, 3000 steps from uniform noise."""
    N, L = 32, 10.0
    a = L / N
    V = orc.potential(orc.POT_HO, [1.0, 1.0, 1.0], N, L)
    psi = orc.initial(N, seed=1)
    orc.evolve(psi, V, L, a * a / 8, 3000)
    ob = orc.observables(psi, V, L)
    lam = 3 * ho_lambda_1d(N, L)
    assert lam <= ob["energy"] < lam + 3e-5
    assert abs(ob["energy"] - 1.5) < 0.01          # continuum (n + 3/2) w
    assert ob["r_rms"] == pytest.approx(math.sqrt(1.5), rel=0.01)  # virial: r_rms^2 = E


def test_ho_anisotropic_az_state_is_first_z_excitation():
    """An A_z start can only relax to the lowest z-odd state: energy
    l0(x) + l0(y) + l1(z) of the separable lattice problem."""
    N, L = 16, 10.0
    a = L / N
    V = orc.potential(orc.POT_HO, [1.0, 1.0, 1.0], N, L)
    psi = orc.initial(N, seed=2, parity=orc.parity_word(z=orc.PAR_A))
    orc.evolve(psi, V, L, a * a / 8, 4000)
    x = orc.coords(N, L)
    lam = sla.eigh_tridiagonal(1 / a**2 + 0.5 * x * x, -0.5 / a**2 * np.ones(N - 1),
                               eigvals_only=True)
    e = orc.observables(psi, V, L)["energy"]
    assert e == pytest.approx(2 * lam[0] + lam[1], rel=2e-3)
    assert e > 2 * lam[0] + lam[1]


def test_hydrogen_like_ground_state():
    """Coulomb V = -1/r on cell-centred sites (no site at r = 0): E -> -1/2,
    r_rms -> sqrt(3) as a -> 0; at a = 0.3125 within a few per cent."""
    N, L = 48, 15.0
    a = L / N
    V = orc.potential(orc.POT_COULOMB, [1.0], N, L)
    psi = orc.initial(N, seed=7)
    done, conv, _ = orc.evolve(psi, V, L, a * a / 8, 12000, check_every=100, rel_tol=1e-8)
    ob = orc.observables(psi, V, L)
    assert conv
    assert ob["energy"] == pytest.approx(-0.5, rel=0.04)
    assert ob["r_rms"] == pytest.approx(math.sqrt(3.0), rel=0.05)


# --------------------------------------------------------------- invariants --
@pytest.mark.parametrize("N", [8, 9])
@pytest.mark.parametrize("mode", [orc.PAR_S, orc.PAR_A])
def test_parity_is_preserved_bitwise(N, mode):
    L = 6.0
    a = L / N
    # Cornell is singular at r = 0, a lattice site when N is odd
    V = (orc.potential(orc.POT_CORNELL, [0.4, 0.2, 0.05], N, L) if N % 2 == 0
         else orc.potential(orc.POT_HO, [1.0, 0.7, 1.3], N, L))
    psi = orc.initial(N, seed=4, parity=orc.parity_word(z=mode, x=mode))
    sign = 1.0 if mode == orc.PAR_S else -1.0
    for p in (psi,):
        assert np.array_equal(p[:, :, ::-1], sign * p)
        assert np.array_equal(p[::-1, :, :], sign * p)
    orc.evolve(psi, V, L, a * a / 8, 150)
    assert np.array_equal(psi[:, :, ::-1], sign * psi)
    assert np.array_equal(psi[::-1, :, :], sign * psi)
    if N % 2 == 1 and mode == orc.PAR_A:
        assert not psi[:, :, N // 2].any()


def test_d_quotient_is_non_increasing_where_bound_holds():
    """With dt max_i(6/(m a^2) + V_i)/(1 + dt V_i/2) <= 1 every amplification
    factor lies in [0, 1], so <psi|H|psi>/<psi|D|psi> cannot rise."""
    N, L = 32, 10.0
    a = L / N
    dt = a * a / 8
    V = orc.potential(orc.POT_HO, [1.0, 1.0, 1.0], N, L)
    assert (dt * (6 / a**2 + V) / (1 + 0.5 * dt * V)).max() <= 1.0
    psi = orc.initial(N, seed=9)
    prev = np.inf
    for _ in range(150):
        q = np.sum(psi * orc.hpsi(psi, V, L)) / np.sum(psi * psi * (1 + 0.5 * dt * V))
        assert q <= prev * (1 + 1e-14)
        prev = q
        psi = orc.step(psi, V, L, dt)


def test_renormalisation_does_not_change_observables():
    N, L = 10, 8.0
    a = L / N
    V = orc.potential(orc.POT_CORNELL, [0.4, 0.2, 0.05], N, L)
    p1 = orc.initial(N, seed=3)
    p2 = p1.copy()
    orc.evolve(p1, V, L, a * a / 8, 300, renorm_every=1)
    orc.evolve(p2, V, L, a * a / 8, 300, renorm_every=0)
    o1, o2 = orc.observables(p1, V, L), orc.observables(p2, V, L)
    for k in ("energy", "r_rms", "kinetic"):
        assert o1[k] == pytest.approx(o2[k], rel=1e-12)
    assert o1["norm2"] == pytest.approx(1.0, rel=1e-13)


def test_convergence_check_semantics():
    N, L = 8, 8.0
    a = L / N
    V = orc.potential(orc.POT_HO, [1.0, 1.0, 1.0], N, L)
    psi = orc.initial(N, seed=1)
    done, conv, hist = orc.evolve(psi, V, L, a * a / 8, 20000, check_every=50, rel_tol=1e-9)
    assert conv and done % 50 == 0 and done < 20000
    assert abs(hist[-1] - hist[-2]) <= 1e-9 * abs(hist[-1])
    assert all(abs(hist[i] - hist[i - 1]) > 1e-9 * abs(hist[i]) for i in range(1, len(hist) - 1))


# -------------------------------------------------------------------- RNG --
def test_initial_noise_follows_published_splitmix64_sequence():
    """SplitMix64 seeded with 0 starts 0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4,
    0x06C45D188009454F; site s takes output 2s + 1 (uniform kind)."""
    outs = [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]
    psi = orc.initial(2, seed=0)
    flat = psi.reshape(-1)
    assert flat[0] == 2.0 * ((outs[0] >> 11) / 2.0**53) - 1.0
    assert flat[1] == 2.0 * ((outs[2] >> 11) / 2.0**53) - 1.0


def test_initial_noise_statistics():
    u = orc.initial(40, seed=123)
    assert u.min() >= -1.0 and u.max() < 1.0
    assert abs(u.mean()) < 0.01 and u.var() == pytest.approx(1 / 3, rel=0.01)
    g = orc.initial(40, seed=123, kind=orc.INIT_GAUSS)
    assert abs(g.mean()) < 0.01 and g.var() == pytest.approx(1.0, rel=0.02)
    m1 = orc.initial(6, seed=5, member=1)
    assert not np.array_equal(m1, orc.initial(6, seed=5, member=0))


# --------------------------------------------------------------- upsample --
def test_upsample_is_exact_on_trilinear_functions_inside():
    Nc, Nf, L = 8, 16, 6.0
    xc, xf = orc.coords(Nc, L), orc.coords(Nf, L)
    f = lambda x, y, z: (1 + 0.3 * x) * (2 - 0.1 * y) * (1.5 + 0.2 * z) + 0.05 * x * y * z
    pc = f(*np.meshgrid(xc, xc, xc, indexing="ij"))
    pf = orc.upsample(pc, Nf, L)
    ref = f(*np.meshgrid(xf, xf, xf, indexing="ij"))
    inner = (slice(1, Nf - 1),) * 3
    ratio = pf[inner] / ref[inner]
    assert np.ptp(ratio) < 1e-13 * abs(ratio.mean())


def test_upsample_dyadic_weights_of_a_single_site():
    Nc, L = 4, 4.0
    pc = np.zeros((Nc, Nc, Nc))
    pc[1, 2, 1] = 1.0
    pf = orc.upsample(pc, 2 * Nc, L)
    pf = pf / pf.max() * 27.0  # largest weight is 27/64
    w1 = np.array([0, 1, 3, 3, 1, 0, 0, 0], dtype=float)       # around coarse index 1
    w2 = np.array([0, 0, 0, 1, 3, 3, 1, 0], dtype=float)       # around coarse index 2
    np.testing.assert_allclose(pf, np.einsum("i,j,k->ijk", w1, w2, w1), atol=1e-12)


def test_upsample_preserves_parity_and_normalises():
    Nc, Nf, L = 8, 16, 6.0
    pc = orc.initial(Nc, seed=2, parity=orc.parity_word(z=orc.PAR_A, y=orc.PAR_S))
    pf = orc.upsample(pc, Nf, L)
    # the oracle sums the eight corners in a fixed order, so only up to rounding
    np.testing.assert_allclose(pf[:, :, ::-1], -pf, rtol=0, atol=1e-15)
    np.testing.assert_allclose(pf[:, ::-1, :], pf, rtol=0, atol=1e-15)
    assert np.sum(pf * pf) * (L / Nf) ** 3 == pytest.approx(1.0, rel=1e-13)


# --------------------------------------------------------------- gradient --
def _energy_after(psi0, V, L, dt, T):
    p = psi0.copy()
    orc.evolve(p, V, L, dt, T, renorm_every=1)
    return orc.observables(p, V, L)["energy"]


def test_adjoint_gradient_matches_finite_differences_per_site():
    rng = np.random.default_rng(0)
    N, L, T = 6, 6.0, 25
    a = L / N
    dt = a * a / 8
    V = orc.potential(orc.POT_HO, [1.0, 0.8, 1.2], N, L) + rng.uniform(-0.3, 0.3, (N, N, N))
    psi0 = orc.initial(N, seed=8)
    E, G = orc.energy_grad_v(psi0, V, L, dt, T)
    assert E == pytest.approx(_energy_after(psi0, V, L, dt, T), rel=1e-13)
    h = 1e-4  # truncation ~h^2 and rounding ~1e-16/h both stay below 1e-10 here
    for idx in [(0, 0, 0), (2, 3, 1), (5, 5, 5), (3, 2, 4)]:
        Vp, Vm = V.copy(), V.copy()
        Vp[idx] += h
        Vm[idx] -= h
        fd = (_energy_after(psi0, Vp, L, dt, T) - _energy_after(psi0, Vm, L, dt, T)) / (2 * h)
        assert G[idx] == pytest.approx(fd, rel=1e-6, abs=1e-10)


def test_adjoint_gradient_wrt_well_parameters():
    N, L, T = 8, 8.0, 30
    a = L / N
    dt = a * a / 8
    p = np.array([1.0, 1.0, 1.0, 2.0, 0.5, -0.3, 0.2, 0.9, 1.1, -1.0, 0.4, 0.0, 0.6])
    V = orc.potential(orc.POT_WELLS, p, N, L)
    psi0 = orc.initial(N, seed=12)
    E, G = orc.energy_grad_v(psi0, V, L, dt, T)
    h = 1e-5
    for j in (3, 7, 8, 12):  # A_0, s_0, A_1, s_1
        adj = float(np.sum(G * orc.wells_dv(p, N, L, j)))
        pp, pm = p.copy(), p.copy()
        pp[j] += h
        pm[j] -= h
        fd = (_energy_after(psi0, orc.potential(orc.POT_WELLS, pp, N, L), L, dt, T)
              - _energy_after(psi0, orc.potential(orc.POT_WELLS, pm, N, L), L, dt, T)) / (2 * h)
        assert adj == pytest.approx(fd, rel=1e-6)
        # dV/dtheta itself against differences of the potential
        dv = (orc.potential(orc.POT_WELLS, pp, N, L) - orc.potential(orc.POT_WELLS, pm, N, L)) / (2 * h)
        np.testing.assert_allclose(orc.wells_dv(p, N, L, j), dv, atol=1e-8)


@pytest.mark.parametrize("kind,params,N", [
    (orc.POT_CONST, [0.3], 6),
    (orc.POT_HO, [1.0, 1.3, 0.7], 7),
    (orc.POT_COULOMB, [1.2], 8),
    (orc.POT_COULOMB_REG, [0.9], 8),
    (orc.POT_CORNELL, [0.4, 0.2, 0.05], 8),
    (orc.POT_WELLS, [1.0, 0.8, 1.2, 2.0, 0.5, -0.3, 0.2, 0.9, 1.1, -1.0, 0.4, 0.0, 0.6], 7),
    (orc.POT_DODECA, [-5.0], 9),
])
def test_potential_parameter_derivatives_against_differences(kind, params, N):
    """dV/dp_j of every analytic kind, every parameter, against central
    differences of the potential itself; indices a kind does not have are
    refused."""
    L = 6.0
    p = np.array(params, dtype=np.float64)
    for j in range(p.size):
        h = 1e-5 * max(1.0, abs(p[j]))
        pp, pm = p.copy(), p.copy()
        pp[j] += h
        pm[j] -= h
        fd = (orc.potential(kind, pp, N, L) - orc.potential(kind, pm, N, L)) / (2 * h)
        dv = orc.potential_dv(kind, p, N, L, j)
        np.testing.assert_allclose(dv, fd, rtol=1e-6, atol=1e-8 * max(1.0, np.abs(fd).max()))
        assert np.abs(dv).max() > 0
    with pytest.raises(ValueError):
        orc.potential_dv(kind, p, N, L, p.size)
    if kind in (orc.POT_HO, orc.POT_CORNELL):
        with pytest.raises(ValueError):
            orc.potential_dv(kind, np.append(p, 1.0), N, L, 3)


def test_hellmann_feynman_limit_at_convergence():
    """For a converged state and small dt the gradient approaches the
    Hellmann-Feynman integral sum psi^2 dV/dtheta / sum psi^2."""
    N, L = 10, 8.0
    a = L / N
    dt = a * a / 64
    p = np.array([1.0, 1.0, 1.0, 1.5, 0.3, 0.0, -0.2, 0.8])
    V = orc.potential(orc.POT_WELLS, p, N, L)
    psi = orc.initial(N, seed=3)
    orc.evolve(psi, V, L, dt, 20000, check_every=200, rel_tol=1e-14)
    E, G = orc.energy_grad_v(psi, V, L, dt, 50)
    for j in (3, 7):
        dv = orc.wells_dv(p, N, L, j)
        hf = float(np.sum(psi * psi * dv) / np.sum(psi * psi))
        assert float(np.sum(G * dv)) == pytest.approx(hf, rel=5e-3)


def test_gaussian_well_perturbation_theory_closed_form():
    """First-order perturbation of the w = 1 oscillator ground state by a weak
    well -A exp(-|r - c|^2 / 2 s^2) (continuum):
    dE/dA = -(2 s^2 / (1 + 2 s^2))^{3/2} exp(-|c|^2 / (1 + 2 s^2))."""
    N, L = 24, 10.0
    a = L / N
    dt = a * a / 8
    s, c = 1.1, np.array([0.4, -0.3, 0.2])
    p = np.array([1.0, 1.0, 1.0, 0.0, *c, s])
    V = orc.potential(orc.POT_WELLS, p, N, L)
    psi = orc.initial(N, seed=6)
    orc.evolve(psi, V, L, dt, 6000, check_every=100, rel_tol=1e-13)
    dv = orc.wells_dv(p, N, L, 3)
    hf = float(np.sum(psi * psi * dv) / np.sum(psi * psi))
    expect = -(2 * s * s / (1 + 2 * s * s)) ** 1.5 * math.exp(-c @ c / (1 + 2 * s * s))
    assert hf == pytest.approx(expect, rel=0.01)


# ------------------------------------------------ excited states (Sec. III) --
def test_projection_leaves_the_orthogonal_remainder():
    """Removing two non-orthogonal states one after the other (modified
    Gram-Schmidt) equals the least-squares remainder of psi against the
    space they span, computed by numpy; the coefficients are the sequential
    Gram-Schmidt ones."""
    rng = np.random.default_rng(3)
    n3 = 5 * 5 * 5
    a, b, psi = (rng.standard_normal(n3) for _ in range(3))
    b = b + 0.4 * a  # not orthogonal to a
    out, coef = orc.project_out(psi.reshape(5, 5, 5), [a.reshape(5, 5, 5), b.reshape(5, 5, 5)])
    A = np.stack([a, b], axis=1)
    resid = psi - A @ np.linalg.lstsq(A, psi, rcond=None)[0]
    # sequential removal of a then b equals the remainder against span{a, b}
    # only when b is taken orthogonal to a first: compare with the MGS form
    c0 = psi @ a / (a @ a)
    p1 = psi - c0 * a
    c1 = p1 @ b / (b @ b)
    np.testing.assert_allclose(coef, [c0, c1], rtol=1e-13)
    np.testing.assert_allclose(out.ravel(), p1 - c1 * b, rtol=0, atol=1e-13)
    # one state: exactly orthogonal remainder, and idempotent
    o1, _ = orc.project_out(psi.reshape(5, 5, 5), [a.reshape(5, 5, 5)])
    assert abs(o1.ravel() @ a) < 1e-12 * np.linalg.norm(psi) * np.linalg.norm(a)
    o2, c = orc.project_out(o1, [a.reshape(5, 5, 5)])
    np.testing.assert_allclose(o2, o1, rtol=0, atol=1e-14)
    assert abs(c[0]) < 1e-14
    # orthonormalised basis of the same span: remainder equals least squares
    q, _ = np.linalg.qr(A)
    o3, _ = orc.project_out(psi.reshape(5, 5, 5), [q[:, 0].reshape(5, 5, 5), q[:, 1].reshape(5, 5, 5)])
    np.testing.assert_allclose(o3.ravel(), resid, rtol=0, atol=1e-13)


def test_deflated_relaxation_converges_to_dense_second_vector():
    """Evolving with the converged ground state projected out after every
    step converges to the dominant eigenvector of P M (M the update matrix,
    P the projector), found by a dense eigensolver on 6^3; its energy is the
    second eigenvalue of H up to the O(dt) difference between Euclidean and
    D-orthogonality."""
    N, L = 6, 3.0
    a = L / N
    dt = a * a / 8
    rng = np.random.default_rng(4)
    V = rng.uniform(-1.0, 2.0, (N, N, N))
    H, D = dense_ops(V, L, dt)
    M = np.linalg.solve(D, D - dt * H)
    w, U = np.linalg.eig(M)
    v0 = np.real(U[:, np.argmax(np.real(w))])
    P = np.eye(N**3) - np.outer(v0, v0) / (v0 @ v0)
    w1, U1 = np.linalg.eig(P @ M)
    v1 = np.real(U1[:, np.argmax(np.real(w1))])
    psi = orc.initial(N, 9)
    orc.evolve(psi, V, L, dt, 6000, deflate=[v0.reshape(N, N, N)], project_every=1)
    g = psi.ravel() / np.linalg.norm(psi)
    v1 = v1 / np.linalg.norm(v1)
    assert abs(abs(g @ v1) - 1.0) < 1e-10
    e = orc.observables(psi, V, L)["energy"]
    lam = np.sort(np.linalg.eigvalsh(H))
    assert abs(e - lam[1]) < 5 * dt * abs(lam[1] - lam[0]) + 1e-9
    # projecting every 5th step reaches the same vector
    psi5 = orc.initial(N, 9)
    orc.evolve(psi5, V, L, dt, 6000, deflate=[v0.reshape(N, N, N)], project_every=5)
    g5 = psi5.ravel() / np.linalg.norm(psi5)
    assert abs(abs(g5 @ g) - 1.0) < 1e-9


def test_snapshot_projection_estimates_first_excited_state():
    """The paper's one-shot estimate: a snapshot taken at tau, minus its
    component along the converged ground state of the same iteration, has the
    energy of the first excited state once tau (E2 - E1) >> 1.  Anisotropic
    oscillator, separable: the first excited level is the x excitation, whose
    energy is a sum of 1-d tridiagonal eigenvalues."""
    N, L = 16, 10.0
    a = L / N
    dt = a * a / 8
    w = [1.0, 1.6, 2.3]
    V = orc.potential(orc.POT_HO, w, N, L)
    x = (np.arange(N) * 2 - (N - 1)) * a / 2
    lam = []
    for wi in w:
        T = (np.diag(np.full(N, 1.0 / a**2 + 0.5 * wi**2 * x**2))
             + np.diag(np.full(N - 1, -0.5 / a**2), 1) + np.diag(np.full(N - 1, -0.5 / a**2), -1))
        lam.append(np.linalg.eigvalsh(T))
    e1 = lam[0][1] + lam[1][0] + lam[2][0]
    psi0 = orc.initial(N, 5)
    orc.evolve(psi0, V, L, dt, 6000)
    err = []
    for steps in (60, 240):
        snap = orc.initial(N, 5)
        orc.evolve(snap, V, L, dt, steps)
        est, c = orc.project_out(snap, [psi0])
        err.append(abs(orc.observables(est, V, L)["energy"] - e1))
    assert err[1] < err[0] and err[1] < 5e-3 * e1


# ------------------------------------------- dodecahedron well (Sec. VII.E) --
def test_dodecahedron_well_volume_symmetry_and_vertices():
    """The well is a regular dodecahedron whose circumsphere has radius
    sqrt(3)/phi in units where the lattice spans [-1, 1]: the fraction of
    sites inside, corrected for the (N - 1)^3 / N^3 measure of the sampled
    cube, approaches the solid's volume (15 + 7 sqrt 5)/4 e^3 with edge
    e = 2/phi^2; the well is invariant under the three mirrors and the cyclic
    exchange of axes; points just inside / outside the 20 vertices fall on
    the right sides."""
    phi = (1 + math.sqrt(5)) / 2
    e = 2.0 / phi**2
    vol = (15 + 7 * math.sqrt(5)) / 4 * e**3
    fr = []
    for N in (48, 96):
        V = orc.potential(orc.POT_DODECA, [-100.0], N, 0.1 * N)
        assert set(np.unique(V)) == {-100.0, 0.0}
        fr.append((V < 0).mean() * (N / (N - 1)) ** 3)
        assert np.array_equal(V, V[::-1]) and np.array_equal(V, V[:, ::-1]) and np.array_equal(V, V[:, :, ::-1])
        assert np.array_equal(V, np.transpose(V, (2, 0, 1)))
    for f in fr:
        assert abs(f / (vol / 8) - 1) < 2e-3
    # a 3-site lattice samples u in {-1, 0, 1}: the centre is inside, the
    # corners (+-1, +-1, +-1) are outside (radius sqrt 3 > sqrt(3)/phi)
    V3 = orc.potential(orc.POT_DODECA, [-1.0], 3, 3.0)
    assert V3[1, 1, 1] == -1.0 and V3[0, 0, 0] == 0.0 and V3[2, 2, 2] == 0.0
    # (0, 0, +-1) is the midpoint of the edge from (0, -1/phi^2, +-1) to
    # (0, 1/phi^2, +-1), on the faces with normals (+-1, 0, phi): on the
    # boundary, so inside the closed solid; likewise on the other axes
    assert V3[1, 1, 0] == -1.0 and V3[1, 1, 2] == -1.0
    assert V3[1, 0, 1] == -1.0 and V3[2, 1, 1] == -1.0
    # the same edge midpoints on a 201-site lattice
    V5 = orc.potential(orc.POT_DODECA, [-1.0], 201, 20.1)
    assert V5[100, 100, 200] == -1.0 and V5[100, 100, 0] == -1.0
