"""Seeded synthetic workloads: lattice sizes, boxes, time steps and potential
parameters of the benchmark configurations.

This module only generates input parameters.  It holds none of the method's
arithmetic (no update, reduction or potential evaluation), so both the GPU
path and the CPU oracle may take their inputs from it.

Potential kinds are numbered as in the library header: 0 constant,
1 harmonic oscillator (wx, wy, wz), 2 Coulomb -Z/r, 3 the paper's regulated
Coulomb (Sec. VII.C), 4 Cornell-type -k/r + s r + g z^2, 5 oscillator plus
Gaussian wells (wx, wy, wz, then A, cx, cy, cz, s per well), 6 the
dodecahedron well of Sec. VII.E (depth).
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Sequence

import numpy as np

POT_CONST, POT_HO, POT_COULOMB, POT_COULOMB_REG, POT_CORNELL, POT_WELLS, POT_DODECA = range(7)


@dataclass
class Lattice:
    N: int
    L: float
    pot_kind: int
    pot_params: List[float]
    mass: float = 1.0
    dt_over_a2: float = 1.0 / 8.0
    v_inf: float = 0.0
    seed: int = 0
    parity: int = 0

    @property
    def a(self) -> float:
        return self.L / self.N

    @property
    def dt(self) -> float:
        return self.dt_over_a2 * self.a * self.a

    @property
    def sites(self) -> int:
        return self.N ** 3


def parity_word(x: int = 0, y: int = 0, z: int = 0) -> int:
    """2 bits per axis: 0 free, 1 symmetric (S_i), 2 antisymmetric (A_i)."""
    return (x & 3) | ((y & 3) << 2) | ((z & 3) << 4)


def ho_32() -> Lattice:
    """Isotropic oscillator V = r^2/2 on 32^3, L = 10, dt = a^2/8, FP64,
    uniform noise, 3000 steps, renormalised every step."""
    return Lattice(32, 10.0, POT_HO, [1.0, 1.0, 1.0], seed=1)


def coulomb_128(odd_z: bool = False) -> Lattice:
    """V = -1/r on 128^3, L = 40 (no site at r = 0), dt = a^2/8; the even
    start is S_z-symmetrised noise, the odd one the same noise made A_z."""
    return Lattice(128, 40.0, POT_COULOMB, [1.0], seed=2,
                   parity=parity_word(z=2 if odd_z else 1))


CORNELL_PARAMS = [0.4, 0.2, 0.05]


def cornell(N: int) -> Lattice:
    """V = -0.4/r + 0.2 r + 0.05 z^2 on L = 30 (levels 128, 256, 512)."""
    return Lattice(N, 30.0, POT_CORNELL, list(CORNELL_PARAMS), seed=3)


BATCH_SIDES = (48, 64, 96, 128, 160)


def random_wells(rng: np.random.Generator, n_wells: int = 8, w_range=(0.5, 2.0)) -> List[float]:
    """Oscillator frequencies, then per well (A, cx, cy, cz, s), drawn in that
    order: w in U[0.5, 2], A in U[0, 3], c in U[-3, 3]^3, s in U[0.3, 1.5]."""
    p = [float(v) for v in rng.uniform(*w_range, size=3)]
    for _ in range(n_wells):
        A = float(rng.uniform(0.0, 3.0))
        c = [float(v) for v in rng.uniform(-3.0, 3.0, size=3)]
        s = float(rng.uniform(0.3, 1.5))
        p += [A, *c, s]
    return p


def wells_batch(count: int = 64, seed: int = 4, sides: Sequence[int] = BATCH_SIDES,
                L: float = 12.0) -> List[Lattice]:
    """Batch of random oscillator-plus-wells potentials on uneven lattices.
    numpy PCG64(seed) draws, per member in order: the side N from `sides`,
    then the potential parameters as in random_wells."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for m in range(count):
        N = int(rng.choice(np.asarray(sides)))
        out.append(Lattice(N, L, POT_WELLS, random_wells(rng), seed=seed, ))
    return out


def gradient_wells(N: int = 256, seed: int = 5) -> Lattice:
    """Fixed-seed eight-well potential with wx = wy = wz = 1 on L = 12; the 16
    differentiated parameters are (A_k, s_k), k = 1..8."""
    rng = np.random.Generator(np.random.PCG64(seed))
    p = random_wells(rng)
    p[0:3] = [1.0, 1.0, 1.0]
    return Lattice(N, 12.0, POT_WELLS, p, seed=seed)


def gradient_param_indices(n_wells: int = 8) -> List[int]:
    """Positions of A_k and s_k in the parameter vector of kind 5."""
    idx = []
    for k in range(n_wells):
        idx += [3 + 5 * k, 3 + 5 * k + 4]
    return idx


# ------------------------------------------- the paper's own setups (Sec. VII) --
def paper_coulomb(N: int = 512, a: float = 0.05, dt_over_a2: float = 0.25,
                  parity: int = 0) -> Lattice:
    """Regulated Coulomb potential of Sec. VII.C (0 for r < a, -1/r + 1/a
    beyond), m = 1, dt = a^2/4: 512^3 at a = 0.05 (L = 25.6 Bohr radii;
    printed binding energies -0.499 and -0.122) and, by the multi-resolution
    chain of Sec. VII.G, 1024^3 at a = 0.025 (-0.499632).  V at infinity is
    1/a, so the binding energy is E - 1/a."""
    return Lattice(N, N * a, POT_COULOMB_REG, [1.0], dt_over_a2=dt_over_a2, v_inf=1.0 / a,
                   seed=11, parity=parity)


def paper_coulomb_az() -> Lattice:
    """The A_z start of Sec. VII.F: regulated Coulomb on 256^3, a = 0.2,
    dt = 0.01 (= a^2/4); printed E_1 = -0.12507 and, for the next state odd
    in z, E_2 = -0.055360."""
    return Lattice(256, 256 * 0.2, POT_COULOMB_REG, [1.0], dt_over_a2=0.25, v_inf=5.0, seed=12,
                   parity=parity_word(z=2))


def paper_ho_512() -> Lattice:
    """Isotropic oscillator of Sec. VII.D: 512^3, a = 0.02 (L = 10.24),
    dt = 1e-4 (= a^2/4); printed E_0 = 1.49996."""
    return Lattice(512, 10.24, POT_HO, [1.0, 1.0, 1.0], dt_over_a2=0.25, seed=13)


def paper_dodeca(N: int = 128) -> Lattice:
    """Dodecahedron well of Sec. VII.E, V = -100 inside: a = 0.1,
    dt = 0.001 (= a^2/10); printed E_0 = -99.78 and E_1 = -99.55 on 128^3,
    E_0 = -99.97 on 512^3."""
    return Lattice(N, N * 0.1, POT_DODECA, [-100.0], dt_over_a2=0.1, seed=14)
