"""The allocation-free upsample (fdtd_upsample_noalloc) against fdtd_upsample:
the same fine state bit for bit, the same observables and the same
relaxation afterwards, on two calls in a row, the second with a smaller
fine lattice (the static scratch keeps the first call's partial sums); the
handles' allocation counters do not move during the call."""
import ctypes as C
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

from paper_0904_0939_amd import fdtd as F  # noqa: E402
from paper_0904_0939_amd import workloads as W  # noqa: E402
from paper_0904_0939_amd.solver import Solver  # noqa: E402


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def coarse_state(N, L, dtype, seed, parity=0):
    """Even sides only (coarse and fine): an odd side puts a site at r = 0,
    where -0.4/r is infinite."""
    c = Solver(N, L, dtype=dtype)
    c.set_potential(F.POT_CORNELL, W.CORNELL_PARAMS)
    c.set_initial(seed, parity=parity)
    c.evolve(40)
    return c


def fine_handle(N, L, dtype):
    f = Solver(N, L, dtype=dtype)
    f.set_potential(F.POT_CORNELL, W.CORNELL_PARAMS)
    return f


@pytest.mark.parametrize("calls", [[(48, "bf16", 96, "f32", 0), (20, "f32", 30, "f64", 0)],
                                   [(64, "f32", 128, "bf16", W.parity_word(z=2)),
                                    (34, "f64", 66, "f32", W.parity_word(x=2))]])
def test_noalloc_upsample_equals_upsample_on_two_calls(calls):
    L = 12.0
    for Nc, cd, Nf, fd, par in calls:  # the second call is the smaller one
        say(f"case: upsample_noalloc {Nc}^3 {cd} -> {Nf}^3 {fd} parity {par}")
        c = coarse_state(Nc, L, cd, seed=Nc, parity=par)
        ref = fine_handle(Nf, L, fd)
        F.fdtd_upsample(c.h, 0, ref.h, 0)
        got = fine_handle(Nf, L, fd)
        a0 = got.counters()["allocations"]
        F.fdtd_upsample_noalloc(c.h, 0, got.h, 0)
        assert got.counters()["allocations"] == a0
        assert np.array_equal(got.state(), ref.state())
        assert got.observables() == ref.observables()
        ref.evolve(25)
        got.evolve(25)
        assert np.array_equal(got.state(), ref.state())
        for h in (c, ref, got):
            h.close()


def test_noalloc_upsample_rejects_a_fine_side_beyond_the_scratch():
    say("case: upsample_noalloc size limit")
    c = coarse_state(16, 12.0, "f32", seed=1)
    big = F.fdtd_create(F.fdtd_config(1621, F.F32, 1621.0, 1.0, 0.1, 0.0, 0, 0, None))
    try:
        st = F.lib().fdtd_upsample_noalloc(C.c_void_p(c.h), 0, C.c_void_p(big), 0)
        assert st == F.EINVAL and "1620" in F.fdtd_last_error()
    finally:
        F.fdtd_destroy(big)
        c.close()
