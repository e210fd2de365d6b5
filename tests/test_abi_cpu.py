"""C-ABI contract checks that need no GPU: the library loads, exports every
function include/fdtd.h declares, and its host-side validation returns the
documented status codes."""
import ctypes as C
import os

import pytest

from paper_0904_0939_amd import fdtd as F


def cfg(N=16, L=8.0, dt_over=0.125, mass=1.0, dtype=F.F32, history=0):
    a = L / N
    return F.fdtd_config(N, dtype, L, mass, dt_over * mass * a * a, 0.0, 0, history, None)


def status_of(fn, *args):
    return getattr(F.lib(), fn)(*args)


def test_library_exports_every_header_function():
    lib = F.lib()
    names = F.header_functions()
    assert len(names) >= 20
    for n in names:
        assert hasattr(lib, n), n


def test_library_is_built_for_gfx950_only():
    blob = open(F.LIB_PATH, "rb").read()
    assert b"gfx950" in blob


def test_potential_kind_numbering_matches_the_oracle():
    import oracle
    from paper_0904_0939_amd import workloads as W

    for name in ("POT_CONST", "POT_HO", "POT_COULOMB", "POT_COULOMB_REG", "POT_CORNELL",
                 "POT_WELLS", "POT_DODECA"):
        assert getattr(F, name) == getattr(oracle, name) == getattr(W, name)
    hdr = open(F.HEADER).read()
    for i, name in enumerate(["CONST", "HO", "COULOMB", "COULOMB_REG", "CORNELL", "WELLS",
                              "DODECA"]):
        assert f"FDTD_POT_{name} = {i}" in hdr


def test_create_rejects_unstable_time_step():
    h = C.c_void_p()
    c = cfg(dt_over=1.0 / 3.0 * 1.0000001)
    assert status_of("fdtd_create", C.byref(c), C.byref(h)) == F.EUNSTABLE
    assert "stability" in F.fdtd_last_error()
    c = cfg(dt_over=0.33, mass=2.0)
    assert status_of("fdtd_create", C.byref(c), C.byref(h)) == F.OK
    F.fdtd_destroy(h.value)


@pytest.mark.parametrize("field,value", [("n", 1), ("box_len", -1.0), ("mass", 0.0),
                                         ("dt", float("nan")), ("psi_dtype", 7),
                                         ("history", -2)])
def test_create_rejects_bad_config(field, value):
    c = cfg()
    setattr(c, field, value)
    h = C.c_void_p()
    assert status_of("fdtd_create", C.byref(c), C.byref(h)) == F.EINVAL
    assert h.value is None


def test_batch_requires_one_dtype():
    arr = (F.fdtd_config * 2)(cfg(dtype=F.F32), cfg(dtype=F.F64))
    h = C.c_void_p()
    assert status_of("fdtd_create_batch", arr, 2, C.byref(h)) == F.EINVAL
    assert status_of("fdtd_create_batch", arr, 0, C.byref(h)) == F.EINVAL


def test_call_order_and_workspace_checks_without_device():
    h = F.fdtd_create(cfg())
    try:
        opts = F.fdtd_evolve_opts(10, 1, 0, 0, 0, 0.0)
        assert status_of("fdtd_evolve", h, C.byref(opts), None, None) == F.ENOTREADY
        obs = F.fdtd_obs()
        assert status_of("fdtd_observables", h, C.byref(obs)) == F.ENOTREADY
        need = F.fdtd_workspace_size(h)
        assert need > 2 * 16**3 * 4 + 16**3 * 4
        assert status_of("fdtd_bind_workspace", h, C.c_void_p(4096), need - 1) == F.ENOMEM
        assert status_of("fdtd_bind_workspace", h, None, need) == F.EINVAL
        bad = F.fdtd_evolve_opts(-1, 1, 0, 0, 0, 0.0)
        assert status_of("fdtd_evolve", h, C.byref(bad), None, None) == F.EINVAL
        assert status_of("fdtd_set_initial", h, 0, 9, 0, 0, None, 0, 0) == F.EINVAL
        assert status_of("fdtd_set_initial", h, 0, 0, 0, 3 << 4, None, 0, 0) == F.EINVAL
        assert status_of("fdtd_set_initial", h, 5, 0, 0, 0, None, 0, 0) == F.EINVAL
        assert status_of("fdtd_set_potential_analytic", h, 0, 99, None, 0) == F.EINVAL
        p = (C.c_double * 4)(1, 1, 1, 1)
        assert status_of("fdtd_set_potential_analytic", h, 0, F.POT_WELLS, p, 4) == F.EINVAL
        assert status_of("fdtd_energy_grad", h, 0, 1, None, 0, None, 0, None, None, None) == F.EINVAL
        assert status_of("fdtd_set_projection_states", h, 0, None, 2, F.F64, 0) == F.EINVAL
        assert status_of("fdtd_set_projection_states", h, 0, C.c_void_p(64), 17, F.F64, 0) == F.EINVAL
        assert status_of("fdtd_set_projection_states", h, 1, C.c_void_p(64), 1, F.F64, 0) == F.EINVAL
        assert status_of("fdtd_project", h, 0, None) == F.ENOTREADY
        bad = F.fdtd_evolve_opts(10, 1, 0, 0, 0, 0.0, -1, 0)
        assert status_of("fdtd_evolve", h, C.byref(bad), None, None) == F.EINVAL
    finally:
        F.fdtd_destroy(h)


def test_tuning_validation_is_host_side():
    h = F.fdtd_create(cfg(N=18))  # 18 % 4 != 0
    try:
        t = F.fdtd_get_tuning(h)
        assert t.vz == 1  # default falls back to scalar lanes
        for bad in [F.fdtd_tuning(4, 1, 8, 0, 1, 1), F.fdtd_tuning(1, 3, 8, 0, 1, 1),
                    F.fdtd_tuning(1, 1, -1, 0, 1, 1), F.fdtd_tuning(1, 1, 8, -1, 1, 1),
                    F.fdtd_tuning(2, 1, 8, 0, 1, 1), F.fdtd_tuning(1, 1, 8, 0, 1, 2),
                    F.fdtd_tuning(1, 1, 8, 0, 1, 0)]:
            assert status_of("fdtd_set_tuning", h, C.byref(bad)) == F.EINVAL
        F.fdtd_set_tuning(h, F.fdtd_tuning(1, 4, 5, 7, 0, 1))
        assert F.fdtd_get_tuning(h).as_dict() == {"vz": 1, "ry": 4, "xchunk": 5, "grid": 7,
                                                  "xcd_remap": 0, "depth": 1, "variant": 0,
                                                  "persist": 0, "vfuse": 0, "tblock": 0,
                                                  "tile": 0}
        # persistent launches: variant 0 only, bounded step count
        for bad in [F.fdtd_tuning(1, 1, 8, 0, 1, 1, 2, 8), F.fdtd_tuning(1, 1, 8, 0, 1, 1, 0, -1),
                    F.fdtd_tuning(1, 1, 8, 0, 1, 1, 0, 65537)]:
            assert status_of("fdtd_set_tuning", h, C.byref(bad)) == F.EINVAL
        F.fdtd_set_tuning(h, F.fdtd_tuning(1, 2, 0, 0, 1, 1, 0, 64))
        assert F.fdtd_get_tuning(h).persist == 64
        assert status_of("fdtd_set_tuning", h, C.byref(F.fdtd_tuning(1, 2, 0, 0, 1, 1, 0, 0, 2))) == F.EINVAL
        # the LDS-tile variant needs full-width vectors
        assert status_of("fdtd_set_tuning", h, C.byref(F.fdtd_tuning(1, 1, 8, 0, 1, 1, 1))) == F.EINVAL
    finally:
        F.fdtd_destroy(h)


def test_depths_four_and_five_are_for_two_step_passes_of_fp32_arithmetic_states():
    """depths 4 and 5 (an 8-slot register ring) exist for the two-step pass of
    F32 and BF16 states only: one-step shapes and F64 handles refuse them, and
    6 is refused everywhere."""
    f32 = F.fdtd_create(cfg(N=64, dtype=F.F32))
    f64 = F.fdtd_create(cfg(N=64, dtype=F.F64))
    try:
        for depth in (4, 5):
            ok = F.fdtd_tuning(4, 1, 0, 0, 1, depth, 0, 0, 0, 2)
            F.fdtd_set_tuning(f32, ok)
            assert F.fdtd_get_tuning(f32).depth == depth
            one_step = F.fdtd_tuning(4, 1, 0, 0, 1, depth, 0, 0, 0, 0)
            assert status_of("fdtd_set_tuning", f32, C.byref(one_step)) == F.EINVAL
            assert "depth 4 or 5" in F.fdtd_last_error()
        for h, bad in ((f64, F.fdtd_tuning(2, 1, 0, 0, 1, 4, 0, 0, 0, 2)),
                       (f64, F.fdtd_tuning(2, 1, 0, 0, 1, 5, 0, 0, 0, 2)),
                       (f32, F.fdtd_tuning(4, 1, 0, 0, 1, 6, 0, 0, 0, 2))):
            assert status_of("fdtd_set_tuning", h, C.byref(bad)) == F.EINVAL
    finally:
        F.fdtd_destroy(f32)
        F.fdtd_destroy(f64)


def test_write_through_variant_rules_and_default():
    """variant 3 (variant 0 with written-through stores): full vectors, ry <=
    2, no persistence; the default for a single lattice whose two state
    buffers and V fit in 512 MiB, else variant 0."""
    small = F.fdtd_create(cfg(N=64, dtype=F.F32))
    big = F.fdtd_create(cfg(N=512, L=40.0, dtype=F.F32))   # 1.5 GiB of fields
    odd = F.fdtd_create(cfg(N=18, dtype=F.F32))            # scalar lanes
    f64 = F.fdtd_create(cfg(N=256, L=30.0, dtype=F.F64))   # 384 MiB
    arr = (F.fdtd_config * 2)(cfg(N=16), cfg(N=24))
    hb = C.c_void_p()
    assert status_of("fdtd_create_batch", arr, 2, C.byref(hb)) == F.OK
    try:
        assert F.fdtd_get_tuning(small).variant == 3
        assert F.fdtd_get_tuning(f64).variant == 3
        assert F.fdtd_get_tuning(big).variant == 0
        assert F.fdtd_get_tuning(odd).variant == 0
        assert F.fdtd_get_tuning(hb.value).variant == 0
        for bad in [F.fdtd_tuning(1, 1, 0, 0, 1, 1, 3), F.fdtd_tuning(4, 4, 0, 0, 1, 1, 3),
                    F.fdtd_tuning(4, 2, 0, 0, 1, 1, 3, 8), F.fdtd_tuning(4, 2, 0, 0, 1, 1, 4)]:
            assert status_of("fdtd_set_tuning", small, C.byref(bad)) == F.EINVAL
        F.fdtd_set_tuning(big, F.fdtd_tuning(4, 2, 0, 0, 1, 3, 3))
        assert F.fdtd_get_tuning(big).variant == 3
    finally:
        for h in (small, big, odd, f64, hb.value):
            F.fdtd_destroy(h)


def test_two_step_passes_validation():
    """tblock = 2: full vectors, ry = 1, variant 0, persistent passes
    allowed (up to 32768 per launch); any side (tiles of the (y, z) plane),
    every dtype; the wide tile (tile = 1) for F32 and BF16 two-step passes
    only."""
    h32 = F.fdtd_create(cfg(N=64, dtype=F.F32))
    h64 = F.fdtd_create(cfg(N=64, dtype=F.F64))
    hb = F.fdtd_create(cfg(N=64, dtype=F.BF16))
    big = F.fdtd_create(cfg(N=516, L=40.0, dtype=F.F32))
    try:
        ok32 = F.fdtd_tuning(4, 1, 0, 0, 1, 2, 0, 0, 1, 2)
        F.fdtd_set_tuning(h32, ok32)
        assert F.fdtd_get_tuning(h32).tblock == 2
        for bad in [F.fdtd_tuning(4, 1, 0, 0, 1, 1, 0, 0, 1, 1),   # tblock 1
                    F.fdtd_tuning(4, 2, 0, 0, 1, 1, 0, 0, 1, 2),   # ry 2
                    F.fdtd_tuning(1, 1, 0, 0, 1, 1, 0, 0, 1, 2),   # scalar lanes
                    F.fdtd_tuning(4, 1, 0, 0, 1, 1, 2, 0, 1, 2),   # variant 2
                    F.fdtd_tuning(4, 1, 0, 0, 1, 1, 0, 32769, 1, 2)]:  # too many passes
            assert status_of("fdtd_set_tuning", h32, C.byref(bad)) == F.EINVAL
        F.fdtd_set_tuning(h32, F.fdtd_tuning(4, 1, 0, 0, 1, 2, 0, 8, 1, 2))  # persistent passes
        assert F.fdtd_get_tuning(h32).persist == 8
        F.fdtd_set_tuning(h64, F.fdtd_tuning(2, 1, 0, 0, 1, 3, 0, 0, 1, 2))
        F.fdtd_set_tuning(hb, F.fdtd_tuning(8, 1, 0, 0, 1, 2, 0, 0, 1, 2))
        assert status_of("fdtd_set_tuning", hb, C.byref(F.fdtd_tuning(1, 1, 0, 0, 1, 1, 0, 0, 1, 2))) == F.EINVAL
        F.fdtd_set_tuning(big, F.fdtd_tuning(4, 1, 0, 0, 1, 1, 0, 0, 1, 2))
        assert F.fdtd_get_tuning(big).tblock == 2
        # tile shapes: 1 (16 x 128) with tblock = 2 on F32 / BF16 states only
        F.fdtd_set_tuning(h32, F.fdtd_tuning(4, 1, 0, 0, 1, 4, 0, 0, 0, 2, 1))
        assert F.fdtd_get_tuning(h32).tile == 1
        F.fdtd_set_tuning(hb, F.fdtd_tuning(8, 1, 0, 0, 1, 3, 0, 8, 1, 2, 1))
        assert F.fdtd_get_tuning(hb).tile == 1
        for h, bad in [(h64, F.fdtd_tuning(2, 1, 0, 0, 1, 3, 0, 0, 1, 2, 1)),   # F64
                       (h32, F.fdtd_tuning(4, 2, 0, 0, 1, 1, 0, 0, 1, 0, 1)),   # one step per pass
                       (h32, F.fdtd_tuning(4, 1, 0, 0, 1, 2, 0, 0, 1, 2, 2))]:  # no tile 2
            assert status_of("fdtd_set_tuning", h, C.byref(bad)) == F.EINVAL
            assert "tile" in F.fdtd_last_error()
    finally:
        for h in (h32, h64, hb, big):
            F.fdtd_destroy(h)


def test_status_strings_and_null_handles():
    for s in range(7):
        assert F.fdtd_status_string(s).startswith("FDTD_")
    assert status_of("fdtd_destroy", None) == F.OK
    assert status_of("fdtd_synchronize", None) == F.EINVAL
    assert status_of("fdtd_create", None, None) == F.EINVAL


def test_tuning_rejects_too_many_sites_per_lane():
    h = F.fdtd_create(cfg(N=32, dtype=F.BF16))
    try:
        assert status_of("fdtd_set_tuning", h, C.byref(F.fdtd_tuning(8, 2, 8, 0, 1, 2))) == F.EINVAL
        F.fdtd_set_tuning(h, F.fdtd_tuning(8, 1, 8, 0, 1, 1, 1))
        assert status_of("fdtd_set_tuning", h, C.byref(F.fdtd_tuning(8, 1, 8, 0, 1, 1, 2))) == F.EINVAL
        big = F.fdtd_create(cfg(N=2200, L=2200.0, dtype=F.F32))
        assert status_of("fdtd_set_tuning", big, C.byref(F.fdtd_tuning(4, 1, 8, 0, 1, 1, 1))) == F.EINVAL
        F.fdtd_destroy(big)
        h64 = F.fdtd_create(cfg(N=32, dtype=F.F64))
        assert status_of("fdtd_set_tuning", h64, C.byref(F.fdtd_tuning(2, 4, 8, 0, 1, 2))) == F.EINVAL
        F.fdtd_destroy(h64)
        F.fdtd_set_tuning(h, F.fdtd_tuning(8, 1, 8, 0, 1, 3))
    finally:
        F.fdtd_destroy(h)


def test_default_vector_width_follows_dtype():
    for dt, vz in ((F.F64, 2), (F.F32, 4), (F.BF16, 8)):
        h = F.fdtd_create(cfg(N=32, dtype=dt))
        assert F.fdtd_get_tuning(h).vz == vz
        assert F.fdtd_get_tuning(h).persist == 0
        assert F.fdtd_get_tuning(h).vfuse == 1
        F.fdtd_destroy(h)


def test_default_vectors_per_lane_follow_lattice_size():
    """One vector per lane on small single lattices (FP32 up to 176^3, FP64
    up to 96^3), two above and on batches; BF16 lanes hold 8 sites, one
    vector."""
    for dt, N, L, ry in ((F.F32, 128, 40.0, 1), (F.F32, 176, 40.0, 1), (F.F32, 192, 40.0, 2),
                         (F.F32, 512, 40.0, 2), (F.F64, 96, 30.0, 1), (F.F64, 128, 30.0, 2),
                         (F.BF16, 256, 30.0, 1), (F.F32, 18, 8.0, 2)):
        h = F.fdtd_create(cfg(N=N, L=L, dtype=dt))
        assert F.fdtd_get_tuning(h).ry == ry, (dt, N)
        F.fdtd_destroy(h)
    arr = (F.fdtd_config * 2)(cfg(N=16), cfg(N=24))
    hb = C.c_void_p()
    assert status_of("fdtd_create_batch", arr, 2, C.byref(hb)) == F.OK
    assert F.fdtd_get_tuning(hb.value).ry == 2
    F.fdtd_destroy(hb.value)


def test_batches_default_to_persistent_launches():
    arr = (F.fdtd_config * 3)(cfg(N=16), cfg(N=24), cfg(N=32))
    h = C.c_void_p()
    assert status_of("fdtd_create_batch", arr, 3, C.byref(h)) == F.OK
    assert F.fdtd_get_tuning(h.value).persist == 64
    F.fdtd_destroy(h.value)


def test_product_path_has_no_oracle_dependency():
    """The package never imports, links or runs the CPU oracle."""
    root = os.path.dirname(F.__file__)
    for dirpath, _, files in os.walk(root):
        for fn in files:
            if fn.endswith((".py", ".cpp", ".hip", ".h")):
                text = open(os.path.join(dirpath, fn)).read()
                assert "import oracle" not in text and "from oracle" not in text, fn
                assert "liboracle" not in text and "fdtd_oracle" not in text, fn


def test_tune_cache_file_round_trip_and_errors(tmp_path):
    """The autotuner's cache file is written and read back without a GPU;
    a malformed line is rejected and leaves the cache as it was; an empty
    file clears it."""
    entries = ["gfx950/256cu:1:512 4 2 0 0 1 1 3 0 1 0 0",
               "gfx950/256cu:0:64:96 2 1 128 0 1 2 0 64 1 2 0",
               "gfx950/256cu:1:1024 4 1 0 0 1 4 0 0 0 2 1"]
    good = tmp_path / "good.txt"
    good.write_text("# shapes\n" + entries[0] + "\n\n   \n" + "\n".join(entries[1:]) + "\n")
    F.fdtd_tune_cache_load(str(good))
    out = tmp_path / "out.txt"

    def saved():
        F.fdtd_tune_cache_save(str(out))
        text = out.read_text().splitlines()
        assert text[0].startswith("#")
        return sorted(line for line in text if line and not line.startswith("#"))

    assert saved() == sorted(entries)
    bad = tmp_path / "bad.txt"
    for text in ("gfx950/256cu:1:512 4 2 0 0 1 1 3 0 1 0\n",      # a field missing
                 "gfx950/256cu:1:512 4 2 0 0 1 1 3 0 1 0 0 7\n",  # one too many
                 "gfx950/256cu:1:512 4 x 0 0 1 1 3 0 1 0 0\n"):   # not an integer
        bad.write_text(entries[0] + "\n" + text)
        assert status_of("fdtd_tune_cache_load", os.fsencode(str(bad))) == F.EINVAL
        assert "line 2" in F.lib().fdtd_last_error().decode()
    assert saved() == sorted(entries)
    assert status_of("fdtd_tune_cache_load", os.fsencode(str(tmp_path / "missing.txt"))) == F.EINVAL
    assert status_of("fdtd_tune_cache_save", os.fsencode(str(tmp_path / "no" / "dir.txt"))) == F.EINVAL
    assert status_of("fdtd_tune_cache_load", None) == F.EINVAL
    empty = tmp_path / "empty.txt"
    empty.write_text("")
    F.fdtd_tune_cache_load(str(empty))
    assert saved() == []


def test_evolve_flags_are_validated_before_any_device_work():
    h = F.fdtd_create(cfg())
    try:
        bad = F.fdtd_evolve_opts(10, 1, 0, 0, 0, 0.0, 0, 2)  # unknown flag
        assert status_of("fdtd_evolve", h, C.byref(bad), None, None) == F.EINVAL
        bad = F.fdtd_evolve_opts(10, 1, 5, 0, 0, 0.0, 0, F.EVOLVE_ASYNC)  # async + check
        assert status_of("fdtd_evolve", h, C.byref(bad), None, None) == F.EINVAL
        assert "ASYNC" in F.fdtd_last_error()
        ok = F.fdtd_evolve_opts(10, 1, 0, 0, 1, 0.0, 0, F.EVOLVE_ASYNC)
        assert status_of("fdtd_evolve", h, C.byref(ok), None, None) == F.ENOTREADY
    finally:
        F.fdtd_destroy(h)


def test_counters_start_at_zero():
    h = F.fdtd_create(cfg())
    try:
        assert F.fdtd_get_counters(h) == {"graph_captures": 0, "graph_replays": 0, "allocations": 0}
        assert status_of("fdtd_get_counters", h, None) == F.EINVAL
        assert status_of("fdtd_get_counters", None, C.byref(F.fdtd_counters())) == F.EINVAL
    finally:
        F.fdtd_destroy(h)


def _header(magic=0x314B435044544446, version=1, dtype=F.F32, n=16, step=5, scale=0.5,
            parity=0, L=8.0, dt=None):
    import struct

    a = L / n
    dt = 0.125 * a * a if dt is None else dt
    return struct.pack("<QiiqqdIIdd16x", magic, version, dtype, n, step, scale, parity, 0, L, dt)


def test_checkpoint_record_size_and_header_checks_without_device():
    """Record = 80-byte header + the stored state; a load checks the header
    (magic, version, dtype, N, L, dt, step, scale, parity) before it touches
    the device."""
    h = F.fdtd_create(cfg(N=16, dtype=F.F32))
    try:
        assert F.fdtd_checkpoint_size(h, 0) == 80 + 4 * 16**3
        assert status_of("fdtd_checkpoint_size", h, 1, C.byref(C.c_size_t())) == F.EINVAL
        assert status_of("fdtd_checkpoint_save", h, 0, C.c_void_p(64), 0) == F.ENOTREADY
        for hd in (_header(magic=1), _header(version=2), _header(dtype=F.F64), _header(n=15),
                   _header(L=8.5), _header(dt=1e-5), _header(step=-1), _header(scale=0.0),
                   _header(scale=float("inf")), _header(parity=1 << 6)):
            buf = C.create_string_buffer(hd + bytes(4 * 16**3))
            assert status_of("fdtd_checkpoint_load", h, 0, buf, 0) == F.EINVAL
        good = C.create_string_buffer(_header() + bytes(4 * 16**3))
        # a valid record gets as far as the device
        assert status_of("fdtd_checkpoint_load", h, 0, good, 0) == F.EHIP
        assert status_of("fdtd_checkpoint_load", h, 0, None, 0) == F.EINVAL
    finally:
        F.fdtd_destroy(h)


def test_gradient_workspace_size_and_binding_checks_without_device():
    """fdtd_grad_workspace_size covers ceil(T/k) checkpoints, min(k, T) + 1
    recomputed states and two adjoint fields of N^3 storage values, plus the
    dE/dV sums; it grows with T and k; binds need 256-byte alignment."""
    h = F.fdtd_create(cfg(N=16, dtype=F.F32))
    h64 = F.fdtd_create(cfg(N=16, dtype=F.F64))
    try:
        fb = 16**3 * 4
        a = F.fdtd_grad_workspace_size(h, 50, 10)
        assert a >= (5 + 11 + 2) * fb + 16**3 * (8 + 4)
        assert F.fdtd_grad_workspace_size(h, 100, 10) - a >= 5 * fb
        assert F.fdtd_grad_workspace_size(h, 50, 25) - a >= (25 - 10) * fb - 5 * fb
        assert F.fdtd_grad_workspace_size(h64, 50, 10) > a
        n = C.c_size_t()
        assert status_of("fdtd_grad_workspace_size", h, 0, 10, C.byref(n)) == F.EINVAL
        assert status_of("fdtd_grad_workspace_size", h, 10, 0, C.byref(n)) == F.EINVAL
        assert status_of("fdtd_bind_grad_workspace", h, C.c_void_p(4100), 1 << 20) == F.EINVAL
        F.fdtd_bind_grad_workspace(h, None, 0)
    finally:
        F.fdtd_destroy(h)
        F.fdtd_destroy(h64)
