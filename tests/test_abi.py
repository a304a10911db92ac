"""Host-only checks of the C ABI: the library loads, exports every function
include/lbe.h declares, and rejects bad parameters before touching a GPU."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lbe.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(lb_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    from paper_1109_3277_amd import binding
    if not os.path.exists(binding.LIB_PATH):
        from paper_1109_3277_amd import build
        build.build()
    return binding.load_library()


def test_header_declares_the_api():
    names = _declared()
    for n in ("lb_create", "lb_init_fields", "lb_add_ellipsoids", "lb_step", "lb_read_fields",
              "lb_read_particles", "lb_stats", "lb_destroy", "lb_workspace_bytes", "lb_last_error"):
        assert n in names


def test_library_exports_every_declared_symbol(lib):
    from paper_1109_3277_amd import binding
    names = _declared()
    for n in names:
        assert hasattr(lib, n), n
    assert set(binding.EXPORTED) <= set(names)


def test_workspace_bytes_validates(lib):
    from paper_1109_3277_amd import binding as B
    ok = B.make_params((32, 32, 64), 1.0, 0.08, max_particles=1, max_radius=8.0)
    n = lib.lb_workspace_bytes(C.byref(ok))
    N = 32 * 32 * 64
    assert n >= 2 * 2 * 19 * N * 8 + 2 * N * 8 + 2 * N * 4
    for bad in (B.make_params((2, 32, 64), 1.0, 0.08), B.make_params((8, 8, 8), 0.5, 0.08),
                B.make_params((8, 8, 8), float("nan"), 0.08), B.make_params((8, 8, 8), 1.0, float("inf")),
                B.make_params((8, 8, 8), 1.0, 0.08, psi_kind=2), B.make_params((8, 8, 8), 1.0, 0.08, precision=7),
                B.make_params((8, 8, 8), 1.0, 0.08, max_particles=-1),
                B.make_params((8, 8, 8), 1.0, 0.08, max_particles=2),
                B.make_params((8, 8, 8), 1.0, 0.08, max_particles=2, max_radius=4.0)):
        assert lib.lb_workspace_bytes(C.byref(bad)) == 0
    # the largest boxes: one population plane (N values of 8 bytes) must stay below 4 GiB
    big = lib.lb_workspace_bytes(C.byref(B.make_params((1024, 1024, 511), 1.0, 0.08)))
    assert big >= 2 * 2 * 19 * 1024 * 1024 * 511 * 8
    for dims in ((1024, 1024, 512), (2 ** 31 - 1, 2 ** 31 - 1, 2 ** 31 - 1), (2 ** 20, 2 ** 20, 3)):
        assert lib.lb_workspace_bytes(C.byref(B.make_params(dims, 1.0, 0.08))) == 0
    # reduced storage needs less memory
    n16 = lib.lb_workspace_bytes(C.byref(B.make_params((32, 32, 64), 1.0, 0.08, precision="fp16_dev")))
    assert n16 < n / 2


def test_create_rejects_bad_arguments_without_gpu(lib):
    from paper_1109_3277_amd import binding as B
    h = C.c_void_p()
    bad = B.make_params((8, 8, 2), 1.0, 0.08)
    assert lib.lb_create(C.byref(bad), C.c_void_p(256), 1 << 20, None, C.byref(h)) == B.LB_EINVAL
    assert not h.value
    assert b"dimension" in lib.lb_last_error(None)
    ok = B.make_params((8, 8, 8), 1.0, 0.08)
    assert lib.lb_create(C.byref(ok), None, 1 << 20, None, C.byref(h)) == B.LB_EINVAL
    need = lib.lb_workspace_bytes(C.byref(ok))
    assert lib.lb_create(C.byref(ok), C.c_void_p(256), need - 1, None, C.byref(h)) == B.LB_ENOMEM
    assert lib.lb_create(C.byref(ok), C.c_void_p(256 + 8), need, None, C.byref(h)) == B.LB_EINVAL
    assert lib.lb_create(None, C.c_void_p(256), need, None, C.byref(h)) == B.LB_EINVAL


def test_null_handle_calls_are_rejected(lib):
    from paper_1109_3277_amd import binding as B
    assert lib.lb_step(None, 1) == B.LB_EINVAL
    assert lib.lb_init_fields(None, None, None, None) == B.LB_EINVAL
    assert lib.lb_set_particle_motion(None, 0, None, None, None) == B.LB_EINVAL
    assert lib.lb_num_particles(None) == B.LB_EINVAL
    lib.lb_destroy(None)


def test_batch_workspace_and_create_validate(lib):
    from paper_1109_3277_amd import binding as B
    a = B.make_params((32, 32, 64), 1.0, 0.08, precision="fp32", max_particles=1, max_radius=8.0)
    b = B.make_params((40, 48, 96), 1.0, 0.08, precision="fp32", max_particles=1, max_radius=12.0)
    arr = (B.lb_params * 2)(a, b)
    n = lib.lb_batch_workspace_bytes(2, arr)
    assert n >= lib.lb_workspace_bytes(C.byref(a)) + lib.lb_workspace_bytes(C.byref(b))
    assert lib.lb_batch_workspace_bytes(0, arr) == 0
    assert lib.lb_batch_workspace_bytes(2, None) == 0
    mixed = (B.lb_params * 2)(a, B.make_params((32, 32, 64), 1.0, 0.08, precision="fp64"))
    assert lib.lb_batch_workspace_bytes(2, mixed) == 0
    bad = (B.lb_params * 2)(a, B.make_params((32, 32, 2), 1.0, 0.08, precision="fp32"))
    assert lib.lb_batch_workspace_bytes(2, bad) == 0
    h = C.c_void_p()
    assert lib.lb_create_batch(2, arr, None, n, None, C.byref(h)) == B.LB_EINVAL
    assert lib.lb_create_batch(2, arr, C.c_void_p(256), n - 1, None, C.byref(h)) == B.LB_ENOMEM
    assert lib.lb_create_batch(2, arr, C.c_void_p(256 + 8), n, None, C.byref(h)) == B.LB_EINVAL
    assert lib.lb_create_batch(2, mixed, C.c_void_p(256), n, None, C.byref(h)) == B.LB_EINVAL
    assert b"precision" in lib.lb_last_error(None)
    assert lib.lb_batch_size(None) == B.LB_EINVAL
    assert lib.lb_batch_system(None, 0, C.byref(h)) == B.LB_EINVAL
    assert lib.lb_batch_tune(None, None) == B.LB_EINVAL


def test_per_system_calls_reject_bad_handles(lib):
    from paper_1109_3277_amd import binding as B
    assert lib.lb_init_fields_sys(None, 0, None, None, None) == B.LB_EINVAL
    assert lib.lb_add_ellipsoids_sys(None, 0, 0, None, None, None, None, None) == B.LB_EINVAL
    assert lib.lb_read_fields_sys(None, 0, None, None, None, None) == B.LB_EINVAL
    assert lib.lb_read_particles_sys(None, 0, None, None, None, None, None, None) == B.LB_EINVAL
    assert lib.lb_stats_sys(None, 0, None) == B.LB_EINVAL


def test_probe_copy_lives_outside_the_method_library(lib):
    """The counter-calibration copy is a separate library, not part of the ABI."""
    assert not hasattr(lib, "lb_probe_copy")
    from paper_1109_3277_amd import build
    if not os.path.exists(build.PROBE_LIB):
        build.build()
    probe = C.CDLL(build.PROBE_LIB)
    assert hasattr(probe, "lbe_probe_copy")


def test_pair_interactions_reject_bad_handles(lib):
    from paper_1109_3277_amd import binding as B
    assert lib.lb_set_pair_interactions(None, 1, 100.0, 2.0 / 3.0) == B.LB_EINVAL


def test_device_readout_rejects_bad_handles(lib):
    from paper_1109_3277_amd import binding as B
    assert lib.lb_read_fields_dev(None, None, None, None, None) == B.LB_EINVAL


def test_domain_size_and_noalloc_stats_reject_bad_handles(lib):
    """Eq. (12) observable and the allocation-free diagnostics: no handle or
    no output is rejected before any GPU work."""
    from paper_1109_3277_amd import binding as B
    out = (C.c_double * 8)()
    assert lib.lb_domain_size(None, out) == B.LB_EINVAL
    assert lib.lb_stats_noalloc(None, None) == B.LB_EINVAL
