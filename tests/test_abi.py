"""The C ABI: libvi.so loads without a GPU and exports every function that
include/vi.h declares; the binding's signature table covers them all; the
host-side argument checks reject bad parameters without touching a GPU."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "vi.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\**\s+\**(vi_[a-z0-9_]+)\s*\(",
                       src, flags=re.M)
    return sorted(set(names))


@pytest.fixture(scope="module")
def libvi():
    from paper_1503_05528_amd import build
    if not os.path.exists(build.LIB):
        build.build()
    from paper_1503_05528_amd import vi
    return vi.lib()


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("vi_create", "vi_nnf_search", "vi_reconstruct", "vi_inpaint_level",
                     "vi_inpaint", "vi_destroy"):
        assert required in names


def test_library_exports_every_declared_symbol(libvi):
    for name in declared_functions():
        assert hasattr(libvi, name), name


def test_binding_covers_the_header():
    from paper_1503_05528_amd import vi
    assert sorted(vi.SIGNATURES) == declared_functions()


def test_params_default_and_validation_on_host(libvi):
    from paper_1503_05528_amd import vi
    p = vi.default_params()
    assert (p.lambda_, p.pm_iters, p.n_jf, list(p.jf_steps)[:3]) == (50, 10, 3, [4, 2, 1])
    # the pass form is the library's choice unless set; below -1 is refused
    assert p.wide_pass_max == -1 and p.reduce_dims == 0
    assert vi.footprint_bytes(vi.default_params(wide_pass_max=0), 854, 480, 100, 0.05) > 0
    assert vi.footprint_bytes(vi.default_params(wide_pass_max=-2), 854, 480, 100, 0.05) == 0
    assert vi.footprint_bytes(p, 854, 480, 100, 0.05) > 854 * 480 * 100 * 36
    bad = vi.default_params(patch=(3, 3, 3))
    assert vi.footprint_bytes(bad, 854, 480, 100, 0.05) == 0
    bad = vi.default_params(levels=6)
    assert vi.footprint_bytes(bad, 64, 64, 10, 0.05) == 0  # coarsest level too small
    # volumes: at least one patch per axis, fewer than 2^31 voxels (32-bit
    # voxel indices); the largest admissible one is sized without overflow
    assert vi.footprint_bytes(p, 4, 480, 100, 0.05) == 0
    assert vi.footprint_bytes(p, 32767, 32767, 5, 0.05) == 0
    big = vi.footprint_bytes(p, 2048, 1024, 1023, 0.01)
    assert big > 2048 * 1024 * 1023 * 36
    h = C.c_void_p()
    # null inputs are rejected before any device work
    st = libvi.vi_create(C.byref(h), C.byref(p), 32, 32, 8, None, None, None)
    assert st == -1 and not h.value
    assert b"null" in libvi.vi_last_error()
