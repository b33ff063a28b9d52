"""Host-only checks of the C ABI: the library loads and exports every entry
point that include/gpnufft.h declares; host-only calls behave as documented."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "gpnufft.h")
LIB = os.path.join(ROOT, "paper_2407_03608_amd", "libgpnufft.so")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_\s\*]*?\b(gp_[a-z0-9_]+)\s*\(", src, flags=re.M)
    return sorted(set(names))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        from paper_2407_03608_amd import build
        build.build(verbose=False)
    return ctypes.CDLL(LIB)


def test_header_declares_the_boundary():
    names = declared_functions()
    for n in ["gp_plan", "gp_matvec", "gp_cg_solve", "gp_posterior_mean", "gp_plan_destroy",
              "gp_last_error", "gp_plan_info", "gp_plan_query", "gp_opts_init",
              "gp_cg_solve_refined", "gp_plan_set_stream"]:
        assert n in names


def test_every_declared_symbol_is_exported(lib):
    for n in declared_functions():
        assert hasattr(lib, n), f"{n} declared in gpnufft.h but not exported"


def test_binding_covers_the_exports():
    from paper_2407_03608_amd import gp
    assert sorted(gp.EXPORTS) == declared_functions()


def test_opts_init_defaults_and_structure_sizes(lib):
    from paper_2407_03608_amd import gp
    o = gp.GpOpts()
    lib.gp_opts_init.argtypes = [ctypes.POINTER(gp.GpOpts)]
    assert lib.gp_opts_init(ctypes.byref(o)) == 0
    assert o.precision == gp.GP_FP64 and o.n_sigma == -1 and o.n_t == -1
    assert o.M == 0 and o.dw == 0.0 and not o.stream
    lib.gp_opts_init.argtypes = [ctypes.c_void_p]
    assert lib.gp_opts_init(None) == gp.GP_EINVAL


def test_invalid_arguments_fail_before_touching_the_device(lib):
    from paper_2407_03608_amd import gp
    lib.gp_plan.argtypes = [ctypes.c_int, ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p,
                            ctypes.c_void_p, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                            ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p)]
    lib.gp_last_error.restype = ctypes.c_char_p
    h = ctypes.c_void_p()
    dummy = ctypes.c_void_p(16)
    assert lib.gp_plan(4, 10, dummy, dummy, dummy, 1.5, 0.1, 1e-6, None, ctypes.byref(h)) == gp.GP_EINVAL
    assert b"d must be" in lib.gp_last_error()
    assert lib.gp_plan(2, 0, dummy, dummy, dummy, 1.5, 0.1, 1e-6, None, ctypes.byref(h)) == gp.GP_EINVAL
    assert lib.gp_plan(2, 10, dummy, dummy, dummy, -1.0, 0.1, 1e-6, None, ctypes.byref(h)) == gp.GP_EDOMAIN
    assert lib.gp_plan(2, 10, dummy, dummy, dummy, 1.5, -0.1, 1e-6, None, ctypes.byref(h)) == gp.GP_EDOMAIN
    assert lib.gp_plan(2, 10, dummy, dummy, dummy, 1.5, 0.1, 0.0, None, ctypes.byref(h)) == gp.GP_EDOMAIN
    assert lib.gp_plan(2, 10, None, dummy, dummy, 1.5, 0.1, 1e-6, None, ctypes.byref(h)) == gp.GP_EINVAL
    lib.gp_matvec.argtypes = [ctypes.c_void_p] * 3 + [ctypes.c_int]
    assert lib.gp_matvec(None, None, None, 0) == gp.GP_EINVAL
    lib.gp_plan_destroy.argtypes = [ctypes.c_void_p]
    assert lib.gp_plan_destroy(None) == 0
