"""Host-side checks of the C ABI (no kernel launches): the library loads,
exports every entry point the header declares, and rejects bad problem
descriptions before touching a device."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mfpff.h")
LIB = os.path.join(ROOT, "paper_2005_00331_amd", "libmfpff.so")


def declared():
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"\b(mfpff_[a-z_]+)\s*\(", txt)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.fail("libmfpff.so is not built; run __graft_entry__.build()")
    import torch  # noqa: F401  (same HIP runtime as torch)
    return ctypes.CDLL(LIB)


def test_header_declares_the_boundary():
    names = declared()
    for n in ["mfpff_create", "mfpff_set_linearization", "mfpff_apply_jacobian", "mfpff_vcycle",
              "mfpff_gmres_solve", "mfpff_residual", "mfpff_residual_param_vjp", "mfpff_newton_step",
              "mfpff_destroy", "mfpff_last_error"]:
        assert n in names


def test_library_exports_every_declared_symbol(lib):
    for name in declared():
        assert hasattr(lib, name), name


def test_binding_covers_every_symbol():
    from paper_2005_00331_amd import binding
    assert sorted(binding.EXPORTS) == declared()


def test_invalid_problems_rejected_without_device(lib):
    from paper_2005_00331_amd import binding
    binding.load_library()
    lib = binding._lib
    h = ctypes.c_void_p()
    good = binding.make_problem(2, [(4, 1), (8, 1)], eps=0.25)
    for field, bad in [("dim", 5), ("n_levels", 0), ("cheb_degree", 0), ("restart", 0), ("vcycle_prec", 7)]:
        p = binding.make_problem(2, [(4, 1), (8, 1)], eps=0.25)
        setattr(p, field, bad)
        assert lib.mfpff_create(ctypes.byref(p), None, ctypes.byref(h)) == 1
    p = binding.make_problem(2, [(4, 1), (8, 2)], eps=0.25)       # neither an h- nor a p-step
    assert lib.mfpff_create(ctypes.byref(p), None, ctypes.byref(h)) == 1
    p = binding.make_problem(2, [(8, 5)], eps=0.25)                # degree above 4
    assert lib.mfpff_create(ctypes.byref(p), None, ctypes.byref(h)) == 1
    assert lib.mfpff_create(None, None, ctypes.byref(h)) == 1
    assert good.dim == 2


def test_null_context_paths(lib):
    from paper_2005_00331_amd import binding
    binding.load_library()
    L = binding._lib
    assert L.mfpff_last_error(None) == b"null context"
    L.mfpff_destroy(None)
    d = binding.LevelDesc()
    assert L.mfpff_level_info(None, 0, ctypes.byref(d)) == 1
