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
    for n in ["mfpff_setup_mesh_levels", "mfpff_set_linearization", "mfpff_apply_jacobian", "mfpff_vcycle",
              "mfpff_gmres_solve", "mfpff_residual", "mfpff_residual_param_vjp", "mfpff_newton_step",
              "mfpff_destroy", "mfpff_last_error", "mfpff_sizes"]:
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
    for field, bad in [("dim", 5), ("n_levels", 0), ("cheb_degree", 0), ("restart", 0), ("vcycle_prec", 7),
                       ("split", 3), ("pdas_project", 2), ("contraction", 2), ("slit", 2), ("kappa", -1.0), ("kappa", 1.0),
                       ("kappa", float("nan"))]:
        p = binding.make_problem(2, [(4, 1), (8, 1)], eps=0.25)
        setattr(p, field, bad)
        assert lib.mfpff_setup_mesh_levels(ctypes.byref(p), None, ctypes.byref(h)) == 1
    p = binding.make_problem(2, [(4, 1), (8, 2)], eps=0.25)       # neither an h- nor a p-step
    assert lib.mfpff_setup_mesh_levels(ctypes.byref(p), None, ctypes.byref(h)) == 1
    p = binding.make_problem(2, [(7, 1)], eps=0.25, slit=True)     # the slit needs an even N
    assert lib.mfpff_setup_mesh_levels(ctypes.byref(p), None, ctypes.byref(h)) == 1
    p = binding.make_problem(2, [(3, 1), (6, 1)], eps=0.25, slit=True)  # ... on every level
    assert lib.mfpff_setup_mesh_levels(ctypes.byref(p), None, ctypes.byref(h)) == 1
    p = binding.make_problem(2, [(8, 5)], eps=0.25)                # degree above 4
    assert lib.mfpff_setup_mesh_levels(ctypes.byref(p), None, ctypes.byref(h)) == 1
    assert lib.mfpff_setup_mesh_levels(None, None, ctypes.byref(h)) == 1
    assert good.dim == 2


def test_null_context_paths(lib):
    from paper_2005_00331_amd import binding
    binding.load_library()
    L = binding._lib
    assert L.mfpff_last_error(None) == b"null context"
    L.mfpff_destroy(None)
    d = binding.LevelDesc()
    assert L.mfpff_level_info(None, 0, ctypes.byref(d)) == 1
    nn, nd = ctypes.c_size_t(), ctypes.c_size_t()
    assert L.mfpff_sizes(None, 0, ctypes.byref(nn), ctypes.byref(nd)) == 1
    assert L.mfpff_debug_bounds_hits() == -1   # the regular library has no index checks


def _c_struct_fields(name):
    """(type, field) pairs of a typedef struct in the header, arrays as (type, field, length)."""
    txt = open(HEADER).read()
    end = re.search(r"\}\s*" + name + ";", txt).start()
    body = txt[txt.rindex("typedef struct {", 0, end) + len("typedef struct {"):end]
    body = re.sub(r"/\*.*?\*/", "", body, flags=re.S)
    out = []
    for decl in body.split(";"):
        decl = " ".join(decl.split())
        if not decl:
            continue
        m = re.match(r"(unsigned long long|long long|double|int|mfpff_\w+) (.*)", decl)
        assert m, decl
        for v in m.group(2).split(","):
            v = v.strip()
            a = re.match(r"(\w+)\[(\w+)\]", v)
            out.append((m.group(1), a.group(1), a.group(2)) if a else (m.group(1), v))
    return out


def test_problem_structure_matches_header():
    """The ctypes structures mirror the header field by field, in order and type."""
    import ctypes as C
    from paper_2005_00331_amd import binding
    ctype = {"int": C.c_int, "double": C.c_double, "unsigned long long": C.c_ulonglong, "long long": C.c_longlong,
             "mfpff_pdas_info": binding.PdasInfo}
    for cname, pyst in (("mfpff_problem", binding.Problem), ("mfpff_solve_info", binding.SolveInfo),
                        ("mfpff_level_desc", binding.LevelDesc), ("mfpff_pdas_info", binding.PdasInfo),
                        ("mfpff_load_info", binding.LoadInfo)):
        cf = _c_struct_fields(cname)
        pf = pyst._fields_
        assert len(cf) == len(pf), cname
        for c, (pname, ptype) in zip(cf, pf):
            assert pname.rstrip("_") == c[1], (cname, pname, c)
            if len(c) == 3:
                n = int(c[2]) if c[2].isdigit() else getattr(binding, c[2].replace("MFPFF_", ""))
                assert ptype._type_ is ctype[c[0]] and ptype._length_ == n, (cname, pname)
            else:
                assert ptype is ctype[c[0]], (cname, pname, c[0])
