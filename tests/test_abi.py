"""The C-ABI library: it loads, exports every function include/fv.h declares, and rejects
bad arguments on the host before touching a device (no compute calls here)."""
import ctypes as C
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fv.h")
LIB = os.path.join(ROOT, "paper_1912_07645_amd", "libfv.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = set(re.findall(r"\b(fv_[a-z0-9_]+)\s*\(", text))
    return sorted(names)


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ("fv_create", "fv_evolve", "fv_stats_accumulate", "fv_stats_read",
                 "fv_evolve_multi", "fv_destroy"):
        assert must in names


def test_library_exports_every_declared_symbol():
    assert os.path.exists(LIB), "build libfv.so first (python -m paper_1912_07645_amd.build)"
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True,
                         check=True).stdout
    exported = set(re.findall(r"\bT (fv_[a-z0-9_]+)", out))
    missing = [n for n in declared_functions() if n not in exported]
    assert not missing, missing
    lib = C.CDLL(LIB)
    for n in declared_functions():
        assert hasattr(lib, n)


def test_header_compiles_as_c():
    src = '#include "fv.h"\nint main(void){ return (int)sizeof(fv_grid) > 0 ? 0 : 1; }\n'
    r = subprocess.run(["gcc", "-std=c99", "-Wall", "-Werror", "-I", os.path.join(ROOT, "include"),
                        "-x", "c", "-", "-fsyntax-only"], input=src, text=True, capture_output=True)
    assert r.returncode == 0, r.stderr


def test_argument_validation_without_device():
    import paper_1912_07645_amd.fv as fv
    eq = fv.make_equation("euler")
    bad_grids = [fv.make_grid(0, (8,)), fv.make_grid(4, (8,)), fv.make_grid(1, (0,)),
                 fv.make_grid(1, (8, 2)), fv.make_grid(2, (8, 8), hi=(1.0, 0.0))]
    for g in bad_grids:
        with pytest.raises(fv.FVError) as e:
            fv.fv_create(g, eq, 0, 0, 0)
        assert e.value.status == fv.FV_EINVAL
    g = fv.make_grid(1, (8,))
    with pytest.raises(fv.FVError) as e:
        fv.fv_create(g, fv.make_equation("advection"), fv.FLUX["hllc"], 0, 0)
    assert e.value.status == fv.FV_ENOTSUP
    with pytest.raises(fv.FVError) as e:
        fv.fv_create(g, fv.make_equation("euler", gamma=1.0), 0, 0, 0)
    assert e.value.status == fv.FV_EINVAL
    for flux, recon, integ in ((7, 0, 0), (0, 4, 0), (0, 0, 3), (-1, 0, 0)):
        with pytest.raises(fv.FVError) as e:
            fv.fv_create(g, eq, flux, recon, integ)
        assert e.value.status == fv.FV_EINVAL
    with pytest.raises(fv.FVError) as e:                 # entropy-conservative: Burgers, Euler
        fv.fv_create(g, fv.make_equation("advection"), fv.FLUX["ec"], 0, 0)
    assert e.value.status == fv.FV_ENOTSUP
    with pytest.raises(fv.FVError) as e:                 # fourth-order EC: cell values only
        fv.fv_create(g, eq, fv.FLUX["ec4"], fv.RECON["muscl_minmod"], 0)
    assert e.value.status == fv.FV_ENOTSUP
    mhd = fv.make_equation("mhd", gamma=5.0 / 3.0)
    for flux in ("hllc", "roe", "godunov", "ec", "ec4"):  # ideal MHD: Rusanov and HLL only
        with pytest.raises(fv.FVError) as e:
            fv.fv_create(g, mhd, fv.FLUX[flux], 0, 0)
        assert e.value.status == fv.FV_ENOTSUP
    with pytest.raises(fv.FVError) as e:
        fv.fv_create(g, fv.make_equation("mhd", gamma=1.0), 0, 0, 0)
    assert e.value.status == fv.FV_EINVAL
    with pytest.raises(fv.FVError) as e:
        fv.fv_create(g, fv.make_equation(5), 0, 0, 0)
    assert e.value.status == fv.FV_EINVAL
    with pytest.raises(fv.FVError) as e:
        fv.fv_create(g, fv.make_equation("swe"), fv.FLUX["godunov"], 0, 0)
    assert e.value.status == fv.FV_ENOTSUP
    assert fv.fv_num_fields(None) == -1
    with pytest.raises(fv.FVError):
        fv.fv_evolve(None, None, 1, None, 1.0, 0.5, 10)


def test_product_path_has_no_cpu_fallback():
    """The binding never imports the oracle, and the oracle never imports the binding."""
    pkg = os.path.join(ROOT, "paper_1912_07645_amd")
    for f in os.listdir(pkg):
        if f.endswith(".py"):
            text = open(os.path.join(pkg, f)).read()
            assert "import oracle" not in text and "from oracle" not in text, f
    for f in os.listdir(os.path.join(ROOT, "oracle")):
        if f.endswith((".py", ".c")):
            text = open(os.path.join(ROOT, "oracle", f)).read()
            assert "paper_1912_07645_amd" not in text, f


def test_functionals_reject_null_arguments_without_device():
    import paper_1912_07645_amd.fv as fv
    L = fv.lib
    pts = (C.c_int64 * 1)(0)
    assert L.fv_point_pdf(None, None, 1, 0, 1, pts, 0.0, 1.0, 4, None) == fv.FV_EINVAL
    assert L.fv_joint_pdf(None, None, 1, 0, 0, 1, pts, 0.0, 1.0, 0.0, 1.0, 4, None) == fv.FV_EINVAL
    assert L.fv_structure_shell(None, None, 1, 2, 2, 0, None) == fv.FV_EINVAL
