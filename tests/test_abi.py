"""The C interface: every function declared in include/lbm.h is exported by
the built library and bound by the Python layer (no GPU needed)."""
import ctypes
import os
import re

from paper_1004_4414_amd import lbm

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "lbm.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(lb_[a-z_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for core in ("lb_create", "lb_add_particles", "lb_step", "lb_observables"):
        assert core in names


def test_library_exports_every_declared_function():
    assert os.path.exists(lbm.LIB_PATH), "build the HIP library first"
    L = ctypes.CDLL(lbm.LIB_PATH)
    for name in declared_functions():
        assert hasattr(L, name), name


def test_binding_covers_every_declared_function():
    assert sorted(lbm.ENTRY_POINTS) == declared_functions()
    lbm.lib()


def test_host_only_calls():
    p = lbm.make_params(dict(lbm_defaults()), "fp32")
    assert p.nx == 16
    assert abs(lbm.contact_angle_to_color(135.0) - 45.0 / 442.0) < 1e-15
    assert lbm.footprint_bytes(lbm_defaults(nx=256, ny=256, nz=256), 4806, 5.0) > 5 * 2 ** 30


def lbm_defaults(**kw):
    from paper_1004_4414_amd import workloads as W
    return W.params(**kw)
