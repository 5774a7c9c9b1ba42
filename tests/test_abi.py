"""CPU checks of the C ABI boundary: the library loads without a GPU and exports
every entry point that include/accfem.h declares."""
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared():
    h = open(os.path.join(ROOT, "include", "accfem.h")).read()
    h = re.sub(r"/\*.*?\*/", "", h, flags=re.S)
    return sorted(set(re.findall(r"\b(fem_[a-z_]+)\s*\(", h)))


def test_header_declares_the_boundary():
    names = declared()
    for f in ("fem_create", "fem_set_actuation", "fem_set_lumen", "fem_solve", "fem_contacts"):
        assert f in names


def test_library_exports_every_declared_symbol():
    from paper_2503_06922_amd import fem
    if not os.path.exists(fem._LIB_PATH):
        pytest.fail("libaccfem.so is not built (run __graft_entry__.build())")
    L = fem.lib()
    missing = [n for n in declared() if not hasattr(L, n)]
    assert not missing, missing
    assert set(declared()) <= set(fem.EXPORTED)


def test_create_rejects_bad_parameters_without_touching_the_gpu():
    """Argument validation runs before any device call, so it is testable on the CPU."""
    import numpy as np
    from paper_2503_06922_amd import fem
    from workloads import robots_for_config
    rb = robots_for_config(0)
    base = fem.params_from_batch(rb)
    for bad in ({"E": -1.0}, {"r_in": 2e-3}, {"contact_capacity": 0}, {"max_newton": 0},
                {"beta0": 0.0}, {"n_elem": np.array([0], np.int32)}, {"cable_angle": np.zeros(9)},
                {"guide_len": 0.5, "base_dir": np.array([[0.0, 0.6, 0.8]])}):
        p = dict(base)
        p.update(bad)
        with pytest.raises(fem.FemError) as e:
            fem.Context(p)
        assert e.value.status == fem.FEM_E_INVAL
