"""Values the paper prints, kept as cited fixtures under tests/golden/, against the workload
generator and the oracle's element rigidities."""
import json
import os

import numpy as np
import pytest

from oracle import solver, beam
from workloads import make_config

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def test_table1_robot_section_drives_the_shaft_elements():
    """The batched workload's robots: the elements proximal to the flexible tip carry Table I's
    robot section (EA = E A, EI = E I, GJ = E/(2(1+nu)) 2I), the distal 70 mm the tube
    section of the robot's own radii and modulus."""
    with open(os.path.join(GOLDEN, "table1_robot.json")) as f:
        g = json.load(f)
    rb, _, _ = make_config(3)
    assert rb.shaft_E == g["young_modulus_Pa"]
    assert rb.shaft_A == g["area_m2"]
    assert rb.shaft_I == g["second_moment_m4"]
    assert rb.tip_len == g["flexible_tip_length_m"]
    EA_t, EI_t, GJ_t = beam.section_stiffness(rb.r_out, rb.r_in, rb.E, rb.nu)
    for b in (0, 1, 4095):
        EA, EI, GJ = solver.element_rigidities(rb, b)
        n_e = int(rb.n_elem[b])
        l0 = rb.length[b] / n_e
        tip = (np.arange(n_e) + 0.5) * l0 >= rb.length[b] - g["flexible_tip_length_m"]
        assert tip.any() and (~tip).any()
        assert np.all(EA[~tip] == pytest.approx(510e6 * 5.551e-6, rel=1e-15))
        assert np.all(EI[~tip] == pytest.approx(510e6 * 5.041e-12, rel=1e-15))
        assert np.all(GJ[~tip] == pytest.approx(510e6 / (2 * (1 + rb.nu)) * 2 * 5.041e-12, rel=1e-15))
        assert np.all(EA[tip] == EA_t) and np.all(EI[tip] == EI_t) and np.all(GJ[tip] == GJ_t)
        # the tip section is much softer than the shaft
        assert EI_t < 0.1 * 510e6 * 5.041e-12
