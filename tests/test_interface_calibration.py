"""The walls/interface and dielectric-drop workloads start from the coexisting bulk
densities of a flat Shan-Chen interface at G = 4 (WALL_RHO_MAJ, WALL_RHO_MIN).  They are
what oracle/calibrate_interface.py prints: a 2 x 2 x 64 column relaxed on the oracle until
the profile stops changing.  The check keeps the constants tied to that run, and to the
symmetry of the mixture (each phase's minority density equals the other's)."""
import pytest

from oracle.calibrate_interface import calibrate
from paper_1712_08494_amd import workloads as wl


def test_interface_densities_are_the_calibrated_ones():
    a_maj, b_min, a_min, b_maj = calibrate(steps=20000)
    assert a_maj == pytest.approx(b_maj, abs=1e-7) and b_min == pytest.approx(a_min, abs=1e-7)
    assert abs(a_maj - wl.WALL_RHO_MAJ) < 1e-5 and abs(b_min - wl.WALL_RHO_MIN) < 1e-5, (a_maj, b_min)
