"""The shape measurement of the dielectric-drop validation on synthetic drops whose half-
lengths are known: tanh profiles around ellipses with a = 30, b = 33 and a circle of
radius 32, centred between sites or on a site."""
import numpy as np
import pytest

from tests.test_gpu_okonski import pressure, shape


@pytest.mark.parametrize("a,b,centre", [(30.0, 33.0, 63.5), (32.0, 32.0, 63.5), (31.0, 32.5, 64.0)])
def test_shape_recovers_half_lengths(a, b, centre):
    n = 128
    z, y = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    # distance to the ellipse along the radial direction, in sites (close to the normal
    # distance for these nearly round shapes); the profile is symmetric around c = 0
    th = np.arctan2(z - centre, y - centre)
    r_edge = a * b / np.sqrt((b * np.cos(th)) ** 2 + (a * np.sin(th)) ** 2)
    d = np.hypot(y - centre, z - centre) - r_edge
    inside = (0.5 * (1.0 - np.tanh(d / 2.0)))[:, :, None] * np.ones((1, 1, 4))
    ra = 1.41401 - 1.40148 * inside
    rb = 0.01253 + 1.40148 * inside
    ga, gb, (yc, zc) = shape(ra, rb)
    assert abs(yc - centre) < 1e-6 and abs(zc - centre) < 1e-6
    assert abs(ga - a) < 0.01 and abs(gb - b) < 0.01


def test_pressure_equation_of_state():
    # pure phases: cs^2 rho (psi_b = 0 and psi_a = 0 at zero density)
    assert pressure(np.array(1.2), np.array(0.0), 4.0) == pytest.approx(0.4)
    # a mixed site adds cs^2 G psi_a psi_b
    ra, rb, G = 0.7, 0.4, 4.0
    want = (ra + rb) / 3 + G * (1 - np.exp(-ra)) * (1 - np.exp(-rb)) / 3
    assert pressure(np.array(ra), np.array(rb), G) == pytest.approx(want, rel=1e-15)
