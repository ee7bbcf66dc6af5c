"""Bulk densities of a flat Shan-Chen interface at G = 4 (test infrastructure).

Runs the oracle on a periodic 2 x 2 x 64 column with fluid a in one half and fluid b in the
other (mean total density 1.386, tanh profiles of width 2, no ions, no field) for 35000
steps, after which the profile no longer changes (below 1e-12), and prints the majority and
minority densities in the middle of each bulk.  The walls/interface and dielectric-drop workloads start from these
values (WALL_RHO_MAJ, WALL_RHO_MIN in paper_1712_08494_amd/workloads.py), so their
interfaces start close to the equilibrium profile.

    python -m oracle.calibrate_interface
"""
import numpy as np

from oracle import oracle as orc
from paper_1712_08494_amd import workloads as wl


def calibrate(G=4.0, nz=64, steps=35000, total=1.386, lo=0.026):
    cfg = wl.EKConfig(2, 2, nz, G=G, precision="fp64")
    z = np.arange(nz)
    s = 0.5 * (np.tanh((z - nz / 4) / 2.0) - np.tanh((z - 3 * nz / 4) / 2.0))  # 1 in the middle half
    hi = total - lo
    ra = lo + (hi - lo) * (1 - s)
    rb = lo + (hi - lo) * s
    inp = wl.uniform(cfg, 0.5, 0.5, 0.0, 0.0)
    inp.rho_a = np.broadcast_to(ra[:, None, None], (nz, 2, 2)).copy()
    inp.rho_b = np.broadcast_to(rb[:, None, None], (nz, 2, 2)).copy()
    o = orc.Oracle(cfg, inp)
    o.step(steps)
    a, b = o.field("rho_a")[:, 0, 0], o.field("rho_b")[:, 0, 0]
    return a[0], b[0], a[nz // 2], b[nz // 2]


if __name__ == "__main__":
    a_maj, b_min, a_min, b_maj = calibrate()
    print(f"fluid a bulk: rho_a {a_maj:.5f} rho_b {b_min:.5f}")
    print(f"fluid b bulk: rho_a {a_min:.5f} rho_b {b_maj:.5f}")
