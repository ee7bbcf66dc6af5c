"""CPU checks of the C ABI: the built library loads without a GPU and exports every
function that include/ek.h declares; the host-only lattice table is a valid D3Q19 set
equal (as a set of velocity/weight pairs) to the oracle's independent table."""
import os
import re

import numpy as np

from oracle import oracle as orc
from paper_1712_08494_amd import ek

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "ek.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(ek_[a-z_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    L = ek.load()
    names = declared_functions()
    assert "ek_init" in names and "ek_step" in names and "ek_poisson" in names and "ek_observables" in names
    for n in names:
        assert hasattr(L, n), n
    assert set(names) == set(ek.EXPORTS)


def test_lattice_table_matches_oracle_set():
    cg, wg = ek.lattice()
    co, wo = orc.lattice()
    assert sorted(zip(map(tuple, cg.tolist()), wg.tolist())) == sorted(zip(map(tuple, co.tolist()), wo.tolist()))
    # opposite velocities are 18 - d in the library's order
    for d in range(19):
        assert np.array_equal(cg[18 - d], -cg[d])


def test_status_strings():
    L = ek.load()
    assert L.ek_status_str(0) == b"ok"
    assert L.ek_status_str(ek.EK_ENOCONV).startswith(b"Poisson")
