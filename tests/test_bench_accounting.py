"""bench.py's byte accounting, which its roofline figures divide by the measured times: the
compulsory traffic per site of each pass (populations, ions and potential read and written
once, one byte of solid mask where there are solids, the Poisson row's potential, charge and
permittivity), counted from the storage sizes rather than re-typed."""
import bench


def test_algorithmic_bytes_per_site():
    for s, pops in ((4, 2 * 19 * 4), (8, 2 * 19 * 8)):
        ions, phi = 2 * s, 8
        # fused pass at tau = 1: populations written, ions read and written, potential read
        assert bench.algorithmic_bytes("k_fused", s, True, 0) == pops + 2 * ions + phi
        assert bench.algorithmic_bytes("k_fused", s, True, 1) == pops + 2 * ions + phi + 1
        # tau != 1 also reads the populations
        assert bench.algorithmic_bytes("k_fused", s, False, 0) == 2 * pops + 2 * ions + phi
        assert bench.algorithmic_bytes("k_moments", s, True, 1) == pops + 1
        sweep = 2 * 8 + s + s  # potential read and written, charge and permittivity read
        for k in ("k_sor", "k_sor_black_from", "k_mg_prolong_red_fine"):
            assert bench.algorithmic_bytes(k, s) == sweep / 2  # one colour of a sweep
        assert bench.algorithmic_bytes("k_sor_rb", s) == sweep
        assert bench.sweep_bytes(s) == sweep
        # the whole step outside the solve: populations and ions both ways, potential, mask
        assert bench.step_bytes(s, 1) == 2 * pops + 2 * ions + phi + 1
    assert bench.algorithmic_bytes("k_mg_smooth", 4) == 0.0  # intermediates are not counted
