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


def test_traffic_record_matches_the_kernel_source():
    """The counter summary of the headline kernel is read back with its figures only while
    the kernel source is the one it was taken on; the committed record is of the current
    source, and its per-launch bytes are its per-site fetch and write counts (KiB per
    dispatch, scaled by the copy calibration) times the sites."""
    import re
    recorded, src = bench.measured_traffic("k_fused", "colloids", 256, "fp32")
    assert recorded is not None, src
    rec = {}
    with open(src) as fh:
        for line in fh:
            m = re.match(r"- (\w+): (.+)", line.strip())
            if m:
                rec[m.group(1)] = m.group(2)
    scaled = (float(rec["fetch_kib_per_launch"]) * float(rec["fetch_scale"])
              + float(rec["write_kib_per_launch"]) * float(rec["write_scale"])) * 1024
    assert abs(scaled - recorded) <= 1e-3 * recorded
    per_site = recorded / int(rec["sites"])
    assert bench.algorithmic_bytes("k_fused", 4, True, 1) < per_site < 3 * bench.algorithmic_bytes("k_fused", 4, True, 1)


def test_more_than_one_gpu_is_refused():
    import os
    import subprocess
    import sys
    root = os.path.dirname(os.path.abspath(bench.__file__))
    p = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert p.returncode == 2
    assert "one GPU" in p.stderr and p.stdout == ""
