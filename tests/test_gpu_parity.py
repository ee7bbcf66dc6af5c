"""GPU parity: the HIP library (through the C ABI) against the FP64 oracle on the same
seeded inputs, field by field, plus properties that hold at any size."""
import numpy as np
import pytest

from oracle import oracle as orc
from paper_1712_08494_amd import ek
from paper_1712_08494_amd import workloads as wl
from tests.parity import TOL, compare, max_rel, oracle_from_sim, phi_err

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU visible")
    ek.load()
    torch.cuda.init()
    yield


def _pair(cfg, inp):
    return ek.EKSim(cfg, inp), orc.Oracle(cfg, inp)


def _announce(msg):
    print(msg, flush=True)


# --------------------------------------------------------------------------------
# Mixture with noise (32^3 periodic, G = 3.6, SOR to 1e-10): FP64 and FP32.
# --------------------------------------------------------------------------------
@pytest.mark.parametrize("precision,solver", [("fp64", "mg"), ("fp64", "sor"), ("fp32", "auto")])
def test_mixture_noise_32(precision, solver):
    cfg, inp = wl.mixture_noise(n=32, precision=precision)
    cfg.poisson_solver = solver
    _announce(f"mixture_noise 32^3 {precision} {solver}")
    sim, o = _pair(cfg, inp)
    compare(sim, o, precision, "t=0")
    for t in (10, 40):
        sim.step(t)
        o.step(t)
        errs = compare(sim, o, precision, f"after {t}")
        _announce(f"  {precision} errors {errs}")


def test_ragged_tile_periodic():
    """Odd sizes that leave partial workgroups and partial XCD slabs."""
    cfg, inp = wl.mixture_noise(shape=(10, 7, 5), precision="fp64", G=4.4)
    _announce("ragged 10x7x5 fp64")
    sim, o = _pair(cfg, inp)
    sim.step(25)
    o.step(25)
    compare(sim, o, "fp64", "ragged")


def _sweep_colours(shape):
    """The lattice Gauss-Seidel colouring: red-black, or three colours when a periodic y or z
    axis has odd length >= 3 (the axis colour is the parity except 2 on its last index)."""
    nz, ny, nx = shape
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    if not ((ny >= 3 and ny % 2) or (nz >= 3 and nz % 2)):
        return (x + y + z) % 2, 2
    cy = np.where((ny >= 3) & (ny % 2 == 1) & (y == ny - 1), 2, y % 2)
    cz = np.where((nz >= 3) & (nz % 2 == 1) & (z == nz - 1), 2, z % 2)
    return (x % 2 + cy + cz) % 3, 3


@pytest.mark.parametrize("shape", [(10, 7, 5), (8, 9, 6), (6, 4, 7), (8, 6, 4)])
def test_sor_sweep_is_a_proper_colour_ordered_sweep(shape):
    """One SOR sweep of the library equals a colour-by-colour sweep computed here (periodic,
    FP64), and the colouring leaves no two neighbours in one pass: with an odd periodic axis
    two colours cannot, so the library sweeps three."""
    nx, ny, nz = shape
    cfg, inp = wl.mixture_noise(shape=shape, precision="fp64", G=4.4)
    cfg.poisson_solver = "sor"
    cfg.sor_omega = 1.25
    cfg.poisson_tol = 1e-2  # leave the starting potential far from converged
    _announce(f"one SOR sweep {nx}x{ny}x{nz} fp64")
    sim = ek.EKSim(cfg, inp)
    phi0, q, eps = sim.field("phi"), sim.field("q"), sim.field("eps")
    col, ncol = _sweep_colours(phi0.shape)
    for ax in range(3):
        if phi0.shape[ax] > 1:
            assert not np.any(col == np.roll(col, 1, axis=ax)), "neighbours share a colour"
    st, iters, _ = sim.poisson(1e-15, 1)
    assert iters == 1
    phi1 = sim.field("phi")
    ref, src = phi0.copy(), q - q.mean()
    for c in range(ncol):
        diag, off = np.zeros_like(ref), np.zeros_like(ref)
        for ax in range(3):
            if ref.shape[ax] == 1:
                continue
            for sh in (1, -1):
                ef = 0.5 * (eps + np.roll(eps, sh, axis=ax))
                diag += ef
                off += ef * np.roll(ref, sh, axis=ax)
        m = col == c
        ref[m] += cfg.sor_omega * ((off + src)[m] / diag[m] - ref[m])
    ref -= ref.mean()
    scale = np.abs(phi1).max()
    change = np.abs(phi1 - phi0).max() / scale
    err = np.abs(phi1 - ref).max() / scale
    _announce(f"  {ncol} colours: sweep changed phi by {change:.2e}, differs from the ordered sweep by {err:.2e}")
    assert change > 1e-6
    assert err < 1e-12
    sim.close()


# --------------------------------------------------------------------------------
# Charged walls and an interface with solvation and permittivity contrast.
# --------------------------------------------------------------------------------
@pytest.mark.parametrize("precision,solver", [("fp64", "mg"), ("fp64", "sor"), ("fp32", "auto")])
def test_walls_interface_small(precision, solver):
    cfg, inp = wl.walls_interface(shape=(16, 12, 32), precision=precision)
    cfg.poisson_solver = solver
    _announce(f"walls_interface 16x12x32 {precision} {solver}")
    sim, o = _pair(cfg, inp)
    compare(sim, o, precision, "t=0")
    sim.step(30)
    o.step(30)
    errs = compare(sim, o, precision, "after 30")
    _announce(f"  errors {errs}")


def test_walls_odd_periodic_axis_three_colour_sor():
    """Charged walls with an odd periodic y axis (7): no red-black colouring exists, the SOR
    solver sweeps in three colours; parity with the oracle after 30 steps (FP64)."""
    cfg, inp = wl.walls_interface(shape=(8, 7, 13), precision="fp64")
    _announce("walls_interface 8x7x13 fp64 (three-colour SOR)")
    sim, o = _pair(cfg, inp)
    compare(sim, o, "fp64", "t=0")
    sim.step(30)
    o.step(30)
    errs = compare(sim, o, "fp64", "after 30")
    _announce(f"  errors {errs}")


# --------------------------------------------------------------------------------
# Resolved charged spheres under a field.
# --------------------------------------------------------------------------------
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_colloids_small(precision):
    cfg, inp = wl.colloids(shape=(32, 32, 32), count=6, radius=3.5, precision=precision, field=(1e-3, 0, 0),
                           seed=7)
    if precision == "fp64":
        cfg.poisson_tol = 1e-12  # the particle force integrates the field; keep phi at the oracle's accuracy
    _announce(f"colloids 32^3 x6 {precision}")
    sim, o = _pair(cfg, inp)
    np.testing.assert_array_equal(sim.field("solid"), o.field("solid"))
    np.testing.assert_allclose(sim.field("psi_s"), o.field("psi_s"), rtol=0, atol=0)
    compare(sim, o, precision, "t=0")
    sim.step(20)
    o.step(20)
    errs = compare(sim, o, precision, "after 20")
    pg, po = sim.particles(), o.particles()
    # The net force on a sphere is a small difference of O(1) link momenta (about 700
    # links of magnitude 0.03 give a net force near 0.02): FP32 rounding of the
    # populations is amplified by that cancellation, hence 2e-3 in FP32.
    tol = 2e-3 if precision == "fp32" else 1e-8
    # displacement, velocity and the last step's force, relative to their largest component
    disp_g, disp_o = pg[:, 0:3] - inp.particles[:, 0:3], po[:, 0:3] - inp.particles[:, 0:3]
    perr = {"x": np.abs(disp_g - disp_o).max() / np.abs(disp_o).max(),
            "v": np.abs(pg[:, 3:6] - po[:, 3:6]).max() / np.abs(po[:, 3:6]).max(),
            "F": np.abs(pg[:, 6:9] - po[:, 6:9]).max() / np.abs(po[:, 6:9]).max()}
    _announce(f"  errors {errs} particles {perr}")
    for k, e in perr.items():
        assert e <= tol, (k, e)


def test_body_force_walls_fp64():
    cfg = wl.EKConfig(4, 2, 18, walls_z=True, body_accel=(1e-6, 0, 0), G=0.0, name="poiseuille")
    inp = wl.uniform(cfg, 0.5, 0.5, 0.0, 0.0)
    _announce("poiseuille 4x2x18 fp64")
    sim, o = _pair(cfg, inp)
    sim.step(500)
    o.step(500)
    compare(sim, o, "fp64", "poiseuille")
    np.testing.assert_allclose(sim.field("ux"), o.field("ux"), rtol=1e-9, atol=1e-15)


# --------------------------------------------------------------------------------
# Full size of the benchmark workload (128^3 walls + interface, FP32): one step from the
# library's state, against the oracle taking the same step from that state.
# --------------------------------------------------------------------------------
def test_walls_interface_128_one_step():
    cfg, inp = wl.walls_interface(n=128, precision="fp32")
    _announce("walls_interface 128^3 fp32: 3 steps then one-step parity")
    sim = ek.EKSim(cfg, inp)
    sim.step(3)
    o = oracle_from_sim(cfg, inp, sim)
    sim.step(1)
    o.step(1)
    errs = compare(sim, o, "fp32", "128^3 one step")
    _announce(f"  errors {errs}")


# --------------------------------------------------------------------------------
# Properties at any size
# --------------------------------------------------------------------------------
@pytest.mark.parametrize("precision,tol", [("fp64", 1e-12), ("fp32", 2e-6)])
def test_conservation(precision, tol):
    cfg, inp = wl.walls_interface(shape=(32, 32, 64), precision=precision)
    sim = ek.EKSim(cfg, inp)
    a = sim.observables()
    sim.step(50)
    b = sim.observables()
    for k in ["sum_rho_a", "sum_rho_b", "sum_n_plus", "sum_n_minus"]:
        assert abs(b[k] - a[k]) <= tol * abs(a[k]), (k, a[k], b[k])
    assert b["nonfinite"] == 0 and b["negative_ions"] == 0


def test_deterministic_bitwise():
    cfg, inp = wl.colloids(shape=(32, 32, 32), count=4, radius=3.0, precision="fp32", seed=11)
    out = []
    for _ in range(2):
        sim = ek.EKSim(cfg, inp)
        sim.step(10)
        out.append([sim.field(k) for k in ("rho_a", "n_plus", "phi")] + [sim.particles()])
        sim.close()
    for a, b in zip(*out):
        assert np.array_equal(a, b)


@pytest.mark.parametrize("walls", [False, True])
def test_multigrid_matches_sor_128(walls):
    """Both solvers reach the same discrete solution on the full-size lattice."""
    if walls:
        cfg, inp = wl.walls_interface(n=128, precision="fp64")
    else:
        cfg, inp = wl.colloids(shape=(128, 128, 128), count=25, precision="fp64", seed=5)
    _announce(f"multigrid vs SOR 128^3 walls={walls}")
    out = {}
    for solver in ("mg", "sor"):
        cfg.poisson_solver = solver
        cfg.poisson_tol = 1e-10
        sim = ek.EKSim(cfg, inp)
        st, it, rel = sim.poisson(1e-11, 20000)
        assert st == ek.EK_OK and rel <= 1e-11
        out[solver] = sim.field("phi")
        levels = sim.observables()["poisson_mg_levels"]
        assert (levels >= 5) == (solver == "mg")
        _announce(f"  {solver}: {it} iterations, levels {levels}")
        sim.close()
    assert phi_err(out["mg"], out["sor"]) < 1e-8


def test_poisson_entry_and_noconv():
    cfg, inp = wl.mixture_noise(n=16, precision="fp64")
    sim = ek.EKSim(cfg, inp)
    st, it, rel = sim.poisson(1e-12, 5000)
    assert st == ek.EK_OK and rel <= 1e-12
    o = orc.Oracle(cfg, inp)
    assert phi_err(sim.field("phi"), o.field("phi")) < 1e-9
    sim.step(1)
    st, it, rel = sim.poisson(1e-14, 1)
    assert st == ek.EK_ENOCONV and it == 1 and rel > 1e-14


def test_invalid_parameters():
    cfg, inp = wl.mixture_noise(n=8, precision="fp64")
    cfg.tau = 0.5
    with pytest.raises(ek.EKError) as e:
        ek.EKSim(cfg, inp)
    assert e.value.status == ek.EK_EINVAL
    cfg2, inp2 = wl.mixture_noise(shape=(7, 4, 4), precision="fp64")
    with pytest.raises(ek.EKError):
        ek.EKSim(cfg2, inp2)


def test_nonfinite_detected():
    cfg, inp = wl.mixture_noise(n=8, precision="fp64")
    inp.n_plus[0, 0, 0] = np.nan
    with pytest.raises(ek.EKError):
        ek.EKSim(cfg, inp)


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_cycle_graph_matches_direct_launches(precision):
    """A solve replays one captured V-cycle graph per cycle; per-sweep timing (level 2)
    makes the same context launch the cycle kernel by kernel.  Both give bitwise the same
    fields, replay after replay, with host reads and synchronisation between the steps."""
    cfg, inp = wl.walls_interface(shape=(64, 64, 64), precision=precision)
    _announce(f"V-cycle graph vs direct launches, walls 64^3 {precision}")
    a, b = ek.EKSim(cfg, inp), ek.EKSim(cfg, inp)
    b.set_timing(2)
    for rep in range(5):
        a.step(3)
        b.step(3)
        for name in ("rho_a", "n_plus", "n_minus", "phi"):
            assert np.array_equal(a.field(name), b.field(name)), (rep, name)
        assert a.observables()["poisson_total"] == b.observables()["poisson_total"]
    a.close()
    b.close()


@pytest.mark.parametrize("case,shape", [("walls_fp32", None), ("walls_fp64", None), ("colloids_fp32", None),
                                        ("walls_fp32", (2, 1, 1, 3, 3, 3, 10)), ("walls_fp64", (1, 3, 0, 2, 2, 2, 6))])
def test_colour_split_solve_is_bit_identical_to_site_order(case, shape, monkeypatch):
    """Multigrid solves run on colour-split copies of the potential and charge, with the
    lattice interpolation fused with the first red pass after it; the same arithmetic in
    the same order as the separate site-order launches (EK_POISSON_SITE_ORDER=1), so the
    states agree bit for bit, iteration counts included (default V-cycle and two other
    shapes: one and three lattice sweeps after the coarse-grid correction)."""
    if case == "colloids_fp32":
        cfg, inp = wl.colloids(shape=(32, 32, 32), count=4, radius=3.0, precision="fp32", seed=11)
    else:
        cfg, inp = wl.walls_interface(shape=(32, 32, 64), precision=case.split("_")[1])
    _announce(f"colour-split vs site-order multigrid: {case} {shape or 'default shape'}")
    a = ek.EKSim(cfg, inp)
    monkeypatch.setenv("EK_POISSON_SITE_ORDER", "1")
    b = ek.EKSim(cfg, inp)
    monkeypatch.delenv("EK_POISSON_SITE_ORDER")
    if shape is not None:
        for sim in (a, b):
            sim.set_multigrid(*shape, omega=1.15)
    assert a.device_bytes() > b.device_bytes()
    for k in ("phi", "rho_a", "n_plus", "n_minus"):
        assert np.array_equal(a.field(k), b.field(k)), f"t=0 {k}"
    a.step(8)
    b.step(8)
    for k in ("phi", "rho_a", "rho_b", "n_plus", "n_minus", "ux"):
        assert np.array_equal(a.field(k), b.field(k)), k
    oa, ob = a.observables(), b.observables()
    assert oa["poisson_total"] == ob["poisson_total"] > 0
    a.close()
    b.close()


@pytest.mark.parametrize("case,shape", [("walls_fp32", None), ("walls_fp64", (2, 1, 1, 3, 3, 3, 10)),
                                        ("walls_fp32", (2, 2, 1, 2, 3, 3, 10)), ("colloids_fp32", None),
                                        ("mixture_fp64", None)])
def test_one_pass_sweep_is_bit_identical_to_two_passes(case, shape, monkeypatch):
    """With EK_POISSON_ONE_PASS=1 a lattice sweep of the V-cycle on colour-split fields runs
    in one pass (k_sor_rb: a z-marching tile with the planes in LDS, writing to a second
    buffer); by default it runs as the two colour passes in place.  The rows are the same
    arithmetic in the same order, so the states agree bit for bit, iteration counts
    included.  Shapes: the default (two one-pass sweeps per cycle), two sweeps before the
    correction and none after the fused one, and an odd count (two in one pass, the last
    in two)."""
    if case == "colloids_fp32":
        cfg, inp = wl.colloids(shape=(64, 64, 64), count=12, radius=4.0, precision="fp32", seed=11)
    elif case == "mixture_fp64":
        cfg, inp = wl.mixture_noise(shape=(64, 32, 32), precision="fp64")
    else:
        cfg, inp = wl.walls_interface(shape=(128, 16, 32) if shape else (64, 64, 64), precision=case.split("_")[1])
    _announce(f"one-pass vs two-pass lattice sweeps: {case} {shape or 'default shape'}")
    monkeypatch.setenv("EK_POISSON_ONE_PASS", "1")
    a = ek.EKSim(cfg, inp)
    monkeypatch.delenv("EK_POISSON_ONE_PASS")
    b = ek.EKSim(cfg, inp)
    if shape is not None:
        for sim in (a, b):
            sim.set_multigrid(*shape, omega=1.15)
    a.step(3)
    b.step(3)
    for sim in (a, b):
        sim.set_timing(3)
    a.step(5)
    b.step(5)
    ka, kb = a.kernel_timing(), b.kernel_timing()
    assert ka["k_sor_rb"][1] > 0 and kb["k_sor_rb"][1] == 0, (ka["k_sor_rb"], kb["k_sor_rb"])
    for k in ("phi", "rho_a", "rho_b", "n_plus", "n_minus", "ux"):
        assert np.array_equal(a.field(k), b.field(k)), k
    oa, ob = a.observables(), b.observables()
    assert oa["poisson_total"] == ob["poisson_total"] > 0
    a.close()
    b.close()


def test_cycle_control_meets_tolerance_every_step():
    """The multigrid solve launches the cycles recent solves needed before it reads back the
    start residual; every step must still end below the tolerance, and the count it records
    is what was needed, so running k0 cycles does not lock k0 in: after the start-up
    transient the cycles per step fall back (walls 64^3 FP32, tolerance 1e-8)."""
    cfg, inp = wl.walls_interface(shape=(64, 64, 64), precision="fp32")
    _announce("cycle control: walls 64^3 fp32, 60 steps")
    sim = ek.EKSim(cfg, inp)
    counts = []
    for _ in range(60):
        sim.step(1)
        o = sim.observables()
        assert 0.0 < o["poisson_rel"] <= cfg.poisson_tol, o["poisson_rel"]
        counts.append(o["poisson_iters"])
    _announce(f"  cycles per step: {counts}")
    assert max(counts[-20:]) <= max(counts[:10])
    assert min(counts[-20:]) < max(counts[:10])
    sim.close()
