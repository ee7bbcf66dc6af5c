"""GPU tests of the boundary calls: a context in a caller-owned workspace, the Poisson
mode without host read-back, and the observables' field mask."""
import numpy as np
import pytest

from paper_1712_08494_amd import ek
from paper_1712_08494_amd import workloads as wl

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU visible")
    ek.load()
    torch.cuda.init()
    yield


def _announce(msg):
    print(msg, flush=True)


@pytest.mark.parametrize("case", ["walls_fp32", "colloids_fp32", "mixture_fp64"])
def test_workspace_context_matches_library_allocation(case):
    """The whole step on a torch-owned workspace: bit-identical to the library-allocated
    context, with the library allocating no device memory for it."""
    import torch
    if case == "walls_fp32":
        cfg, inp = wl.walls_interface(shape=(32, 32, 64), precision="fp32")
    elif case == "colloids_fp32":
        cfg, inp = wl.colloids(shape=(32, 32, 32), count=4, radius=3.0, precision="fp32", seed=11)
    else:
        cfg, inp = wl.mixture_noise(n=32, precision="fp64")
    _announce(f"workspace context {case}")
    a = ek.EKSim(cfg, inp)
    torch.cuda.synchronize()
    b = ek.EKSim(cfg, inp, workspace=True)
    assert b.workspace is not None and b.workspace.numel() >= b.device_bytes()
    for sim in (a, b):
        sim.step(12)
    for k in ("rho_a", "rho_b", "n_plus", "n_minus", "phi", "ux"):
        assert np.array_equal(a.field(k), b.field(k)), k
    if a.np:
        assert np.array_equal(a.particles(), b.particles())
    oa, ob = a.observables(), b.observables()
    assert oa["poisson_total"] == ob["poisson_total"]
    a.close()
    b.close()


def test_fixed_cycles_step_without_readback():
    """poisson_cycles > 0: every step runs that many V-cycles and reads nothing back; the
    residuals stay on the device and the observables report them.  With enough cycles the
    result agrees with the solve to tolerance."""
    cfg, inp = wl.walls_interface(shape=(64, 64, 64), precision="fp32")
    _announce("fixed V-cycles: walls 64^3 fp32")
    ref = ek.EKSim(cfg, inp)
    cfg.poisson_cycles = 6
    fx = ek.EKSim(cfg, inp)
    ref.step(20)
    fx.step(20)
    o = fx.observables()
    assert o["poisson_iters"] == 6 and o["poisson_total"] == 6 * 20
    assert 0.0 < o["poisson_rel"] <= o["poisson_rel_max"] < 1e-7, o
    assert o["poisson_rel0"] > o["poisson_rel"]
    o2 = fx.observables()
    assert o2["poisson_rel_max"] == 0.0  # cleared by the previous call, no step since
    fx.step(1)
    assert 0.0 < fx.observables()["poisson_rel_max"] < 1e-7
    ref.step(1)
    for k in ("rho_a", "n_plus", "n_minus"):
        a, b = fx.field(k), ref.field(k)
        m = np.abs(b) > 0
        assert np.max(np.abs(a - b)[m] / np.abs(b)[m]) < 1e-5, k
    pa, pb = fx.field("phi"), ref.field("phi")
    assert np.abs(pa - pb).max() < 1e-4 * np.abs(pb).max()
    fx.close()
    ref.close()


def test_fixed_cycles_rejected_without_multigrid():
    cfg, inp = wl.mixture_noise(shape=(10, 6, 6), precision="fp64")
    cfg.poisson_cycles = 3
    with pytest.raises(ek.EKError) as e:
        ek.EKSim(cfg, inp)
    assert e.value.status == ek.EK_EINVAL


def test_observables_field_mask():
    cfg, inp = wl.colloids(shape=(24, 24, 24), count=2, radius=3.0, precision="fp32", seed=5)
    sim = ek.EKSim(cfg, inp)
    sim.step(3)
    names = ["phi", "rho_a", "n_minus", "Ez", "solid"]
    o = sim.observables(fields=names)
    for n in names:
        assert np.array_equal(o["fields"][n], sim.field(n)), n
    assert o["sum_rho_a"] == sim.observables()["sum_rho_a"]
    sim.close()
