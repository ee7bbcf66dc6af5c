"""The tau = 1 moment state (ek_params.moment_state): per site and component the density
and the equilibrium velocity of the last collision stand for the 19 post-collision
populations, and the moments pass gathers the streamed populations from them.  It is
the same computation as the population path (the same equilibrium expression, the same
summation order), so the two agree bit for bit; the oracle check covers it
independently."""
import numpy as np
import pytest

from oracle import oracle as orc
from paper_1712_08494_amd import ek
from paper_1712_08494_amd import workloads as wl
from tests.parity import compare

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU visible")
    ek.load()
    yield


FIELDS = ("rho_a", "rho_b", "n_plus", "n_minus", "phi", "ux", "uy", "uz")


def _case(name, precision):
    if name == "mixture":
        return wl.mixture_noise(n=32, precision=precision)
    if name == "walls":
        return wl.walls_interface(shape=(16, 12, 32), precision=precision)
    cfg, inp = wl.droplet(32, seed=5, precision=precision, field=1e-3, radius=8)
    cfg.eps_b = 2.0 * cfg.eps_a
    return cfg, inp


def _snapshot(sim):
    out = {k: sim.field(k) for k in FIELDS}
    out["f_a"] = sim.populations(0)
    out["f_b"] = sim.populations(1)
    return out


@pytest.mark.parametrize("name,precision", [("mixture", "fp64"), ("mixture", "fp32"), ("walls", "fp64"),
                                            ("walls", "fp32"), ("droplet", "fp32")])
def test_moment_state_matches_populations(name, precision):
    cfg, inp = _case(name, precision)
    print(f"moment state vs populations: {name} {precision} {cfg.nx}x{cfg.ny}x{cfg.nz}", flush=True)
    # the moment state takes the plain collision (no exact-mass rest population in FP32)
    cfg.fp32_plain_collision = True
    pop = ek.EKSim(cfg, inp)
    cfg.moment_state = True
    ms = ek.EKSim(cfg, inp)
    for s0, s1 in ((_snapshot(pop), _snapshot(ms)),):
        for k in s0:
            assert np.array_equal(s0[k], s1[k]), f"t=0 {k}"
    for step in (1, 9):
        pop.step(step)
        ms.step(step)
        a, b = _snapshot(pop), _snapshot(ms)
        for k in a:
            assert np.array_equal(a[k], b[k]), f"after {pop.observables()['steps']} steps, {k}: max diff " \
                                               f"{np.abs(a[k] - b[k]).max():.3e}"
    oa, ob = pop.observables(), ms.observables()
    for k in ("sum_rho_a", "sum_rho_b", "sum_n_plus", "sum_n_minus", "mom_x", "mom_y", "mom_z", "poisson_total"):
        assert oa[k] == ob[k], (k, oa[k], ob[k])
    ba, bb = pop.device_bytes(), ms.device_bytes()
    print(f"  device bytes {ba / 2**20:.1f} MiB with populations, {bb / 2**20:.1f} MiB with the moment state",
          flush=True)
    assert bb < ba
    pop.close()
    ms.close()


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_moment_state_vs_oracle(precision):
    cfg, inp = wl.walls_interface(shape=(16, 12, 32), precision=precision)
    cfg.moment_state = True
    print(f"moment state walls_interface 16x12x32 {precision} vs the oracle", flush=True)
    sim, o = ek.EKSim(cfg, inp), orc.Oracle(cfg, inp)
    sim.step(30)
    o.step(30)
    errs = compare(sim, o, precision, "after 30")
    print(f"  errors {errs}", flush=True)
    sim.close()


def test_moment_state_rejections():
    import torch
    cfg, inp = wl.mixture_noise(n=16, precision="fp64")
    cfg.moment_state = True
    cfg.tau = 0.8
    with pytest.raises(ek.EKError) as e:
        ek.EKSim(cfg, inp)
    assert e.value.status == ek.EK_EINVAL
    cfg, inp = wl.colloids(shape=(32, 32, 32), count=2, radius=3.5, precision="fp32", seed=7)
    cfg.moment_state = True
    with pytest.raises(ek.EKError) as e:
        ek.EKSim(cfg, inp)
    assert e.value.status == ek.EK_EINVAL
    cfg, inp = wl.mixture_noise(n=16, precision="fp64", G=0.0)
    cfg.moment_state = True
    sim = ek.EKSim(cfg, inp)
    with pytest.raises(ek.EKError) as e:
        sim.forward_checkpointed(2, 1)
    assert e.value.status == ek.EK_EINVAL
    sim.close()
    reps = wl.replica_sweep(count=2, seed=4, precision="fp32", sizes=(32,))
    for c, _ in reps:
        c.moment_state = True
    with pytest.raises(ek.EKError):
        ek.EKBatch([c for c, _ in reps], [i for _, i in reps], cycles=2)
