"""Batched replicas (one graph launch per step for all replicas) against the FP64 oracle
run of each replica, and against the same replicas stepped one context at a time."""
import numpy as np
import pytest

from oracle import oracle as orc
from paper_1712_08494_amd import ek
from paper_1712_08494_amd import workloads as wl
from tests.parity import compare, phi_err

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU visible")
    ek.load()
    yield


def _replicas(precision):
    # uneven sizes (16^3, 24^3, 32^3) and swept field, salt and coupling
    spec = [(16, 1e-3, 1e-2, 3.2), (24, 3e-4, 1e-3, 3.9), (32, 1e-4, 3e-4, 4.1), (16, 5e-4, 2e-3, 3.6)]
    return [wl.droplet(L, seed=40 + k, precision=precision, field=f, salt=s, G=G) for k, (L, f, s, G) in enumerate(spec)]


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_batch_matches_oracle(precision):
    reps = _replicas(precision)
    print(f"batch of {len(reps)} replicas, {precision}", flush=True)
    b = ek.EKBatch([c for c, _ in reps], [i for _, i in reps], cycles=8)
    b.step(20)
    b.sync()
    last, worst = b.residuals()
    print("  residuals last", last, "worst", worst, flush=True)
    assert np.all(last < 1e-9) and np.all(worst < 1e-7)  # worst: the first step has no extrapolated start
    for r, (cfg, inp) in enumerate(reps):
        o = orc.Oracle(cfg, inp)
        o.step(20)
        errs = compare(b.replica(r), o, precision, f"replica {r}")
        print(f"  replica {r} {cfg.name}: {errs}", flush=True)
    b.close()


def test_batch_matches_serial_contexts():
    reps = _replicas("fp64")
    b = ek.EKBatch([c for c, _ in reps], [i for _, i in reps], cycles=10)
    b.step(15)
    b.sync()
    for r, (cfg, inp) in enumerate(reps):
        cfg.poisson_tol = 1e-12
        sim = ek.EKSim(cfg, inp)
        sim.step(15)
        for name in ("rho_a", "rho_b", "n_plus", "n_minus"):
            a, s = b.replica(r).field(name), sim.field(name)
            assert np.max(np.abs(a - s) / np.abs(s)) < 1e-10, (r, name)
        assert phi_err(b.replica(r).field("phi"), sim.field("phi")) < 1e-8
        sim.close()
    b.close()


def test_batch_replica_is_borrowed():
    reps = _replicas("fp32")[:2]
    b = ek.EKBatch([c for c, _ in reps], [i for _, i in reps], cycles=2)
    rep = b.replica(0)
    with pytest.raises(ek.EKError) as e:
        rep.step(1)
    assert e.value.status == ek.EK_ESTATE
    b.close()


def test_batch_rejects_walls():
    cfg, inp = wl.walls_interface(shape=(16, 16, 16), precision="fp32")
    with pytest.raises(ek.EKError) as e:
        ek.EKBatch([cfg], [inp])
    assert e.value.status == ek.EK_EINVAL


def test_batch_autotune_restores_state_and_meets_its_bound():
    """ek_batch_autotune tries (shape, cycles) candidates from a saved state: afterwards the
    replicas hold the state they had, the chosen configuration keeps the worst residual
    within the bound, and the run continues bit for bit as a batch given that
    configuration by ek_batch_set_cycle."""
    reps = _replicas("fp32")
    cfgs, inps = [c for c, _ in reps], [i for _, i in reps]
    b = ek.EKBatch(cfgs, inps, cycles=4)
    b.step(3)
    before = [b.replica(r).field("rho_a") for r in range(len(reps))]
    shape, omega, cycles, ms = b.autotune(trial_steps=5, max_residual=1e-7)
    print(f"tuned: shape {shape} omega {omega} cycles {cycles} {ms:.3f} ms/step", flush=True)
    for r in range(len(reps)):
        assert np.array_equal(b.replica(r).field("rho_a"), before[r]), r
    b.residuals()
    b.step(10)
    _, worst = b.residuals()
    assert worst.max() <= 1e-7 * 1.5, worst.max()  # steps beyond the trial, same regime
    ref = ek.EKBatch(cfgs, inps, cycles=4)
    ref.step(3)
    ref.set_cycle(shape, omega, cycles)
    ref.step(10)
    for r in range(len(reps)):
        for name in ("rho_a", "n_plus", "phi"):
            assert np.array_equal(b.replica(r).field(name), ref.replica(r).field(name)), (r, name)
    b.close()
    ref.close()
