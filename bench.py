"""Benchmark of the coupled electrokinetic lattice step on one MI355X.

One step = moments + charge/permittivity + variable-permittivity Poisson solve + total
force + fused ion/force/collide/stream sweep + particle update: the whole per-timestep
sweep of the method.  Headline workload: a 256^3 periodic binary mixture with 200
resolved charged spheres (radius 4, surface charge uniform in [1e-3, 5e-3]) in the
applied field E_x = 1e-4, FP32 populations; inputs are seeded synthetic fields.

Prints one JSON line.  value = lattice-site updates per second (MLUPS) of the whole step
with all state resident in HBM.  "roofline" rates the kernel with the largest device time
per step, chosen among every kernel of the step (HIP events around each launch, on the
library's stream): its algorithmic bytes per launch over its mean launch time.
"roofline_step" rates the whole step: the method's compulsory bytes per site update
(populations, ions and potential once each way, the solid mask, and 24 B for each executed
lattice sweep of the Poisson solve) at the step rate.  "cpu_baseline" times the FP64 CPU
oracle on a bounded sample of the same workload, with all host cores and with one.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E
METRIC = "coupled-step MLUPS + % HBM roofline; FP32/FP64 speedup at stated error; bwd/fwd ratio"


# Algorithmic bytes per lattice site of one launch: the part of the method's compulsory
# traffic that the kernel carries (s = bytes of a population or ion value, 4 in FP32 and 8
# in FP64; the potential is FP64; `mask` = 1 byte of solid mask where there are solids).
# Intermediates that a kernel writes and the next reads (moment slots, charge,
# permittivity, physical velocity, multigrid levels) are not algorithmic.
def algorithmic_bytes(kernel, s, tau_one=True, mask=0):
    pops = 2 * 19 * s
    if kernel == "k_fused":      # populations written (and read when tau != 1), ions read + written, potential read
        return pops * (1 if tau_one else 2) + 4 * s + 8 + mask
    if kernel == "k_moments":    # populations read
        return pops + mask
    if kernel in ("k_sor", "k_sor_black_from", "k_mg_prolong_red_fine"):
        # one red-black colour pass over the lattice: half of a sweep's potential read +
        # write (16), charge (s) and permittivity (s)
        return (16 + 2 * s) / 2
    if kernel == "k_sor_rb":     # a whole red-black sweep in one pass
        return 16 + 2 * s
    return 0.0


def step_bytes(s, mask=0):
    """The method's compulsory traffic per site update outside the Poisson solve."""
    return 2 * 19 * 2 * s + 2 * 2 * s + 8 + mask


def sweep_bytes(s):
    """Compulsory traffic of one executed lattice sweep of the Poisson solve."""
    return 16 + 2 * s


# HBM traffic of a kernel, from rocprofv3 counter runs (FETCH_SIZE, then WRITE_SIZE, each
# scaled by what the same counter reads for a device copy of known size).  The summary
# records a hash of the kernel source it was taken on; once the source has changed the
# figure no longer describes the kernel and is reported as null.
KERNEL_SOURCE = os.path.join(ROOT, "paper_1712_08494_amd", "csrc", "ek_kernels.hip")


def traffic_summary_path(kernel, workload, n, precision):
    return os.path.join(ROOT, "profiles", f"{kernel}_{workload}_{n}_{precision}_hbm_traffic.md")


def measured_traffic(kernel, workload, n, precision):
    import hashlib
    path = traffic_summary_path(kernel, workload, n, precision)
    if not os.path.exists(path):
        return None, "no counter summary"
    rec = {}
    with open(path) as fh:
        for line in fh:
            if line.startswith("- ") and ": " in line:
                k, v = line[2:].strip().split(": ", 1)
                rec[k.strip("`")] = v.strip().strip("`")
    with open(KERNEL_SOURCE, "rb") as fh:
        sha = hashlib.sha256(fh.read()).hexdigest()
    if rec.get("kernel_source_sha256") != sha:
        return None, "kernel source changed since the counters were taken"
    return float(rec["hbm_bytes_per_launch"]), path


def copy_calibration(mib, repeats=3):
    """Device-to-device copies of a known size, for scaling the HBM byte counters."""
    import torch
    x = torch.ones(mib << 18, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    torch.cuda.synchronize()
    for _ in range(repeats):
        y.copy_(x)
    torch.cuda.synchronize()
    log(f"copy calibration: {repeats} copies of {mib} MiB")


def build_workload(name, precision, n, **kw):
    from paper_1712_08494_amd import workloads as wl
    if name == "walls_interface":
        return wl.walls_interface(n=n, precision=precision)
    if name == "colloids":
        return wl.colloids(n=n, precision=precision, **kw)
    if name == "mixture_noise":
        return wl.mixture_noise(n=n, precision=precision)
    raise SystemExit(f"unknown workload {name}")


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def run_gpu(cfg, inp, steps, warmup, kernel_steps=20, autotune=0):
    """Warm-up, then `steps` timed steps with no events inside; then `kernel_steps` more
    with an event pair around every kernel launch (timing level 3).  Events between
    kernels of a few microseconds stretch the step, so they stay out of the timed region.
    With autotune > 0 the library's V-cycle autotuner runs after the warm-up (that many
    trial steps per candidate shape, state restored) and its choice is returned."""
    import torch
    from paper_1712_08494_amd import ek
    sim = ek.EKSim(cfg, inp)
    sim.step(warmup)
    tuned = None
    if autotune:
        best, shapes, ms = sim.autotune_multigrid(autotune)
        tuned = {"shape": list(shapes[best][0]), "omega": shapes[best][1], "index": best,
                 "ms_per_step": [round(t, 4) for t in ms]}
    torch.cuda.synchronize()
    ob0 = sim.observables()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.step(steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ob1 = sim.observables()
    kt = {}
    if kernel_steps:
        sim.set_timing(3)
        sim.step(kernel_steps)
        kt = sim.kernel_timing()
        sim.set_timing(0)
    sim.close()
    return t1 - t0, kt, ob0, ob1, tuned


def kernel_table(kt, kernel_steps, N, s, tau_one, mask):
    """Per-kernel device time per step, launches per step, mean launch time and, for the
    kernels that carry algorithmic traffic, that traffic's rate."""
    table = {}
    for name, (ms, cnt) in kt.items():
        if not cnt:
            continue
        row = {"us_per_step": round(1e3 * ms / kernel_steps, 1), "launches_per_step": round(cnt / kernel_steps, 2),
               "us_per_launch": round(1e3 * ms / cnt, 2)}
        b = algorithmic_bytes(name, s, tau_one, mask)
        if b:
            row["algorithmic_bytes_per_site"] = b
            row["GBps"] = round(b * N / (ms / 1e3 / cnt) / 1e9, 1)
        table[name] = row
    return table


def run_secondary(name, precision, n, steps, warmup):
    """Step rate of another workload (no per-kernel timing)."""
    cfg, inp = build_workload(name, precision, n)
    log(f"gpu {precision}: {cfg.name}, {warmup} warm-up + {steps} timed steps")
    dt, _, _, ob1, _ = run_gpu(cfg, inp, steps, warmup, kernel_steps=0)
    return {"workload": f"{name} {cfg.nx}x{cfg.ny}x{cfg.nz}", "precision": precision,
            "mlups": round(cfg.n_sites * steps / dt / 1e6, 2), "ms_per_step": round(1e3 * dt / steps, 4),
            "poisson_iterations_last_solve": ob1["poisson_iters"]}


def run_moment_state(workload, precision, n, steps, warmup):
    """The tau = 1 moment state (density and u_e per site instead of the populations) on
    a workload without particles: step rate against the population path, device memory,
    and a bitwise comparison after a few steps with the population path taking the same
    (plain FP32) collision."""
    import numpy as np
    from paper_1712_08494_amd import ek
    out = {}
    for ms in (False, True):
        cfg, inp = build_workload(workload, precision, n)
        cfg.moment_state = ms
        log(f"gpu {'moment-state' if ms else 'population'} run, {cfg.name}")
        dt, _, _, _, _ = run_gpu(cfg, inp, steps, warmup, kernel_steps=0)
        out["moment_state" if ms else "populations"] = round(cfg.n_sites * steps / dt / 1e6, 2)
    cfg, inp = build_workload(workload, precision, n)
    cfg.moment_state = True
    a = ek.EKSim(cfg, inp)
    cfg.moment_state = False
    cfg.fp32_plain_collision = True  # the moment state's collision: compared bit for bit
    b = ek.EKSim(cfg, inp)
    bytes_ms, bytes_pop = a.device_bytes(), b.device_bytes()
    a.step(5)
    b.step(5)
    same = all(np.array_equal(a.field(k), b.field(k)) for k in ("rho_a", "rho_b", "n_plus", "n_minus", "phi"))
    a.close()
    b.close()
    return {"workload": f"{workload} {cfg.nx}x{cfg.ny}x{cfg.nz} {precision}", "mlups": out["moment_state"],
            "mlups_populations": out["populations"],
            "speedup_over_populations": round(out["moment_state"] / out["populations"], 3),
            "device_mib": round(bytes_ms / 2**20, 1), "device_mib_populations": round(bytes_pop / 2**20, 1),
            "bitwise_equal_to_populations_after_5_steps": bool(same)}


def run_moving(n, steps, warmup, speed=0.05):
    """The colloid workload with its spheres projected anew after every step (reproject),
    each launched at `speed` lattice units per step in a random direction so that sites are
    covered and uncovered throughout: step rate, the projection's device time per step, and
    the sites whose solid mark changed, against the same spheres kept on the set-up mask."""
    import numpy as np
    from paper_1712_08494_amd import ek
    res = {}
    for rp in (False, True):
        cfg, inp = build_workload("colloids", "fp32", n)
        cfg.reproject = rp
        r = np.random.Generator(np.random.PCG64(17))
        v = r.normal(size=(inp.particles.shape[0], 3))
        inp.particles[:, 3:6] = speed * v / np.linalg.norm(v, axis=1, keepdims=True)
        log(f"gpu moving spheres, {cfg.name}, reproject {rp}")
        sim = ek.EKSim(cfg, inp)
        solid0 = sim.field("solid")
        sim.close()
        dt, kt, _, _, _ = run_gpu(cfg, inp, steps, warmup, kernel_steps=5)
        key = "reproject" if rp else "set_up_mask"
        res[key] = {"mlups": round(cfg.n_sites * steps / dt / 1e6, 2), "ms_per_step": round(1e3 * dt / steps, 4)}
        if rp:
            ms, cnt = kt.get("k_reproject", (0.0, 0))
            res[key]["k_reproject_us_per_step"] = round(1e3 * ms / 5, 1) if cnt else None
            sim = ek.EKSim(cfg, inp)
            sim.step(warmup + steps)
            res[key]["sites_converted_over_run"] = int(np.sum(sim.field("solid") != solid0))
            sim.close()
    count = inp.particles.shape[0]
    return {"workload": f"colloids {n}x{n}x{n}, {count} spheres moving at {speed} per step, FP32", **res}


def run_fft_compare(n, steps, warmup):
    """The paper's lagged Fourier Poisson scheme against converged multigrid solves on a
    periodic charged droplet (n^3, radius 0.21 n, permittivity ratio 4, FP32): step rate of
    each, Poisson device time per step, and how far the lagged potential drifts from the
    converged one.  (On resolved colloids the lagged scheme diverges, and the library
    refuses it there.)"""
    import numpy as np
    import torch
    from paper_1712_08494_amd import ek
    from paper_1712_08494_amd import workloads as wl
    out = {"workload": f"droplet {n}x{n}x{n}, radius {round(0.21 * n)}, eps_b/eps_a 4, E_z 5e-4, FP32",
           "steps": steps}
    phis = {}
    for solver in ("mg", "fft"):
        cfg, inp = wl.droplet(n, seed=5, precision="fp32", field=5e-4, radius=round(0.21 * n))
        cfg.eps_b = 4.0 * cfg.eps_a
        cfg.poisson_solver = solver
        log(f"gpu Poisson comparison: {solver}, droplet {n}^3")
        sim = ek.EKSim(cfg, inp)
        sim.step(warmup)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sim.step(steps)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        sim.set_timing(1)
        sim.step(5)
        pois_ms = sim.timing()["poisson"][0] / 5
        phis[solver] = sim.field("phi")
        out[solver] = {"mlups": round(cfg.n_sites * steps / dt / 1e6, 2), "ms_per_step": round(1e3 * dt / steps, 3),
                       "poisson_ms_per_step": round(pois_ms, 3)}
        sim.close()
    out["fft_over_mg"] = round(out["fft"]["mlups"] / out["mg"]["mlups"], 3)
    d = np.abs(phis["fft"] - phis["mg"]).max() / np.abs(phis["mg"]).max()
    out["phi_max_rel_diff_after_run"] = float(f"{d:.3e}")
    return out


def field_errors(a, b):
    """Max relative difference of the fluid and ion densities where b is non-zero, and
    max |dphi| / max |phi|; a, b: objects with .field(name)."""
    import numpy as np
    out = {}
    for name in ("rho_a", "rho_b", "n_plus", "n_minus"):
        x, y = a.field(name), b.field(name)
        m = np.abs(y) > 0
        out[name] = float(f"{np.max(np.abs(x - y)[m] / np.abs(y)[m]):.3e}")
    px, py = a.field("phi"), b.field("phi")
    out["phi"] = float(f"{np.abs(px - py).max() / np.abs(py).max():.3e}")
    return out


def precision_error_vs_oracle(cfg, inp, steps):
    """The error the FP32/FP64 speedup is quoted at: the GPU FP32 path and the GPU FP64
    path against the FP64 CPU oracle, from the same inputs after `steps` steps."""
    from dataclasses import replace
    from oracle import oracle as orc
    from paper_1712_08494_amd import ek
    o = orc.Oracle(cfg, inp)
    o.step(steps)
    out = {"workload": f"{cfg.name}", "steps": steps}
    for prec in ("fp32", "fp64"):
        sim = ek.EKSim(replace(cfg, precision=prec), inp)
        sim.step(steps)
        out[prec] = field_errors(sim, o)
        sim.close()
    o.close()
    return out


def cpu_info():
    model = None
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"nproc": len(os.sched_getaffinity(0)), "cpu_count": os.cpu_count(), "model": model}


def cpu_baseline(cfg, inp, target_s=20.0):
    """Time the FP64 oracle on a bounded sample of the workload with all host cores and
    with one: one untimed step (the first solve after set-up starts from a converged
    potential), then whole steps up to about target_s per run."""
    from oracle import oracle as orc
    res = {}
    for threads in (0, 1):
        log(f"cpu baseline: oracle set-up ({'all cores' if threads == 0 else '1 core'})")
        o = orc.Oracle(cfg, inp, n_threads=threads)
        used = orc.num_threads() if threads == 0 else 1
        o.step(1)
        t0 = time.perf_counter()
        o.step(1)
        per = time.perf_counter() - t0
        steps = 1
        extra = int(max(0, min(9, target_s / max(per, 1e-6) - 1)))
        if extra:
            t0 = time.perf_counter()
            o.step(extra)
            per = (time.perf_counter() - t0 + per) / (extra + 1)
            steps += extra
        o.close()
        log(f"cpu baseline: {per:.3f} s/step over {steps} step(s) with {used} thread(s)")
        res[used] = (per, steps)
    all_threads = max(res)
    per, steps = res[all_threads]
    per1, steps1 = res[1]
    return {"value": round(cfg.n_sites / per / 1e6, 4), "unit": "MLUPS", "cores": all_threads, "kind": "oracle",
            "value_1core": round(cfg.n_sites / per1 / 1e6, 4), "host": cpu_info(),
            "sample": f"{cfg.nx}x{cfg.ny}x{cfg.nz} box of the same workload ({cfg.name}: sphere density, "
                      f"charges, salt, field as in the full box), FP64, Poisson CG to {cfg.poisson_tol_oracle:g}; "
                      f"{steps} timed step(s) with {all_threads} OpenMP threads and {steps1} with 1, each after "
                      f"set-up and one untimed step"}


def run_batched(count, steps, cycles, seed=4, tune_residual=None):
    """The replica sweep (droplets of sizes 32^3, 48^3, 64^3 with swept field, salt and
    coupling; FP32) as one batch with one graph launch per step, and the same replicas
    stepped one context after another."""
    import torch
    from paper_1712_08494_amd import ek
    from paper_1712_08494_amd import workloads as wl
    reps = wl.replica_sweep(count=count, seed=seed, precision="fp32")
    cfgs = [c for c, _ in reps]
    sites = sum(c.n_sites for c in cfgs)
    log(f"batched: {count} replicas, {sites} sites, {cycles} V-cycles per step")
    b = ek.EKBatch(cfgs, [i for _, i in reps], cycles=cycles)
    b.step(3)
    tuned = None
    if tune_residual:
        shape, omega, tc, tms = b.autotune(trial_steps=10, max_residual=tune_residual)
        tuned = {"shape": shape, "omega": omega, "v_cycles_per_step": tc, "trial_ms_per_step": round(tms, 3),
                 "max_residual": tune_residual}
        cycles = tc
        log(f"batched: autotuner chose shape {shape}, omega {omega}, {tc} V-cycles per step")
    b.residuals()  # restart the worst-residual tracker after the start-up steps
    t0 = time.perf_counter()
    b.step(steps)
    b.sync()
    tb = time.perf_counter() - t0
    last, worst = b.residuals()
    b.close()
    log(f"batched: {1e3 * tb / steps:.3f} ms per step of all replicas")
    sims = [ek.EKSim(c, i) for c, i in reps]
    for sm in sims:
        sm.step(3)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        for sm in sims:
            sm.step(1)
    torch.cuda.synchronize()
    ts = time.perf_counter() - t0
    its = sum(sm.observables()["poisson_total"] for sm in sims) / (len(sims) * (steps + 3))
    for sm in sims:
        sm.close()
    log(f"serial: {1e3 * ts / steps:.3f} ms per step of all replicas")
    # equal work: serial contexts running the batch's fixed cycle count per step (no read-back)
    from dataclasses import replace
    sims = [ek.EKSim(replace(c, poisson_cycles=cycles), i) for c, i in reps]
    for sm in sims:
        sm.step(3)
        sm.observables()  # restart the largest-residual record after the start-up steps
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        for sm in sims:
            sm.step(1)
    torch.cuda.synchronize()
    te = time.perf_counter() - t0
    worst_e = max(sm.observables()["poisson_rel_max"] for sm in sims)
    for sm in sims:
        sm.close()
    log(f"serial, {cycles} fixed V-cycles: {1e3 * te / steps:.3f} ms per step of all replicas")
    return {"workload": f"{count} droplet replicas of 32^3/48^3/64^3 (FP32)", "sites": sites, "steps": steps,
            "v_cycles_per_step": cycles, "mlups": round(sites * steps / tb / 1e6, 2),
            "serial_mlups": round(sites * steps / ts / 1e6, 2), "batched_over_serial": round(ts / tb, 3),
            "serial_v_cycles_per_step": round(its, 2), "worst_rel_residual": float(worst.max()),
            "last_rel_residual": float(last.max()),
            "serial_equal_cycles_mlups": round(sites * steps / te / 1e6, 2),
            "batched_over_serial_equal_cycles": round(te / tb, 3),
            "serial_equal_cycles_worst_rel_residual": float(worst_e), "autotune": tuned}


def droplet_deformation(ra, rb, background=0.1):
    """(b - a)/(b + a) from the second moments of the b excess about the box centre, a
    along y and b along z; works on numpy arrays and on torch tensors."""
    import numpy as np
    nz, ny, _ = rb.shape
    if not isinstance(rb, np.ndarray):
        import torch
        z = torch.arange(nz, dtype=rb.dtype, device=rb.device)[:, None, None] - (nz - 1) / 2
        y = torch.arange(ny, dtype=rb.dtype, device=rb.device)[None, :, None] - (ny - 1) / 2
        sq = torch.sqrt
        total = torch.sum
    else:
        z = np.arange(nz)[:, None, None] - (nz - 1) / 2
        y = np.arange(ny)[None, :, None] - (ny - 1) / 2
        sq, total = np.sqrt, np.sum
    w = rb - background
    a = sq(total(w * y * y))
    b = sq(total(w * z * z))
    return (b - a) / (b + a)


def run_adjoint(n=96, steps=500, every=50, fd=True, tune=100):
    """Reverse mode on the differentiation workload: a charged droplet (radius 20 in a
    periodic 96^3 box, permittivity ratio 4, E_z = 5e-4, FP64), 500 steps with a
    checkpoint every 50, and the gradient of its deformation with respect to (E_z,
    eps_b/eps_a, G) by the adjoint sweep, next to central differences of GPU runs.
    With tune > 0 the V-cycle autotuner first picks the shape for this workload (that many
    trial steps per candidate, after 20 steps from the initial state); every timed run,
    forward and reverse, uses it."""
    import torch
    from dataclasses import replace
    from paper_1712_08494_amd import ek
    from paper_1712_08494_amd import workloads as wl
    cfg, inp = wl.droplet(n, seed=5, precision="fp64", field=5e-4, salt=1e-3, G=3.6, radius=20)
    cfg.eps_b = 4.0 * cfg.eps_a
    cfg.poisson_tol = 1e-10
    N = cfg.n_sites
    log(f"adjoint: droplet {n}^3, {steps} steps, checkpoints every {every}")
    shape, tuned = None, None
    if tune:
        st = ek.EKSim(cfg, inp)
        st.step(20)
        best, cands, ms = st.autotune_multigrid(tune)
        st.close()
        shape = cands[best]
        tuned = {"shape": list(shape[0]), "omega": shape[1], "ms_per_step": round(ms[best], 4),
                 "default_ms_per_step": round(ms[0], 4)}
        log(f"adjoint: autotuned V-cycle {shape} ({ms[best]:.3f} ms/step, default {ms[0]:.3f})")

    def new_sim(c):
        s = ek.EKSim(c, inp)
        if shape is not None:
            s.set_multigrid(*shape[0], omega=shape[1])
        return s

    sim = new_sim(cfg)
    sim.step(2)
    sim.close()  # warm the library and the allocator
    sim = new_sim(cfg)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.step(steps)
    torch.cuda.synchronize()
    t_plain = time.perf_counter() - t0
    sim.close()
    sim = new_sim(cfg)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.forward_checkpointed(steps, every)
    torch.cuda.synchronize()
    t_fwd = time.perf_counter() - t0
    dev = torch.device("cuda")
    ra = torch.from_numpy(sim.field("rho_a")).to(dev).requires_grad_(True)
    rb = torch.from_numpy(sim.field("rho_b")).to(dev).requires_grad_(True)
    D = droplet_deformation(ra, rb)
    D.backward()
    adj_f = torch.zeros((2, 19, N), dtype=torch.float64, device=dev)
    for comp, t in ((0, ra), (1, rb)):
        if t.grad is not None:
            adj_f[comp] = t.grad.reshape(1, N)
    adj_n = torch.zeros((2, N), dtype=torch.float64, device=dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    grad, _, _ = sim.adjoint(adj_f, adj_n, initial=False)
    torch.cuda.synchronize()
    t_bwd = time.perf_counter() - t0
    sim.close()
    g = {"E_z": grad["E_ext"][2], "eps_ratio": grad["eps_b"] * cfg.eps_a, "G": grad["G"]}
    log(f"adjoint: forward {t_fwd:.2f} s (plain {t_plain:.2f} s), backward {t_bwd:.2f} s")
    out = {"workload": f"droplet {n}^3 radius 20, eps ratio 4, E_z 5e-4, FP64, {steps} steps, checkpoint every "
                       f"{every}, Poisson tolerance {cfg.poisson_tol:g}",
           "objective": "deformation (b - a)/(b + a) from second moments of the b excess",
           "D": float(D.detach()), "fwd_ms": round(1e3 * t_fwd, 1), "fwd_plain_ms": round(1e3 * t_plain, 1),
           "bwd_ms": round(1e3 * t_bwd, 1), "bwd_fwd_ratio": round(t_bwd / t_fwd, 3),
           "grad": {k: float(v) for k, v in g.items()}, "multigrid_autotune": tuned}
    # the same workload from an FP32 context: FP32 forward run, FP64 sweep over segments
    # restarted from its checkpoints
    cfg32 = replace(cfg, precision="fp32")
    s32 = new_sim(cfg32)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s32.forward_checkpointed(steps, every)
    torch.cuda.synchronize()
    t_fwd32 = time.perf_counter() - t0
    ra32 = torch.from_numpy(s32.field("rho_a")).to(dev).requires_grad_(True)
    rb32 = torch.from_numpy(s32.field("rho_b")).to(dev).requires_grad_(True)
    D32 = droplet_deformation(ra32, rb32)
    D32.backward()
    adj32 = torch.zeros((2, 19, N), dtype=torch.float64, device=dev)
    for comp, t in ((0, ra32), (1, rb32)):
        if t.grad is not None:
            adj32[comp] = t.grad.reshape(1, N)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    grad32, _, _ = s32.adjoint(adj32, adj_n, initial=False)
    torch.cuda.synchronize()
    t_bwd32 = time.perf_counter() - t0
    s32.close()
    g32 = {"E_z": grad32["E_ext"][2], "eps_ratio": grad32["eps_b"] * cfg.eps_a, "G": grad32["G"]}
    log(f"adjoint FP32: forward {t_fwd32:.2f} s, backward {t_bwd32:.2f} s")
    out["fp32"] = {"D": float(D32.detach()), "fwd_ms": round(1e3 * t_fwd32, 1), "bwd_ms": round(1e3 * t_bwd32, 1),
                   "grad": {k: float(v) for k, v in g32.items()},
                   "grad_rel_diff_to_fp64": {k: abs(g32[k] - g[k]) / abs(g[k]) for k in g}}
    if fd:
        def D_at(**kw):
            s2 = ek.EKSim(replace(cfg, **kw), inp)
            s2.step(steps)
            v = float(droplet_deformation(s2.field("rho_a"), s2.field("rho_b")))
            s2.close()
            return v
        # central differences at several relative steps: the step the workload names
        # (1e-4) and smaller ones, which show where the difference quotient settles
        fds, rels = {}, {}
        for key, base, steps_rel in (("E_z", cfg.E_ext[2], (1e-2, 1e-4)), ("eps_ratio", 4.0, (1e-4, 1e-5)),
                                     ("G", cfg.G, (1e-4, 1e-5, 1e-6))):
            fds[key], rels[key] = {}, {}
            for rel_h in steps_rel:
                h = rel_h * base
                vals = []
                for sgn in (1, -1):
                    if key == "E_z":
                        vals.append(D_at(E_ext=(0.0, 0.0, base + sgn * h)))
                    elif key == "eps_ratio":
                        vals.append(D_at(eps_b=(base + sgn * h) * cfg.eps_a))
                    else:
                        vals.append(D_at(G=base + sgn * h))
                fd = (vals[0] - vals[1]) / (2 * h)
                fds[key][f"{rel_h:g}"] = fd
                rels[key][f"{rel_h:g}"] = abs(g[key] - fd) / abs(fd) if fd != 0 else None
                log(f"adjoint: dD/d{key} {g[key]:.6e} vs central difference (relative step {rel_h:g}) {fd:.6e}")
        out["fd"] = fds
        out["fd_rel_err"] = rels
        out["fd_note"] = ("the donor-cell ion flux n max(u, 0) is not differentiable where a link velocity is 0, "
                          "and the resting fluid around the drop sits there: difference quotients in G scatter "
                          "around the adjoint value instead of converging (with a uniform drift they converge to "
                          "it within 1e-7, see the reverse-mode tests)")
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="colloids")
    ap.add_argument("--n", type=int, default=256)
    ap.add_argument("--precision", default="fp32")
    ap.add_argument("--kernel-steps", type=int, default=20,
                    help="steps after the timed region with an event pair around every kernel launch")
    ap.add_argument("--no-fp64", action="store_true", help="skip the FP64 run used for the FP32/FP64 speedup")
    ap.add_argument("--no-error", action="store_true", help="skip the FP32/FP64 error against the oracle")
    ap.add_argument("--error-n", type=int, default=48, help="box of the error check (same sphere density)")
    ap.add_argument("--error-steps", type=int, default=20)
    ap.add_argument("--no-secondary", action="store_true", help="skip the walls/interface 128^3 legs")
    ap.add_argument("--no-moment-state", action="store_true", help="skip the tau = 1 moment-state run")
    ap.add_argument("--no-moving", action="store_true", help="skip the moving-colloid (reproject) comparison")
    ap.add_argument("--no-fft", action="store_true", help="skip the lagged Fourier Poisson comparison")
    ap.add_argument("--fft-n", type=int, default=128)
    ap.add_argument("--fft-steps", type=int, default=50)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--cpu-n", type=int, default=64, help="box of the CPU sample (same sphere density)")
    ap.add_argument("--no-batched", action="store_true", help="skip the batched-vs-serial replica sweep")
    ap.add_argument("--batched-replicas", type=int, default=64)
    ap.add_argument("--batched-steps", type=int, default=50)
    ap.add_argument("--batched-cycles", type=int, default=4)
    ap.add_argument("--batched-tune-residual", type=float, default=1e-8,
                    help="autotune the batch for this worst relative residual (0: fixed --batched-cycles)")
    ap.add_argument("--no-adjoint", action="store_true", help="skip the reverse-mode leg")
    ap.add_argument("--autotune", type=int, default=100,
                    help="after the warm-up of the headline run and of its FP64 twin, let the library pick the "
                         "V-cycle shape (trial steps per candidate; 0: the default shape)")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="after the run, copy a buffer of this size three times (byte-counter scale)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: runs on one GPU only (asked for --gpus {args.gpus}); the multi-GPU "
              "decomposition is a design note, not an implemented path.", file=sys.stderr)
        sys.exit(2)

    import torch
    if not torch.cuda.is_available():
        raise SystemExit("bench.py needs a GPU")
    torch.cuda.set_device(0)

    cfg, inp = build_workload(args.workload, args.precision, args.n)
    log(f"gpu {args.precision}: {cfg.name}, {args.warmup} warm-up + {args.steps} timed steps")
    dt, kt, ob0, ob1, tuned = run_gpu(cfg, inp, args.steps, args.warmup, args.kernel_steps, args.autotune)
    if tuned:
        log(f"autotuned V-cycle: {tuned}")
    log(f"gpu {args.precision}: {1e3 * dt / args.steps:.3f} ms/step")
    N = cfg.n_sites
    mlups = N * args.steps / dt / 1e6
    s = 4 if args.precision == "fp32" else 8
    has_particles = inp.particles is not None and len(inp.particles) > 0
    mask = 1 if (has_particles or cfg.walls_z) else 0
    tau_one = cfg.tau == 1.0

    # the dominant kernel: largest device time per step among all kernels of the step
    table = kernel_table(kt, args.kernel_steps, N, s, tau_one, mask)
    dom = max(table, key=lambda k: table[k]["us_per_step"])
    ms_dom, cnt_dom = kt[dom]
    avg_s = ms_dom / 1e3 / cnt_dom
    bpsite = algorithmic_bytes(dom, s, tau_one, mask)
    achieved = bpsite * N / avg_s / 1e9
    if args.copy_calibration_mib:
        copy_calibration(args.copy_calibration_mib)
    traffic, traffic_src = measured_traffic(dom, args.workload, args.n, args.precision)

    # executed lattice sweeps per step (two colour passes each) and the whole step's rate
    passes = sum(kt[k][1] for k in ("k_sor", "k_sor_black_from", "k_mg_prolong_red_fine") if k in kt)
    passes += 2 * kt.get("k_sor_rb", (0.0, 0))[1]
    sweeps = passes / 2 / args.kernel_steps if args.kernel_steps else None
    cycles = (ob1["poisson_total"] - ob0["poisson_total"]) / args.steps
    step_b = step_bytes(s, mask) + (sweeps or 0.0) * sweep_bytes(s)
    step_gbs = step_b * N * args.steps / dt / 1e9

    drift = None
    if has_particles:
        d = [ob1[f"drift_{c}"] - ob0[f"drift_{c}"] for c in "xyz"]
        v = [x / args.steps for x in d]
        E = cfg.E_ext
        drift = {"particles": len(inp.particles), "mean_displacement_over_timed_steps": d,
                 "mean_velocity": v, "steps_since_init_at_end": ob1["steps"],
                 "mean_displacement_since_init": [ob1[f"drift_{c}"] for c in "xyz"],
                 "mobility_along_field": v[0] / E[0] if E[0] else None}

    fp64, tuned64 = None, None
    if not args.no_fp64 and args.precision == "fp32":
        cfg64, inp64 = build_workload(args.workload, "fp64", args.n)
        steps64 = max(10, args.steps // 2)
        log("gpu fp64 run for the FP32/FP64 speedup")
        dt64, _, _, _, tuned64 = run_gpu(cfg64, inp64, steps64, args.warmup, kernel_steps=0, autotune=args.autotune)
        fp64 = N * steps64 / dt64 / 1e6
        log(f"gpu fp64: {1e3 * dt64 / steps64:.3f} ms/step")

    error = None
    if not args.no_error and args.workload == "colloids":
        # the same workload in a smaller box with the same sphere density, against the oracle
        count = max(1, round(200 * (args.error_n / 256.0) ** 3))
        cfg_e, inp_e = build_workload("colloids", "fp32", args.error_n, count=count)
        log(f"error check: {cfg_e.name}, {args.error_steps} steps against the oracle")
        error = precision_error_vs_oracle(cfg_e, inp_e, args.error_steps)

    secondary = None
    if not args.no_secondary:
        secondary = {"walls_interface_128_fp32": run_secondary("walls_interface", "fp32", 128, 100, 10),
                     "walls_interface_128_fp64": run_secondary("walls_interface", "fp64", 128, 50, 10)}
        secondary["walls_interface_128_fp32_fp64_speedup"] = round(
            secondary["walls_interface_128_fp32"]["mlups"] / secondary["walls_interface_128_fp64"]["mlups"], 3)

    moment = None
    if not args.no_moment_state:
        moment = run_moment_state("walls_interface", "fp32", 128, 100, 10)

    moving = None
    if not args.no_moving:
        moving = run_moving(args.n, 30, 5)

    fft = None
    if not args.no_fft:
        fft = run_fft_compare(args.fft_n, args.fft_steps, 5)

    batched = None
    if not args.no_batched:
        batched = run_batched(args.batched_replicas, args.batched_steps, args.batched_cycles,
                              tune_residual=args.batched_tune_residual or None)

    adjoint = None
    if not args.no_adjoint:
        adjoint = run_adjoint()

    cpu = None
    if not args.no_cpu_baseline:
        if args.workload == "colloids":
            count = max(1, round(200 * (args.cpu_n / 256.0) ** 3))
            cfg_c, inp_c = build_workload("colloids", "fp64", args.cpu_n, count=count)
        else:
            cfg_c, inp_c = build_workload(args.workload, "fp64", args.cpu_n)
        cpu = cpu_baseline(cfg_c, inp_c, args.cpu_seconds)

    out = {
        "metric": METRIC,
        "value": round(mlups, 2),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1e3 * dt / args.steps, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if args.precision == "fp32" else "f64",
        "data": "synthetic",
        "config": {"workload": f"{args.workload} {cfg.nx}x{cfg.ny}x{cfg.nz}", "sites": N,
                   "particles": len(inp.particles) if has_particles else 0, "precision": args.precision,
                   "field": list(cfg.E_ext), "poisson_tol": cfg.poisson_tol,
                   "poisson_solver": "multigrid" if ob1["poisson_mg_levels"] else "sor",
                   "poisson_v_cycles_per_step": round(cycles, 2),
                   "poisson_start_residual": ob1["poisson_rel0"], "multigrid_autotune": tuned},
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": round(traffic) if traffic else None, "traffic_unit": "bytes per launch",
                     "traffic_bytes_per_site": round(traffic / N, 1) if traffic else None,
                     "traffic_source": os.path.relpath(traffic_src, ROOT) if traffic else traffic_src,
                     "algorithmic_bytes_per_site": bpsite, "us_per_launch": round(avg_s * 1e6, 3),
                     "launches_per_step": round(cnt_dom / args.kernel_steps, 2),
                     "timed_over": f"{args.kernel_steps} steps after the timed region, an event pair per launch"},
        "roofline_step": {"bound": "hbm", "achieved": round(step_gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                          "frac": round(step_gbs / HBM_PEAK_GBS, 4), "bytes_per_site_update": round(step_b, 1),
                          "lattice_sweeps_per_step": round(sweeps, 2) if sweeps is not None else None,
                          "definition": "(populations, ions and potential once each way, solid mask, and 24 B "
                                        "(FP32) per executed lattice sweep of the Poisson solve) x MLUPS"},
        "kernels": table,
        "electrophoretic_drift": drift,
        "fp64_mlups": round(fp64, 2) if fp64 else None,
        "fp32_fp64_speedup": round(mlups / fp64, 3) if fp64 else None,
        "fp64_multigrid_autotune": tuned64,
        "precision_error_vs_oracle": error,
        "secondary": secondary,
        "moment_state": moment,
        "moving_colloids": moving,
        "lagged_fourier_poisson": fft,
        "batched": batched,
        "adjoint": adjoint,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
