"""Python binding of ``libek.so`` (the C ABI in ``include/ek.h``).

Argument marshalling only: every step of the method runs in the library's HIP kernels.
The binding fails loudly when the library is not built; there is no fallback.
PyTorch supplies the HIP stream the context runs on (its current stream by default).
"""
import ctypes
import os
from dataclasses import replace

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libek.so")

EK_OK, EK_EINVAL, EK_ENOMEM, EK_EHIP, EK_ENOCONV, EK_ENONFINITE, EK_ESTATE = 0, -1, -2, -3, -4, -5, -6
EK_FP64, EK_FP32 = 0, 1
POISSON_SOLVERS = {"auto": 0, "sor": 1, "mg": 2, "fft": 3}
FIELDS = {"rho_a": 0, "rho_b": 1, "n_plus": 2, "n_minus": 3, "phi": 4, "ux": 5, "uy": 6, "uz": 7, "q": 8,
          "eps": 9, "psi_s": 10, "solid": 11, "Ex": 12, "Ey": 13, "Ez": 14}
TIMING_CLASSES = ["moments", "poisson", "force", "fused", "particle", "iter", "smooth"]


class EKParams(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
        ("walls_z", ctypes.c_int32), ("precision", ctypes.c_int32), ("poisson_maxit", ctypes.c_int32),
        ("poisson_solver", ctypes.c_int32), ("subsample", ctypes.c_int32), ("move_particles", ctypes.c_int32),
        ("tau", ctypes.c_double), ("G", ctypes.c_double), ("rho0", ctypes.c_double),
        ("rho_ref", ctypes.c_double * 2), ("D", ctypes.c_double), ("beta", ctypes.c_double),
        ("dmu", ctypes.c_double * 2), ("drho_a", ctypes.c_double), ("solvation_sign", ctypes.c_double),
        ("eps_a", ctypes.c_double), ("eps_b", ctypes.c_double), ("eps_p", ctypes.c_double),
        ("E_ext", ctypes.c_double * 3), ("body_accel", ctypes.c_double * 3), ("sigma_wall", ctypes.c_double * 2),
        ("poisson_tol", ctypes.c_double), ("sor_omega", ctypes.c_double), ("particle_rho", ctypes.c_double),
        ("k_hertz", ctypes.c_double), ("eta", ctypes.c_double), ("phi_history", ctypes.c_int32),
        ("moment_state", ctypes.c_int32), ("sweep_band", ctypes.c_int32), ("poisson_cycles", ctypes.c_int32),
        ("fp32_plain_collision", ctypes.c_int32), ("polarization", ctypes.c_int32), ("reproject", ctypes.c_int32),
    ]


class EKParticle(ctypes.Structure):
    _fields_ = [("x", ctypes.c_double * 3), ("v", ctypes.c_double * 3), ("radius", ctypes.c_double),
                ("charge", ctypes.c_double)]


class EKObs(ctypes.Structure):
    _fields_ = [
        ("sum_rho", ctypes.c_double * 2), ("sum_n", ctypes.c_double * 2), ("sum_q", ctypes.c_double),
        ("momentum", ctypes.c_double * 3), ("max_u", ctypes.c_double), ("source_mean", ctypes.c_double),
        ("poisson_rel", ctypes.c_double), ("poisson_iters", ctypes.c_int64), ("poisson_total", ctypes.c_int64),
        ("poisson_mg_levels", ctypes.c_int32), ("steps", ctypes.c_int64), ("drift", ctypes.c_double * 3), ("pmomentum", ctypes.c_double * 3),
        ("nonfinite", ctypes.c_int32), ("negative_ions", ctypes.c_int32), ("poisson_rel0", ctypes.c_double),
        ("poisson_rel_max", ctypes.c_double),
    ]


N_KERNELS = 23


class EKTiming(ctypes.Structure):
    _fields_ = [("ms", ctypes.c_double * 7), ("count", ctypes.c_int64 * 7),
                ("kernel_ms", ctypes.c_double * N_KERNELS), ("kernel_count", ctypes.c_int64 * N_KERNELS)]


EXPORTS = ["ek_lattice", "ek_min_image", "ek_kernel_name", "ek_workspace_bytes", "ek_init_ws", "ek_observables_device", "ek_init", "ek_step", "ek_poisson", "ek_observables", "ek_get_field",
           "ek_get_populations", "ek_get_particles", "ek_device_bytes", "ek_set_timing", "ek_get_timing",
           "ek_destroy", "ek_status_str", "ek_last_error", "ek_batch_init", "ek_batch_step", "ek_batch_sync",
           "ek_batch_residuals", "ek_batch_replica", "ek_batch_destroy", "ek_batch_last_error",
           "ek_batch_set_cycle", "ek_batch_autotune",
           "ek_forward_ckpt", "ek_adjoint", "ek_set_field", "ek_set_multigrid", "ek_autotune_candidates",
           "ek_autotune_multigrid"]

_lib = None


class EKError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{msg} (status {status})")
        self.status = status


def load(path=LIB_PATH):
    """Load libek.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} not found: build it with paper_1712_08494_amd.build.build()")
    # PyTorch ships its own HIP runtime with the same soname as the system one; importing
    # it first makes libek bind to that already-loaded runtime, so the process holds a
    # single HIP runtime (two would each try to own the device).
    import torch  # noqa: F401
    L = ctypes.CDLL(path)
    dp = ctypes.POINTER(ctypes.c_double)
    vp = ctypes.c_void_p
    L.ek_lattice.argtypes = [ctypes.POINTER(ctypes.c_int32), dp]
    L.ek_lattice.restype = ctypes.c_int32
    L.ek_min_image.argtypes = [ctypes.c_double, ctypes.c_int32]
    L.ek_min_image.restype = ctypes.c_double
    L.ek_kernel_name.argtypes = [ctypes.c_int32]
    L.ek_kernel_name.restype = ctypes.c_char_p
    L.ek_init.argtypes = [ctypes.POINTER(EKParams), dp, dp, dp, dp, ctypes.POINTER(EKParticle), ctypes.c_int32, vp,
                          ctypes.POINTER(vp)]
    L.ek_init.restype = ctypes.c_int32
    L.ek_step.argtypes = [vp, ctypes.c_int32]
    L.ek_step.restype = ctypes.c_int32
    L.ek_poisson.argtypes = [vp, ctypes.c_double, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32), dp]
    L.ek_poisson.restype = ctypes.c_int32
    L.ek_workspace_bytes.argtypes = [ctypes.POINTER(EKParams), ctypes.POINTER(EKParticle), ctypes.c_int32,
                                     ctypes.POINTER(ctypes.c_size_t)]
    L.ek_workspace_bytes.restype = ctypes.c_int32
    L.ek_init_ws.argtypes = [ctypes.POINTER(EKParams), dp, dp, dp, dp, ctypes.POINTER(EKParticle), ctypes.c_int32,
                             vp, ctypes.c_size_t, vp, ctypes.POINTER(vp)]
    L.ek_init_ws.restype = ctypes.c_int32
    L.ek_observables.argtypes = [vp, ctypes.POINTER(EKObs), ctypes.c_uint32, dp]
    L.ek_observables_device.argtypes = [vp, vp]
    L.ek_observables_device.restype = ctypes.c_int32
    L.ek_observables.restype = ctypes.c_int32
    L.ek_get_field.argtypes = [vp, ctypes.c_int32, dp]
    L.ek_get_field.restype = ctypes.c_int32
    L.ek_get_populations.argtypes = [vp, ctypes.c_int32, dp]
    L.ek_get_populations.restype = ctypes.c_int32
    L.ek_get_particles.argtypes = [vp, dp]
    L.ek_get_particles.restype = ctypes.c_int32
    L.ek_device_bytes.argtypes = [vp, ctypes.POINTER(ctypes.c_size_t)]
    L.ek_device_bytes.restype = ctypes.c_int32
    L.ek_set_timing.argtypes = [vp, ctypes.c_int32]
    L.ek_set_timing.restype = ctypes.c_int32
    L.ek_get_timing.argtypes = [vp, ctypes.POINTER(EKTiming)]
    L.ek_get_timing.restype = ctypes.c_int32
    L.ek_destroy.argtypes = [vp]
    L.ek_destroy.restype = ctypes.c_int32
    L.ek_status_str.argtypes = [ctypes.c_int32]
    L.ek_status_str.restype = ctypes.c_char_p
    L.ek_last_error.argtypes = [vp]
    L.ek_last_error.restype = ctypes.c_char_p
    pdp = ctypes.POINTER(dp)
    L.ek_batch_init.argtypes = [ctypes.POINTER(EKParams), ctypes.c_int32, pdp, pdp, pdp, pdp, ctypes.c_int32,
                                ctypes.POINTER(vp)]
    L.ek_batch_init.restype = ctypes.c_int32
    L.ek_batch_step.argtypes = [vp, ctypes.c_int32]
    L.ek_batch_step.restype = ctypes.c_int32
    L.ek_batch_sync.argtypes = [vp]
    L.ek_batch_sync.restype = ctypes.c_int32
    L.ek_batch_residuals.argtypes = [vp, dp, dp]
    L.ek_batch_residuals.restype = ctypes.c_int32
    L.ek_batch_set_cycle.argtypes = [vp, ctypes.POINTER(ctypes.c_int32), ctypes.c_double, ctypes.c_int32]
    L.ek_batch_set_cycle.restype = ctypes.c_int32
    L.ek_batch_autotune.argtypes = [vp, ctypes.c_int32, ctypes.c_double, ctypes.POINTER(ctypes.c_int32),
                                    dp, dp]
    L.ek_batch_autotune.restype = ctypes.c_int32
    L.ek_batch_replica.argtypes = [vp, ctypes.c_int32, ctypes.POINTER(vp)]
    L.ek_batch_replica.restype = ctypes.c_int32
    L.ek_batch_destroy.argtypes = [vp]
    L.ek_batch_destroy.restype = ctypes.c_int32
    L.ek_batch_last_error.argtypes = [vp]
    L.ek_batch_last_error.restype = ctypes.c_char_p
    L.ek_forward_ckpt.argtypes = [vp, ctypes.c_int32, ctypes.c_int32]
    L.ek_forward_ckpt.restype = ctypes.c_int32
    L.ek_adjoint.argtypes = [vp, vp, vp, dp, vp, vp]
    L.ek_adjoint.restype = ctypes.c_int32
    L.ek_set_field.argtypes = [vp, ctypes.POINTER(ctypes.c_double)]
    L.ek_set_field.restype = ctypes.c_int32
    L.ek_set_multigrid.argtypes = [vp] + [ctypes.c_int32] * 7 + [ctypes.c_double]
    L.ek_set_multigrid.restype = ctypes.c_int32
    L.ek_autotune_candidates.argtypes = [ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_double)]
    L.ek_autotune_candidates.restype = ctypes.c_int32
    L.ek_autotune_multigrid.argtypes = [vp, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32),
                                        ctypes.POINTER(ctypes.c_double)]
    L.ek_autotune_multigrid.restype = ctypes.c_int32
    _lib = L
    return L


def lattice():
    """The library's D3Q19 velocities (19x3) and weights (19)."""
    L = load()
    c = np.zeros((19, 3), dtype=np.int32)
    w = np.zeros(19)
    L.ek_lattice(c.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), w.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    return c, w


def autotune_candidates():
    """The V-cycle shapes the autotuner tries, the default first: (7 sweep counts in the
    argument order of set_multigrid, omega)."""
    L = load()
    n = L.ek_autotune_candidates(None, None)
    shapes = (ctypes.c_int32 * (7 * n))()
    om = (ctypes.c_double * n)()
    L.ek_autotune_candidates(shapes, om)
    return [(tuple(shapes[7 * k:7 * k + 7]), om[k]) for k in range(n)]


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _c64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def params_from_config(cfg):
    """Pack a workloads.EKConfig into the ek_params struct."""
    p = EKParams()
    p.nx, p.ny, p.nz = cfg.nx, cfg.ny, cfg.nz
    p.walls_z = int(bool(cfg.walls_z))
    p.precision = EK_FP32 if cfg.precision == "fp32" else EK_FP64
    p.poisson_maxit = int(cfg.poisson_maxit)
    p.poisson_solver = POISSON_SOLVERS[cfg.poisson_solver]
    p.subsample = int(cfg.subsample)
    p.move_particles = int(bool(cfg.move_particles))
    p.tau, p.G, p.rho0 = cfg.tau, cfg.G, cfg.rho0
    p.rho_ref[0] = p.rho_ref[1] = 0.0
    p.D, p.beta = cfg.D, cfg.beta
    p.dmu[0], p.dmu[1] = cfg.dmu_plus, cfg.dmu_minus
    p.drho_a, p.solvation_sign = cfg.drho_a, cfg.solvation_sign
    p.eps_a, p.eps_b, p.eps_p = cfg.eps_a, cfg.eps_b, cfg.eps_p
    for k in range(3):
        p.E_ext[k] = cfg.E_ext[k]
        p.body_accel[k] = cfg.body_accel[k]
    p.sigma_wall[0], p.sigma_wall[1] = cfg.sigma_wall
    p.poisson_tol = cfg.poisson_tol
    p.sor_omega = float(getattr(cfg, "sor_omega", 0.0))
    p.particle_rho, p.k_hertz, p.eta = cfg.particle_rho, cfg.k_hertz, cfg.eta
    p.phi_history = int(getattr(cfg, "phi_history", 0))
    p.moment_state = int(bool(getattr(cfg, "moment_state", False)))
    p.sweep_band = int(getattr(cfg, "sweep_band", 0))
    p.poisson_cycles = int(getattr(cfg, "poisson_cycles", 0))
    p.fp32_plain_collision = int(bool(getattr(cfg, "fp32_plain_collision", False)))
    p.polarization = int(bool(getattr(cfg, "polarization", False)))
    p.reproject = int(bool(getattr(cfg, "reproject", False)))
    return p


def current_stream_handle():
    """Raw hipStream_t of PyTorch's current stream on the current device."""
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


class EKSim:
    """A simulation context on the GPU.  Fields come back as (nz, ny, nx) float64 arrays."""

    def __init__(self, cfg, inputs, stream=None, params=None, workspace=False):
        """workspace=True: the context's device memory is one torch uint8 tensor held by
        this object (ek_workspace_bytes / ek_init_ws); otherwise the library allocates it."""
        L = load()
        self.cfg = cfg
        self.shape = (cfg.nz, cfg.ny, cfg.nx)
        self.N = cfg.nx * cfg.ny * cfg.nz
        self._p = params if params is not None else params_from_config(cfg)
        ra, rb = _c64(inputs.rho_a), _c64(inputs.rho_b)
        npl, nmi = _c64(inputs.n_plus), _c64(inputs.n_minus)
        parts = inputs.particles
        self.np = 0 if parts is None else int(parts.shape[0])
        arr = (EKParticle * max(self.np, 1))()
        for j in range(self.np):
            for k in range(3):
                arr[j].x[k] = parts[j, k]
                arr[j].v[k] = parts[j, 3 + k]
            arr[j].radius = parts[j, 6]
            arr[j].charge = parts[j, 7]
        if stream is None:
            stream = current_stream_handle()
        self._stream = stream
        h = ctypes.c_void_p()
        self.workspace = None
        if workspace:
            import torch
            nb = ctypes.c_size_t(0)
            st = L.ek_workspace_bytes(ctypes.byref(self._p), arr if self.np else None, self.np, ctypes.byref(nb))
            if st != EK_OK:
                raise EKError(st, "ek_workspace_bytes")
            self.workspace = torch.empty(nb.value, dtype=torch.uint8, device="cuda")
            st = L.ek_init_ws(ctypes.byref(self._p), _dp(ra), _dp(rb), _dp(npl), _dp(nmi), arr if self.np else None,
                              self.np, ctypes.c_void_p(self.workspace.data_ptr()), nb.value, stream, ctypes.byref(h))
        else:
            st = L.ek_init(ctypes.byref(self._p), _dp(ra), _dp(rb), _dp(npl), _dp(nmi),
                           arr if self.np else None, self.np, stream, ctypes.byref(h))
        self._h = h
        if st != EK_OK:
            msg = self.last_error()
            self.close()
            raise EKError(st, "ek_init: " + msg)

    def last_error(self):
        if not self._h:
            return ""
        return load().ek_last_error(self._h).decode()

    def _check(self, st, what, allow=()):
        if st != EK_OK and st not in allow:
            raise EKError(st, f"{what}: {self.last_error()}")
        return st

    def close(self):
        if getattr(self, "_h", None):
            load().ek_destroy(self._h)
            self._h = None
        self.workspace = None  # after ek_destroy: the context no longer uses it

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def step(self, n=1, allow_noconv=False):
        return self._check(load().ek_step(self._h, int(n)), "ek_step", (EK_ENOCONV,) if allow_noconv else ())

    def poisson(self, tol, maxit):
        it = ctypes.c_int32(0)
        rel = ctypes.c_double(0.0)
        st = load().ek_poisson(self._h, float(tol), int(maxit), ctypes.byref(it), ctypes.byref(rel))
        self._check(st, "ek_poisson", (EK_ENOCONV,))
        return st, it.value, rel.value

    def observables(self, fields=()):
        """FP64 totals and diagnostics; with field names, also those fields (ek_observables'
        field mask) under the key "fields" as {name: (nz, ny, nx) array}."""
        o = EKObs()
        ids = sorted(FIELDS[f] for f in fields)
        mask = 0
        for k in ids:
            mask |= 1 << k
        buf = np.zeros(len(ids) * self.N) if ids else None
        st = load().ek_observables(self._h, ctypes.byref(o), mask, _dp(buf) if ids else None)
        self._check(st, "ek_observables", (EK_ENONFINITE,))
        out = {
            "status": st,
            "sum_rho_a": o.sum_rho[0], "sum_rho_b": o.sum_rho[1], "sum_n_plus": o.sum_n[0],
            "sum_n_minus": o.sum_n[1], "sum_q": o.sum_q, "mom_x": o.momentum[0], "mom_y": o.momentum[1],
            "mom_z": o.momentum[2], "max_u": o.max_u, "source_mean": o.source_mean, "poisson_rel": o.poisson_rel,
            "poisson_iters": o.poisson_iters, "poisson_total": o.poisson_total,
            "poisson_mg_levels": o.poisson_mg_levels, "steps": o.steps,
            "drift_x": o.drift[0], "drift_y": o.drift[1], "drift_z": o.drift[2], "pmom_x": o.pmomentum[0],
            "pmom_y": o.pmomentum[1], "pmom_z": o.pmomentum[2], "nonfinite": o.nonfinite,
            "negative_ions": o.negative_ions, "poisson_rel0": o.poisson_rel0, "poisson_rel_max": o.poisson_rel_max,
        }
        if ids:
            names = {v: k for k, v in FIELDS.items()}
            out["fields"] = {names[k]: buf[j * self.N:(j + 1) * self.N].reshape(self.shape) for j, k in enumerate(ids)}
        return out

    def observables_device(self, out):
        """The totals of observables() written by the library into `out`, a contiguous float64
        GPU tensor of at least 11 values, on the context's stream, with no allocation and no
        synchronisation (ek_observables_device)."""
        import torch
        if not (out.is_cuda and out.dtype == torch.float64 and out.is_contiguous() and out.numel() >= 11):
            raise TypeError("out must be a contiguous float64 GPU tensor of at least 11 values")
        self._check(load().ek_observables_device(self._h, ctypes.c_void_p(out.data_ptr())), "ek_observables_device")

    def field(self, name):
        out = np.zeros(self.N)
        self._check(load().ek_get_field(self._h, FIELDS[name], _dp(out)), "ek_get_field")
        return out.reshape(self.shape)

    def populations(self, comp):
        """(19, nz, ny, nx) in the library's velocity order (see lattice())."""
        out = np.zeros(19 * self.N)
        self._check(load().ek_get_populations(self._h, int(comp), _dp(out)), "ek_get_populations")
        return out.reshape((19,) + self.shape)

    def particles(self):
        out = np.zeros((max(self.np, 1), 9))
        self._check(load().ek_get_particles(self._h, _dp(out)), "ek_get_particles")
        return out[: self.np]

    def device_bytes(self):
        b = ctypes.c_size_t(0)
        load().ek_device_bytes(self._h, ctypes.byref(b))
        return b.value

    def set_timing(self, on):
        self._check(load().ek_set_timing(self._h, int(on)), "ek_set_timing")

    def timing(self):
        t = EKTiming()
        self._check(load().ek_get_timing(self._h, ctypes.byref(t)), "ek_get_timing")
        return {name: (t.ms[k], t.count[k]) for k, name in enumerate(TIMING_CLASSES)}

    def kernel_timing(self):
        """Per-kernel totals of timing level 3: {kernel name: (ms, launches)}."""
        t = EKTiming()
        L = load()
        self._check(L.ek_get_timing(self._h, ctypes.byref(t)), "ek_get_timing")
        return {L.ek_kernel_name(k).decode(): (t.kernel_ms[k], t.kernel_count[k]) for k in range(N_KERNELS)}

    def set_field(self, E_ext):
        """Change the external field from the next step on (ek_set_field)."""
        e = (ctypes.c_double * 3)(*[float(v) for v in E_ext])
        self._check(load().ek_set_field(self._h, e), "ek_set_field")
        self.cfg = replace(self.cfg, E_ext=tuple(float(v) for v in E_ext))

    def set_multigrid(self, fine_pre=1, fine_post=2, coarse_pre=1, coarse_post=2, tail_pre=3, tail_post=3,
                      coarsest=10, omega=1.2):
        """V-cycle shape: sweeps before/after the correction on the lattice, on the launched
        coarse grids and on the tail kernel's upper grid, coarsest-grid sweeps, and the
        relaxation of the smoothing sweeps."""
        self._check(load().ek_set_multigrid(self._h, fine_pre, fine_post, coarse_pre, coarse_post, tail_pre,
                                            tail_post, coarsest, float(omega)), "ek_set_multigrid")

    def autotune_multigrid(self, trial_steps=100):
        """Time every candidate V-cycle shape over trial_steps steps from the current state,
        restore the state and keep the fastest shape.  Returns (best index, the candidates
        as (sweep counts, omega), milliseconds per step of each).  A step runs a whole
        number of cycles, so a window of a few steps can favour a shape that happens to
        save a cycle there; about 100 steps track the long-run rate."""
        cands = autotune_candidates()
        best = ctypes.c_int32(-1)
        ms = (ctypes.c_double * len(cands))()
        self._check(load().ek_autotune_multigrid(self._h, int(trial_steps), ctypes.byref(best), ms),
                    "ek_autotune_multigrid")
        return best.value, cands, list(ms)

    def forward_checkpointed(self, nsteps, every, allow_noconv=False):
        """nsteps steps keeping a checkpoint every `every` steps, for adjoint()."""
        return self._check(load().ek_forward_ckpt(self._h, int(nsteps), int(every)), "ek_forward_ckpt",
                           (EK_ENOCONV,) if allow_noconv else ())

    def adjoint(self, adj_f, adj_n, initial=True):
        """Reverse the last forward_checkpointed run.  adj_f (2, 19, N) and adj_n (2, N) are
        float64 tensors on the GPU holding dL/d(populations) and dL/d(n+, n-) at its end.
        Returns (gradient dict, dL/df at the start or None, dL/dn at the start or None)."""
        import torch
        for t in (adj_f, adj_n):
            if not (t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()):
                raise TypeError("adj_f and adj_n must be contiguous float64 GPU tensors")
        if adj_f.numel() != 2 * 19 * self.N or adj_n.numel() != 2 * self.N:
            raise ValueError("adj_f must hold 2 x 19 x N values and adj_n 2 x N")
        f0 = torch.empty_like(adj_f) if initial else None
        n0 = torch.empty_like(adj_n) if initial else None
        g = np.zeros(6)
        st = load().ek_adjoint(self._h, ctypes.c_void_p(adj_f.data_ptr()), ctypes.c_void_p(adj_n.data_ptr()), _dp(g),
                               ctypes.c_void_p(f0.data_ptr()) if initial else None,
                               ctypes.c_void_p(n0.data_ptr()) if initial else None)
        self._check(st, "ek_adjoint", (EK_ENOCONV,))
        grad = {"E_ext": g[0:3].copy(), "eps_a": g[3], "eps_b": g[4], "G": g[5]}
        return grad, f0, n0


class _Borrowed(EKSim):
    """A replica context owned by a batch: export calls only."""

    def __init__(self, handle, cfg):
        self._h = handle
        self.cfg = cfg
        self.shape = (cfg.nz, cfg.ny, cfg.nx)
        self.N = cfg.nx * cfg.ny * cfg.nz
        self.np = 0

    def close(self):
        self._h = None


class EKBatch:
    """Many periodic replicas advanced together, one graph launch per step."""

    def __init__(self, cfgs, inputs, cycles=4):
        L = load()
        n = len(cfgs)
        self.cfgs = list(cfgs)
        params = (EKParams * n)()
        for r, c in enumerate(cfgs):
            params[r] = params_from_config(c)
        self._keep = []
        ptrs = []
        for name in ("rho_a", "rho_b", "n_plus", "n_minus"):
            arrs = [_c64(getattr(inp, name)) for inp in inputs]
            self._keep.append(arrs)
            ptrs.append((ctypes.POINTER(ctypes.c_double) * n)(*[_dp(a) for a in arrs]))
        h = ctypes.c_void_p()
        st = L.ek_batch_init(params, n, ptrs[0], ptrs[1], ptrs[2], ptrs[3], int(cycles), ctypes.byref(h))
        self._h = h
        self.n = n
        self._keep = None
        if st != EK_OK:
            msg = L.ek_batch_last_error(h).decode() if h else ""
            self.close()
            raise EKError(st, "ek_batch_init: " + msg)

    def close(self):
        if getattr(self, "_h", None):
            load().ek_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def step(self, n=1):
        st = load().ek_batch_step(self._h, int(n))
        if st != EK_OK:
            raise EKError(st, "ek_batch_step: " + load().ek_batch_last_error(self._h).decode())

    def set_cycle(self, shape, omega, cycles):
        """V-cycle shape (seven sweep counts), relaxation and V-cycles per step (ek_batch_set_cycle)."""
        sh = (ctypes.c_int32 * 7)(*[int(v) for v in shape])
        st = load().ek_batch_set_cycle(self._h, sh, float(omega), int(cycles))
        if st != EK_OK:
            raise EKError(st, "ek_batch_set_cycle: " + load().ek_batch_last_error(self._h).decode())

    def autotune(self, trial_steps=20, max_residual=1e-8):
        """Pick the fastest (shape, cycles per step) meeting max_residual (ek_batch_autotune);
        returns (shape, omega, cycles, ms per step)."""
        best = (ctypes.c_int32 * 8)()
        om = ctypes.c_double(0.0)
        ms = ctypes.c_double(0.0)
        st = load().ek_batch_autotune(self._h, int(trial_steps), float(max_residual), best, ctypes.byref(om),
                                      ctypes.byref(ms))
        if st != EK_OK:
            raise EKError(st, "ek_batch_autotune: " + load().ek_batch_last_error(self._h).decode())
        return list(best[:7]), om.value, best[7], ms.value

    def sync(self):
        load().ek_batch_sync(self._h)

    def residuals(self):
        last = np.zeros(self.n)
        worst = np.zeros(self.n)
        load().ek_batch_residuals(self._h, _dp(last), _dp(worst))
        return last, worst

    def replica(self, r):
        h = ctypes.c_void_p()
        st = load().ek_batch_replica(self._h, int(r), ctypes.byref(h))
        if st != EK_OK:
            raise EKError(st, "ek_batch_replica")
        return _Borrowed(h, self.cfgs[r])


def _ek_run_function():
    import torch

    class EKRun(torch.autograd.Function):
        """T steps of the method as a differentiable function of (E_z, eps_b / eps_a, G).
        forward(params, cfg, inputs, nsteps, every) runs a checkpointed forward pass of a
        periodic context built from cfg (in its precision) with those three parameters
        replaced, and returns the fluid densities rho^a, rho^b at the end as (nz, ny, nx)
        GPU tensors; backward runs the library's adjoint sweep (FP64; for an FP32 context
        along segments restarted from its FP32 checkpoints)."""

        @staticmethod
        def forward(ctx, params, cfg, inputs, nsteps, every):
            from dataclasses import replace
            ez, ratio, G = (float(v) for v in params.detach().cpu().tolist())
            c2 = replace(cfg, E_ext=(cfg.E_ext[0], cfg.E_ext[1], ez), eps_b=ratio * cfg.eps_a, G=G)
            sim = EKSim(c2, inputs)
            sim.forward_checkpointed(nsteps, every)
            ctx.sim, ctx.eps_a = sim, cfg.eps_a
            dev = torch.device("cuda")
            return (torch.from_numpy(sim.field("rho_a")).to(dev), torch.from_numpy(sim.field("rho_b")).to(dev))

        @staticmethod
        def backward(ctx, g_ra, g_rb):
            sim = ctx.sim
            N = sim.N
            dev = torch.device("cuda")
            adj_f = torch.zeros((2, 19, N), dtype=torch.float64, device=dev)
            # rho^s = sum_d f^s_d: the same sensitivity for every population of a component
            if g_ra is not None:
                adj_f[0] = g_ra.reshape(1, N).to(torch.float64)
            if g_rb is not None:
                adj_f[1] = g_rb.reshape(1, N).to(torch.float64)
            adj_n = torch.zeros((2, N), dtype=torch.float64, device=dev)
            grad, _, _ = sim.adjoint(adj_f, adj_n, initial=False)
            sim.close()
            out = torch.tensor([grad["E_ext"][2], grad["eps_b"] * ctx.eps_a, grad["G"]], dtype=torch.float64)
            return out, None, None, None, None

    return EKRun


def ek_run(params, cfg, inputs, nsteps, every):
    """Differentiable run: see EKRun (params = tensor([E_z, eps_b / eps_a, G]))."""
    return _ek_run_function().apply(params, cfg, inputs, nsteps, every)
