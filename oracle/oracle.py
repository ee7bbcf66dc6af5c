"""ctypes binding of the FP64 CPU oracle in ``ek_oracle.c``.

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the CPU-baseline leg of
``bench.py`` may use this module; the HIP library and its Python binding never import
it.  The oracle has its own parameter struct and lattice tables; a configuration object
from ``paper_1712_08494_amd.workloads`` (plain numbers, no arithmetic of the method)
is translated into that struct here.
"""
import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
BUILD_DIR = os.path.join(HERE, "_build")
LIB_PATH = os.path.join(BUILD_DIR, "libekoracle.so")
SRC = os.path.join(HERE, "ek_oracle.c")

FIELDS = {
    "rho_a": 0, "rho_b": 1, "n_plus": 2, "n_minus": 3, "phi": 4, "ux": 5, "uy": 6, "uz": 7,
    "q": 8, "eps": 9, "psi_s": 10, "solid": 11, "Ex": 12, "Ey": 13, "Ez": 14, "owner": 15,
    "q_c": 16, "Phi_a_x": 17, "Phi_a_y": 18, "Phi_a_z": 19, "Phi_b_x": 20, "Phi_b_y": 21,
    "Phi_b_z": 22, "J_plus_x": 23, "J_plus_y": 24, "J_plus_z": 25, "J_minus_x": 26,
    "J_minus_y": 27, "J_minus_z": 28, "A_plus_x": 29, "A_plus_y": 30, "A_plus_z": 31,
    "A_minus_x": 32, "A_minus_y": 33, "A_minus_z": 34, "upx": 35, "upy": 36, "upz": 37,
}
OBS = ["sum_rho_a", "sum_rho_b", "sum_n_plus", "sum_n_minus", "sum_q", "mom_x", "mom_y", "mom_z",
       "max_u", "poisson_iters", "poisson_rel", "source_mean", "drift_x", "drift_y", "drift_z",
       "pmom_x", "pmom_y", "pmom_z"]


class OrParams(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
        ("walls_z", ctypes.c_int32), ("poisson_maxit", ctypes.c_int32), ("subsample", ctypes.c_int32),
        ("move_particles", ctypes.c_int32), ("n_threads", ctypes.c_int32),
        ("tau", ctypes.c_double), ("G", ctypes.c_double), ("rho0", ctypes.c_double),
        ("D", ctypes.c_double), ("beta", ctypes.c_double),
        ("dmu_plus", ctypes.c_double), ("dmu_minus", ctypes.c_double), ("drho_a", ctypes.c_double),
        ("solvation_sign", ctypes.c_double),
        ("eps_a", ctypes.c_double), ("eps_b", ctypes.c_double), ("eps_p", ctypes.c_double),
        ("E_ext", ctypes.c_double * 3), ("body_accel", ctypes.c_double * 3),
        ("sigma_wall", ctypes.c_double * 2), ("poisson_tol", ctypes.c_double),
        ("particle_rho", ctypes.c_double), ("k_hertz", ctypes.c_double), ("eta", ctypes.c_double),
        ("poisson_lagged", ctypes.c_int32), ("polarization", ctypes.c_int32), ("reproject", ctypes.c_int32),
    ]


def build(verbose=False):
    """Compile the oracle with gcc (OpenMP).  Always recompiles."""
    os.makedirs(BUILD_DIR, exist_ok=True)
    tmp = LIB_PATH + ".tmp"
    cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-o", tmp, SRC, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.check_call(cmd)
    os.replace(tmp, LIB_PATH)
    return LIB_PATH


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        L = ctypes.CDLL(LIB_PATH)
        dp = ctypes.POINTER(ctypes.c_double)
        L.or_create.restype = ctypes.c_void_p
        L.or_create.argtypes = [ctypes.POINTER(OrParams), dp, dp, dp, dp, dp, ctypes.c_int32]
        L.or_destroy.argtypes = [ctypes.c_void_p]
        L.or_step.argtypes = [ctypes.c_void_p, ctypes.c_int32]
        L.or_step.restype = ctypes.c_int
        L.or_poisson.argtypes = [ctypes.c_void_p, ctypes.c_double, ctypes.c_int32,
                                 ctypes.POINTER(ctypes.c_int32), dp]
        L.or_poisson.restype = ctypes.c_int
        L.or_poisson_lagged.argtypes = [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int32), dp]
        L.or_poisson_lagged.restype = ctypes.c_int
        L.or_get_field.argtypes = [ctypes.c_void_p, ctypes.c_int32, dp]
        L.or_get_field.restype = ctypes.c_int
        L.or_get_populations.argtypes = [ctypes.c_void_p, ctypes.c_int32, dp]
        L.or_set_state.argtypes = [ctypes.c_void_p, dp, dp, dp, dp, dp, dp]
        L.or_set_field.argtypes = [ctypes.c_void_p, dp]
        L.or_set_field.restype = ctypes.c_int
        L.or_get_particles.argtypes = [ctypes.c_void_p, dp]
        L.or_observables.argtypes = [ctypes.c_void_p, dp]
        L.or_lattice.argtypes = [ctypes.POINTER(ctypes.c_int32), dp]
        L.or_lattice.restype = ctypes.c_int
        L.or_equilibrium.argtypes = [ctypes.c_double, dp, dp]
        L.or_num_threads.restype = ctypes.c_int
        _lib = L
    return _lib


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _c64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def lattice():
    """The oracle's D3Q19 velocities (19x3 int) and weights (19)."""
    c = np.zeros((19, 3), dtype=np.int32)
    w = np.zeros(19)
    lib().or_lattice(c.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), _dp(w))
    return c, w


def equilibrium(rho, u):
    u = _c64(np.asarray(u, dtype=np.float64).reshape(3))
    out = np.zeros(19)
    lib().or_equilibrium(float(rho), _dp(u), _dp(out))
    return out


def params_from_config(cfg, n_threads=0):
    p = OrParams()
    p.nx, p.ny, p.nz = cfg.nx, cfg.ny, cfg.nz
    p.walls_z = int(bool(cfg.walls_z))
    p.poisson_maxit = int(cfg.poisson_maxit_oracle)
    p.subsample = int(cfg.subsample)
    p.move_particles = int(bool(cfg.move_particles))
    p.n_threads = int(n_threads)
    p.tau, p.G, p.rho0 = cfg.tau, cfg.G, cfg.rho0
    p.D, p.beta = cfg.D, cfg.beta
    p.dmu_plus, p.dmu_minus, p.drho_a = cfg.dmu_plus, cfg.dmu_minus, cfg.drho_a
    p.solvation_sign = cfg.solvation_sign
    p.eps_a, p.eps_b, p.eps_p = cfg.eps_a, cfg.eps_b, cfg.eps_p
    for k in range(3):
        p.E_ext[k] = cfg.E_ext[k]
        p.body_accel[k] = cfg.body_accel[k]
    p.sigma_wall[0], p.sigma_wall[1] = cfg.sigma_wall
    p.poisson_tol = cfg.poisson_tol_oracle
    p.particle_rho, p.k_hertz, p.eta = cfg.particle_rho, cfg.k_hertz, cfg.eta
    p.poisson_lagged = int(cfg.poisson_solver == "fft")
    p.polarization = int(bool(getattr(cfg, "polarization", False)))
    p.reproject = int(bool(getattr(cfg, "reproject", False)))
    return p


class Oracle:
    """One oracle simulation.  Fields are returned as (nz, ny, nx) float64 arrays."""

    def __init__(self, cfg, inputs, n_threads=0):
        self.cfg = cfg
        self.shape = (cfg.nz, cfg.ny, cfg.nx)
        self.N = cfg.nx * cfg.ny * cfg.nz
        self._p = params_from_config(cfg, n_threads)
        ra, rb = _c64(inputs.rho_a), _c64(inputs.rho_b)
        npl, nmi = _c64(inputs.n_plus), _c64(inputs.n_minus)
        parts = _c64(inputs.particles if inputs.particles is not None else np.zeros((0, 8)))
        self.np = parts.shape[0]
        pp = _dp(parts) if self.np else None
        self._h = lib().or_create(ctypes.byref(self._p), _dp(ra), _dp(rb), _dp(npl), _dp(nmi), pp, self.np)
        if not self._h:
            raise RuntimeError("oracle: or_create failed")

    def close(self):
        if self._h:
            lib().or_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def step(self, n=1):
        return lib().or_step(self._h, int(n))

    def poisson(self, tol, maxit):
        it = ctypes.c_int32(0)
        rel = ctypes.c_double(0.0)
        st = lib().or_poisson(self._h, float(tol), int(maxit), ctypes.byref(it), ctypes.byref(rel))
        return st, it.value, rel.value

    def poisson_lagged(self):
        """One lagged Fourier solve for the current state from its potential; returns
        (status, CG iterations, relative residual of the finite-volume equation)."""
        it = ctypes.c_int32(0)
        rel = ctypes.c_double(0.0)
        st = lib().or_poisson_lagged(self._h, ctypes.byref(it), ctypes.byref(rel))
        return st, it.value, rel.value

    def field(self, name):
        out = np.zeros(self.N)
        if lib().or_get_field(self._h, FIELDS[name], _dp(out)) != 0:
            raise KeyError(name)
        return out.reshape(self.shape)

    def populations(self, comp):
        """(19, nz, ny, nx) in the oracle's velocity order (see lattice())."""
        out = np.zeros(19 * self.N)
        lib().or_get_populations(self._h, int(comp), _dp(out))
        return out.reshape((19,) + self.shape)

    def set_state(self, fa, fb, n_plus, n_minus, phi, particles=None):
        fa, fb = _c64(fa), _c64(fb)
        npl, nmi, ph = _c64(n_plus), _c64(n_minus), _c64(phi)
        pp = None
        if particles is not None and self.np:
            parts = _c64(particles)
            pp = _dp(parts)
        lib().or_set_state(self._h, _dp(fa), _dp(fb), _dp(npl), _dp(nmi), _dp(ph), pp)

    def set_field(self, E_ext):
        e = _c64(np.asarray(E_ext, dtype=float).reshape(3))
        if lib().or_set_field(self._h, _dp(e)) != 0:
            raise ValueError("oracle: field undefined for this configuration")

    def particles(self):
        out = np.zeros((max(self.np, 1), 9))
        lib().or_get_particles(self._h, _dp(out))
        return out[: self.np]

    def observables(self):
        out = np.zeros(len(OBS))
        lib().or_observables(self._h, _dp(out))
        return dict(zip(OBS, out.tolist()))


def num_threads():
    return lib().or_num_threads()
