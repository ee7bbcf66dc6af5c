"""Seeded synthetic workloads: parameter sets and initial fields.

This module holds plain numbers and seeded random draws only.  It contains none of the
arithmetic of the lattice method (no equilibrium, no force, no flux, no solver), so the
HIP library and the CPU oracle can both be fed from it without sharing any of the
method's code.  Fields are float64 arrays of shape (nz, ny, nx), x fastest.

The workloads stand in for the paper's quasi-1D / quasi-2D boxes and its 3-D cube
(Sec. III): cubic boxes with the same ingredients (binary Shan-Chen mixture, monovalent
salt, permittivity contrast, charged walls or resolved charged spheres, applied field).
The paper uses no public dataset.
"""
from dataclasses import dataclass, field, replace
from typing import Optional, Tuple

import numpy as np

# Bjerrum length 1.3 lattice units (Sec. III D): eps = 1 / (4 pi l_B) with beta = e = 1.
EPS_FLUID = 1.0 / (4.0 * np.pi * 1.3)


@dataclass
class EKConfig:
    nx: int
    ny: int
    nz: int
    walls_z: bool = False
    precision: str = "fp64"          # "fp64" or "fp32" (populations as deviations)
    tau: float = 1.0                 # Sec. III A
    G: float = 3.6                   # fluid/fluid Shan-Chen coupling
    rho0: float = 1.0                # pseudopotential reference density
    D: float = 0.01                  # ion diffusivity, Sec. II C
    beta: float = 1.0
    dmu_plus: float = 0.0            # Gibbs transfer energies
    dmu_minus: float = 0.0
    drho_a: float = 1.0              # bulk rho^a difference between the phases
    solvation_sign: float = 1.0      # +1: the printed discrete solvation flux
    eps_a: float = EPS_FLUID
    eps_b: float = EPS_FLUID
    eps_p: float = EPS_FLUID / 8.0   # relative permittivities 10 / 80, Sec. III D
    phi_history: int = 0             # Poisson warm start: 0 the library default
    moment_state: bool = False       # tau = 1 only: store density and u_e per site instead of populations
    sweep_band: int = 0              # workgroup band of the stencil sweeps: 0 or -1 plain order
    poisson_cycles: int = 0          # > 0: that many V-cycles per step, no host read-back
    fp32_plain_collision: bool = False  # FP32: the plain collision instead of the exact-mass one
    polarization: bool = False       # the external field polarises the dielectric (Poisson source)
    reproject: bool = False          # moving particles projected anew every step (cover / uncover)
    E_ext: Tuple[float, float, float] = (0.0, 0.0, 0.0)
    body_accel: Tuple[float, float, float] = (0.0, 0.0, 0.0)
    sigma_wall: Tuple[float, float] = (0.0, 0.0)
    poisson_tol: float = 1e-10       # relative residual of the GPU solve
    poisson_maxit: int = 20000
    sor_omega: float = 0.0           # SOR relaxation of the "sor" solver; 0: from the lattice size
    poisson_solver: str = "auto"     # "auto" (multigrid where possible), "sor", "mg", or "fft" (the
                                     # lagged Fourier scheme, one solve per step, periodic lattices)
    poisson_tol_oracle: float = 1e-12
    poisson_maxit_oracle: int = 200000
    subsample: int = 8               # sub-cells per axis for the solid fraction
    move_particles: bool = True
    particle_rho: float = 5.0        # Sec. II E
    k_hertz: float = 1.0             # Sec. II E
    eta: float = 1.0 / 6.0           # dynamic viscosity used by lubrication
    name: str = "custom"

    @property
    def n_sites(self):
        return self.nx * self.ny * self.nz


@dataclass
class EKInputs:
    rho_a: np.ndarray
    rho_b: np.ndarray
    n_plus: np.ndarray
    n_minus: np.ndarray
    particles: Optional[np.ndarray] = None   # (n, 8): x, y, z, vx, vy, vz, radius, charge
    extra: dict = field(default_factory=dict)


def _rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def _neutralise(n_plus, n_minus, extra_charge=0.0, mask=None):
    """Rescale n- so that sum(n+) - sum(n-) + extra_charge = 0 in float64."""
    if mask is None:
        mask = np.ones_like(n_plus, dtype=bool)
    tot_p = n_plus[mask].sum() + extra_charge
    tot_m = n_minus[mask].sum()
    n_minus = n_minus.copy()
    n_minus[mask] *= tot_p / tot_m
    return n_minus


# ---------------------------------------------------------------------------------
# Workload 1: small periodic mixture with noise (parity case).
# ---------------------------------------------------------------------------------
def mixture_noise(n=32, seed=1, precision="fp64", G=3.6, shape=None):
    nx, ny, nz = shape if shape is not None else (n, n, n)
    cfg = EKConfig(nx, ny, nz, precision=precision, G=G, poisson_tol=1e-10, name=f"mixture_noise_{nx}x{ny}x{nz}")
    r = _rng(seed)
    sh = (nz, ny, nx)
    rho_a = 0.5 + r.uniform(-0.01, 0.01, sh)
    rho_b = 0.5 + r.uniform(-0.01, 0.01, sh)
    n_plus = 1e-3 + r.uniform(-1e-5, 1e-5, sh)
    n_minus = 1e-3 + r.uniform(-1e-5, 1e-5, sh)
    n_minus = _neutralise(n_plus, n_minus)
    return cfg, EKInputs(rho_a, rho_b, n_plus, n_minus)


# ---------------------------------------------------------------------------------
# Workload 2: charged walls in z and a flat interface between the two fluids.
# Phase densities are the coexisting bulk densities of a flat Shan-Chen interface at
# the paper's coupling G = 4.0 and mean total density 1.386: a 64-site column relaxed for
# 35000 steps on the CPU reference (oracle/calibrate_interface.py prints them).
# ---------------------------------------------------------------------------------
WALL_G = 4.0
WALL_RHO_MAJ = 1.41527
WALL_RHO_MIN = 0.01112


def _bisect(f, lo, hi, it=200):
    flo = f(lo)
    for _ in range(it):
        mid = 0.5 * (lo + hi)
        fm = f(mid)
        if (fm > 0) == (flo > 0):
            lo, flo = mid, fm
        else:
            hi = mid
    return 0.5 * (lo + hi)


def pb_column(nz, zi, rho_a_z, salt, sigma, eps_a, eps_b, dmu_p, dmu_m, drho, sign=1.0):
    """Equilibrium ion profiles n+(z), n-(z) of a column with charged walls (planes at
    z = 1/2 and nz - 3/2) and a sharp interface at z = zi between fluid a (below) and b
    (above), from closed-form Poisson-Boltzmann pieces (beta = e = 1):
      - ions are Boltzmann distributed in the potential psi and the solvation energy
        U+- = sign * dmu+- rho^a / drho_a, so the two bulks differ by the Donnan step
        psi_b - psi_a = U+_a - U+_b;
      - at the interface each side follows tanh((psi - psi_bulk)/4) ~ exp(-kappa |z - zi|),
        kappa^2 = 2 n / eps, with psi and eps psi' continuous (one scalar root);
      - at each wall the Gouy-Chapman solution with sinh(psi0 / 2) = sigma / sqrt(8 eps n).
    The pieces are superposed; they overlap negligibly when the walls are far from the
    interface compared with the Debye length.  Returns arrays of length nz (wall layers 0)."""
    z = np.arange(nz, dtype=np.float64)
    U_p = sign * dmu_p * rho_a_z / drho
    U_m = sign * dmu_m * rho_a_z / drho
    Ua_p, Ub_p = sign * dmu_p * rho_a_z[1] / drho, sign * dmu_p * rho_a_z[-2] / drho
    Ua_m, Ub_m = sign * dmu_m * rho_a_z[1] / drho, sign * dmu_m * rho_a_z[-2] / drho
    psi_a = 0.0
    psi_b = Ua_p - Ub_p  # equals Ub_m - Ua_m when dmu+ = -dmu-
    ka, kb = np.sqrt(2 * salt / eps_a), np.sqrt(2 * salt / eps_b)
    g = lambda p0: eps_a * ka * np.sinh((p0 - psi_a) / 2) + eps_b * kb * np.sinh((p0 - psi_b) / 2)
    lo, hi = min(psi_a, psi_b), max(psi_a, psi_b)
    psi0 = _bisect(g, lo, hi) if hi > lo else psi_a
    dz = z - zi
    dev = np.where(dz < 0,
                   4 * np.arctanh(np.tanh((psi0 - psi_a) / 4) * np.exp(-ka * np.abs(dz))),
                   4 * np.arctanh(np.tanh((psi0 - psi_b) / 4) * np.exp(-kb * np.abs(dz))))
    bulk = np.where(dz < 0, psi_a, psi_b)
    for zw, k, e in ((0.5, ka, eps_a), (nz - 1.5, kb, eps_b)):
        p0 = 2 * np.arcsinh(sigma / np.sqrt(8 * e * salt))
        dev = dev + 4 * np.arctanh(np.tanh(p0 / 4) * np.exp(-k * np.abs(z - zw)))
    psi = bulk + dev
    n_p = salt * np.exp(-(psi - psi_a) - (U_p - Ua_p))
    n_m = salt * np.exp(+(psi - psi_a) - (U_m - Ua_m))
    n_p[0] = n_p[-1] = n_m[0] = n_m[-1] = 0.0
    return n_p, n_m


def walls_interface(n=128, seed=2, precision="fp32", shape=None, salt=1e-3, sigma=-1e-3, eps_ratio=2.0,
                    dmu=2.0, width=1.0):
    nx, ny, nz = shape if shape is not None else (n, n, n)
    zi = nz // 2
    drho = WALL_RHO_MAJ - WALL_RHO_MIN
    cfg = EKConfig(nx, ny, nz, walls_z=True, precision=precision, G=WALL_G, dmu_plus=dmu, dmu_minus=-dmu,
                   drho_a=drho, eps_a=EPS_FLUID, eps_b=eps_ratio * EPS_FLUID, sigma_wall=(sigma, sigma),
                   poisson_tol=1e-8, name=f"walls_interface_{nx}x{ny}x{nz}")
    r = _rng(seed)
    sh = (nz, ny, nx)
    z = np.arange(nz, dtype=np.float64)
    # fluid a below the interface plane, fluid b above it
    s = 0.5 * (1.0 + np.tanh((z - (zi - 0.5)) / width))
    ra_z = WALL_RHO_MAJ + (WALL_RHO_MIN - WALL_RHO_MAJ) * s
    rb_z = WALL_RHO_MIN + (WALL_RHO_MAJ - WALL_RHO_MIN) * s
    rho_a = ra_z[:, None, None] + r.uniform(-1e-4, 1e-4, sh)
    rho_b = rb_z[:, None, None] + r.uniform(-1e-4, 1e-4, sh)
    # ions start at the equilibrium double layers (walls and interface)
    np_z, nm_z = pb_column(nz, zi - 0.5, ra_z, salt, sigma, cfg.eps_a, cfg.eps_b, dmu, -dmu, drho)
    n_plus = np_z[:, None, None] * (1.0 + r.uniform(-1e-4, 1e-4, sh))
    n_minus = nm_z[:, None, None] * (1.0 + r.uniform(-1e-4, 1e-4, sh))
    fluid = np.ones(sh, dtype=bool)
    fluid[0] = False
    fluid[-1] = False
    n_plus[~fluid] = 0.0
    n_minus[~fluid] = 0.0
    # exact neutrality with the two charged walls
    wall_charge = (sigma + sigma) * nx * ny
    n_minus = _neutralise(n_plus, n_minus, extra_charge=wall_charge, mask=fluid)
    return cfg, EKInputs(rho_a, rho_b, n_plus, n_minus)


# ---------------------------------------------------------------------------------
# Workload 3: resolved charged spheres in a periodic binary mixture under a field.
# ---------------------------------------------------------------------------------
def place_spheres(rng, count, radius, shape, min_gap=2.0, max_tries=200000):
    """Uniform random centres, rejection-sampled so that centre distances (minimum
    image) are at least 2 r + min_gap."""
    nx, ny, nz = shape
    L = np.array([nx, ny, nz], dtype=np.float64)
    centres = []
    tries = 0
    while len(centres) < count:
        tries += 1
        if tries > max_tries:
            raise RuntimeError("could not place spheres")
        c = rng.uniform(0.0, 1.0, 3) * L
        ok = True
        for o in centres:
            d = c - o
            d -= L * np.round(d / L)
            if np.dot(d, d) < (2 * radius + min_gap) ** 2:
                ok = False
                break
        if ok:
            centres.append(c)
    return np.array(centres)


def colloids(n=256, seed=3, precision="fp32", count=200, radius=4.0, shape=None, salt=1e-3,
             field=(1e-4, 0.0, 0.0), G=3.6):
    nx, ny, nz = shape if shape is not None else (n, n, n)
    cfg = EKConfig(nx, ny, nz, precision=precision, G=G, E_ext=tuple(field), poisson_tol=1e-8,
                   name=f"colloids_{nx}x{ny}x{nz}_{count}")
    r = _rng(seed)
    sh = (nz, ny, nx)
    centres = place_spheres(r, count, radius, (nx, ny, nz))
    sigma = r.uniform(1e-3, 5e-3, count)
    Q = 4.0 * np.pi * radius ** 2 * sigma
    parts = np.zeros((count, 8))
    parts[:, 0:3] = centres
    parts[:, 6] = radius
    parts[:, 7] = Q
    rho_a = 0.5 + r.uniform(-0.01, 0.01, sh)
    rho_b = 0.5 + r.uniform(-0.01, 0.01, sh)
    n_plus = salt * np.ones(sh)
    n_minus = salt * np.ones(sh) + Q.sum() / float(nx * ny * nz)
    return cfg, EKInputs(rho_a, rho_b, n_plus, n_minus, particles=parts)


# ---------------------------------------------------------------------------------
# Workload 4: a sweep of independent droplet replicas of uneven size.
# ---------------------------------------------------------------------------------
def droplet(L, seed=4, precision="fp32", field=1e-4, salt=1e-3, G=3.6, dmu=-4.0, width=2.0, shape=None, radius=None):
    """A drop of fluid b (radius L/5 unless given) in fluid a, centred in a periodic cube: inside
    (rho_a, rho_b) = (0.1, 0.9), outside swapped, tanh profile of width 2; both ion
    species Boltzmann-partitioned by the solvation energy dmu rho_a / drho_a (same
    energy for both, so the fluid stays neutral), mean salt `salt`; field along z."""
    nx, ny, nz = shape if shape is not None else (L, L, L)
    drho = 0.8
    cfg = EKConfig(nx, ny, nz, precision=precision, G=G, dmu_plus=dmu, dmu_minus=dmu, drho_a=drho,
                   E_ext=(0.0, 0.0, field), poisson_tol=1e-8, name=f"droplet_{nx}x{ny}x{nz}")
    r = _rng(seed)
    sh = (nz, ny, nx)
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    d = np.sqrt((x - nx / 2 + 0.5) ** 2 + (y - ny / 2 + 0.5) ** 2 + (z - nz / 2 + 0.5) ** 2)
    R = min(nx, ny, nz) / 5.0 if radius is None else float(radius)
    inside = 0.5 * (1.0 - np.tanh((d - R) / width))
    rho_a = 0.9 - 0.8 * inside + r.uniform(-1e-3, 1e-3, sh)
    rho_b = 0.1 + 0.8 * inside + r.uniform(-1e-3, 1e-3, sh)
    boltz = np.exp(-(dmu / drho) * rho_a)
    n = salt * boltz / boltz.mean()
    return cfg, EKInputs(rho_a, rho_b, n.copy(), n.copy())


def dielectric_droplet(l=128, lx=4, radius=None, chi=0.5, field=0.05, precision="fp64", seed=6, width=2.0,
                       noise=1e-4):
    """The ion-free dielectric drop of Sec. III B: a quasi-two-dimensional periodic box
    lx x l x l, a cylinder of fluid b (radius l/4 unless given) along x in fluid a, the two
    bulk densities of the flat-interface calibration at G = 4.0, tanh profile of the given
    width, uniform rho noise of the given amplitude.  Permittivity contrast
    chi = (eps_a - eps_b) / (eps_a + eps_b) with eps_a the fluid default; the field E_z
    polarises the dielectric."""
    eps_b = EPS_FLUID * (1.0 - chi) / (1.0 + chi)
    cfg = EKConfig(lx, l, l, precision=precision, G=WALL_G, eps_a=EPS_FLUID, eps_b=eps_b, E_ext=(0.0, 0.0, field),
                   polarization=True, poisson_tol=1e-10, name=f"dielectric_droplet_{lx}x{l}x{l}")
    r = _rng(seed)
    sh = (l, l, lx)
    z, y = np.meshgrid(np.arange(l), np.arange(l), indexing="ij")
    d = np.hypot(y - l / 2 + 0.5, z - l / 2 + 0.5)
    R = l / 4.0 if radius is None else float(radius)
    inside = (0.5 * (1.0 - np.tanh((d - R) / width)))[:, :, None]
    rho_a = WALL_RHO_MAJ + (WALL_RHO_MIN - WALL_RHO_MAJ) * inside + r.uniform(-noise, noise, sh)
    rho_b = WALL_RHO_MIN + (WALL_RHO_MAJ - WALL_RHO_MIN) * inside + r.uniform(-noise, noise, sh)
    zero = np.zeros(sh)
    return cfg, EKInputs(rho_a, rho_b, zero.copy(), zero.copy())


def replica_sweep(count=64, seed=4, precision="fp32", sizes=(32, 48, 64)):
    """Replica sizes drawn from `sizes`; field E_z log-uniform in [1e-5, 1e-3], salt
    log-uniform in [1e-4, 1e-2], G uniform in [3.0, 4.2]."""
    r = _rng(seed)
    out = []
    for k in range(count):
        L = int(r.choice(sizes))
        field = float(10 ** r.uniform(-5, -3))
        salt = float(10 ** r.uniform(-4, -2))
        G = float(r.uniform(3.0, 4.2))
        out.append(droplet(L, seed=seed * 1000 + k, precision=precision, field=field, salt=salt, G=G))
    return out


# ---------------------------------------------------------------------------------
# Small deterministic fields used by the pins.
# ---------------------------------------------------------------------------------
def uniform(cfg, rho_a=0.5, rho_b=0.5, n_plus=1e-3, n_minus=1e-3):
    sh = (cfg.nz, cfg.ny, cfg.nx)
    return EKInputs(np.full(sh, float(rho_a)), np.full(sh, float(rho_b)), np.full(sh, float(n_plus)),
                    np.full(sh, float(n_minus)))


def with_precision(cfg, precision):
    return replace(cfg, precision=precision)
