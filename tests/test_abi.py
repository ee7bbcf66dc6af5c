"""CPU checks of the C ABI: the built library loads without a GPU and exports every
function that include/ek.h declares; the host-only lattice table is a valid D3Q19 set
equal (as a set of velocity/weight pairs) to the oracle's independent table."""
import os
import re

import numpy as np

from oracle import oracle as orc
from paper_1712_08494_amd import ek

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "ek.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(ek_[a-z_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    L = ek.load()
    names = declared_functions()
    assert "ek_init" in names and "ek_step" in names and "ek_poisson" in names and "ek_observables" in names
    for n in names:
        assert hasattr(L, n), n
    assert set(names) == set(ek.EXPORTS)


def test_lattice_table_matches_oracle_set():
    cg, wg = ek.lattice()
    co, wo = orc.lattice()
    assert sorted(zip(map(tuple, cg.tolist()), wg.tolist())) == sorted(zip(map(tuple, co.tolist()), wo.tolist()))
    # opposite velocities are 18 - d in the library's order
    for d in range(19):
        assert np.array_equal(cg[18 - d], -cg[d])


def test_status_strings():
    L = ek.load()
    assert L.ek_status_str(0) == b"ok"
    assert L.ek_status_str(ek.EK_ENOCONV).startswith(b"Poisson")


def _stepping_min_image(d, n):
    """Reference: step by whole periods while outside [-n/2, n/2] (finite d only)."""
    L = float(n)
    while d > 0.5 * L:
        d -= L
    while d < -0.5 * L:
        d += L
    return d


def test_min_image_closed_form_equals_stepping():
    """The particle geometry's minimum image takes whole periods off at once: equal to the
    stepping loop for finite separations, NaN (not an endless loop) for non-finite ones."""
    L = ek.load()
    rng = np.random.default_rng(11)
    for n in (1, 2, 7, 24, 255, 256, 1000):
        ds = np.concatenate([rng.uniform(-3.5 * n, 3.5 * n, 4000), rng.uniform(-0.6 * n, 0.6 * n, 4000),
                             np.array([0.5 * n, -0.5 * n, 1.5 * n, -1.5 * n, 0.0, n, -n, 2.5 * n, 1e-300]),
                             np.nextafter(0.5 * n, np.inf) + np.arange(3) * n])
        for d in ds:
            assert L.ek_min_image(float(d), n) == _stepping_min_image(float(d), n), (d, n)
    for bad in (np.inf, -np.inf, np.nan):
        assert np.isnan(L.ek_min_image(bad, 64))


def _init_status(cfg, inp, params=None):
    """ek_init's status for a configuration that fails its argument checks, which run
    before any device call (so this needs no GPU)."""
    import ctypes
    L = ek.load()
    p = ek.params_from_config(cfg) if params is None else params
    parts = inp.particles if inp.particles is not None else np.zeros((0, 8))
    arr = (ek.EKParticle * len(parts))()
    for j, row in enumerate(parts):
        for k in range(3):
            arr[j].x[k], arr[j].v[k] = row[k], row[3 + k]
        arr[j].radius, arr[j].charge = row[6], row[7]
    h = ctypes.c_void_p()
    a = [np.ascontiguousarray(x, dtype=np.float64) for x in (inp.rho_a, inp.rho_b, inp.n_plus, inp.n_minus)]
    st = L.ek_init(ctypes.byref(p), *[ek._dp(x) for x in a], arr, len(parts), None, ctypes.byref(h))
    msg = L.ek_last_error(h).decode() if h else ""
    L.ek_destroy(h)
    return st, msg


def test_init_rejects_non_finite_particles_and_fft_with_particles():
    from paper_1712_08494_amd import workloads as wl
    cfg = wl.EKConfig(16, 16, 16)
    inp = wl.uniform(cfg)
    for col, bad in ((0, np.inf), (1, np.nan), (4, np.inf), (6, np.nan), (7, np.inf), (6, -1.0)):
        parts = np.array([[8.0, 8.0, 8.0, 0.0, 0.0, 0.0, 3.0, 0.1]])
        parts[0, col] = bad
        inp.particles = parts
        st, msg = _init_status(cfg, inp)
        assert st == ek.EK_EINVAL and "particle 0" in msg, (col, bad, msg)
    inp.particles = np.array([[8.0, 8.0, 8.0, 0.0, 0.0, 0.0, 3.0, 0.1]])
    cfg.poisson_solver = "fft"
    st, msg = _init_status(cfg, inp)
    assert st == ek.EK_EINVAL and "lagged Fourier" in msg, msg


def test_init_rejects_polarization_where_undefined():
    """The polarisation source is refused with the lagged Fourier scheme (whose right-hand
    side has no such term), with a field normal to walls (the wall faces carry no
    displacement) and with a flag other than 0 or 1; checked before any device work."""
    from paper_1712_08494_amd import workloads as wl
    cfg = wl.EKConfig(16, 16, 16, polarization=True, E_ext=(0.0, 0.0, 1e-3), poisson_solver="fft")
    st, msg = _init_status(cfg, wl.uniform(cfg))
    assert st == ek.EK_EINVAL and "polarisation" in msg, msg
    cfg = wl.EKConfig(16, 16, 16, walls_z=True, polarization=True, E_ext=(0.0, 0.0, 1e-3))
    st, msg = _init_status(cfg, wl.uniform(cfg))
    assert st == ek.EK_EINVAL and "normal to the walls" in msg, msg
    cfg = wl.EKConfig(16, 16, 16, polarization=True)
    p = ek.params_from_config(cfg)
    p.polarization = 2
    st, msg = _init_status(cfg, wl.uniform(cfg), params=p)
    assert st == ek.EK_EINVAL and "polarization" in msg, msg


def test_init_rejects_reproject_where_unsupported():
    """Projecting moving particles anew needs them to move, and every axis long enough for
    the box of sites a step can change (2 ceil(r) + 9); checked before any device work."""
    from paper_1712_08494_amd import workloads as wl
    cfg = wl.EKConfig(28, 20, 20, reproject=True, move_particles=False)
    inp = wl.uniform(cfg)
    inp.particles = np.array([[7.3, 9.6, 7.9, 0.0, 0.0, 0.0, 3.5, 0.0]])
    st, msg = _init_status(cfg, inp)
    assert st == ek.EK_EINVAL and "move_particles" in msg, msg
    cfg = wl.EKConfig(28, 20, 16, reproject=True)
    inp = wl.uniform(cfg)
    inp.particles = np.array([[7.3, 9.6, 7.9, 0.0, 0.0, 0.0, 3.5, 0.0]])
    st, msg = _init_status(cfg, inp)
    assert st == ek.EK_EINVAL and "axis" in msg, msg
    cfg = wl.EKConfig(28, 20, 20, reproject=True)
    st, msg = _init_status(cfg, wl.uniform(cfg))
    assert st == ek.EK_EINVAL and "particles" in msg, msg


def test_workspace_bytes_is_a_host_computation():
    """ek_workspace_bytes needs no GPU: it counts the buffers of the context's layout (the
    particle geometry is built on the host for the boundary links)."""
    import ctypes
    from paper_1712_08494_amd import workloads as wl
    L = ek.load()

    def ws(cfg, parts=None):
        p = ek.params_from_config(cfg)
        n = 0 if parts is None else len(parts)
        arr = (ek.EKParticle * max(n, 1))()
        for j in range(n):
            for k in range(3):
                arr[j].x[k] = parts[j][k]
            arr[j].radius, arr[j].charge = parts[j][6], parts[j][7]
        b = ctypes.c_size_t(0)
        st = L.ek_workspace_bytes(ctypes.byref(p), arr if n else None, n, ctypes.byref(b))
        return st, b.value

    st32, b32 = ws(wl.EKConfig(32, 32, 32, precision="fp32"))
    st64, b64 = ws(wl.EKConfig(32, 32, 32, precision="fp64"))
    assert st32 == 0 and st64 == 0
    N = 32 ** 3
    # two population buffers of 2 x 19 values per site, plus ions, moments and potentials
    assert 2 * 2 * 19 * 4 * N < b32 < b64 and b64 > 2 * 2 * 19 * 8 * N
    stp, bp = ws(wl.EKConfig(32, 32, 32, precision="fp32"), [[16.0, 16.0, 16.0, 0, 0, 0, 4.0, 0.5]])
    assert stp == 0 and bp > b32  # the particle geometry adds per-site arrays and link records
    stf, _ = ws(wl.EKConfig(32, 32, 32, poisson_solver="fft"))
    assert stf == ek.EK_EINVAL
    stb, _ = ws(wl.EKConfig(7, 4, 4))
    assert stb == ek.EK_EINVAL
