"""Seeded synthetic inputs shared by the GPU library's tests/benchmarks and the oracle.

This module only builds inputs: grid sizes, material maps, the electron bunch,
probe positions and smooth initial fields.  It holds none of the time-stepping
arithmetic of the method and imports neither the GPU package nor the oracle.

The workloads follow the structure of the paper's simulation model (Sec. III:
a relativistic electron bunch travelling parallel to a silver film described
by the Drude model of Eq. 1), in the frame used throughout this project:
film normal along z, bunch moving along +x.

Workloads (all seeded, ``seed = 1505040070 + index``):
  0 ``slab20nm_32x32x32_pec``       32^3, dx 5 nm, PEC, Ag slab z-cells 8..11,
                                     1000 particles, 30 keV, 200 steps
  1 ``film30nm_256x128x128_cpml8``  256x128x128, dx 2 nm, 8-cell CPML, 30 nm film,
                                     1e6 particles, 50 keV, 5000 steps
  3 ``film20nm_128x64x64_cpml8``    128x64x64, dx 2 nm, 8-cell CPML, 20 nm film with
                                     +-5 % seeded map noise, 1e5 particles, 2000 steps
  4 ``grating40nm_512x256x256_cpml12`` 512x256x256, dx 1 nm, 12-cell CPML, 40 nm film
                                     with 10 nm grooves at 100 nm period, 1e7
                                     particles, 100 keV, 20000 steps, sort every 20
  2 ``batched16``                   16 instances, 5..80 nm films, U(20,80) keV
  - ``grating40nm_shard2of8_64x256x256`` rank 2's x-slab of workload 4 under an
                                     8-way split (the busiest rank: 48 % of the
                                     bunch); periodic x faces stand in for halos
"""
from dataclasses import dataclass, field
from typing import Optional

import numpy as np

# CODATA 2018 constants used to define inputs (loading energies, dt).
C_LIGHT = 299792458.0
E_CHARGE = 1.602176634e-19
M_E = 9.1093837015e-31
MEC2_EV = M_E * C_LIGHT ** 2 / E_CHARGE

PEC, PERIODIC, CPML = 0, 1, 2
SEED0 = 1505040070

# Silver Drude constants of the workloads (rad/s, 1/s), eps_inf = 1.
AG_WP = 1.37e16
AG_GAMMA = 3.2e13


@dataclass
class Bunch:
    x: np.ndarray
    y: np.ndarray
    z: np.ndarray
    ux: np.ndarray
    uy: np.ndarray
    uz: np.ndarray
    q: float
    m: float
    w: float

    @property
    def n(self):
        return int(self.x.shape[0])

    def subset(self, idx):
        return Bunch(self.x[idx], self.y[idx], self.z[idx], self.ux[idx], self.uy[idx],
                     self.uz[idx], self.q, self.m, self.w)


@dataclass
class Workload:
    name: str
    nx: int
    ny: int
    nz: int
    dx: float
    dt: float
    bc: tuple
    npml: int
    wp_map: np.ndarray  # (nx, ny, nz) rad/s
    gamma_map: np.ndarray  # (nx, ny, nz) 1/s
    bunch: Optional[Bunch]
    probes: np.ndarray  # (nprobe, 3) metres
    omega: np.ndarray  # (nfreq,) rad/s
    steps: int
    sort_every: int = 0
    pml: tuple = (3.0, 1.0, 1.0, 0.0)  # grading order m, sigma scale, kappa_max, alpha_max
    meta: dict = field(default_factory=dict)

    @property
    def cells(self):
        return self.nx * self.ny * self.nz


def courant_dt(dx):
    """dt = 0.5 dx / (c sqrt 3): half the 3D vacuum Courant limit."""
    return 0.5 * dx / (C_LIGHT * np.sqrt(3.0))


def beam_u(kinetic_ev):
    """gamma v (m/s) of an electron with the given kinetic energy."""
    g = 1.0 + kinetic_ev / MEC2_EV
    return C_LIGHT * np.sqrt(g * g - 1.0)


def truncated_normal(rng, n, cut=3.0):
    """Standard normal samples, entries beyond +-cut redrawn until inside."""
    g = rng.standard_normal(n)
    bad = np.abs(g) > cut
    while bad.any():
        g[bad] = rng.standard_normal(int(bad.sum()))
        bad = np.abs(g) > cut
    return g


def gaussian_bunch(rng, n, center, sigma, kinetic_ev, charge=1e-15):
    """Cold electron bunch along +x, Gaussian positions truncated at 3 sigma."""
    pos = [center[a] + sigma[a] * truncated_normal(rng, n) for a in range(3)]
    u = beam_u(kinetic_ev)
    return Bunch(pos[0], pos[1], pos[2], np.full(n, u), np.zeros(n), np.zeros(n),
                 -E_CHARGE, M_E, charge / (n * E_CHARGE))


def aloof_center(top_z, gap, sigma_z, cut=3.0):
    """Height of a bunch centre whose truncated lower edge (cut sigma below the
    centre) clears the film top by `gap`: the bunch travels wholly above the
    surface, as an aloof beam "N nm above the surface" does."""
    return top_z + gap + cut * sigma_z


def film_maps(nx, ny, nz, k0, k1, wp=AG_WP, gamma=AG_GAMMA):
    """Drude maps with metal in the z-cells k0 <= k < k1 (full x, y)."""
    wpm = np.zeros((nx, ny, nz))
    gm = np.zeros((nx, ny, nz))
    wpm[:, :, k0:k1] = wp
    gm[:, :, k0:k1] = gamma
    return wpm, gm


def spectrum_omegas(wp=AG_WP, nfreq=64, lo=0.3, hi=1.0):
    """nfreq angular frequencies spaced linearly over [lo, hi] * wp."""
    return wp * np.linspace(lo, hi, nfreq)


def slab_tiny(with_bunch=True):
    """32^3 cells, dx = 5 nm, PEC walls, Ag slab in z-cells 8..11, 200 steps."""
    n, dx = 32, 5e-9
    wpm, gm = film_maps(n, n, n, 8, 12)
    rng = np.random.default_rng(SEED0 + 0)
    bunch = None
    if with_bunch:
        # centre 10 nm above the film top (z = 60 nm), y centred, x = 40 nm
        bunch = gaussian_bunch(rng, 1000, (40e-9, 80e-9, 70e-9), (5e-9,) * 3, 30e3)
    probes = np.array([[16 * dx, 16 * dx, 62e-9], [20 * dx, 16 * dx, 62e-9],
                       [24 * dx, 16 * dx, 62e-9]])
    return Workload("slab20nm_32x32x32_pec", n, n, n, dx, courant_dt(dx), (PEC,) * 3, 0,
                    wpm, gm, bunch, probes, spectrum_omegas(), 200)


def film_production(nparticles=1_000_000, seed_index=1):
    """256x128x128, dx = 2 nm, 8-cell CPML, 30 nm film, 50 keV bunch 8 nm above
    the surface (gap to the bunch's truncated lower edge)."""
    nx, ny, nz, dx, npml = 256, 128, 128, 2e-9, 8
    top = nz // 2
    wpm, gm = film_maps(nx, ny, nz, top - 15, top)
    rng = np.random.default_rng(SEED0 + seed_index)
    sig = (20e-9, 5e-9, 5e-9)
    center = (npml * dx + 3 * sig[0], ny * dx / 2, aloof_center(top * dx, 8e-9, sig[2]))
    bunch = gaussian_bunch(rng, nparticles, center, sig, 50e3)
    zp = top * dx + 2e-9
    probes = np.array([[nx * dx * f, ny * dx / 2, zp] for f in (0.5, 0.625, 0.75)])
    return Workload("film30nm_256x128x128_cpml8", nx, ny, nz, dx, courant_dt(dx),
                    (CPML,) * 3, npml, wpm, gm, bunch, probes, spectrum_omegas(), 5000,
                    sort_every=20)


def film_adjoint(nparticles=100_000):
    """128x64x64, dx = 2 nm, 8-cell CPML, 20 nm film, maps with +-5 % noise."""
    nx, ny, nz, dx, npml = 128, 64, 64, 2e-9, 8
    top = nz // 2
    wpm, gm = film_maps(nx, ny, nz, top - 10, top)
    rng = np.random.default_rng(SEED0 + 3)
    metal = wpm > 0
    wpm[metal] *= 1.0 + 0.05 * rng.standard_normal(int(metal.sum()))
    gm[metal] *= 1.0 + 0.05 * rng.standard_normal(int(metal.sum()))
    sig = (20e-9, 5e-9, 5e-9)
    center = (npml * dx + 3 * sig[0], ny * dx / 2, aloof_center(top * dx, 8e-9, sig[2]))
    bunch = gaussian_bunch(rng, nparticles, center, sig, 50e3)
    zp = top * dx + 2e-9
    probes = np.array([[nx * dx * f, ny * dx / 2, zp] for f in (0.5, 0.625, 0.75)])
    return Workload("film20nm_128x64x64_cpml8", nx, ny, nz, dx, courant_dt(dx), (CPML,) * 3,
                    npml, wpm, gm, bunch, probes, np.array([0.68 * AG_WP]), 2000,
                    sort_every=20, meta={"omega0": 0.68 * AG_WP})


def grating_large(nparticles=10_000_000):
    """512x256x256, dx = 1 nm, 12-cell CPML, 40 nm film with a 1D grating on top.

    Grooves 10 nm deep and 50 nm wide, period 100 nm along x, invariant in y.
    """
    nx, ny, nz, dx, npml = 512, 256, 256, 1e-9, 12
    top = nz // 2
    wpm, gm = film_maps(nx, ny, nz, top - 40, top)
    xc = (np.arange(nx) + 0.5) * dx
    groove = np.mod(xc, 100e-9) >= 50e-9
    wpm[groove, :, top - 10:top] = 0.0
    gm[groove, :, top - 10:top] = 0.0
    rng = np.random.default_rng(SEED0 + 4)
    sig = (50e-9, 10e-9, 10e-9)
    center = (npml * dx + 3 * sig[0], ny * dx / 2, aloof_center(top * dx, 5e-9, sig[2]))
    bunch = gaussian_bunch(rng, nparticles, center, sig, 100e3)
    zp = top * dx + 2e-9
    probes = np.array([[nx * dx * f, ny * dx / 2, zp] for f in (0.5, 0.625, 0.75)])
    return Workload("grating40nm_512x256x256_cpml12", nx, ny, nz, dx, courant_dt(dx),
                    (CPML,) * 3, npml, wpm, gm, bunch, probes, spectrum_omegas(), 20000,
                    sort_every=20)


def grating_shard(nshards=8, rank=2, nparticles=10_000_000):
    """One rank's share of the grating workload under an x-slab split.

    Cells [rank * nx / nshards, (rank + 1) * nx / nshards) of the 512-cell x
    axis with the film, grooves and the bunch particles inside them (positions
    shifted to the slab).  The slab's x faces are periodic here: on one GPU
    that reads the one neighbour plane per face a halo exchange would deliver
    (the exchange itself is not modelled).  Rank 2 holds the bunch centre, so
    it carries the most particles of the split.
    """
    full = grating_large(nparticles)
    w = full.nx // nshards
    x0 = rank * w
    b = full.bunch
    keep = np.nonzero((b.x >= x0 * full.dx) & (b.x < (x0 + w) * full.dx))[0]
    sub = b.subset(keep)
    sub.x = sub.x - x0 * full.dx
    zp = full.probes[0, 2]
    probes = np.array([[w * full.dx / 2, full.ny * full.dx / 2, zp]])
    return Workload(f"grating40nm_shard{rank}of{nshards}_{w}x{full.ny}x{full.nz}", w, full.ny, full.nz,
                    full.dx, full.dt, (PERIODIC, CPML, CPML), full.npml,
                    np.ascontiguousarray(full.wp_map[x0:x0 + w]),
                    np.ascontiguousarray(full.gamma_map[x0:x0 + w]), sub, probes, full.omega,
                    full.steps, sort_every=full.sort_every)


def batched_sweep(nparticles=200_000):
    """16 instances: film 5..80 nm, energy U(20, 80) keV, grids 128x64x64..192x96x96.

    Each grid dimension grows linearly with the film thickness and is rounded
    to a multiple of 16.
    """
    rng = np.random.default_rng(SEED0 + 2)
    energies = rng.uniform(20e3, 80e3, 16)
    out = []
    dx, npml = 2e-9, 8
    for i, t_nm in enumerate(range(5, 85, 5)):
        f = (t_nm - 5) / 75.0
        nx = int(round((128 + 64 * f) / 16)) * 16
        ny = int(round((64 + 32 * f) / 16)) * 16
        nz = ny
        top = nz // 2
        tc = int(round(t_nm * 1e-9 / dx))
        wpm, gm = film_maps(nx, ny, nz, top - tc, top)
        sig = (20e-9, 5e-9, 5e-9)
        center = (npml * dx + 3 * sig[0], ny * dx / 2, aloof_center(top * dx, 8e-9, sig[2]))
        bunch = gaussian_bunch(rng, nparticles, center, sig, float(energies[i]))
        zp = top * dx + 2e-9
        probes = np.array([[nx * dx * q, ny * dx / 2, zp] for q in (0.5, 0.625, 0.75)])
        out.append(Workload(f"film{t_nm}nm_{nx}x{ny}x{nz}_cpml8", nx, ny, nz, dx,
                            courant_dt(dx), (CPML,) * 3, npml, wpm, gm, bunch, probes,
                            spectrum_omegas(), 3000, sort_every=20,
                            meta={"thickness_nm": t_nm, "energy_ev": float(energies[i])}))
    return out


# Drude constants of the paper's own workload (Sec. III), eps_inf = 1.
PAPER_WP = 1.2e16
PAPER_GAMMA = 1.45e13


def paper_film(d_nm, dx=2e-9, t_fs=40.0, gap_nm=10.0, kinetic_ev=100e3, nparticles=4000,
               npml=10, current_density=1e9, below_nm=100.0, above_nm=100.0, probe_um=1.5,
               gamma=PAPER_GAMMA, past_probe_nm=None, ny=4, pml_alpha=0.0, f_thz=(500.0, 1800.0, 1.0)):
    """The paper's geometry (Sec. III): film normal along x, bunch along +z,
    periodic y, Ez probe on the film surface 1.5 um downstream of the bunch start.

    x: CPML | 100 nm vacuum | film d | 100 nm vacuum | CPML (the surface modes
    decay over ~30 nm into vacuum; with 30-50 nm gaps the layers pulled the
    thin-film lower branch by ~100 THz).  y: 4 periodic cells,
    the bunch uniform across them (a sheet beam: the modes it drives have no y
    wavenumber, as in the dispersion relation of Table 1).  z: long enough that
    the bunch stays clear of the far layer for t_fs.  Bunch: Gaussian in x
    (sigma 2 nm, centre gap_nm above the film) and z (sigma 5 nm), 3-sigma
    truncated, cold, along +z, with the peak current density of Sec. III
    (100 kA/cm^2 = 1e9 A/m^2): Q = J ly 2 pi sx sz / v.  At that density the
    bunch's space charge is negligible and it moves on straight lines.
    probe_um: one distance or several (one probe each, same run); the first
    is the paper's.  past_probe_nm: end the domain this far past the last probe
    instead (the bunch then leaves through the far absorbing layer and the
    probes record the surface modes ringing down; long records stay
    affordable).  ny: periodic cells across the beam (the sheet bunch drives
    no y wavenumber, so one cell is the same problem).  pml_alpha: CFS shift
    alpha_max of the layers (S/m).  f_thz: (first, last, step) of the probe
    DFT grid in THz.
    """
    rng = np.random.default_rng(SEED0 + 5)
    i0 = npml + int(round(below_nm * 1e-9 / dx))
    i1 = i0 + int(round(d_nm * 1e-9 / dx))
    nx = i1 + int(round(above_nm * 1e-9 / dx)) + npml
    dt = courant_dt(dx)
    pz = np.atleast_1d(np.asarray(probe_um, dtype=np.float64))
    g = 1.0 + kinetic_ev / MEC2_EV
    v = C_LIGHT * np.sqrt(1.0 - 1.0 / (g * g))
    steps = int(np.ceil(t_fs * 1e-15 / dt))
    z0 = (npml + 12) * dx + 15e-9
    zps = z0 + pz * 1e-6
    zp = zps[0]
    if past_probe_nm is None:
        z_end = max(z0 + v * steps * dt + 80e-9, zps.max() + 200e-9)
    else:
        z_end = zps.max() + past_probe_nm * 1e-9
    nz = int(np.ceil(z_end / dx)) + npml
    wpm = np.zeros((nx, ny, nz))
    gm = np.zeros((nx, ny, nz))
    wpm[i0:i1] = PAPER_WP
    gm[i0:i1] = gamma
    top = i1 * dx
    xs = top + gap_nm * 1e-9 + 2e-9 * truncated_normal(rng, nparticles)
    ys = rng.uniform(0.0, ny * dx, nparticles)
    zs = z0 + 5e-9 * truncated_normal(rng, nparticles)
    u = beam_u(kinetic_ev)
    charge = current_density * ny * dx * 2 * np.pi * 2e-9 * 5e-9 / v
    bunch = Bunch(xs, ys, zs, np.zeros(nparticles), np.zeros(nparticles), np.full(nparticles, u),
                  -E_CHARGE, M_E, charge / (nparticles * E_CHARGE))
    probes = np.array([[top + 1e-9, (ny // 2) * dx, z] for z in zps])
    omega = 2 * np.pi * 1e12 * np.arange(*f_thz)
    return Workload(f"paperfilm{d_nm}nm_{nx}x{ny}x{nz}", nx, ny, nz, dx, dt, (CPML, PERIODIC, CPML),
                    npml, wpm, gm, bunch, probes, omega, steps,
                    pml=(3.0, 1.0, 1.0, float(pml_alpha)), sort_every=20,
                    meta={"thickness_nm": d_nm, "z0": z0, "z_probe": zp, "z_probes": zps, "v": v,
                          "film_top": top, "gamma": gamma})


# ---------------------------------------------------------------------------
# Smooth initial fields (sampled by each side at its own Yee positions)
# ---------------------------------------------------------------------------

class CavityField:
    """Sum of divergence-free PEC-cavity mode shapes with seeded amplitudes.

    Ex ~ cos(kx x) sin(ky y) sin(kz z), Ey ~ sin cos sin, Ez ~ sin sin cos with
    k_a = pi m_a / L_a and amplitude vector orthogonal to k: tangential E
    vanishes on every wall of the box [0,Lx]x[0,Ly]x[0,Lz].
    """

    def __init__(self, L, seed, nmodes=6, mmax=3, amplitude=1.0):
        rng = np.random.default_rng(seed)
        self.L = np.asarray(L, dtype=np.float64)
        self.modes = []
        for _ in range(nmodes):
            m = rng.integers(1, mmax + 1, size=3)
            k = np.pi * m / self.L
            a = rng.standard_normal(3)
            a -= k * (a @ k) / (k @ k)
            self.modes.append((k, amplitude * a / np.linalg.norm(a)))

    def __call__(self, comp, X, Y, Z):
        out = np.zeros(np.broadcast(X, Y, Z).shape)
        for k, a in self.modes:
            cx, sx = np.cos(k[0] * X), np.sin(k[0] * X)
            cy, sy = np.cos(k[1] * Y), np.sin(k[1] * Y)
            cz, sz = np.cos(k[2] * Z), np.sin(k[2] * Z)
            if comp == 0:
                out += a[0] * cx * sy * sz
            elif comp == 1:
                out += a[1] * sx * cy * sz
            else:
                out += a[2] * sx * sy * cz
        return out


class GaussianPulse:
    """A localized smooth E pulse: E_c = A_c exp(-|r - r0|^2 / (2 w^2))."""

    def __init__(self, center, width, amplitude):
        self.c = np.asarray(center, dtype=np.float64)
        self.w = float(width)
        self.a = np.asarray(amplitude, dtype=np.float64)

    def __call__(self, comp, X, Y, Z):
        r2 = (X - self.c[0]) ** 2 + (Y - self.c[1]) ** 2 + (Z - self.c[2]) ** 2
        return self.a[comp] * np.exp(-r2 / (2 * self.w ** 2))


def yee_positions(kind, comp, n, dx):
    """Meshgrids (X, Y, Z) in metres of component `comp` of E or H on the full
    staggered lattice of an (nx, ny, nz)-cell box: E_c sits at half cells along
    c, H_c at half cells across c.  Shapes match the full-lattice extents."""
    axes = []
    for a in range(3):
        half = (a == comp) if kind == "E" else (a != comp)
        if half:
            axes.append((np.arange(n[a]) + 0.5) * dx)
        else:
            axes.append(np.arange(n[a] + 1) * dx)
    return np.meshgrid(*axes, indexing="ij")


def sample_field(fn, kind, n, dx):
    """The three components of `fn` sampled on the full staggered lattice."""
    return [fn(c, *yee_positions(kind, c, n, dx)) for c in range(3)]
