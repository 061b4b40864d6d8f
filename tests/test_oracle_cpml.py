"""Pins of the oracle's absorbing layers (convolutional PML, the stand-in for
the split-field PML of Sec. III) and of its FP64 diagnostics.

None of these restates the oracle's code:

* uniform layer: with the same recursion coefficients (b, c, kappa) at every
  position of a periodic axis, a single Fourier mode's state (E, H and the two
  memories) evolves by a fixed 4 x 4 map whose eigenvalues are the roots of the
  z-domain dispersion relation of the stretched Yee scheme,
      (lam - 1)^2 / lam = -(2 S sin(k dx/2))^2 s(lam)^2,
      s(lam) = 1/kappa + c / (1 - b / lam),
  S = c0 dt / dx.  The field at a node over time must be a combination of
  exactly those four geometric sequences (least squares at round-off).  The
  relation is derived from the recursion psi' = b psi + c d, d -> d/kappa +
  psi' and the leapfrog, for a plane wave along the stretched axis;
* graded kappa layers without conductivity: a real coordinate stretching
  makes the Yee scheme a lossless scheme whose conserved energy weights every
  stored component by the product of the kappa values at its own staggered
  position, E^n . W E^{n+1} eps0 + H^{n+1/2} . W H^{n+1/2} mu0 (the staggered
  Yee energy); it must stay constant to round-off, which it does only if each
  derivative uses kappa at the right (node or half node) position;
* coefficient tables: c b^q must equal the integral over step q of the
  continuous CPML kernel, the inverse transform of 1/s(w) - 1/kappa with
  s(w) = kappa + sigma / (alpha + i w eps0),
      zeta(t) = -(sigma / (eps0 kappa^2)) exp(-(sigma/kappa + alpha) t / eps0),
  (recursive convolution with a piecewise-constant derivative, Roden & Gedney
  2000), evaluated here by numerical quadrature at each position's depth;
* diagnostics: field energy and bunch moments against values worked out by
  hand for constant fields and a handful of particles.
"""
import numpy as np
import pytest
from scipy.integrate import quad

from pic_inputs import yee_positions

PER, CPML = 1, 2


def _setup(po, n, dx=2e-9):
    c0, mu0, eps0 = po.constants()
    return c0, mu0, eps0, dx, 0.5 * dx / (c0 * np.sqrt(3.0))


def _uniform_coeffs(dt, eps0, sig_dt_eps0=0.5, kappa=1.7, alp_dt_eps0=0.1):
    """(b, c, kappa) of a layer with the given sigma dt/eps0, kappa, alpha dt/eps0."""
    sig = sig_dt_eps0 * eps0 / dt
    alp = alp_dt_eps0 * eps0 / dt
    b = np.exp(-(sig / kappa + alp) * dt / eps0)
    c = sig * (b - 1.0) / (sig * kappa + kappa * kappa * alp)
    return b, c, kappa


CASES = [(a, p) for a in range(3) for p in range(3) if p != a]


@pytest.mark.parametrize("axis,pol", CASES)
def test_uniform_cpml_mode_spans_the_dispersion_roots(oracle_mod, axis, pol):
    po = oracle_mod
    nax, m, steps = 16, 3, 60
    n = [2, 2, 2]
    n[axis] = nax
    c0, mu0, eps0, dx, dt = _setup(po, n)
    b, c, kap = _uniform_coeffs(dt, eps0)
    s = po.OracleSim(*n, dx, dt, bc=(PER, PER, PER))
    s.test_uniform_cpml(axis, b, c, kap)
    k = 2 * np.pi * m / (nax * dx)
    X = yee_positions("E", pol, tuple(n), dx)
    s.E[pol][...] = np.cos(k * X[axis])
    node = (1, 1, 1)
    series = [s.E[pol][node]]
    for _ in range(steps):
        s.step(1)
        series.append(s.E[pol][node])
    series = np.array(series)
    # p(lam) = (lam-1)^2 (lam-b)^2 + Q lam ((1/kappa + c) lam - b/kappa)^2
    Q = (2 * c0 * dt / dx * np.sin(k * dx / 2)) ** 2
    p = np.polyadd(np.polymul(np.polymul([1, -1], [1, -1]), np.polymul([1, -b], [1, -b])),
                   Q * np.polymul([1, 0], np.polymul([1 / kap + c, -b / kap], [1 / kap + c, -b / kap])))
    lam = np.roots(p)
    V = np.vander(lam, steps + 1, increasing=True).T  # V[n, j] = lam_j^n
    A, *_ = np.linalg.lstsq(V, series.astype(complex), rcond=None)
    resid = np.abs(V @ A - series).max() / np.abs(series).max()
    osc = lam[np.argmax(np.abs(np.angle(lam)))]
    print(f"axis {axis} pol {pol}: oscillating root |lam| = {abs(osc):.6f}, "
          f"w dt = {abs(np.angle(osc)):.6f}, residual {resid:.2e}")
    assert np.all(np.abs(lam) < 1.0)  # the layer damps every mode
    assert resid < 1e-11
    # the lossy recursion matters: a lossless (b = 1, c = 0) reading is far off
    lam0 = np.roots(np.polyadd(np.polymul([1, -1], [1, -1]), Q / kap ** 2 * np.array([0, 1, 0])))
    V0 = np.vander(lam0, steps + 1, increasing=True).T
    A0, *_ = np.linalg.lstsq(V0, series.astype(complex), rcond=None)
    assert np.abs(V0 @ A0 - series).max() / np.abs(series).max() > 1e-2


def test_uniform_cpml_every_axis_and_polarisation(oracle_mod):
    for axis, pol in CASES:
        test_uniform_cpml_mode_spans_the_dispersion_roots(oracle_mod, axis, pol)


def _kappa_at(pos, n, L, kmax, m):
    """kappa at position pos (cells) of an axis with layers of L cells at both ends."""
    rho = np.where(pos < L, L - pos, np.where(pos > n - L, pos - (n - L), 0.0))
    return 1.0 + (kmax - 1.0) * (np.clip(rho, 0, None) / L) ** m


def test_kappa_graded_layers_conserve_the_weighted_yee_energy(oracle_mod):
    po = oracle_mod
    n = (11, 9, 10)
    L, kmax, mgrad = 3, 4.0, 3.0
    c0, mu0, eps0, dx, dt = _setup(po, n)
    s = po.OracleSim(*n, dx, dt, bc=(CPML, CPML, CPML), npml=L, pml=(mgrad, 0.0, kmax, 0.0))
    rng = np.random.default_rng(1505040070 + 601)
    W = {}
    for kind in ("E", "H"):
        for comp in range(3):
            X = yee_positions(kind, comp, n, 1.0)  # positions in cells
            w = np.ones_like(X[0])
            for a in range(3):
                w = w * _kappa_at(X[a], n[a], L, kmax, mgrad)
            W[kind, comp] = w
            arr = s.E[comp] if kind == "E" else s.H[comp]
            v = rng.standard_normal(arr.shape) * (1.0 if kind == "E" else 1.0 / 377.0)
            # PEC walls behind the layers: tangential E and normal H are zero there
            for a in range(3):
                on_nodes = (a != comp) if kind == "E" else (a == comp)
                if on_nodes:
                    sl = [slice(None)] * 3
                    sl[a] = [0, n[a]]
                    v[tuple(sl)] = 0.0
            arr[...] = v
    energies = []
    for _ in range(80):
        E0 = [s.E[q].copy() for q in range(3)]
        s.step(1)
        F = sum(eps0 * np.sum(W["E", q] * E0[q] * s.E[q]) + mu0 * np.sum(W["H", q] * s.H[q] ** 2)
                for q in range(3))
        energies.append(F)
    energies = np.array(energies)
    drift = np.abs(energies - energies[0]).max() / energies[0]
    print(f"weighted Yee energy drift over 80 steps: {drift:.2e}")
    assert drift < 1e-12
    # the same energy with unit weights is not conserved: the stretching acts
    assert not np.allclose(s.E[0], 0.0)


def test_cpml_coefficients_are_the_recursive_convolution_of_the_kernel(oracle_mod):
    po = oracle_mod
    n = (24, 2, 2)
    L, mgrad, scale, kmax, amax = 7, 3.0, 1.3, 3.0, 3e6
    c0, mu0, eps0, dx, dt = _setup(po, n)
    s = po.OracleSim(*n, dx, dt, bc=(CPML, PER, PER), npml=L, pml=(mgrad, scale, kmax, amax))
    eta0 = mu0 * c0
    smax = scale * 0.8 * (mgrad + 1.0) / (eta0 * dx)
    checked = 0
    for h in (0, 1):
        b, c, kap = s.cpml_profile(0, h)
        pos = np.arange(len(b)) + 0.5 * h
        for i, x in enumerate(pos):
            rho = L - x if x < L else (x - (n[0] - L) if x > n[0] - L else 0.0)
            if rho <= 0.0:
                assert (b[i], c[i], kap[i]) == (1.0, 0.0, 1.0)
                continue
            r = rho / L
            sig, k_, alp = smax * r ** mgrad, 1.0 + (kmax - 1.0) * r ** mgrad, amax * (1.0 - r)
            assert abs(kap[i] - k_) <= 1e-13 * k_
            zeta = lambda u: -(sig * dt / (eps0 * k_ ** 2)) * np.exp(-(sig / k_ + alp) * dt / eps0 * u)  # noqa: E731
            for q in range(4):
                ref = quad(zeta, q, q + 1, epsabs=0.0, epsrel=1e-13)[0]
                assert abs(c[i] * b[i] ** q - ref) <= 1e-11 * abs(ref), (h, i, q)
            checked += 1
    assert checked == 4 * L  # L E-type and L H-type positions in each of the two layers


def test_diagnostics_by_hand(oracle_mod):
    """Energy of constant fields and moments of five particles, worked out by hand."""
    po = oracle_mod
    n = (5, 4, 3)
    c0, mu0, eps0, dx, dt = _setup(po, n)
    s = po.OracleSim(*n, dx, dt, bc=(0, PER, CPML), npml=1)
    ev, hv = (3.0, -2.0, 1.5), (0.01, 0.02, -0.03)
    for q in range(3):
        s.E[q][...] = ev[q]
        s.H[q][...] = hv[q]
    # stored entries, the periodic copies at y-node 4 excluded:
    # Ex (5,5,4) -> 5*4*4 = 80, Ey (6,4,4) -> 96, Ez (6,5,3) -> 6*4*3 = 72,
    # Hx (6,4,3) -> 72, Hy (5,5,3) -> 5*4*3 = 60, Hz (5,4,4) -> 80
    nE, nH = (80, 96, 72), (72, 60, 80)
    energy = 0.5 * dx ** 3 * (eps0 * sum(nE[q] * ev[q] ** 2 for q in range(3)) +
                              mu0 * sum(nH[q] * hv[q] ** 2 for q in range(3)))
    xs = np.array([0.5, 1.5, 2.0, 4.0, 4.95]) * dx
    ys = np.array([1.0, 3.0, 2.0, 2.0, 0.5]) * dx
    zs = np.array([1.0, 1.0, 2.0, 2.0, 1.5]) * dx
    ux = np.array([1e7, 2e7, 3e7, 2e7, 9e7])
    uy = np.array([0.0, 1e6, -1e6, 4e6, 0.0])
    uz = np.zeros(5)
    s.set_particles(xs, ys, zs, ux, uy, uz, -1.602176634e-19, 9.1093837015e-31, 1.0)
    d = s.diag()
    assert abs(d["energy"] - energy) <= 1e-14 * energy
    assert d["count"] == 5
    # by hand, in cells: mean x = (0.5+1.5+2+4+4.95)/5 = 2.59, mean square 47.0025/5 = 9.4005,
    # rms^2 = 9.4005 - 2.59^2 = 2.6924; y: 1.7, 18.25/5 - 1.7^2 = 0.76; z: 1.5, 12.25/5 - 2.25 = 0.2
    assert np.allclose(d["mean"], np.array([2.59, 1.7, 1.5]) * dx, rtol=1e-14, atol=0)
    assert np.allclose(d["rms"], np.sqrt([2.6924, 0.76, 0.2]) * dx, rtol=1e-12, atol=0)
    assert np.allclose(d["umean"], [3.4e7, 0.8e6, 0.0], rtol=1e-14, atol=1e-30)
    # one step in zero fields: the fifth particle (x = 4.95 cells, u = 9e7 m/s,
    # 0.083 cells per step) leaves through the x wall and drops out; the others
    # move by dt u / gamma
    for q in range(3):
        s.E[q][...] = 0.0
        s.H[q][...] = 0.0
    s.step(1)
    d = s.diag()
    g = np.sqrt(1 + (ux ** 2 + uy ** 2) / c0 ** 2)
    x1, y1 = xs + dt * ux / g, ys + dt * uy / g
    assert d["count"] == 4
    assert np.allclose(d["mean"][:2], [x1[:4].mean(), y1[:4].mean()], rtol=1e-13, atol=0)
    assert abs(d["rms"][0] - x1[:4].std()) <= 1e-12 * x1[:4].std()
