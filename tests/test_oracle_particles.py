"""Pins of the oracle's particle, deposit, probe and boundary parts.

Expected values come from closed forms (Boris rotation angle, exact
impulse under pure E, E x B drift), exactness properties (affine gather),
conservation laws checked with an independent brute-force charge density,
and continuum physics (surface plasmon at wp/sqrt(2), CPML reflection).
"""
import numpy as np
import pytest

import pic_inputs as pi


def test_boris_pure_magnetic_rotation(oracle_mod):
    """E = 0: |u| is conserved and u turns about B by 2 atan(|q| B dt / (2 gamma m))."""
    po = oracle_mod
    c = po.constants()[0]
    q, m, dt = -pi.E_CHARGE, pi.M_E, 1e-15
    B = np.array([0.0, 0.0, 50.0])
    u = np.array([0.6 * c, 0.2 * c, 0.1 * c])
    g = np.sqrt(1 + (u @ u) / c ** 2)
    u1 = po.boris(q, m, dt, np.zeros(3), B, u)
    assert abs(np.linalg.norm(u1) / np.linalg.norm(u) - 1) < 1e-15
    ang = np.arctan2(u[0] * u1[1] - u[1] * u1[0], u[0] * u1[0] + u[1] * u1[1])
    expect = -np.sign(q) * 2 * np.arctan(abs(q) * 50.0 * dt / (2 * g * m))
    assert abs(ang - expect) < 1e-13
    assert u1[2] == u[2]


def test_boris_pure_electric_impulse(oracle_mod):
    """B = 0: u^{n+1/2} = u^{n-1/2} + q E dt / m exactly."""
    po = oracle_mod
    q, m, dt = -pi.E_CHARGE, pi.M_E, 2e-18
    E = np.array([3e9, -1e9, 5e8])
    u = np.array([1e8, 2e7, -3e7])
    u1 = po.boris(q, m, dt, E, np.zeros(3), u)
    assert np.allclose(u1, u + q * E * dt / m, rtol=1e-15, atol=1e-9)


def test_boris_exb_drift(oracle_mod):
    """Crossed E, B (E << cB): the gyro-averaged velocity is E x B / B^2."""
    po = oracle_mod
    c = po.constants()[0]
    q, m = -pi.E_CHARGE, pi.M_E
    B = np.array([0.0, 0.0, 10.0])
    E = np.array([1e5, 0.0, 0.0])  # drift 1e4 m/s along -y
    wc = abs(q) * 10.0 / m
    dt = 2 * np.pi / wc / 400
    u = np.zeros(3)
    vs = []
    for _ in range(400 * 20):
        u = po.boris(q, m, dt, E, B, u)
        vs.append(u / np.sqrt(1 + (u @ u) / c ** 2))
    v = np.mean(vs, axis=0)
    drift = np.cross(E, B) / (B @ B)
    assert np.abs(v - drift).max() < 2e-3 * np.linalg.norm(drift)


def test_free_particle_moves_at_u_over_gamma(oracle_mod):
    """No field (a vanishing charge): each step moves x by dt u / gamma, with
    gamma = sqrt(1 + |u|^2 / c^2), folded on periodic axes."""
    po = oracle_mod
    c = po.constants()[0]
    n, dx = 12, 5e-9
    dt = pi.courant_dt(dx)
    z = np.zeros((n, n, n))
    o = po.OracleSim(n, n, n, dx, dt, bc=(po.PERIODIC,) * 3, wp_map=z, gamma_map=z)
    u = np.array([[0.9 * c, -0.4 * c, 0.25 * c], [-0.1 * c, 0.05 * c, 2.5 * c]])
    x0 = np.array([[3.3 * dx, 7.1 * dx, 0.4 * dx], [10.9 * dx, 1.2 * dx, 5.5 * dx]])
    o.set_particles(x0[:, 0], x0[:, 1], x0[:, 2], u[:, 0], u[:, 1], u[:, 2], -pi.E_CHARGE, pi.M_E, 1e-30)
    steps = 40
    o.step(steps)
    P = o.particles()
    g = np.sqrt(1 + (u * u).sum(1) / c ** 2)
    expect = np.mod(x0 + steps * dt * u / g[:, None], n * dx)
    got = np.stack(P[:3], axis=1)
    assert np.abs(got - expect).max() < 1e-9 * dx
    assert np.array_equal(np.stack(P[3:6], axis=1), u)


def test_gather_is_exact_on_affine_fields(oracle_mod):
    """Trilinear interpolation on each component's staggered lattice reproduces
    any affine field exactly; B^n averages the two stored H time levels."""
    po = oracle_mod
    c, mu0, eps0 = po.constants()
    n = (8, 7, 9)
    dx = 3e-9
    s = po.OracleSim(*n, dx, 1e-18)
    rng = np.random.default_rng(11)
    coefE = rng.standard_normal((3, 4))
    coefH = rng.standard_normal((3, 4))
    coefHp = rng.standard_normal((3, 4))

    def aff(cf, X, Y, Z):
        return cf[0] + cf[1] * X / dx + cf[2] * Y / dx + cf[3] * Z / dx

    for q in range(3):
        s.E[q][...] = aff(coefE[q], *pi.yee_positions("E", q, n, dx))
        s.H[q][...] = aff(coefH[q], *pi.yee_positions("H", q, n, dx))
        s.Hprev[q][...] = aff(coefHp[q], *pi.yee_positions("H", q, n, dx))
    for _ in range(50):
        p = (np.array([1.0, 1.0, 1.0]) + rng.random(3) * (np.array(n) - 2.0)) * dx
        E, B = s.gather(p)
        for q in range(3):
            assert abs(E[q] - aff(coefE[q], *p)) < 1e-12 * 20
            Bref = mu0 * 0.5 * (aff(coefH[q], *p) + aff(coefHp[q], *p))
            assert abs(B[q] - Bref) < 1e-12 * 20 * mu0


def _cic_rho(n, dx, pos, qw, periodic=(False,) * 3):
    """Brute-force node-centred cloud-in-cell charge density."""
    rho = np.zeros((n[0] + 1, n[1] + 1, n[2] + 1))
    X = np.asarray(pos) / dx
    i0 = np.floor(X).astype(int)
    f = X - i0
    for a in (0, 1):
        for b in (0, 1):
            for cc in (0, 1):
                w = (f[0] if a else 1 - f[0]) * (f[1] if b else 1 - f[1]) * (f[2] if cc else 1 - f[2])
                idx = [i0[0] + a, i0[1] + b, i0[2] + cc]
                for d in range(3):
                    if periodic[d]:
                        idx[d] %= n[d]
                rho[tuple(idx)] += qw * w / dx ** 3
    return rho


def _div_nodes(Jb, n, dx):
    """Node divergence of an edge field on the full lattice (zero beyond the box)."""
    div = np.zeros((n[0] + 1, n[1] + 1, n[2] + 1))
    jx = np.zeros((n[0] + 2, n[1] + 1, n[2] + 1))
    jx[1:-1] = Jb[0]
    jy = np.zeros((n[0] + 1, n[1] + 2, n[2] + 1))
    jy[:, 1:-1] = Jb[1]
    jz = np.zeros((n[0] + 1, n[1] + 1, n[2] + 2))
    jz[:, :, 1:-1] = Jb[2]
    div += (jx[1:] - jx[:-1]) / dx
    div += (jy[:, 1:] - jy[:, :-1]) / dx
    div += (jz[:, :, 1:] - jz[:, :, :-1]) / dx
    return div


@pytest.mark.parametrize("move", [(0.13, 0.0, 0.0), (0.7, -0.4, 0.25), (-0.95, 0.9, -0.6),
                                  (0.05, 0.02, -0.99)])
def test_single_move_deposit_conserves_charge(oracle_mod, move):
    """Esirkepov deposit: (rho1 - rho0)/dt + div J = 0 at every node (checked with an
    independent CIC density) and sum_edges J dV = q w (x1 - x0)/dt per axis."""
    po = oracle_mod
    n = (8, 8, 8)
    dx, dt = 2e-9, 1e-18
    s = po.OracleSim(*n, dx, dt)
    s.set_particles([0.0], [0.0], [0.0], [0.0], [0.0], [0.0], -pi.E_CHARGE, pi.M_E, 5.0)
    qw = -pi.E_CHARGE * 5.0
    p0 = np.array([3.4, 4.71, 3.05]) * dx
    p1 = p0 + np.array(move) * dx
    s.deposit_move(p0, p1)
    Jb = [a.copy() for a in s.Jb]
    cont = (_cic_rho(n, dx, p1, qw) - _cic_rho(n, dx, p0, qw)) / dt + _div_nodes(Jb, n, dx)
    scale = abs(qw) / dx ** 3 / dt
    assert np.abs(cont).max() < 1e-13 * scale
    for a in range(3):
        total = Jb[a].sum() * dx ** 3
        assert abs(total - qw * (p1[a] - p0[a]) / dt) < 1e-12 * abs(qw) * dx / dt


def test_gauss_law_constant_in_vacuum_with_bunch(oracle_mod):
    """With charge-conserving deposition, G = eps0 div E - rho stays equal to its
    initial value -rho^0 at every interior node (E^0 = 0) while no particle
    leaves the box."""
    po = oracle_mod
    c = po.constants()[0]
    n = (24, 16, 16)
    dx = 5e-9
    dt = pi.courant_dt(dx)
    s = po.OracleSim(*n, dx, dt)
    rng = np.random.default_rng(5)
    N = 60
    b = pi.gaussian_bunch(rng, N, (5 * dx, 8 * dx, 8 * dx), (dx, dx, dx), 200e3)
    # add transverse momentum so particles cross cells in every direction
    uy = 0.1 * c * rng.standard_normal(N)
    uz = 0.1 * c * rng.standard_normal(N)
    s.set_particles(b.x, b.y, b.z, b.ux, uy, uz, b.q, b.m, b.w)
    G0 = s.gauss()
    rho0 = s.rho()
    for _ in range(6):
        s.step(10)
        assert s.particles()[6].all()
        G = s.gauss()
        assert np.abs(G - G0)[1:-1, 1:-1, 1:-1].max() < 1e-12 * np.abs(rho0).max()


def test_gauss_law_with_metal_polarization(oracle_mod):
    """Inside and around a Drude slab, eps0 div E + div P - rho is conserved,
    with P accumulated from the Drude current (D = eps0 E + P, Eq. 2)."""
    po = oracle_mod
    w = pi.slab_tiny()
    s = po.OracleSim(w.nx, w.ny, w.nz, w.dx, w.dt, bc=w.bc, wp_map=w.wp_map,
                     gamma_map=w.gamma_map)
    b = w.bunch
    sel = np.arange(0, b.n, 10)
    bb = b.subset(sel)
    # push some charge through the slab
    s.set_particles(bb.x, bb.y, bb.z - 25e-9, bb.ux, bb.uy, -0.3 * bb.ux, bb.q, bb.m, bb.w * 1e3)
    G0 = s.gauss()
    s.step(80)
    G = s.gauss()
    scale = np.abs(s.rho()).max() + np.abs(G0).max()
    assert np.abs(G - G0)[1:-1, 1:-1, 1:-1].max() < 1e-9 * scale
    assert np.abs(np.concatenate([p.ravel() for p in s.P])).max() > 0


def test_probe_dft_of_exact_cavity_mode(oracle_mod):
    """For the exact discrete cavity mode E^n = cos(n th) E^0, the probe
    accumulator equals dt E0_p sum_{n=1}^N cos(n th) exp(-i w n dt), summed here
    in closed form as two geometric series."""
    po = oracle_mod
    c, mu0, eps0 = po.constants()
    n = (10, 10, 10)
    dx = 5e-9
    dt = pi.courant_dt(dx)
    k = np.pi * np.array([1, 1, 2]) / (np.array(n) * dx)
    K = 2 / dx * np.sin(k * dx / 2)
    A = np.array([0.3, 0.5, 0.0])
    A -= K * (A @ K) / (K @ K)
    s = po.OracleSim(*n, dx, dt)
    for q in range(3):
        X = pi.yee_positions("E", q, n, dx)
        Y = pi.yee_positions("H", q, n, dx)
        shE = np.ones_like(X[0])
        shH = np.ones_like(Y[0])
        for a in range(3):
            shE = shE * (np.cos if a == q else np.sin)(k[a] * X[a])
            shH = shH * (np.sin if a == q else np.cos)(k[a] * Y[a])
        s.E[q][...] = A[q] * shE
        s.H[q][...] = dt / (2 * mu0) * np.cross(K, A)[q] * shH
    th = 2 * np.arcsin(c * dt / dx * np.sqrt(np.sum(np.sin(k * dx / 2) ** 2)))
    probes = np.array([[3 * dx, 4 * dx, 3.3 * dx], [7 * dx, 2 * dx, 6.9 * dx]])
    om = np.array([0.5, 1.0, 1.3]) * th / dt
    s.set_probes(probes, om)
    e0 = []
    for p in probes:
        i, j, kk = int(np.floor(p[0] / dx + 0.5)), int(np.floor(p[1] / dx + 0.5)), int(np.floor(p[2] / dx))
        e0.append(s.E[2][i, j, kk])
    N = 400
    s.step(N)
    F = s.probe()

    def geo(z):  # sum_{n=1}^N z^n
        return z * (1 - z ** N) / (1 - z) if abs(1 - z) > 1e-14 else N

    for pi_, E0p in enumerate(e0):
        for mi, w in enumerate(om):
            a = np.exp(1j * (th - w * dt))
            b = np.exp(1j * (-th - w * dt))
            ref = dt * E0p * 0.5 * (geo(a) + geo(b))
            assert abs(F[pi_, mi] - ref) < 1e-9 * dt * N * abs(E0p) + 1e-300


def _spp_rel_error(po, refine):
    """Surface-plasmon ring-down of one flat Drude/vacuum interface at fixed
    physical k and wp; returns (w_measured / w_continuum - 1, w_continuum / wp)."""
    import os
    import sys
    sys.path.insert(0, os.path.dirname(__file__))
    import dispersion
    c = po.constants()[0]
    nx, ny, nz = 64 * refine, 1, 120 * refine
    dx = 5e-9 / refine
    dt = pi.courant_dt(dx)
    k = 2 * np.pi / (nx * dx)
    wp = 0.1 * k * c
    wpm = np.zeros((nx, ny, nz))
    wpm[:, :, : nz // 2] = wp
    s = po.OracleSim(nx, ny, nz, dx, dt, bc=(po.PERIODIC, po.PERIODIC, po.PEC), wp_map=wpm,
                     gamma_map=np.zeros_like(wpm))
    # quasi-static surface-charge field: E = -grad(cos(kx) exp(-k|z - z0|))
    z0 = nz // 2 * dx
    X, Y, Z = pi.yee_positions("E", 0, (nx, ny, nz), dx)
    s.E[0][...] = np.sin(k * X) * np.exp(-k * np.abs(Z - z0))
    X, Y, Z = pi.yee_positions("E", 2, (nx, ny, nz), dx)
    s.E[2][...] = np.sign(Z - z0) * np.cos(k * X) * np.exp(-k * np.abs(Z - z0))
    s.set_probes(np.array([[0.0, 0.0, z0 + 10e-9]]), np.array([1.0]))
    steps = 26000 * refine
    series = np.empty(steps)
    for t in range(steps):
        s.step(1)
        series[t] = s.probe_values()[0]
    win = np.hanning(steps)
    spec = np.abs(np.fft.rfft((series - series.mean()) * win, n=16 * steps))
    freqs = np.fft.rfftfreq(16 * steps, dt) * 2 * np.pi
    band = (freqs > 0.5 * wp) & (freqs < 0.9 * wp)
    w_meas = freqs[band][np.argmax(spec[band])]
    w_theory = dispersion.single_interface_at_k(wp, k)
    return w_meas / w_theory - 1, w_theory / wp


@pytest.mark.slow
def test_single_interface_surface_plasmon_converges_to_continuum(oracle_mod):
    """A flat Drude/vacuum interface (Eq. 1, eps_inf = 1) at k c = 10 wp rings at
    the surface-plasmon frequency, whose continuum single-interface root here
    is 0.70622 wp (-> wp/sqrt(2) as k c/wp grows).  The grid-aligned interface
    (tangential E on the interface plane counted as vacuum) gives a first-order
    error in dx: it must halve when dx halves, and the Richardson-extrapolated
    frequency must match the continuum root."""
    po = oracle_mod
    e1, ratio = _spp_rel_error(po, 1)
    e2, _ = _spp_rel_error(po, 2)
    assert abs(ratio - 0.70622) < 2e-4
    assert abs(ratio * np.sqrt(2) - 1) < 2e-3
    assert abs(e1) < 0.035 and abs(e2) < 0.016
    assert 0.35 < e2 / e1 < 0.6
    assert abs(2 * e2 - e1) < 5e-3


def test_cpml_reflection_below_minus_40_db(oracle_mod):
    """A broadband pulse leaving a CPML-terminated box (m = 3 grading,
    sigma_max = 0.8 (m+1)/(eta0 dx), 8 cells) matches the same pulse in a box so
    large that its walls are not yet felt, to better than 1 % (-40 dB) of the peak."""
    po = oracle_mod
    dx = 5e-9
    dt = pi.courant_dt(dx)
    small, npml, big = 48, 8, 208
    pulse_w = 3 * dx
    runs = {}
    for nn, bc, npm in ((small, po.CPML, npml), (big, po.PEC, 0)):
        n = (nn, 1, nn)
        s = po.OracleSim(*n, dx, dt, bc=(bc, po.PERIODIC, bc), npml=npm)
        ctr = np.array([nn / 2 * dx, 0.0, nn / 2 * dx])
        X, Y, Z = pi.yee_positions("E", 1, n, dx)
        s.E[1][...] = np.exp(-((X - ctr[0]) ** 2 + (Z - ctr[2]) ** 2) / (2 * pulse_w ** 2))
        s.step(300)
        off = (nn - small) // 2
        runs[nn] = s.E[1][off + npml: off + small - npml + 1, 0, off + npml: off + small - npml + 1].copy()
    err = np.abs(runs[small] - runs[big]).max()
    assert err < 1e-2, err
    # and the pulse really has left: the big-box field in the window is small too
    assert np.abs(runs[big]).max() < 0.2


def test_table1_theory_column_reproduced(request):
    """The thin-film/electron-line crossings reproduce the theory column of the
    paper's Table 1 (printed to 1 THz) within 1.5 THz."""
    import os, sys
    sys.path.insert(0, os.path.dirname(__file__))
    import dispersion
    path = os.path.join(os.path.dirname(__file__), "golden", "table1_theory.txt")
    rows = np.loadtxt(path)
    beta = dispersion.beta_of(100e3)
    for d, lo, hi in rows:
        wl, wh = dispersion.film_modes_on_line(1.2e16, d * 1e-9, beta)
        fl, fh = wl / (2 * np.pi * 1e12), wh / (2 * np.pi * 1e12)
        if np.isnan(hi):
            # merged modes at 150 nm: both branches within 1.5 THz of the single value
            assert abs(fl - lo) < 1.5 and abs(fh - lo) < 1.5
        else:
            assert abs(fl - lo) < 1.5 and abs(fh - hi) < 1.5
    # thick-film limit and the large-k limit wp/sqrt(2) of Eq. 1
    w_inf = dispersion.single_interface_on_line(1.2e16, beta)
    assert abs(w_inf / (2 * np.pi * 1e12) - 1225.25) < 0.1
    k_big = 1e3 * 1.2e16 / dispersion.C
    assert abs(dispersion.single_interface_at_k(1.2e16, k_big) / (1.2e16 / np.sqrt(2)) - 1) < 1e-6
