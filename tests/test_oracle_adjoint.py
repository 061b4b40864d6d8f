"""Pins of the oracle's adjoint and gradient (the differentiable form).

The adjoint is the transpose of one linear field step (H, Drude J, E with
CPML memories and periodic copies; the bunch current held fixed).  It is
pinned by
  * the dot-product identity <y, M x> = <M^T y, x> for every pair of state
    blocks (E, H, J and each CPML memory), so a coupling transposed to the
    wrong block, a dropped term, a sign or an index shift fails on its own;
  * central finite differences of the probe spectral power L in FP64 with the
    bunch current prescribed, on seeded metal cells, for dL/dwp and dL/dgamma;
  * L itself against the oracle's forward probe DFT (a separate code path);
  * the closed form dL/dwp = 0 where wp = 0 (the Drude cb coefficient of Eq. 6
    is quadratic in wp).
"""
import numpy as np
import pytest

import pic_inputs as pi


def _blocks(o, adjoint):
    """Named views of every state array of the linear step (forward or adjoint)."""
    out = {}
    E, H, J = (o.Ea, o.Ha, o.Ja) if adjoint else (o.E, o.H, o.J)
    for c in range(3):
        out[f"E{c}"] = E[c]
        out[f"H{c}"] = H[c]
        out[f"J{c}"] = J[c]
        for f in "EH":
            for a in range(3):
                v = o.psi(f, c, a, adjoint=adjoint)
                if v is not None:
                    out[f"psi{f}{c}{a}"] = v
    return out


def _make(po, n, bc, npml, pml, rng, metal_frac=0.5):
    dx = 3e-9
    dt = pi.courant_dt(dx)
    wp = np.where(rng.random(n) < metal_frac, pi.AG_WP * (1 + 0.2 * rng.random(n)), 0.0)
    g = pi.AG_GAMMA * (1 + 3 * rng.random(n)) * 50  # strong damping so ca differs from 1
    return po.OracleSim(*n, dx, dt, bc=bc, npml=npml, pml=pml, wp_map=wp, gamma_map=g)


CASES = [
    # alpha_max of a few 1e6 S/m is comparable with sigma_max (~1e7 S/m at 3 nm)
    ((5, 4, 6), ("CPML", "PERIODIC", "PEC"), 2, (3.0, 1.0, 2.5, 3e6)),
    ((6, 5, 4), ("CPML", "CPML", "CPML"), 2, (2.0, 1.3, 1.7, 1e6)),
    ((4, 5, 3), ("PERIODIC", "PERIODIC", "PERIODIC"), 0, (3.0, 1.0, 1.0, 0.0)),
    ((4, 3, 5), ("PEC", "PEC", "CPML"), 2, (3.0, 1.0, 1.0, 0.0)),
]


@pytest.mark.parametrize("case", range(len(CASES)))
def test_adjoint_step_is_transpose_blockwise(oracle_mod, case):
    po = oracle_mod
    n, bcn, npml, pml = CASES[case]
    bc = tuple(getattr(po, b) for b in bcn)
    rng = np.random.default_rng(pi.SEED0 + 700 + case)
    o = _make(po, n, bc, npml, pml, rng)
    names = list(_blocks(o, False))
    X0 = {k: rng.standard_normal(v.shape) for k, v in _blocks(o, False).items()}
    Y0 = {k: rng.standard_normal(v.shape) for k, v in _blocks(o, False).items()}
    couplings = 0
    for src in names:
        # forward M applied to x nonzero only in block src
        for k, v in _blocks(o, False).items():
            v[...] = X0[k] if k == src else 0.0
        o.step(1)
        Mx = {k: v.copy() for k, v in _blocks(o, False).items()}
        for dst in names:
            lhs = float(np.sum(Y0[dst] * Mx[dst]))
            o.adj_zero()
            A = _blocks(o, True)
            A[dst][...] = Y0[dst]
            o.adj_step()
            rhs = float(np.sum(_blocks(o, True)[src] * X0[src]))
            scale = float(np.sum(np.abs(Y0[dst] * Mx[dst]))) + 1e-300
            assert abs(lhs - rhs) <= 1e-12 * scale, (src, dst, lhs, rhs)
            if lhs != 0.0:
                couplings += 1
    # the step couples E, H, J and the memories in many directions; an adjoint
    # that misses a coupling would show zero here where the forward is not
    assert couplings >= len(names)


def _grad_setup(po, nsteps):
    """Film between CPML layers, periodic in y; a bunch over it; seeded map noise."""
    nx, ny, nz, dx, npml = 20, 8, 18, 2e-9, 4
    top = 9
    wp, g = pi.film_maps(nx, ny, nz, top - 3, top)
    rng = np.random.default_rng(pi.SEED0 + 710)
    metal = wp > 0
    wp[metal] *= 1.0 + 0.05 * rng.standard_normal(int(metal.sum()))
    g[metal] *= 1.0 + 0.05 * rng.standard_normal(int(metal.sum()))
    dt = pi.courant_dt(dx)
    bc = (po.CPML, po.PERIODIC, po.CPML)
    probes = np.array([[12 * dx, 4 * dx, (top + 1.3) * dx], [15 * dx, 4 * dx, (top + 0.7) * dx]])
    w0 = 0.68 * pi.AG_WP
    bunch = pi.gaussian_bunch(rng, 300, (7 * dx, 4 * dx, (top + 3) * dx), (1.5 * dx,) * 3, 50e3,
                              charge=1e-16)
    pulse = pi.GaussianPulse(np.array([10.0, 4.0, 13.0]) * dx, 2.0 * dx, [3e6, 0.0, -2e6])
    E0 = pi.sample_field(pulse, "E", (nx, ny, nz), dx)

    def make(wpm, gm):
        o = po.OracleSim(nx, ny, nz, dx, dt, bc=bc, npml=npml, wp_map=wpm, gamma_map=gm)
        for c in range(3):
            o.E[c][...] = E0[c]
        o.set_probes(probes, np.array([w0]))
        return o

    rec = make(wp, g)
    b = bunch
    rec.set_particles(b.x, b.y, b.z, b.ux, b.uy, b.uz, b.q, b.m, b.w)
    hist = rec.run_record_jb(nsteps)
    return make, wp, g, hist, w0, rng


def _L(o):
    return float(np.sum(np.abs(o.probe()) ** 2))


def test_gradient_matches_central_differences(oracle_mod):
    po = oracle_mod
    N = 90
    make, wp, g, hist, w0, rng = _grad_setup(po, N)
    assert np.abs(hist).max() > 0  # the bunch does drive the grid
    o = make(wp, g)
    o.prescribe_jb(hist)
    L, gw, gg = o.grad(N, w0)
    assert L > 0

    def L_of(wpm, gm):
        s = make(wpm, gm)
        s.prescribe_jb(hist)
        s.step(N)
        return _L(s)

    cells = np.argwhere(wp > 0)
    pick = cells[rng.choice(len(cells), 16, replace=False)]
    # Relative steps: L moves by ~1e-11 of itself per unit relative change of
    # one cell's gamma, so its central difference needs a larger step than wp's
    # to stay clear of FP64 round-off; truncation stays O(h^2) in both.
    for (i, j, k) in pick:
        for name, base, grad, h in (("wp", wp, gw, 1e-4), ("gamma", g, gg, 1e-2)):
            d = h * base[i, j, k]
            up, dn = base.copy(), base.copy()
            up[i, j, k] += d
            dn[i, j, k] -= d
            fd = (L_of(up, g) - L_of(dn, g)) / (2 * d) if name == "wp" else \
                 (L_of(wp, up) - L_of(wp, dn)) / (2 * d)
            ad = grad[i, j, k]
            # O(h^2) truncation, plus the round-off of L (~1e-14 L over the run) over 2d
            assert abs(ad - fd) <= 1e-6 * abs(fd) + 1e-14 * L / d, (name, (i, j, k), ad, fd)


def test_gradient_L_matches_forward_probe_dft(oracle_mod):
    po = oracle_mod
    N = 60
    make, wp, g, hist, w0, _ = _grad_setup(po, N)
    a = make(wp, g)
    a.prescribe_jb(hist)
    L, gw, gg = a.grad(N, w0)
    b = make(wp, g)
    b.prescribe_jb(hist)
    b.step(N)
    assert abs(L - _L(b)) <= 1e-13 * _L(b)
    # forward state after grad() is the state after N steps
    for c in range(3):
        np.testing.assert_array_equal(a.E[c], b.E[c])
    # dcb/dwp = 4 dt eps0 wp / (2 + gamma dt) vanishes in vacuum; J = 0 there too
    assert np.all(gw[wp == 0] == 0.0)
    assert np.all(gg[wp == 0] == 0.0)
    assert np.abs(gw[wp > 0]).max() > 0 and np.abs(gg[wp > 0]).max() > 0


def test_gradient_is_zero_without_probe_signal(oracle_mod):
    """No field and no source: L = 0 and both gradients vanish identically."""
    po = oracle_mod
    n = (8, 6, 8)
    wp, g = pi.film_maps(*n, 2, 4)
    o = po.OracleSim(*n, 2e-9, pi.courant_dt(2e-9), wp_map=wp, gamma_map=g)
    o.set_probes(np.array([[8e-9, 6e-9, 10e-9]]), np.array([1e16]))
    L, gw, gg = o.grad(20, 1e16)
    assert L == 0.0 and not gw.any() and not gg.any()


def test_box_record_replays_the_particle_run(oracle_mod):
    """The bunch current recorded on a box that holds every deposit, then
    prescribed in a fresh run without particles, reproduces the particle run's
    fields bit for bit (the source the gradient holds fixed)."""
    po = oracle_mod
    n, dx = (20, 10, 16), 3e-9
    dt = pi.courant_dt(dx)
    wp, g = pi.film_maps(*n, 4, 7, wp=pi.AG_WP, gamma=pi.AG_GAMMA)
    rng = np.random.default_rng(pi.SEED0 + 760)
    b = pi.gaussian_bunch(rng, 300, (5 * dx, 5 * dx, 10 * dx), (1.2 * dx, dx, dx), 50e3, charge=1e-16)
    bc = (po.CPML, po.PERIODIC, po.CPML)
    run = po.OracleSim(*n, dx, dt, bc=bc, npml=3, wp_map=wp, gamma_map=g)
    run.set_particles(b.x, b.y, b.z, b.ux, b.uy, b.uz, b.q, b.m, b.w)
    lo, ext = (0, 1, 5), (20, 8, 10)
    hist, outside = run.run_record_jb_box(40, lo, ext)
    assert outside == 0.0 and np.abs(hist).max() > 0
    rep = po.OracleSim(*n, dx, dt, bc=bc, npml=3, wp_map=wp, gamma_map=g)
    rep.prescribe_jb_box(lo, ext, hist)
    rep.step(40)
    for c in range(3):
        np.testing.assert_array_equal(rep.E[c], run.E[c])
        np.testing.assert_array_equal(rep.H[c], run.H[c])
    # a box that misses part of the bunch reports what it missed
    run2 = po.OracleSim(*n, dx, dt, bc=bc, npml=3, wp_map=wp, gamma_map=g)
    run2.set_particles(b.x, b.y, b.z, b.ux, b.uy, b.uz, b.q, b.m, b.w)
    _, outside2 = run2.run_record_jb_box(5, (0, 1, 5), (20, 8, 5))
    assert outside2 > 0.0
