"""Pins of the oracle's field and Drude parts against closed forms.

Every expected value here is derived independently of the oracle's code:
exact discrete Yee eigen-solutions with analytic discrete wavenumbers,
the closed-form solution of the uniform-plasma recursion, a step matrix
assembled from face/edge incidence, and continuum physics limits.
"""
import itertools

import numpy as np
import pytest

from pic_inputs import yee_positions


def _consts(po):
    return po.constants()


def _mode_shapes(kind, n, dx, k, trig_own, trig_other):
    """Per component c: product over axes of trig_own(k x) along c, trig_other across."""
    out = []
    for c in range(3):
        X = yee_positions(kind, c, n, dx)
        v = np.ones_like(X[0])
        for a in range(3):
            f = trig_own if a == c else trig_other
            v = v * f(k[a] * X[a])
        out.append(v)
    return out


@pytest.mark.parametrize("m", [(1, 2, 1), (2, 1, 3)])
def test_pec_cavity_mode_is_exact_discrete_eigenmode(oracle_mod, m):
    """Closed-form Yee dispersion sin(w dt/2) = (c dt/dx) sqrt(sum sin^2(k dx/2)).

    With E ~ A cos/sin cavity shapes, A orthogonal to the discrete
    wavenumber K = (2/dx) sin(k dx/2), and H^{-1/2} = dt/(2 mu0) (K x A),
    the leapfrog gives E^n = cos(n w dt) E^0 exactly.
    """
    po = oracle_mod
    c, mu0, eps0 = _consts(po)
    n = (12, 10, 8)
    dx = 5e-9
    dt = 0.5 * dx / (c * np.sqrt(3))
    k = np.pi * np.array(m) / (np.array(n) * dx)
    K = 2.0 / dx * np.sin(k * dx / 2)
    A = np.array([1.0, -0.3, 0.7])
    A -= K * (A @ K) / (K @ K)
    shE = _mode_shapes("E", n, dx, k, np.cos, np.sin)
    shH = _mode_shapes("H", n, dx, k, np.sin, np.cos)
    s = po.OracleSim(*n, dx, dt)
    KxA = np.cross(K, A)
    E0 = [A[q] * shE[q] for q in range(3)]
    for q in range(3):
        s.E[q][...] = E0[q]
        s.H[q][...] = dt / (2 * mu0) * KxA[q] * shH[q]
    theta = 2 * np.arcsin(c * dt / dx * np.sqrt(np.sum(np.sin(k * dx / 2) ** 2)))
    scale = max(np.abs(e).max() for e in E0)
    worst = 0.0
    for step in range(1, 301):
        s.step(1)
        for q in range(3):
            worst = max(worst, np.abs(s.E[q] - np.cos(step * theta) * E0[q]).max() / scale)
    assert worst < 1e-11, worst


def test_periodic_plane_wave_phase_advance(oracle_mod):
    """Travelling wave in a fully periodic box advances by the exact Yee phase."""
    po = oracle_mod
    c, mu0, eps0 = _consts(po)
    n = (10, 8, 6)
    dx = 4e-9
    dt = 0.5 * dx / (c * np.sqrt(3))
    m = np.array([1, -2, 1])
    k = 2 * np.pi * m / (np.array(n) * dx)
    K = 2.0 / dx * np.sin(k * dx / 2)
    A = np.array([0.4, 1.0, -0.2])
    A -= K * (A @ K) / (K @ K)
    Om = c * np.linalg.norm(K)
    w = 2 / dt * np.arcsin(Om * dt / 2)
    B = np.cross(K, A) / (mu0 * Om)
    s = po.OracleSim(*n, dx, dt, bc=(po.PERIODIC,) * 3)

    def phase(kind, q, t):
        X = yee_positions(kind, q, n, dx)
        return k[0] * X[0] + k[1] * X[1] + k[2] * X[2] - w * t

    for q in range(3):
        s.E[q][...] = A[q] * np.cos(phase("E", q, 0.0))
        s.H[q][...] = B[q] * np.cos(phase("H", q, -0.5 * dt))
    for step in (1, 37, 120):
        s.step(step - s.nstep)
        for q in range(3):
            ref = A[q] * np.cos(phase("E", q, step * dt))
            assert np.abs(s.E[q] - ref).max() < 1e-11 * np.abs(A).max()
        for q in range(3):
            ref = B[q] * np.cos(phase("H", q, (step - 0.5) * dt))
            assert np.abs(s.H[q] - ref).max() < 1e-11 * np.abs(B).max()


def _uniform_plasma(po, wp, gamma, wpdt, steps, E0=1.0):
    c, mu0, eps0 = _consts(po)
    dx = 1e-9
    dt = wpdt / wp
    n = (2, 2, 2)
    s = po.OracleSim(*n, dx, dt, bc=(po.PERIODIC,) * 3, wp_map=np.full(n, wp),
                     gamma_map=np.full(n, gamma))
    s.E[0][...] = E0
    series = [E0]
    for _ in range(steps):
        s.step(1)
        series.append(s.E[0][0, 0, 0])
        assert np.ptp(s.E[0][:2, :2, :2]) == 0.0  # stays uniform
    return np.array(series), dt


def test_lossless_plasma_oscillation_closed_form(oracle_mod):
    """k = 0 mode of a lossless Drude medium (Eqs. 6, 8 with gamma = 0).

    Eliminating J gives E^{n+1} - 2E^n + E^{n-1} = -(wp dt)^2 E^n, so with
    J^{-1/2} = 0: E^n = E0 [cos(n th) - (wp dt)^2/(2 sin th) sin(n th)],
    cos th = 1 - (wp dt)^2/2, and th/dt -> wp as dt -> 0.
    """
    po = oracle_mod
    wp, wpdt = 1.37e16, 0.05
    E, dt = _uniform_plasma(po, wp, 0.0, wpdt, 2000)
    th = np.arccos(1 - wpdt ** 2 / 2)
    nn = np.arange(E.size)
    ref = np.cos(nn * th) - wpdt ** 2 / (2 * np.sin(th)) * np.sin(nn * th)
    assert np.abs(E - ref).max() < 1e-11
    # continuum limit: discrete frequency within the O((wp dt)^2) Yee error of wp
    assert abs(th / (wp * dt) - 1) < wpdt ** 2 / 24 * 1.01


def test_damped_drude_mode_follows_eq6_eq8_recurrence(oracle_mod):
    """k = 0 mode of a collisional Drude medium, exactly (round-off).

    With curl H = 0, Eq. 6 (J^{n+1/2} = ca J^{n-1/2} + cb E^n, ca = (2 - g dt)/(2 + g dt),
    cb = 2 dt eps0 wp^2/(2 + g dt)) and Eq. 8 (E^{n+1} = E^n - (dt/eps0) J^{n+1/2})
    form a 2x2 linear map of (E^n, J^{n-1/2}); iterated in FP64 from J^{-1/2} = 0 it
    must reproduce the oracle's uniform field step by step.  A different time
    level of E in Eq. 6, or a wrong ca / cb, changes the sequence at first order.
    """
    po = oracle_mod
    _, _, eps0 = _consts(po)
    wp, wpdt = 1.3e16, 0.05
    gamma = 0.3 * wp
    E, dt = _uniform_plasma(po, wp, gamma, wpdt, 600)
    ca = (2 - gamma * dt) / (2 + gamma * dt)
    cb = 2 * dt * eps0 * wp ** 2 / (2 + gamma * dt)
    e, j = 1.0, 0.0
    ref = [e]
    for _ in range(E.size - 1):
        j = ca * j + cb * e
        e = e - dt / eps0 * j
        ref.append(e)
    ref = np.array(ref)
    assert np.abs(E - ref).max() < 1e-12
    assert np.abs(ref).min() < 0.5  # the mode does oscillate and decay over the run


def _fit_recurrence(E):
    """Least-squares (p, q) of E^{n+1} = p E^n - q E^{n-1}."""
    Amat = np.stack([E[1:-1], -E[:-2]], axis=1)
    sol, *_ = np.linalg.lstsq(Amat, E[2:], rcond=None)
    return sol


def test_collisional_damping_and_frequency(oracle_mod):
    """Damped plasma oscillation: amplitude decays at gamma/2 and oscillates at
    sqrt(wp^2 - gamma^2/4) (continuum solution of Eq. 4), up to the scheme's
    O((wp dt)^2) and O((gamma dt)^3) errors."""
    po = oracle_mod
    wp, wpdt = 1.0e16, 0.04
    gamma = 0.2 * wp
    E, dt = _uniform_plasma(po, wp, gamma, wpdt, 3000)
    p, q = _fit_recurrence(E)
    R = np.sqrt(q)
    th = np.arccos(p / (2 * R))
    decay = -np.log(R) / dt
    assert abs(decay / (gamma / 2) - 1) < 1e-5
    freq = th / dt
    cont = np.sqrt(wp ** 2 - gamma ** 2 / 4)
    assert abs(freq / cont - 1) < 2 * wpdt ** 2 / 24


def test_overdamped_drude_relaxes_at_dc_conductivity_rate(oracle_mod):
    """gamma >> wp: a Drude metal behaves as a conductor with sigma = eps0 wp^2/gamma,
    so E relaxes at the slow root s = gamma/2 - sqrt(gamma^2/4 - wp^2) ~ wp^2/gamma.
    This fixes the ADE's fixed point J* = eps0 wp^2 E / gamma."""
    po = oracle_mod
    wp = 1.0e15
    gamma = 40 * wp
    wpdt = 0.004  # gamma dt = 0.16
    E, dt = _uniform_plasma(po, wp, gamma, wpdt, 8000)
    nn = np.arange(E.size)
    sel = slice(2000, 8000)
    slope = np.polyfit(nn[sel] * dt, np.log(E[sel]), 1)[0]
    s_slow = gamma / 2 - np.sqrt(gamma ** 2 / 4 - wp ** 2)
    assert abs(-slope / s_slow - 1) < 5e-3
    assert abs(s_slow / (wp ** 2 / gamma) - 1) < 1e-2


# ---------------------------------------------------------------------------
# Dense step matrix from face/edge incidence (brute force on tiny grids)
# ---------------------------------------------------------------------------

def _edges_faces(n, periodic):
    """Physical E edges and H faces of an n-cell box.

    Edge (b, idx): along axis b, half-integer coordinate idx[b] + 1/2 on b,
    node coordinates on the other two.  Face (a, idx): normal a, node along a,
    half-integer on the others.  On a periodic axis node n is node 0.
    """
    def rng(a, half):
        if half or periodic[a]:
            return range(n[a])
        return range(n[a] + 1)

    edges, faces = [], []
    for b in range(3):
        for idx in itertools.product(*[rng(a, a == b) for a in range(3)]):
            edges.append((b, idx))
    for a in range(3):
        for idx in itertools.product(*[rng(d, d != a) for d in range(3)]):
            faces.append((a, idx))
    return edges, faces


def _norm_idx(n, periodic, idx):
    return tuple((i % n[a]) if periodic[a] else i for a, i in enumerate(idx))


def _curl_incidence(n, periodic, edges, faces):
    """C[f, e]: circulation of E around face f (right-hand rule about its normal)."""
    eid = {e: i for i, e in enumerate(edges)}
    C = np.zeros((len(faces), len(edges)))
    for fi, (a, idx) in enumerate(faces):
        b, c = (a + 1) % 3, (a + 2) % 3
        loop = []
        lo = list(idx)
        loop.append((+1, b, tuple(lo)))               # along +b at c low
        hi_b = list(idx)
        hi_b[b] += 1
        loop.append((+1, c, tuple(hi_b)))             # along +c at b high
        hi_c = list(idx)
        hi_c[c] += 1
        loop.append((-1, b, tuple(hi_c)))             # back along b at c high
        loop.append((-1, c, tuple(lo)))               # back along c at b low
        for sgn, comp, pos in loop:
            key = (comp, _norm_idx(n, periodic, pos))
            if key in eid:
                C[fi, eid[key]] += sgn
    return C


def _updated_edge(n, periodic, e):
    b, idx = e
    for a in range(3):
        if a == b or periodic[a]:
            continue
        if idx[a] == 0 or idx[a] == n[a]:
            return False
    return True


def _edge_cell(n, e):
    b, idx = e
    return tuple(min(idx[a], n[a] - 1) for a in range(3))


def _assemble(n, periodic, dx, dt, wp, gamma, consts):
    c, mu0, eps0 = consts
    edges, faces = _edges_faces(n, periodic)
    C = _curl_incidence(n, periodic, edges, faces) / dx
    ne, nf = len(edges), len(faces)
    mask = np.diag([1.0 if _updated_edge(n, periodic, e) else 0.0 for e in edges])
    ca = np.zeros(ne)
    cb = np.zeros(ne)
    for i, e in enumerate(edges):
        cell = _edge_cell(n, e)
        g, w = gamma[cell], wp[cell]
        # time-centred discretisation of dJ/dt + g J = eps0 wp^2 E at t = n dt
        ca[i] = (1 - g * dt / 2) / (1 + g * dt / 2)
        cb[i] = eps0 * w * w * dt / (1 + g * dt / 2)
    I_e, I_f = np.eye(ne), np.eye(nf)
    # state (E, H, J) -> (E', H', J')
    Hn = np.hstack([-(dt / mu0) * C, I_f, np.zeros((nf, ne))])
    # PEC-wall tangential edges are inert: neither E nor J is ever updated there
    upd = np.diag(mask)
    Jn = np.hstack([np.diag(cb * upd), np.zeros((ne, nf)), np.diag(np.where(upd > 0, ca, 1.0))])
    En = np.hstack([I_e, np.zeros((ne, nf)), np.zeros((ne, ne))]) + mask @ (
        (dt / eps0) * C.T @ Hn - (dt / eps0) * Jn)
    return edges, faces, np.vstack([En, Hn, Jn])


def _oracle_matrix(po, n, periodic, dx, dt, wp, gamma, edges, faces):
    bc = tuple(po.PERIODIC if p else po.PEC for p in periodic)
    s = po.OracleSim(*n, dx, dt, bc=bc, wp_map=wp, gamma_map=gamma)

    def store_positions(kind, comp, idx):
        node_axes = [a for a in range(3) if (a != comp if kind == "E" else a == comp)]
        opts = []
        for a in range(3):
            ch = [idx[a]]
            if periodic[a] and a in node_axes and idx[a] == 0:
                ch.append(n[a])
            opts.append(ch)
        return list(itertools.product(*opts))

    state = [("E", e) for e in edges] + [("H", f) for f in faces] + [("J", e) for e in edges]
    M = np.zeros((len(state), len(state)))
    for col, (kind, (comp, idx)) in enumerate(state):
        for arr in s.E + s.H + s.J + s.P + s.Hprev:
            arr[...] = 0.0
        tgt = {"E": s.E, "H": s.H, "J": s.J}[kind][comp]
        for pos in store_positions("H" if kind == "H" else "E", comp, idx):
            tgt[pos] = 1.0
        s.step(1)
        for row, (k2, (c2, i2)) in enumerate(state):
            M[row, col] = {"E": s.E, "H": s.H, "J": s.J}[k2][c2][i2]
    return M


@pytest.mark.parametrize("periodic", [(False, False, False), (True, True, True),
                                      (True, False, True)])
def test_step_matrix_equals_incidence_assembly(oracle_mod, periodic):
    """The oracle's one-step linear map equals the map built from the
    face/edge incidence matrix C (H' = H - dt/mu0 C E, E' = E + dt/eps0
    (C^T H' - J')), including the Drude recursion on owned edges."""
    po = oracle_mod
    consts = _consts(po)
    c = consts[0]
    n = (3, 2, 3)
    dx = 5e-9
    dt = 0.5 * dx / (c * np.sqrt(3))
    rng = np.random.default_rng(7)
    wp = np.where(rng.random(n) < 0.5, rng.uniform(0.5e16, 1.5e16, n), 0.0)
    gamma = np.where(wp > 0, rng.uniform(1e13, 1e15, n), 0.0)
    edges, faces, Mref = _assemble(n, periodic, dx, dt, wp, gamma, consts)
    M = _oracle_matrix(po, n, periodic, dx, dt, wp, gamma, edges, faces)
    ne, nf = len(edges), len(faces)
    blocks = [slice(0, ne), slice(ne, ne + nf), slice(ne + nf, 2 * ne + nf)]
    for rb in blocks:
        for cb_ in blocks:
            ref = Mref[rb, cb_]
            got = M[rb, cb_]
            scale = max(np.abs(ref).max(), 1e-300)
            assert np.abs(got - ref).max() <= 1e-12 * scale + 1e-300, (rb, cb_)


def test_vacuum_step_is_lossless_and_drude_is_dissipative(oracle_mod):
    """Spectral radius of the assembled-and-checked step map: |lambda| = 1 for the
    vacuum leapfrog under the Courant limit, <= 1 with lossy Drude edges."""
    po = oracle_mod
    consts = _consts(po)
    c = consts[0]
    n = (3, 3, 2)
    dx = 5e-9
    dt = 0.5 * dx / (c * np.sqrt(3))
    per = (False, False, False)
    zero = np.zeros(n)
    edges, faces, Mref = _assemble(n, per, dx, dt, zero, zero, consts)
    M = _oracle_matrix(po, n, per, dx, dt, zero, zero, edges, faces)
    ne, nf = len(edges), len(faces)
    EH = M[: ne + nf, : ne + nf]
    lam = np.abs(np.linalg.eigvals(EH))
    # modes with a non-trivial curl sit on the unit circle; gradient modes at 1
    assert lam.max() < 1 + 1e-9
    rng = np.random.default_rng(3)
    wp = rng.uniform(0.5e16, 1.5e16, n)
    gamma = rng.uniform(1e14, 1e15, n)
    M2 = _oracle_matrix(po, n, per, dx, dt, wp, gamma, edges, faces)
    lam2 = np.abs(np.linalg.eigvals(M2))
    assert lam2.max() < 1 + 1e-9
