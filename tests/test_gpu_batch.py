"""Batched simulations (pic_batch_*) vs the same simulations stepped alone.

Fields-only members must be bitwise identical to their plain runs (the batch
runs the same per-cell code, only the launch is shared), both through the
captured graph and through direct batched launches.  With particles the
float atomics of the deposit make results order-dependent at round-off, so
members are compared with their plain runs at 1e-5 and with the oracle at
the 1e-3 particle tolerance.
"""
import dataclasses
import numpy as np
import pytest

import pic_inputs as pi
from oracle import pic_oracle as po
from paper_1505_04007_amd import native

pytestmark = pytest.mark.gpu


def _rel(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def _members(with_bunch, sort_every=10):
    """Three uneven grids with different films, boundaries and bunches."""
    specs = [((40, 24, 32), (native.BC_CPML,) * 3, 5, (10, 14), 30e3),
             ((64, 20, 28), (native.BC_CPML, native.BC_PERIODIC, native.BC_CPML), 4, (8, 13), 60e3),
             ((37, 19, 27), (native.BC_PEC,) * 3, 0, (6, 9), 90e3)]
    out = []
    for q, (n, bc, npml, (k0, k1), ev) in enumerate(specs):
        dx = 3e-9
        wpm, gm = pi.film_maps(*n, k0, k1)
        bunch = None
        if with_bunch:
            rng = np.random.default_rng(pi.SEED0 + 60 + q)
            bunch = pi.gaussian_bunch(rng, 400 + 100 * q, (10 * dx, n[1] / 2 * dx, (k1 + 3) * dx),
                                      (1.5 * dx,) * 3, ev)
        w = pi.Workload(f"member{q}", *n, dx, pi.courant_dt(dx), bc, npml, wpm, gm, bunch,
                        np.array([[n[0] / 2 * dx, n[1] / 2 * dx, (k1 + 0.4) * dx]]),
                        pi.spectrum_omegas(nfreq=6), 60, sort_every=sort_every if with_bunch else 0)
        pulse = pi.GaussianPulse(np.array(n) * dx * np.array([0.45, 0.5, 0.7]), 2.5 * dx,
                                 [2e5, -1e5, 3e5])
        E = pi.sample_field(pulse, "E", n, dx)
        out.append((w, [e[: n[0], : n[1], : n[2]] for e in E]))
    return out


def _sims(members):
    return [native.from_workload(w, init_E=E) for w, E in members]


@pytest.mark.parametrize("use_graph", [True, False])
def test_fields_only_batch_is_bitwise_plain(use_graph):
    members = _members(False)
    plain = _sims(members)
    for s in plain:
        s.step(37)
    sims = _sims(members)
    b = native.Batch(sims, use_graph=use_graph)
    b.step(37)
    for s, p in zip(sims, plain):
        for which in (native.FIELD_E, native.FIELD_H, native.FIELD_JPOL):
            assert np.array_equal(s.fields(which), p.fields(which))
        assert np.array_equal(s.probe(), p.probe())
        assert s.stats()["steps"] == 37
    b.close()


def test_batch_with_bunches_matches_plain_and_oracle():
    members = _members(True, sort_every=10)
    plain = _sims(members)
    for s in plain:
        s.step(45)
    sims = _sims(members)
    b = native.Batch(sims, use_graph=True)
    b.step(45)
    for s, p in zip(sims, plain):
        assert _rel(s.fields(native.FIELD_E), p.fields(native.FIELD_E)) <= 1e-5
        assert s.stats()["pushes"] == p.stats()["pushes"]
    w, E = members[0]
    o = po.OracleSim(w.nx, w.ny, w.nz, w.dx, w.dt, bc=w.bc, npml=w.npml, pml=w.pml,
                     wp_map=w.wp_map, gamma_map=w.gamma_map)
    Ef = pi.sample_field(pi.GaussianPulse(np.array((w.nx, w.ny, w.nz)) * w.dx * np.array([0.45, 0.5, 0.7]),
                                          2.5 * w.dx, [2e5, -1e5, 3e5]), "E", (w.nx, w.ny, w.nz), w.dx)
    for c in range(3):
        for a in range(3):
            if a != c:
                sl = [slice(None)] * 3
                sl[a] = 0
                Ef[c][tuple(sl)] = 0.0
                sl[a] = (w.nx, w.ny, w.nz)[a]
                Ef[c][tuple(sl)] = 0.0
        o.E[c][...] = Ef[c]
    bb = w.bunch
    o.set_particles(bb.x, bb.y, bb.z, bb.ux, bb.uy, bb.uz, bb.q, bb.m, bb.w)
    o.step(45)
    Eo = np.stack([o.E[c][: w.nx, : w.ny, : w.nz] for c in range(3)])
    assert _rel(sims[0].fields(native.FIELD_E), Eo) <= 1e-3
    b.close()


def test_batch_mixing_members_with_and_without_a_bunch():
    """A member without particles takes no part in the batched sorts: a batch
    of two bunches and one fields-only grid, replayed over four sort periods
    and stepped on without the graph, matches its plain runs, the fields-only
    member bit for bit."""
    members = _members(True, sort_every=10)
    w1, E1 = members[1]
    members[1] = (dataclasses.replace(w1, bunch=None, sort_every=0), E1)
    plain = _sims(members)
    for s in plain:
        s.step(45)
    sims = _sims(members)
    b = native.Batch(sims, use_graph=True)
    b.step(45)
    for q, (s, p) in enumerate(zip(sims, plain)):
        if q == 1:
            for which in (native.FIELD_E, native.FIELD_H, native.FIELD_JPOL):
                assert np.array_equal(s.fields(which), p.fields(which))
            assert s.stats()["pushes"] == 0
        else:
            assert _rel(s.fields(native.FIELD_E), p.fields(native.FIELD_E)) <= 1e-5
            assert s.stats()["pushes"] == p.stats()["pushes"] > 0
            Ps, Pp = s.particles(), p.particles()
            assert np.abs(Ps[:3] - Pp[:3]).max() <= 1e-5 * w1.dx
    b.close()


def test_batch_rejects_mismatched_members():
    m1 = _members(True, sort_every=10)[:1]
    m2 = _members(True, sort_every=7)[1:2]
    sims = _sims(m1) + _sims(m2)
    with pytest.raises(native.PicError) as ei:
        native.Batch(sims)
    assert ei.value.status == native.PIC_EINVAL
    with pytest.raises(native.PicError):
        native.Batch([sims[0], sims[0]])


def test_batch_rejects_the_fixed_point_deposit():
    w, E = _members(True, sort_every=10)[0]
    sim = native.from_workload(w, init_E=E, deposit_mode=2)
    with pytest.raises(native.PicError) as ei:
        native.Batch([sim])
    assert ei.value.status == native.PIC_ENOTSUP
