"""The one-pass field sweep against the separate H and E launches (GPU).

With field_sweep = 1 pic_step fuses each step's E update with the next
step's H update where it can; field_sweep = 0 (the default) keeps the
separate launches.  The
per-cell arithmetic is the same, so fields-only runs must agree bitwise: E, H,
J_pol, probe spectra and probe series, on every boundary kind, CPML layers
with kappa > 1 and alpha > 0, grids whose x extent fills several wavefronts
(ragged and whole), y and z extents ragged against the sweep's 4-row,
16-plane blocks, and step counts that leave a plain step before the sweeps
or not.  With a bunch the two paths differ only by the FP32 atomics' order.
One oracle parity case runs the sweep with a bunch.
"""
import dataclasses

import numpy as np
import pytest

import pic_inputs as pi
from paper_1505_04007_amd import native

pytestmark = pytest.mark.gpu

KAPPA_ALPHA = (3.0, 1.2, 3.0, 2e6)


def _case(nx, ny, nz, bc, npml, film=True, pml=None, seed=3):
    dx = 4e-9
    if film:
        wpm, gm = pi.film_maps(nx, ny, nz, max(1, nz // 3), max(2, nz // 3 + 5))
    else:
        wpm = gm = np.zeros((nx, ny, nz))
    probes = np.array([[0.55 * nx * dx, 0.45 * ny * dx, 0.6 * nz * dx], [0.2 * nx * dx, 0.8 * ny * dx, 0.3 * nz * dx]])
    w = pi.Workload(f"fused_{nx}x{ny}x{nz}", nx, ny, nz, dx, pi.courant_dt(dx), bc, npml, wpm, gm, None, probes,
                    pi.spectrum_omegas(nfreq=16), 0)
    if pml is not None:
        w = dataclasses.replace(w, pml=pml)
    n = (nx, ny, nz)
    pulse = pi.GaussianPulse(np.array(n) * dx * np.array([0.4, 0.55, 0.6]), 2.5 * dx, [3e5, -2e5, 1e5])
    Efull = pi.sample_field(pulse, "E", n, dx)
    return w, [Efull[c][:nx, :ny, :nz] for c in range(3)]


def _run(w, E0, steps, sweep, **kw):
    sim = native.from_workload(w, with_bunch=False, init_E=E0, series_len=steps, field_sweep=sweep, **kw)
    sim.step(steps)
    F, ser = sim.probe(series=True)
    out = {"E": sim.fields(native.FIELD_E), "H": sim.fields(native.FIELD_H),
           "J": sim.fields(native.FIELD_JPOL), "F": F, "series": ser, "hcur": sim.stats()["hcur"]}
    sim.close()
    return out


def _assert_same(a, b):
    assert a["hcur"] == b["hcur"]
    for k in ("E", "H", "J", "F", "series"):
        assert np.array_equal(a[k], b[k]), (k, float(np.max(np.abs(a[k] - b[k]))))


CASES = [
    # x extent: partial wavefront, several wavefronts, exact multiple of 64
    (37, 19, 27, (native.BC_CPML, native.BC_PERIODIC, native.BC_PEC), 5, None),
    (70, 9, 33, (native.BC_PERIODIC, native.BC_CPML, native.BC_CPML), 3, None),
    (128, 6, 17, (native.BC_CPML,) * 3, 2, None),
    (37, 19, 27, (native.BC_PERIODIC,) * 3, 0, None),
    (130, 11, 21, (native.BC_PEC,) * 3, 0, None),
    (37, 19, 27, (native.BC_CPML,) * 3, 6, KAPPA_ALPHA),
    (65, 5, 40, (native.BC_CPML, native.BC_PERIODIC, native.BC_CPML), 5, KAPPA_ALPHA),
]


@pytest.mark.parametrize("nx,ny,nz,bc,npml,pml", CASES)
@pytest.mark.parametrize("steps", [7, 40])
def test_sweep_is_bitwise_equal_to_separate_launches(nx, ny, nz, bc, npml, pml, steps):
    w, E0 = _case(nx, ny, nz, bc, npml, pml=pml)
    a = _run(w, E0, steps, 1)
    b = _run(w, E0, steps, 0)
    _assert_same(a, b)
    assert np.abs(a["J"]).max() > 0  # the film's Drude current took part


def test_sweep_on_the_widest_grid_it_takes():
    """1024 cells along x (16 wavefronts per workgroup), periodic x."""
    w, E0 = _case(1024, 6, 20, (native.BC_PERIODIC, native.BC_CPML, native.BC_PEC), 2)
    _assert_same(_run(w, E0, 9, 1), _run(w, E0, 9, 0))


def test_calls_of_every_length_chain_to_the_same_state():
    """One call of 23 steps, and calls of 1, 2, 3, 4, 5 and 8 steps (the short
    ones without sweeps), end in the same bits as the separate launches."""
    w, E0 = _case(70, 9, 33, (native.BC_PERIODIC, native.BC_CPML, native.BC_CPML), 3)
    ref = _run(w, E0, 23, 0)
    sim = native.from_workload(w, with_bunch=False, init_E=E0, series_len=23, field_sweep=1)
    for n in (1, 2, 3, 4, 5, 8):
        sim.step(n)
    F, ser = sim.probe(series=True)
    got = {"E": sim.fields(native.FIELD_E), "H": sim.fields(native.FIELD_H), "J": sim.fields(native.FIELD_JPOL),
           "F": F, "series": ser, "hcur": sim.stats()["hcur"]}
    sim.close()
    _assert_same(got, ref)


def test_caller_buffers_hold_the_state_after_a_call():
    """With E and H in caller (torch) memory the sweep alternates E with a
    second block inside a call and ends every call back in the caller's."""
    import torch
    w, E0 = _case(37, 19, 27, (native.BC_CPML, native.BC_PERIODIC, native.BC_PEC), 5)
    sim = native.from_workload(w, with_bunch=False, init_E=E0, device_fields=True, field_sweep=1)
    sim.step(11)
    torch.cuda.synchronize()
    dev = sim.device_E().cpu().numpy()  # (3, nz, ny, nx)
    host = sim.fields(native.FIELD_E)    # (3, nx, ny, nz)
    assert np.array_equal(np.transpose(dev, (0, 3, 2, 1)).astype(np.float64), host)
    ref = _run(w, E0, 11, 0)
    assert np.array_equal(host, ref["E"])
    sim.close()


@pytest.mark.parametrize("sort_every", [1, 3, 20])
def test_sweep_with_a_bunch_matches_separate_launches(sort_every):
    """Bunch over a slab (the push reads the sweep's time-centred H, the sweep
    reads the push's current, re-sorts inside the chain): within FP32 atomic
    reordering of the separate launches."""
    w = dataclasses.replace(pi.slab_tiny(), sort_every=sort_every)
    runs = []
    for sweep in (1, 0):
        sim = native.from_workload(w, field_sweep=sweep)
        sim.step(60)
        runs.append((sim.fields(native.FIELD_E), sim.fields(native.FIELD_H), sim.particles(), sim.probe()))
        sim.close()
    (Ea, Ha, Pa, Fa), (Eb, Hb, Pb, Fb) = runs
    rel = lambda x, y: np.linalg.norm(x - y) / np.linalg.norm(y)
    assert rel(Ea, Eb) <= 1e-5 and rel(Ha, Hb) <= 1e-5 and rel(Fa, Fb) <= 1e-5
    live = np.isfinite(Pb[0])
    assert np.array_equal(np.isfinite(Pa[0]), live)
    for c in range(6):  # x, y, z, ux, uy, uz
        assert rel(Pa[c, live], Pb[c, live]) <= 1e-5, c


def test_sweep_with_a_bunch_matches_the_oracle():
    """The tiny bunch over the slab, 200 steps through the sweep, against the
    FP64 oracle at the particle parity tests' 1e-3."""
    from oracle import pic_oracle as po
    w = pi.slab_tiny()
    b = w.bunch
    o = po.OracleSim(w.nx, w.ny, w.nz, w.dx, w.dt, bc=w.bc, npml=w.npml, pml=w.pml, wp_map=w.wp_map,
                     gamma_map=w.gamma_map)
    o.set_particles(b.x, b.y, b.z, b.ux, b.uy, b.uz, b.q, b.m, b.w)
    o.set_probes(w.probes, w.omega)
    o.step(200)
    sim = native.from_workload(w, field_sweep=1)
    sim.step(200)
    rel = lambda x, y: np.linalg.norm(x - y) / np.linalg.norm(y)
    n = (w.nx, w.ny, w.nz)
    E = sim.fields(native.FIELD_E)
    Eo = np.stack([o.E[c][: n[0], : n[1], : n[2]] for c in range(3)])
    assert rel(E, Eo) <= 1e-3
    assert rel(sim.probe(), o.probe()) <= 1e-3
    sim.close()
