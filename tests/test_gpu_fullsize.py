"""Parity at the benchmark's full size, in its launch configuration.

The 512 x 256 x 256-cell grating workload (12-cell CPML, 40 nm film with
grooves, 1e7-particle bunch) with the tile the autotuner picks for it:
  * fields: a few steps of the whole grid against the oracle (which needs
    ~10 GB of host memory and ~1 s per step here), element by element;
  * particles: one step of the whole 1e7-particle bunch on both sides, every
    particle's push compared, and the deposited current edge by edge (E^1 =
    -J_b from fields at rest isolates the deposit at full bunch density).
"""
import numpy as np
import pytest

import pic_inputs as pi
from oracle import pic_oracle as po
from paper_1505_04007_amd import native

pytestmark = pytest.mark.gpu


def _rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def _pulse(w, center, width, amp):
    """Separable Gaussian E pulse on the full staggered lattice, zero on walls."""
    n = (w.nx, w.ny, w.nz)
    out = []
    for c in range(3):
        f = []
        for a in range(3):
            x = (np.arange(n[a]) + 0.5) * w.dx if a == c else np.arange(n[a] + 1) * w.dx
            g = np.exp(-(x - center[a]) ** 2 / (2 * width ** 2))
            if a != c:
                g[0] = 0.0
                g[-1] = 0.0  # tangential E on the PEC wall behind each CPML layer
            f.append(g)
        out.append(amp[c] * f[0][:, None, None] * f[1][None, :, None] * f[2][None, None, :])
    return out


def _oracle(w, E):
    o = po.OracleSim(w.nx, w.ny, w.nz, w.dx, w.dt, bc=w.bc, npml=w.npml, pml=w.pml,
                     wp_map=w.wp_map, gamma_map=w.gamma_map)
    for c in range(3):
        o.E[c][...] = E[c]
    return o


def _center(w):
    return np.array([w.nx * 0.55, w.ny * 0.5, w.nz * 0.5 + 6]) * w.dx


def test_full_grid_fields_match_oracle():
    w = pi.grating_large(nparticles=1)
    w.bunch = None
    E = _pulse(w, _center(w), 6 * w.dx, [2e6, -1e6, 3e6])
    g = native.from_workload(w, init_E=[e[: w.nx, : w.ny, : w.nz] for e in E])
    tile = g.tune(reps=5)
    print(f"tile {tile['fx']}x{tile['fy']} order {tile['order']}", flush=True)
    o = _oracle(w, E)
    del E
    steps = 4
    o.step(steps)
    g.step(steps)
    Eg = g.fields(native.FIELD_E)
    Eo = np.stack([o.E[c][: w.nx, : w.ny, : w.nz] for c in range(3)])
    eE = _rel(Eg, Eo)
    del Eg, Eo
    Hg = g.fields(native.FIELD_H)
    Ho = np.stack([o.H[c][: w.nx, : w.ny, : w.nz] for c in range(3)])
    eH = _rel(Hg, Ho)
    print(f"full grid after {steps} steps: E rel {eE:.2e}, H rel {eH:.2e}", flush=True)
    assert eE <= 1e-5 and eH <= 1e-5


@pytest.mark.parametrize("pulse", [False, True], ids=["fields_at_rest", "strong_pulse"])
def test_full_bunch_first_step_matches_oracle(pulse):
    """Every one of the 1e7 particles pushed and deposited by both sides for one
    step, in the bench's launch configuration (tuned tile, wavefront-reduced
    FP32 deposit, bunch sorted at init).

    fields_at_rest: E = H = 0, so nothing acts on the bunch and the Drude
    current stays 0: E^1 is minus the deposited bunch current (V/m), and the
    deposit at the bench bunch's full density (~10^3 particles per cell, as
    many FP32 atomic contributions per edge) is compared edge by edge.
    strong_pulse: a 1e11 V/m pulse over the bunch; every particle's position
    and kick, and E^1 - E^0 edge by edge over the bunch box.  The whole grid's
    E^1 is held to the particle tolerance 1e-3 either way.
    """
    w = pi.grating_large()
    n = (w.nx, w.ny, w.nz)
    b = w.bunch
    if pulse:
        c = _center(w)
        c[0] = 200 * w.dx
        E = _pulse(w, c, 30 * w.dx, [1e11, 5e10, -8e10])
    else:
        E = [np.zeros((w.nx + (q != 0), w.ny + (q != 1), w.nz + (q != 2))) for q in range(3)]
    print(f"full bunch, one step, pulse={pulse}: {b.n} particles", flush=True)
    g = native.from_workload(w, init_E=[e[: w.nx, : w.ny, : w.nz] for e in E])
    g.tune(reps=5)
    g.step(1)
    P = g.particles()
    Eg = g.fields(native.FIELD_E)
    assert g.stats()["pushes"] == b.n
    g.close()
    o = _oracle(w, E)
    o.set_particles(b.x, b.y, b.z, b.ux, b.uy, b.uz, b.q, b.m, b.w)
    o.step(1)
    assert o.timing()["pushes"] == b.n
    # particles, all of them
    Po = np.stack(o.particles()[:6])
    u0 = np.stack([b.ux, b.uy, b.uz])
    umax = np.abs(u0).max()
    dpos = np.abs(P[:3] - Po[:3]).max() / w.dx
    du = np.abs(P[3:] - Po[3:]).max() / umax
    print(f"  all pushes: max |dx| {dpos:.2e} cells, max |du| {du:.2e} |u|", flush=True)
    assert dpos <= 1e-4 and du <= 1e-6
    if pulse:
        kick_o = Po[3:] - u0
        dk = np.abs((P[3:] - u0) - kick_o).max() / np.abs(kick_o).max()
        print(f"  kick max {np.abs(kick_o).max() / umax:.2e} |u|, error {dk:.2e} of it", flush=True)
        assert np.abs(kick_o).max() > 5e-5 * umax and dk <= 1e-2
    del P, Po, u0
    # E^1 - E^0 over the bunch box: cells the initial bunch spans, +-3
    lo = [max(int(np.floor(v.min() / w.dx)) - 3, 0) for v in (b.x, b.y, b.z)]
    hi = [min(int(np.floor(v.max() / w.dx)) + 4, m) for v, m in zip((b.x, b.y, b.z), n)]
    box = (slice(lo[0], hi[0]), slice(lo[1], hi[1]), slice(lo[2], hi[2]))
    Eo = np.stack([o.E[q][: w.nx, : w.ny, : w.nz] for q in range(3)])
    whole = _rel(Eg, Eo)
    D = np.stack([Eg[q][box] - E[q][: w.nx, : w.ny, : w.nz][box] for q in range(3)])
    Do = np.stack([Eo[q][box] - E[q][: w.nx, : w.ny, : w.nz][box] for q in range(3)])
    edge = np.abs(D - Do).max() / np.abs(Do).max()
    boxl2 = _rel(D, Do)
    print(f"  E^1 - E^0 over the bunch box {[h - l for l, h in zip(lo, hi)]}: max edge error "
          f"{edge:.2e} of the largest, rel-L2 {boxl2:.2e}; whole grid E rel-L2 {whole:.2e}", flush=True)
    assert np.abs(Do).max() > 0
    assert edge <= 2e-4 and boxl2 <= 1e-4
    assert whole <= 1e-3


def test_full_batched_sweep_matches_its_plain_runs():
    """The 16-instance sweep (films 5-80 nm, grids 128x64x64 to 192x96x96,
    2e5 particles each) as one batch with its captured graph: every member's
    fields, pushes and probe spectra equal its own plain run to the FP32
    deposit's rounding (the per-cell arithmetic is the plain kernels')."""
    ws = pi.batched_sweep()
    steps = 45
    plain = []
    for w in ws:
        s = native.from_workload(w)
        s.step(steps)
        plain.append((s.fields(native.FIELD_E), s.stats()["pushes"], s.probe()))
        s.close()
    sims = [native.from_workload(w) for w in ws]
    b = native.Batch(sims, use_graph=True)
    b.step(steps)
    worst = 0.0
    for s, (E, pushes, F) in zip(sims, plain):
        e = _rel(s.fields(native.FIELD_E), E)
        worst = max(worst, e)
        assert e <= 1e-5
        assert s.stats()["pushes"] == pushes
        assert np.abs(s.probe() - F).max() <= 1e-4 * np.abs(F).max()
    print(f"16 members after {steps} steps: worst E rel-L2 against the plain run {worst:.2e}", flush=True)
    b.close()


def test_full_adjoint_workload_properties():
    """The adjoint workload at its full size (128x64x64, 20 nm film with map
    noise, 1e5 particles, 2000 steps): L equals the probe power of the same
    forward run, the gradients vanish outside the metal and are finite, and
    the checkpointed reverse pass (interval 45) agrees with the store-all one."""
    w = pi.film_adjoint()
    w0 = w.meta["omega0"]
    N = w.steps
    a = native.from_workload(w)
    L, gw, gg = a.grad(w0, N)
    F = a.probe()[:, 0]
    assert abs(L - float(np.sum(np.abs(F) ** 2))) <= 1e-9 * L
    metal = w.wp_map > 0
    assert np.all(gw[~metal] == 0) and np.all(gg[~metal] == 0)
    assert np.all(np.isfinite(gw)) and np.abs(gw[metal]).max() > 0
    b = native.from_workload(w)
    L2, gw2, gg2 = b.grad(w0, N, ckpt_every=45)
    assert abs(L2 - L) <= 1e-4 * L
    assert np.linalg.norm(gw2 - gw) <= 1e-3 * np.linalg.norm(gw)
    assert np.linalg.norm(gg2 - gg) <= 1e-3 * np.linalg.norm(gg)
