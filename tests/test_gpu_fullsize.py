"""Parity at the benchmark's full size, in its launch configuration.

The 512 x 256 x 256-cell grating workload (12-cell CPML, 40 nm film with
grooves, 1e7-particle bunch) with the tile the autotuner picks for it:
  * fields: a few steps of the whole grid against the oracle (which needs
    ~10 GB of host memory and ~1 s per step here), element by element;
  * particles: after one step the push of every particle depends only on the
    initial fields, so a sample of the bunch pushed by the oracle must match
    the GPU's push of the whole bunch particle by particle.
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


def test_full_bunch_first_push_matches_oracle_sample():
    w = pi.grating_large()
    # a strong pulse (1e11 V/m) over the bunch: one step's kick must stand well
    # above the FP32 resolution of u (6e-8 |u|)
    c = _center(w)
    c[0] = 200 * w.dx
    E = _pulse(w, c, 30 * w.dx, [1e11, 5e10, -8e10])
    g = native.from_workload(w, init_E=[e[: w.nx, : w.ny, : w.nz] for e in E])
    g.tune(reps=5)
    g.step(1)
    P = g.particles()
    rng = np.random.default_rng(pi.SEED0 + 740)
    idx = np.sort(rng.choice(w.bunch.n, 20000, replace=False))
    sub = w.bunch.subset(idx)
    o = _oracle(w, E)
    del E
    o.set_particles(sub.x, sub.y, sub.z, sub.ux, sub.uy, sub.uz, sub.q, sub.m, sub.w)
    o.step(1)
    Po = np.stack(o.particles()[:6])
    assert g.stats()["pushes"] == w.bunch.n
    u0 = np.stack([sub.ux, sub.uy, sub.uz])
    umax = np.abs(u0).max()
    kick_o = Po[3:] - u0
    kick_g = P[3:, idx] - u0
    dpos = np.abs(P[:3, idx] - Po[:3]).max() / w.dx
    dk = np.abs(kick_g - kick_o).max() / np.abs(kick_o).max()
    print(f"sampled pushes: max |dx| {dpos:.2e} cells, kick max {np.abs(kick_o).max() / umax:.2e} |u|, "
          f"kick error {dk:.2e} of it", flush=True)
    assert np.abs(kick_o).max() > 5e-5 * umax  # the field does act on the sample
    assert dpos <= 1e-4                          # FP32 positions of ~300 cells
    assert dk <= 1e-2                            # FP32 storage of u: 6e-8 |u| against the kick
    assert np.abs(P[3:, idx] - Po[3:]).max() <= 1e-6 * umax
