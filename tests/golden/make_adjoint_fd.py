"""Central differences of the probe spectral power on the adjoint workload,
written by the FP64 oracle alone (test infrastructure; it reads nothing else).

Workload `pic_inputs.film_adjoint()`: 128 x 64 x 64 cells of 2 nm, 8-cell
CPML, a 20 nm silver film whose per-cell wp and gamma carry +-5 % seeded
noise, a 1e5-particle 50 keV bunch, probes 2 nm above the film, 2000 steps,
objective L = sum_p |F_p(0.68 wp)|^2 (the differentiable form of the step,
with the bunch current held at what the forward run deposited).

1. One run with the bunch records the bunch current of every step on a box
   that holds every deposit (the oracle reports anything outside it; the
   script stops if there is any).
2. With that current prescribed, one run of 2000 steps per perturbed map:
   wp and gamma of 32 seeded metal cells moved by +-h of their value
   (h = 1e-4 for wp, 1e-2 for gamma, whose effect per cell is ~1e4 times
   weaker), and (L+ - L-)/(2 h v) per cell and map.
The unperturbed L of the prescribed run must equal the particle run's L.

Output: adjoint_fd_film20nm_128x64x64.json beside this script.  About an hour
on 8 host threads (128 runs of 2000 steps of 0.52M cells).
Run: python tests/golden/make_adjoint_fd.py
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import pic_inputs as pi  # noqa: E402
from oracle import pic_oracle as po  # noqa: E402

OUT = os.path.join(HERE, "adjoint_fd_film20nm_128x64x64.json")
NCELLS = 32
H_WP, H_GAMMA = 1e-4, 1e-2
MARGIN = 4  # cells around the initial bunch across the beam


def make(w, wp, g):
    o = po.OracleSim(w.nx, w.ny, w.nz, w.dx, w.dt, bc=w.bc, npml=w.npml, pml=w.pml, wp_map=wp,
                     gamma_map=g)
    o.set_probes(w.probes, w.omega)
    return o


def main():
    w = pi.film_adjoint()
    N = w.steps
    w0 = float(w.meta["omega0"])
    b = w.bunch
    lo = [0, int(np.floor(b.y.min() / w.dx)) - MARGIN, int(np.floor(b.z.min() / w.dx)) - MARGIN]
    # x: the whole axis, nodes 0..nx (the bunch leaves through the +x wall)
    hi = [w.nx + 1, int(np.floor(b.y.max() / w.dx)) + MARGIN + 1, int(np.floor(b.z.max() / w.dx)) + MARGIN + 1]
    ext = [h - l for l, h in zip(lo, hi)]
    t0 = time.time()
    o = make(w, w.wp_map, w.gamma_map)
    o.set_particles(b.x, b.y, b.z, b.ux, b.uy, b.uz, b.q, b.m, b.w)
    hist, outside = o.run_record_jb_box(N, lo, ext)
    L_part = float(np.sum(np.abs(o.probe()) ** 2))
    print(f"recorded {N} steps of bunch current on box lo {lo} ext {ext} in {time.time() - t0:.0f} s; "
          f"outside {outside:.3e}; L = {L_part:.10e}", flush=True)
    if outside != 0.0:
        raise SystemExit("the box misses part of the deposits: widen MARGIN")
    del o

    def L_of(wp, g):
        s = make(w, wp, g)
        s.prescribe_jb_box(lo, ext, hist)
        s.step(N)
        return float(np.sum(np.abs(s.probe()) ** 2))

    L0 = L_of(w.wp_map, w.gamma_map)
    print(f"prescribed-current L = {L0:.10e} (particle run {L_part:.10e})", flush=True)
    assert abs(L0 - L_part) <= 1e-12 * L_part

    rng = np.random.default_rng(pi.SEED0 + 3000)
    metal = np.argwhere(w.wp_map > 0)
    cells = metal[np.sort(rng.choice(len(metal), NCELLS, replace=False))]
    g_wp, g_gamma = [], []
    for q, (i, j, k) in enumerate(cells):
        row = []
        for base, h, other_first in ((w.wp_map, H_WP, True), (w.gamma_map, H_GAMMA, False)):
            d = h * base[i, j, k]
            up, dn = base.copy(), base.copy()
            up[i, j, k] += d
            dn[i, j, k] -= d
            if other_first:
                Lp, Lm = L_of(up, w.gamma_map), L_of(dn, w.gamma_map)
            else:
                Lp, Lm = L_of(w.wp_map, up), L_of(w.wp_map, dn)
            row.append((Lp - Lm) / (2 * d))
        g_wp.append(row[0])
        g_gamma.append(row[1])
        print(f"cell {q + 1}/{NCELLS} ({i},{j},{k}): dL/dwp {row[0]:.6e}  dL/dgamma {row[1]:.6e}  "
              f"[{time.time() - t0:.0f} s]", flush=True)
    out = {
        "what": "FP64 oracle central differences of L = sum_p |F_p(omega0)|^2 on the adjoint workload",
        "workload": w.name,
        "generator": "tests/golden/make_adjoint_fd.py (oracle only)",
        "steps": N,
        "omega0": w0,
        "h_wp": H_WP,
        "h_gamma": H_GAMMA,
        "bunch_current_box": {"lo": lo, "ext": ext},
        "L": L0,
        "cells": cells.tolist(),
        "dL_dwp": g_wp,
        "dL_dgamma": g_gamma,
    }
    with open(OUT, "w") as f:
        json.dump(out, f, indent=1)
    print(f"wrote {OUT} in {time.time() - t0:.0f} s", flush=True)


if __name__ == "__main__":
    main()
