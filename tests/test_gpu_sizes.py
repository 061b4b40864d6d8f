"""pic_query_sizes against what pic_init allocates (pic_stats.device_bytes).

The query sees only the grid, the particle count and the options; the Drude
state depends on the maps and is its per-cell figure times the cells of the
bounding box of wp > 0.  Both must give the context's allocation exactly.
"""
import numpy as np
import pytest

import pic_inputs as pi
from paper_1505_04007_amd import native

pytestmark = pytest.mark.gpu


def _box_cells(wp):
    m = wp > 0
    if not m.any():
        return 0
    idx = [np.nonzero(m.any(axis=tuple(b for b in range(3) if b != a)))[0] for a in range(3)]
    return int(np.prod([i.max() - i.min() + 1 for i in idx]))


def _ragged(with_bunch):
    nx, ny, nz, dx = 37, 19, 30, 4e-9
    wp, g = pi.film_maps(nx, ny, nz, 9, 14)
    bunch = None
    if with_bunch:
        rng = np.random.default_rng(pi.SEED0 + 950)
        bunch = pi.gaussian_bunch(rng, 777, (12 * dx, ny / 2 * dx, 18.5 * dx), (2 * dx, 2 * dx, 1.5 * dx),
                                  60e3, charge=1e-16)
    return pi.Workload("sizes_37x19x30", nx, ny, nz, dx, pi.courant_dt(dx),
                       (native.BC_CPML, native.BC_PERIODIC, native.BC_CPML), 4, wp, g, bunch,
                       np.array([[20 * dx, 9 * dx, 15.2 * dx], [5 * dx, 3 * dx, 20.9 * dx]]),
                       pi.spectrum_omegas(nfreq=8), 50, sort_every=5)


CASES = {
    "fields_only": (lambda: _ragged(False), {}),
    "bunch_series_diag": (lambda: _ragged(True), dict(series_len=40, diag=True)),
    "bunch_device_fields": (lambda: _ragged(True), dict(device_fields=True)),
    "bunch_fixed_point": (lambda: _ragged(True), dict(deposit_mode=2)),
    "pec_slab_tiny": (pi.slab_tiny, {}),
}


@pytest.mark.parametrize("case", list(CASES))
def test_query_matches_the_allocation(case):
    make, kw = CASES[case]
    w = make()
    q = native.workload_sizes(w, **kw)
    sim = native.from_workload(w, **kw)
    got = sim.stats()["device_bytes"]
    expect = q["device_bytes"] + _box_cells(w.wp_map) * q["bytes_per_metal_box_cell"]
    assert got == expect, (case, got, expect)
