"""pic_grad_noalloc (every device buffer carved from the library's static
scratch, no device allocation) against pic_grad on identical contexts.

Both run the same kernels in the same order: the store-all form of the
reverse pass, a bunch with the fixed-point deposit (deposit_mode 2, exact
integer sums, so the forward run is bitwise reproducible) and FP64 gradient
accumulation per cell without atomics.  The two calls must therefore agree
bit for bit, in L, in both gradient maps and in the state the simulation is
left in.  Two calls in a row on one device, the second on a smaller grid
with fewer steps, show that what the first call left in the shared scratch
does not leak into the second.
"""
import numpy as np
import pytest

import pic_inputs as pi
from paper_1505_04007_amd import native

pytestmark = pytest.mark.gpu


def _workload(nx, ny, nz, seed):
    dx = 2e-9
    k0, k1 = nz // 3, nz // 3 + 4
    wp, g = pi.film_maps(nx, ny, nz, k0, k1)
    rng = np.random.default_rng(pi.SEED0 + 930 + seed)
    metal = wp > 0
    wp[metal] *= 1.0 + 0.05 * rng.standard_normal(int(metal.sum()))
    g[metal] *= 1.0 + 0.05 * rng.standard_normal(int(metal.sum()))
    bunch = pi.gaussian_bunch(rng, 300, (7 * dx, ny / 2 * dx, (k1 + 3) * dx),
                              (2 * dx, 1.5 * dx, 1.5 * dx), 50e3, charge=1e-16)
    probes = np.array([[0.5 * nx * dx, ny / 2 * dx, (k1 + 1.4) * dx],
                       [0.7 * nx * dx, ny / 2 * dx, (k1 + 0.6) * dx]])
    bc = (native.BC_CPML, native.BC_PERIODIC, native.BC_CPML)
    return pi.Workload(f"noalloc_{nx}x{ny}x{nz}", nx, ny, nz, dx, pi.courant_dt(dx), bc, 3, wp, g,
                       bunch, probes, np.array([0.68 * pi.AG_WP]), 0, sort_every=10)


@pytest.mark.parametrize("shape_steps", [((40, 12, 28), 120), ((24, 12, 20), 70)])
def test_noalloc_equals_pic_grad(shape_steps):
    (nx, ny, nz), N = shape_steps
    w = _workload(nx, ny, nz, seed=nx)
    print(f"noalloc vs pic_grad: {w.name}, {N} steps, deposit_mode 2", flush=True)
    a = native.from_workload(w, deposit_mode=2)
    b = native.from_workload(w, deposit_mode=2)
    w0 = w.omega[0]
    La, gwa, gga = a.grad(w0, N, ckpt_every=0)
    Lb, gwb, ggb = b.grad_noalloc(w0, N)
    print(f"  L = {La:.6e} / {Lb:.6e}, max|dL/dwp| = {np.abs(gwa).max():.3e}", flush=True)
    assert La > 0 and np.abs(gwa).max() > 0 and np.abs(gga).max() > 0
    assert Lb == La
    np.testing.assert_array_equal(gwb, gwa)
    np.testing.assert_array_equal(ggb, gga)
    assert b.stats()["steps"] == a.stats()["steps"] == N
    for f in (native.FIELD_E, native.FIELD_H, native.FIELD_JPOL):
        np.testing.assert_array_equal(b.fields(f), a.fields(f))
    np.testing.assert_array_equal(b.particles(), a.particles())
    np.testing.assert_array_equal(b.probe(), a.probe())


def test_noalloc_refuses_what_does_not_fit():
    """A run whose snapshots exceed the static scratch is refused before any
    step is taken, with the sizes in the message."""
    w = _workload(64, 64, 40, seed=3)
    s = native.from_workload(w, with_bunch=False)
    with pytest.raises(native.PicError) as err:
        s.grad_noalloc(w.omega[0], 4000)
    assert err.value.status == native.PIC_EINVAL
    assert "static scratch" in str(err.value)
    assert s.stats()["steps"] == 0
    # the context is still usable, and a run that fits goes through
    L, gw, gg = s.grad_noalloc(w.omega[0], 5)
    assert s.stats()["steps"] == 5 and np.isfinite(L)
