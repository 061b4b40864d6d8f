"""Field-kernel tile autotuner (pic_tune, pic_batch_tune).

Every tile shape runs the same per-cell arithmetic, so fields-only results
are bitwise identical whichever shape is chosen; the tuner times shapes from
a saved state and restores it, so tuning leaves the simulation as it was.
"""
import numpy as np
import pytest

import pic_inputs as pi
from paper_1505_04007_amd import native

pytestmark = pytest.mark.gpu

NSHAPES = 16


def _ragged(bc, npml):
    nx, ny, nz, dx = 37, 19, 27, 4e-9
    wpm, gm = pi.film_maps(nx, ny, nz, 9, 14)
    probes = np.array([[20 * dx, 9 * dx, 15.2 * dx]])
    w = pi.Workload("ragged", nx, ny, nz, dx, pi.courant_dt(dx), bc, npml, wpm, gm, None, probes,
                    pi.spectrum_omegas(nfreq=8), 60)
    pulse = pi.GaussianPulse(np.array((nx, ny, nz)) * dx * np.array([0.4, 0.5, 0.6]), 2.5 * dx,
                             [3e5, -2e5, 1e5])
    E = pi.sample_field(pulse, "E", (nx, ny, nz), dx)
    return w, [e[:nx, :ny, :nz] for e in E]


def _fields(s):
    return [s.fields(f) for f in (native.FIELD_E, native.FIELD_H, native.FIELD_JPOL)]


@pytest.mark.parametrize("bc,npml", [((native.BC_CPML, native.BC_PERIODIC, native.BC_CPML), 4),
                                     ((native.BC_PERIODIC,) * 3, 0)])
def test_every_tile_shape_gives_identical_fields(bc, npml):
    w, E = _ragged(bc, npml)
    ref = native.from_workload(w, init_E=E)
    ref.step(40)
    want = _fields(ref)
    for shape in range(NSHAPES):
        s = native.from_workload(w, init_E=E)
        r = s.tune(force=shape)
        assert r["tile"] == shape
        s.step(40)
        for a, b in zip(_fields(s), want):
            assert np.array_equal(a, b), shape
        assert np.array_equal(s.probe(), ref.probe())


def test_timed_tuning_leaves_the_state_unchanged():
    w, E = _ragged((native.BC_CPML,) * 3, 4)
    a = native.from_workload(w, init_E=E)
    b = native.from_workload(w, init_E=E)
    a.step(11)
    b.step(11)
    before = _fields(a)
    r = a.tune(reps=5)
    assert 0 <= r["tile"] < NSHAPES and len(r["ms"]) == NSHAPES and min(r["ms"]) > 0
    for x, y in zip(_fields(a), before):
        assert np.array_equal(x, y)
    a.step(29)
    b.step(29)
    for x, y in zip(_fields(a), _fields(b)):
        assert np.array_equal(x, y)
    assert np.array_equal(a.probe(), b.probe())
    assert a.stats()["steps"] == 40


def test_tuning_with_a_bunch_keeps_results():
    w = pi.slab_tiny()
    a = native.from_workload(w)
    b = native.from_workload(w)
    a.step(30)
    b.step(30)
    a.tune(reps=3)
    a.step(30)
    b.step(30)
    Ea, Eb = a.fields(native.FIELD_E), b.fields(native.FIELD_E)
    assert np.linalg.norm(Ea - Eb) <= 1e-5 * np.linalg.norm(Eb)  # deposit atomics: order only
    assert a.stats()["pushes"] == b.stats()["pushes"]


def test_batch_tune_keeps_members_equal_to_plain_runs():
    specs = [((native.BC_CPML, native.BC_PERIODIC, native.BC_CPML), 4), ((native.BC_PERIODIC,) * 3, 0)]
    members = [_ragged(bc, npml) for bc, npml in specs]
    plain = [native.from_workload(w, init_E=E) for w, E in members]
    for s in plain:
        s.step(33)
    for use_graph in (True, False):
        sims = [native.from_workload(w, init_E=E) for w, E in members]
        b = native.Batch(sims, use_graph=use_graph)
        b.step(3)
        r = b.tune(reps=3)
        assert 0 <= r["tile"] < NSHAPES
        b.step(30)
        for s, p in zip(sims, plain):
            for x, y in zip(_fields(s), _fields(p)):
                assert np.array_equal(x, y)
        b.tune(force=11)
        b.close()


def test_tune_rejects_bad_arguments():
    w, E = _ragged((native.BC_PEC,) * 3, 0)
    s = native.from_workload(w, init_E=E)
    for reps, force in ((0, -1), (5, NSHAPES), (5, -2)):
        with pytest.raises(native.PicError) as ei:
            s.tune(reps=reps, force=force)
        assert ei.value.status == native.PIC_EINVAL


def test_sampled_timing_counts_the_sampled_steps_and_every_sort():
    """timing = 3 from step 0 over 30 steps with a sort every 5: the launches
    of steps 0, 3, ..., 27 (10 each) and all 6 sorts (pic_init's and those
    before steps 5, 10, ..., 25); timing = 1 every launch.
    Results are those of an untimed run."""
    import dataclasses
    w = dataclasses.replace(pi.slab_tiny(), sort_every=5)
    out = {}
    for t in (0, 1, 3):
        sim = native.from_workload(w, timing=t)
        sim.step(30)
        out[t] = (sim.timing(), sim.fields(native.FIELD_E))
        sim.close()
    per_step = ("h_update", "push_deposit", "e_update", "probe")
    for fam in per_step:
        assert out[1][0][fam][1] == 30 and out[3][0][fam][1] == 10, fam
        assert out[3][0][fam][0] > 0, fam
        assert out[0][0][fam] == (0.0, 0), fam
    assert out[1][0]["sort"][1] == 6 and out[3][0]["sort"][1] == 6
    rel = np.linalg.norm(out[3][1] - out[0][1]) / np.linalg.norm(out[0][1])
    assert rel <= 1e-5  # the FP32 deposit's atomics order aside, the same run
