"""Surface-plasmon frequencies in the paper's geometry on the GPU (Table 1).

The paper's probe (1.5 um downstream, 40 fs): thin films, where the two
branches lie far apart, show both peaks at the dispersion-relation crossings
within the record's resolution 1/T = 25 THz.

Every thickness of Table 1 (the sweep of tests/table1_sweep.py: a long-path
probe 6 um downstream, 190 fs, 2 nm and 1 nm cells): the lower-corner edge
rule detunes the film's two surfaces by -/+ a h, the single-interface shift
that the 150 nm film measures, and the branches follow
wbar -/+ sqrt((a h)^2 + c^2).  That model must fit every kept peak to within
the peak's own location uncertainty, and its extrapolation wbar -/+ c must
meet both crossings to within the uncertainty propagated through the fit.
The paper's own PIC column is printed beside each row; it is not a pin (the
paper's bunch and domain are not fully specified).  The decay of the probe
field with the collision frequency (Sec. IV) is checked against the
quasi-static surface-mode root of the Drude metal.
"""
import numpy as np
import pytest

import pic_inputs as pi
import table1_sweep as ts

pytestmark = pytest.mark.gpu

H_NM = (2.0, 1.0)


@pytest.mark.parametrize("d_nm", [20, 40])
def test_thin_film_branches_match_dispersion_crossings(d_nm):
    r = ts.run_film(d_nm, dx=2e-9, t_fs=40.0)
    lo, hi = ts.theory_thz(d_nm)
    paper = ts.golden_pic()[d_nm]
    print(f"d = {d_nm} nm: measured {r['lower']:.0f} / {r['upper']:.0f} THz, theory {lo:.0f} / {hi:.0f}, "
          f"paper PIC {paper[0]:.0f} / {paper[1]:.0f}", flush=True)
    assert r["live"] == 4000  # the bunch stays in the box, on a straight line
    res = 1e3 / r["record_fs"]  # THz
    assert abs(r["lower"] - lo) <= res
    assert abs(r["upper"] - hi) <= res


def sweep_peaks(d_nm):
    out = {}
    for h in H_NM:
        print(f"sweep run: d = {d_nm} nm, {h:g} nm cells", flush=True)
        r = ts.run_sweep(d_nm, h * 1e-9)
        assert r["live"] == 0  # the whole bunch has left through the far layer
        out[h] = ts.branch_peaks(r)
    return out


@pytest.fixture(scope="module")
def single_interface():
    return sweep_peaks(ts.SINGLE)


def test_single_interface_converges_first_order_to_the_crossing(single_interface):
    th = ts.theory_thz(ts.SINGLE)[0]
    f2, f1 = (single_interface[h]["lower"][0] for h in H_NM)
    ws, tol = ts.single_interface_with_tolerance(single_interface)
    print(f"d = {ts.SINGLE} nm: 2 nm {f2:.1f}, 1 nm {f1:.1f}, extrapolated {ws:.1f} +- {tol:.1f}, "
          f"theory {th:.1f}, paper PIC {ts.golden_pic()[ts.SINGLE][0]:.0f} THz", flush=True)
    assert f2 < f1 < th  # approached from below
    assert abs(th - f1) < 0.6 * abs(th - f2)  # the error halves with the cell
    assert abs(ws - th) <= tol


@pytest.mark.parametrize("d_nm", [20, 30, 40, 50, 60, 70, 80])
def test_film_branches_extrapolate_to_the_dispersion_crossings(d_nm, single_interface):
    meas = sweep_peaks(d_nm)
    (lo, hi), tol, resid, obs, us = ts.crossings_with_tolerance(meas, single_interface)
    th = ts.theory_thz(d_nm)
    paper = ts.golden_pic()[d_nm]
    kept = ", ".join(f"{h:g} nm {'upper' if s > 0 else 'lower'} {f:.1f}" for h, s, f in obs)
    print(f"d = {d_nm} nm: extrapolated {lo:.1f} +- {tol[0]:.1f} / {hi:.1f} +- {tol[1]:.1f}, "
          f"theory {th[0]:.1f} / {th[1]:.1f}, paper PIC {paper[0]:.0f} / {paper[1]:.0f} THz; "
          f"peaks {kept}; residuals {np.round(resid, 2).tolist()}", flush=True)
    assert len(obs) >= 3 or d_nm >= 70  # both branches seen wherever the upper is not washed out
    assert np.all(np.abs(resid) <= us)
    assert abs(lo - th[0]) <= tol[0]
    assert abs(hi - th[1]) <= tol[1]


def test_decay_rate_grows_with_the_collision_frequency():
    """Sec. IV: the probe field decays faster for a larger collision frequency.
    Thick film (one interface): the decay rate rises linearly in gamma with the
    slope 1/2 that the quasi-static surface-mode root of the Drude metal gives
    (eps(w) = -1 with Eq. 1: w = wp/sqrt(2) - i gamma/2); thin film: it rises
    too, on top of the two branches' beating."""
    g0 = pi.PAPER_GAMMA
    facs = np.array([1.0, 2.0, 4.0, 8.0])
    thick = np.array([ts.run_decay(150, g0 * f)[0] for f in facs])
    slope = np.polyfit(g0 * facs, thick, 1)[0]
    print("d = 150 nm: decay rates " + ", ".join(f"{r:.3e}" for r in thick) + f" 1/s, slope {slope:.3f}",
          flush=True)
    assert np.all(np.diff(thick) > 0)
    assert 0.4 < slope < 0.6
    thin = [ts.run_decay(50, g0 * f)[0] for f in (1.0, 4.0)]
    print(f"d = 50 nm: decay rates {thin[0]:.3e}, {thin[1]:.3e} 1/s", flush=True)
    assert thin[1] > thin[0]
