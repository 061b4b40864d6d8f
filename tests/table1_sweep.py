"""Physics validation in the paper's geometry (Sec. III-IV, Table 1).

A 100 keV sheet bunch glides over a Drude film (wp = 1.2e16 rad/s,
gamma = 1.45e13 1/s) with the film normal along x and the bunch along z;
Ez is sampled on the film surface downstream.  The probe spectrum peaks
where the film's two surface-mode branches cross the electron line
w = beta c k: the "theoretical value" columns of Table 1, computed here by
tests/dispersion.py.

Two measurements.

1. The paper's probe, 1.5 um downstream, 40 fs record (`run_film`): the
   library's FP64 probe DFT (F(w) = sum_n dt Ez^n exp(-i w n dt), 1 THz grid),
   its two strongest local maxima.  Good for thin films only: the wake rings
   at the probe only while wave packets launched upstream still arrive, for
   tau = (L / v)(v / v_g - 1) after the bunch has passed (L the path from the
   bunch's start to the probe, v_g the branch's group velocity).  At
   L = 1.5 um that is 30-40 fs for the 70-80 nm branches, a spectral width of
   ~30 THz, above their 19-34 THz splitting, whatever the record length.

2. The Table 1 sweep (`run_sweep`, every thickness): a second probe 6 um
   downstream (tau x4), a 190 fs record that ends after the bunch has left
   through the far layer, one periodic cell across the sheet beam (the modes
   have no y wavenumber), CFS layers (see `sweep_workload`).  The lower branch
   is the strongest local maximum of the library's probe DFT near its crossing;
   the upper branch, longer-lived and much weaker in thick films, is read from
   the Hann-tapered ring-down after the passage (the taper removes the
   lower branch's -13 dB side lobes that hide it), and kept when it stands
   above the -30 dB floor that a single-branch (150 nm) film shows there.

Discretisation error.  Under the lower-corner edge rule a cell owns the E
edges at its low corner, so the film's bottom surface has its tangential-E
nodes in the metal and its top surface has them in vacuum.  The two surfaces'
single-interface modes are detuned, first order in the cell size h, by
-/+ delta(h) = -/+ a h, and the film's coupled branches sit at

    w(h) = wbar -/+ sqrt((a h)^2 + c^2),   c = half the continuum splitting

(two coupled surface modes: the top-surface mode, the one the bunch drives,
leans on the lower branch, so the upper one fades as delta grows past c).
a is the single-interface shift, measured on the 150 nm film (its peak
converges at first order to the single-interface crossing: a = f(h/2) -
f(h) per h/2); wbar and c are fitted by least squares to every branch peak
kept at every cell size, and wbar -/+ c are the extrapolated crossings.  The
tolerance propagates a peak-location uncertainty u through that fit (sum of
the absolute changes when each input, a's two peaks included, moves by u):
u = 1 / (4 T) for a peak of the untapered record of length T, 1 / (2 T_w) for
one of the tapered ring-down of length T_w (the Hann main lobe is twice as
wide).

Run as a script (GPU) for the whole table:  python tests/table1_sweep.py
[--fine] [d_nm ...]  (--fine adds 0.5 nm cells for 70, 80 and 150 nm).
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))
sys.path.insert(0, HERE)

import pic_inputs as pi  # noqa: E402
from dispersion import beta_of, film_modes_on_line  # noqa: E402

THICKNESSES = (20, 30, 40, 50, 60, 70, 80, 150)


def theory_thz(d_nm, kinetic_ev=100e3):
    lo, hi = film_modes_on_line(pi.PAPER_WP, d_nm * 1e-9, beta_of(kinetic_ev))
    return lo / (2 * np.pi * 1e12), hi / (2 * np.pi * 1e12)


def golden_pic():
    out = {}
    for line in open(os.path.join(HERE, "golden", "table1_pic.txt")):
        if line.startswith("#") or not line.strip():
            continue
        d, lo, hi = line.split()
        out[int(d)] = (float(lo), float(hi))
    return out


def two_peaks(f, a):
    """Frequencies of the two largest local maxima of a(f), ascending."""
    i = np.where((a[1:-1] > a[:-2]) & (a[1:-1] >= a[2:]))[0] + 1
    if i.size == 0:
        return np.nan, np.nan
    top = i[np.argsort(a[i])[::-1][:2]]
    fs = np.sort(f[top])
    if fs.size == 1:
        return fs[0], np.nan
    return fs[0], fs[1]


def dominant_peak(f, a):
    i = np.where((a[1:-1] > a[:-2]) & (a[1:-1] >= a[2:]))[0] + 1
    return f[i[np.argmax(a[i])]] if i.size else np.nan


def resolvable(d_nm, t_fs=40.0):
    lo, hi = theory_thz(d_nm)
    return np.isfinite(hi) and (hi - lo) > 2e3 / t_fs


def run_film(d_nm, dx=2e-9, t_fs=40.0):
    """Simulate one film on the GPU; returns the measured branches (THz)."""
    from paper_1505_04007_amd import native
    w = pi.paper_film(d_nm, dx=dx, t_fs=t_fs)
    sim = native.from_workload(w)
    sim.step(w.steps)
    F = sim.probe()[0]
    f = w.omega / (2 * np.pi * 1e12)
    a = np.abs(F)
    if resolvable(d_nm, t_fs):
        lo, hi = two_peaks(f, a)
    else:
        lo, hi = dominant_peak(f, a), np.nan
    st = sim.stats()
    sim.close()
    return {"d_nm": d_nm, "lower": lo, "upper": hi, "cells": w.cells, "steps": w.steps,
            "live": st["live"], "record_fs": w.steps * w.dt * 1e15}


def decay_rate(w, ez):
    """Temporal decay rate (1/s) of the probe's surface-mode ringing after the
    bunch has passed: the record band-passed to +-150 THz around its
    strongest peak, its Hilbert envelope, and a straight-line fit of the
    envelope's logarithm from 6 fs after the bunch's passage to 4 fs before
    the end of the record."""
    from scipy.signal import hilbert
    t = (np.arange(ez.size) + 1) * w.dt
    spec = np.fft.rfft(ez)
    f = np.fft.rfftfreq(ez.size, w.dt)
    band = (f > 0.5e15) & (f < 1.8e15)
    f0 = f[band][np.argmax(np.abs(spec[band]))]
    env = np.abs(hilbert(np.fft.irfft(spec * (np.abs(f - f0) < 0.15e15), n=ez.size)))
    t_pass = (w.meta["z_probe"] - w.meta["z0"]) / w.meta["v"]
    sel = (t > t_pass + 6e-15) & (t < t[-1] - 4e-15)
    return -np.polyfit(t[sel], np.log(env[sel]), 1)[0], f0


def run_decay(d_nm, gamma, dx=2e-9, t_fs=40.0):
    """The paper's setup with collision frequency `gamma`: decay rate (1/s)
    and frequency (Hz) of the probe Ez after the bunch has passed (Sec. IV)."""
    from paper_1505_04007_amd import native
    w = pi.paper_film(d_nm, dx=dx, t_fs=t_fs, gamma=gamma)
    sim = native.from_workload(w, series_len=w.steps)
    sim.step(w.steps)
    _, ser = sim.probe(series=True)
    sim.close()
    return decay_rate(w, np.asarray(ser, dtype=np.float64).reshape(-1))


# ---------------------------------------------------------------------------
# Table 1 sweep: long-path probe, two cell sizes, two-surface extrapolation
# ---------------------------------------------------------------------------

SWEEP_PROBES_UM = (1.5, 6.0)  # the paper's probe, then the long-path one
SWEEP_RECORD_FS = 190.0
SWEEP_PAST_NM = 300.0
SWEEP_ALPHA = 5e5  # S/m
SWEEP_GRID_THZ = (800.0, 1600.0, 0.5)
LONG = 1  # index of the long-path probe
LOWER_BAND = (-60.0, 15.0)  # THz around the lower crossing
UPPER_BAND = (-15.0, 60.0)  # THz around the upper crossing
FLOOR_DB = -30.0  # single-branch floor of the tapered ring-down
RINGDOWN_MARGIN_FS = 5.0
SINGLE = 150  # the film whose two surfaces no longer couple


def sweep_workload(d_nm, dx):
    """The paper's film with the sweep's probes and record.  The layers carry
    a CFS shift alpha_max = 5e5 S/m: with alpha = 0, a record of this length
    grows without bound where the Drude film meets the CPML (the film running
    through the layer, or its end faces against it): the known instability of
    classical PMLs on plasmonic guides that carry backward modes (Becache,
    Joly & Vinoles, Math. Comp. 2018).  The shift gives up most of the
    layer's absorption of propagating waves at these frequencies, which this
    problem, all evanescent fields, does not need."""
    return pi.paper_film(d_nm, dx=dx, t_fs=SWEEP_RECORD_FS, past_probe_nm=SWEEP_PAST_NM,
                         probe_um=SWEEP_PROBES_UM, ny=1, pml_alpha=SWEEP_ALPHA, f_thz=SWEEP_GRID_THZ)


def run_sweep(d_nm, dx):
    """One sweep run on the GPU: the library's probe spectra and series."""
    from paper_1505_04007_amd import native
    w = sweep_workload(d_nm, dx)
    sim = native.from_workload(w, series_len=w.steps)
    sim.step(w.steps)
    F, ser = sim.probe(series=True)
    st = sim.stats()
    sim.close()
    return {"w": w, "F": F, "series": np.asarray(ser, np.float64).reshape(w.steps, -1),
            "live": st["live"], "d_nm": d_nm, "dx": dx}


def local_max(f, a, lo, hi):
    """Strongest local maximum of a(f) with lo <= f <= hi, refined by a parabola
    through log a at it and its neighbours; (f, level in dB re max a).
    (nan, -inf) when there is none."""
    i = np.where((a[1:-1] > a[:-2]) & (a[1:-1] >= a[2:]))[0] + 1
    i = i[(f[i] >= lo) & (f[i] <= hi)]
    if i.size == 0:
        return np.nan, -np.inf
    j = i[np.argmax(a[i])]
    y0, y1, y2 = np.log(a[j - 1:j + 2])
    p = 0.5 * (y0 - y2) / (y0 - 2 * y1 + y2)
    return float(f[j] + p * (f[j + 1] - f[j])), float(20 * np.log10(a[j] / a.max()))


def ringdown_spectrum(r, probe=LONG, df_thz=0.1):
    """|F| of the probe's Ez after the bunch has passed it (plus a margin),
    Hann-tapered, zero-padded to a df_thz grid; (f THz, |F|, T_w s)."""
    w = r["w"]
    dt = w.dt
    t = (np.arange(r["series"].shape[0]) + 1) * dt
    t_pass = (w.meta["z_probes"][probe] - w.meta["z0"]) / w.meta["v"]
    x = r["series"][t > t_pass + RINGDOWN_MARGIN_FS * 1e-15, probe]
    x = x * np.hanning(x.size)
    n = int(round(1.0 / (df_thz * 1e12 * dt)))
    F = np.fft.rfft(x, n=n)
    f = np.fft.rfftfreq(n, dt) / 1e12
    keep = (f >= SWEEP_GRID_THZ[0]) & (f <= SWEEP_GRID_THZ[1])
    return f[keep], np.abs(F[keep]), x.size * dt


def branch_peaks(r, probe=LONG):
    """Measured branches of one run: {"lower": (f, dB, u), "upper": (f, dB, u)
    or None}, u the location uncertainty (THz) of each."""
    w = r["w"]
    lo, hi = theory_thz(r["d_nm"])
    f = w.omega / (2 * np.pi * 1e12)
    T = w.steps * w.dt
    flo, dblo = local_max(f, np.abs(r["F"][probe]), lo + LOWER_BAND[0], lo + LOWER_BAND[1])
    out = {"lower": (flo, dblo, 1e-12 / (4 * T)), "upper": None}
    if np.isfinite(hi) and hi - lo > 5.0:
        fh, ah, Tw = ringdown_spectrum(r, probe)
        # outside the lower branch's tapered main lobe (half width 2 / T_w)
        start = max(hi + UPPER_BAND[0], flo + 2e-12 / Tw)
        fu, dbu = local_max(fh, ah, start, hi + UPPER_BAND[1])
        if dbu >= FLOOR_DB:
            out["upper"] = (fu, dbu, 1e-12 / (2 * Tw))
    return out


def single_interface_shift(peaks_by_h):
    """From the 150 nm film's peak at two or more cell sizes h (nm):
    f(h) = ws - a h fitted; returns (ws, a)."""
    hs = np.array(sorted(peaks_by_h))
    fs = np.array([peaks_by_h[h] for h in hs])
    A = np.stack([np.ones_like(hs), -hs], axis=1)
    ws, a = np.linalg.lstsq(A, fs, rcond=None)[0]
    return float(ws), float(a)


def fit_crossings(obs, a):
    """obs: [(h nm, -1 lower / +1 upper, f THz)]; fits wbar, c of
    w = wbar + sign sqrt((a h)^2 + c^2); returns (lower, upper, residuals)."""
    from scipy.optimize import least_squares

    def res(x):
        return np.array([x[0] + s * np.sqrt((a * h) ** 2 + x[1] ** 2) - y for h, s, y in obs])

    ys = [y for _, _, y in obs]
    x0 = [np.mean(ys) if any(s > 0 for _, s, _ in obs) else max(ys) + 30.0, 30.0]
    fit = least_squares(res, x0, bounds=([0.0, 0.0], [1e4, 2e3]), xtol=1e-12, ftol=1e-12)
    wb, c = fit.x
    return float(wb - c), float(wb + c), res(fit.x)


def crossings_with_tolerance(meas, single):
    """meas: {h: branch_peaks(...)} of one film; single: {h: branch_peaks(...)}
    of the 150 nm film.  Returns the extrapolated (lower, upper), their
    tolerances, the fit residuals, the observations used and their u."""
    obs, us = [], []
    for h in sorted(meas):
        m = meas[h]
        obs.append([h, -1, m["lower"][0]])
        us.append(m["lower"][2])
        if m["upper"] is not None:
            obs.append([h, 1, m["upper"][0]])
            us.append(m["upper"][2])
    sp = {h: single[h]["lower"][0] for h in single}
    su = {h: single[h]["lower"][2] for h in single}

    def solve(o, s):
        return np.array(fit_crossings(o, single_interface_shift(s)[1])[:2])

    base = solve(obs, sp)
    tol = np.zeros(2)
    for k, u in enumerate(us):
        o = [list(x) for x in obs]
        o[k][2] += u
        tol += np.abs(solve(o, sp) - base)
    for h in sp:
        s = dict(sp)
        s[h] += su[h]
        tol += np.abs(solve(obs, s) - base)
    _, _, resid = fit_crossings(obs, single_interface_shift(sp)[1])
    return base, tol, resid, obs, np.array(us)


def single_interface_with_tolerance(single):
    """The 150 nm film: the first-order extrapolation ws of its peak and the
    tolerance (each peak moved by its u)."""
    sp = {h: single[h]["lower"][0] for h in single}
    ws, _ = single_interface_shift(sp)
    tol = 0.0
    for h in sp:
        s = dict(sp)
        s[h] += single[h]["lower"][2]
        tol += abs(single_interface_shift(s)[0] - ws)
    return ws, tol


def _run_logged(d_nm, h):
    print(f"  run: {d_nm} nm film, {h:g} nm cells", flush=True)
    return run_sweep(d_nm, h * 1e-9)


def main(argv):
    args = [a for a in argv[1:] if not a.startswith("--")]
    fine = "--fine" in argv
    thick = [int(a) for a in args] or list(THICKNESSES)
    gp = golden_pic()
    hs = {d: ([2.0, 1.0, 0.5] if fine and d in (70, 80, SINGLE) else [2.0, 1.0]) for d in set(thick) | {SINGLE}}
    single = {h: branch_peaks(_run_logged(SINGLE, h)) for h in hs[SINGLE]}
    ws, wtol = single_interface_with_tolerance(single)
    print(f"single interface ({SINGLE} nm film): peaks " +
          ", ".join(f"{h:g} nm {single[h]['lower'][0]:.1f}" for h in hs[SINGLE]) +
          f"; shift a = {single_interface_shift({h: single[h]['lower'][0] for h in single})[1]:.2f} THz/nm")
    print("frequencies in THz; long-path probe (6 um) unless marked")
    print(f"{'d_nm':>5} | {'theory':>15} | {'extrapolated':>15} | {'tolerance':>11} | {'paper PIC':>15} | "
          f"per cell size: lower / upper (dB)  | paper's probe (1.5 um), finest cells")
    for d in thick:
        th = theory_thz(d)
        p = gp.get(d, (np.nan, np.nan))
        if d == SINGLE:
            print(f"{d:5d} | {th[0]:7.1f} {'':7s} | {ws:7.1f} {'':7s} | {wtol:5.1f} {'':5s} | {p[0]:7.1f} {'':7s} |")
            continue
        runs = {h: _run_logged(d, h) for h in hs[d]}
        meas = {h: branch_peaks(r) for h, r in runs.items()}
        (elo, ehi), tol, resid, _, _ = crossings_with_tolerance(meas, single)
        cols = "  ".join(f"{h:g}: {m['lower'][0]:.1f} / " +
                         (f"{m['upper'][0]:.1f} ({m['upper'][1]:.0f})" if m["upper"] else "-")
                         for h, m in meas.items())
        paper_probe = branch_peaks(runs[min(hs[d])], probe=0)
        pp = f"{paper_probe['lower'][0]:.1f} / " + (f"{paper_probe['upper'][0]:.1f}" if paper_probe["upper"] else "-")
        print(f"{d:5d} | {th[0]:7.1f} {th[1]:7.1f} | {elo:7.1f} {ehi:7.1f} | {tol[0]:5.1f} {tol[1]:5.1f} | "
              f"{p[0]:7.1f} {p[1]:7.1f} | {cols} | {pp}   (fit residual <= {np.abs(resid).max():.2f})",
              flush=True)


if __name__ == "__main__":
    main(sys.argv)
