"""Surface-plasmon dispersion theory used as an analytic pin (test tool).

A lossless Drude film (Eq. 1 with gamma = 0, eps_inf = 1) of thickness d in
vacuum carries two TM surface modes.  With the decay constants
kd = sqrt(k^2 - w^2/c^2) in vacuum and km = sqrt(k^2 - eps_m w^2/c^2) in the
metal, the textbook insulator/metal/insulator conditions read
    (eps_m kd + km) / (eps_m kd - km) = +exp(-km d)   (lower-frequency branch)
    (eps_m kd + km) / (eps_m kd - km) = -exp(-km d)   (upper-frequency branch)
An electron moving parallel to the film at speed beta c excites the modes
where they cross its line w = beta c k (Sec. IV, Fig. 2 and Table 1).
"""
import numpy as np
from scipy.optimize import brentq

C = 299792458.0
MEC2_EV = 510998.95


def beta_of(kinetic_ev):
    g = 1.0 + kinetic_ev / MEC2_EV
    return np.sqrt(1.0 - 1.0 / (g * g))


def _mismatch(w, k, wp, d, sign):
    eps = 1.0 - (wp / w) ** 2
    kd = np.sqrt(max(k * k - (w / C) ** 2, 0.0))
    km = np.sqrt(k * k - eps * (w / C) ** 2)
    return (eps * kd + km) / (eps * kd - km) - sign * np.exp(-km * d)


def film_modes_on_line(wp, d, beta, nscan=20000):
    """Angular frequencies where the thin-film TM modes meet w = beta c k.

    Returns (lower, upper); a branch with no crossing returns nan.
    """
    out = []
    for sign in (+1.0, -1.0):
        ws = np.linspace(0.05 * wp, 0.999 * wp, nscan)
        f = np.array([_mismatch(w, w / (beta * C), wp, d, sign) for w in ws])
        roots = []
        for i in range(nscan - 1):
            if not (np.isfinite(f[i]) and np.isfinite(f[i + 1])):
                continue
            if f[i] == 0.0 or f[i] * f[i + 1] < 0.0:
                # skip the pole where eps kd = km
                a, b = ws[i], ws[i + 1]
                r = brentq(lambda w: _mismatch(w, w / (beta * C), wp, d, sign), a, b,
                           xtol=1e-6, rtol=1e-15)
                if abs(_mismatch(r, r / (beta * C), wp, d, sign)) < 1e-6:
                    roots.append(r)
        out.append(roots[0] if roots else np.nan)
    return tuple(out)


def single_interface_on_line(wp, beta):
    """Thick-film limit: one interface, k^2 = (w/c)^2 eps/(1+eps) on w = beta c k.

    Closed form w^2 = wp^2 (a - 1)/(2a - 1) ... solved here numerically from
    eps kd + km = 0 to stay independent of any algebra.
    """
    def f(w):
        eps = 1.0 - (wp / w) ** 2
        k = w / (beta * C)
        kd = np.sqrt(k * k - (w / C) ** 2)
        km = np.sqrt(k * k - eps * (w / C) ** 2)
        return eps * kd + km
    return brentq(f, 0.05 * wp, wp / np.sqrt(2.0) * (1 - 1e-12), xtol=1e-6, rtol=1e-15)


def single_interface_at_k(wp, k):
    """SPP frequency of one flat Drude/vacuum interface at wavenumber k."""
    def f(w):
        eps = 1.0 - (wp / w) ** 2
        kd = np.sqrt(k * k - (w / C) ** 2)
        km = np.sqrt(k * k - eps * (w / C) ** 2)
        return eps * kd + km
    hi = min(wp / np.sqrt(2.0), k * C) * (1 - 1e-12)
    return brentq(f, 1e-3 * wp, hi, xtol=1e-6, rtol=1e-15)
