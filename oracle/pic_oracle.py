"""ctypes wrapper of the FP64 CPU oracle (test infrastructure only).

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
import this module.  It loads ``liboracle.so`` built from ``oracle.c`` and
exposes the oracle's state as numpy arrays on the full staggered Yee lattice:

    E[0] (nx, ny+1, nz+1)   E[1] (nx+1, ny, nz+1)   E[2] (nx+1, ny+1, nz)
    H[0] (nx+1, ny, nz)     H[1] (nx, ny+1, nz)     H[2] (nx, ny, nz+1)

All quantities are SI and float64.  Boundary codes: 0 PEC, 1 periodic,
2 CPML backed by PEC.
"""
import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
# the library this module loads; a test that plants a mistake in a copy of the
# oracle points a separate instance of this module at that copy's build
LIB_PATH = os.path.join(HERE, "liboracle.so")
_LIB = None

PEC, PERIODIC, CPML = 0, 1, 2
_dp = ctypes.POINTER(ctypes.c_double)


def _load():
    global _LIB
    if _LIB is not None:
        return _LIB
    path = LIB_PATH
    if not os.path.exists(path):
        from . import build as _b  # type: ignore
        _b.build()
    lib = ctypes.CDLL(path)
    lib.osim_create.restype = ctypes.c_void_p
    lib.osim_create.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                ctypes.POINTER(ctypes.c_int), ctypes.c_int, _dp,
                                ctypes.c_double, ctypes.c_double, _dp, _dp]
    lib.osim_destroy.argtypes = [ctypes.c_void_p]
    lib.osim_field_ptr.restype = _dp
    lib.osim_field_ptr.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int,
                                   ctypes.POINTER(ctypes.c_int)]
    lib.osim_step.argtypes = [ctypes.c_void_p, ctypes.c_long]
    lib.osim_get_step.restype = ctypes.c_long
    lib.osim_get_step.argtypes = [ctypes.c_void_p]
    lib.osim_set_particles.argtypes = [ctypes.c_void_p, ctypes.c_long] + [_dp] * 6 + [
        ctypes.c_double] * 3
    lib.osim_get_particles.argtypes = [ctypes.c_void_p, ctypes.c_int, _dp]
    lib.osim_set_probes.argtypes = [ctypes.c_void_p, ctypes.c_int, _dp, ctypes.c_int, _dp]
    lib.osim_probe.argtypes = [ctypes.c_void_p, _dp, _dp]
    lib.osim_probe_values.argtypes = [ctypes.c_void_p, _dp]
    lib.osim_gather.argtypes = [ctypes.c_void_p, _dp, _dp, _dp]
    lib.osim_deposit_move.argtypes = [ctypes.c_void_p, _dp, _dp]
    lib.oracle_boris.argtypes = [ctypes.c_double, ctypes.c_double, ctypes.c_double, _dp, _dp, _dp]
    lib.osim_rho.argtypes = [ctypes.c_void_p, _dp]
    lib.osim_gauss.argtypes = [ctypes.c_void_p, _dp]
    lib.osim_diag.argtypes = [ctypes.c_void_p, _dp]
    lib.osim_timing.argtypes = [ctypes.c_void_p, _dp]
    lib.oracle_constants.argtypes = [_dp]
    lib.osim_jb_size.restype = ctypes.c_long
    lib.osim_jb_size.argtypes = [ctypes.c_void_p]
    lib.osim_prescribe_jb.argtypes = [ctypes.c_void_p, _dp, ctypes.c_long]
    lib.osim_run_record_jb.argtypes = [ctypes.c_void_p, ctypes.c_long, _dp]
    lib.osim_adj_zero.argtypes = [ctypes.c_void_p]
    lib.osim_adj_step.argtypes = [ctypes.c_void_p]
    lib.osim_adj_ptr.restype = _dp
    lib.osim_adj_ptr.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                 ctypes.POINTER(ctypes.c_int)]
    lib.osim_grad.argtypes = [ctypes.c_void_p, ctypes.c_long, ctypes.c_double, _dp, _dp, _dp]
    lib.osim_run_record_jb_box.restype = ctypes.c_double
    lib.osim_run_record_jb_box.argtypes = [ctypes.c_void_p, ctypes.c_long, ctypes.POINTER(ctypes.c_int),
                                           ctypes.POINTER(ctypes.c_int), _dp]
    lib.osim_prescribe_jb_box.argtypes = [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int),
                                          ctypes.POINTER(ctypes.c_int), _dp, ctypes.c_long]
    lib.osim_test_uniform_cpml.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_double,
                                           ctypes.c_double, ctypes.c_double]
    lib.osim_cpml_profile.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, _dp, _dp, _dp]
    _LIB = lib
    return lib


def _p(a):
    return a.ctypes.data_as(_dp)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def constants():
    """(c, mu0, eps0) as the oracle defines them."""
    out = np.zeros(3)
    _load().oracle_constants(_p(out))
    return tuple(out)


def boris(q, m, dt, E, B, u):
    """One relativistic Boris step of u = gamma v (m/s) under E, B (SI)."""
    E, B = _f64(E), _f64(B)
    u = _f64(u).copy()
    _load().oracle_boris(q, m, dt, _p(E), _p(B), _p(u))
    return u


class OracleSim:
    """One FP64 FDTD-PIC simulation on the full Yee lattice."""

    def __init__(self, nx, ny, nz, dx, dt, bc=(PEC, PEC, PEC), npml=0,
                 pml=(3.0, 1.0, 1.0, 0.0), wp_map=None, gamma_map=None):
        lib = _load()
        self.n = (int(nx), int(ny), int(nz))
        self.dx, self.dt = float(dx), float(dt)
        self.bc = tuple(int(b) for b in bc)
        shape = self.n
        wp = _f64(np.zeros(shape) if wp_map is None else wp_map)
        g = _f64(np.zeros(shape) if gamma_map is None else gamma_map)
        assert wp.shape == shape and g.shape == shape
        bc_arr = (ctypes.c_int * 3)(*self.bc)
        pml_arr = _f64(pml)
        self._h = lib.osim_create(nx, ny, nz, bc_arr, int(npml), _p(pml_arr), self.dx, self.dt,
                                  _p(wp), _p(g))
        self._lib = lib
        self.np = 0

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            self._lib.osim_destroy(h)
            self._h = None

    def _field(self, which, comp):
        ext = (ctypes.c_int * 3)()
        ptr = self._lib.osim_field_ptr(self._h, which, comp, ext)
        shape = tuple(ext)
        return np.ctypeslib.as_array(ptr, shape=shape)

    # live views into the oracle's arrays (writable)
    @property
    def E(self):
        return [self._field(0, c) for c in range(3)]

    @property
    def H(self):
        return [self._field(1, c) for c in range(3)]

    @property
    def J(self):
        return [self._field(2, c) for c in range(3)]

    @property
    def P(self):
        return [self._field(3, c) for c in range(3)]

    @property
    def Jb(self):
        return [self._field(4, c) for c in range(3)]

    @property
    def Hprev(self):
        return [self._field(5, c) for c in range(3)]

    def step(self, n=1):
        self._lib.osim_step(self._h, int(n))

    @property
    def nstep(self):
        return self._lib.osim_get_step(self._h)

    def set_particles(self, x, y, z, ux, uy, uz, q, m, w):
        arrs = [_f64(a) for a in (x, y, z, ux, uy, uz)]
        self._keep = arrs
        self.np = len(arrs[0])
        self._lib.osim_set_particles(self._h, self.np, *[_p(a) for a in arrs], float(q), float(m),
                                     float(w))

    def particles(self):
        """(x, y, z, ux, uy, uz, alive) as float64 arrays."""
        out = []
        for w in range(7):
            a = np.zeros(max(self.np, 1))
            self._lib.osim_get_particles(self._h, w, _p(a))
            out.append(a[: self.np])
        out[6] = out[6].astype(bool)
        return out

    def set_probes(self, xyz, omega):
        xyz = _f64(np.asarray(xyz).reshape(-1, 3))
        om = _f64(omega)
        self._probe_shape = (xyz.shape[0], om.shape[0])
        self._lib.osim_set_probes(self._h, xyz.shape[0], _p(xyz), om.shape[0], _p(om))

    def probe(self):
        """Complex FP64 accumulators F[p, m] = sum_n dt Ez_p^n exp(-i w_m n dt)."""
        npb, nf = self._probe_shape
        re = np.zeros(max(npb * nf, 1))
        im = np.zeros(max(npb * nf, 1))
        self._lib.osim_probe(self._h, _p(re), _p(im))
        return (re[: npb * nf] + 1j * im[: npb * nf]).reshape(npb, nf)

    def probe_values(self):
        npb = self._probe_shape[0]
        out = np.zeros(max(npb, 1))
        self._lib.osim_probe_values(self._h, _p(out))
        return out[:npb]

    def gather(self, pos):
        pos = _f64(pos)
        E = np.zeros(3)
        B = np.zeros(3)
        self._lib.osim_gather(self._h, _p(pos), _p(E), _p(B))
        return E, B

    def deposit_move(self, p0, p1):
        p0, p1 = _f64(p0), _f64(p1)
        self._lib.osim_deposit_move(self._h, _p(p0), _p(p1))

    def rho(self):
        out = np.zeros((self.n[0] + 1, self.n[1] + 1, self.n[2] + 1))
        self._lib.osim_rho(self._h, _p(out))
        return out

    def gauss(self):
        out = np.zeros((self.n[0] + 1, self.n[1] + 1, self.n[2] + 1))
        self._lib.osim_gauss(self._h, _p(out))
        return out

    def diag(self):
        """dict(energy, count, mean[3], rms[3], umean[3])."""
        out = np.zeros(11)
        self._lib.osim_diag(self._h, _p(out))
        return {"energy": out[0], "count": out[1], "mean": out[2:5], "rms": out[5:8],
                "umean": out[8:11]}

    def timing(self):
        out = np.zeros(4)
        self._lib.osim_timing(self._h, _p(out))
        return {"field_s": out[0], "particle_s": out[1], "pushes": int(out[2]),
                "threads": int(out[3])}

    # ---- bunch current as a prescribed source, and the adjoint ----
    def jb_size(self):
        """Doubles in one J_b snapshot (the three E-edge arrays back to back)."""
        return int(self._lib.osim_jb_size(self._h))

    def run_record_jb(self, n):
        """Step n times and return J_b^{n+1/2} of each step, shape (n, jb_size)."""
        out = np.zeros((int(n), self.jb_size()))
        self._lib.osim_run_record_jb(self._h, int(n), _p(out))
        return out

    def prescribe_jb(self, hist):
        """Use hist[r] as the bunch current of the r-th next step (no particle push)."""
        hist = _f64(hist)
        assert hist.ndim == 2 and hist.shape[1] == self.jb_size()
        self._lib.osim_prescribe_jb(self._h, _p(hist), hist.shape[0])

    def run_record_jb_box(self, n, lo, ext):
        """Step n times recording J_b^{n+1/2} on the cell box [lo, lo + ext) of each
        component: returns (records (n, 3, *ext), largest |J_b| seen outside the box)."""
        lo_c = (ctypes.c_int * 3)(*[int(v) for v in lo])
        ext_c = (ctypes.c_int * 3)(*[int(v) for v in ext])
        out = np.zeros((int(n), 3) + tuple(int(v) for v in ext))
        outside = self._lib.osim_run_record_jb_box(self._h, int(n), lo_c, ext_c, _p(out))
        return out, float(outside)

    def prescribe_jb_box(self, lo, ext, hist):
        """Use hist[r] (3, *ext) on the box as the bunch current of the r-th next step."""
        hist = _f64(hist)
        assert hist.shape[1:] == (3,) + tuple(int(v) for v in ext)
        lo_c = (ctypes.c_int * 3)(*[int(v) for v in lo])
        ext_c = (ctypes.c_int * 3)(*[int(v) for v in ext])
        self._lib.osim_prescribe_jb_box(self._h, lo_c, ext_c, _p(hist), hist.shape[0])

    def _adj(self, which, c, a=0):
        ext = (ctypes.c_int * 3)()
        ptr = self._lib.osim_adj_ptr(self._h, which, c, a, ext)
        if not ptr:
            return None
        return np.ctypeslib.as_array(ptr, shape=tuple(ext))

    @property
    def Ea(self):
        return [self._adj(0, c) for c in range(3)]

    @property
    def Ha(self):
        return [self._adj(1, c) for c in range(3)]

    @property
    def Ja(self):
        return [self._adj(2, c) for c in range(3)]

    def psi(self, field, c, a, adjoint=False):
        """CPML memory of component c along axis a ('E' or 'H'); None if absent."""
        which = {"E": 3, "H": 4}[field] + (2 if adjoint else 0)
        return self._adj(which, c, a)

    def adj_zero(self):
        self._lib.osim_adj_zero(self._h)

    def adj_step(self):
        """Apply the transpose of one field step (bunch current fixed) to the adjoint state."""
        self._lib.osim_adj_step(self._h)

    def grad(self, nsteps, omega0):
        """Run nsteps forward, then the adjoint back.  Returns (L, dL/dwp, dL/dgamma)
        for L = sum over probes of |F_p(omega0)|^2, with the bunch current held at
        the values of this forward run."""
        L = np.zeros(1)
        gw = np.zeros(self.n)
        gg = np.zeros(self.n)
        self._lib.osim_grad(self._h, int(nsteps), float(omega0), _p(L), _p(gw), _p(gg))
        return float(L[0]), gw, gg

    # ---- test-only access to the absorbing layers' coefficient tables ----
    def test_uniform_cpml(self, axis, b, c, kappa):
        """Give axis `axis` the same CPML recursion (b, c, kappa) at every E-type
        and H-type position (test-only; the step's arithmetic is unchanged)."""
        self._lib.osim_test_uniform_cpml(self._h, int(axis), float(b), float(c), float(kappa))

    def cpml_profile(self, axis, h):
        """(b, c, kappa) tables of an axis: h = 0 E-type at nodes 0..n, h = 1
        H-type at i + 1/2, i = 0..n-1 (b = 1, c = 0, kappa = 1 outside the layers)."""
        n = self.n[axis] + (0 if h else 1)
        b, c, k = np.zeros(n), np.zeros(n), np.zeros(n)
        self._lib.osim_cpml_profile(self._h, int(axis), int(h), _p(b), _p(c), _p(k))
        return b, c, k
