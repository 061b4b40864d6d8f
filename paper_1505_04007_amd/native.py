"""ctypes binding of libpic.so (include/pic.h): argument marshalling only.

Every step of the simulation runs in the library's HIP kernels; this module
converts numpy inputs to the C structs, passes torch's current HIP stream,
and converts outputs back.  Importing it fails loudly if the library has not
been built.
"""
import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpic.so")

PIC_OK, PIC_EINVAL, PIC_ENOMEM, PIC_EDEVICE, PIC_EUNSTABLE, PIC_ESTATE, PIC_ENOTSUP = (
    0, -1, -2, -3, -4, -5, -6)
STATUS_NAMES = {0: "PIC_OK", -1: "PIC_EINVAL", -2: "PIC_ENOMEM", -3: "PIC_EDEVICE",
                -4: "PIC_EUNSTABLE", -5: "PIC_ESTATE", -6: "PIC_ENOTSUP"}
BC_PEC, BC_PERIODIC, BC_CPML = 0, 1, 2
FIELD_E, FIELD_H, FIELD_JPOL, FIELD_JB = 0, 1, 2, 3
KERNEL_FAMILIES = ("h_update", "push_deposit", "e_update", "probe", "sort", "field_sweep")

_dp = ctypes.POINTER(ctypes.c_double)


class PicGrid(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("bc", ctypes.c_int32 * 3), ("npml", ctypes.c_int32),
                ("pml_m", ctypes.c_double), ("pml_sigma_scale", ctypes.c_double),
                ("pml_kappa_max", ctypes.c_double), ("pml_alpha_max", ctypes.c_double)]


class PicParticles(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("x", _dp), ("y", _dp), ("z", _dp),
                ("ux", _dp), ("uy", _dp), ("uz", _dp),
                ("q", ctypes.c_double), ("m", ctypes.c_double), ("weight", ctypes.c_double)]


class PicDeviceBuffers(ctypes.Structure):
    _fields_ = [("E", ctypes.c_void_p * 3), ("H", (ctypes.c_void_p * 3) * 2)]


class PicOpts(ctypes.Structure):
    _fields_ = [("stream", ctypes.c_void_p), ("nprobe", ctypes.c_int32), ("probe_xyz", _dp),
                ("nfreq", ctypes.c_int32), ("omega", _dp), ("series_len", ctypes.c_int64),
                ("sort_every", ctypes.c_int32), ("check_every", ctypes.c_int32),
                ("init_E", _dp * 3), ("init_H", _dp * 3), ("diag", ctypes.c_int32),
                ("timing", ctypes.c_int32), ("deposit_mode", ctypes.c_int32),
                ("bufs", ctypes.POINTER(PicDeviceBuffers)), ("field_sweep", ctypes.c_int32)]


class PicDiag(ctypes.Structure):
    _fields_ = [("field_energy", ctypes.c_double), ("count", ctypes.c_double),
                ("mean", ctypes.c_double * 3), ("rms", ctypes.c_double * 3),
                ("umean", ctypes.c_double * 3), ("gauss_max", ctypes.c_double),
                ("rho0_max", ctypes.c_double), ("checked_nodes", ctypes.c_int64)]


class PicStats(ctypes.Structure):
    _fields_ = [("steps", ctypes.c_int64), ("pushes", ctypes.c_int64), ("live", ctypes.c_int64),
                ("pbox", ctypes.c_int32 * 6), ("hcur", ctypes.c_int32), ("device_bytes", ctypes.c_int64)]


class PicBufferSizes(ctypes.Structure):
    _fields_ = [("field_elems", ctypes.c_int64), ("field_bytes", ctypes.c_int64),
                ("device_bytes", ctypes.c_int64), ("bytes_per_metal_box_cell", ctypes.c_int64)]


class PicTuneOut(ctypes.Structure):
    _fields_ = [("tile", ctypes.c_int32), ("fx", ctypes.c_int32), ("fy", ctypes.c_int32),
                ("order", ctypes.c_int32), ("nshapes", ctypes.c_int32), ("ms", ctypes.c_double * 16)]


EXPORTS = ("pic_abi_version", "pic_init", "pic_step", "pic_probe", "pic_grad", "pic_tune",
           "pic_read_fields", "pic_read_particles", "pic_diag", "pic_stats", "pic_timing",
           "pic_destroy", "pic_last_error", "pic_batch_create", "pic_batch_step", "pic_batch_tune",
           "pic_batch_destroy", "pic_batch_last_error", "pic_query_sizes", "pic_grad_noalloc")


def _tune_dict(t):
    return {"tile": t.tile, "fx": t.fx, "fy": t.fy, "order": t.order, "ms": list(t.ms)[: t.nshapes]}

_LIB = None


def load():
    """Load libpic.so; raises if it is missing (there is no fallback path)."""
    global _LIB
    if _LIB is not None:
        return _LIB
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built: run __graft_entry__.build() or "
                          "python paper_1505_04007_amd/csrc/build.py")
    # torch ships its own HIP runtime with the same soname as ROCm's.  Loading
    # torch first makes libpic.so bind to that instance, so the process holds
    # one HIP runtime and torch's streams are valid handles for the library.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = ctypes.CDLL(LIB_PATH)
    vp = ctypes.c_void_p
    lib.pic_abi_version.restype = ctypes.c_int
    lib.pic_init.restype = ctypes.c_int
    lib.pic_init.argtypes = [ctypes.POINTER(vp), ctypes.POINTER(PicGrid), ctypes.c_double,
                             ctypes.c_double, _dp, _dp, ctypes.POINTER(PicParticles),
                             ctypes.POINTER(PicOpts)]
    lib.pic_step.restype = ctypes.c_int
    lib.pic_step.argtypes = [vp, ctypes.c_int64]
    lib.pic_probe.restype = ctypes.c_int
    lib.pic_probe.argtypes = [vp, _dp, _dp, _dp]
    lib.pic_grad.restype = ctypes.c_int
    lib.pic_grad.argtypes = [vp, ctypes.c_double, ctypes.c_int64, ctypes.c_int64, _dp, _dp, _dp]
    lib.pic_grad_noalloc.restype = ctypes.c_int
    lib.pic_grad_noalloc.argtypes = [vp, ctypes.c_double, ctypes.c_int64, _dp, _dp, _dp]
    lib.pic_read_fields.restype = ctypes.c_int
    lib.pic_read_fields.argtypes = [vp, ctypes.c_int, _dp]
    lib.pic_read_particles.restype = ctypes.c_int
    lib.pic_read_particles.argtypes = [vp, _dp]
    lib.pic_diag.restype = ctypes.c_int
    lib.pic_diag.argtypes = [vp, ctypes.POINTER(PicDiag)]
    lib.pic_stats.restype = ctypes.c_int
    lib.pic_stats.argtypes = [vp, ctypes.POINTER(PicStats)]
    lib.pic_timing.restype = ctypes.c_int
    lib.pic_timing.argtypes = [vp, _dp, ctypes.POINTER(ctypes.c_int64), ctypes.c_int]
    lib.pic_destroy.restype = None
    lib.pic_destroy.argtypes = [vp]
    lib.pic_last_error.restype = ctypes.c_char_p
    lib.pic_last_error.argtypes = [vp]
    lib.pic_batch_create.restype = ctypes.c_int
    lib.pic_batch_create.argtypes = [ctypes.POINTER(vp), ctypes.POINTER(vp), ctypes.c_int32,
                                     ctypes.c_int32]
    lib.pic_batch_step.restype = ctypes.c_int
    lib.pic_batch_step.argtypes = [vp, ctypes.c_int64]
    lib.pic_batch_destroy.restype = None
    lib.pic_batch_destroy.argtypes = [vp]
    lib.pic_tune.restype = ctypes.c_int
    lib.pic_tune.argtypes = [vp, ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(PicTuneOut)]
    lib.pic_batch_tune.restype = ctypes.c_int
    lib.pic_batch_tune.argtypes = [vp, ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(PicTuneOut)]
    lib.pic_batch_last_error.restype = ctypes.c_char_p
    lib.pic_batch_last_error.argtypes = [vp]
    lib.pic_query_sizes.restype = ctypes.c_int
    lib.pic_query_sizes.argtypes = [ctypes.POINTER(PicGrid), ctypes.c_int64, ctypes.POINTER(PicOpts),
                                    ctypes.POINTER(PicBufferSizes)]
    _LIB = lib
    return lib


class PicError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


def _p(a):
    return a.ctypes.data_as(_dp) if a is not None else None


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def to_compact(arr_xyz):
    """(nx, ny, nz) array -> compact layout (x fastest) as float64."""
    return _f64(np.asarray(arr_xyz).transpose(2, 1, 0))


def from_compact(flat, n):
    """compact layout (x fastest) -> (nx, ny, nz) array."""
    return np.asarray(flat).reshape(n[2], n[1], n[0]).transpose(2, 1, 0)


def current_stream_handle():
    """torch's current HIP stream as a raw handle (0 = default) when a GPU is present."""
    try:
        import torch
        if torch.cuda.is_available():
            return int(torch.cuda.current_stream().cuda_stream)
    except Exception:
        pass
    return 0


class Simulation:
    """One FDTD-PIC simulation held by a pic_ctx on the GPU.

    Arguments mirror pic_init: grid sizes/boundaries, cell size dx (m), time
    step dt (s), per-cell Drude maps (nx, ny, nz) in rad/s and 1/s, an
    optional bunch, probe positions (m) and DFT frequencies (rad/s).

    device_fields=True: E and both H levels live in torch tensors this object
    allocates (pic_opts.bufs), readable on the GPU without copies through
    device_E() and device_H().
    """

    def __init__(self, nx, ny, nz, dx, dt, wp_map, gamma_map, bc=(BC_PEC,) * 3, npml=0,
                 pml=(3.0, 1.0, 1.0, 0.0), bunch=None, probes=None, omega=None, series_len=0,
                 sort_every=0, check_every=0, init_E=None, init_H=None, diag=False, timing=False,
                 deposit_mode=0, device_fields=False, stream=None, field_sweep=0):
        self._lib = load()
        self._E_dev = self._H_dev = None
        self.n = (int(nx), int(ny), int(nz))
        self.dx, self.dt = float(dx), float(dt)
        g = PicGrid(nx, ny, nz, (ctypes.c_int32 * 3)(*[int(b) for b in bc]), int(npml), *pml)
        self._keep = []
        wp = to_compact(wp_map)
        gm = to_compact(gamma_map)
        self._keep += [wp, gm]
        parts = None
        self.np = 0
        if bunch is not None and bunch.n > 0:
            arrs = [_f64(a) for a in (bunch.x, bunch.y, bunch.z, bunch.ux, bunch.uy, bunch.uz)]
            self._keep += arrs
            parts = PicParticles(bunch.n, *[_p(a) for a in arrs], bunch.q, bunch.m, bunch.w)
            self.np = bunch.n
        o = PicOpts()
        o.stream = current_stream_handle() if stream is None else stream
        self.nprobe = 0 if probes is None else int(np.asarray(probes).reshape(-1, 3).shape[0])
        self.nfreq = 0 if omega is None else int(np.asarray(omega).size)
        if self.nprobe:
            pxyz = _f64(np.asarray(probes).reshape(-1, 3))
            self._keep.append(pxyz)
            o.nprobe, o.probe_xyz = self.nprobe, _p(pxyz)
        if self.nfreq:
            om = _f64(omega)
            self._keep.append(om)
            o.nfreq, o.omega = self.nfreq, _p(om)
        o.series_len = int(series_len)
        o.sort_every = int(sort_every)
        o.check_every = int(check_every)
        for d in range(3):
            if init_E is not None:
                a = to_compact(init_E[d])
                self._keep.append(a)
                o.init_E[d] = _p(a)
            if init_H is not None:
                a = to_compact(init_H[d])
                self._keep.append(a)
                o.init_H[d] = _p(a)
        o.diag = int(bool(diag))
        o.timing = int(timing)
        o.deposit_mode = int(deposit_mode)
        o.field_sweep = int(field_sweep)
        if device_fields:
            import torch
            shape = (int(nz), int(ny), int(nx))
            self._E_dev = torch.empty((3,) + shape, dtype=torch.float32, device="cuda")
            self._H_dev = torch.empty((2, 3) + shape, dtype=torch.float32, device="cuda")
            bufs = PicDeviceBuffers()
            for d in range(3):
                bufs.E[d] = self._E_dev[d].data_ptr()
                for p in range(2):
                    bufs.H[p][d] = self._H_dev[p, d].data_ptr()
            self._keep.append(bufs)
            o.bufs = ctypes.pointer(bufs)
        h = ctypes.c_void_p()
        st = self._lib.pic_init(ctypes.byref(h), ctypes.byref(g), self.dx, self.dt, _p(wp),
                                _p(gm), ctypes.byref(parts) if parts is not None else None,
                                ctypes.byref(o))
        self._h = None
        if st != PIC_OK:
            raise PicError(st, self._lib.pic_last_error(None).decode())
        self._h = h
        self._keep = []

    def _check(self, st):
        if st != PIC_OK:
            raise PicError(st, self._lib.pic_last_error(self._h).decode())

    def close(self):
        if getattr(self, "_h", None):
            self._lib.pic_destroy(self._h)
            self._h = None

    def __del__(self):
        self.close()

    def step(self, n=1):
        self._check(self._lib.pic_step(self._h, int(n)))

    def fields(self, which):
        """(3, nx, ny, nz) float64 in SI units (compact Yee layout positions)."""
        N = self.n[0] * self.n[1] * self.n[2]
        out = np.zeros(3 * N)
        self._check(self._lib.pic_read_fields(self._h, int(which), _p(out)))
        return np.stack([from_compact(out[d * N:(d + 1) * N], self.n) for d in range(3)])

    def particles(self):
        """(6, n) float64: x, y, z (m, NaN once lost), ux, uy, uz (m/s), original order."""
        out = np.zeros(6 * max(self.np, 1))
        self._check(self._lib.pic_read_particles(self._h, _p(out)))
        return out[: 6 * self.np].reshape(6, self.np)

    def probe(self, series=False):
        nf = self.nprobe * self.nfreq
        re = np.zeros(max(nf, 1))
        im = np.zeros(max(nf, 1))
        st = self.stats()["steps"]
        ser = np.zeros(max(st * self.nprobe, 1)) if series else None
        self._check(self._lib.pic_probe(self._h, _p(re), _p(im), _p(ser)))
        F = (re[:nf] + 1j * im[:nf]).reshape(self.nprobe, self.nfreq)
        if series:
            return F, ser
        return F

    def diag(self):
        d = PicDiag()
        self._check(self._lib.pic_diag(self._h, ctypes.byref(d)))
        return {"energy": d.field_energy, "count": d.count, "mean": np.array(d.mean),
                "rms": np.array(d.rms), "umean": np.array(d.umean), "gauss_max": d.gauss_max,
                "rho0_max": d.rho0_max, "checked_nodes": d.checked_nodes}

    def stats(self):
        s = PicStats()
        self._check(self._lib.pic_stats(self._h, ctypes.byref(s)))
        return {"steps": s.steps, "pushes": s.pushes, "live": s.live, "pbox": tuple(s.pbox), "hcur": s.hcur,
                "device_bytes": s.device_bytes}

    def device_E(self):
        """E (V/m) as a torch tensor (3, nz, ny, nx) on the GPU, the library's own
        storage (device_fields=True); ordered after the steps on the context's stream."""
        if self._E_dev is None:
            raise PicError(PIC_EINVAL, "created without device_fields=True")
        return self._E_dev

    def device_H(self):
        """eta0 H (V/m) at the current half step, (3, nz, ny, nx), the library's own
        storage (device_fields=True)."""
        if self._H_dev is None:
            raise PicError(PIC_EINVAL, "created without device_fields=True")
        return self._H_dev[self.stats()["hcur"]]

    def timing(self, reset=False):
        ms = np.zeros(len(KERNEL_FAMILIES))
        cnt = (ctypes.c_int64 * len(KERNEL_FAMILIES))()
        self._check(self._lib.pic_timing(self._h, _p(ms), cnt, int(bool(reset))))
        return {name: (float(ms[i]), int(cnt[i])) for i, name in enumerate(KERNEL_FAMILIES)}

    def tune(self, reps=20, force=-1):
        """pic_tune: pick the field kernels' tile shape (force >= 0: that shape)."""
        t = PicTuneOut()
        self._check(self._lib.pic_tune(self._h, int(reps), int(force), ctypes.byref(t)))
        return _tune_dict(t)

    def grad(self, omega0, nsteps, ckpt_every=0):
        """pic_grad: advance nsteps and return (L, dL/dwp, dL/dgamma), maps (nx, ny, nz)."""
        N = self.n[0] * self.n[1] * self.n[2]
        L = np.zeros(1)
        gw = np.zeros(N)
        gg = np.zeros(N)
        self._check(self._lib.pic_grad(self._h, float(omega0), int(nsteps), int(ckpt_every), _p(L),
                                       _p(gw), _p(gg)))
        return float(L[0]), from_compact(gw, self.n), from_compact(gg, self.n)

    def grad_noalloc(self, omega0, nsteps):
        """pic_grad_noalloc: pic_grad's store-all form with no device allocation."""
        N = self.n[0] * self.n[1] * self.n[2]
        L = np.zeros(1)
        gw = np.zeros(N)
        gg = np.zeros(N)
        self._check(self._lib.pic_grad_noalloc(self._h, float(omega0), int(nsteps), _p(L), _p(gw),
                                               _p(gg)))
        return float(L[0]), from_compact(gw, self.n), from_compact(gg, self.n)


def spp_power(make_sim, omega0, nsteps, ckpt_every=0):
    """A torch.autograd.Function-backed map (wp_map, gamma_map) -> L.

    ``make_sim(wp, gamma)`` builds a fresh Simulation from numpy maps (nx, ny,
    nz).  Calling the returned function with two float64 tensors runs pic_grad
    once: its forward pass yields L and the adjoint's gradients, which the
    backward pass scales by the incoming gradient.
    """
    import torch

    class SppPower(torch.autograd.Function):
        @staticmethod
        def forward(ctx, wp, gamma):
            sim = make_sim(wp.detach().cpu().double().numpy(), gamma.detach().cpu().double().numpy())
            L, gw, gg = sim.grad(omega0, nsteps, ckpt_every)
            ctx.save_for_backward(torch.from_numpy(gw).to(wp.device), torch.from_numpy(gg).to(gamma.device))
            return torch.tensor(L, dtype=torch.float64, device=wp.device)

        @staticmethod
        def backward(ctx, g):
            gw, gg = ctx.saved_tensors
            return g * gw, g * gg

    return SppPower.apply


def query_sizes(nx, ny, nz, bc=(BC_PEC,) * 3, npml=0, pml=(3.0, 1.0, 1.0, 0.0), nparticles=0,
                nprobe=0, nfreq=0, series_len=0, diag=False, device_fields=False, deposit_mode=0,
                field_sweep=0):
    """pic_query_sizes: device memory pic_init needs (a dict of pic_buffer_sizes).

    device_fields=True counts E and H as caller memory (as Simulation(...,
    device_fields=True) provides them); the query reads only which entries are
    set and how they are laid out, so placeholders with the layout of those
    tensors (each field one block, components nx*ny*nz apart) stand in."""
    lib = load()
    g = PicGrid(nx, ny, nz, (ctypes.c_int32 * 3)(*[int(b) for b in bc]), int(npml), *pml)
    o = PicOpts()
    o.nprobe, o.nfreq, o.series_len, o.diag = int(nprobe), int(nfreq), int(series_len), int(bool(diag))
    o.deposit_mode = int(deposit_mode)
    o.field_sweep = int(field_sweep)
    if device_fields:
        N = 4 * int(nx) * int(ny) * int(nz)
        bufs = PicDeviceBuffers()
        for d in range(3):
            bufs.E[d] = 4096 + d * N
            for p in range(2):
                bufs.H[p][d] = 4096 + (3 + 3 * p + d) * N
        o.bufs = ctypes.pointer(bufs)
    out = PicBufferSizes()
    st = lib.pic_query_sizes(ctypes.byref(g), int(nparticles), ctypes.byref(o), ctypes.byref(out))
    if st != PIC_OK:
        raise PicError(st, lib.pic_last_error(None).decode())
    return {"field_elems": out.field_elems, "field_bytes": out.field_bytes, "device_bytes": out.device_bytes,
            "bytes_per_metal_box_cell": out.bytes_per_metal_box_cell}


def workload_sizes(w, with_bunch=True, **kw):
    """query_sizes for a pic_inputs.Workload, with what from_workload passes."""
    return query_sizes(w.nx, w.ny, w.nz, bc=w.bc, npml=w.npml, pml=w.pml,
                       nparticles=w.bunch.n if (with_bunch and w.bunch is not None) else 0,
                       nprobe=len(w.probes), nfreq=len(w.omega), **kw)


def from_workload(w, with_bunch=True, **kw):
    """Simulation for a pic_inputs.Workload."""
    return Simulation(w.nx, w.ny, w.nz, w.dx, w.dt, w.wp_map, w.gamma_map, bc=w.bc, npml=w.npml,
                      pml=w.pml, bunch=w.bunch if with_bunch else None, probes=w.probes,
                      omega=w.omega, sort_every=kw.pop("sort_every", w.sort_every), **kw)


class Batch:
    """Several Simulations advanced together (pic_batch_*): one launch per kernel
    family per step for all members, optionally replaying a captured HIP graph
    of one sort period.  The member Simulations stay readable and must outlive
    the batch."""

    def __init__(self, sims, use_graph=True):
        self._lib = load()
        self.sims = list(sims)
        arr = (ctypes.c_void_p * len(self.sims))(*[s._h.value for s in self.sims])
        h = ctypes.c_void_p()
        st = self._lib.pic_batch_create(ctypes.byref(h), arr, len(self.sims), int(bool(use_graph)))
        self._h = None
        if st != PIC_OK:
            raise PicError(st, self._lib.pic_batch_last_error(None).decode())
        self._h = h

    def step(self, n=1):
        st = self._lib.pic_batch_step(self._h, int(n))
        if st != PIC_OK:
            raise PicError(st, self._lib.pic_batch_last_error(self._h).decode())

    def tune(self, reps=10, force=-1):
        """pic_batch_tune: one tile shape for all members' field launches."""
        t = PicTuneOut()
        st = self._lib.pic_batch_tune(self._h, int(reps), int(force), ctypes.byref(t))
        if st != PIC_OK:
            raise PicError(st, self._lib.pic_batch_last_error(self._h).decode())
        return _tune_dict(t)

    def close(self):
        if getattr(self, "_h", None):
            self._lib.pic_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        self.close()
