"""ctypes binding of libnct.so (include/nct.h): argument marshalling only.

Every computation runs in the HIP library.  torch provides device memory and
the stream.  If libnct.so is missing, or no GPU is present, the calls raise:
there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import math
import os
from ctypes import POINTER, c_double, c_int, c_void_p
from typing import Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libnct.so")

NCT_OK, NCT_ERR_ARG, NCT_ERR_UNSUPPORTED, NCT_ERR_OOM, NCT_ERR_HIP, NCT_ERR_NONFINITE, NCT_ERR_STATE = range(7)
NCT_GAUGE_LENGTH, NCT_GAUGE_VELOCITY = 0, 1
NCT_FP64, NCT_FP32_MIXED = 0, 1
STATUS_NAMES = {0: "NCT_OK", 1: "NCT_ERR_ARG", 2: "NCT_ERR_UNSUPPORTED", 3: "NCT_ERR_OOM",
                4: "NCT_ERR_HIP", 5: "NCT_ERR_NONFINITE", 6: "NCT_ERR_STATE"}
KERNEL_CLASSES = ["plane_stage", "xpass", "plane_fwd", "density", "fields", "proj", "obs", "adjoint",
                  "orth"]
OBS_NAMES = ["t", "N_e", "M_x", "M_y", "M_z", "E_total", "E_kin", "E_loc", "E_NL", "E_H",
             "E_xc", "E_Z", "max_norm_err"]


class Channel(ctypes.Structure):
    _fields_ = [("l", c_int), ("twoj", c_int), ("energy", c_double), ("rc", c_double)]


class Pulse(ctypes.Structure):
    _fields_ = [("A", c_double), ("omega", c_double), ("t0", c_double), ("tau", c_double),
                ("phase", c_double), ("e1", c_double * 3), ("e2", c_double * 3)]


class BField(ctypes.Structure):
    _fields_ = [("B0", c_double * 3), ("npulses", c_int), ("pulses", POINTER(Pulse))]


class AtomDensity(ctypes.Structure):
    _fields_ = [("Z", c_double), ("sigma", c_double), ("moment", c_double * 3)]


class LaserPulse(ctypes.Structure):
    _fields_ = [("A", c_double), ("omega", c_double), ("t0", c_double), ("tau", c_double),
                ("phase", c_double), ("pol", c_double * 3)]


class Params(ctypes.Structure):
    _fields_ = [("n", c_int * 3), ("cell", c_double * 3), ("nstates", c_int),
                ("occ", POINTER(c_double)), ("natoms", c_int), ("positions", POINTER(c_double)),
                ("nchannels", c_int), ("channels", POINTER(Channel)), ("r_sphere", c_double),
                ("xc", c_int), ("hartree", c_int), ("m_threshold", c_double), ("dt", c_double),
                ("taylor_order", c_int), ("precision", c_int), ("tape_steps", c_int),
                ("overlap", c_int), ("stream", c_void_p)]


class NctError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(code, code)}: {msg}")
        self.code = code


_LIB = None


def lib():
    """Load libnct.so (raises if it has not been built)."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"libnct.so not built at {LIB_PATH}; run __graft_entry__.build()")
        L = ctypes.CDLL(LIB_PATH)
        L.nct_create_system.argtypes = [POINTER(Params), POINTER(c_void_p)]
        L.nct_create_system.restype = c_int
        L.nct_destroy_system.argtypes = [c_void_p]
        L.nct_destroy_system.restype = None
        L.nct_last_error.argtypes = [c_void_p]
        L.nct_last_error.restype = ctypes.c_char_p
        L.nct_set_potentials.argtypes = [c_void_p, c_void_p, POINTER(BField), c_void_p]
        L.nct_set_potentials.restype = c_int
        L.nct_set_laser.argtypes = [c_void_p, c_int, POINTER(LaserPulse)]
        L.nct_set_laser.restype = c_int
        L.nct_set_kpoints.argtypes = [c_void_p, c_void_p]
        L.nct_set_kpoints.restype = c_int
        L.nct_set_laser_gauge.argtypes = [c_void_p, c_int]
        L.nct_set_laser_gauge.restype = c_int
        L.nct_dm_initialization.argtypes = [c_void_p, POINTER(AtomDensity), c_void_p, c_int]
        L.nct_dm_initialization.restype = c_int
        L.nct_ground_state.argtypes = [c_void_p, c_void_p, c_int, c_double, c_int, POINTER(c_double)]
        L.nct_ground_state.restype = c_int
        L.nct_density_magnetization.argtypes = [c_void_p, c_void_p, c_double, c_void_p,
                                                POINTER(c_double), c_int]
        L.nct_density_magnetization.restype = c_int
        L.nct_density_magnetization_static.argtypes = [c_void_p, c_void_p, c_double, c_void_p,
                                                       POINTER(c_double), c_int]
        L.nct_density_magnetization_static.restype = c_int
        L.nct_get_fields.argtypes = [c_void_p, c_double, c_void_p]
        L.nct_get_fields.restype = c_int
        L.nct_apply_hamiltonian.argtypes = [c_void_p, c_void_p, c_void_p, c_double]
        L.nct_apply_hamiltonian.restype = c_int
        L.nct_step.argtypes = [c_void_p, c_void_p, c_double, c_int, POINTER(c_double), c_int]
        L.nct_step.restype = c_int
        L.nct_magnetization_seed.argtypes = [c_void_p, c_void_p, POINTER(c_double), c_void_p]
        L.nct_magnetization_seed.restype = c_int
        L.nct_backward_step.argtypes = [c_void_p, c_int, c_void_p, c_double, c_void_p, c_void_p,
                                        POINTER(c_double), POINTER(c_double)]
        L.nct_backward_step.restype = c_int
        L.nct_set_watchdog.argtypes = [c_void_p, c_double]
        L.nct_set_watchdog.restype = c_int
        L.nct_set_timing.argtypes = [c_void_p, c_int]
        L.nct_set_timing.restype = c_int
        L.nct_set_timing_sample.argtypes = [c_void_p, c_int]
        L.nct_set_timing_sample.restype = c_int
        L.nct_get_timing.argtypes = [c_void_p, c_int, POINTER(c_double), POINTER(ctypes.c_longlong),
                                     POINTER(c_double), POINTER(c_double)]
        L.nct_get_timing.restype = c_int
        L.nct_version.argtypes = []
        L.nct_version.restype = ctypes.c_char_p
        _LIB = L
    return _LIB


def _dptr(x: np.ndarray):
    return x.ctypes.data_as(POINTER(c_double))


def _tptr(t) -> Optional[int]:
    if t is None:
        return None
    import torch
    if not t.is_cuda:
        raise ValueError("expected a device tensor")
    if not t.is_contiguous():
        raise ValueError("expected a contiguous tensor")
    return t.data_ptr()


class System:
    """One nct_system.  States are torch tensors [S, 2, nx, ny, nz] (complex128 or complex64)."""

    def __init__(self, n: Sequence[int], cell: Sequence[float], nstates: int, occ=None,
                 positions=None, channels=(), r_sphere: float = 2.5, xc: int = 1,
                 hartree: int = 1, m_threshold: float = 1e-12, dt: float = 0.05,
                 taylor_order: int = 4, precision: int = NCT_FP64, tape_steps: int = 0,
                 overlap: bool = False, stream=None):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("nct.System needs a GPU (no CPU fallback)")
        L = lib()
        self._keep = []
        p = Params()
        p.n = (c_int * 3)(*[int(v) for v in n])
        p.cell = (c_double * 3)(*[float(v) for v in cell])
        p.nstates = int(nstates)
        if occ is not None:
            occ = np.ascontiguousarray(occ, dtype=np.float64)
            self._keep.append(occ)
            p.occ = _dptr(occ)
        pos = np.ascontiguousarray(np.zeros((0, 3)) if positions is None else positions,
                                   dtype=np.float64).reshape(-1, 3)
        self._keep.append(pos)
        p.natoms = int(pos.shape[0])
        p.positions = _dptr(pos) if pos.size else None
        chans = (Channel * max(1, len(channels)))()
        for k, c in enumerate(channels):
            chans[k] = Channel(int(c.l), int(c.twoj), float(c.energy), float(c.rc))
        self._keep.append(chans)
        p.nchannels = len(channels)
        p.channels = ctypes.cast(chans, POINTER(Channel)) if len(channels) else None
        p.r_sphere = float(r_sphere)
        p.xc, p.hartree = int(xc), int(hartree)
        p.m_threshold = float(m_threshold)
        p.dt = float(dt)
        p.taylor_order = int(taylor_order)
        p.precision = int(precision)
        p.tape_steps = int(tape_steps)
        p.overlap = int(bool(overlap))
        if stream is None:
            stream = torch.cuda.current_stream()
        self.stream = stream
        p.stream = c_void_p(stream.cuda_stream)
        self.params = p
        h = c_void_p()
        rc = L.nct_create_system(ctypes.byref(p), ctypes.byref(h))
        if rc != NCT_OK:
            raise NctError(rc, L.nct_last_error(None).decode())
        self.h = h
        self.n = tuple(int(v) for v in n)
        self.N = int(np.prod(self.n))
        self.S = int(nstates)
        self.precision = int(precision)
        self.dtype = torch.complex128 if precision == NCT_FP64 else torch.complex64
        self.npulses = 0
        self.bfield_args = ((0.0, 0.0, 0.0), [])  # (B0, pulses) last given to set_potentials

    # ------------------------------------------------------------------ helpers
    def _check(self, rc: int):
        if rc != NCT_OK:
            raise NctError(rc, lib().nct_last_error(self.h).decode())

    def close(self):
        if getattr(self, "h", None) is not None and self.h.value:
            lib().nct_destroy_system(self.h)
            self.h = c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def new_states(self):
        import torch
        return torch.empty((self.S, 2) + self.n, dtype=self.dtype, device="cuda")

    # ------------------------------------------------------------------ C ABI
    def set_potentials(self, v_ext=None, B0=None, pulses=None, fields=None):
        bf = None
        if B0 is not None or pulses is not None:
            pl = list(pulses or [])
            arr = (Pulse * max(1, len(pl)))()
            for k, q in enumerate(pl):
                arr[k] = Pulse(q.A, q.omega, q.t0, q.tau, getattr(q, "phase", 0.0),
                               (c_double * 3)(*q.e1), (c_double * 3)(*q.e2))
            b0 = tuple(float(v) for v in (B0 if B0 is not None else (0.0, 0.0, 0.0)))
            bf = BField((c_double * 3)(*b0), len(pl), ctypes.cast(arr, POINTER(Pulse)) if pl else None)
            self._keep.append(arr)
            self.npulses = len(pl)
            self.bfield_args = (b0, list(pl))
        self._check(lib().nct_set_potentials(self.h, _tptr(v_ext),
                                             ctypes.byref(bf) if bf is not None else None,
                                             _tptr(fields)))

    def set_laser(self, pulses=None):
        """Uniform electric pulses (objects with A, omega, t0, tau, phase, pol); None or [] removes."""
        pl = list(pulses or [])
        arr = (LaserPulse * max(1, len(pl)))()
        for k, q in enumerate(pl):
            arr[k] = LaserPulse(q.A, q.omega, q.t0, q.tau, getattr(q, "phase", 0.0),
                                (c_double * 3)(*q.pol))
        self._check(lib().nct_set_laser(self.h, len(pl), ctypes.cast(arr, POINTER(LaserPulse)) if pl else None))

    def dm_initialization(self, atoms, rho_v=None, update_fields: bool = True):
        """Initial spin-density matrix from per-atom (Z, sigma, moment) (objects with those
        attributes, in the order of the atom positions)."""
        arr = (AtomDensity * max(1, len(atoms)))()
        for k, a in enumerate(atoms):
            arr[k] = AtomDensity(a.Z, a.sigma, (c_double * 3)(*a.moment))
        self._check(lib().nct_dm_initialization(self.h, ctypes.cast(arr, POINTER(AtomDensity)),
                                                _tptr(rho_v), int(update_fields)))

    def ground_state(self, psi, niter: int, tau: float, keep_fields: bool = False):
        """Imaginary-time ground state in place; returns the total energy after each iteration."""
        e = np.zeros(max(int(niter), 1))
        self._check(lib().nct_ground_state(self.h, _tptr(psi), int(niter), float(tau),
                                           int(keep_fields), _dptr(e)))
        return e[:int(niter)]

    def set_laser_gauge(self, gauge: str):
        """"length" (isolated systems) or "velocity" (periodic systems)."""
        code = {"length": NCT_GAUGE_LENGTH, "velocity": NCT_GAUGE_VELOCITY}.get(gauge, -1)
        self._check(lib().nct_set_laser_gauge(self.h, code))

    def set_kpoints(self, kvec=None):
        """Bloch vector [S, 3] of each state (None: Gamma only); k-weights go into occ."""
        if kvec is None:
            self._check(lib().nct_set_kpoints(self.h, None))
            return
        k = np.ascontiguousarray(np.asarray(kvec, dtype=np.float64).reshape(-1, 3))
        self._check(lib().nct_set_kpoints(self.h, k.ctypes.data_as(c_void_p)))

    def density_magnetization(self, psi, t: float = 0.0, rho_v=None, totals: bool = False,
                              update_fields: bool = False):
        tot = np.zeros(4)
        self._check(lib().nct_density_magnetization(self.h, _tptr(psi), float(t), _tptr(rho_v),
                                                     _dptr(tot) if totals else None,
                                                     int(update_fields)))
        return tot if totals else None

    def density_magnetization_static(self, psi, t: float = 0.0, rho_v=None, totals: bool = False,
                                     update_fields: bool = False):
        """nct_density_magnetization_static: the same results with every temporary in the
        library's static device array (no allocation during the call)."""
        tot = np.zeros(4)
        self._check(lib().nct_density_magnetization_static(self.h, _tptr(psi), float(t), _tptr(rho_v),
                                                            _dptr(tot) if totals else None,
                                                            int(update_fields)))
        return tot if totals else None

    def get_fields(self, t: float, out):
        self._check(lib().nct_get_fields(self.h, float(t), _tptr(out)))

    def apply_hamiltonian(self, psi, hpsi, t: float = 0.0):
        self._check(lib().nct_apply_hamiltonian(self.h, _tptr(psi), _tptr(hpsi), float(t)))

    def step(self, psi, t0: float, nsteps: int, obs: bool = False, tape: bool = False):
        out = np.zeros((max(nsteps, 1), 13)) if obs else None
        self._check(lib().nct_step(self.h, _tptr(psi), float(t0), int(nsteps),
                                   _dptr(out) if obs else None, int(tape)))
        return out[:nsteps] if obs else None

    def magnetization_seed(self, psi, w, lam):
        wv = np.ascontiguousarray(w, dtype=np.float64)
        self._check(lib().nct_magnetization_seed(self.h, _tptr(psi), _dptr(wv), _tptr(lam)))

    def backward_step(self, tape_index: int, psi_n, t_n: float, lam_np1, lam_n, dLdtheta=None):
        dLdB = np.zeros(6)
        self._check(lib().nct_backward_step(self.h, int(tape_index), _tptr(psi_n), float(t_n),
                                            _tptr(lam_np1), _tptr(lam_n), _dptr(dLdB),
                                            _dptr(dLdtheta) if dLdtheta is not None else None))
        return dLdB

    def set_watchdog(self, max_rel_drift: float):
        """Largest relative drift of N_e over one nct_step call (<= 0: finiteness only)."""
        self._check(lib().nct_set_watchdog(self.h, float(max_rel_drift)))

    def set_timing(self, mask: int):
        """Bit k of mask instruments kernel class k (KERNEL_CLASSES); -1 = all, 0 = off."""
        self._check(lib().nct_set_timing(self.h, int(mask)))

    def set_timing_sample(self, every: int):
        """Record one launch in every `every` of each timed class."""
        self._check(lib().nct_set_timing_sample(self.h, int(every)))

    def timing(self):
        """{class: (ms, launches, algorithmic bytes, flops)} since the last set_timing."""
        out = {}
        for k, name in enumerate(KERNEL_CLASSES):
            ms, cnt, by, fl = c_double(), ctypes.c_longlong(), c_double(), c_double()
            self._check(lib().nct_get_timing(self.h, k, ctypes.byref(ms), ctypes.byref(cnt),
                                             ctypes.byref(by), ctypes.byref(fl)))
            out[name] = (ms.value, cnt.value, by.value, fl.value)
        return out


def system_from_workload(w, precision: int = NCT_FP64, tape_steps: int = 0, dt=None,
                         taylor_order=None, overlap: bool = False, stream=None) -> System:
    """Create a System for a seeded workload and upload its v_ext and B field."""
    import torch
    s = System(w.n, w.L, w.nstates, occ=w.occ, positions=w.positions, channels=w.channels,
               r_sphere=w.r_sphere, xc=w.xc, hartree=w.hartree, m_threshold=w.m_threshold,
               dt=w.dt if dt is None else dt,
               taylor_order=w.taylor_order if taylor_order is None else taylor_order,
               precision=precision, tape_steps=tape_steps, overlap=overlap, stream=stream)
    v = torch.from_numpy(np.ascontiguousarray(w.v_ext)).to("cuda")
    s.set_potentials(v_ext=v, B0=w.bfield.B0, pulses=w.bfield.pulses)
    if getattr(w, "laser", None):
        s.set_laser(w.laser)
        s.set_laser_gauge(getattr(w, "laser_gauge", "length"))
    if getattr(w, "kvec", None) is not None:
        s.set_kpoints(w.kvec)
    torch.cuda.synchronize()
    return s


def states_to_device(psi0: np.ndarray, precision: int = NCT_FP64):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(psi0))
    if precision == NCT_FP32_MIXED:
        t = t.to(torch.complex64)
    return t.to("cuda").contiguous()


def version() -> str:
    return lib().nct_version().decode()


def _pulses_with(pulses, theta):
    import dataclasses
    k = len(pulses)
    out = []
    for i, p in enumerate(pulses):
        out.append(dataclasses.replace(p, A=float(theta[i]), omega=float(theta[k + i])))
    return out


def _segment_adjoint_recompute(s, psi, t_c, n, dt, lam, grad, sub_every):
    """Reverse sweep over one checkpointed segment of n steps without a multi-step tape: the
    segment is re-run keeping its state every sub_every steps; each of those sub-segments is
    re-run keeping the state of every step; then nct_backward_step runs step by step in recompute
    mode (it re-runs its own step from psi_n with a one-step tape).  State sets held on the GPU:
    n / sub_every sub-checkpoints and sub_every step states."""
    subs = []
    t = t_c
    j0 = 0
    while j0 < n:
        m = min(sub_every, n - j0)
        subs.append((psi.clone(), t, m))
        if j0 + m < n:
            s.step(psi, t, m)
        t += m * dt
        j0 += m
    del psi
    while subs:
        psi_s, t_s, m = subs.pop()
        states = [psi_s]
        p = psi_s.clone()
        for j in range(m - 1):
            s.step(p, t_s + j * dt, 1)
            states.append(p.clone())
        del p
        for j in reversed(range(m)):
            s.backward_step(-1, states[j], t_s + j * dt, lam, lam, grad)
            states[j] = None
        del states, psi_s


def _make_pulse_mz():
    import torch

    class PulseMz(torch.autograd.Function):
        """L = M_z(t0 + nsteps dt) = int m_z dV as a function of the pulse parameters
        theta = (A_1..A_k, omega_1..omega_k) of the external field B_ext(t).

        forward: runs the trajectory with nct_step, keeping a copy of the states every
        checkpoint_every steps (in host memory when checkpoint_on_host).  backward: seeds
        lam = 2 dV f sigma_z psi_T (nct_magnetization_seed), then for each segment in reverse:
        * if the system's tape holds a whole segment (tape_steps >= checkpoint_every), re-runs it
          with the tape on (nct_step(tape=1)) and calls nct_backward_step step by step;
        * otherwise (systems too large for a multi-step tape) takes the two-level schedule of
          _segment_adjoint_recompute with sub-segments of sub_every steps (default about
          sqrt(checkpoint_every)).
        The library adds dL/dB . dB/dtheta into the gradient.  backward re-applies the field of its
        own forward call (theta and B0 are kept in ctx), so other forward calls on the same system
        in between (finite differences, line searches) do not change the gradient; the field the
        system held before backward is restored.  progress, if given, is called as
        progress(done_segments, total_segments) after each segment of the backward sweep.
        """

        @staticmethod
        def forward(ctx, theta, system, psi0, pulses, nsteps, checkpoint_every, t0=0.0,
                    B0=(0.0, 0.0, 0.0), checkpoint_on_host=False, sub_every=None, progress=None):
            th = theta.detach().cpu().double().numpy()
            system.set_potentials(B0=B0, pulses=_pulses_with(pulses, th))
            dt = float(system.params.dt)
            psi = psi0.detach().clone()
            ckpts = []
            t = float(t0)
            done = 0
            while done < nsteps:
                n = min(int(checkpoint_every), nsteps - done)
                ckpts.append((psi.to("cpu") if checkpoint_on_host else psi.clone(), t, n))
                system.step(psi, t, n)
                t += n * dt
                done += n
            tot = system.density_magnetization(psi, t, totals=True)
            ctx.system = system
            ctx.ckpts = ckpts
            ctx.psi_final = psi
            ctx.npar = 2 * len(pulses)
            ctx.field = (tuple(float(v) for v in B0), _pulses_with(pulses, th))
            ctx.sub_every = int(sub_every) if sub_every else max(1, int(round(math.sqrt(checkpoint_every))))
            ctx.progress = progress
            return torch.tensor(float(tot[3]), dtype=torch.float64)

        @staticmethod
        def backward(ctx, gout):
            s = ctx.system
            dt = float(s.params.dt)
            held = s.bfield_args
            s.set_potentials(B0=ctx.field[0], pulses=ctx.field[1])
            try:
                lam = torch.empty_like(ctx.psi_final)
                s.magnetization_seed(ctx.psi_final, (0.0, 0.0, 1.0), lam)
                grad = np.zeros(ctx.npar)
                taped = int(s.params.tape_steps) >= max(n for _, _, n in ctx.ckpts)
                total = len(ctx.ckpts)
                for k, (psi_c, t_c, n) in enumerate(reversed(ctx.ckpts)):
                    psi = psi_c.to(ctx.psi_final.device).clone()
                    if taped:
                        s.step(psi, t_c, n, tape=True)
                        for j in reversed(range(n)):
                            s.backward_step(j, None, t_c + j * dt, lam, lam, grad)
                    else:
                        _segment_adjoint_recompute(s, psi, t_c, n, dt, lam, grad, ctx.sub_every)
                    del psi
                    if ctx.progress is not None:
                        ctx.progress(k + 1, total)
            finally:
                s.set_potentials(B0=held[0], pulses=held[1])
            g = torch.from_numpy(grad * float(gout))
            return g, None, None, None, None, None, None, None, None, None, None

    return PulseMz


_PULSE_MZ = None


def pulse_mz(theta, system, psi0, pulses, nsteps, checkpoint_every, t0=0.0, B0=(0.0, 0.0, 0.0),
             checkpoint_on_host=False, sub_every=None, progress=None):
    """Differentiable final M_z with respect to the pulse parameters (see PulseMz)."""
    global _PULSE_MZ
    if _PULSE_MZ is None:
        _PULSE_MZ = _make_pulse_mz()
    return _PULSE_MZ.apply(theta, system, psi0, pulses, nsteps, checkpoint_every, t0, B0,
                           checkpoint_on_host, sub_every, progress)
