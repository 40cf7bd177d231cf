"""Seeded synthetic inputs for the non-collinear real-time TDDFT step.

This module only draws random numbers and shapes them into the inputs of a
time step: the grid, the initial two-component spinor states, atom positions,
the external (ionic) local potential as a real-space field, the projector
channel table and the magnetic-field pulse parameters.  It holds none of the
method's arithmetic (no Hamiltonian, density, exchange-correlation, Hartree,
projector or propagator code): the CPU oracle and the HIP library each build
those from these inputs on their own.

The paper's systems (Fe clusters, bcc Fe, NiO; Results section) need real
pseudopotentials and ground states that are not available here, so seeded
synthetic systems with the same shapes stand in for them:

* states: complex Gaussian noise per grid point, smoothed in G space by
  exp(-|G|^2 sigma^2 / 2) (sigma = 1 bohr), orthonormalised in FP64 with the
  inner product  <a|b> = dV sum_r sum_s a*(r,s) b(r,s);
* tiny case: both spinor components random; other cases: psi_i = phi_i x chi,
  chi = (cos 15deg, sin 15deg) for 3S/4 states (spin along
  (sin 30deg, 0, cos 30deg)) and chi = (-sin 15deg, cos 15deg) for S/4 states,
  so the net moment is S/2 tilted 30 degrees from z;
* atoms: uniform positions with minimum-image separation >= 5 bohr, or a
  jittered bcc lattice for the solid-like case;
* local potential: a periodic sum of attractive Gaussians
  -D exp(-|r-R|^2 / 2w^2), depth D ~ U[1,3] Ha, width w = 1 bohr;
* projector channels: s, p1/2, p3/2, d3/2, d5/2 (18 projectors per atom),
  Gaussian radial form, with spin-orbit strength lambda_so entering the
  channel energies as E_lj = E_l + lambda_so <L.S>_j  (Eq. for the
  pseudo spin-orbit term in the spin-orbit implementation section).
"""
from __future__ import annotations

import dataclasses
import math
import os
from concurrent.futures import ThreadPoolExecutor
from typing import List, Optional, Sequence, Tuple

import numpy as np
import scipy.fft as sfft
import scipy.linalg

SEED_BASE = 21908


@dataclasses.dataclass
class Channel:
    """One Kleinman-Bylander channel (l, j = twoj/2) with energy and radial width."""
    l: int
    twoj: int
    energy: float
    rc: float


@dataclasses.dataclass
class Pulse:
    """Circularly polarised Gaussian pulse.

    B(t) = A exp(-(t-t0)^2 / (2 tau^2)) [cos(w (t-t0) + phase) e1 + sin(w (t-t0) + phase) e2]
    """
    A: float
    omega: float
    t0: float
    tau: float
    phase: float = 0.0
    e1: Tuple[float, float, float] = (1.0, 0.0, 0.0)
    e2: Tuple[float, float, float] = (0.0, 1.0, 0.0)


@dataclasses.dataclass
class BField:
    B0: Tuple[float, float, float] = (0.0, 0.0, 0.0)
    pulses: List[Pulse] = dataclasses.field(default_factory=list)


@dataclasses.dataclass
class LaserPulse:
    """Uniform electric pulse (optical excitation, magnetic component neglected).

    E(t) = A pol cos(omega t + phase) exp(-(t-t0)^2 / (2 tau^2))
    """
    A: float
    omega: float
    t0: float
    tau: float
    phase: float = 0.0
    pol: Tuple[float, float, float] = (0.0, 0.0, 1.0)


# unit conversions for the laser parameters quoted in eV and fs
EV_HA = 1.0 / 27.211386245988
FS_AU = 41.341373335


@dataclasses.dataclass
class Workload:
    name: str
    n: Tuple[int, int, int]
    L: Tuple[float, float, float]
    nstates: int
    occ: np.ndarray                 # [S] float64
    positions: np.ndarray           # [natoms, 3] float64 (bohr)
    depths: np.ndarray              # [natoms] Gaussian local-potential depths (Ha)
    widths: np.ndarray              # [natoms] Gaussian widths (bohr)
    v_ext: np.ndarray               # [nx, ny, nz] float64 (Ha)
    channels: List[Channel]
    r_sphere: float
    psi0: np.ndarray                # [S, 2, nx, ny, nz] complex128
    bfield: BField
    dt: float
    nsteps: int
    xc: int = 1
    hartree: int = 1
    m_threshold: float = 1e-12
    taylor_order: int = 4
    checkpoint_every: int = 0
    laser: List[LaserPulse] = dataclasses.field(default_factory=list)
    kvec: Optional[np.ndarray] = None   # [S, 3] Bloch vector of each state (None: Gamma only)
    laser_gauge: str = "length"         # "length" (isolated) or "velocity" (periodic)

    @property
    def natoms(self) -> int:
        return int(self.positions.shape[0])

    @property
    def npoints(self) -> int:
        return int(self.n[0] * self.n[1] * self.n[2])


def kb_channels(lambda_so: float = 0.05, e_s: float = 1.0, e_p: float = 0.5,
                e_d: float = -0.3, rc: float = 0.7) -> List[Channel]:
    """The 18-projector channel table: s, p1/2, p3/2, d3/2, d5/2.

    <L.S> = l/2 for j = l+1/2 and -(l+1)/2 for j = l-1/2, so that
    2/(2l+1) (E_{l+1/2} - E_{l-1/2}) = lambda_so.
    """
    def e(l, twoj, base):
        ls = l / 2.0 if twoj == 2 * l + 1 else -(l + 1) / 2.0
        return base + lambda_so * ls
    return [Channel(0, 1, e_s, rc),
            Channel(1, 1, e(1, 1, e_p), rc), Channel(1, 3, e(1, 3, e_p), rc),
            Channel(2, 3, e(2, 3, e_d), rc), Channel(2, 5, e(2, 5, e_d), rc)]


def _rngs(case: int):
    ss = np.random.SeedSequence(SEED_BASE + 100 * case).spawn(4)
    return [np.random.default_rng(s) for s in ss]


def _periodic_gauss_1d(x: np.ndarray, c: float, w: float, L: float) -> np.ndarray:
    """Sum over periodic images of exp(-(x - c - kL)^2 / (2 w^2))."""
    out = np.zeros_like(x)
    kmax = int(math.ceil(12.0 * w / L)) + 1
    for k in range(-kmax, kmax + 1):
        out += np.exp(-((x - c - k * L) ** 2) / (2.0 * w * w))
    return out


def gaussian_local_potential(n, L, positions, depths, widths) -> np.ndarray:
    """Real-space external potential v(r) = -sum_a D_a sum_images exp(-|r-R_a|^2/2w_a^2).

    The image sum of a Gaussian factorises over the three axes of an
    orthorhombic cell, so it is built from 1D periodised Gaussians.
    """
    axes = [np.arange(n[d]) * (L[d] / n[d]) for d in range(3)]
    v = np.zeros(tuple(n), dtype=np.float64)
    for R, D, w in zip(positions, depths, widths):
        gx = _periodic_gauss_1d(axes[0], R[0], w, L[0])
        gy = _periodic_gauss_1d(axes[1], R[1], w, L[1])
        gz = _periodic_gauss_1d(axes[2], R[2], w, L[2])
        v -= D * gx[:, None, None] * gy[None, :, None] * gz[None, None, :]
    return v


def _workers() -> int:
    """Host threads for input generation (the cores this process may run on)."""
    try:
        return max(1, len(os.sched_getaffinity(0)))
    except AttributeError:  # pragma: no cover - non-Linux hosts
        return max(1, os.cpu_count() or 1)


def _smooth_noise(rng, count: int, n, L, sigma: float = 1.0) -> np.ndarray:
    """Complex normal noise on the grid, smoothed by exp(-|G|^2 sigma^2/2).

    Row i draws its 2N normals (interleaved real and imaginary parts) from its own child generator
    rng.spawn(count)[i], so rows can be drawn on several threads with a result that does not
    depend on the thread count."""
    N = int(np.prod(n))
    z = np.empty((count, N), dtype=np.complex128)
    zr = z.view(np.float64)                       # [count, 2N]: re, im, re, im, ...
    kids = rng.spawn(count)

    def draw(i):
        kids[i].standard_normal(out=zr[i])

    with ThreadPoolExecutor(max_workers=_workers()) as ex:
        list(ex.map(draw, range(count)))
    z = z.reshape((count,) + tuple(n))
    g2 = np.zeros(tuple(n))
    for d in range(3):
        g = 2.0 * np.pi * np.fft.fftfreq(n[d], d=L[d] / n[d])
        sh = [1, 1, 1]
        sh[d] = n[d]
        g2 = g2 + (g ** 2).reshape(sh)
    filt = np.exp(-0.5 * g2 * sigma * sigma)
    w = _workers()
    z = sfft.fftn(z, axes=(-3, -2, -1), workers=w, overwrite_x=True)
    z *= filt
    return sfft.ifftn(z, axes=(-3, -2, -1), workers=w, overwrite_x=True)


def _orthonormal_columns(vecs: np.ndarray, dV: float) -> np.ndarray:
    """Orthonormalise the rows of vecs [count, M] under <a|b> = dV sum a* b in FP64.

    Cholesky QR applied twice (Fukaya, Nakatsukasa, Yanagisawa and Yamamoto, "CholeskyQR2",
    2014): with G = dV conj(Z) Z^T = L L^H, the rows of conj(L)^-1 Z are orthonormal; the
    second pass removes the rounding left by the first.  The Cholesky factor has a positive
    real diagonal, so the result is unique (no sign or phase convention of a library)."""
    q = np.ascontiguousarray(vecs, dtype=np.complex128)
    for _ in range(2):
        G = dV * (q.conj() @ q.T)
        Lc = scipy.linalg.cholesky(G, lower=True)
        q = scipy.linalg.solve_triangular(Lc.conj(), q, lower=True, overwrite_b=True,
                                          check_finite=False)
    return q


def random_spinors_full(rng, S: int, n, L) -> np.ndarray:
    """Both spinor components random (tiny case)."""
    N = int(np.prod(n))
    dV = float(np.prod(L)) / N
    z = _smooth_noise(rng, 2 * S, n, L).reshape(S, 2 * N)
    q = _orthonormal_columns(z, dV)
    return q.reshape((S, 2) + tuple(n))


def tilted_product_spinors(rng, S: int, n, L, tilt_deg: float = 30.0) -> np.ndarray:
    """psi_i = phi_i (x) chi_{+/-}, 3S/4 along n = (sin t, 0, cos t), S/4 along -n."""
    N = int(np.prod(n))
    dV = float(np.prod(L)) / N
    z = _smooth_noise(rng, S, n, L).reshape(S, N)
    phi = _orthonormal_columns(z, dV).reshape((S,) + tuple(n))
    h = math.radians(tilt_deg) / 2.0
    chi_p = np.array([math.cos(h), math.sin(h)])
    chi_m = np.array([-math.sin(h), math.cos(h)])
    nplus = (3 * S + 3) // 4
    psi = np.empty((S, 2) + tuple(n), dtype=np.complex128)
    for i in range(S):
        chi = chi_p if i < nplus else chi_m
        psi[i, 0] = chi[0] * phi[i]
        psi[i, 1] = chi[1] * phi[i]
    return psi


def localized_product_spinors(rng, S: int, n, L, sigma_env: float, tilt_deg: float = 30.0) -> np.ndarray:
    """Like tilted_product_spinors, with every orbital multiplied by a Gaussian envelope of width
    sigma_env about the cell centre before orthonormalisation: a cluster isolated in its box."""
    N = int(np.prod(n))
    dV = float(np.prod(L)) / N
    env = np.ones(tuple(n))
    for d in range(3):
        x = np.arange(n[d]) * (L[d] / n[d]) - 0.5 * L[d]
        sh = [1, 1, 1]
        sh[d] = n[d]
        env = env * np.exp(-0.5 * (x / sigma_env) ** 2).reshape(sh)
    z = (_smooth_noise(rng, S, n, L) * env[None]).reshape(S, N)
    phi = _orthonormal_columns(z, dV).reshape((S,) + tuple(n))
    h = math.radians(tilt_deg) / 2.0
    chi_p = np.array([math.cos(h), math.sin(h)])
    chi_m = np.array([-math.sin(h), math.cos(h)])
    nplus = (3 * S + 3) // 4
    psi = np.empty((S, 2) + tuple(n), dtype=np.complex128)
    for i in range(S):
        chi = chi_p if i < nplus else chi_m
        psi[i, 0] = chi[0] * phi[i]
        psi[i, 1] = chi[1] * phi[i]
    return psi


def localized_full_spinors(rng, S: int, n, L, sigma_env: float) -> np.ndarray:
    """Both spinor components random, in a Gaussian envelope of width sigma_env about the cell
    centre, orthonormalised in FP64: generic local polarisation (0 < zeta < 1) with density tails
    that reach large rs."""
    N = int(np.prod(n))
    dV = float(np.prod(L)) / N
    env = np.ones(tuple(n))
    for d in range(3):
        x = np.arange(n[d]) * (L[d] / n[d]) - 0.5 * L[d]
        sh = [1, 1, 1]
        sh[d] = n[d]
        env = env * np.exp(-0.5 * (x / sigma_env) ** 2).reshape(sh)
    z = (_smooth_noise(rng, 2 * S, n, L) * env[None]).reshape(S, 2 * N)
    return _orthonormal_columns(z, dV).reshape((S, 2) + tuple(n))


def central_positions(rng, natoms: int, L, radius: float, min_sep: float) -> np.ndarray:
    """Atoms uniform in a ball of the given radius about the cell centre, pairwise >= min_sep."""
    c = 0.5 * np.asarray(L, dtype=np.float64)
    pos: List[np.ndarray] = []
    tries = 0
    while len(pos) < natoms:
        tries += 1
        if tries > 100000:
            raise RuntimeError("could not place atoms with the requested separation")
        u = rng.uniform(-1.0, 1.0, 3)
        if np.dot(u, u) > 1.0:
            continue
        p = c + radius * u
        if all(np.linalg.norm(p - q) >= min_sep for q in pos):
            pos.append(p)
    return np.array(pos).reshape(natoms, 3)


def separated_positions(rng, natoms: int, L, min_sep: float = 5.0) -> np.ndarray:
    L = np.asarray(L, dtype=np.float64)
    pos: List[np.ndarray] = []
    tries = 0
    while len(pos) < natoms:
        tries += 1
        if tries > 100000:
            raise RuntimeError("could not place atoms with the requested separation")
        p = rng.uniform(0.0, 1.0, 3) * L
        ok = True
        for q in pos:
            d = p - q
            d -= L * np.round(d / L)
            if np.linalg.norm(d) < min_sep:
                ok = False
                break
        if ok:
            pos.append(p)
    return np.array(pos).reshape(natoms, 3)


def bcc_positions(rng, L: float, cells: int = 2, jitter: float = 0.05) -> np.ndarray:
    a = L / cells
    pos = []
    for i in range(cells):
        for j in range(cells):
            for k in range(cells):
                base = np.array([i, j, k], dtype=np.float64) * a
                pos.append(base)
                pos.append(base + 0.5 * a)
    pos = np.array(pos) + rng.normal(0.0, jitter, (len(pos), 3))
    return np.mod(pos, L)


def monkhorst_pack(L, grid=(2, 2, 2)) -> np.ndarray:
    """Monkhorst-Pack k-points of an orthorhombic cell: k_d = (2 pi / L_d)((2 i + 1 - q_d)/(2 q_d))."""
    axes = [2.0 * math.pi / L[d] * (2.0 * np.arange(grid[d]) + 1.0 - grid[d]) / (2.0 * grid[d])
            for d in range(3)]
    return np.array([[a, b, c] for a in axes[0] for b in axes[1] for c in axes[2]])


@dataclasses.dataclass
class AtomDensity:
    """Atomic charge Z in a Gaussian of width sigma and the atom's moment (initial spin density)."""
    Z: float
    sigma: float
    moment: Tuple[float, float, float] = (0.0, 0.0, 0.0)


def atom_densities(w, Z: float = 4.0, sigma: float = 1.0, tilt_deg: float = 30.0):
    """Initial atomic data for a workload: the states' electrons shared over the atoms, each with a
    moment of half its charge along the 30-degree tilt of the initial spinors."""
    na = max(len(w.positions), 1)
    Zs = float(np.sum(w.occ)) / na if Z is None else Z
    t = math.radians(tilt_deg)
    mom = (0.5 * Zs * math.sin(t), 0.0, 0.5 * Zs * math.cos(t))
    return [AtomDensity(Zs, sigma, mom) for _ in range(na)]


def circular_pulses(t_centers: Sequence[float], omegas: Sequence[float], A: float, tau: float):
    return [Pulse(A=A, omega=w, t0=t, tau=tau) for t, w in zip(t_centers, omegas)]


def make_system(n=(8, 8, 8), L=(6.0, 6.0, 6.0), nstates=4, natoms=0, case=7,
                projectors=True, lambda_so=0.05, r_sphere=2.5, rc=0.7,
                full_spinors=True, bfield: Optional[BField] = None, dt=0.05,
                nsteps=4, xc=1, hartree=1, min_sep=None, name="custom",
                depth_range=(1.0, 3.0), width=1.0, taylor_order=4,
                laser: Optional[List[LaserPulse]] = None, localized: Optional[float] = None,
                localized_full: bool = False) -> Workload:
    """A seeded system of arbitrary (small) shape, for tests."""
    r_pos, r_depth, r_states, _ = _rngs(case)
    n = tuple(int(v) for v in n)
    L = tuple(float(v) for v in L)
    if natoms > 0 and localized is not None:
        sep = min_sep if min_sep is not None else min(4.2, 0.3 * min(L))
        pos = central_positions(r_pos, natoms, L, 0.2 * min(L), sep)
    elif natoms > 0:
        sep = min_sep if min_sep is not None else min(5.0, 0.45 * min(L))
        pos = separated_positions(r_pos, natoms, L, sep)
    else:
        pos = np.zeros((0, 3))
    depths = r_depth.uniform(depth_range[0], depth_range[1], max(natoms, 0))
    widths = np.full(max(natoms, 0), width)
    v_ext = gaussian_local_potential(n, L, pos, depths, widths)
    if localized is not None and localized_full:
        psi0 = localized_full_spinors(r_states, nstates, n, L, localized)
    elif localized is not None:
        psi0 = localized_product_spinors(r_states, nstates, n, L, localized)
    elif full_spinors:
        psi0 = random_spinors_full(r_states, nstates, n, L)
    else:
        psi0 = tilted_product_spinors(r_states, nstates, n, L)
    chans = kb_channels(lambda_so=lambda_so, rc=rc) if (projectors and natoms > 0) else []
    return Workload(name=name, n=n, L=L, nstates=nstates, occ=np.ones(nstates),
                    positions=pos, depths=depths, widths=widths, v_ext=v_ext,
                    channels=chans, r_sphere=r_sphere, psi0=psi0,
                    bfield=bfield if bfield is not None else BField(),
                    dt=dt, nsteps=nsteps, xc=xc, hartree=hartree,
                    taylor_order=taylor_order, laser=list(laser) if laser else [])


def workload(case: int) -> Workload:
    """The five benchmark-shaped systems (0-indexed).

    0 tiny 16^3 x 8 spinors, 4 Gaussians, no projectors, B = (0,0,0.01), 20 steps
    1 magnetic-cluster-like 48^3 x 64, 4 atoms x 18 KB+SOC projectors, field free, 200 steps
    2 solid-like 64^3 x 256, 16 atoms bcc 2x2x2 (+0.05 bohr jitter), circular pulse, 1000 steps
    3 gradient case 32^3 x 32, 2 atoms, 4 circular pulse components, 200 steps, checkpoint 20
    4 large 96^3 x 512, 32 atoms, 4 circular pulse components, 500 steps, checkpoint 25
    6 k-point solid: the solid-like system of case 2 sampled on a 2x2x2 Monkhorst-Pack grid,
      8 k-points x 32 states (weights 1/8 in the occupations), the same 256 states in total
    5 laser-driven cluster 48^3 x 64, 4 atoms within 5 bohr of the centre, states in a Gaussian
      envelope (sigma 3.5 bohr) about the centre, z-polarised electric pulse A = 1 a.u.,
      omega = 10 eV, t0 = 0.1 fs, tau = 0.5 fs (the parameters of the paper's cluster runs),
      200 steps
    7 reduced system that keeps every term of the step, for long trajectories against the oracle:
      16^3 grid (h = 0.42 bohr, L = 6.72), 8 spinor states tilted as in cases 1-4, 2 atoms x 18
      KB+SOC projectors (minimum-image separation >= 4 bohr), Gaussian local potential, exchange
      + Hartree, the circular pulse of case 2 (A = 0.005, omega = 0.5, t0 = 25, tau = 5), 1000
      steps of dt = 0.05 (the pulse's whole envelope)
    """
    r_pos, r_depth, r_states, _r_jit = _rngs(case)
    if case == 7:
        n, L, S, natoms = (16, 16, 16), (6.72,) * 3, 8, 2
        pos = separated_positions(r_pos, natoms, L, 4.0)
        depths = r_depth.uniform(1.0, 3.0, natoms)
        widths = np.ones(natoms)
        v_ext = gaussian_local_potential(n, L, pos, depths, widths)
        psi0 = tilted_product_spinors(r_states, S, n, L)
        bf = BField(pulses=[Pulse(A=0.005, omega=0.5, t0=25.0, tau=5.0)])
        return Workload("reduced-16^3x8-2x18KB-pulse", n, L, S, np.ones(S), pos, depths, widths,
                        v_ext, kb_channels(), 2.5, psi0, bf, 0.05, 1000)
    if case == 6:
        w = workload(2)
        nk, per = 8, 32
        w.name = "kpoints-solid-64^3x8kx32-16x18KB"
        w.kvec = np.repeat(monkhorst_pack(w.L), per, axis=0)
        w.occ = np.full(nk * per, 1.0 / nk)
        return w
    if case == 5:
        n, L, S, natoms = (48, 48, 48), (20.0,) * 3, 64, 4
        pos = central_positions(r_pos, natoms, L, 5.0, 4.2)
        depths = r_depth.uniform(1.0, 3.0, natoms)
        widths = np.ones(natoms)
        v_ext = gaussian_local_potential(n, L, pos, depths, widths)
        psi0 = localized_product_spinors(r_states, S, n, L, 3.5)
        laser = [LaserPulse(A=1.0, omega=10.0 * EV_HA, t0=0.1 * FS_AU, tau=0.5 * FS_AU)]
        return Workload("laser-cluster-48^3x64-4x18KB", n, L, S, np.ones(S), pos, depths, widths,
                        v_ext, kb_channels(), 2.5, psi0, BField(), 0.05, 200, laser=laser)
    if case == 0:
        n, L, S, natoms = (16, 16, 16), (10.0,) * 3, 8, 4
        pos = separated_positions(r_pos, natoms, L, 2.0)
        depths = r_depth.uniform(1.0, 3.0, natoms)
        widths = np.ones(natoms)
        v_ext = gaussian_local_potential(n, L, pos, depths, widths)
        psi0 = random_spinors_full(r_states, S, n, L)
        return Workload("tiny-16^3x8-fp64", n, L, S, np.ones(S), pos, depths, widths,
                        v_ext, [], 2.5, psi0, BField(B0=(0.0, 0.0, 0.01)), 0.05, 20)
    if case == 1:
        n, L, S, natoms = (48, 48, 48), (20.0,) * 3, 64, 4
        pos = separated_positions(r_pos, natoms, L, 5.0)
        bf = BField()
        nsteps, ck = 200, 0
    elif case == 2:
        n, L, S = (64, 64, 64), (26.88,) * 3, 256
        pos = bcc_positions(_r_jit, L[0], 2, 0.05)
        natoms = pos.shape[0]
        bf = BField(pulses=[Pulse(A=0.005, omega=0.5, t0=25.0, tau=5.0)])
        nsteps, ck = 1000, 0
    elif case == 3:
        n, L, S, natoms = (32, 32, 32), (13.44,) * 3, 32, 2
        pos = separated_positions(r_pos, natoms, L, 5.0)
        bf = BField(pulses=circular_pulses([1.25, 3.75, 6.25, 8.75], [0.25, 0.5, 0.75, 1.0], 0.01, 1.0))
        nsteps, ck = 200, 20
    elif case == 4:
        n, L, S, natoms = (96, 96, 96), (40.32,) * 3, 512, 32
        pos = separated_positions(r_pos, natoms, L, 5.0)
        bf = BField(pulses=circular_pulses([(k - 0.5) * 6.25 for k in range(1, 5)],
                                           [0.25, 0.5, 0.75, 1.0], 0.01, 2.5))
        nsteps, ck = 500, 25
    else:
        raise ValueError("unknown case %d" % case)
    depths = r_depth.uniform(1.0, 3.0, natoms)
    widths = np.ones(natoms)
    v_ext = gaussian_local_potential(n, L, pos, depths, widths)
    psi0 = tilted_product_spinors(r_states, S, n, L)
    names = {1: "cluster-48^3x64-4x18KB", 2: "solid-64^3x256-16x18KB",
             3: "grad-32^3x32-2x18KB", 4: "large-96^3x512-32x18KB"}
    w = Workload(names[case], n, L, S, np.ones(S), pos, depths, widths, v_ext,
                 kb_channels(), 2.5, psi0, bf, 0.05, nsteps)
    w.checkpoint_every = ck
    return w
