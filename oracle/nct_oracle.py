"""Plain FP64 CPU oracle for one non-collinear real-time TDDFT time step.

TEST INFRASTRUCTURE ONLY.  Only tests/, __graft_entry__.smoke() and the
cpu_baseline leg of bench.py may import this module.  It shares no code with
the HIP library or its Python binding; the only common ingredient is the
seeded input generator (paper_2506_21908_amd.inputs), which holds none of the
method's arithmetic.

Everything here is slow on purpose: whole-array numpy with complex128/float64,
library FFTs (scipy.fft) as the only primitive, explicit sums in the order the
equations state them.  Atomic units throughout, mu_B = 1/2 (Sec. 2.1).

Sources (paper arXiv 2506.21908, "Spin non-collinear real-time TDDFT ... INQ"):
  * non-collinear Kohn-Sham Hamiltonian          Eq. (HNC-SDFT), Eq. (TDSDFT)
  * spin-density matrix and its 4-vector         Sec. 3.1, Eqs. (rho1-3), (density4)
  * locally collinear adiabatic LSDA             Eqs. (LC+ALDA2), (LC+ALDA), Sec. 3.3
  * Zeeman term mu_B sigma.b_ext                 Eq. (zeeman_potential), Sec. 3.4
  * Kleinman-Bylander + spin-orbit projectors    Eqs. (Vps), (Vps-soc), spinor harmonics, Sec. 3.5
  * Hartree potential                            Eq. (KSpot)
  * uniform electric (laser) pulse               Sec. 4.7, pulse profile of Figs. (fe2-laser), (fe6-laser)
  * initial spin-density matrix (DMInitialization)  Sec. 3.2 and its algorithm figure (alg:mag_init)
  * ground state by self-consistent imaginary-time propagation with Cholesky orthonormalisation
    (the paper's ground-state solver is not specified; reading in the design notes)
  * k-point sampling (state index i = (n, k))    Sec. 2.1 (Eq. KSDFT), Sec. 5; states are held as
    the periodic parts u of psi = exp(i k.r) u, kinetic 1/2 |G + k|^2, projector
    Bloch phases exp(-/+ i k.d) on the sphere points; k-weights enter the occupations
The paper names no propagator, Taylor order, Poisson solver or LDA
parametrisation; the readings taken here are:
  * propagator: enforced time-reversal symmetry (ETRS) with a truncated Taylor
    exponential of order K (default 4), predictor built from a second
    half-step of the same exponential;
  * exchange-correlation: Slater exchange (spin-scaled), locally collinear;
    b_xc = 0 where |m| < threshold; with xc = 2 also the Perdew-Wang 1992
    (PW92) LSDA correlation in the same locally collinear form;
  * Hartree: FFT Poisson solve with the G = 0 term dropped;
  * projectors: radial form r^l exp(-r^2/2rc^2) cut at r_sphere, normalised by
    the continuum radial integral; channel energies absorb the KB denominator;
  * laser: length gauge for an isolated system, v_E(r, t) = E(t).(r - c) with c the
    cell centre (potential energy of a charge -1 in the field E), evaluated like
    B(t): at t_n for H_n and t_{n+1} for H~; its energy int v_E n is part of E_loc.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Callable, List, Optional, Sequence

import numpy as np
import scipy.fft as sfft
from scipy.special import gamma as _gamma, gammainc as _gammainc

MU_B = 0.5           # Bohr magneton in atomic units (Sec. 2.1)
SLATER_C = (6.0 / math.pi) ** (1.0 / 3.0)
FFT_WORKERS = -1


# ----------------------------------------------------------------------------
# grid
# ----------------------------------------------------------------------------
@dataclass
class Grid:
    n: tuple
    L: tuple

    @property
    def N(self) -> int:
        return int(self.n[0] * self.n[1] * self.n[2])

    @property
    def volume(self) -> float:
        return float(self.L[0] * self.L[1] * self.L[2])

    @property
    def dV(self) -> float:
        return self.volume / self.N

    def axis(self, d: int) -> np.ndarray:
        return np.arange(self.n[d]) * (self.L[d] / self.n[d])

    def gvec(self, d: int) -> np.ndarray:
        """G_d = 2 pi fftfreq(n_d, h_d): the plane-wave basis of the periodic cell."""
        return 2.0 * math.pi * np.fft.fftfreq(self.n[d], d=self.L[d] / self.n[d])

    def g2(self) -> np.ndarray:
        gx, gy, gz = self.gvec(0), self.gvec(1), self.gvec(2)
        return gx[:, None, None] ** 2 + gy[None, :, None] ** 2 + gz[None, None, :] ** 2


def fft3(f):
    return sfft.fftn(f, axes=(-3, -2, -1), workers=FFT_WORKERS)


def ifft3(f):
    return sfft.ifftn(f, axes=(-3, -2, -1), workers=FFT_WORKERS)


# ----------------------------------------------------------------------------
# kinetic energy:  -1/2 nabla^2  is  1/2 |G|^2  in the plane-wave basis (Eq. TDSDFT)
# ----------------------------------------------------------------------------
def kinetic(psi: np.ndarray, grid: Grid, kvec: Optional[np.ndarray] = None) -> np.ndarray:
    """T psi = IFFT(1/2 |G|^2 FFT psi); with Bloch vectors kvec[S, 3] (psi holding the periodic
    parts u_i of psi_i = exp(i k_i.r) u_i) the factor is 1/2 |G + k_i|^2."""
    if kvec is None:
        return ifft3(0.5 * grid.g2() * fft3(psi))
    out = np.empty_like(psi)
    G = [grid.gvec(d) for d in range(3)]
    for i in range(psi.shape[0]):
        k = kvec[i]
        g2 = ((G[0] + k[0])[:, None, None] ** 2 + (G[1] + k[1])[None, :, None] ** 2
              + (G[2] + k[2])[None, None, :] ** 2)
        out[i] = ifft3(0.5 * g2 * fft3(psi[i]))
    return out


# ----------------------------------------------------------------------------
# spin-density matrix (Sec. 3.1)
# ----------------------------------------------------------------------------
def spin_density(psi: np.ndarray, occ: np.ndarray) -> np.ndarray:
    """rho_v = {rho_uu, rho_dd, Re rho_ud, Im rho_ud},  rho_ud = sum_i f_i psi_iu psi_id^*.

    psi has shape [S, 2, nx, ny, nz]; component 0 is spin up, 1 spin down.
    """
    up, dn = psi[:, 0], psi[:, 1]
    f = occ.reshape(-1, 1, 1, 1)
    rho_uu = np.sum(f * (up * up.conj()).real, axis=0)
    rho_dd = np.sum(f * (dn * dn.conj()).real, axis=0)
    rho_ud = np.sum(f * up * dn.conj(), axis=0)
    return np.stack([rho_uu, rho_dd, rho_ud.real, rho_ud.imag])


def charge_and_magnetization(rho_v: np.ndarray):
    """n = rho_uu + rho_dd;  m_x = 2 Re rho_ud, m_y = -2 Im rho_ud, m_z = rho_uu - rho_dd (Eqs. rho1-3)."""
    n = rho_v[0] + rho_v[1]
    m = np.stack([2.0 * rho_v[2], -2.0 * rho_v[3], rho_v[0] - rho_v[1]])
    return n, m


# ----------------------------------------------------------------------------
# exchange: spin-polarised Slater exchange in the locally collinear form
# (Eqs. LC+ALDA2 and LC+ALDA; b = (v_up - v_dn)/2 as in Sec. 2.1)
# ----------------------------------------------------------------------------
def slater_exchange(n: np.ndarray, m: np.ndarray, thr: float = 1e-12):
    """Returns (vbar, b_xc[3], e_x) with e_x the exchange energy per volume.

    n_up,dn = (n +/- |m|)/2 (clamped at 0);
    e_x = -(3/4)(6/pi)^(1/3) (n_up^(4/3) + n_dn^(4/3));  v_s = -(6/pi)^(1/3) n_s^(1/3);
    vbar = (v_up + v_dn)/2;  b_xc = (v_up - v_dn)/2 * m/|m|,  zero where |m| < thr.
    """
    mu = np.sqrt(m[0] ** 2 + m[1] ** 2 + m[2] ** 2)
    nu = np.maximum(0.5 * (n + mu), 0.0)
    nd = np.maximum(0.5 * (n - mu), 0.0)
    v_up = -SLATER_C * np.cbrt(nu)
    v_dn = -SLATER_C * np.cbrt(nd)
    e_x = -0.75 * SLATER_C * (nu ** (4.0 / 3.0) + nd ** (4.0 / 3.0))
    vbar = 0.5 * (v_up + v_dn)
    bmag = 0.5 * (v_up - v_dn)
    big = mu >= thr
    safe_mu = np.where(big, mu, 1.0)
    bxc = np.where(big, bmag / safe_mu, 0.0) * m
    return vbar, bxc, e_x


# ----------------------------------------------------------------------------
# correlation: PW92 LSDA correlation (J. P. Perdew and Y. Wang, Phys. Rev. B 45,
# 13244 (1992)), applied in the locally collinear form of Eqs. LC+ALDA2 / LC+ALDA
# ----------------------------------------------------------------------------
# (A, alpha1, beta1, beta2, beta3, beta4) of G(rs) with p = 1, PW92 Table I
PW92_PARA = (0.031091, 0.21370, 7.5957, 3.5876, 1.6382, 0.49294)    # eps_c(rs, zeta = 0)
PW92_FERRO = (0.015545, 0.20548, 14.1189, 6.1977, 3.3662, 0.62517)  # eps_c(rs, zeta = 1)
PW92_ALPHA = (0.016887, 0.11125, 10.357, 3.6231, 0.88026, 0.49671)  # -alpha_c(rs)
PW92_FPP0 = 1.709921                                                # f''(0)
PW92_NMIN = 1e-30


def pw92_G(rs, par):
    """G = -2A(1 + a1 rs) ln[1 + 1/(2A(b1 rs^1/2 + b2 rs + b3 rs^3/2 + b4 rs^2))] and dG/drs."""
    A, a1, b1, b2, b3, b4 = par
    srs = np.sqrt(rs)
    q0 = -2.0 * A * (1.0 + a1 * rs)
    q1 = 2.0 * A * (b1 * srs + b2 * rs + b3 * rs * srs + b4 * rs * rs)
    q1p = A * (b1 / srs + 2.0 * b2 + 3.0 * b3 * srs + 4.0 * b4 * rs)
    lg = np.log1p(1.0 / q1)
    return q0 * lg, -2.0 * A * a1 * lg - q0 * q1p / (q1 * q1 + q1)


def _cbrt(x):
    """Real cube root; for the complex-step derivative (complex x near the positive real axis)
    the principal root, with a zero imaginary part where the real part is 0 (the derivative of
    the clamped channel is taken as 0 there)."""
    if not np.iscomplexobj(x):
        return np.cbrt(x)
    r = np.where(x.real > 0, x, 1.0) ** (1.0 / 3.0)
    return np.where(x.real > 0, r, 0.0)


def pw92_f(zeta):
    """Spin interpolation f(zeta) = [(1+z)^(4/3) + (1-z)^(4/3) - 2] / (2^(4/3) - 2) and f'."""
    d = 2.0 ** (4.0 / 3.0) - 2.0
    up, dn = 1.0 + zeta, 1.0 - zeta
    f = (up * _cbrt(up) + dn * _cbrt(dn) - 2.0) / d if np.iscomplexobj(zeta) else \
        (up ** (4.0 / 3.0) + dn ** (4.0 / 3.0) - 2.0) / d
    fp = (4.0 / 3.0) * (_cbrt(up) - _cbrt(dn)) / d
    return f, fp


def pw92_eps(rs, zeta):
    """eps_c(rs, zeta) of PW92 Eq. (8) with its derivatives (eps, d eps/d rs, d eps/d zeta)."""
    e0, d0 = pw92_G(rs, PW92_PARA)
    e1, d1 = pw92_G(rs, PW92_FERRO)
    ma, dma = pw92_G(rs, PW92_ALPHA)
    ac, dac = -ma, -dma
    f, fp = pw92_f(zeta)
    z4 = zeta ** 4
    eps = e0 + ac * f * (1.0 - z4) / PW92_FPP0 + (e1 - e0) * f * z4
    deps_rs = d0 * (1.0 - f * z4) + d1 * f * z4 + dac * f * (1.0 - z4) / PW92_FPP0
    deps_z = (4.0 * zeta ** 3 * f * (e1 - e0 - ac / PW92_FPP0)
              + fp * (z4 * (e1 - e0) + (1.0 - z4) * ac / PW92_FPP0))
    return eps, deps_rs, deps_z


def pw92_correlation(n: np.ndarray, m: np.ndarray, thr: float = 1e-12):
    """Returns (vbar_c, b_c[3], e_c) with e_c = n eps_c the correlation energy per volume.

    zeta = |m|/n (clamped to [0, 1]), rs = (3/(4 pi n))^(1/3);
    v_up/dn = eps - (rs/3) d eps/d rs - (zeta -/+ 1) d eps/d zeta;
    vbar_c = (v_up + v_dn)/2,  b_c = (v_up - v_dn)/2 m/|m| = (d eps/d zeta) m/|m|  (zero where
    |m| < thr);  nothing where n <= 1e-30.
    """
    mu = np.sqrt(m[0] ** 2 + m[1] ** 2 + m[2] ** 2)
    ok = n > PW92_NMIN
    ns = np.where(ok, n, 1.0)
    rs = np.cbrt(3.0 / (4.0 * math.pi * ns))
    zeta = np.clip(mu / ns, 0.0, 1.0)
    eps, drs, dz = pw92_eps(rs, zeta)
    vbar = np.where(ok, eps - rs / 3.0 * drs - zeta * dz, 0.0)
    big = ok & (mu >= thr)
    safe_mu = np.where(big, mu, 1.0)
    bc = np.where(big, dz / safe_mu, 0.0) * m
    ec = np.where(ok, n * eps, 0.0)
    return vbar, bc, ec


def pw92_correlation_jvp(n, m, dn, dm, thr: float = 1e-12):
    """Directional derivative of (vbar_c, b_c) of pw92_correlation along (dn, dm).

    In (n, |m|) the potentials are vbar_c(n, mu) and bmag_c(n, mu) = d eps/d zeta; their
    derivatives along (dn, dmu), dmu = mhat.dm, come from one complex-step evaluation
    (Squire & Trapp, SIAM Rev. 40, 110 (1998)): d f = Im f(n + i h dn, mu + i h dmu) / h,
    exact to rounding for these analytic formulas; the clamp of zeta to [0, 1] acts on the real
    part.  d b_c = d bmag mhat + bmag d mhat, as for exchange; b_c = 0 where |m| < thr (and there
    dmu = 0)."""
    mu = np.sqrt(m[0] ** 2 + m[1] ** 2 + m[2] ** 2)
    big = mu >= thr
    safe_mu = np.where(big, mu, 1.0)
    mhat = np.where(big, 1.0, 0.0) * m / safe_mu
    dmu = np.sum(mhat * dm, axis=0)
    ok = n > PW92_NMIN
    scale = max(float(np.max(np.abs(dn))), float(np.max(np.abs(dmu))), 1e-300)
    h = 1e-20 / scale
    nc = np.where(ok, n, 1.0) + 1j * h * np.where(ok, dn, 0.0)
    muc = mu + 1j * h * dmu
    rs = _cbrt(3.0 / (4.0 * math.pi * nc))
    zr = (muc / nc).real
    zeta = np.where(zr < 0.0, 0.0, np.where(zr > 1.0, 1.0, muc / nc))
    eps, drs, dz = pw92_eps(rs, zeta)
    vbar = eps - rs / 3.0 * drs - zeta * dz
    dvbar = np.where(ok, vbar.imag / h, 0.0)
    dbmag = np.where(ok & big, dz.imag / h, 0.0)
    bmag = np.where(ok & big, dz.real, 0.0)
    dmhat = np.where(big, 1.0, 0.0) * (dm - mhat * dmu) / safe_mu
    return dvbar, dbmag * mhat + bmag * dmhat


def slater_exchange_jvp(n, m, dn, dm, thr: float = 1e-12):
    """Directional derivative of (vbar, b_xc) along (dn, dm).

    With dmu = mhat.dm, dn_up = (dn + dmu)/2, dn_dn = (dn - dmu)/2,
    dv_s = -(1/3)(6/pi)^(1/3) n_s^(-2/3) dn_s (zero on a clamped channel),
    d vbar = (dv_up + dv_dn)/2,  d bmag = (dv_up - dv_dn)/2,
    d mhat = (dm - mhat (mhat.dm))/|m|,  d b_xc = d bmag mhat + bmag d mhat.
    """
    mu = np.sqrt(m[0] ** 2 + m[1] ** 2 + m[2] ** 2)
    big = mu >= thr
    safe_mu = np.where(big, mu, 1.0)
    mhat = np.where(big, 1.0, 0.0) * m / safe_mu
    dmu = np.sum(mhat * dm, axis=0)
    nu = 0.5 * (n + mu)
    nd = 0.5 * (n - mu)
    pos_u = nu > 0
    pos_d = nd > 0
    su = np.where(pos_u, nu, 1.0)
    sd = np.where(pos_d, nd, 1.0)
    dvu = np.where(pos_u, -(SLATER_C / 3.0) * su ** (-2.0 / 3.0), 0.0) * 0.5 * (dn + dmu)
    dvd = np.where(pos_d, -(SLATER_C / 3.0) * sd ** (-2.0 / 3.0), 0.0) * 0.5 * (dn - dmu)
    dvbar = 0.5 * (dvu + dvd)
    v_up = -SLATER_C * np.cbrt(np.maximum(nu, 0.0))
    v_dn = -SLATER_C * np.cbrt(np.maximum(nd, 0.0))
    bmag = 0.5 * (v_up - v_dn)
    dbmag = 0.5 * (dvu - dvd)
    dmhat = np.where(big, 1.0, 0.0) * (dm - mhat * dmu) / safe_mu
    dbxc = np.where(big, 1.0, 0.0) * (dbmag * mhat + bmag * dmhat)
    return dvbar, dbxc


# ----------------------------------------------------------------------------
# Hartree (Eq. KSpot): v_H(G) = 4 pi n(G) / |G|^2, G = 0 dropped
# ----------------------------------------------------------------------------
def hartree(n: np.ndarray, grid: Grid) -> np.ndarray:
    g2 = grid.g2()
    kern = np.zeros_like(g2)
    nz = g2 > 0
    kern[nz] = 4.0 * math.pi / g2[nz]
    return ifft3(kern * fft3(n)).real


# ----------------------------------------------------------------------------
# external magnetic field B(t) (Zeeman coupling only, Sec. 3.4)
# ----------------------------------------------------------------------------
@dataclass
class PulseSpec:
    A: float
    omega: float
    t0: float
    tau: float
    phase: float = 0.0
    e1: tuple = (1.0, 0.0, 0.0)
    e2: tuple = (0.0, 1.0, 0.0)


@dataclass
class FieldSpec:
    B0: tuple = (0.0, 0.0, 0.0)
    pulses: List[PulseSpec] = field(default_factory=list)

    def B(self, t: float) -> np.ndarray:
        out = np.array(self.B0, dtype=np.float64)
        for p in self.pulses:
            s = t - p.t0
            g = math.exp(-s * s / (2.0 * p.tau * p.tau))
            ph = p.omega * s + p.phase
            out = out + p.A * g * (math.cos(ph) * np.array(p.e1) + math.sin(ph) * np.array(p.e2))
        return out

    def dB_dtheta(self, t: float) -> np.ndarray:
        """[2*npulses, 3]: derivatives w.r.t. (A_1..A_k, omega_1..omega_k)."""
        k = len(self.pulses)
        out = np.zeros((2 * k, 3))
        for i, p in enumerate(self.pulses):
            s = t - p.t0
            g = math.exp(-s * s / (2.0 * p.tau * p.tau))
            ph = p.omega * s + p.phase
            e1, e2 = np.array(p.e1), np.array(p.e2)
            out[i] = g * (math.cos(ph) * e1 + math.sin(ph) * e2)
            out[k + i] = p.A * g * s * (-math.sin(ph) * e1 + math.cos(ph) * e2)
        return out


@dataclass
class LaserPulseSpec:
    A: float
    omega: float
    t0: float
    tau: float
    phase: float = 0.0
    pol: tuple = (0.0, 0.0, 1.0)


@dataclass
class LaserSpec:
    """Uniform electric field E(t) = sum_k A_k pol_k cos(omega_k t + phase_k)
    exp(-(t - t0_k)^2 / (2 tau_k^2))  (pulse profile of the optical runs, Sec. 4.7).

    gauge "length": v_E = E(t).(r - c) (isolated systems);  gauge "velocity": the kinetic momentum
    of every state is shifted by the vector potential A(t) = -int_0^t E dt' (periodic systems):
    1/2 |G + k + A|^2 and projector phases exp(+/- i (k + A).d)."""
    pulses: List[LaserPulseSpec] = field(default_factory=list)
    gauge: str = "length"

    def A(self, t: float) -> np.ndarray:
        """Vector potential -int_0^t E(t') dt' by adaptive quadrature (scipy.integrate.quad)."""
        from scipy.integrate import quad
        out = np.zeros(3)
        if t == 0.0 or not self.pulses:
            return out
        for d in range(3):
            f = lambda tt: float(self.E(tt)[d])
            val, _ = quad(f, 0.0, t, epsabs=1e-14, epsrel=1e-12, limit=400)
            out[d] = -val
        return out

    def E(self, t: float) -> np.ndarray:
        out = np.zeros(3)
        for p in self.pulses:
            g = math.exp(-(t - p.t0) ** 2 / (2.0 * p.tau * p.tau))
            out = out + p.A * math.cos(p.omega * t + p.phase) * g * np.array(p.pol, dtype=np.float64)
        return out


def laser_potential(grid: "Grid", E: np.ndarray) -> np.ndarray:
    """v_E(r) = E.(r - c): length-gauge potential energy of an electron (charge -1) in the uniform
    field E, with r the grid point i*h and c the cell centre (the jump of this sawtooth sits on
    the cell faces, where an isolated system has no density)."""
    v = np.zeros(grid.n)
    for d in range(3):
        x = grid.axis(d) - 0.5 * grid.L[d]
        sh = [1, 1, 1]
        sh[d] = grid.n[d]
        v = v + E[d] * x.reshape(sh)
    return v


# ----------------------------------------------------------------------------
# spinor spherical harmonics and projectors (Sec. 3.5)
# ----------------------------------------------------------------------------
def ylm(l: int, m: int, u: np.ndarray) -> np.ndarray:
    """Complex spherical harmonic Y_l^m (Condon-Shortley phase) of unit vectors u[..., 3]."""
    x, y, z = u[..., 0], u[..., 1], u[..., 2]
    if abs(m) > l:
        return np.zeros(x.shape, dtype=np.complex128)
    pi = math.pi
    if l == 0:
        return np.full(x.shape, 0.5 / math.sqrt(pi), dtype=np.complex128)
    if l == 1:
        if m == 0:
            return math.sqrt(3.0 / (4 * pi)) * z + 0j
        return -m * math.sqrt(3.0 / (8 * pi)) * (x + 1j * m * y)
    if l == 2:
        if m == 0:
            return math.sqrt(5.0 / (16 * pi)) * (3 * z * z - 1) + 0j
        if abs(m) == 1:
            return -m * math.sqrt(15.0 / (8 * pi)) * z * (x + 1j * m * y)
        s = 1 if m > 0 else -1
        return math.sqrt(15.0 / (32 * pi)) * (x + 1j * s * y) ** 2
    raise NotImplementedError("l > 2")


def spinor_harmonic_coefficients(l: int, twoj: int, twomj: int):
    """Coefficients of Phi_{l,j}^{m_j} = c_up Y_l^{m_j-1/2} chi_up + c_dn Y_l^{m_j+1/2} chi_dn.

    From the spinor-harmonic formula of Sec. 3.5, read with m = m_j - 1/2 for
    j = l + 1/2 and m = m_j + 1/2 for j = l - 1/2:
      j = l + 1/2:  c_up =  sqrt((l + m_j + 1/2)/(2l+1)),  c_dn = +sqrt((l - m_j + 1/2)/(2l+1))
      j = l - 1/2:  c_up =  sqrt((l - m_j + 1/2)/(2l+1)),  c_dn = -sqrt((l + m_j + 1/2)/(2l+1))
    Returns (c_up, m_up, c_dn, m_dn) with integer m's.
    """
    mj = twomj / 2.0
    m_up = (twomj - 1) // 2
    m_dn = (twomj + 1) // 2
    if twoj == 2 * l + 1:
        c_up = math.sqrt((l + mj + 0.5) / (2 * l + 1))
        c_dn = math.sqrt((l - mj + 0.5) / (2 * l + 1))
    elif twoj == 2 * l - 1:
        c_up = math.sqrt((l - mj + 0.5) / (2 * l + 1))
        c_dn = -math.sqrt((l + mj + 0.5) / (2 * l + 1))
    else:
        raise ValueError("j must be l +/- 1/2")
    return c_up, m_up, c_dn, m_dn


def radial_norm(l: int, rc: float, rs: float) -> float:
    """sqrt of int_0^rs (r^l exp(-r^2/2rc^2))^2 r^2 dr = (rc^(2l+3)/2) gamma_lower(l+3/2, rs^2/rc^2)."""
    a = l + 1.5
    val = 0.5 * rc ** (2 * l + 3) * _gammainc(a, (rs / rc) ** 2) * _gamma(a)
    return math.sqrt(val)


@dataclass
class AtomProjectors:
    idx: np.ndarray        # [Ns] flat grid indices (C order) inside the sphere
    beta: np.ndarray       # [P, 2, Ns] complex projector values
    energy: np.ndarray     # [P] KB energies
    disp: np.ndarray = None  # [Ns, 3] minimum-image displacement r - R_a of each sphere point


def build_projectors(grid: Grid, positions: np.ndarray, channels: Sequence,
                     r_sphere: float) -> List[AtomProjectors]:
    """beta_{a,p}(r, s) = f_l(|d|) Phi_{l j}^{m_j}(d/|d|)_s / norm_l,  d = min-image(r - R_a), |d| < r_sphere.

    This is the |delta V phi> factor of Eq. (Vps) with the KB denominator
    absorbed into the channel energy; channels are (l, twoj, energy, rc).
    """
    out: List[AtomProjectors] = []
    if len(channels) == 0:
        return out
    X, Y, Z = np.meshgrid(grid.axis(0), grid.axis(1), grid.axis(2), indexing="ij")
    r = np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1)
    L = np.array(grid.L, dtype=np.float64)
    for R in positions:
        d = r - R
        d -= L * np.round(d / L)
        dist = np.sqrt(np.sum(d * d, axis=1))
        sel = np.nonzero(dist < r_sphere)[0]
        dd = d[sel]
        ds = dist[sel]
        u = np.zeros_like(dd)
        nzr = ds > 0
        u[nzr] = dd[nzr] / ds[nzr, None]
        u[~nzr] = np.array([0.0, 0.0, 1.0])
        betas, energies = [], []
        for ch in channels:
            l, twoj, energy, rc = ch.l, ch.twoj, ch.energy, ch.rc
            f = ds ** l * np.exp(-ds * ds / (2.0 * rc * rc)) / radial_norm(l, rc, r_sphere)
            for twomj in range(-twoj, twoj + 1, 2):
                c_up, m_up, c_dn, m_dn = spinor_harmonic_coefficients(l, twoj, twomj)
                b = np.stack([f * c_up * ylm(l, m_up, u), f * c_dn * ylm(l, m_dn, u)])
                betas.append(b)
                energies.append(energy)
        out.append(AtomProjectors(sel, np.array(betas), np.array(energies, dtype=np.float64), dd.copy()))
    return out


def _bloch_phase(ap: AtomProjectors, kvec: Optional[np.ndarray], S: int):
    """[S, Ns] exp(i k_i.d) for the sphere points of one atom (ones without Bloch vectors)."""
    if kvec is None:
        return None
    return np.exp(1j * (kvec @ ap.disp.T))


def projections(psi: np.ndarray, projs: List[AtomProjectors], grid: Grid,
                kvec: Optional[np.ndarray] = None):
    """C_{a,p,i} = dV sum_{r in sphere a} sum_s conj(beta_{a,p}(r,s)) psi_i(r,s).

    For Bloch states psi_i = exp(i k_i.r) u_i held as u_i, the sphere about the atom image at
    R_a + L sees exp(i k_i.(R_a + L + d)) u_i(r): up to the factor exp(i k_i.(R_a + L)), which
    cancels between the projection and the scatter, C uses exp(i k_i.d) u_i(r)."""
    S = psi.shape[0]
    flat = psi.reshape(S, 2, -1)
    out = []
    for ap in projs:
        sub = flat[:, :, ap.idx]                        # [S, 2, Ns]
        ph = _bloch_phase(ap, kvec, S)
        if ph is not None:
            sub = sub * ph[:, None, :]
        out.append(grid.dV * np.einsum("psk,isk->pi", ap.beta.conj(), sub))
    return out


def apply_nonlocal(psi: np.ndarray, projs: List[AtomProjectors], grid: Grid,
                   kvec: Optional[np.ndarray] = None) -> np.ndarray:
    """V_NL psi_i = sum_a sum_p beta_{a,p} E_{a,p} C_{a,p,i}   (Eqs. Vps, Vps-soc);
    for Bloch states the scattered rows carry exp(-i k_i.d)."""
    S = psi.shape[0]
    out = np.zeros((S, 2, grid.N), dtype=np.complex128)
    for ap, C in zip(projs, projections(psi, projs, grid, kvec)):
        ec = ap.energy[:, None] * C                     # [P, S]
        add = np.einsum("psk,pi->isk", ap.beta, ec)
        ph = _bloch_phase(ap, kvec, S)
        if ph is not None:
            add = add * ph.conj()[:, None, :]
        out[:, :, ap.idx] += add
    return out.reshape(psi.shape)


# ----------------------------------------------------------------------------
# local 2x2 potential (Eq. HNC-SDFT; V_xc matrix of Sec. 3.3; Eq. zeeman_potential)
# ----------------------------------------------------------------------------
def apply_local(psi: np.ndarray, v: np.ndarray, b: np.ndarray) -> np.ndarray:
    """[v + b.sigma] psi:  up' = (v+b_z) up + (b_x - i b_y) dn;  dn' = (b_x + i b_y) up + (v - b_z) dn."""
    up, dn = psi[:, 0], psi[:, 1]
    out = np.empty_like(psi)
    out[:, 0] = (v + b[2]) * up + (b[0] - 1j * b[1]) * dn
    out[:, 1] = (b[0] + 1j * b[1]) * up + (v - b[2]) * dn
    return out


# ----------------------------------------------------------------------------
# system description and self-consistent fields
# ----------------------------------------------------------------------------
@dataclass
class System:
    grid: Grid
    occ: np.ndarray
    v_ext: np.ndarray
    projs: List[AtomProjectors]
    bfield: FieldSpec
    xc: int = 1
    hartree: int = 1
    thr: float = 1e-12
    dt: float = 0.05
    K: int = 4
    laser: LaserSpec = field(default_factory=LaserSpec)
    kvec: Optional[np.ndarray] = None   # [S, 3] Bloch vector of each state (None: Gamma only)


@dataclass
class Fields:
    v: np.ndarray          # total scalar potential
    b: np.ndarray          # [3] total magnetic field (b_xc + mu_B B)
    vH: np.ndarray
    vbar: np.ndarray
    bxc: np.ndarray
    ex: np.ndarray
    n: np.ndarray
    m: np.ndarray
    B: np.ndarray
    vE: np.ndarray = None  # laser potential at t (zeros without a laser or in the velocity gauge)
    A: np.ndarray = None   # velocity-gauge vector potential at t (None in the length gauge)


def fields_from_density(sysd: System, rho_v: np.ndarray, t: float) -> Fields:
    """v = v_ext + v_E(t) + v_H[n] + vbar_xc[n, m];  b = b_xc[n, m] + mu_B B(t)  (Eq. HNC-SDFT and
    its b_s; v_E the laser potential, zero without a laser)."""
    n, m = charge_and_magnetization(rho_v)
    grid = sysd.grid
    vH = hartree(n, grid) if sysd.hartree else np.zeros_like(n)
    if sysd.xc:
        vbar, bxc, ex = slater_exchange(n, m, sysd.thr)
        if sysd.xc >= 2:
            vc, bc, ec = pw92_correlation(n, m, sysd.thr)
            vbar, bxc, ex = vbar + vc, bxc + bc, ex + ec
    else:
        vbar, bxc, ex = np.zeros_like(n), np.zeros_like(m), np.zeros_like(n)
    B = sysd.bfield.B(t)
    A = None
    if sysd.laser.gauge == "velocity":
        vE = np.zeros_like(n)
        A = sysd.laser.A(t) if sysd.laser.pulses else None
    else:
        vE = laser_potential(grid, sysd.laser.E(t))
    v = sysd.v_ext + vE + vH + vbar
    b = bxc + MU_B * B[:, None, None, None]
    return Fields(v, b, vH, vbar, bxc, ex, n, m, B, vE, A)


def effective_kvec(sysd: System, F: Fields, S: int) -> Optional[np.ndarray]:
    """Bloch vectors of the states, shifted by the velocity-gauge vector potential if any."""
    if F.A is None:
        return sysd.kvec
    base = np.zeros((S, 3)) if sysd.kvec is None else sysd.kvec
    return base + F.A[None, :]


def apply_hamiltonian(sysd: System, psi: np.ndarray, F: Fields) -> np.ndarray:
    """H psi = T psi + [v + b.sigma] psi + V_NL psi  (Eq. TDSDFT with the pseudopotential of Eq. Vps)."""
    kv = effective_kvec(sysd, F, psi.shape[0])
    out = kinetic(psi, sysd.grid, kv) + apply_local(psi, F.v, F.b)
    if sysd.projs:
        out = out + apply_nonlocal(psi, sysd.projs, sysd.grid, kv)
    return out


# ----------------------------------------------------------------------------
# propagator: truncated Taylor exponential and ETRS
# ----------------------------------------------------------------------------
def taylor_exp(applyH: Callable, x: np.ndarray, a: float, K: int) -> np.ndarray:
    """T_K(-i a H) x = sum_{k=0}^{K} x_k,  x_0 = x,  x_{k+1} = (-i a/(k+1)) H x_k."""
    total = x.copy()
    xk = x
    for k in range(K):
        xk = (-1j * a / (k + 1)) * applyH(xk)
        total = total + xk
    return total


def etrs_step(sysd: System, psi: np.ndarray, t: float):
    """One step t -> t + dt.

    H_n from rho(psi_n) and B(t_n):      phi = T(-i dt/2 H_n) psi_n
    predictor:                           psi~ = T(-i dt/2 H_n) phi
    H~ from rho(psi~) and B(t_{n+1}):    psi_{n+1} = T(-i dt/2 H~) phi
    """
    a = 0.5 * sysd.dt
    F_n = fields_from_density(sysd, spin_density(psi, sysd.occ), t)
    H_n = lambda x: apply_hamiltonian(sysd, x, F_n)
    phi = taylor_exp(H_n, psi, a, sysd.K)
    psi_p = taylor_exp(H_n, phi, a, sysd.K)
    F_p = fields_from_density(sysd, spin_density(psi_p, sysd.occ), t + sysd.dt)
    H_p = lambda x: apply_hamiltonian(sysd, x, F_p)
    return taylor_exp(H_p, phi, a, sysd.K)


# ----------------------------------------------------------------------------
# observables
# ----------------------------------------------------------------------------
OBS_NAMES = ["t", "N_e", "M_x", "M_y", "M_z", "E_total", "E_kin", "E_loc", "E_NL",
             "E_H", "E_xc", "E_Z", "max_norm_err"]


def observables(sysd: System, psi: np.ndarray, t: float) -> np.ndarray:
    """Row of 13 doubles: t, N_e, M, energies and the largest |<psi_i|psi_i> - 1|.

    E = sum_i f_i <psi_i|T|psi_i> + int (v_ext + v_E(t)) n + sum_i f_i sum_p E_p |C_p,i|^2
        + mu_B B.M + 1/2 int v_H n + int e_x.
    """
    grid = sysd.grid
    dV = grid.dV
    rho_v = spin_density(psi, sysd.occ)
    F = fields_from_density(sysd, rho_v, t)
    n, m = F.n, F.m
    Ne = n.sum() * dV
    M = m.reshape(3, -1).sum(axis=1) * dV
    f = sysd.occ
    kv = effective_kvec(sysd, F, psi.shape[0])
    Tpsi = kinetic(psi, grid, kv)
    ekin = float(np.sum(f * np.real(np.sum(psi.conj() * Tpsi, axis=(1, 2, 3, 4)))) * dV)
    eloc = float(np.sum((sysd.v_ext + F.vE) * n) * dV)
    enl = 0.0
    if sysd.projs:
        for ap, C in zip(sysd.projs, projections(psi, sysd.projs, grid, kv)):
            enl += float(np.sum(f[None, :] * ap.energy[:, None] * np.abs(C) ** 2))
    eh = float(0.5 * np.sum(F.vH * n) * dV)
    exc = float(np.sum(F.ex) * dV)
    ez = float(MU_B * np.dot(F.B, M))
    norms = np.real(np.sum(psi.conj() * psi, axis=(1, 2, 3, 4))) * dV
    etot = ekin + eloc + enl + eh + exc + ez
    return np.array([t, Ne, M[0], M[1], M[2], etot, ekin, eloc, enl, eh, exc, ez,
                     float(np.max(np.abs(norms - 1.0)))])


def run(sysd: System, psi0: np.ndarray, nsteps: int, t0: float = 0.0, record: bool = True):
    """Propagate nsteps; returns (psi_final, obs[nsteps+1, 13])."""
    psi = psi0.copy()
    t = t0
    rows = [observables(sysd, psi, t)] if record else []
    for _ in range(nsteps):
        psi = etrs_step(sysd, psi, t)
        t += sysd.dt
        if record:
            rows.append(observables(sysd, psi, t))
    return psi, (np.array(rows) if record else None)


# ----------------------------------------------------------------------------
# initial spin-density matrix (Sec. 3.2, DMInitialization) and the ground state
# ----------------------------------------------------------------------------
@dataclass
class AtomDensitySpec:
    """Atomic charge Z (electrons) in a Gaussian of width sigma, and the atom's moment (mu_B)."""
    Z: float
    sigma: float
    moment: tuple = (0.0, 0.0, 0.0)


def dm_initialization(grid: Grid, positions: np.ndarray, atoms: List[AtomDensitySpec]) -> np.ndarray:
    """rho_v of the initialisation algorithm: every grid point belongs to its nearest atom
    (Voronoi partition, minimum image, ties to the lowest atom index); with d the distance to that
    atom, n = n_a(d) = Z_a (2 pi sigma_a^2)^(-3/2) exp(-d^2 / 2 sigma_a^2) and the local
    polarisation vector m = M_a / Z_a (the atom's moment per electron),
    rho_v = n {(1 + m_z)/2, (1 - m_z)/2, m_x/2, -m_y/2}  (ComputeSpinDensity, Eq. density4)."""
    X, Y, Z = np.meshgrid(grid.axis(0), grid.axis(1), grid.axis(2), indexing="ij")
    r = np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1)
    L = np.array(grid.L, dtype=np.float64)
    best = np.full(r.shape[0], np.inf)
    owner = np.zeros(r.shape[0], dtype=np.int64)
    for a, R in enumerate(np.asarray(positions, dtype=np.float64)):
        d = r - R
        d -= L * np.round(d / L)
        d2 = (d[:, 0] * d[:, 0] + d[:, 1] * d[:, 1]) + d[:, 2] * d[:, 2]
        closer = d2 < best
        best[closer] = d2[closer]
        owner[closer] = a
    rho = np.zeros((4, r.shape[0]))
    for a, spec in enumerate(atoms):
        sel = owner == a
        n = spec.Z * (2.0 * math.pi * spec.sigma ** 2) ** -1.5 * np.exp(-best[sel] / (2.0 * spec.sigma ** 2))
        m = np.asarray(spec.moment, dtype=np.float64) / spec.Z
        rho[0, sel] = n * (1.0 + m[2]) / 2.0
        rho[1, sel] = n * (1.0 - m[2]) / 2.0
        rho[2, sel] = n * m[0] / 2.0
        rho[3, sel] = -n * m[1] / 2.0
    return rho.reshape((4,) + tuple(grid.n))


def k_blocks(kvec: Optional[np.ndarray], S: int):
    """Runs [i0, i1) of consecutive states that share one Bloch vector (a single run at Gamma).
    States of different k are orthogonal through their Bloch factors, not through their periodic
    parts, so orthonormalisation acts within each run."""
    if kvec is None:
        return [(0, S)]
    kvec = np.asarray(kvec)
    runs, i0 = [], 0
    for i in range(1, S + 1):
        if i == S or not np.array_equal(kvec[i], kvec[i0]):
            runs.append((i0, i))
            i0 = i
    return runs


def orthonormalize(psi: np.ndarray, dV: float, kvec: Optional[np.ndarray] = None) -> np.ndarray:
    """Psi <- Psi L^(-H) with L L^H = dV Psi^H Psi (Cholesky), within each run of states of one
    Bloch vector: orthonormal states spanning the same space (the overlap and the triangular
    solve are library primitives)."""
    import scipy.linalg
    S = psi.shape[0]
    flat = psi.reshape(S, -1)
    out = np.empty_like(flat)
    for i0, i1 in k_blocks(kvec, S):
        f = flat[i0:i1]
        ovl = dV * (f.conj() @ f.T)
        Lc = scipy.linalg.cholesky(ovl, lower=True)
        # rows of the result: psi_new_j = sum_i psi_i (L^-H)_ij, i.e. new = conj(L)^-1 f
        out[i0:i1] = scipy.linalg.solve_triangular(Lc.conj(), f, lower=True)
    return out.reshape(psi.shape)


def ground_state(sysd: System, psi0: np.ndarray, niter: int, tau: float,
                 rho_init: Optional[np.ndarray] = None):
    """Self-consistent imaginary-time propagation: each iteration applies T_K(-tau H[rho]) (the
    Taylor polynomial of exp(-tau H), K = sysd.K) to the states, orthonormalises them (within each
    run of one Bloch vector), and takes the new density; the first iteration uses rho_init if given (e.g. from dm_initialization).
    Returns (psi, total energies after each iteration)."""
    psi = orthonormalize(psi0, sysd.grid.dV, sysd.kvec)
    rho = spin_density(psi, sysd.occ) if rho_init is None else rho_init
    energies = []
    for _ in range(niter):
        F = fields_from_density(sysd, rho, 0.0)
        H = lambda x: apply_hamiltonian(sysd, x, F)
        psi = taylor_exp(H, psi, -1j * tau, sysd.K)
        psi = orthonormalize(psi, sysd.grid.dV, sysd.kvec)
        rho = spin_density(psi, sysd.occ)
        energies.append(observables(sysd, psi, 0.0)[5])
    return psi, np.array(energies)


# ----------------------------------------------------------------------------
# tangent-linear (forward-mode) derivative of the discrete trajectory
# ----------------------------------------------------------------------------
def _density_jvp(psi, dpsi, occ):
    """d rho_v for psi -> psi + dpsi (rho is sesquilinear)."""
    up, dn = psi[:, 0], psi[:, 1]
    dup, ddn = dpsi[:, 0], dpsi[:, 1]
    f = occ.reshape(-1, 1, 1, 1)
    d_uu = np.sum(f * 2.0 * (dup * up.conj()).real, axis=0)
    d_dd = np.sum(f * 2.0 * (ddn * dn.conj()).real, axis=0)
    d_ud = np.sum(f * (dup * dn.conj() + up * ddn.conj()), axis=0)
    return np.stack([d_uu, d_dd, d_ud.real, d_ud.imag])


def _fields_jvp(sysd: System, rho_v, drho_v, dB):
    n, m = charge_and_magnetization(rho_v)
    dn, dm = charge_and_magnetization(drho_v)
    dvH = hartree(dn, sysd.grid) if sysd.hartree else np.zeros_like(n)
    if sysd.xc:
        dvbar, dbxc = slater_exchange_jvp(n, m, dn, dm, sysd.thr)
        if sysd.xc >= 2:
            dvc, dbc = pw92_correlation_jvp(n, m, dn, dm, sysd.thr)
            dvbar, dbxc = dvbar + dvc, dbxc + dbc
    else:
        dvbar, dbxc = np.zeros_like(n), np.zeros_like(m)
    return dvH + dvbar, dbxc + MU_B * np.asarray(dB)[:, None, None, None]


def _taylor_jvp(applyH, applydH, x, dx, a, K):
    """Derivative of T_K(-i a H) x along (dx, dH):  dx_{k+1} = (-i a/(k+1)) (H dx_k + dH x_k)."""
    total, dtotal = x.copy(), dx.copy()
    xk, dxk = x, dx
    for k in range(K):
        c = -1j * a / (k + 1)
        nxk = c * applyH(xk)
        ndxk = c * (applyH(dxk) + applydH(xk))
        xk, dxk = nxk, ndxk
        total = total + xk
        dtotal = dtotal + dxk
    return total, dtotal


def etrs_step_jvp(sysd: System, psi, dpsi, t, dB_n, dB_np1):
    a = 0.5 * sysd.dt
    rho = spin_density(psi, sysd.occ)
    F_n = fields_from_density(sysd, rho, t)
    dv_n, db_n = _fields_jvp(sysd, rho, _density_jvp(psi, dpsi, sysd.occ), dB_n)
    H_n = lambda x: apply_hamiltonian(sysd, x, F_n)
    dH_n = lambda x: apply_local(x, dv_n, db_n)
    phi, dphi = _taylor_jvp(H_n, dH_n, psi, dpsi, a, sysd.K)
    pp, dpp = _taylor_jvp(H_n, dH_n, phi, dphi, a, sysd.K)
    rho_p = spin_density(pp, sysd.occ)
    F_p = fields_from_density(sysd, rho_p, t + sysd.dt)
    dv_p, db_p = _fields_jvp(sysd, rho_p, _density_jvp(pp, dpp, sysd.occ), dB_np1)
    H_p = lambda x: apply_hamiltonian(sysd, x, F_p)
    dH_p = lambda x: apply_local(x, dv_p, db_p)
    return _taylor_jvp(H_p, dH_p, phi, dphi, a, sysd.K)


def total_mz(sysd: System, psi) -> float:
    n, m = charge_and_magnetization(spin_density(psi, sysd.occ))
    return float(np.sum(m[2]) * sysd.grid.dV)


def mz_gradient_tangent_linear(sysd: System, psi0, nsteps: int, t0: float = 0.0):
    """d M_z(t0 + nsteps dt) / d theta for theta = (A_1..A_k, omega_1..omega_k), by forward mode.

    One tangent run per parameter, exact for the discrete trajectory.
    """
    npar = 2 * len(sysd.bfield.pulses)
    grads = np.zeros(npar)
    for kpar in range(npar):
        psi = psi0.copy()
        dpsi = np.zeros_like(psi0)
        t = t0
        for _ in range(nsteps):
            dBn = sysd.bfield.dB_dtheta(t)[kpar]
            dBp = sysd.bfield.dB_dtheta(t + sysd.dt)[kpar]
            psi, dpsi = etrs_step_jvp(sysd, psi, dpsi, t, dBn, dBp)
            t += sysd.dt
        up, dn = psi[:, 0], psi[:, 1]
        dup, ddn = dpsi[:, 0], dpsi[:, 1]
        f = sysd.occ.reshape(-1, 1, 1, 1)
        dmz = np.sum(f * 2.0 * ((dup * up.conj()).real - (ddn * dn.conj()).real))
        grads[kpar] = float(dmz) * sysd.grid.dV
    return grads


# ----------------------------------------------------------------------------
# construction from a seeded workload
# ----------------------------------------------------------------------------
def system_from_workload(w, dt: Optional[float] = None) -> System:
    grid = Grid(tuple(w.n), tuple(w.L))
    projs = build_projectors(grid, w.positions, w.channels, w.r_sphere) if w.channels else []
    bf = FieldSpec(tuple(w.bfield.B0),
                   [PulseSpec(p.A, p.omega, p.t0, p.tau, p.phase, tuple(p.e1), tuple(p.e2))
                    for p in w.bfield.pulses])
    laser = LaserSpec([LaserPulseSpec(p.A, p.omega, p.t0, p.tau, p.phase, tuple(p.pol))
                       for p in getattr(w, "laser", [])], getattr(w, "laser_gauge", "length"))
    return System(grid=grid, occ=np.asarray(w.occ, dtype=np.float64), v_ext=w.v_ext,
                  projs=projs, bfield=bf, xc=w.xc, hartree=w.hartree, thr=w.m_threshold,
                  dt=w.dt if dt is None else dt, K=w.taylor_order, laser=laser,
                  kvec=None if getattr(w, "kvec", None) is None else np.asarray(w.kvec, dtype=np.float64))
