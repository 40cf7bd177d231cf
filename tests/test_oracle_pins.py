"""Pins of the CPU oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: a closed
form, a value printed in the paper, a textbook formula, a library routine
(scipy) or brute force on a tiny grid.  None of these tests needs a GPU.
"""
import math
import os

import numpy as np
import pytest
import scipy.linalg
from scipy.integrate import quad
from scipy.special import sph_harm_y

from oracle import nct_oracle as O
from paper_2506_21908_amd import inputs as I

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
HA_EV = 27.211386245988


def _free_system(n=(6, 6, 6), L=(5.0, 5.0, 5.0), xc=0, hartree=0, B0=(0, 0, 0), dt=0.05,
                 K=4, v_ext=None, projs=None, occ=None):
    grid = O.Grid(n, L)
    return O.System(grid=grid, occ=np.ones(1) if occ is None else occ,
                    v_ext=np.zeros(n) if v_ext is None else v_ext,
                    projs=[] if projs is None else projs,
                    bfield=O.FieldSpec(tuple(B0), []), xc=xc, hartree=hartree, dt=dt, K=K)


def _plane_wave(grid, kint, chi):
    """exp(i k.r)/sqrt(Omega) (x) chi with k = 2 pi kint / L."""
    X, Y, Z = np.meshgrid(grid.axis(0), grid.axis(1), grid.axis(2), indexing="ij")
    k = [2 * math.pi * kint[d] / grid.L[d] for d in range(3)]
    pw = np.exp(1j * (k[0] * X + k[1] * Y + k[2] * Z)) / math.sqrt(grid.volume)
    psi = np.stack([chi[0] * pw, chi[1] * pw])[None]
    return psi, 0.5 * sum(kk * kk for kk in k)


def _taylor_scalar(z, K):
    return sum(z ** k / math.factorial(k) for k in range(K + 1))


# ---------------------------------------------------------------- kinetic / FFT
def test_kinetic_plane_wave_closed_form():
    """-1/2 nabla^2 exp(ik.r) = k^2/2 exp(ik.r) for k on the reciprocal lattice (mixed radix 2/3 grid)."""
    grid = O.Grid((6, 4, 12), (3.0, 4.5, 5.0))
    for kint in [(1, 0, 0), (0, 1, 2), (-2, 1, -5), (3, 2, 6)]:
        psi, eps = _plane_wave(grid, kint, (1.0, 0.0))
        Tpsi = O.kinetic(psi, grid)
        if abs(kint[0]) * 2 == grid.n[0] or abs(kint[2]) * 2 == grid.n[2]:
            # Nyquist modes: fftfreq assigns -n/2, same |G|^2
            pass
        assert np.allclose(Tpsi, eps * psi, atol=1e-12 * max(1.0, eps))


def test_kinetic_dense_dft_matrix():
    """Kinetic operator from explicit DFT matrices (no FFT library) on a 4x6x3 grid."""
    n, L = (4, 6, 3), (2.0, 3.3, 1.7)
    grid = O.Grid(n, L)
    rng = np.random.default_rng(0)
    f = rng.standard_normal(n) + 1j * rng.standard_normal(n)

    def dft(m):
        j = np.arange(m)
        return np.exp(-2j * math.pi * np.outer(j, j) / m)

    def freq(m, Ld):
        k = np.arange(m)
        k = np.where(k <= (m - 1) // 2, k, k - m)   # signed index; Nyquist (even m) -> -m/2
        return 2 * math.pi * k / Ld

    F = np.kron(np.kron(dft(n[0]), dft(n[1])), dft(n[2]))
    gx, gy, gz = (freq(n[d], L[d]) for d in range(3))
    g2 = (gx[:, None, None] ** 2 + gy[None, :, None] ** 2 + gz[None, None, :] ** 2).ravel()
    Tdense = np.linalg.inv(F) @ np.diag(0.5 * g2) @ F
    ref = (Tdense @ f.ravel()).reshape(n)
    got = O.kinetic(f[None, None], grid)[0, 0]
    assert np.allclose(got, ref, atol=1e-12)


# ---------------------------------------------------------------- density conventions
def test_spinor_direction_to_magnetization():
    """Spinor (cos t/2, e^{i p} sin t/2) has m = n (sin t cos p, sin t sin p, cos t) (Eqs. rho1-3)."""
    grid = O.Grid((2, 2, 2), (1.0, 1.0, 1.0))
    for th, ph in [(0.3, 0.0), (1.1, 2.0), (2.9, -1.3), (math.pi / 2, math.pi / 2)]:
        chi = np.array([math.cos(th / 2), np.exp(1j * ph) * math.sin(th / 2)])
        psi = np.broadcast_to(chi[None, :, None, None, None], (1, 2, 2, 2, 2)).copy() * 0.7
        n, m = O.charge_and_magnetization(O.spin_density(psi, np.ones(1)))
        exp_m = 0.49 * np.array([math.sin(th) * math.cos(ph), math.sin(th) * math.sin(ph), math.cos(th)])
        assert np.allclose(n, 0.49)
        assert np.allclose(m.reshape(3, -1), exp_m[:, None])


def test_spin_density_map_golden():
    """rho_v of a pure spinor state equals the ComputeSpinDensity map of the initialisation algorithm."""
    rows = np.loadtxt(os.path.join(GOLDEN, "spin_density_map.txt"))
    for th, ph, n, *exp in rows:
        th, ph = math.radians(th), math.radians(ph)
        chi = math.sqrt(n) * np.array([math.cos(th / 2), np.exp(1j * ph) * math.sin(th / 2)])
        psi = chi.reshape(1, 2, 1, 1, 1)
        rho = O.spin_density(psi, np.ones(1)).ravel()
        assert np.allclose(rho, exp, atol=1e-14)


def test_magnetization_bounded_by_density():
    w = I.make_system(n=(6, 6, 6), L=(5.0,) * 3, nstates=5, case=3)
    n, m = O.charge_and_magnetization(O.spin_density(w.psi0, w.occ))
    assert np.all(np.sqrt((m ** 2).sum(0)) <= n * (1 + 1e-12))


# ---------------------------------------------------------------- exchange
def test_slater_unpolarised_textbook():
    """m = 0: v_x = -(3n/pi)^(1/3), e_x = -(3/4)(3/pi)^(1/3) n^(4/3) (Dirac/Slater exchange)."""
    n = np.array([1e-4, 0.01, 0.3, 2.0])
    m = np.zeros((3, 4))
    vbar, bxc, ex = O.slater_exchange(n, m)
    assert np.allclose(vbar, -(3 * n / math.pi) ** (1 / 3), rtol=1e-14)
    assert np.allclose(ex, -0.75 * (3 / math.pi) ** (1 / 3) * n ** (4 / 3), rtol=1e-14)
    assert np.all(bxc == 0)


def test_slater_full_polarisation_scaling():
    """Fully polarised gas: e_x(n, |m|=n) = 2^(1/3) e_x(n, 0) (spin scaling of exchange)."""
    n = np.array([0.01, 0.5, 3.0])
    m = np.stack([np.zeros(3), np.zeros(3), n])
    _, _, ex1 = O.slater_exchange(n, m)
    _, _, ex0 = O.slater_exchange(n, np.zeros((3, 3)))
    assert np.allclose(ex1, 2 ** (1 / 3) * ex0, rtol=1e-13)


def test_slater_potential_is_energy_derivative():
    """v_s = d e_x / d n_s by central differences; b along m with magnitude (v_up - v_dn)/2."""
    rng = np.random.default_rng(1)
    n = rng.uniform(0.05, 1.0, 20)
    mhat = rng.standard_normal((3, 20))
    mhat /= np.linalg.norm(mhat, axis=0)
    mu = n * rng.uniform(0.05, 0.9, 20)
    m = mhat * mu
    vbar, bxc, _ = O.slater_exchange(n, m)
    h = 1e-6

    def ex_of(nu, nd):
        nn = nu + nd
        mm = mhat * (nu - nd)
        return O.slater_exchange(nn, mm)[2]
    nu, nd = (n + mu) / 2, (n - mu) / 2
    vu = (ex_of(nu + h, nd) - ex_of(nu - h, nd)) / (2 * h)
    vd = (ex_of(nu, nd + h) - ex_of(nu, nd - h)) / (2 * h)
    assert np.allclose(vbar, 0.5 * (vu + vd), rtol=1e-8)
    assert np.allclose(bxc, 0.5 * (vu - vd) * mhat, rtol=1e-7, atol=1e-10)
    # zero local torque: b_xc x m = 0 pointwise (locally collinear functional)
    assert np.allclose(np.cross(bxc.T, m.T), 0, atol=1e-14)


def test_slater_vxc_matrix_eigenpairs():
    """The 2x2 V_xc = vbar + b_xc.sigma has eigenvalues v_up, v_dn with eigenvectors along +/- mhat."""
    n = np.array([0.7])
    m = np.array([[0.1], [-0.2], [0.25]])
    vbar, bxc, _ = O.slater_exchange(n, m)
    mu = np.linalg.norm(m)
    v_up = -O.SLATER_C * ((n[0] + mu) / 2) ** (1 / 3)
    v_dn = -O.SLATER_C * ((n[0] - mu) / 2) ** (1 / 3)
    sx = np.array([[0, 1], [1, 0]]); sy = np.array([[0, -1j], [1j, 0]]); sz = np.diag([1, -1])
    V = vbar[0] * np.eye(2) + bxc[0, 0] * sx + bxc[1, 0] * sy + bxc[2, 0] * sz
    ev, vec = np.linalg.eigh(V)
    assert np.allclose(sorted(ev), sorted([v_up, v_dn]), rtol=1e-13)
    # eigenvector of the lower eigenvalue v_up has spin along +mhat
    s = vec[:, 0]
    spin = np.real([s.conj() @ sx @ s, s.conj() @ sy @ s, s.conj() @ sz @ s])
    assert np.allclose(spin, m[:, 0] / mu, atol=1e-12)


def test_slater_below_threshold_zero_field():
    n = np.array([0.5, 0.5])
    m = np.array([[1e-14, 0.0], [0.0, 0.0], [0.0, 0.0]])
    _, bxc, _ = O.slater_exchange(n, m, thr=1e-12)
    assert np.all(bxc == 0)


def test_slater_jvp_matches_central_differences():
    rng = np.random.default_rng(2)
    n = rng.uniform(0.1, 1.0, 30)
    m = rng.standard_normal((3, 30)) * 0.2 * n
    dn = rng.standard_normal(30)
    dm = rng.standard_normal((3, 30))
    h = 1e-6
    vp, bp, _ = O.slater_exchange(n + h * dn, m + h * dm)
    vm, bm, _ = O.slater_exchange(n - h * dn, m - h * dm)
    dv, db = O.slater_exchange_jvp(n, m, dn, dm)
    assert np.allclose(dv, (vp - vm) / (2 * h), rtol=1e-7, atol=1e-9)
    assert np.allclose(db, (bp - bm) / (2 * h), rtol=1e-7, atol=1e-9)


# ---------------------------------------------------------------- Hartree
# ---------------------------------------------------------------- PW92 correlation (xc = 2)
def test_pw92_high_density_limit():
    """eps_c -> c0 ln rs - c1 as rs -> 0 with the exact Gell-Mann-Brueckner coefficient
    c0 = (1 - ln 2)/pi^2 (half of it when fully polarised) and PW92's c1 = 0.046644."""
    c0 = (1.0 - math.log(2.0)) / math.pi ** 2
    for z, c in ((0.0, c0), (1.0, 0.5 * c0)):
        rs = 1e-8
        e1 = float(O.pw92_eps(np.array(rs), np.array(z))[0])
        e2 = float(O.pw92_eps(np.array(rs * 1.01), np.array(z))[0])
        # PW92 prints A to 5 significant digits (0.031091, 0.015545)
        assert abs((e2 - e1) / math.log(1.01) / c - 1.0) < 5e-5
    e = float(O.pw92_eps(np.array(1e-6), np.array(0.0))[0])
    assert abs(-(e - c0 * math.log(1e-6)) - 0.046644) < 5e-6


def test_pw92_uniform_gas_textbook_values():
    """Unpolarised correlation energies of the uniform electron gas (Ceperley-Alder, as fitted by
    PW92): -0.0448, -0.0282, -0.0186 Ha at rs = 2, 5, 10."""
    for rs, ref in ((2.0, -0.0448), (5.0, -0.0282), (10.0, -0.0186)):
        assert abs(float(O.pw92_eps(np.array(rs), np.array(0.0))[0]) - ref) < 2e-4


def test_pw92_spin_interpolation():
    f = lambda z: float(O.pw92_f(np.array(z))[0])
    fp = lambda z: float(O.pw92_f(np.array(z))[1])
    assert f(0.0) == 0.0 and abs(f(1.0) - 1.0) < 1e-15 and abs(f(-1.0) - 1.0) < 1e-15
    h = 1e-4
    assert abs((f(h) - 2 * f(0.0) + f(-h)) / h ** 2 - O.PW92_FPP0) < 1e-6
    for z in (0.2, 0.7, 0.95):
        assert abs((f(z + 1e-6) - f(z - 1e-6)) / 2e-6 - fp(z)) < 1e-8


def test_pw92_potentials_are_energy_derivatives():
    """v_up/dn = d(n eps_c)/d n_up/dn (central differences), through the locally collinear map
    (n, m) -> (vbar_c, b_c) with eigenvalues v_up, v_dn of the 2x2 V_c along +/- mhat."""
    def e_of(nu, nd):
        n = nu + nd
        rs = (3.0 / (4.0 * math.pi * n)) ** (1.0 / 3.0)
        return n * float(O.pw92_eps(np.array(rs), np.array((nu - nd) / n))[0])
    mhat = np.array([0.3, -0.4, math.sqrt(1 - 0.25)])
    for n, z in ((0.5, 0.0), (0.05, 0.3), (0.002, 0.8), (1.3, 0.97)):
        nu, nd = 0.5 * n * (1 + z), 0.5 * n * (1 - z)
        h = 1e-6 * n
        vu = (e_of(nu + h, nd) - e_of(nu - h, nd)) / (2 * h)
        vd = (e_of(nu, nd + h) - e_of(nu, nd - h)) / (2 * h)
        m = (z * n * mhat)[:, None, None, None]
        vbar, bc, ec = O.pw92_correlation(np.full((1, 1, 1), n), m)
        b = bc[:, 0, 0, 0]
        if z > 0:
            assert np.linalg.norm(np.cross(b, mhat)) < 1e-15      # no local torque
        bm = float(np.dot(b, mhat))
        assert abs(float(vbar.ravel()[0]) + bm - vu) < 1e-7
        assert abs(float(vbar.ravel()[0]) - bm - vd) < 1e-7
        assert abs(float(ec.ravel()[0]) - e_of(nu, nd)) < 1e-15


def test_hartree_cosine_closed_form():
    """n = cos(G.r) gives v_H = (4 pi/|G|^2) cos(G.r); a constant density gives v_H = 0."""
    grid = O.Grid((8, 6, 12), (4.0, 3.0, 6.0))
    X, Y, Z = np.meshgrid(grid.axis(0), grid.axis(1), grid.axis(2), indexing="ij")
    G = np.array([2 * math.pi * 1 / 4.0, 2 * math.pi * 2 / 3.0, 2 * math.pi * -1 / 6.0])
    n = np.cos(G[0] * X + G[1] * Y + G[2] * Z)
    vH = O.hartree(n + 0.3, grid)
    assert np.allclose(vH, 4 * math.pi / (G @ G) * n, atol=1e-12)


# ---------------------------------------------------------------- projectors
def test_ylm_matches_scipy():
    rng = np.random.default_rng(3)
    u = rng.standard_normal((50, 3))
    u /= np.linalg.norm(u, axis=1)[:, None]
    theta = np.arccos(u[:, 2])
    phi = np.arctan2(u[:, 1], u[:, 0])
    for l in range(3):
        for m in range(-l, l + 1):
            assert np.allclose(O.ylm(l, m, u), sph_harm_y(l, m, theta, phi), atol=1e-14)


def _angular_momentum(l):
    """L_z, L_+, L_- in the |l m> basis ordered m = -l..l (standard ladder algebra)."""
    ms = np.arange(-l, l + 1)
    Lz = np.diag(ms).astype(float)
    Lp = np.zeros((2 * l + 1, 2 * l + 1))
    for i, m in enumerate(ms[:-1]):
        Lp[i + 1, i] = math.sqrt(l * (l + 1) - m * (m + 1))
    return Lz, Lp, Lp.T


@pytest.mark.parametrize("l", [1, 2])
def test_spinor_harmonics_are_LS_eigenvectors(l):
    """Phi_{l,j=l+1/2} has <L.S> = l/2, Phi_{l,j=l-1/2} has -(l+1)/2; P+ + P- = 1 (Eq. Vps-soc)."""
    Lz, Lp, Lm = _angular_momentum(l)
    Sz = np.diag([0.5, -0.5]); Sp = np.array([[0, 1.0], [0, 0]]); Sm = Sp.T
    LS = np.kron(Lz, Sz) + 0.5 * (np.kron(Lp, Sm) + np.kron(Lm, Sp))
    dim = 2 * (2 * l + 1)
    P = {1: np.zeros((dim, dim)), -1: np.zeros((dim, dim))}
    for twoj, sign, ev in [(2 * l + 1, 1, l / 2), (2 * l - 1, -1, -(l + 1) / 2)]:
        for twomj in range(-twoj, twoj + 1, 2):
            cu, mu_, cd, md = O.spinor_harmonic_coefficients(l, twoj, twomj)
            vec = np.zeros(dim)
            if abs(mu_) <= l:
                vec[2 * (mu_ + l) + 0] = cu
            if abs(md) <= l:
                vec[2 * (md + l) + 1] = cd
            assert abs(np.linalg.norm(vec) - 1) < 1e-14
            assert np.allclose(LS @ vec, ev * vec, atol=1e-14)
            # J_z eigenvalue m_j
            Jz = np.kron(Lz, np.eye(2)) + np.kron(np.eye(2 * l + 1), Sz)
            assert np.allclose(Jz @ vec, (twomj / 2) * vec, atol=1e-14)
            P[sign] += np.outer(vec, vec)
    assert np.allclose(P[1] + P[-1], np.eye(dim), atol=1e-14)
    assert np.allclose(LS, (l / 2) * P[1] - ((l + 1) / 2) * P[-1], atol=1e-14)


def test_spinor_harmonic_completeness_pointwise():
    """sum_{j,m_j} Phi(u) Phi(u')^dagger = sum_m Y_lm(u) Y_lm(u')^* 1_2 for l = 1, 2."""
    rng = np.random.default_rng(4)
    u = rng.standard_normal((7, 3)); u /= np.linalg.norm(u, axis=1)[:, None]
    v = rng.standard_normal((7, 3)); v /= np.linalg.norm(v, axis=1)[:, None]
    for l in (1, 2):
        acc = np.zeros((7, 2, 2), dtype=complex)
        for twoj in (2 * l - 1, 2 * l + 1):
            for twomj in range(-twoj, twoj + 1, 2):
                cu, mu_, cd, md = O.spinor_harmonic_coefficients(l, twoj, twomj)
                pu = np.stack([cu * O.ylm(l, mu_, u), cd * O.ylm(l, md, u)], axis=1)
                pv = np.stack([cu * O.ylm(l, mu_, v), cd * O.ylm(l, md, v)], axis=1)
                acc += pu[:, :, None] * pv[:, None, :].conj()
        ref = sum(O.ylm(l, m, u) * O.ylm(l, m, v).conj() for m in range(-l, l + 1))
        assert np.allclose(acc, ref[:, None, None] * np.eye(2)[None], atol=1e-14)


def test_radial_norm_quadrature():
    for l in (0, 1, 2):
        val, _ = quad(lambda r: (r ** l * math.exp(-r * r / (2 * 0.7 ** 2))) ** 2 * r * r, 0, 2.5,
                      epsabs=1e-15, epsrel=1e-13, limit=200)
        assert abs(O.radial_norm(l, 0.7, 2.5) - math.sqrt(val)) < 1e-13


def test_projector_table_shape_and_soc_energies():
    """18 projectors per atom: s(2), p1/2(2), p3/2(4), d3/2(4), d5/2(6); 2/(2l+1)(E+ - E-) = lambda_so."""
    chans = I.kb_channels(lambda_so=0.05)
    assert sum(c.twoj + 1 for c in chans) == 18
    E = {(c.l, c.twoj): c.energy for c in chans}
    for l in (1, 2):
        assert abs(2 / (2 * l + 1) * (E[(l, 2 * l + 1)] - E[(l, 2 * l - 1)]) - 0.05) < 1e-15
    grid = O.Grid((12, 12, 12), (7.0, 7.0, 7.0))
    projs = O.build_projectors(grid, np.array([[3.5, 3.5, 3.5]]), chans, 2.5)
    assert projs[0].beta.shape[0] == 18
    # grid norm approximates the continuum norm 1
    nrm = grid.dV * np.sum(np.abs(projs[0].beta) ** 2, axis=(1, 2))
    assert np.all(np.abs(nrm - 1) < 0.1)


def test_nonlocal_hermitian_and_spin_independent_without_soc():
    w = I.make_system(n=(10, 10, 10), L=(7.0,) * 3, nstates=3, natoms=1, case=5, lambda_so=0.0)
    sysd = O.system_from_workload(w)
    rng = np.random.default_rng(5)
    u = rng.standard_normal(w.psi0.shape) + 1j * rng.standard_normal(w.psi0.shape)
    v = rng.standard_normal(w.psi0.shape) + 1j * rng.standard_normal(w.psi0.shape)
    Vu = O.apply_nonlocal(u, sysd.projs, sysd.grid)
    Vv = O.apply_nonlocal(v, sysd.projs, sysd.grid)
    assert abs(np.vdot(v, Vu) - np.conj(np.vdot(u, Vv))) < 1e-10 * abs(np.vdot(v, Vu))
    U = scipy.linalg.expm(-0.5j * 0.8 * np.array([[0.3, 0.5 - 0.2j], [0.5 + 0.2j, -0.3]]))
    rot = lambda x: np.einsum("st,itxyz->isxyz", U, x)
    assert np.allclose(O.apply_nonlocal(rot(u), sysd.projs, sysd.grid), rot(Vu), atol=1e-11)


# ---------------------------------------------------------------- Zeeman / Larmor
def _gaussian_orbital(grid, spin):
    X, Y, Z = np.meshgrid(grid.axis(0), grid.axis(1), grid.axis(2), indexing="ij")
    c = [grid.L[d] / 2 for d in range(3)]
    g = np.exp(-((X - c[0]) ** 2 + (Y - c[1]) ** 2 + (Z - c[2]) ** 2) / 2.0)
    g = g / math.sqrt(np.sum(g * g) * grid.dV)
    return np.stack([spin[0] * g, spin[1] * g])[None].astype(complex)


@pytest.mark.parametrize("table", ["zeeman_H_1s.txt", "zeeman_Al_3s.txt"])
def test_zeeman_splitting_golden(table):
    """<up|H|up> - <dn|H|dn> = 2 mu_B B_z reproduces the paper's Zeeman tables (Delta E = 2 b)."""
    rows = np.loadtxt(os.path.join(GOLDEN, table))
    grid = O.Grid((12, 12, 12), (8.0, 8.0, 8.0))
    for b_ev, dE_ev in rows:
        Bz = (b_ev / HA_EV) / O.MU_B
        sysd = _free_system(grid.n, grid.L, B0=(0, 0, Bz),
                            v_ext=-np.ones(grid.n) * 0.3)
        levels = []
        for spin in ((1, 0), (0, 1)):
            psi = _gaussian_orbital(grid, spin)
            F = O.fields_from_density(sysd, O.spin_density(psi, sysd.occ), 0.0)
            Hpsi = O.apply_hamiltonian(sysd, psi, F)
            levels.append(np.real(np.vdot(psi, Hpsi)) * grid.dV)
        assert abs((levels[0] - levels[1]) * HA_EV - dE_ev) < 1e-4


def _rotation(axis, angle):
    axis = np.asarray(axis, float) / np.linalg.norm(axis)
    K = np.array([[0, -axis[2], axis[1]], [axis[2], 0, -axis[0]], [-axis[1], axis[0], 0]])
    return np.eye(3) + math.sin(angle) * K + (1 - math.cos(angle)) * K @ K


def test_larmor_exact_discrete_propagator():
    """Uniform spinor, no XC: psi_n = [T_4(-i dt/2 H)]^(2n) psi_0 with H = eps + mu_B B.sigma (2x2)."""
    grid = O.Grid((4, 4, 4), (3.0, 3.0, 3.0))
    B = np.array([0.3, -0.4, 0.5])
    sysd = _free_system(grid.n, grid.L, B0=tuple(B), dt=0.1)
    chi = np.array([0.6, 0.8j])
    psi0, eps = _plane_wave(grid, (0, 0, 0), chi)
    sx = np.array([[0, 1], [1, 0]]); sy = np.array([[0, -1j], [1j, 0]]); sz = np.diag([1.0, -1.0])
    H2 = eps * np.eye(2) + O.MU_B * (B[0] * sx + B[1] * sy + B[2] * sz)
    A = -1j * 0.05 * H2
    T = sum(np.linalg.matrix_power(A, k) / math.factorial(k) for k in range(5))
    psi = psi0
    cur = chi.copy()
    for n in range(10):
        psi = O.etrs_step(sysd, psi, 0.1 * n)
        cur = T @ T @ cur
        assert np.allclose(psi[0, :, 0, 0, 0] * math.sqrt(grid.volume), cur, atol=1e-14)


@pytest.mark.parametrize("xc", [0, 1])
def test_larmor_precession_closed_form(xc):
    """dM/dt = 2 mu_B B x M (Eqs. magrot, MOmega): M rotates about B at |B| a.u., with or without XC."""
    grid = O.Grid((4, 4, 4), (3.0, 3.0, 3.0))
    B = np.array([0.8, 0.0, 0.6]) * 0.5
    dt = 0.02
    sysd = _free_system(grid.n, grid.L, B0=tuple(B), xc=xc, hartree=1, dt=dt)
    th = 1.0
    psi, _ = _plane_wave(grid, (0, 0, 0), np.array([math.cos(th / 2), math.sin(th / 2)]))
    M0 = O.observables(sysd, psi, 0.0)[2:5]
    t = 0.0
    for _ in range(200):
        psi = O.etrs_step(sysd, psi, t)
        t += dt
    M = O.observables(sysd, psi, t)[2:5]
    ref = _rotation(B, np.linalg.norm(B) * t) @ M0
    tol = 1e-9 if xc == 0 else 5e-4
    assert np.allclose(M, ref, atol=tol)
    # sense: the first step moves M along B x M
    psi1 = O.etrs_step(sysd, _plane_wave(grid, (0, 0, 0), np.array([math.cos(th / 2), math.sin(th / 2)]))[0], 0.0)
    dM = O.observables(sysd, psi1, dt)[2:5] - M0
    assert np.dot(dM, np.cross(B, M0)) > 0


def test_larmor_xc_error_is_second_order():
    grid = O.Grid((4, 4, 4), (3.0, 3.0, 3.0))
    B = np.array([0.0, 0.6, 0.8]) * 0.5
    errs = []
    for dt in (0.04, 0.02):
        sysd = _free_system(grid.n, grid.L, B0=tuple(B), xc=1, hartree=1, dt=dt)
        psi, _ = _plane_wave(grid, (0, 0, 0), np.array([math.cos(0.4), math.sin(0.4)]))
        M0 = O.observables(sysd, psi, 0.0)[2:5]
        t = 0.0
        for _ in range(int(round(2.0 / dt))):
            psi = O.etrs_step(sysd, psi, t)
            t += dt
        M = O.observables(sysd, psi, t)[2:5]
        errs.append(np.linalg.norm(M - _rotation(B, np.linalg.norm(B) * t) @ M0))
    assert 3.0 < errs[0] / errs[1] < 5.0


# ---------------------------------------------------------------- propagator pins
def test_plane_wave_exact_phase():
    """Field-free plane wave: psi_n = [T_4(-i eps dt/2)]^(2n) psi_0, -> exp(-i eps t) as K grows."""
    grid = O.Grid((6, 6, 6), (5.0, 5.0, 5.0))
    psi0, eps = _plane_wave(grid, (1, -2, 1), np.array([1.0, 0.0]))
    dt = 0.05
    sysd = _free_system(grid.n, grid.L, dt=dt)
    psi = psi0
    for n in range(1, 9):
        psi = O.etrs_step(sysd, psi, 0.0)
        assert np.allclose(psi, _taylor_scalar(-1j * eps * dt / 2, 4) ** (2 * n) * psi0, atol=1e-14)
    sysd16 = _free_system(grid.n, grid.L, dt=dt, K=16)
    psi = psi0
    for n in range(8):
        psi = O.etrs_step(sysd16, psi, 0.0)
    assert np.allclose(psi, np.exp(-1j * eps * 8 * dt) * psi0, atol=1e-13)


def test_polarised_uniform_gas_phase_with_xc():
    """Fully polarised uniform state with XC+Hartree: v_H = 0 and the phase rate is eps + v_up,
    v_up = -(6 n/pi)^(1/3), n = 1/Omega."""
    grid = O.Grid((4, 4, 4), (3.0, 3.0, 3.0))
    chi = np.array([math.cos(0.35), math.sin(0.35) * np.exp(0.7j)])
    psi0, eps = _plane_wave(grid, (1, 0, 0), chi)
    dt = 0.05
    sysd = _free_system(grid.n, grid.L, dt=dt, xc=1, hartree=1)
    E = eps - (6.0 / math.pi / grid.volume) ** (1 / 3)
    psi = psi0
    for n in range(1, 6):
        psi = O.etrs_step(sysd, psi, 0.0)
        assert np.allclose(psi, _taylor_scalar(-1j * E * dt / 2, 4) ** (2 * n) * psi0, atol=1e-13)


def _dense_H(sysd, v, b):
    """Hamiltonian as a dense matrix built from DFT matrices, 2x2 blocks and projector outer products."""
    n = sysd.grid.n
    N = sysd.grid.N

    def dft(m):
        j = np.arange(m)
        return np.exp(-2j * math.pi * np.outer(j, j) / m)
    F = np.kron(np.kron(dft(n[0]), dft(n[1])), dft(n[2]))
    g2 = sysd.grid.g2().ravel()
    T = np.linalg.inv(F) @ np.diag(0.5 * g2) @ F
    H = np.zeros((2 * N, 2 * N), dtype=complex)
    H[:N, :N] += T + np.diag(v.ravel() + b[2].ravel())
    H[N:, N:] += T + np.diag(v.ravel() - b[2].ravel())
    H[:N, N:] += np.diag(b[0].ravel() - 1j * b[1].ravel())
    H[N:, :N] += np.diag(b[0].ravel() + 1j * b[1].ravel())
    for ap in sysd.projs:
        for p in range(ap.beta.shape[0]):
            vec = np.zeros(2 * N, dtype=complex)
            vec[ap.idx] = ap.beta[p, 0]
            vec[N + ap.idx] = ap.beta[p, 1]
            H += ap.energy[p] * sysd.grid.dV * np.outer(vec, vec.conj())
    return H


def test_frozen_field_step_matches_dense_matrix():
    """Non-self-consistent step equals the dense Taylor polynomial squared; K=16 tends to expm."""
    w = I.make_system(n=(6, 6, 6), L=(6.0,) * 3, nstates=2, natoms=1, case=6, xc=0, hartree=0,
                      bfield=I.BField(B0=(0.2, -0.1, 0.3)), dt=0.05)
    sysd = O.system_from_workload(w)
    F = O.fields_from_density(sysd, O.spin_density(w.psi0, sysd.occ), 0.0)
    H = _dense_H(sysd, F.v, F.b)
    assert np.allclose(H, H.conj().T, atol=1e-12)
    N = sysd.grid.N
    x0 = w.psi0.reshape(2, 2 * N).T
    A = -1j * 0.025 * H
    T = sum(np.linalg.matrix_power(A, k) / math.factorial(k) for k in range(5))
    ref = T @ T @ x0
    got = O.etrs_step(sysd, w.psi0, 0.0).reshape(2, 2 * N).T
    assert np.allclose(got, ref, atol=1e-12)
    sysd.K = 16
    psi = w.psi0
    for _ in range(4):
        psi = O.etrs_step(sysd, psi, 0.0)
    ref = scipy.linalg.expm(-1j * 0.2 * H) @ x0
    assert np.allclose(psi.reshape(2, 2 * N).T, ref, atol=1e-10)


def test_norm_drift_within_taylor_bound():
    """|T_4(i x)|^2 = 1 - x^6/72 + x^8/576 bounds the per-step norm change on a frozen field."""
    w = I.make_system(n=(6, 6, 6), L=(6.0,) * 3, nstates=2, natoms=1, case=6, xc=0, hartree=0,
                      dt=0.05)
    sysd = O.system_from_workload(w)
    F = O.fields_from_density(sysd, O.spin_density(w.psi0, sysd.occ), 0.0)
    ev = np.linalg.eigvalsh(_dense_H(sysd, F.v, F.b))
    x = 0.025 * np.abs(ev)
    g = 1 - x ** 6 / 72 + x ** 8 / 576
    lo, hi = np.min(g) ** 2, np.max(g) ** 2
    psi = O.etrs_step(sysd, w.psi0, 0.0)
    norms = np.real(np.sum(psi.conj() * psi, axis=(1, 2, 3, 4))) * sysd.grid.dV
    assert np.all(norms >= lo - 1e-13) and np.all(norms <= hi + 1e-13)


# ---------------------------------------------------------------- whole-step invariants
def test_su2_covariance_without_soc():
    """Rotating psi_0 and B by the same SU(2)/SO(3) pair rotates M; n and E do not change (Sec. 3.1)."""
    bf = I.BField(B0=(0.05, 0.02, -0.04))
    w = I.make_system(n=(8, 8, 8), L=(7.0,) * 3, nstates=3, natoms=1, case=8, lambda_so=0.0,
                      bfield=bf, dt=0.05)
    sysd = O.system_from_workload(w)
    axis = np.array([0.3, -0.5, 0.81]); axis /= np.linalg.norm(axis)
    ang = 0.9
    sig = [np.array([[0, 1], [1, 0]]), np.array([[0, -1j], [1j, 0]]), np.diag([1.0, -1.0])]
    U = scipy.linalg.expm(-0.5j * ang * sum(a * s for a, s in zip(axis, sig)))
    R = _rotation(axis, ang)
    psiR = np.einsum("st,itxyz->isxyz", U, w.psi0)
    wR = I.make_system(n=(8, 8, 8), L=(7.0,) * 3, nstates=3, natoms=1, case=8, lambda_so=0.0,
                       bfield=I.BField(B0=tuple(R @ np.array(bf.B0))), dt=0.05)
    sysR = O.system_from_workload(wR)
    pa, obs_a = O.run(sysd, w.psi0, 3)
    pb, obs_b = O.run(sysR, psiR, 3)
    na, _ = O.charge_and_magnetization(O.spin_density(pa, sysd.occ))
    nb, _ = O.charge_and_magnetization(O.spin_density(pb, sysd.occ))
    assert np.allclose(na, nb, atol=1e-12)
    assert np.allclose(obs_a[:, 5], obs_b[:, 5], atol=1e-11)
    for row_a, row_b in zip(obs_a, obs_b):
        assert np.allclose(R @ row_a[2:5], row_b[2:5], atol=1e-12)


def test_energy_conservation_second_order():
    """Static field: total energy drift falls ~4x when dt halves (ETRS is second order)."""
    drifts = []
    for dt in (0.04, 0.02):
        w = I.make_system(n=(8, 8, 8), L=(7.0,) * 3, nstates=3, natoms=1, case=9, dt=dt,
                          bfield=I.BField(B0=(0.0, 0.0, 0.05)))
        sysd = O.system_from_workload(w)
        _, obs = O.run(sysd, w.psi0, int(round(0.4 / dt)))
        drifts.append(abs(obs[-1, 5] - obs[0, 5]))
    assert drifts[1] < drifts[0]
    assert 2.5 < drifts[0] / drifts[1] < 6.0


def test_energy_conservation_second_order_with_correlation():
    """xc = 2 (exchange + PW92): the energy still drifts only at second order in dt, which holds
    only if the correlation potentials are the functional derivative of int n eps_c."""
    drifts = []
    for dt in (0.04, 0.02):
        w = I.make_system(n=(8, 8, 8), L=(7.0,) * 3, nstates=3, natoms=1, case=9, dt=dt, xc=2,
                          bfield=I.BField(B0=(0.0, 0.0, 0.05)))
        sysd = O.system_from_workload(w)
        _, obs = O.run(sysd, w.psi0, int(round(0.4 / dt)))
        drifts.append(abs(obs[-1, 5] - obs[0, 5]))
    assert 2.5 < drifts[0] / drifts[1] < 6.0


def test_charge_conserved_and_collinear_limit():
    """N_e is conserved; spin-z product states in B || z with no SOC stay unmixed (collinear limit)."""
    w = I.make_system(n=(8, 8, 8), L=(7.0,) * 3, nstates=2, natoms=1, case=10, lambda_so=0.0,
                      bfield=I.BField(B0=(0.0, 0.0, 0.1)))
    psi0 = w.psi0.copy()
    psi0[0, 1] = 0.0
    psi0[1, 0] = 0.0
    for i in range(2):
        psi0[i] /= math.sqrt(np.sum(np.abs(psi0[i]) ** 2) * (7.0 ** 3 / 512))
    sysd = O.system_from_workload(w)
    psi, obs = O.run(sysd, psi0, 3)
    # projectors sum to a spin-diagonal operator only up to rounding
    assert np.max(np.abs(psi[0, 1])) < 1e-15 * np.max(np.abs(psi[0, 0]))
    assert np.max(np.abs(psi[1, 0])) < 1e-15 * np.max(np.abs(psi[1, 1]))
    assert np.allclose(obs[:, 1], obs[0, 1], rtol=1e-12)
    assert np.allclose(obs[:, 2:4], 0, atol=1e-14)


# ---------------------------------------------------------------- k-points (Sec. 2.1, Sec. 5)
def test_bloch_free_electron_exact_phase():
    """u = const with Bloch vector k: H_k u = |k|^2/2 u, so each half step multiplies by
    T_4(-i |k|^2 dt/4) exactly (no potential, no XC)."""
    grid = O.Grid((8, 8, 8), (5.0, 6.0, 7.0))
    sysd = _free_system(grid.n, grid.L, dt=0.07)
    k = np.array([0.31, -0.44, 0.27])
    sysd.kvec = k[None, :]
    psi0 = np.zeros((1, 2) + grid.n, complex)
    psi0[0, 0] = 0.6 / math.sqrt(grid.volume)
    psi0[0, 1] = 0.8j / math.sqrt(grid.volume)
    eps = 0.5 * float(k @ k)
    g = _taylor_scalar(-1j * eps * 0.035, 4)
    psi = psi0
    for nstep in range(5):
        psi = O.etrs_step(sysd, psi, 0.07 * nstep)
        assert np.allclose(psi, psi0 * g ** (2 * (nstep + 1)), atol=1e-14)


def _kpoint_primitive(lam=0.05):
    return I.make_system(n=(12, 12, 12), L=(6.0, 6.0, 6.0), nstates=2, natoms=1, case=48,
                         lambda_so=lam, full_spinors=True, dt=0.04)


def test_supercell_gamma_equals_two_kpoints():
    """A 2x1x1 supercell at Gamma holding the states exp(i k.r) u_k (k = 0 and pi/L_x, tiled, with
    1/sqrt 2) evolves exactly as the primitive cell sampled at those two k-points with weights
    1/2: kinetic |G + k|^2, projector Bloch phases, k-weighted density, Hartree and exchange."""
    w = _kpoint_primitive()
    prim = O.system_from_workload(w)
    Lx = w.L[0]
    kx = math.pi / Lx
    S = w.nstates
    u = np.concatenate([w.psi0, np.roll(w.psi0[::-1], 3, axis=-1)])   # 2S periodic parts
    kv = np.zeros((2 * S, 3))
    kv[S:, 0] = kx
    prim.kvec = kv
    prim.occ = np.full(2 * S, 0.5)
    sup_grid = O.Grid((24, 12, 12), (2 * Lx, 6.0, 6.0))
    pos = np.concatenate([w.positions, w.positions + np.array([Lx, 0, 0])])
    sup = O.System(grid=sup_grid, occ=np.ones(2 * S), v_ext=np.concatenate([w.v_ext, w.v_ext], axis=0),
                   projs=O.build_projectors(sup_grid, pos, w.channels, w.r_sphere),
                   bfield=prim.bfield, xc=1, hartree=1, dt=w.dt, K=4)
    x = sup_grid.axis(0)
    def to_super(uu):
        big = np.concatenate([uu, uu], axis=2) / math.sqrt(2.0)
        ph = np.exp(1j * np.outer(kv[:, 0], x))                   # [2S, 24]
        return big * ph[:, None, :, None, None]
    psi_s = to_super(u)
    psi_p = u
    for n in range(2):
        psi_s = O.etrs_step(sup, psi_s, n * w.dt)
        psi_p = O.etrs_step(prim, psi_p, n * w.dt)
    assert np.max(np.abs(psi_s - to_super(psi_p))) < 1e-12 * np.max(np.abs(psi_s))
    obs_s = O.observables(sup, psi_s, 2 * w.dt)
    obs_p = O.observables(prim, psi_p, 2 * w.dt)
    # per-cell quantities: the supercell holds two cells
    assert np.allclose(obs_s[1:12], 2 * obs_p[1:12], rtol=1e-11, atol=1e-12)


def test_projector_bloch_phase_shift_by_reciprocal_vector():
    """(u, k) and (exp(-i G0.r) u, k + G0) are the same Bloch state, so V_NL must map them to
    results related by the same factor: the projector phases use the displacement from the atom,
    and the atom position and image drop out.  (The kinetic term is pinned by the free-electron
    and supercell tests; on a finite FFT grid a shift by G0 wraps the highest frequencies.)"""
    w = _kpoint_primitive()
    sysd = O.system_from_workload(w)
    k = np.tile(np.array([0.2, -0.3, 0.45]), (w.nstates, 1))
    G0 = 2 * math.pi * np.array([1, -2, 1]) / np.array(w.L)
    X, Y, Z = np.meshgrid(*[sysd.grid.axis(d) for d in range(3)], indexing="ij")
    ph = np.exp(-1j * (G0[0] * X + G0[1] * Y + G0[2] * Z))
    a = O.apply_nonlocal(w.psi0, sysd.projs, sysd.grid, k)
    b = O.apply_nonlocal(w.psi0 * ph, sysd.projs, sysd.grid, k + G0)
    assert np.max(np.abs(a)) > 1e-3
    assert np.max(np.abs(b - a * ph)) < 1e-13 * np.max(np.abs(a))
    # and V_NL stays Hermitian with Bloch phases
    x = w.psi0
    y = np.roll(w.psi0, 2, axis=-1)
    lhs = np.vdot(x, O.apply_nonlocal(y, sysd.projs, sysd.grid, k))
    rhs = np.vdot(O.apply_nonlocal(x, sysd.projs, sysd.grid, k), y)
    assert abs(lhs - rhs) < 1e-13 * abs(lhs)


# ---------------------------------------------------------------- laser (Sec. 4.7)
def _laser_packet_system(dt, E0):
    grid = O.Grid((28, 28, 40), (14.0, 14.0, 20.0))   # packet tails negligible at the faces
    sysd = _free_system(grid.n, grid.L, dt=dt)
    sysd.laser = O.LaserSpec([O.LaserPulseSpec(A=E0, omega=0.0, t0=0.0, tau=1e9, pol=(0.0, 0.0, 1.0))])
    X, Y, Z = np.meshgrid(grid.axis(0), grid.axis(1), grid.axis(2), indexing="ij")
    c = [grid.L[d] / 2 for d in range(3)]
    g = np.exp(-((X - c[0]) ** 2 + (Y - c[1]) ** 2 + (Z - c[2]) ** 2) / 2.0)
    g = g / math.sqrt(np.sum(g * g) * grid.dV)
    psi = np.stack([g, 0 * g])[None].astype(complex)
    return sysd, psi, (X - c[0], Y - c[1], Z - c[2])


def test_laser_ehrenfest_uniform_acceleration():
    """A packet at rest in a static uniform field: for a linear potential Ehrenfest's theorem is
    exact, so <r> - c = -E t^2/2 (force -E on a charge -1); pins the sign and size of v_E."""
    E0, T = 0.5, 1.2
    sysd, psi, rel = _laser_packet_system(0.04, E0)
    p, obs = O.run(sysd, psi, 30)
    n, _ = O.charge_and_magnetization(O.spin_density(p, sysd.occ))
    dV = sysd.grid.dV
    disp = [float(np.sum(n * r) * dV) for r in rel]
    assert abs(disp[2] + 0.5 * E0 * T * T) < 1e-6
    # transverse: zero but for the packet tail on the unpaired face point x - c = -L/2
    assert abs(disp[0]) < 1e-7 and abs(disp[1]) < 1e-7
    # the energy includes int v_E n: conserved while kinetic energy grows by E^2 T^2/2
    assert abs(obs[-1, 5] - obs[0, 5]) < 1e-6
    assert abs(obs[-1, 6] - obs[0, 6] - 0.5 * E0 * E0 * T * T) < 1e-5
    assert abs(obs[-1, 7] - E0 * disp[2]) < 1e-12


@pytest.mark.parametrize("lam", [0.0, 0.05])
def test_laser_rotates_magnetisation_only_through_soc(lam):
    """Without spin-orbit coupling the electric pulse acts on the charge only: the collinear
    product states keep M along its initial direction (to rounding; |M| follows the Taylor norm
    error).  With SOC the pulse turns M (Sec. 4.7, Eq. SOtorque)."""
    las = [I.LaserPulse(A=0.5, omega=0.4, t0=0.3, tau=0.3, pol=(0.0, 0.0, 1.0))]
    w = I.make_system(n=(12, 12, 12), L=(9.0,) * 3, nstates=3, natoms=2, case=41, lambda_so=lam,
                      dt=0.05, laser=las, localized=1.8, full_spinors=False)
    sysd = O.system_from_workload(w)
    _, obs = O.run(sysd, w.psi0, 12)
    n0 = obs[0, 2:5] / np.linalg.norm(obs[0, 2:5])
    perp = max(np.linalg.norm(np.cross(row[2:5], n0)) for row in obs)
    if lam == 0.0:
        assert perp < 1e-13
    else:
        assert perp > 1e-4


def test_velocity_gauge_ehrenfest_and_free_phase():
    """Velocity gauge: a packet at rest in a static field keeps its canonical momentum while its
    kinetic momentum grows as A(t) = -E t, so <r> - c = -E t^2/2 exactly, periodic boundaries and
    all; and a plane wave picks up exactly the Taylor factors of 1/2 |G + A(t)|^2 with A taken at
    t_n for the first two half steps and t_{n+1} for the third."""
    E0, T = 0.5, 1.2
    sysd, psi, rel = _laser_packet_system(0.04, E0)
    sysd.laser.gauge = "velocity"
    assert np.allclose(sysd.laser.A(0.7), [0.0, 0.0, -E0 * 0.7], atol=1e-14)
    p, obs = O.run(sysd, psi, 30)
    n, _ = O.charge_and_magnetization(O.spin_density(p, sysd.occ))
    disp = [float(np.sum(n * r) * sysd.grid.dV) for r in rel]
    assert abs(disp[2] + 0.5 * E0 * T * T) < 1e-6
    assert abs(obs[-1, 6] - obs[0, 6] - 0.5 * E0 * E0 * T * T) < 1e-5   # kinetic energy of the packet
    grid = O.Grid((8, 8, 8), (5.0, 5.0, 5.0))
    sysw = _free_system(grid.n, grid.L, dt=0.1)
    sysw.laser = O.LaserSpec([O.LaserPulseSpec(A=0.3, omega=0.9, t0=0.2, tau=0.4, phase=0.1,
                                               pol=(0.6, 0.0, 0.8))], "velocity")
    G = np.array([2 * math.pi / 5.0, 0.0, -2 * math.pi / 5.0])
    pw, _ = _plane_wave(grid, (1, 0, -1), np.array([1.0, 0.0]))
    cur = pw
    amp = 1.0 + 0j
    for nstep in range(4):
        t = 0.1 * nstep
        e_n = 0.5 * float(np.sum((G + sysw.laser.A(t)) ** 2))
        e_p = 0.5 * float(np.sum((G + sysw.laser.A(t + 0.1)) ** 2))
        # phi = T(e_n) psi_n, psi_{n+1} = T(e_{n+1}) phi
        amp *= _taylor_scalar(-1j * e_p * 0.05, 4) * _taylor_scalar(-1j * e_n * 0.05, 4)
        cur = O.etrs_step(sysw, cur, t)
        assert np.allclose(cur, amp * pw, atol=1e-13)


# ---------------------------------------------------------------- initialisation and ground state
def test_dm_initialization_voronoi_and_moments():
    """Every point takes its nearest atom (brute force over all atoms and periodic images), the
    ComputeSpinDensity map of that atom's moment per electron, and for compact atomic densities
    the integrated charge and moment are those of the atoms."""
    grid = O.Grid((10, 10, 10), (9.0, 9.0, 9.0))
    pos = np.array([[2.0, 2.5, 2.0], [6.5, 6.0, 7.0], [2.2, 7.0, 6.0]])
    atoms = [O.AtomDensitySpec(6.0, 0.7, (0.0, 0.0, 3.0)), O.AtomDensitySpec(4.0, 0.6, (1.2, -1.6, 0.0)),
             O.AtomDensitySpec(5.0, 0.65, (0.0, 2.0, -2.0))]
    rho = O.dm_initialization(grid, pos, atoms)
    X, Y, Z = np.meshgrid(*[grid.axis(d) for d in range(3)], indexing="ij")
    for idx in [(0, 0, 0), (3, 4, 2), (7, 6, 8), (2, 8, 6), (9, 9, 9), (5, 5, 5)]:
        r = np.array([X[idx], Y[idx], Z[idx]])
        best, owner = np.inf, -1
        for a, R in enumerate(pos):
            for img in np.ndindex(3, 3, 3):
                d = r - R - 9.0 * (np.array(img) - 1)
                if d @ d < best:
                    best, owner = d @ d, a
        sp = atoms[owner]
        n = sp.Z * (2 * math.pi * sp.sigma ** 2) ** -1.5 * math.exp(-best / (2 * sp.sigma ** 2))
        m = np.array(sp.moment) / sp.Z
        expect = n * np.array([(1 + m[2]) / 2, (1 - m[2]) / 2, m[0] / 2, -m[1] / 2])
        assert np.allclose(rho[(slice(None),) + idx], expect, rtol=1e-13, atol=1e-300)
    n, m = O.charge_and_magnetization(rho)
    assert abs(n.sum() * grid.dV - 15.0) < 0.02
    assert np.allclose(m.reshape(3, -1).sum(1) * grid.dV, [1.2, 0.4, 1.0], atol=0.01)


def test_orthonormalize_complex_overlap():
    rng = np.random.default_rng(3)
    psi = rng.standard_normal((4, 2, 3, 3, 3)) + 1j * rng.standard_normal((4, 2, 3, 3, 3))
    out = O.orthonormalize(psi, 0.7)
    f, g = out.reshape(4, -1), psi.reshape(4, -1)
    assert np.abs(0.7 * f.conj() @ f.T - np.eye(4)).max() < 1e-13
    # same span: the projector onto the states is unchanged
    P1 = f.T @ np.linalg.pinv(f.T)
    P0 = g.T @ np.linalg.pinv(g.T)
    assert np.abs(P1 - P0).max() < 1e-12


def test_ground_state_reaches_lowest_eigenvectors_without_interactions():
    """xc = 0, no Hartree, static B, SOC projectors: imaginary-time iterations converge to the
    lowest eigenvectors of the dense Hamiltonian (band energy and spanned space)."""
    # two states: the spectrum of this system has a 0.56 Ha gap above its second level
    w = I.make_system(n=(6, 6, 6), L=(5.0,) * 3, nstates=2, natoms=1, case=61, xc=0, hartree=0,
                      bfield=I.BField(B0=(0.0, 0.05, 0.1)), full_spinors=True)
    sysd = O.system_from_workload(w)
    F = O.fields_from_density(sysd, O.spin_density(w.psi0, sysd.occ), 0.0)
    Hd = _dense_H(sysd, F.v, F.b)
    evals, evecs = np.linalg.eigh(Hd)
    assert evals[2] - evals[1] > 0.5
    psi, E = O.ground_state(sysd, w.psi0, 400, 0.1)
    assert abs(E[-1] - evals[:2].sum()) < 1e-9
    assert np.all(np.diff(E[5:]) < 1e-12)                   # the energy decreases
    f = psi.reshape(2, -1).T * math.sqrt(sysd.grid.dV)
    P = f @ f.conj().T
    Q = evecs[:, :2] @ evecs[:, :2].conj().T
    assert np.abs(P - Q).max() < 1e-6


def test_ground_state_with_kpoints_reaches_lowest_bands_of_each_k():
    """Two k-points x two states, no interaction: each k-run converges to the two lowest
    eigenvectors of its own H_k (a dense matrix from the oracle's H on basis vectors), and the
    energy to the weighted band sum; states of different k are not mixed."""
    w = I.make_system(n=(6, 6, 6), L=(5.0,) * 3, nstates=4, natoms=1, case=61, xc=0, hartree=0,
                      bfield=I.BField(B0=(0.0, 0.05, 0.1)), full_spinors=True)
    k1 = np.array([0.35, -0.2, 0.15])
    w.kvec = np.array([[0.0, 0.0, 0.0], [0.0, 0.0, 0.0], k1, k1])
    w.occ = np.full(4, 0.5)
    sysd = O.system_from_workload(w)
    assert O.k_blocks(sysd.kvec, 4) == [(0, 2), (2, 4)]
    F = O.fields_from_density(sysd, O.spin_density(w.psi0, sysd.occ), 0.0)
    N = sysd.grid.N
    dense = {}
    for k in (np.zeros(3), k1):
        basis = np.eye(2 * N, dtype=complex).reshape((2 * N, 2) + tuple(sysd.grid.n))
        sk = O.System(**{**vars(sysd), "kvec": np.tile(k, (2 * N, 1)), "occ": np.ones(2 * N)})
        Hk = O.apply_hamiltonian(sk, basis, F).reshape(2 * N, 2 * N).T
        assert np.abs(Hk - Hk.conj().T).max() < 1e-12
        dense[tuple(k)] = np.linalg.eigh(Hk)
    psi, E = O.ground_state(sysd, w.psi0, 800, 0.1)
    band = 0.0
    for (i0, i1), k in (((0, 2), np.zeros(3)), ((2, 4), k1)):
        evals, evecs = dense[tuple(k)]
        assert evals[2] - evals[1] > 0.2   # e^(-0.1 x 0.2 x 800) ~ 1e-7 left of the next band
        band += 0.5 * evals[:2].sum()
        f = psi[i0:i1].reshape(2, -1).T * math.sqrt(sysd.grid.dV)
        P = f @ f.conj().T
        Q = evecs[:, :2] @ evecs[:, :2].conj().T
        assert np.abs(P - Q).max() < 1e-6
    assert abs(E[-1] - band) < 1e-9


def test_ground_state_self_consistent_with_exchange_and_hartree():
    """With exchange and Hartree on, the converged states are eigenvectors of the Hamiltonian built
    from their own density (subspace residual H psi - psi Lambda), and the energy settles."""
    w = I.make_system(n=(6, 6, 6), L=(5.0,) * 3, nstates=2, natoms=1, case=61, xc=1, hartree=1,
                      bfield=I.BField(B0=(0.0, 0.05, 0.1)), full_spinors=True)
    sysd = O.system_from_workload(w)
    psi, E = O.ground_state(sysd, w.psi0, 400, 0.1)
    F = O.fields_from_density(sysd, O.spin_density(psi, sysd.occ), 0.0)
    f = psi.reshape(2, -1)
    hf = O.apply_hamiltonian(sysd, psi, F).reshape(2, -1)
    Lam = sysd.grid.dV * f.conj() @ hf.T
    assert np.abs(Lam - Lam.conj().T).max() < 1e-12
    assert np.abs(hf - Lam.T @ f).max() < 1e-6 * np.abs(hf).max()
    assert abs(E[-1] - E[-2]) < 1e-12


def test_pw92_jvp_matches_central_differences():
    """The complex-step tangent of the correlation potentials equals central differences of
    pw92_correlation (a different method), including strongly polarised points."""
    rng = np.random.default_rng(5)
    n = 10.0 ** rng.uniform(-4, 0.5, 40)
    m = rng.standard_normal((3, 40))
    m *= (rng.uniform(0.0, 0.97, 40) * n / np.sqrt(np.sum(m * m, axis=0)))
    dn = rng.standard_normal(40) * n
    dm = rng.standard_normal((3, 40)) * n
    h = 1e-6
    vp, bp, _ = O.pw92_correlation(n + h * dn, m + h * dm)
    vm, bm, _ = O.pw92_correlation(n - h * dn, m - h * dm)
    dv, db = O.pw92_correlation_jvp(n, m, dn, dm)
    fv, fb = (vp - vm) / (2 * h), (bp - bm) / (2 * h)
    assert np.all(np.abs(dv - fv) <= 1e-6 * np.abs(fv) + 1e-9)
    assert np.all(np.abs(db - fb) <= 1e-6 * np.abs(fb) + 1e-9)


def test_pw92_potentials_have_a_symmetric_jacobian():
    """vbar_c = dE/dn and bmag_c = dE/d|m| are derivatives of one energy density, so
    d vbar/d|m| = d bmag/dn: the tangent along |m| of vbar equals the tangent along n of
    bmag (m along z, so that b_c = bmag e_z)."""
    rng = np.random.default_rng(6)
    n = rng.uniform(0.01, 2.0, 25)
    mz = rng.uniform(0.05, 0.9, 25) * n
    m = np.stack([np.zeros(25), np.zeros(25), mz])
    one, zero = np.ones(25), np.zeros(25)
    dv_mu, _ = O.pw92_correlation_jvp(n, m, zero, np.stack([zero, zero, one]))
    _, db_n = O.pw92_correlation_jvp(n, m, one, np.zeros((3, 25)))
    assert np.allclose(dv_mu, db_n[2], rtol=1e-11, atol=1e-14)


def test_lsda_fields_jvp_matches_central_differences():
    """Tangent of the self-consistent fields (Hartree + exchange + PW92 correlation) along a
    density perturbation, against central differences of the fields themselves."""
    w = I.make_system(n=(6, 6, 6), L=(6.0,) * 3, nstates=3, natoms=0, case=62, xc=2)
    sysd = O.system_from_workload(w)
    rho = O.spin_density(w.psi0, sysd.occ)
    rng = np.random.default_rng(7)
    dpsi = rng.standard_normal(w.psi0.shape) + 1j * rng.standard_normal(w.psi0.shape)
    drho = O._density_jvp(w.psi0, dpsi, sysd.occ)
    dv, db = O._fields_jvp(sysd, rho, drho, np.zeros(3))
    h = 1e-6
    Fp = O.fields_from_density(sysd, rho + h * drho, 0.0)
    Fm = O.fields_from_density(sysd, rho - h * drho, 0.0)
    fv, fb = (Fp.v - Fm.v) / (2 * h), (Fp.b - Fm.b) / (2 * h)
    assert np.abs(dv - fv).max() < 1e-7 * np.abs(fv).max()
    assert np.abs(db - fb).max() < 1e-7 * np.abs(fb).max()


# ---------------------------------------------------------------- gradient oracle
def test_tangent_linear_gradient_lsda_matches_central_differences():
    """With PW92 correlation in the self-consistent fields (xc = 2), the forward-mode pulse
    gradient of the discrete trajectory equals central differences of it."""
    bf = I.BField(pulses=I.circular_pulses([0.1, 0.2], [0.5, 1.0], 0.05, 0.1))
    w = I.make_system(n=(6, 6, 6), L=(6.0,) * 3, nstates=2, natoms=1, case=11, bfield=bf, dt=0.05,
                      xc=2)
    sysd = O.system_from_workload(w)
    nsteps = 4
    g = O.mz_gradient_tangent_linear(sysd, w.psi0, nsteps)
    h = 1e-5
    for k in (0, 3):
        vals = []
        for sgn in (1, -1):
            pulses = [O.PulseSpec(**vars(p)) for p in sysd.bfield.pulses]
            if k < 2:
                pulses[k].A += sgn * h
            else:
                pulses[k - 2].omega += sgn * h
            s2 = O.System(**{**vars(sysd), "bfield": O.FieldSpec(sysd.bfield.B0, pulses)})
            psi, _ = O.run(s2, w.psi0, nsteps, record=False)
            vals.append(O.total_mz(s2, psi))
        fd = (vals[0] - vals[1]) / (2 * h)
        assert abs(fd - g[k]) < 1e-7 * max(1.0, abs(g[k])) + 1e-9, (k, fd, g[k])


def test_tangent_linear_gradient_velocity_gauge_matches_central_differences():
    """Periodic system with two k-points under a velocity-gauge laser: the forward-mode B-pulse
    gradient of the discrete trajectory equals central differences of it."""
    bf = I.BField(pulses=I.circular_pulses([0.1, 0.2], [0.5, 1.0], 0.05, 0.1))
    laser = [I.LaserPulse(A=0.5, omega=0.4, t0=0.1, tau=0.4, phase=0.3, pol=(0.2, -0.3, 0.93))]
    w = I.make_system(n=(6, 6, 6), L=(6.0,) * 3, nstates=2, natoms=1, case=11, bfield=bf, dt=0.05,
                      laser=laser, full_spinors=True)
    w.laser_gauge = "velocity"
    w.kvec = np.array([[0.0, 0.0, 0.0], [0.3, -0.2, 0.1]])
    w.occ = np.full(2, 0.5)
    sysd = O.system_from_workload(w)
    nsteps = 4
    g = O.mz_gradient_tangent_linear(sysd, w.psi0, nsteps)
    h = 1e-5
    for k in (1, 2):
        vals = []
        for sgn in (1, -1):
            pulses = [O.PulseSpec(**vars(p)) for p in sysd.bfield.pulses]
            if k < 2:
                pulses[k].A += sgn * h
            else:
                pulses[k - 2].omega += sgn * h
            s2 = O.System(**{**vars(sysd), "bfield": O.FieldSpec(sysd.bfield.B0, pulses)})
            psi, _ = O.run(s2, w.psi0, nsteps, record=False)
            vals.append(O.total_mz(s2, psi))
        fd = (vals[0] - vals[1]) / (2 * h)
        assert abs(fd - g[k]) < 1e-7 * max(1.0, abs(g[k])) + 1e-9, (k, fd, g[k])


def test_tangent_linear_gradient_matches_central_differences():
    bf = I.BField(pulses=I.circular_pulses([0.1, 0.2], [0.5, 1.0], 0.05, 0.1))
    w = I.make_system(n=(6, 6, 6), L=(6.0,) * 3, nstates=2, natoms=1, case=11, bfield=bf, dt=0.05)
    sysd = O.system_from_workload(w)
    nsteps = 6
    g = O.mz_gradient_tangent_linear(sysd, w.psi0, nsteps)
    h = 1e-5
    for k in range(4):
        vals = []
        for sgn in (1, -1):
            pulses = [O.PulseSpec(**vars(p)) for p in sysd.bfield.pulses]
            if k < 2:
                pulses[k].A += sgn * h
            else:
                pulses[k - 2].omega += sgn * h
            s2 = O.System(**{**vars(sysd), "bfield": O.FieldSpec(sysd.bfield.B0, pulses)})
            psi, _ = O.run(s2, w.psi0, nsteps, record=False)
            vals.append(O.total_mz(s2, psi))
        fd = (vals[0] - vals[1]) / (2 * h)
        assert abs(fd - g[k]) < 1e-7 * max(1.0, abs(g[k])) + 1e-9, (k, fd, g[k])
