"""Parity of the HIP path (through the C ABI) with the CPU FP64 oracle.

FP64 bar: relative error <= 1e-10 in n, m and energies (trajectories), <= 1e-12 for a single
H application.  FP32-mixed bar: <= 1e-5 relative over the tiny trajectory.
"""
import math
import sys

import numpy as np
import pytest

from oracle import nct_oracle as O
from paper_2506_21908_amd import inputs as I
from parity_metrics import max_rel, nm_errors

pytestmark = pytest.mark.gpu


def say(msg):
    print(f"[case] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def nct_mod():
    from paper_2506_21908_amd import nct
    return nct


def rel(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def random_fields(n, seed):
    rng = np.random.default_rng(seed)
    f = rng.uniform(-0.5, 0.5, (4,) + tuple(n))
    return f


# ------------------------------------------------------------------ single H application
@pytest.mark.parametrize("n,S", [((8, 8, 8), 3), ((12, 16, 12), 5), ((16, 8, 16), 2),
                                 ((24, 16, 24), 3), ((16, 16, 16), 4), ((32, 32, 32), 2),
                                 ((48, 48, 48), 2), ((64, 64, 64), 1), ((96, 96, 96), 1)])
def test_apply_hamiltonian_frozen_fields(torch_cuda, n, S):
    """H psi = T psi + [v + b.sigma] psi with frozen random fields, no projectors."""
    torch = torch_cuda
    nct = nct_mod()
    say(f"apply_H frozen n={n} S={S}")
    L = tuple(0.45 * v for v in n)
    w = I.make_system(n=n, L=L, nstates=S, case=20, natoms=0)
    F = random_fields(n, 1)
    sysd = O.system_from_workload(w)
    ref = O.kinetic(w.psi0, sysd.grid) + O.apply_local(w.psi0, F[0], F[1:])
    s = nct.system_from_workload(w)
    s.set_potentials(fields=torch.from_numpy(F).cuda())
    psi = nct.states_to_device(w.psi0)
    hpsi = torch.empty_like(psi)
    s.apply_hamiltonian(psi, hpsi, 0.0)
    got = hpsi.cpu().numpy()
    assert rel(got, ref) < 1e-12


@pytest.mark.parametrize("n,S,natoms", [((16, 16, 16), 5, 2), ((24, 24, 24), 17, 3),
                                        ((12, 16, 12), 3, 1)])
def test_apply_hamiltonian_projectors(torch_cuda, n, S, natoms):
    """Kleinman-Bylander + spin-orbit projectors (MFMA contraction and scatter), ragged S."""
    torch = torch_cuda
    nct = nct_mod()
    say(f"apply_H projectors n={n} S={S} natoms={natoms}")
    L = tuple(0.5 * v for v in n)
    w = I.make_system(n=n, L=L, nstates=S, case=21, natoms=natoms, min_sep=5.0)
    F = random_fields(n, 2)
    sysd = O.system_from_workload(w)
    ref = (O.kinetic(w.psi0, sysd.grid) + O.apply_local(w.psi0, F[0], F[1:])
           + O.apply_nonlocal(w.psi0, sysd.projs, sysd.grid))
    s = nct.system_from_workload(w)
    s.set_potentials(fields=torch.from_numpy(F).cuda())
    psi = nct.states_to_device(w.psi0)
    hpsi = torch.empty_like(psi)
    s.apply_hamiltonian(psi, hpsi, 0.0)
    assert rel(hpsi.cpu().numpy(), ref) < 1e-12
    # nonlocal part alone (removes the kinetic and local parts from both sides)
    nl_ref = O.apply_nonlocal(w.psi0, sysd.projs, sysd.grid)
    nl_got = hpsi.cpu().numpy() - (O.kinetic(w.psi0, sysd.grid) + O.apply_local(w.psi0, F[0], F[1:]))
    assert rel(nl_got, nl_ref) < 1e-10


def test_apply_hamiltonian_projectors_mixed(torch_cuda):
    """FP32-mixed H application (FP32 FFT, local multiply and MFMA projector GEMMs)."""
    torch = torch_cuda
    nct = nct_mod()
    say("apply_H projectors mixed n=(16,16,16) S=5 natoms=2")
    n = (16, 16, 16)
    w = I.make_system(n=n, L=(8.0,) * 3, nstates=5, case=21, natoms=2, min_sep=5.0)
    F = random_fields(n, 2)
    sysd = O.system_from_workload(w)
    ref = (O.kinetic(w.psi0, sysd.grid) + O.apply_local(w.psi0, F[0], F[1:])
           + O.apply_nonlocal(w.psi0, sysd.projs, sysd.grid))
    s = nct.system_from_workload(w, precision=nct.NCT_FP32_MIXED)
    s.set_potentials(fields=torch.from_numpy(F).cuda())
    psi = nct.states_to_device(w.psi0, nct.NCT_FP32_MIXED)
    hpsi = torch.empty_like(psi)
    s.apply_hamiltonian(psi, hpsi, 0.0)
    err = rel(hpsi.cpu().numpy().astype(np.complex128), ref)
    say(f"  mixed rel err {err:.2e}")
    assert err < 2e-6


def test_density_and_scf_fields(torch_cuda):
    """rho_v (Eq. density4), exchange and Hartree fields and totals match the oracle."""
    torch = torch_cuda
    nct = nct_mod()
    say("density + fields, 16x12x16? -> (12,16,12)")
    bf = I.BField(B0=(0.01, -0.02, 0.03))
    w = I.make_system(n=(12, 16, 12), L=(7.0, 8.0, 7.0), nstates=5, case=22, natoms=2,
                      bfield=bf, min_sep=3.0, projectors=False)
    sysd = O.system_from_workload(w)
    rho_ref = O.spin_density(w.psi0, sysd.occ)
    F = O.fields_from_density(sysd, rho_ref, 0.7)
    s = nct.system_from_workload(w)
    psi = nct.states_to_device(w.psi0)
    rho = torch.empty((4,) + w.n, dtype=torch.float64, device="cuda")
    tot = s.density_magnetization(psi, 0.7, rho_v=rho, totals=True, update_fields=True)
    assert rel(rho.cpu().numpy(), rho_ref) < 1e-13
    n, m = O.charge_and_magnetization(rho_ref)
    dV = sysd.grid.dV
    assert abs(tot[0] - n.sum() * dV) < 1e-12 * abs(n.sum() * dV)
    assert np.allclose(tot[1:], m.reshape(3, -1).sum(1) * dV, atol=1e-12)
    fields = torch.empty((4,) + w.n, dtype=torch.float64, device="cuda")
    s.get_fields(0.7, fields)
    got = fields.cpu().numpy()
    assert rel(got[0], F.v) < 1e-12
    assert rel(got[1:], F.b) < 1e-12


# ------------------------------------------------------------------ trajectories
def _compare_traj(obs_gpu, obs_ref, tol):
    # rows: t N_e Mx My Mz Etot Ekin Eloc ENL EH Exc EZ maxnorm
    assert np.allclose(obs_gpu[:, 0], obs_ref[:, 0], atol=1e-12)
    e_N = np.max(np.abs(obs_gpu[:, 1] - obs_ref[:, 1])) / abs(obs_ref[0, 1])
    e_M = np.max(np.abs(obs_gpu[:, 2:5] - obs_ref[:, 2:5])) / max(np.max(np.abs(obs_ref[:, 2:5])), 1.0)
    scaleE = max(np.max(np.abs(obs_ref[:, 5:12])), 1.0)
    e_E = np.max(np.abs(obs_gpu[:, 5:12] - obs_ref[:, 5:12])) / scaleE
    say(f"  errors: N_e {e_N:.2e}  M {e_M:.2e}  E {e_E:.2e}")
    assert e_N < tol and e_M < tol and e_E < tol


def _final_nm_errors(psi_gpu, psi_ref, occ):
    """Point by point: max |dn| / max n and max |dm| / max n over the grid."""
    en, em, l2n, l2m = nm_errors(psi_gpu, psi_ref, occ)
    say(f"  n, m max-abs {en:.2e} {em:.2e} (L2 {l2n:.2e} {l2m:.2e})")
    return en, em


def test_step_tiny_workload_fp64(torch_cuda):
    """16^3 x 8 spinors, 4 Gaussians, XC + Hartree, B = (0,0,0.01), 20 steps: FP64 <= 1e-10."""
    nct = nct_mod()
    w = I.workload(0)
    say(f"step {w.name} 20 steps fp64")
    sysd = O.system_from_workload(w)
    psi_ref, obs_ref = O.run(sysd, w.psi0, w.nsteps)
    s = nct.system_from_workload(w)
    psi = nct.states_to_device(w.psi0)
    obs = s.step(psi, 0.0, w.nsteps, obs=True)
    _compare_traj(obs, obs_ref[1:], 1e-10)
    en, em = _final_nm_errors(psi.cpu().numpy(), psi_ref, sysd.occ)
    say(f"  final n {en:.2e} m {em:.2e}")
    assert en < 1e-10 and em < 1e-10


def test_step_projectors_pulse_fp64(torch_cuda):
    """Projectors with SOC, circular pulse, product spinors tilted 30 deg: 6 steps FP64."""
    nct = nct_mod()
    bf = I.BField(pulses=I.circular_pulses([0.1, 0.2], [0.5, 1.0], 0.05, 0.1))
    w = I.make_system(n=(16, 16, 16), L=(8.0,) * 3, nstates=6, natoms=2, case=23, bfield=bf,
                      full_spinors=False, min_sep=4.0)
    say("step projectors+pulse 16^3 S=6 6 steps")
    sysd = O.system_from_workload(w)
    psi_ref, obs_ref = O.run(sysd, w.psi0, 6)
    s = nct.system_from_workload(w)
    psi = nct.states_to_device(w.psi0)
    obs = s.step(psi, 0.0, 6, obs=True)
    _compare_traj(obs, obs_ref[1:], 1e-10)
    en, em = _final_nm_errors(psi.cpu().numpy(), psi_ref, sysd.occ)
    assert en < 1e-10 and em < 1e-10


@pytest.mark.parametrize("K", [1, 2, 8])
def test_step_taylor_orders(torch_cuda, K):
    nct = nct_mod()
    w = I.make_system(n=(8, 8, 8), L=(6.0,) * 3, nstates=3, natoms=1, case=24,
                      bfield=I.BField(B0=(0.0, 0.05, 0.02)), taylor_order=K, dt=0.02)
    say(f"step taylor K={K}")
    sysd = O.system_from_workload(w)
    psi_ref, obs_ref = O.run(sysd, w.psi0, 3)
    s = nct.system_from_workload(w)
    psi = nct.states_to_device(w.psi0)
    obs = s.step(psi, 0.0, 3, obs=True)
    _compare_traj(obs, obs_ref[1:], 1e-10)


def test_step_cluster_workload_fp64_one_step(torch_cuda):
    """Full-size magnetic-cluster system (48^3 x 64 spinors, 4 atoms x 18 projectors): one step."""
    nct = nct_mod()
    w = I.workload(1)
    say(f"step {w.name} 1 step fp64 (oracle ~1 min)")
    sysd = O.system_from_workload(w)
    psi_ref, obs_ref = O.run(sysd, w.psi0, 1)
    s = nct.system_from_workload(w)
    psi = nct.states_to_device(w.psi0)
    obs = s.step(psi, 0.0, 1, obs=True)
    _compare_traj(obs, obs_ref[1:], 1e-10)
    got = psi.cpu().numpy()
    en, em = _final_nm_errors(got, psi_ref, sysd.occ)
    ep = max_rel(got, psi_ref)
    say(f"  final n {en:.2e} m {em:.2e} psi {ep:.2e} (max-abs)")
    assert en < 1e-10 and em < 1e-10 and ep < 1e-10


def test_step_overlap_groups_bitwise(torch_cuda):
    """The two-stream state-group schedule gives bit-identical trajectories (same kernels per state)."""
    nct = nct_mod()
    bf = I.BField(pulses=I.circular_pulses([0.1], [0.5], 0.05, 0.1))
    w = I.make_system(n=(16, 16, 16), L=(8.0,) * 3, nstates=9, natoms=2, case=27, bfield=bf,
                      full_spinors=False, min_sep=4.0)
    say("overlap groups S=9")
    out = []
    for ov in (False, True):
        s = nct.system_from_workload(w, overlap=ov)
        psi = nct.states_to_device(w.psi0)
        obs = s.step(psi, 0.0, 3, obs=True)
        out.append((psi.cpu().numpy(), obs))
    assert np.array_equal(out[0][0], out[1][0])
    assert np.array_equal(out[0][1], out[1][1])


def test_step_tiny_workload_mixed(torch_cuda):
    """FP32-mixed form on the tiny system: n, m, E within 1e-5 of the FP64 oracle over 20 steps."""
    nct = nct_mod()
    w = I.workload(0)
    say("step tiny mixed")
    sysd = O.system_from_workload(w)
    psi_ref, obs_ref = O.run(sysd, w.psi0, w.nsteps)
    s = nct.system_from_workload(w, precision=nct.NCT_FP32_MIXED)
    psi = nct.states_to_device(w.psi0, nct.NCT_FP32_MIXED)
    obs = s.step(psi, 0.0, w.nsteps, obs=True)
    _compare_traj(obs, obs_ref[1:], 1e-5)
    en, em = _final_nm_errors(psi.cpu().numpy().astype(np.complex128), psi_ref, sysd.occ)
    say(f"  final n {en:.2e} m {em:.2e}")
    assert en < 1e-5 and em < 1e-5


def test_frozen_field_step(torch_cuda):
    """Frozen total fields: step equals the oracle Taylor-ETRS with the same fixed H."""
    torch = torch_cuda
    nct = nct_mod()
    say("frozen-field step")
    w = I.make_system(n=(8, 8, 8), L=(6.0,) * 3, nstates=2, natoms=1, case=25, dt=0.05)
    F = random_fields(w.n, 3) * 0.4
    sysd = O.system_from_workload(w)
    H = lambda x: (O.kinetic(x, sysd.grid) + O.apply_local(x, F[0], F[1:])
                   + O.apply_nonlocal(x, sysd.projs, sysd.grid))
    ref = w.psi0
    for _ in range(3):
        phi = O.taylor_exp(H, ref, 0.025, 4)
        ref = O.taylor_exp(H, phi, 0.025, 4)
    s = nct.system_from_workload(w)
    s.set_potentials(fields=torch.from_numpy(F).cuda())
    psi = nct.states_to_device(w.psi0)
    s.step(psi, 0.0, 3)
    assert rel(psi.cpu().numpy(), ref) < 1e-12


def test_apply_hamiltonian_96_mixed(torch_cuda):
    """96^2 planes in FP32 (two-half plane pass at its largest LDS footprint).  The oracle sees
    the same FP32-rounded states and fields, so only the kernel's FP32 arithmetic is measured; the
    error of an FP32 FFT round trip grows like u log2(N) (u = 2^-24, the FP32 unit roundoff), and
    the bound 8 u log2(N) (about 9.4e-6 for N = 96^3) stays inside the FP32-mixed tolerance of
    1e-5."""
    torch = torch_cuda
    nct = nct_mod()
    n = (96, 96, 96)
    say("apply_H mixed 96^3")
    w = I.make_system(n=n, L=(40.0,) * 3, nstates=1, case=28, natoms=0)
    F = random_fields(n, 5).astype(np.float32).astype(np.float64)
    psi32 = w.psi0.astype(np.complex64)
    psi_in = psi32.astype(np.complex128)
    sysd = O.system_from_workload(w)
    ref = O.kinetic(psi_in, sysd.grid) + O.apply_local(psi_in, F[0], F[1:])
    s = nct.system_from_workload(w, precision=nct.NCT_FP32_MIXED)
    s.set_potentials(fields=torch.from_numpy(F).cuda())
    psi = nct.states_to_device(psi32, nct.NCT_FP32_MIXED)
    hpsi = torch.empty_like(psi)
    s.apply_hamiltonian(psi, hpsi, 0.0)
    tol = 8 * 2.0 ** -24 * np.log2(np.prod(n))
    err = rel(hpsi.cpu().numpy().astype(np.complex128), ref)
    say(f"  rel err {err:.2e} (tol {tol:.2e})")
    assert err < tol


@pytest.mark.parametrize("xc", [0, 1])
def test_step_single_state_and_noncubic_projectors(torch_cuda, xc):
    """S = 1 (15 padded states in every MFMA tile) on a 12x16x12 grid with projectors and a
    static field, against the oracle.  One spinor is fully polarised at every point, so the
    minority density n_- = (n - |m|)/2 is zero up to rounding and Slater's n_-^(1/3) magnifies
    rounding noise: with exchange on, the oracle itself moves by ~1e-10 in psi when its input
    is perturbed at 1e-16.  The bound on psi is then a small multiple of that measured
    sensitivity; without exchange the dynamics is well conditioned and psi must agree to 1e-12.
    Observables are insensitive in both cases."""
    nct = nct_mod()
    say(f"S=1 non-cubic projectors xc={xc}")
    w = I.make_system(n=(12, 16, 12), L=(6.5, 8.0, 6.5), nstates=1, natoms=1, case=29,
                      bfield=I.BField(B0=(0.03, 0.0, -0.02)), full_spinors=True, xc=xc)
    sysd = O.system_from_workload(w)
    psi_ref, obs_ref = O.run(sysd, w.psi0, 4)
    rng = np.random.default_rng(1)
    psi_p, _ = O.run(sysd, w.psi0 * (1 + 1e-16 * rng.standard_normal(w.psi0.shape)), 4)
    sens = rel(psi_p, psi_ref)
    s = nct.system_from_workload(w)
    psi = nct.states_to_device(w.psi0)
    obs = s.step(psi, 0.0, 4, obs=True)
    _compare_traj(obs, obs_ref[1:], 1e-10)
    err = rel(psi.cpu().numpy(), psi_ref)
    say(f"  psi err {err:.2e}, oracle sensitivity {sens:.2e}")
    assert err < max(10 * sens, 1e-12)
    if xc == 0:
        assert sens < 1e-14


def test_tape_and_backward_argument_errors(torch_cuda):
    torch = torch_cuda
    nct = nct_mod()
    say("tape errors")
    w = I.make_system(n=(8, 8, 8), L=(6.0,) * 3, nstates=2, case=31)
    s = nct.system_from_workload(w, tape_steps=2)
    psi = nct.states_to_device(w.psi0)
    lam = torch.zeros_like(psi)
    with pytest.raises(nct.NctError) as e:       # nothing taped yet
        s.backward_step(0, None, 0.0, lam, lam)
    assert e.value.code == nct.NCT_ERR_STATE
    with pytest.raises(nct.NctError) as e:       # more steps than the tape holds
        s.step(psi, 0.0, 3, tape=True)
    assert e.value.code == nct.NCT_ERR_ARG
    s.step(psi, 0.0, 2, tape=True)
    with pytest.raises(nct.NctError) as e:       # index beyond the record
        s.backward_step(2, None, 0.1, lam, lam)
    assert e.value.code == nct.NCT_ERR_STATE
    with pytest.raises(nct.NctError) as e:       # time does not match the record
        s.backward_step(1, None, 0.3, lam, lam)
    assert e.value.code == nct.NCT_ERR_ARG
    with pytest.raises(nct.NctError) as e:       # recompute mode needs psi_n
        s.backward_step(-1, None, 0.0, lam, lam)
    assert e.value.code == nct.NCT_ERR_ARG


def test_frozen_nonfinite_fields_detected(torch_cuda):
    torch = torch_cuda
    nct = nct_mod()
    say("frozen NaN field")
    w = I.make_system(n=(8, 8, 8), L=(6.0,) * 3, nstates=2, case=32)
    F = random_fields(w.n, 6)
    F[0, 1, 1, 1] = np.nan
    s = nct.system_from_workload(w)
    s.set_potentials(fields=torch.from_numpy(F).cuda())
    psi = nct.states_to_device(w.psi0)
    with pytest.raises(nct.NctError) as e:
        s.step(psi, 0.0, 1)
    assert e.value.code == nct.NCT_ERR_NONFINITE


# ------------------------------------------------------------------ error handling
def test_error_codes(torch_cuda):
    nct = nct_mod()
    say("error codes")
    with pytest.raises(nct.NctError) as e:
        nct.System((10, 16, 16), (5.0, 5.0, 5.0), 2)
    assert e.value.code == nct.NCT_ERR_UNSUPPORTED
    with pytest.raises(nct.NctError) as e:
        nct.System((8, 8, 8), (5.0, 5.0, 5.0), 0)
    assert e.value.code == nct.NCT_ERR_ARG
    with pytest.raises(nct.NctError) as e:
        nct.System((8, 8, 8), (5.0, 5.0, 5.0), 2, taylor_order=0)
    assert e.value.code == nct.NCT_ERR_ARG
    s = nct.System((8, 8, 8), (5.0, 5.0, 5.0), 2)
    psi = s.new_states()
    with pytest.raises(nct.NctError) as e:      # fields not computed yet
        s.apply_hamiltonian(psi, s.new_states())
    assert e.value.code == nct.NCT_ERR_STATE
    with pytest.raises(nct.NctError) as e:
        s.apply_hamiltonian(psi, psi)
    assert e.value.code == nct.NCT_ERR_ARG
    with pytest.raises(nct.NctError) as e:
        s.step(psi, 0.0, -1)
    assert e.value.code == nct.NCT_ERR_ARG


def test_nonfinite_detected(torch_cuda):
    """A NaN in the initial states is reported as NCT_ERR_NONFINITE."""
    torch = torch_cuda
    nct = nct_mod()
    say("nonfinite")
    w = I.make_system(n=(8, 8, 8), L=(6.0,) * 3, nstates=2, case=26)
    s = nct.system_from_workload(w)
    psi0 = w.psi0.copy()
    psi0[0, 0, 1, 2, 3] = np.nan
    psi = nct.states_to_device(psi0)
    with pytest.raises(nct.NctError) as e:
        s.step(psi, 0.0, 1)
    assert e.value.code == nct.NCT_ERR_NONFINITE


def test_watchdog_stops_unstable_propagation(torch_cuda):
    """A time step far outside the Taylor polynomial's stability range (x = E_max dt / 2 ~ 6.6
    against 2.83 for K = 4) makes the norm grow from the first steps: nct_step reports
    NCT_ERR_NONFINITE naming the step at which the electron count left its bound; with the bound
    lifted (finiteness only) the same call succeeds as long as the numbers stay finite."""
    nct = nct_mod()
    say("watchdog: unstable time step")
    w = I.make_system(n=(8, 8, 8), L=(6.0,) * 3, nstates=2, case=33, dt=0.5)
    s = nct.system_from_workload(w)
    psi = nct.states_to_device(w.psi0)
    with pytest.raises(nct.NctError) as e:
        s.step(psi, 0.0, 6)
    assert e.value.code == nct.NCT_ERR_NONFINITE
    assert "step" in str(e.value) and "drifted" in str(e.value)
    s.set_watchdog(0.0)
    psi = nct.states_to_device(w.psi0)
    s.step(psi, 0.0, 1)
    with pytest.raises(nct.NctError) as e:
        s.set_watchdog(float("nan"))
    assert e.value.code == nct.NCT_ERR_ARG
