"""k-point sampling (Bloch vectors per state, Sec. 2.1 and Sec. 5) on the GPU against the oracle."""
import math
import sys
import time

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


def rel(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def _errors(obs, ref, psi, psi_ref, occ):
    e_N = np.max(np.abs(obs[:, 1] - ref[:, 1])) / abs(ref[0, 1])
    e_M = np.max(np.abs(obs[:, 2:5] - ref[:, 2:5])) / max(np.max(np.abs(ref[:, 2:5])), 1.0)
    e_E = np.max(np.abs(obs[:, 5:12] - ref[:, 5:12])) / max(np.max(np.abs(ref[:, 5:12])), 1.0)
    en, em, _, _ = nm_errors(psi, psi_ref, occ)  # point by point over the grid
    return e_N, e_M, e_E, en, em


def _kpoint_system(n=(16, 12, 16), L=(8.0, 6.0, 8.0), nk=3, per=2, case=50, **kw):
    w = I.make_system(n=n, L=L, nstates=nk * per, natoms=2, case=case, full_spinors=True,
                      min_sep=3.0, **kw)
    rng = np.random.default_rng(case)
    kpts = rng.uniform(-1.0, 1.0, (nk, 3)) * np.pi / np.array(L)
    w.kvec = np.repeat(kpts, per, axis=0)
    wk = rng.uniform(0.5, 1.5, nk)
    w.occ = np.repeat(wk / wk.sum(), per) * nk
    return w


def test_kpoints_apply_hamiltonian_frozen_fields(torch_cuda):
    """H_k psi (1/2 |G + k|^2, local 2x2 potential, projectors with Bloch phases) on a non-cubic
    grid against the oracle."""
    torch = torch_cuda
    from paper_2506_21908_amd import nct
    say("H_k psi, frozen fields, 16x12x16")
    w = _kpoint_system()
    sysd = O.system_from_workload(w)
    F = np.random.default_rng(7).uniform(-0.4, 0.4, (4,) + w.n)
    ref = (O.kinetic(w.psi0, sysd.grid, sysd.kvec) + O.apply_local(w.psi0, F[0], F[1:])
           + O.apply_nonlocal(w.psi0, sysd.projs, sysd.grid, sysd.kvec))
    s = nct.system_from_workload(w)
    s.set_potentials(fields=torch.from_numpy(F).cuda())
    psi = nct.states_to_device(w.psi0)
    hpsi = torch.empty_like(psi)
    s.apply_hamiltonian(psi, hpsi, 0.0)
    assert rel(hpsi.cpu().numpy(), ref) < 1e-12


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_kpoints_step_vs_oracle(torch_cuda, prec):
    """3 k-points x 2 states with k-weights, SOC projectors and a B pulse: 6 steps."""
    from paper_2506_21908_amd import nct
    say(f"k-point steps {prec}")
    bf = I.BField(B0=(0.0, 0.01, 0.02), pulses=I.circular_pulses([0.1], [0.8], 0.05, 0.2))
    w = _kpoint_system(bfield=bf)
    sysd = O.system_from_workload(w)
    psi_ref, obs_ref = O.run(sysd, w.psi0, 6)
    pf = nct.NCT_FP64 if prec == "fp64" else nct.NCT_FP32_MIXED
    s = nct.system_from_workload(w, precision=pf)
    psi = nct.states_to_device(w.psi0, pf)
    obs = s.step(psi, 0.0, 6, obs=True)
    errs = _errors(obs, obs_ref[1:], psi.cpu().numpy().astype(np.complex128), psi_ref, sysd.occ)
    say("  N_e %.2e M %.2e E %.2e n %.2e m %.2e" % errs)
    assert max(errs) < (1e-10 if prec == "fp64" else 1e-5)
    if prec == "fp64":
        assert rel(psi.cpu().numpy(), psi_ref) < 1e-10


def test_kpoints_supercell_equivalence_on_gpu(torch_cuda):
    """A 2x1x1 supercell at Gamma (24x12x12) and the primitive cell (12x12x12) sampled at
    k = 0, pi/L_x with weights 1/2, both on the GPU: the supercell states stay the tiled,
    phased primitive ones over 3 steps."""
    from paper_2506_21908_amd import nct
    say("supercell equivalence")
    w = I.make_system(n=(12, 12, 12), L=(6.0, 6.0, 6.0), nstates=2, natoms=1, case=48,
                      full_spinors=True, dt=0.04)
    S = w.nstates
    Lx = w.L[0]
    u = np.concatenate([w.psi0, np.roll(w.psi0[::-1], 3, axis=-1)])
    kv = np.zeros((2 * S, 3))
    kv[S:, 0] = math.pi / Lx
    prim = I.make_system(n=(12, 12, 12), L=(6.0, 6.0, 6.0), nstates=2 * S, natoms=1, case=48,
                         full_spinors=True, dt=0.04)
    prim.psi0 = u
    prim.kvec = kv
    prim.occ = np.full(2 * S, 0.5)
    x = np.arange(24) * (2 * Lx / 24)
    def to_super(uu):
        big = np.concatenate([uu, uu], axis=2) / math.sqrt(2.0)
        return big * np.exp(1j * np.outer(kv[:, 0], x))[:, None, :, None, None]
    sup = I.make_system(n=(24, 12, 12), L=(2 * Lx, 6.0, 6.0), nstates=2 * S, natoms=0, case=48,
                        dt=0.04)
    sup.positions = np.concatenate([w.positions, w.positions + np.array([Lx, 0, 0])])
    sup.channels = w.channels
    sup.v_ext = np.concatenate([w.v_ext, w.v_ext], axis=0)
    sup.psi0 = to_super(u)
    sup.occ = np.ones(2 * S)
    sp = nct.system_from_workload(prim)
    ss = nct.system_from_workload(sup)
    pp = nct.states_to_device(prim.psi0)
    ps = nct.states_to_device(sup.psi0)
    sp.step(pp, 0.0, 3)
    ss.step(ps, 0.0, 3)
    got = ps.cpu().numpy()
    assert rel(got, to_super(pp.cpu().numpy())) < 1e-11


def test_kpoints_overlap_groups_bitwise(torch_cuda):
    """The two-group overlap schedule offsets the states of its second group; the Bloch vectors
    must follow (bitwise equal to the one-group run)."""
    from paper_2506_21908_amd import nct
    say("k-points with overlap groups")
    w = _kpoint_system(n=(16, 16, 16), L=(8.0,) * 3, nk=4, per=4, case=51)
    out = []
    for ov in (False, True):
        s = nct.system_from_workload(w, overlap=ov)
        psi = nct.states_to_device(w.psi0)
        s.step(psi, 0.0, 2)
        out.append(psi.cpu().numpy())
    assert np.array_equal(out[0], out[1])


def test_kpoints_gradient_vs_oracle_tangent_linear(torch_cuda):
    """Adjoint (checkpointed) B-pulse gradient with k-points against the oracle's forward mode."""
    torch = torch_cuda
    from paper_2506_21908_amd import nct
    say("gradient with k-points")
    pulses = I.circular_pulses([0.1, 0.2], [0.5, 1.0], 0.05, 0.15)
    w = _kpoint_system(n=(12, 12, 12), L=(7.0,) * 3, nk=2, per=2, case=52,
                       bfield=I.BField(pulses=pulses))
    sysd = O.system_from_workload(w)
    nsteps = 6
    g_ref = O.mz_gradient_tangent_linear(sysd, w.psi0, nsteps)
    s = nct.system_from_workload(w, tape_steps=3)
    theta = torch.tensor([p.A for p in pulses] + [p.omega for p in pulses], dtype=torch.float64,
                         requires_grad=True)
    psi0 = nct.states_to_device(w.psi0)
    L = nct.pulse_mz(theta, s, psi0, pulses, nsteps, 3)
    L.backward()
    g = theta.grad.numpy()
    say(f"  adjoint {g}\n  oracle  {g_ref}")
    assert np.allclose(g, g_ref, rtol=1e-8, atol=1e-12 * np.max(np.abs(g_ref)))


def test_kpoint_workload_one_step_vs_oracle(torch_cuda):
    """The k-point solid (64^3, 8 Monkhorst-Pack k-points x 32 states, 16 atoms x 18 projectors):
    one FP64 step against the oracle."""
    from paper_2506_21908_amd import nct
    w = I.workload(6)
    say(f"{w.name}: 1 FP64 step vs oracle")
    sysd = O.system_from_workload(w)
    t0 = time.time()
    psi_ref, obs_ref = O.run(sysd, w.psi0, 1)
    say(f"  oracle {time.time() - t0:.1f} s")
    s = nct.system_from_workload(w)
    psi = nct.states_to_device(w.psi0)
    obs = s.step(psi, 0.0, 1, obs=True)
    got = psi.cpu().numpy()
    errs = _errors(obs, obs_ref[1:], got, psi_ref, sysd.occ) + (max_rel(got, psi_ref),)
    say("  N_e %.2e M %.2e E %.2e n %.2e m %.2e psi %.2e (max-abs)" % errs)
    assert max(errs) < 1e-10
