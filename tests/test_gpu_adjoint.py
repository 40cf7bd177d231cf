"""Adjoint (reverse-mode) time step on the GPU against the oracle's tangent-linear step and
against central finite differences of the GPU trajectory."""
import sys

import numpy as np
import pytest

from oracle import nct_oracle as O
from paper_2506_21908_amd import inputs as I

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


def _rand_states(shape, seed):
    rng = np.random.default_rng(seed)
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


def _inner(a, b):
    return float(np.real(np.vdot(a, b)))


@pytest.mark.parametrize("frozen,xc", [(False, 1), (True, 1), (False, 2)])
def test_backward_step_dot_product(torch_cuda, frozen, xc):
    """Re<lam_n, dpsi_n> = Re<lam_{n+1}, J dpsi_n>, with J the oracle's tangent-linear step,
    and dL/dB(t_n), dL/dB(t_n+dt) against the oracle's response to dB (xc = 2: with the PW92
    correlation response)."""
    torch = torch_cuda
    from paper_2506_21908_amd import nct
    say(f"backward dot product frozen={frozen} xc={xc}")
    bf = I.BField(B0=(0.01, 0.0, 0.02), pulses=I.circular_pulses([0.1], [0.7], 0.05, 0.2))
    w = I.make_system(n=(12, 12, 12), L=(7.0,) * 3, nstates=4, natoms=1, case=40, bfield=bf,
                      full_spinors=False, xc=xc)
    sysd = O.system_from_workload(w)
    t_n = 0.1
    lam1 = _rand_states(w.psi0.shape, 1)
    dpsi = _rand_states(w.psi0.shape, 2)
    s = nct.system_from_workload(w, tape_steps=1)
    if frozen:
        rng = np.random.default_rng(3)
        F = rng.uniform(-0.3, 0.3, (4,) + w.n)
        s.set_potentials(fields=torch.from_numpy(F).cuda())
        H = lambda x: (O.kinetic(x, sysd.grid) + O.apply_local(x, F[0], F[1:])
                       + O.apply_nonlocal(x, sysd.projs, sysd.grid))
        Z = lambda x: np.zeros_like(x)
        a = 0.5 * w.dt
        phi, dphi = O._taylor_jvp(H, Z, w.psi0, dpsi, a, 4)
        _, dnext = O._taylor_jvp(H, Z, phi, dphi, a, 4)
    else:
        _, dnext = O.etrs_step_jvp(sysd, w.psi0, dpsi, t_n, np.zeros(3), np.zeros(3))
    psi = nct.states_to_device(w.psi0)
    lam_in = nct.states_to_device(lam1)
    lam_out = torch.empty_like(lam_in)
    dLdB = s.backward_step(-1, psi, t_n, lam_in, lam_out)
    lhs = _inner(lam_out.cpu().numpy(), dpsi)
    rhs = _inner(lam1, dnext)
    say(f"  <lam_n, dpsi> = {lhs:.15e}  <lam_n+1, J dpsi> = {rhs:.15e}")
    assert abs(lhs - rhs) < 1e-10 * abs(rhs)
    if not frozen:
        for j in range(6):
            e = np.zeros(3)
            e[j % 3] = 1.0
            dBn, dBp = (e, np.zeros(3)) if j < 3 else (np.zeros(3), e)
            _, dn2 = O.etrs_step_jvp(sysd, w.psi0, np.zeros_like(dpsi), t_n, dBn, dBp)
            ref = _inner(lam1, dn2)
            assert abs(dLdB[j] - ref) < 1e-10 * max(abs(ref), 1e-3), (j, dLdB[j], ref)
    # taped mode gives the same result as recompute mode
    psi2 = nct.states_to_device(w.psi0)
    s.step(psi2, t_n, 1, tape=True)
    lam_out2 = torch.empty_like(lam_in)
    dLdB2 = s.backward_step(0, None, t_n, lam_in, lam_out2)
    assert torch.equal(lam_out, lam_out2)
    assert np.array_equal(dLdB, dLdB2)


@pytest.mark.parametrize("xc", [1, 2])
def test_pulse_gradient_vs_oracle_tangent_linear(torch_cuda, xc):
    """dM_z(T)/d(A_k, omega_k) through the checkpointed adjoint equals the oracle's forward-mode
    gradient of the same discrete trajectory (xc = 2: LSDA)."""
    torch = torch_cuda
    from paper_2506_21908_amd import nct
    say(f"pulse gradient vs oracle tangent-linear, 12^3 x 4, 8 steps, xc={xc}")
    pulses = I.circular_pulses([0.1, 0.25], [0.5, 1.0], 0.05, 0.15)
    bf = I.BField(pulses=pulses)
    w = I.make_system(n=(12, 12, 12), L=(7.0,) * 3, nstates=4, natoms=1, case=41, bfield=bf,
                      full_spinors=False, xc=xc)
    sysd = O.system_from_workload(w)
    nsteps = 8
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


def test_pulse_gradient_grad_workload_vs_fd(torch_cuda):
    """Gradient workload (32^3 x 32 spinors, 2 atoms x 18 projectors, 4 circular pulse
    components, 200 steps, checkpoint every 20): adjoint vs central differences h = 1e-6."""
    torch = torch_cuda
    from paper_2506_21908_amd import nct
    w = I.workload(3)
    say(f"{w.name}: adjoint vs FD, {w.nsteps} steps")
    pulses = w.bfield.pulses
    s = nct.system_from_workload(w, tape_steps=w.checkpoint_every)
    psi0 = nct.states_to_device(w.psi0)
    th0 = np.array([p.A for p in pulses] + [p.omega for p in pulses])
    theta = torch.tensor(th0, dtype=torch.float64, requires_grad=True)
    L = nct.pulse_mz(theta, s, psi0, pulses, w.nsteps, w.checkpoint_every)
    L.backward()
    g = theta.grad.numpy()
    h = 1e-6
    fd = np.zeros_like(th0)
    for k in range(len(th0)):
        vals = []
        for sg in (1, -1):
            th = th0.copy()
            th[k] += sg * h
            vals.append(float(nct.pulse_mz(torch.tensor(th), s, psi0, pulses, w.nsteps,
                                           w.checkpoint_every)))
        fd[k] = (vals[0] - vals[1]) / (2 * h)
    say(f"  L = {float(L):.12f}\n  adjoint {g}\n  FD      {fd}")
    scale = np.max(np.abs(g))
    assert np.all(np.abs(g - fd) < 1e-5 * scale + 1e-9)


def test_pulse_gradient_grad_workload_vs_oracle_short(torch_cuda):
    """Same workload, first 10 steps: adjoint vs the oracle tangent-linear gradient."""
    torch = torch_cuda
    from paper_2506_21908_amd import nct
    w = I.workload(3)
    nsteps = 10
    say(f"{w.name}: adjoint vs oracle tangent-linear, {nsteps} steps")
    sysd = O.system_from_workload(w)
    g_ref = O.mz_gradient_tangent_linear(sysd, w.psi0, nsteps)
    pulses = w.bfield.pulses
    s = nct.system_from_workload(w, tape_steps=5)
    theta = torch.tensor([p.A for p in pulses] + [p.omega for p in pulses], dtype=torch.float64,
                         requires_grad=True)
    L = nct.pulse_mz(theta, s, nct.states_to_device(w.psi0), pulses, nsteps, 5)
    L.backward()
    g = theta.grad.numpy()
    say(f"  adjoint {g}\n  oracle  {g_ref}")
    assert np.allclose(g, g_ref, rtol=1e-8, atol=1e-10 * np.max(np.abs(g_ref)))


def test_pulse_gradient_mixed_precision(torch_cuda):
    """FP64 and FP32-mixed adjoint gradients against the oracle's tangent-linear gradient of the
    same discrete trajectory (FP64 to 1e-8, FP32-mixed to 1e-4 relative to the largest
    component)."""
    torch = torch_cuda
    from paper_2506_21908_amd import nct
    say("mixed-precision gradient vs oracle tangent-linear")
    pulses = I.circular_pulses([0.1, 0.25], [0.5, 1.0], 0.05, 0.15)
    w = I.make_system(n=(16, 16, 16), L=(8.0,) * 3, nstates=6, natoms=2, case=42,
                      bfield=I.BField(pulses=pulses), full_spinors=False, min_sep=4.0)
    g_ref = O.mz_gradient_tangent_linear(O.system_from_workload(w), w.psi0, 8)
    for prec, tol in ((nct.NCT_FP64, 1e-8), (nct.NCT_FP32_MIXED, 1e-4)):
        s = nct.system_from_workload(w, precision=prec, tape_steps=4)
        theta = torch.tensor([p.A for p in pulses] + [p.omega for p in pulses],
                             dtype=torch.float64, requires_grad=True)
        L = nct.pulse_mz(theta, s, nct.states_to_device(w.psi0, prec), pulses, 8, 4)
        L.backward()
        g = theta.grad.numpy()
        err = np.max(np.abs(g - g_ref)) / np.max(np.abs(g_ref))
        say(f"  precision {prec}: adjoint {g}\n  oracle {g_ref}\n  rel err {err:.2e}")
        assert err < tol


def test_pulse_gradient_backward_after_another_forward(torch_cuda):
    """backward uses the pulse of its own forward call: a second forward with a perturbed theta
    between L = pulse_mz(theta) and L.backward() (as a finite-difference probe or a line search
    would run) leaves the gradient equal to the oracle's at theta, and the system gets back the
    field it held before backward."""
    torch = torch_cuda
    from paper_2506_21908_amd import nct
    say("pulse gradient with an interleaved forward call")
    pulses = I.circular_pulses([0.1, 0.25], [0.5, 1.0], 0.05, 0.15)
    w = I.make_system(n=(12, 12, 12), L=(7.0,) * 3, nstates=4, natoms=1, case=41,
                      bfield=I.BField(pulses=pulses), full_spinors=False, xc=1)
    g_ref = O.mz_gradient_tangent_linear(O.system_from_workload(w), w.psi0, 6)
    s = nct.system_from_workload(w, tape_steps=3)
    psi0 = nct.states_to_device(w.psi0)
    th = np.array([p.A for p in pulses] + [p.omega for p in pulses])
    theta = torch.tensor(th, dtype=torch.float64, requires_grad=True)
    L = nct.pulse_mz(theta, s, psi0, pulses, 6, 3)
    other = th * np.array([1.7, 0.6, 1.3, 0.8])
    L2 = nct.pulse_mz(torch.tensor(other), s, psi0, pulses, 6, 3)
    assert abs(float(L2) - float(L)) > 1e-9          # the probe really changed the field
    held = s.bfield_args
    L.backward()
    g = theta.grad.numpy()
    say(f"  adjoint {g}\n  oracle  {g_ref}")
    assert np.allclose(g, g_ref, rtol=1e-8, atol=1e-12 * np.max(np.abs(g_ref)))
    assert s.bfield_args[1] == held[1]


def test_pulse_gradient_two_level_schedule(torch_cuda):
    """The schedule for systems too large for a multi-step tape (host checkpoints every 6 steps,
    sub-segments of 2, recompute-mode backward steps) gives the oracle's tangent-linear gradient
    and the taped schedule's gradient."""
    torch = torch_cuda
    from paper_2506_21908_amd import nct
    say("pulse gradient, two-level recompute schedule")
    pulses = I.circular_pulses([0.1, 0.25], [0.5, 1.0], 0.05, 0.15)
    w = I.make_system(n=(12, 12, 12), L=(7.0,) * 3, nstates=4, natoms=1, case=41,
                      bfield=I.BField(pulses=pulses), full_spinors=False, xc=1)
    nsteps = 13
    g_ref = O.mz_gradient_tangent_linear(O.system_from_workload(w), w.psi0, nsteps)
    th = [p.A for p in pulses] + [p.omega for p in pulses]
    grads = {}
    seen = []
    for name, tape in (("taped", 6), ("recompute", 0)):
        s = nct.system_from_workload(w, tape_steps=tape)
        theta = torch.tensor(th, dtype=torch.float64, requires_grad=True)
        L = nct.pulse_mz(theta, s, nct.states_to_device(w.psi0), pulses, nsteps, 6,
                         checkpoint_on_host=(tape == 0), sub_every=2,
                         progress=(lambda k, n: seen.append((k, n))) if tape == 0 else None)
        L.backward()
        grads[name] = theta.grad.numpy()
        s.close()
    say(f"  taped {grads['taped']}\n  recompute {grads['recompute']}\n  oracle {g_ref}")
    assert seen == [(1, 3), (2, 3), (3, 3)]
    scale = np.max(np.abs(g_ref))
    assert np.allclose(grads["recompute"], g_ref, rtol=1e-8, atol=1e-12 * scale)
    assert np.allclose(grads["recompute"], grads["taped"], rtol=1e-12, atol=1e-14 * scale)
