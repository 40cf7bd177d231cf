"""LSDA (Slater exchange + PW92 correlation, locally collinear; xc = 2) on the GPU against the
oracle."""
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


def test_lsda_fields_vs_oracle(torch_cuda):
    """v = v_ext + v_H + vbar_x + vbar_c and b = b_x + b_c with generic local polarisation
    (0 < zeta < 1; a fully polarised point is ill-conditioned for Slater exchange, whose
    n_dn^(1/3) magnifies the rounding of n_dn = 0) and density tails reaching large rs."""
    torch = torch_cuda
    from paper_2506_21908_amd import nct
    say("lsda fields")
    w = I.make_system(n=(12, 16, 12), L=(7.0, 8.0, 7.0), nstates=3, case=45, natoms=2, xc=2,
                      projectors=False, localized=1.5, localized_full=True)
    sysd = O.system_from_workload(w)
    F = O.fields_from_density(sysd, O.spin_density(w.psi0, sysd.occ), 0.0)
    s = nct.system_from_workload(w)
    psi = nct.states_to_device(w.psi0)
    s.density_magnetization(psi, 0.0, update_fields=True)
    out = torch.empty((4,) + w.n, dtype=torch.float64, device="cuda")
    s.get_fields(0.0, out)
    got = out.cpu().numpy()
    assert rel(got[0], F.v) < 1e-12
    assert rel(got[1:], F.b) < 1e-12
    # the correlation part is really there
    _, _, ec = O.pw92_correlation(F.n, F.m)
    assert abs(np.sum(ec)) > 1e-3 * abs(np.sum(F.ex))


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_lsda_step_vs_oracle(torch_cuda, prec):
    from paper_2506_21908_amd import nct
    say(f"lsda step {prec}")
    bf = I.BField(B0=(0.01, 0.0, 0.02), pulses=I.circular_pulses([0.15], [0.6], 0.05, 0.2))
    w = I.make_system(n=(16, 16, 16), L=(8.0,) * 3, nstates=6, natoms=2, case=46, xc=2, bfield=bf,
                      full_spinors=False, min_sep=4.0)
    sysd = O.system_from_workload(w)
    psi_ref, obs_ref = O.run(sysd, w.psi0, 8)
    pf = nct.NCT_FP64 if prec == "fp64" else nct.NCT_FP32_MIXED
    s = nct.system_from_workload(w, precision=pf)
    psi = nct.states_to_device(w.psi0, pf)
    obs = s.step(psi, 0.0, 8, obs=True)
    errs = _errors(obs, obs_ref[1:], psi.cpu().numpy().astype(np.complex128), psi_ref, sysd.occ)
    say("  N_e %.2e M %.2e E %.2e n %.2e m %.2e" % errs)
    assert max(errs) < (1e-10 if prec == "fp64" else 1e-5)


def test_lsda_cluster_workload_one_step_vs_oracle(torch_cuda):
    from paper_2506_21908_amd import nct
    w = I.workload(1)
    w.xc = 2
    say(f"{w.name} with PW92: 1 FP64 step vs oracle")
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
