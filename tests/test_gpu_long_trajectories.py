"""Long trajectories of the HIP path against the oracle's stored reference trajectories.

The references (tests/golden/long_*.npz) are written by tests/golden/make_long_trajectories.py,
which calls only the CPU oracle and the seeded input generator.

* Reduced system that keeps every term of the step (16^3 x 8 spinors, 2 atoms x 18 KB+SOC
  projectors, Gaussian local potential, exchange + Hartree, circular B pulse), 1000 steps with
  Slater exchange and with PW92 correlation added: the FP32-mixed form must stay within 1e-5 of
  the FP64 oracle over the whole window (the FP32 target), the FP64 path within 1e-10.
* Magnetic-cluster system at full size (48^3 x 64 spinors, 4 atoms x 18 projectors), its 200
  steps: the FP64 path within 1e-10 of the oracle in n, m and E (the FP64 target), and the
  FP32-mixed form within 1e-5.

Observables are compared after every step; n and m of the final state point by point over the
grid; the final states entry by entry (all of them for the reduced system, a seeded sample of
4096 entries for the cluster).
"""
import os
import sys
import time

import numpy as np
import pytest

from oracle import nct_oracle as O
from paper_2506_21908_amd import inputs as I
from parity_metrics import max_rel, rho_errors, traj_errors

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def say(msg):
    print(f"[case] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def load(tag):
    path = os.path.join(GOLDEN, f"long_{tag}.npz")
    with np.load(path, allow_pickle=False) as z:
        return {k: z[k] for k in z.files}


def check_inputs(w, ref):
    """The seeded inputs are the ones the reference was written from: the oracle's observables of
    the initial state reproduce row 0 of the stored trajectory."""
    sysd = O.system_from_workload(w)
    row0 = O.observables(sysd, w.psi0, 0.0)
    err = max_rel(row0, ref["obs"][0])
    assert err < 1e-12, f"input generator changed since the reference was written ({err:.2e})"


def run_gpu(w, precision, nsteps):
    from paper_2506_21908_amd import nct
    s = nct.system_from_workload(w, precision=precision)
    psi = nct.states_to_device(w.psi0, precision)
    t0 = time.time()
    obs = s.step(psi, 0.0, nsteps, obs=True)
    say(f"  {nsteps} steps on the GPU in {time.time() - t0:.2f} s")
    out = psi.cpu().numpy().astype(np.complex128)
    s.close()
    return obs, out


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
@pytest.mark.parametrize("xc", [1, 2])
def test_reduced_system_1000_steps_vs_oracle(torch_cuda, xc, prec):
    from paper_2506_21908_amd import nct
    ref = load(f"reduced16_xc{xc}")
    w = I.workload(7)
    w.xc = xc
    nsteps = int(ref["nsteps"])
    say(f"{w.name} xc={xc} {prec}: {nsteps} steps vs oracle")
    check_inputs(w, ref)
    pf = nct.NCT_FP64 if prec == "fp64" else nct.NCT_FP32_MIXED
    obs, psi = run_gpu(w, pf, nsteps)
    e_N, e_M, e_E = traj_errors(obs, ref["obs"][1:])
    e_n, e_m = rho_errors(O.spin_density(psi, w.occ), ref["rho_final"])
    e_psi = max_rel(psi, ref["psi_final"])
    drift = float(np.max(np.abs(ref["obs"][:, 5] - ref["obs"][0, 5])))
    say(f"  over {nsteps} steps: N_e {e_N:.2e} M {e_M:.2e} E {e_E:.2e}; final n {e_n:.2e} "
        f"m {e_m:.2e} psi {e_psi:.2e} (max-abs); M_z(T) gpu {obs[-1, 4]:.12f} oracle "
        f"{ref['obs'][-1, 4]:.12f}; oracle energy excursion {drift:.2e} Ha")
    assert np.allclose(obs[:, 0], ref["obs"][1:, 0], atol=1e-9)
    tol = 1e-10 if prec == "fp64" else 1e-5
    assert max(e_N, e_M, e_E, e_n, e_m, e_psi) < tol


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_cluster_workload_200_steps_vs_oracle(torch_cuda, prec):
    from paper_2506_21908_amd import nct
    ref = load("cluster48_fp64")
    w = I.workload(1)
    nsteps = int(ref["nsteps"])
    say(f"{w.name} {prec}: {nsteps} steps vs oracle")
    check_inputs(w, ref)
    pf = nct.NCT_FP64 if prec == "fp64" else nct.NCT_FP32_MIXED
    obs, psi = run_gpu(w, pf, nsteps)
    e_N, e_M, e_E = traj_errors(obs, ref["obs"][1:])
    e_n, e_m = rho_errors(O.spin_density(psi, w.occ), ref["rho_final"])
    e_psi = max_rel(psi.reshape(-1)[ref["psi_index"]], ref["psi_sample"])
    say(f"  over {nsteps} steps: N_e {e_N:.2e} M {e_M:.2e} E {e_E:.2e}; final n {e_n:.2e} "
        f"m {e_m:.2e} (max-abs over the grid) psi {e_psi:.2e} (4096 sampled entries); "
        f"E(T) gpu {obs[-1, 5]:.12f} oracle {ref['obs'][-1, 5]:.12f}")
    tol = 1e-10 if prec == "fp64" else 1e-5
    assert max(e_N, e_M, e_E, e_n, e_m, e_psi) < tol
