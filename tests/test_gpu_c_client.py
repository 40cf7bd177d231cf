"""The library used from plain C (examples/c_step.c, built by __graft_entry__.build()): a
self-consistent 20-step run with projectors.  The program checks charge, norm and energy
conservation itself; here its observables are also compared with the same system run through
the Python binding."""
import math
import os
import subprocess
import sys
import tempfile
from types import SimpleNamespace

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
EXE = os.path.join(ROOT, "paper_2506_21908_amd", "examples", "c_step")


def _same_system_through_python(nct):
    """The C program's system, built with the same formulas in numpy."""
    import torch
    n, S, L = 16, 4, 8.0
    h = L / n
    pos = np.array([[4.1, 3.9, 4.0]])
    ch = [SimpleNamespace(l=l, twoj=tj, energy=e, rc=0.7)
          for l, tj, e in ((0, 1, 1.0), (1, 1, 0.45), (1, 3, 0.525), (2, 3, -0.33), (2, 5, -0.28))]
    s = nct.System((n,) * 3, (L,) * 3, S, positions=pos, channels=ch, r_sphere=2.5, xc=1, hartree=1,
                   m_threshold=1e-12, dt=0.05, taylor_order=4)
    ax = np.arange(n) * h
    X, Y, Z = np.meshgrid(ax, ax, ax, indexing="ij")
    d2 = (X - pos[0, 0]) ** 2 + (Y - pos[0, 1]) ** 2 + (Z - pos[0, 2]) ** 2
    s.set_potentials(v_ext=torch.from_numpy(-2.0 * np.exp(-d2 / 2.0)).cuda(), B0=(0.0, 0.0, 0.02))
    psi = np.zeros((S, 2, n, n, n), dtype=np.complex128)
    for i in range(S):
        th, ph = 0.5 + 0.4 * i, 0.7 * i
        g = np.exp(-d2 / (2.0 * (1.2 + 0.3 * i)))
        k = 2.0 * math.pi / L * (i % 2)
        psi[i, 0] = g * math.cos(0.5 * th) * np.exp(1j * k * X)
        psi[i, 1] = g * math.sin(0.5 * th) * np.exp(1j * (k * X + ph))
        psi[i] /= math.sqrt(np.sum(np.abs(psi[i]) ** 2) * h ** 3)
    d = nct.states_to_device(psi)
    obs = s.step(d, 0.0, 20, obs=True)
    s.close()
    return obs


def test_c_client_runs_and_matches_binding():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    if not os.path.exists(EXE):
        pytest.fail("examples/c_step not built (run __graft_entry__.build())")
    from paper_2506_21908_amd import nct
    print("[case] plain C client, 16^3 x 4 spinors, 20 steps", flush=True)
    sys.stdout.flush()
    with tempfile.TemporaryDirectory() as tmp:
        path = os.path.join(tmp, "obs.bin")
        r = subprocess.run([EXE, path], capture_output=True, text=True, timeout=120)
        print(r.stdout, r.stderr, flush=True)
        assert r.returncode == 0, r.stderr
        obs_c = np.fromfile(path, dtype=np.float64).reshape(20, 13)
    obs_py = _same_system_through_python(nct)
    err = np.max(np.abs(obs_c[:, 1:12] - obs_py[:, 1:12])) / np.max(np.abs(obs_py[:, 1:12]))
    print(f"[case]   C vs Python binding: max rel obs difference {err:.2e}", flush=True)
    assert err < 1e-12
