"""Write the oracle's long reference trajectories (tests/golden/long_*.npz).

Calls only the CPU oracle (oracle/) and the seeded input generator: no value here comes from the
HIP library.  The GPU tests in tests/test_gpu_long_trajectories.py compare both precisions of the
HIP path with these files.

  reduced  the 16^3 x 8 system that keeps every term of the step (2 atoms x 18 KB+SOC
           projectors, Gaussian local potential, exchange + Hartree, circular B pulse), 1000
           ETRS steps of dt = 0.05, once with Slater exchange (xc = 1) and once with PW92
           correlation added (xc = 2): the window of the FP32-mixed target (1e-5 over 1000 steps)
  cluster  the magnetic-cluster system (48^3 x 64 spinors, 4 atoms x 18 projectors, field free),
           its full 200 steps in FP64: the window of the FP64 target (1e-10 in n, m and E)

Each file holds the oracle's observables after every step (row 0: the initial state), the spin
density of the final state and the final states (all of them for the reduced system; a seeded
sample of 4096 entries for the cluster, whose full state set is 226 MB), plus the observables of
the initial state so that a changed input generator is detected.

usage: python tests/golden/make_long_trajectories.py [reduced] [cluster] [--workers W]
"""
import argparse
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import nct_oracle as O  # noqa: E402
from paper_2506_21908_amd import inputs as I  # noqa: E402

SAMPLE = 4096


def sample_index(shape, count, seed=2506):
    """Seeded flat indices into a state array of the given shape (the same set on both sides)."""
    rng = np.random.default_rng(seed)
    return np.sort(rng.choice(int(np.prod(shape)), size=count, replace=False))


def path_for(tag: str) -> str:
    return os.path.join(HERE, f"long_{tag}.npz")


def reduced(xc: int):
    w = I.workload(7)
    w.xc = xc
    return w


def write(tag: str, w, nsteps: int, full_psi: bool):
    sysd = O.system_from_workload(w)
    t0 = time.time()
    psi = w.psi0.copy()
    rows = [O.observables(sysd, psi, 0.0)]
    t = 0.0
    for k in range(nsteps):
        psi = O.etrs_step(sysd, psi, t)
        t += sysd.dt
        rows.append(O.observables(sysd, psi, t))
        if (k + 1) % 10 == 0:
            print(f"[{tag}] step {k + 1}/{nsteps}  {time.time() - t0:.0f} s", flush=True)
    rho = O.spin_density(psi, sysd.occ)
    out = {"obs": np.array(rows), "rho_final": rho, "nsteps": np.array(nsteps),
           "xc": np.array(w.xc), "name": np.array(w.name)}
    if full_psi:
        out["psi_final"] = psi
    else:
        idx = sample_index(psi.shape, SAMPLE)
        out["psi_index"] = idx
        out["psi_sample"] = psi.reshape(-1)[idx]
    np.savez_compressed(path_for(tag), **out)
    print(f"[{tag}] wrote {path_for(tag)} in {time.time() - t0:.0f} s", flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("which", nargs="*", default=["reduced", "cluster"])
    ap.add_argument("--workers", type=int, default=-1, help="scipy.fft workers of the oracle")
    args = ap.parse_args()
    O.FFT_WORKERS = args.workers
    if "reduced" in args.which:
        for xc in (1, 2):
            write(f"reduced16_xc{xc}", reduced(xc), 1000, full_psi=True)
    if "cluster" in args.which:
        write("cluster48_fp64", I.workload(1), 200, full_psi=False)


if __name__ == "__main__":
    main()
