"""Point-by-point error measures shared by the GPU parity tests.

Every measure is a maximum over grid points (or state entries) of an absolute difference, divided
by the largest magnitude of the reference, so that one wrong point fails the bar however large the
grid is.  The L2 ratios are returned beside them for context only.
"""
import numpy as np

from oracle import nct_oracle as O


def max_rel(a, b) -> float:
    """max |a - b| / max |b|."""
    return float(np.max(np.abs(a - b)) / max(float(np.max(np.abs(b))), 1e-300))


def nm_errors(psi_a, psi_b, occ):
    """Spin densities of two state sets compared point by point.

    Returns (e_n, e_m, l2_n, l2_m): e_n = max_r |n_a - n_b| / max_r n_b and
    e_m = max_r max_q |m_a,q - m_b,q| / max_r n_b (m may vanish, so it is measured against n);
    l2_* are the corresponding ||.||_2 ratios."""
    na, ma = O.charge_and_magnetization(O.spin_density(psi_a, occ))
    nb, mb = O.charge_and_magnetization(O.spin_density(psi_b, occ))
    scale = float(np.max(np.abs(nb)))
    e_n = float(np.max(np.abs(na - nb))) / scale
    e_m = float(np.max(np.abs(ma - mb))) / scale
    l2n = float(np.linalg.norm(na - nb) / np.linalg.norm(nb))
    l2m = float(np.linalg.norm(ma - mb) / np.linalg.norm(nb))
    return e_n, e_m, l2n, l2m


def rho_errors(rho_a, rho_b):
    """(e_n, e_m) point by point from two spin-density matrices rho_v [4][...]."""
    na, ma = O.charge_and_magnetization(rho_a)
    nb, mb = O.charge_and_magnetization(rho_b)
    scale = float(np.max(np.abs(nb)))
    return float(np.max(np.abs(na - nb))) / scale, float(np.max(np.abs(ma - mb))) / scale


def traj_errors(obs, ref):
    """Relative errors of N_e, M and the energies over a trajectory (rows of the 13 observables):
    e_N = max |dN_e| / |N_e(0)|, e_M = max |dM| / max(max |M|, 1), e_E = max over E_total and
    its parts |dE| / max(max |E|, 1)."""
    e_N = float(np.max(np.abs(obs[:, 1] - ref[:, 1])) / abs(ref[0, 1]))
    e_M = float(np.max(np.abs(obs[:, 2:5] - ref[:, 2:5])) / max(float(np.max(np.abs(ref[:, 2:5]))), 1.0))
    e_E = float(np.max(np.abs(obs[:, 5:12] - ref[:, 5:12])) / max(float(np.max(np.abs(ref[:, 5:12]))), 1.0))
    return e_N, e_M, e_E
