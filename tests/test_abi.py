"""The C ABI library loads and exports what include/nct.h declares (no GPU needed)."""
import ctypes
import os
import re
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "nct.h")
LIB = os.path.join(ROOT, "paper_2506_21908_amd", "libnct.so")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(nct_[a-z_]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for f in ["nct_create_system", "nct_destroy_system", "nct_last_error", "nct_set_potentials",
              "nct_density_magnetization", "nct_apply_hamiltonian", "nct_step",
              "nct_backward_step", "nct_magnetization_seed", "nct_get_fields", "nct_version",
              "nct_set_laser", "nct_set_laser_gauge", "nct_set_kpoints", "nct_dm_initialization",
              "nct_ground_state", "nct_set_timing_sample"]:
        assert f in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libnct.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_ctypes_structs_match_c_layout():
    """sizeof/offsetof of the public structs from gcc equal the ctypes mirrors."""
    from paper_2506_21908_amd import nct
    prog = r'''
#include <stdio.h>
#include <stddef.h>
#include "nct.h"
int main(void) {
  printf("%zu %zu %zu %zu\n", sizeof(nct_channel), sizeof(nct_pulse), sizeof(nct_bfield), sizeof(nct_params));
  printf("%zu %zu %zu %zu %zu %zu %zu\n", offsetof(nct_params, nstates), offsetof(nct_params, occ),
         offsetof(nct_params, r_sphere), offsetof(nct_params, dt), offsetof(nct_params, tape_steps),
         offsetof(nct_params, overlap), offsetof(nct_params, stream));
  printf("%zu %zu\n", offsetof(nct_pulse, e1), offsetof(nct_bfield, pulses));
  printf("%zu %zu\n", sizeof(nct_laser_pulse), offsetof(nct_laser_pulse, pol));
  printf("%zu %zu\n", sizeof(nct_atom_density), offsetof(nct_atom_density, moment));
  return 0;
}
'''
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "t.c")
        exe = os.path.join(d, "t")
        open(c, "w").write(prog)
        subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), c, "-o", exe], check=True)
        out = subprocess.run([exe], capture_output=True, text=True, check=True).stdout.split()
    vals = [int(v) for v in out]
    P = nct.Params
    assert vals[:4] == [ctypes.sizeof(nct.Channel), ctypes.sizeof(nct.Pulse),
                        ctypes.sizeof(nct.BField), ctypes.sizeof(P)]
    assert vals[4:11] == [P.nstates.offset, P.occ.offset, P.r_sphere.offset, P.dt.offset,
                          P.tape_steps.offset, P.overlap.offset, P.stream.offset]
    assert vals[11:13] == [nct.Pulse.e1.offset, nct.BField.pulses.offset]
    assert vals[13:15] == [ctypes.sizeof(nct.LaserPulse), nct.LaserPulse.pol.offset]
    assert vals[15:17] == [ctypes.sizeof(nct.AtomDensity), nct.AtomDensity.moment.offset]


def test_binding_refuses_without_gpu():
    """No CPU fallback: creating a system without a GPU raises."""
    import torch
    if torch.cuda.is_available():
        pytest.skip("GPU present")
    from paper_2506_21908_amd import nct
    with pytest.raises(RuntimeError):
        nct.System((8, 8, 8), (5.0, 5.0, 5.0), 2)


def test_input_generator_is_seeded_and_normalised():
    import numpy as np
    from paper_2506_21908_amd import inputs as I
    a = I.make_system(n=(8, 8, 8), L=(6.0,) * 3, nstates=3, natoms=1, case=12)
    b = I.make_system(n=(8, 8, 8), L=(6.0,) * 3, nstates=3, natoms=1, case=12)
    assert np.array_equal(a.psi0, b.psi0) and np.array_equal(a.positions, b.positions)
    dV = 6.0 ** 3 / 512
    S = a.psi0.reshape(3, -1)
    assert np.allclose(S.conj() @ S.T * dV, np.eye(3), atol=1e-12)
    w = I.workload(0)
    assert w.psi0.shape == (8, 2, 16, 16, 16) and w.nsteps == 20
