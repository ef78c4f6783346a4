"""Host-only checks of the C ABI: libpp.so loads, exports every function declared in
include/pp.h, and the ctypes structs of the binding match the C layout (sizes and offsets
printed by a host C program compiled against the header).  No GPU call is made."""
import ctypes
import os
import re
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pp.h")


def _declared_functions():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:pp_status|const char\*)\s+(pp_\w+)\s*\(", text, re.M)))


def test_header_declares_the_five_calls():
    names = _declared_functions()
    for f in ("pp_init_species", "pp_gather_push_deposit", "pp_field_step", "pp_sort_particles", "pp_diagnostics"):
        assert f in names


def test_library_exports_every_declared_symbol():
    from paper_1211_4575_amd import pp
    L = pp.lib()
    for name in _declared_functions():
        assert hasattr(L, name), name
    assert set(_declared_functions()) == set(pp.EXPORTED)
    assert L.pp_status_str(pp.PP_E_CFL).decode().startswith("c*dt")


def test_struct_layout_matches_header():
    from paper_1211_4575_amd import pp
    src = r"""
#include <stdio.h>
#include <stddef.h>
#include "pp.h"
#define P(T, F) printf(#T "." #F " %zu\n", offsetof(T, F))
int main(void) {
  printf("pp_params %zu\npp_mesh %zu\npp_particles %zu\npp_diag %zu\n", sizeof(pp_params), sizeof(pp_mesh),
         sizeof(pp_particles), sizeof(pp_diag));
  P(pp_params, dt); P(pp_params, shape_order); P(pp_params, alpha); P(pp_params, precision);
  P(pp_params, relax_tol); P(pp_params, relax_max_iter); P(pp_params, rho_background);
  P(pp_particles, cell); P(pp_particles, u); P(pp_particles, id); P(pp_particles, id_alt);
  P(pp_diag, field_E); P(pp_diag, relax_iters); P(pp_diag, flags); P(pp_diag, step);
  return 0;
}
"""
    with tempfile.TemporaryDirectory() as td:
        c = os.path.join(td, "lay.c")
        exe = os.path.join(td, "lay")
        open(c, "w").write(src)
        subprocess.check_call(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), c, "-o", exe])
        out = subprocess.check_output([exe], text=True).split("\n")
    vals = dict(l.split() for l in out if l.strip())
    assert int(vals["pp_params"]) == ctypes.sizeof(pp.pp_params)
    assert int(vals["pp_mesh"]) == ctypes.sizeof(pp.pp_mesh)
    assert int(vals["pp_particles"]) == ctypes.sizeof(pp.pp_particles)
    assert int(vals["pp_diag"]) == ctypes.sizeof(pp.pp_diag)
    for key, v in vals.items():
        if "." in key:
            T, F = key.split(".")
            assert int(v) == getattr(getattr(pp, T), F).offset, key


def test_mmi_generator_binding_marshals_every_argument():
    # an empty range returns before any device work, after the argument checks: the ctypes
    # signature of the loader (quiet flag, lattice pointer, split mode, the pointer tables)
    # reaches the library intact, and a lattice extent below 1 is refused
    import torch
    from paper_1211_4575_amd import inputs_device as ind
    n = (8, 6, 5)
    cells = [torch.empty(1, dtype=torch.int32) for _ in range(4)]
    offs = [[torch.empty(1, dtype=torch.float32) for _ in range(3)] for _ in range(4)]
    us = [[torch.empty(1, dtype=torch.float32) for _ in range(3)] for _ in range(4)]
    for quiet, lattice in ((False, None), (True, None), (True, (2, 2, 5))):
        ind.mmi(1, n, 0, 0, 4.0, 0.01, 0.1, 1836.0, 2, cells, offs, us, None, quiet=quiet, lattice=lattice)
    with pytest.raises(RuntimeError):
        ind.mmi(1, n, 0, 0, 4.0, 0.01, 0.1, 1836.0, 2, cells, offs, us, None, lattice=(0, 2, 5))
