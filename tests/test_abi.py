"""The C-ABI library loads and exports every symbol include/pf.h declares, and
the ctypes structures match the C layout (CPU only: no compute calls)."""
import os
import re
import subprocess
import tempfile

import pytest

import paper_2401_01672_amd as pf

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pf.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[\w\s\*]+?\b(pf_\w+)\s*\(", text, flags=re.M)
    return sorted(set(names))


def test_header_declares_entry_points():
    names = declared_functions()
    for required in ("pf_create", "pf_destroy", "pf_rhs", "pf_rkm_step", "pf_integrate",
                     "pf_set_state", "pf_get_state", "pf_last_error"):
        assert required in names


def test_library_exports_every_declared_symbol():
    L = pf.lib()
    bound = {n for n, _, _ in pf.SIGNATURES}
    for name in declared_functions():
        assert hasattr(L, name), f"{name} declared in pf.h but not exported"
        assert name in bound, f"{name} has no ctypes signature in the binding"
    assert L.pf_abi_version() == 2


def declared_parameters():
    """{function: [parameter declarations]} from include/pf.h."""
    text = re.sub(r"/\*.*?\*/", "", open(HEADER).read(), flags=re.S)
    out = {}
    for m in re.finditer(r"\b(pf_\w+)\s*\(([^;{]*?)\)\s*;", text, flags=re.S):
        args = " ".join(m.group(2).split())
        out[m.group(1)] = [] if args in ("", "void") else [a.strip() for a in args.split(",")]
    return out


def test_binding_arity_matches_header():
    decl = declared_parameters()
    for name, _, args in pf.SIGNATURES:
        assert name in decl, name
        assert len(args) == len(decl[name]), (name, len(args), decl[name])


def test_stream_arguments_of_the_boundary():
    """The state copies, the right-hand side, the batch and the warm start
    take the stream to work on as their last argument."""
    decl = declared_parameters()
    for name in ("pf_set_state", "pf_get_state", "pf_rhs", "pf_warmstart"):
        assert decl[name][-1] == "uintptr_t stream", (name, decl[name])
    assert "uintptr_t stream" in decl["pf_batch_integrate"]


def test_error_paths_without_gpu():
    L = pf.lib()
    import ctypes as C
    h = C.c_void_p()
    P = pf.PFParams()
    P.n1 = 0  # invalid size: rejected before any device call
    rc = L.pf_create(C.byref(P), C.c_void_p(0), C.byref(h))
    assert rc == pf.PF_EINVAL
    assert b"non-NULL" in L.pf_last_error(None) or b"grid" in L.pf_last_error(None)
    assert L.pf_set_loop(None, 16, 1) == pf.PF_EINVAL
    assert L.pf_set_stage_tiles(None, None) == pf.PF_EINVAL
    assert L.pf_num_cells(None) == -1
    L.pf_destroy(None)


def _c_layout():
    src = r'''
#include <stdio.h>
#include <stddef.h>
#include "pf.h"
int main(void) {
  printf("%zu %zu %zu\n", sizeof(pf_params), sizeof(pf_step_info), sizeof(pf_run_stats));
  printf("%zu %zu %zu %zu\n", offsetof(pf_params, h), offsetof(pf_params, lam),
         offsetof(pf_params, tol), offsetof(pf_params, dt_max));
  printf("%zu %zu\n", offsetof(pf_run_stats, ice_count), offsetof(pf_run_stats, status));
  printf("%zu %zu\n", offsetof(pf_params, rho_c_separate), offsetof(pf_params, L));
  return 0;
}
'''
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "l.c")
        exe = os.path.join(d, "l")
        open(c, "w").write(src)
        subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), c, "-o", exe], check=True)
        out = subprocess.run([exe], capture_output=True, text=True, check=True).stdout.split()
    return [int(x) for x in out]


def test_ctypes_structs_match_c_layout():
    import ctypes as C
    v = _c_layout()
    assert v[0] == C.sizeof(pf.PFParams)
    assert v[1] == C.sizeof(pf.PFStepInfo)
    assert v[2] == C.sizeof(pf.PFRunStats)
    assert v[3] == pf.PFParams.h.offset
    assert v[4] == pf.PFParams.lam.offset
    assert v[5] == pf.PFParams.tol.offset
    assert v[6] == pf.PFParams.dt_max.offset
    assert v[7] == pf.PFRunStats.ice_count.offset
    assert v[8] == pf.PFRunStats.status.offset
    assert v[9] == pf.PFParams.rho_c_separate.offset
    assert v[10] == pf.PFParams.L.offset


def test_make_params_from_case():
    import pf_inputs as pi
    c = pi.case_coupled_128()
    P = pf.make_params(c.params, "fp32", c.run)
    assert (P.n1, P.n2, P.n3) == (128, 128, 128)
    assert P.model == 1 and P.precision == 1 and P.dirichlet_faces == 16
    assert P.tol == 1e-6 and abs(P.lam[1] - 2.2) < 1e-15
