"""The C ABI without a GPU: the library loads, exports every function that
include/dpsim.h declares, its struct layout matches the ctypes mirror, and the
host-only entry points (footprint, argument validation) behave."""
import ctypes as C
import os
import re
import subprocess
import tempfile

import numpy as np
import pytest

import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "dpsim.h")


def _lib():
    from paper_1808_04338_amd import _lib as L

    if not os.path.exists(L.LIB_PATH):
        pytest.skip("libdpsim.so not built (run __graft_entry__.build())")
    return L, L.load()


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:dp_status|const char \*)\s*(\w+)\s*\(", text, flags=re.M)))


def test_header_declares_the_hot_path():
    names = declared_functions()
    for f in ("sim_create", "assemble_residual_jacobian", "cpr_fpf_setup", "krylov_solve",
              "newton_step", "timestep", "sim_footprint", "sim_destroy", "batch_timestep"):
        assert f in names


def test_library_exports_every_declared_symbol():
    L, lib = _lib()
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_struct_layout_matches_ctypes():
    L, _ = _lib()
    src = r"""
#include <stdio.h>
#include <stddef.h>
#include "dpsim.h"
int main(void) {
  printf("%zu %zu %zu %zu\n", sizeof(dp_well), sizeof(dp_sim_desc), sizeof(dp_newton_info), sizeof(dp_step_info));
  printf("%zu %zu %zu %zu\n", offsetof(dp_sim_desc, wells), offsetof(dp_sim_desc, precond_precision),
         offsetof(dp_sim_desc, newton_tol), offsetof(dp_well, target));
  return 0;
}
"""
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "t.c")
        exe = os.path.join(d, "t")
        open(c, "w").write(src)
        subprocess.run(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), c, "-o", exe], check=True)
        out = subprocess.run([exe], capture_output=True, text=True, check=True).stdout.split()
    sizes = list(map(int, out))
    assert sizes[0] == C.sizeof(L.DpWell)
    assert sizes[1] == C.sizeof(L.DpSimDesc)
    assert sizes[2] == C.sizeof(L.DpNewtonInfo)
    assert sizes[3] == C.sizeof(L.DpStepInfo)
    assert sizes[4] == L.DpSimDesc.wells.offset
    assert sizes[5] == L.DpSimDesc.precond_precision.offset
    assert sizes[6] == L.DpSimDesc.newton_tol.offset
    assert sizes[7] == L.DpWell.target.offset


def test_footprint_is_host_only_and_grows_with_size():
    from paper_1808_04338_amd import footprint

    _lib()
    f0 = footprint(synth.model_small())
    f1 = footprint(synth.model_layered())
    assert 0 < f0 < f1
    assert footprint(synth.model_small(), "fp32") <= f0 + (1 << 20)


def test_invalid_descriptors_are_rejected():
    from paper_1808_04338_amd import footprint
    from paper_1808_04338_amd._lib import DP_E_INVALID, DpError

    _lib()
    m = synth.model_small()
    bad = dict(m, nx=0)
    with pytest.raises(DpError) as e:
        footprint(bad)
    assert e.value.code == DP_E_INVALID
    w = [dict(m["wells"][0], i=99)]
    with pytest.raises(DpError):
        footprint(dict(m, wells=w))
    # two wells perforating one cell
    w2 = [m["wells"][0], dict(m["wells"][0])]
    with pytest.raises(DpError):
        footprint(dict(m, wells=w2))
    with pytest.raises(DpError):
        footprint(m, gmres_restart=64)


def test_invalid_solver_variants_and_well_options_are_rejected():
    """Descriptor fields the Python mapping cannot produce (set directly on the
    struct) and well options that do not fit the well kind fail in the host-only
    validation with DP_E_INVALID."""
    from paper_1808_04338_amd import _lib as L
    from paper_1808_04338_amd import footprint
    from paper_1808_04338_amd.sim import make_desc

    lib = L.load()
    m = synth.model_small()
    for field, val in (("decoupling", 3), ("decoupling", -1), ("cpr_variant", 2), ("c_r", float("nan")),
                       ("c_r", float("inf"))):
        d, keep = make_desc(m, None)
        setattr(d, field, val)
        nbytes = C.c_size_t()
        assert lib.sim_footprint(C.byref(d), C.byref(nbytes)) == L.DP_E_INVALID, (field, val)
    for bad in (dict(m["wells"][0], control="orate"),  # oil-rate control on an injector
                dict(m["wells"][0], wi=-1.0),
                dict(m["wells"][0], wi=float("nan"))):
        with pytest.raises(L.DpError) as e:
            footprint(dict(m, wells=[bad] + m["wells"][1:]))
        assert e.value.code == L.DP_E_INVALID
    prod = dict(m["wells"][1], control="rate")  # water-rate control on a producer
    with pytest.raises(L.DpError):
        footprint(dict(m, wells=[m["wells"][0], prod]))
    # the valid variants pass
    for dec in ("gj", "abf", "ti"):
        for cpr in ("fpf", "fp"):
            assert footprint(m, decoupling=dec, cpr_variant=cpr) > 0
    ok = dict(m["wells"][1], control="orate", target=1e-3, bhp_limit=1e6)
    assert footprint(dict(m, wells=[m["wells"][0], ok], c_r=4e-10)) > 0


def test_create_rejects_null_workspace_without_touching_a_gpu():
    L, lib = _lib()
    from paper_1808_04338_amd.sim import _dp, make_desc

    m = synth.model_small()
    d, keep = make_desc(m)
    h = C.c_void_p()
    p0 = np.ascontiguousarray(m["p0"])
    sw0 = np.ascontiguousarray(m["sw0"])
    code = lib.sim_create(C.byref(d), _dp(p0), _dp(sw0), None, 0, None, C.byref(h))
    assert code == L.DP_E_INVALID
    assert b"workspace" in lib.sim_last_error(None)
