"""The C-ABI library loads on the host and exports every declared symbol.

No compute call is made (there may be no GPU): only dlopen/dlsym, the
argument checks that run on the host before anything touches a device, and
pimc_strerror.
"""

import ctypes as C
import os

import pytest

from paper_1103_4887_amd import _lib as L


def test_library_built():
    assert os.path.exists(L.LIB_PATH), "run __graft_entry__.build() first"


def test_exports_every_declared_function():
    names = L.header_functions()
    assert {"pimc_action", "pimc_sweep", "pimc_param_update", "pimc_grad", "pimc_run_batch",
            "pimc_ctx_create", "pimc_ctx_destroy", "pimc_sync", "pimc_strerror"} <= set(names)
    lib = C.CDLL(L.LIB_PATH)
    for n in names:
        assert hasattr(lib, n), n
    assert set(L._SIGS) >= set(names)


def test_strerror_and_null_arguments():
    lib = L.load()
    assert lib.pimc_strerror(0) == b"ok"
    assert b"box" in lib.pimc_strerror(L.PIMC_ERR_BOX)
    m = L.Model()
    pa = L.Path()
    rng = L.Rng()
    # null context / path are rejected before any device work
    assert lib.pimc_action(None, C.byref(m), C.byref(pa), None, None) == L.PIMC_ERR_ARG
    assert lib.pimc_sweep(None, C.byref(m), C.byref(pa), rng, None, 1, 3, None, None, None) == L.PIMC_ERR_ARG
    assert lib.pimc_grad(None, C.byref(m), C.byref(pa), None, None, None) == L.PIMC_ERR_ARG
    assert lib.pimc_param_update(None, C.byref(m), C.byref(pa), rng, None, None, None) == L.PIMC_ERR_ARG
    assert lib.pimc_run_batch(None, C.byref(m), None, 0, 0, None, 1, 3, None, None) == L.PIMC_ERR_ARG
    assert lib.pimc_sync(None, None) == L.PIMC_ERR_ARG
    assert lib.pimc_set_sweep_tile(None, 4) == L.PIMC_ERR_ARG


def test_struct_layout_matches_header(tmp_path):
    """Every ctypes struct of the binding has the size and field offsets that
    the C compiler gives the header's struct (compiled here with gcc)."""
    import shutil
    import subprocess

    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    structs = {"pimc_model": L.Model, "pimc_path": L.Path, "pimc_rng": L.Rng, "pimc_stats": L.Stats,
               "pimc_batch_stats": L.BatchStats, "pimc_debug": L.Debug, "pimc_batch": L.Batch,
               "pimc_hmc_stats": L.HmcStats, "pimc_init_phase": L.InitPhase}
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "pimc.h"', "int main(void) {"]
    for cname, py in structs.items():
        lines.append(f'  printf("{cname} size %zu\\n", sizeof({cname}));')
        for fname, _ in py._fields_:
            lines.append(f'  printf("{cname} {fname} %zu\\n", offsetof({cname}, {fname}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.dirname(L.HEADER), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {tuple(l.split()[:2]): int(l.split()[2]) for l in out if l.strip()}
    for cname, py in structs.items():
        assert got[(cname, "size")] == C.sizeof(py), cname
        for fname, _ in py._fields_:
            assert got[(cname, fname)] == getattr(py, fname).offset, (cname, fname)
