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


def test_struct_layout_matches_header():
    # sizes fixed by the header's field order (all naturally aligned)
    assert C.sizeof(L.Model) == 8 * (1 + 1 + 4 + 1 + 12 + 8 + 14) + 8
    assert C.sizeof(L.Path) == 8 + 8 + 4 * 8
    assert C.sizeof(L.Rng) == 24
    assert C.sizeof(L.Stats) == 9 * 8
    assert C.sizeof(L.BatchStats) == 9 * 8
    assert C.sizeof(L.Debug) == 6 * 8
    assert C.sizeof(L.Batch) == 8 + 6 * 8
