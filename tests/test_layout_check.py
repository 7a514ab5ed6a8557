"""Host-side bounds check of the sweep kernel's launch shapes (CPU only).

tests/layout_check.cpp is built with the host compiler against the same
ownership, LDS-layout, exchange-offset and shape-choice functions the kernel
and the C ABI use (csrc/layout.hpp), and walks every block and thread of each
launch: every site of a window owned exactly once and updated in its colour,
every neighbour read from where it is published, every LDS and global index
inside its buffer (the block layout of Section 4.3: time-ordered sites split
over threads and, for long windows, over workgroups).

Cases: the launches of the benchmark workloads (every shape the autotuner
tries for the 4096- and 65536-step windows, the 512-window uneven batch),
the FP64 shapes that are refused today (8 sites x 512 threads at M = 4096,
16 tiles x 256 threads at M = 16384, the tiled FP64 parity windows), and a
ragged sweep of window lengths around every tile and workgroup boundary.
A shape too small for its window must be reported, so the check is seen to
detect a broken layout.
"""

from __future__ import annotations

import os
import shutil
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "tests", "layout_check.cpp")
ROCM_INC = "/opt/rocm/include"


@pytest.fixture(scope="module")
def checker(tmp_path_factory):
    cxx = shutil.which("g++")
    if cxx is None or not os.path.isdir(ROCM_INC):
        pytest.skip("host compiler or HIP headers missing")
    exe = str(tmp_path_factory.mktemp("layout") / "layout_check")
    cmd = [cxx, "-std=c++17", "-O2", "-Wall", "-D__HIP_PLATFORM_AMD__", f"-I{ROCM_INC}",
           "-I" + os.path.join(ROOT, "paper_1103_4887_amd", "csrc"), "-I" + os.path.join(ROOT, "include"),
           SRC, "-o", exe]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    return exe


def run(exe, lines):
    p = subprocess.run([exe], input="\n".join(lines) + "\n", capture_output=True, text=True, timeout=600)
    return p.returncode, p.stdout


def single_candidates(M, prec, narrow=False):
    """The (K, T) pairs the launch-shape autotuner times for one window."""
    from paper_1103_4887_amd.autotune import candidates
    return list(candidates(M, prec, narrow))


def test_benchmark_launches(checker):
    from workloads.configs import CONFIGS, batch_sizes
    lines = ["single 256 1 0 0"]                                   # the FP64 window
    for M in (4096, 65536):                                        # every shape the tuner tries
        for K, T in single_candidates(M, "fp32"):
            lines.append(f"single {M} 0 {K} {T}")
        for K, T in single_candidates(M, "fp32", narrow=True):
            lines.append(f"single {M} 0 {K} {T}")
    c = CONFIGS["c4"]
    sizes = batch_sizes(c["B"], c["M_lo"], c["M_hi"], c["data_seed"])
    for K in (0, 4, 8, 16):
        lines.append(f"batch 0 {K} 1 0 " + " ".join(str(int(m)) for m in sizes))
    lines.append("batch 0 16 1 1 " + " ".join(str(int(m)) for m in sizes))
    rc, out = run(checker, lines)
    assert rc == 0, out
    assert "FAIL" not in out
    ok = {ln.split(" K=")[0][3:] for ln in out.splitlines() if ln.startswith("ok ")}
    # the measured launches: the FP64 window, the 4096-step window at 16
    # tiles of 128 threads x 2 sites and automatic, the 65536-step window at
    # 128 tiles of 256 threads x 2 sites, the uneven batch automatic
    for case in ("single 256 1 0 0", "single 4096 0 2 16", "single 4096 0 0 0", "single 65536 0 2 128",
                 "single 65536 0 0 0"):
        assert case in ok, out
    assert any(c.startswith("batch 0 0 1 0 ") for c in ok), out


def test_fp64_wide_and_tiled_shapes(checker):
    """The FP64 shapes that stay refused: their index arithmetic is sound."""
    forced = [
        "forced 4096 1 8 512 1",      # wide single workgroup
        "forced 16384 1 4 256 16",    # 16 time tiles
        "forced 1000 1 4 128 2", "forced 1000 1 4 64 4", "forced 4096 1 4 256 4", "forced 2049 1 4 64 9",
    ]
    lines = forced + [
        "single 16384 1 0 1",         # the oversized window with tiles forced off: no shape
        "single 16384 1 0 0", "single 4096 1 0 0", "single 1025 1 0 0", "single 1000 1 0 2",
        "single 1024 1 0 0",
    ]
    rc, out = run(checker, lines)
    assert rc == 0, out
    for case in forced:
        assert f"ok {case} " in out, out
    assert "(a shape launch_sweep refuses)" in out     # the wide one
    for case in ("single 16384 1 0 1", "single 16384 1 0 0", "single 4096 1 0 0", "single 1025 1 0 0",
                 "single 1000 1 0 2"):
        assert f"refused {case}" in out, out
    assert "ok single 1024 1 0 0 " in out


def test_ragged_windows(checker):
    lines = []
    for M in list(range(1, 300)) + list(range(1010, 1040)) + list(range(4090, 4100)) + [8191, 8192, 8193]:
        lines.append(f"single {M} 0 0 1")
        if M <= 1024:
            lines.append(f"single {M} 1 0 0")
    for T in (2, 3, 4, 8, 9, 16, 17, 64):
        for K in (2, 4):
            for NT in (64, 128, 192, 256):
                S = NT * K
                for M in ((T - 1) * S + 1, (T - 1) * S + 2, T * S - 1, T * S):
                    lines.append(f"forced {M} 0 {K} {NT} {T}")
    rng = np.random.default_rng(7)
    for _ in range(6):
        sizes = rng.integers(1, 9000, size=int(rng.integers(1, 40)))
        lines.append("batch 0 0 1 0 " + " ".join(str(int(m)) for m in sizes))
        lines.append("batch 1 0 1 0 " + " ".join(str(int(m)) for m in sizes if m <= 1024))
    lines.append("batch 0 0 4 0 " + " ".join(["3000"] * 16))
    lines.append("batch 0 2 8 0 " + " ".join(["8000"] * 8))
    rc, out = run(checker, lines)
    assert rc == 0, out
    assert "FAIL" not in out


def test_extended_kernel_shapes(checker):
    """Exact draws, the initialization phase and the Table 1 constants run in
    shapes of at most 4 sites per thread and 256 threads: the automatic
    choice cuts longer windows into time tiles, and a forced wider shape is
    refused."""
    lines = [f"single {M} {p} 0 0 1" for M in (96, 200, 257, 300, 1024, 2048, 2049, 4096) for p in (0, 1)]
    lines += ["single 4096 0 2 16 1", "single 4096 0 0 4 1", "single 4096 0 0 8 1",
              "single 4096 0 16 1 1", "single 4096 0 8 1 1", "single 4096 0 4 1 1"]
    rc, out = run(checker, lines)
    assert rc == 0, out
    ok = {ln.split(" K=")[0][3:]: ln for ln in out.splitlines() if ln.startswith("ok ")}
    for M in (96, 200, 257, 300, 1024, 2048, 2049, 4096):
        case = f"single {M} 0 0 0 1"
        assert case in ok and (" K=4 " in ok[case] or " K=2 " in ok[case]), out
    assert "T=4" in ok["single 4096 0 0 0 1"], out          # 4 tiles of 256 threads x 4 sites
    for case in ("single 4096 0 16 1 1", "single 4096 0 8 1 1", "single 4096 0 4 1 1",
                 "single 2049 1 0 0 1", "single 4096 1 0 0 1"):
        assert f"refused {case}" in out, out


def test_detects_a_layout_too_small(checker):
    # 2 tiles of 64 threads x 4 sites cannot hold 5001 sites
    rc, out = run(checker, ["forced 5000 0 4 64 2"])
    assert rc == 1
    assert "FAIL" in out
