"""Host code under the address and undefined-behaviour sanitizers (no GPU).

Two drivers built with the host compiler and -fsanitize=address,undefined
(every report is fatal):
  * tests/native/plan_check.cpp: the native hierarchy builder
    (csrc/hierarchy.cpp) and the setup plan (csrc/plan.hpp: CSR validation,
    ELL conversion, graph and symmetry analysis) on seeded block-diffusion
    hierarchies, then malformed copies (unsorted or out-of-range columns,
    broken row pointers, a zero diagonal, a wrong transfer shape) that must be
    refused with MG_ERR_SHAPE before any out-of-bounds read;
  * tests/native/tiles_check.cpp: the fused convolution's tiling
    (csrc/tiles.hpp: 16-bit local columns, per-item metadata) on grid levels,
    an unstructured mesh and random graphs.
A third, tests/native/concurrent_build.cpp, runs under the thread sanitizer:
four threads build hierarchies at once through the builder's shared worker
threads, and each result must equal the same build done alone."""
import os
import shutil
import subprocess

import numpy as np
import pytest
import scipy.sparse as sp

from mginputs import configs as C, hierarchy as H
from tests.test_tiles_host import _ell, _random_graph

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(ROOT, "paper_2608_29082_amd", "csrc")
SAN = ["-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")


def _build(tmp_path_factory, name, srcs, flags=SAN):
    cxx = shutil.which("g++")
    if cxx is None:
        pytest.skip("no host C++ compiler")
    exe = tmp_path_factory.mktemp(name) / name
    subprocess.run([cxx, *flags, "-std=c++17", "-pthread", "-I", os.path.join(ROOT, "include"), "-I", CSRC,
                    *srcs, "-o", str(exe)], check=True)
    return str(exe)


@pytest.fixture(scope="module")
def plan_driver(tmp_path_factory):
    return _build(tmp_path_factory, "plan_check", [os.path.join(HERE, "native", "plan_check.cpp"),
                                                   os.path.join(CSRC, "hierarchy.cpp")])


@pytest.fixture(scope="module")
def tiles_driver(tmp_path_factory):
    return _build(tmp_path_factory, "tiles_check", [os.path.join(HERE, "native", "tiles_check.cpp")])


def _clean(out):
    assert out.returncode == 0, out.stdout + out.stderr
    assert "runtime error" not in out.stderr and "AddressSanitizer" not in out.stderr, out.stderr


@pytest.mark.parametrize("side,nb,seed", [(33, 4, 1), (65, 16, 2), (129, 16, 3), (257, 16, 4)])
def test_plan_and_hierarchy_under_sanitizers(plan_driver, side, nb, seed):
    out = subprocess.run([plan_driver, str(side), str(nb), str(seed)], capture_output=True, text=True,
                         timeout=300, env=ENV)
    _clean(out)
    lines = out.stdout.split("\n")
    assert lines[-2] == "ok"
    assert any(ln.startswith("rowptr-overrun-sorted 2") for ln in lines)


def _run_tiles(driver, path, KM, side):
    out = subprocess.run([driver, path, str(KM), str(side)], capture_output=True, text=True, timeout=300, env=ENV)
    _clean(out)
    tok = out.stdout.split()
    assert tok[0] == "ok" and float(tok[3]) == 0.0 and int(tok[4]) == 1, out.stdout


def test_tiles_under_sanitizers(tiles_driver, tmp_path):
    hier = H.square_hierarchy(129, H.block_field(C.rng(8, 2, 1), 16, -2, 2))
    for A, (KM, side) in zip(hier.A[:3], [(3, 16), (2, 15), (4, 8)]):
        _run_tiles(tiles_driver, _ell(A, str(tmp_path)), KM, side)
    mesh = H.lshape_hierarchy(C.rng(7, 4, 0), target_nodes=120, refinements=2)
    _run_tiles(tiles_driver, _ell(mesh.A[0], str(tmp_path)), 3, 12)
    A = H.square_hierarchy(33).A[0]
    _run_tiles(tiles_driver, _ell(sp.block_diag([A, A]).tocsr(), str(tmp_path)), 3, 8)
    _run_tiles(tiles_driver, _ell(_random_graph(2000, 2, 1), str(tmp_path)), 2, 8)


def test_concurrent_builds_under_thread_sanitizer(tmp_path_factory):
    exe = _build(tmp_path_factory, "concurrent_build",
                 [os.path.join(HERE, "native", "concurrent_build.cpp"), os.path.join(CSRC, "hierarchy.cpp")],
                 flags=["-O1", "-g", "-fsanitize=thread", "-fno-omit-frame-pointer"])
    out = subprocess.run([exe], capture_output=True, text=True, timeout=600,
                         env=dict(os.environ, TSAN_OPTIONS="halt_on_error=1"))
    assert out.returncode == 0, out.stdout + out.stderr
    assert "ThreadSanitizer" not in out.stderr, out.stderr
    assert out.stdout.split() == ["ok", "0"], out.stdout
