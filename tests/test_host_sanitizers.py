"""The library's host-side C++ (argument checks, row-panel table builder)
compiled for the CPU with the address and undefined-behaviour sanitizers and
exercised on valid and broken inputs. Any out-of-bounds access, leak or
undefined arithmetic aborts the sanitized program."""
import os
import shutil
import subprocess

import numpy as np
import pytest
import scipy.sparse as sp

import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1602_02070_amd", "csrc")
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
       "-g", "-O1", "-std=c++17"]


def _gxx():
    if shutil.which("g++") is None:
        pytest.skip("g++ not available")
    return "g++"


def _env():
    env = dict(os.environ)
    env["ASAN_OPTIONS"] = "detect_leaks=1:abort_on_error=0:exitcode=23"
    env["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1:exitcode=24"
    env.pop("LD_PRELOAD", None)
    return env


def test_argument_checks_under_sanitizers(tmp_path):
    exe = str(tmp_path / "validate_fuzz")
    subprocess.run([_gxx(), *SAN, "-I", os.path.join(ROOT, "include"), "-I", CSRC,
                    os.path.join(ROOT, "tests", "validate_fuzz.cpp"),
                    os.path.join(CSRC, "validate.cpp"), "-o", exe], check=True)
    r = subprocess.run([exe], capture_output=True, text=True, env=_env(), timeout=300)
    assert r.returncode == 0, r.stderr[-3000:]
    assert r.stdout.startswith("ok ") and int(r.stdout.split()[1]) > 2000


def test_panel_builder_under_sanitizers(tmp_path):
    exe = str(tmp_path / "panel_sim")
    subprocess.run([_gxx(), *SAN, "-I", CSRC, os.path.join(ROOT, "tests", "panel_sim.cpp"),
                    "-o", exe], check=True)
    rng = np.random.default_rng(0)
    graphs = [synth.knn_laplacian(synth.grid_coords(40, 48), 10)[0],
              synth.knn_laplacian(rng.standard_normal((500, 3)), 5)[0],
              sp.csr_matrix(np.array([[1.0]]))]
    for k, L in enumerate(graphs):
        L = sp.csr_matrix(L)
        L.sort_indices()
        inp, out = str(tmp_path / f"in{k}.bin"), str(tmp_path / f"out{k}.bin")
        x = rng.standard_normal(L.shape[0])
        with open(inp, "wb") as f:
            np.array([L.shape[0], L.nnz], dtype=np.int64).tofile(f)
            L.indptr.astype(np.int32).tofile(f)
            L.indices.astype(np.int32).tofile(f)
            L.data.astype(np.float64).tofile(f)
            (rng.random(L.shape[0]) < 0.3).astype(np.uint8).tofile(f)
            x.tofile(f)
        for umax in (160, 128):
            r = subprocess.run([exe, inp, out, str(umax)], capture_output=True, text=True,
                               env=_env(), timeout=300)
            assert r.returncode == 0, r.stderr[-3000:]
            if not r.stdout.startswith("no_tables"):
                y = np.fromfile(out, dtype=np.float64)
                assert np.allclose(y, L @ x, rtol=1e-12, atol=1e-12)
