"""Host checks of the row-panel tables (the library's panel builder, compiled
for the CPU from its own header, replayed by tests/panel_sim.cpp the way the
kernel walks them).

The replay starts every group of panels with NaN in all LDS slots, stages
what each panel's table names, and forms L_r x from the slots the entries
point at. A missing or misplaced staged row therefore shows up as a NaN or a
wrong value in y, which must equal the plain sparse product L_r x."""
import os
import shutil
import subprocess

import numpy as np
import pytest
import scipy.sparse as sp

import synth
from synth.configs import grid_coords

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def sim(tmp_path_factory):
    if shutil.which("g++") is None:
        pytest.skip("g++ not available")
    d = tmp_path_factory.mktemp("panel_sim")
    exe = str(d / "panel_sim")
    subprocess.run(["g++", "-O2", "-std=c++17", "-Wall", "-Werror",
                    "-I", os.path.join(ROOT, "paper_1602_02070_amd", "csrc"),
                    os.path.join(ROOT, "tests", "panel_sim.cpp"), "-o", exe], check=True)

    def run(L, mask, x, umax):
        L = sp.csr_matrix(L)
        L.sort_indices()
        inp, out = str(d / "in.bin"), str(d / "out.bin")
        with open(inp, "wb") as f:
            np.array([L.shape[0], L.nnz], dtype=np.int64).tofile(f)
            L.indptr.astype(np.int32).tofile(f)
            L.indices.astype(np.int32).tofile(f)
            L.data.astype(np.float64).tofile(f)
            np.asarray(mask, dtype=np.uint8).tofile(f)
            np.asarray(x, dtype=np.float64).tofile(f)
        r = subprocess.run([exe, inp, out, str(umax)], capture_output=True, text=True)
        assert r.returncode == 0, r.stderr
        if r.stdout.startswith("no_tables"):
            return None, None
        stats = dict(zip(r.stdout.split()[::2], map(int, r.stdout.split()[1::2])))
        return np.fromfile(out, dtype=np.float64), stats

    return run


def _check(sim, L, umax, seed=0):
    rng = np.random.default_rng(seed)
    x = rng.standard_normal(L.shape[0])
    mask = rng.random(L.shape[0]) < 0.3
    y, st = sim(L, mask, x, umax)
    assert y is not None
    ref = L @ x
    assert np.abs(y - ref).max() <= 1e-13 * np.abs(ref).max()
    return st


@pytest.mark.parametrize("umax,bound", [(160, 1.4), (128, 1.6)])
def test_video_grid_tables_reproduce_the_product_and_reuse_rows(sim, umax, bound):
    # the 128 x 160 pixel grid of the video workload (10-NN, 20480 rows):
    # with rows kept in LDS across the panels of a group, every row is staged
    # 1.32 (union bound 160, FP32) or 1.52 (128, FP64) times, where
    # raster-order panels without reuse stage |U| / |panel| = 1.84 and 1.91
    L, _ = synth.knn_laplacian(grid_coords(128, 160), 10)
    st = _check(sim, L, umax)
    assert st["max_rows"] <= 64
    assert st["staged"] / L.shape[0] < bound, st


@pytest.mark.parametrize("shape,umax", [((9, 13), 160), ((20, 24), 128), ((7, 7), 160),
                                        ((40, 48), 128)])
def test_small_grids_and_ragged_panel_counts(sim, shape, umax):
    L, _ = synth.knn_laplacian(grid_coords(*shape), 10)
    _check(sim, L, umax, seed=shape[0])


def test_unstructured_graph_and_isolated_rows(sim):
    rng = np.random.default_rng(3)
    L, _ = synth.knn_laplacian(rng.standard_normal((900, 3)), 5)
    assert (np.diff(L.tocsr().indptr) - 1).max() <= 16  # within the table width
    # append 37 isolated rows (diagonal only) and a 2-row component
    iso = sp.diags(rng.uniform(0.5, 2.0, 37))
    pair = sp.csr_matrix(np.array([[1.0, -1.0], [-1.0, 1.0]]))
    _check(sim, sp.block_diag([L, iso, pair]).tocsr(), 160)


def test_one_row_and_too_many_entries(sim):
    y, st = sim(sp.csr_matrix(np.array([[2.5]])), [1], [3.0], 160)
    assert y is not None and y[0] == 7.5 and st["npan"] == 1
    # a row with 17 off-diagonal entries exceeds the table width: no tables
    n = 18
    W = np.zeros((n, n))
    W[0, 1:] = W[1:, 0] = -1.0
    y, _ = sim(sp.csr_matrix(W + np.diag(-W.sum(1))), np.zeros(n), np.ones(n), 160)
    assert y is None
