"""Host logic of tests/accuracy_report.py (CPU): the GPU phase's x-plane parts are joined back
into the whole lattice, gaps and short coverage are refused, and the oracle phase's bounded map
keeps no more results ahead than asked for."""

import concurrent.futures as cf
import os
import sys
import threading
import time

import numpy as np
import pytest

sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
import accuracy_report as A  # noqa: E402


@pytest.fixture
def split_case(monkeypatch):
    # a 64^3 workload at full resolution, split into parts of 24 x-planes (24 + 24 + 16)
    monkeypatch.setitem(A.CASES, "t64", ("c64_fp64", "fp32", 1, 1, ("psi1",), None, 24))
    return "t64"


def _write_parts(tmp_path, case, F, R, parts):
    paths = []
    for p in parts:
        lo = 24 * p
        d = {f"{case}|F@{lo}": F[lo:lo + 24], f"{case}|R@{lo}": R[lo:lo + 24]}
        if p == 0:
            d[f"{case}|psi1"] = np.ones((3, 64, 64, 64), np.float32)
        path = str(tmp_path / f"part{p}.npz")
        np.savez_compressed(path, **d)
        paths.append(path)
    return paths


def test_parts_join_in_any_file_order(tmp_path, split_case):
    assert A.case_parts(split_case) == 3
    rng = np.random.default_rng(1)
    F = rng.random((64, 64, 64), dtype=np.float32)
    R = rng.integers(0, 30, (64, 64, 64), dtype=np.uint8)
    paths = _write_parts(tmp_path, split_case, F, R, [0, 1, 2])
    g = A.load_gpu(paths[::-1])[split_case]
    assert np.array_equal(g["F"], F) and np.array_equal(g["R"], R)
    assert sorted(g) == ["F", "R", "psi1"]


def test_missing_part_is_refused(tmp_path, split_case):
    F = np.zeros((64, 64, 64), np.float32)
    R = np.zeros((64, 64, 64), np.uint8)
    with pytest.raises(SystemExit, match="do not cover"):
        A.load_gpu(_write_parts(tmp_path, split_case, F, R, [0, 2]))
    with pytest.raises(SystemExit, match="lattice is"):
        A.load_gpu(_write_parts(tmp_path, split_case, F, R, [0, 1]))


def test_every_case_has_parts_that_tile_its_lattice():
    for case, (wl, _, fs, _, _, sel, slab) in A.CASES.items():
        n = A.W.CONFIGS[wl]["n"]
        m = (n + fs - 1) // fs
        parts = A.case_parts(case)
        assert parts >= 1
        if slab is not None:
            assert (parts - 1) * slab < m <= parts * slab
        if sel is not None:
            assert sel[0] == 0 and sel[-1] == A.W.CONFIGS[wl]["n_radii"] - 1 and len(sel) >= 5


@pytest.mark.parametrize("ahead", [0, 1, 3])
def test_bounded_map_keeps_order_and_bound(ahead):
    alive = [0, 0]
    lock = threading.Lock()

    def fn(x):
        with lock:
            alive[0] += 1
            alive[1] = max(alive[1], alive[0])
        time.sleep(0.005)
        return x * x

    out = []
    with cf.ThreadPoolExecutor(max(1, ahead)) as ex:
        for r in A.bounded_map(ex, fn, range(12), ahead):
            out.append(r)
            time.sleep(0.01)
            with lock:
                alive[0] -= 1
    assert out == [x * x for x in range(12)]
    assert alive[1] <= ahead + 1
