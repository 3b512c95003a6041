"""The NURSD-vs-RSD-sum gap (NUFFT section: the interpolation error is called
negligible for well-sampled relays), as stored by tests/golden/method_gap.py.

The stored table is the oracle's own report (O1 against the brute-force sum
O2, per workload and upsampling q); these tests check that it is complete,
that it behaves as the sampling argument says (the gap shrinks when the frame
pitch drops below half the shortest wavelength, and is small where the relays
are already sampled that finely), and that its tiny-workload rows are what
the oracle computes now.
"""
import importlib.util
import os

import numpy as np
import pytest

HERE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _table():
    rows = {}
    with open(os.path.join(HERE, "method_gap.txt")) as fh:
        for line in fh:
            if line.startswith("#") or not line.strip():
                continue
            name, q, M, nb, nz, nv, gv, gi = [c.strip() for c in line.split("|")]
            rows[(name, int(q))] = dict(M=int(M), bins=int(nb), planes=int(nz), voxels=int(nv),
                                        gap=float(gv), gap_I=float(gi))
    return rows


def test_table_covers_every_workload():
    rows = _table()
    for key in [("tiny", 1), ("tiny", 2), ("tiny", 4), ("spad", 1), ("spad", 2), ("srsd", 1),
                ("frustum_points", 1), ("srsd_points", 1)]:
        assert key in rows, key
        r = rows[key]
        assert np.isfinite(r["gap"]) and 0 < r["gap"] < 1
        assert r["voxels"] >= 1024


def test_gap_shrinks_with_upsampling():
    rows = _table()
    # the tiny workload's 31.25 mm pitch is above half the shortest wavelength:
    # halving the pitch must cut the gap by a large factor
    assert rows[("tiny", 2)]["gap"] < 0.1 * rows[("tiny", 1)]["gap"]
    assert rows[("tiny", 4)]["gap"] < rows[("tiny", 2)]["gap"]
    # the SPAD frame (7.8 mm) is already far below it: the gap is at the
    # parity tolerance and upsampling does not make it larger
    assert rows[("spad", 1)]["gap"] < 1e-4
    assert rows[("spad", 2)]["gap"] <= rows[("spad", 1)]["gap"]


def test_tiny_rows_reproduce():
    spec = importlib.util.spec_from_file_location("method_gap", os.path.join(HERE, "method_gap.py"))
    mg = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mg)
    rows = _table()
    for q, M, gv, gi, nv in mg.tiny_rows():
        r = rows[("tiny", q)]
        assert r["M"] == M and r["voxels"] == nv
        assert gv == pytest.approx(r["gap"], rel=1e-3)
        assert gi == pytest.approx(r["gap_I"], rel=1e-3)
