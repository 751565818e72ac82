"""Pins for the oracle's Philox4x32-10, uniform maps and Box-Muller normals.

The generator is pinned against an independent implementation (rocRAND's
header-only Philox4x32-10, run on the host), not against itself.
"""

import os
import shutil
import subprocess

import numpy as np
import pytest
from scipy import stats

from oracle import philox as px

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "tests", "native", "philox_rocrand_ref.cpp")
BIN = os.path.join(ROOT, "_build", "philox_rocrand_ref")


def _reference_binary():
    if os.path.exists(BIN) and os.path.getmtime(BIN) >= os.path.getmtime(SRC):
        return BIN
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available to build the rocRAND host reference")
    os.makedirs(os.path.dirname(BIN), exist_ok=True)
    subprocess.run([hipcc, "-O1", "-o", BIN, SRC], check=True, capture_output=True)
    return BIN


def test_philox_matches_rocrand_host_reference():
    exe = _reference_binary()
    rng = np.random.Generator(np.random.PCG64(12345))
    cases = rng.integers(0, 2 ** 32, size=(4000, 6), dtype=np.uint64)
    edge = np.array([[0] * 6, [2 ** 32 - 1] * 6, [1, 0, 0, 0, 0, 0], [0, 0, 0, 1, 0, 0],
                     [0, 0, 0, 0, 1, 0], [0, 0, 0, 0, 0, 1]], dtype=np.uint64)
    cases = np.vstack([edge, cases])
    inp = "\n".join(" ".join(str(int(v)) for v in row) for row in cases) + "\n"
    out = subprocess.run([exe], input=inp, capture_output=True, text=True, check=True).stdout
    ref = np.array([[int(t) for t in line.split()] for line in out.strip().splitlines()],
                   dtype=np.uint64)
    got = np.stack(px.philox4x32_10(*[cases[:, i] for i in range(6)]), axis=1)
    assert ref.shape == got.shape
    assert np.array_equal(ref, got)


def test_counter_layout_separates_purposes_and_indices():
    idx = np.arange(4096, dtype=np.uint64)
    seen = set()
    for purpose in (px.PRIOR, px.PROP, px.ACC, px.RESAMP, px.EXCH):
        for move in (0, 1):
            w = px.words(7, idx, 0, 3, purpose, move)[0]
            seen.update(int(v) for v in w)
    # 20480 draws of a 32-bit word: collisions expected ~0.05, allow a few
    assert len(seen) >= 20480 - 3


def test_uniform_maps_are_exact_and_in_range():
    w = np.array([0, 1, 2 ** 31, 2 ** 32 - 1], dtype=np.uint64)
    u = px.u01_open(w)
    assert np.all(u > 0.0) and np.all(u < 1.0)
    assert u[0] == 2.0 ** -33 and u[-1] == 1.0 - 2.0 ** -33
    v = px.u01_left_closed(w)
    assert v[0] == 0.0 and v[-1] == 1.0 - 2.0 ** -32 and np.all(v < 1.0)


def test_box_muller_normals_are_standard_normal():
    idx = np.arange(1 << 16, dtype=np.uint64)
    z = px.normals(99, idx, 1, px.PROP, 0, 8).reshape(-1)
    assert abs(z.mean()) < 4.0 / np.sqrt(z.size)
    assert abs(z.var() - 1.0) < 4.0 * np.sqrt(2.0 / z.size)
    assert stats.kstest(z, "norm").pvalue > 1e-4
    # coordinates are independent of each other (pairwise correlation ~ 0)
    zz = px.normals(99, idx, 1, px.PROP, 0, 8)
    c = np.corrcoef(zz)
    off = c[~np.eye(8, dtype=bool)]
    assert np.max(np.abs(off)) < 5.0 / np.sqrt(idx.size)
