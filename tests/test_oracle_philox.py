"""Pins of the oracle's test-matrix generator (Section 3.1: Gaussian test
matrix Omega_n; Philox4x32-10 of Salmon et al., SC'11)."""
import os
import shutil
import subprocess
import tempfile

import numpy as np
import pytest
from scipy import stats

from oracle import philox

HERE = os.path.dirname(os.path.abspath(__file__))


def _kat(golden_dir):
    rows = []
    with open(os.path.join(golden_dir, "philox4x32_10_kat.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            w = [int(x, 16) for x in line.split()]
            rows.append((w[:4], w[4:6], w[6:10]))
    return rows


def test_known_answer_vectors(golden_dir):
    rows = _kat(golden_dir)
    assert len(rows) == 3
    for ctr, key, want in rows:
        got = philox.philox4x32_10(*ctr, key[0], key[1])
        assert [int(x) for x in got] == want


def _rocrand_block(inputs):
    """Evaluate Philox4x32-10 with rocRAND's header (built for the host)."""
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available to build the rocRAND cross-check")
    src = os.path.join(HERE, "philox_rocrand_check.cpp")
    with tempfile.TemporaryDirectory() as d:
        exe = os.path.join(d, "prc")
        r = subprocess.run([hipcc, "-O1", "-o", exe, src], capture_output=True, text=True, cwd=d)
        if r.returncode != 0:
            pytest.skip("could not build rocRAND cross-check: " + r.stderr[-400:])
        text = "\n".join(" ".join("%08x" % v for v in row) for row in inputs) + "\n"
        out = subprocess.run([exe], input=text, capture_output=True, text=True, check=True).stdout
    return [[int(x, 16) for x in line.split()] for line in out.strip().splitlines()]


def test_matches_independent_implementation():
    rng = np.random.default_rng(7)
    inputs = [list(map(int, rng.integers(0, 2 ** 32, size=6, dtype=np.uint64))) for _ in range(64)]
    # include the exact counters that Omega uses: (j lo, j hi, group, batch<<8|mode)
    inputs += [[j, 0, g, (3 << 8) | 2, 1234, 0] for j in (0, 1, 99999) for g in (0, 7)]
    want = _rocrand_block(inputs)
    c = np.array(inputs, dtype=np.uint64)
    for row, w in zip(c, want):
        got = philox.philox4x32_10(row[0], row[1], row[2], row[3], int(row[4]), int(row[5]))
        assert [int(x) for x in got] == w


def test_vectorised_matches_scalar():
    seed = (77 << 32) | 5
    bits = philox.omega_bits(seed, 2, 3, 10, 5, 2)
    for jj in range(5):
        for g in range(2):
            x = philox.philox4x32_10(10 + jj, 0, g, (3 << 8) | 2, 5, 77)
            assert [int(v) for v in x] == [int(v) for v in bits[jj, 4 * g:4 * g + 4]]


def test_uniform_range_exact():
    bits = np.array([0, 0xFF, 0x100, 0xFFFFFFFF], dtype=np.uint64)
    u = philox.uniforms(bits)
    assert u[0] == 2.0 ** -24 and u[1] == 2.0 ** -24
    assert u[2] == 2.0 * 2.0 ** -24
    assert u[3] == 1.0
    # exact in float32
    assert np.all(u.astype(np.float32).astype(np.float64) == u)


def test_gaussian_moments_and_ks():
    z = philox.omega(seed=11, mode=0, batch=0, row0=0, nrows=250_000, l=4).ravel()
    n = z.size
    assert abs(z.mean()) < 5.0 / np.sqrt(n)
    assert abs(z.var() - 1.0) < 5.0 * np.sqrt(2.0 / n)
    assert stats.kstest(z, "norm").pvalue > 1e-4
    # columns within one counter group are uncorrelated
    Z = philox.omega(seed=11, mode=1, batch=0, row0=0, nrows=200_000, l=8)
    C = np.corrcoef(Z.T)
    off = C[~np.eye(8, dtype=bool)]
    assert np.max(np.abs(off)) < 5.0 / np.sqrt(200_000)


def test_blocks_are_consistent_and_streams_differ():
    full = philox.omega(5, 1, 0, 0, 300, 30)
    part = philox.omega(5, 1, 0, 123, 50, 30)
    np.testing.assert_array_equal(full[123:173], part)
    # width only truncates columns
    np.testing.assert_array_equal(philox.omega(5, 1, 0, 0, 300, 13), full[:, :13])
    # different mode / batch / seed give different matrices
    assert not np.allclose(full, philox.omega(5, 2, 0, 0, 300, 30))
    assert not np.allclose(full, philox.omega(5, 1, 1, 0, 300, 30))
    assert not np.allclose(full, philox.omega(6, 1, 0, 0, 300, 30))
    # rows beyond 2^32 use the high counter word
    hi = philox.omega(5, 1, 0, 2 ** 32, 4, 8)
    lo = philox.omega(5, 1, 0, 0, 4, 8)
    assert not np.allclose(hi, lo)
