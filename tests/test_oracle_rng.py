"""Pins of the oracle's random streams (Philox4x32-10, uniform and normal maps)."""
import os
import shutil
import subprocess

import numpy as np
import pytest
from scipy import stats

from oracle import oracle as O

HERE = os.path.dirname(os.path.abspath(__file__))


def _kats():
    rows = []
    with open(os.path.join(HERE, "golden", "philox4x32_10_kat.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            w = [int(t, 16) for t in line.split()]
            rows.append((w[0:4], w[4:6], w[6:10]))
    return rows


def test_philox_known_answers():
    for ctr, key, out in _kats():
        assert O.philox(ctr, key).tolist() == out


@pytest.mark.skipif(shutil.which("hipcc") is None, reason="needs hipcc to build the rocRAND helper")
def test_philox_matches_rocrand(tmp_path):
    exe = tmp_path / "rrp"
    subprocess.check_call(["hipcc", "-O1", "-x", "hip", "--offload-arch=gfx950", "-w",
                           os.path.join(HERE, "golden", "rocrand_philox_dump.cpp"), "-o", str(exe)],
                          cwd=str(tmp_path))
    g = np.random.default_rng(7)
    words = g.integers(0, 1 << 32, size=(2000, 6), dtype=np.uint64)
    inp = "\n".join(" ".join("%08x" % v for v in row) for row in words) + "\n"
    res = subprocess.run([str(exe)], input=inp, capture_output=True, text=True, check=True)
    got = [[int(t, 16) for t in line.split()] for line in res.stdout.strip().splitlines()]
    assert len(got) == len(words)
    for row, ref in zip(words, got):
        assert O.philox(row[:4], row[4:6]).tolist() == ref


def test_uniform_is_fp32_exact_and_open():
    for w in [0, 1, 511, 512, 0xFFFFFFFF, 0x80000000, 12345678]:
        u = O.lib().orc_u01(w)
        assert 0.0 < u < 1.0
        assert float(np.float32(u)) == u
    assert O.lib().orc_u01(0) == 2.0 ** -24
    assert O.lib().orc_u01(0xFFFFFFFF) == 1.0 - 2.0 ** -24


def test_uniform_stream_moments_and_ks():
    u = np.array([O.uniform(99, c, d, O.ROLE_THRESH) for c in range(100) for d in range(100)])
    assert stats.kstest(u, "uniform").pvalue > 1e-3
    assert abs(u.mean() - 0.5) < 3 * np.sqrt(1 / 12 / u.size)


def test_normal_moments_and_ks():
    z = np.concatenate([O.normals(5, c, 0, O.ROLE_NU, 0, 1000) for c in range(50)])
    assert stats.kstest(z, "norm").pvalue > 1e-3
    n = z.size
    assert abs(z.mean()) < 3 / np.sqrt(n)
    assert abs(z.var() - 1) < 3 * np.sqrt(2 / n)


def test_normal_layout_box_muller_pairs():
    # d = 2q, 2q+1 of block b come from words (2q, 2q+1): r^2 = -2 ln u1 and
    # the angle 2 pi u2.
    seed, chain, draw, role, sub = 11, 3, 4, O.ROLE_PROP, 2
    z = O.normals(seed, chain, draw, role, sub, 16)
    for b in range(4):
        w = O.philox([chain, draw, (role << 24) | sub, b], [seed & 0xFFFFFFFF, seed >> 32])
        for q in range(2):
            u1 = O.lib().orc_u01(int(w[2 * q]))
            u2 = O.lib().orc_u01(int(w[2 * q + 1]))
            z0, z1 = z[4 * b + 2 * q], z[4 * b + 2 * q + 1]
            assert z0 * z0 + z1 * z1 == pytest.approx(-2 * np.log(u1), rel=1e-13)
            ang = np.arctan2(z1, z0) % (2 * np.pi)
            assert ang == pytest.approx(2 * np.pi * u2, abs=1e-12)


def test_streams_are_distinct():
    a = O.normals(1, 0, 0, O.ROLE_NU, 0, 8)
    for args in [(1, 1, 0, O.ROLE_NU, 0), (1, 0, 1, O.ROLE_NU, 0), (1, 0, 0, O.ROLE_INIT, 0),
                 (1, 0, 0, O.ROLE_NU, 1), (2, 0, 0, O.ROLE_NU, 0)]:
        assert not np.array_equal(a, O.normals(*args, 8))
