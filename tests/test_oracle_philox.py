"""Pins of the oracle's Philox4x32-10 (Salmon et al., SC'11) and its uniform/normal mapping."""

import os

import numpy as np

from oracle import philox

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "philox4x32_10_kat.txt")


def _kat_rows():
    rows = []
    with open(GOLDEN) as fh:
        for line in fh:
            if line.startswith("#") or not line.strip():
                continue
            rows.append([int(w, 16) for w in line.split()])
    return rows


def test_known_answer_vectors():
    rows = _kat_rows()
    assert len(rows) == 3
    for r in rows:
        out = philox.philox4x32_10(r[0], r[1], r[2], r[3], r[4], r[5])
        assert [int(o) for o in out] == r[6:10]


def test_vectorised_matches_scalar_calls():
    ctr = np.arange(1000, dtype=np.uint64) * 7919 + 12345
    out = philox.philox4x32_10(ctr & 0xFFFFFFFF, ctr >> 32, 3, 4, 0xDEADBEEF, 0x01234567)
    for k in (0, 17, 999):
        one = philox.philox4x32_10(int(ctr[k]) & 0xFFFFFFFF, int(ctr[k]) >> 32, 3, 4,
                                   0xDEADBEEF, 0x01234567)
        assert [int(o[k]) for o in out] == [int(x) for x in one]


def test_uniforms_open_interval_and_exact():
    lo = np.array([0, 0xFFFFFFFF, 0x00000FFF, 0], dtype=np.uint64)
    hi = np.array([0, 0xFFFFFFFF, 0, 0x80000000], dtype=np.uint64)
    u = philox.uniforms_from_words(lo, hi)
    assert u[0] == 2.0 ** -53                      # smallest value: (2*0+1) 2^-53
    assert u[1] == 1.0 - 2.0 ** -53                # largest value, still below 1
    assert u[2] == 2.0 ** -53                      # the 12 low bits are dropped
    assert u[3] == 0.5 + 2.0 ** -53
    assert np.all((u > 0) & (u < 1))


def test_uniform_statistics():
    u1, u2 = philox.mode_uniforms(np.arange(200000, dtype=np.uint64), 42)
    for u in (u1, u2):
        assert abs(u.mean() - 0.5) < 5 * np.sqrt(1 / 12 / u.size)
        assert abs(u.var() - 1 / 12) < 0.002
    assert abs(np.corrcoef(u1, u2)[0, 1]) < 0.01
