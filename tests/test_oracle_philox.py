"""Pins the oracle's Philox4x32-10 (Salmon et al., SC'11) against an independent
implementation: PyTorch's header-only engine, compiled and called by this test."""
import subprocess

import numpy as np
import pytest

from tests.inputs import random_words


def _torch_ref(native_bin, rows):
    exe = native_bin("philox_torch_ref.cpp")
    text = "\n".join(" ".join(str(int(v)) for v in r) for r in rows) + "\n"
    out = subprocess.run([exe], input=text, capture_output=True, text=True, check=True).stdout
    return np.array([[int(v) for v in line.split()] for line in out.strip().splitlines()], dtype=np.uint64)


def test_philox_matches_independent_header(native_bin, oracle_lib):
    w = random_words(6 * 400, seed=20110104).reshape(400, 6)
    special = np.array(
        [[0, 0, 0, 0, 0, 0],
         [0xFFFFFFFF] * 6,
         [1, 0, 0, 0, 0, 0],
         [0, 1, 0, 0, 0, 0],
         [0, 0, 1, 0, 0, 0],
         [0, 0, 0, 1, 0, 0],
         [0, 0, 0, 0, 1, 0],
         [0, 0, 0, 0, 0, 1],
         [12345, 7, 0, 2, 1, 0]], dtype=np.uint32)
    rows = np.concatenate([special, w])
    ref = _torch_ref(native_bin, rows)
    got = np.array([oracle_lib.philox4x32_10(r[:4], r[4:]) for r in rows], dtype=np.uint64)
    assert np.array_equal(got, ref)


def test_philox_words_look_uniform(oracle_lib):
    # 4096 blocks along the first counter word: byte histogram chi^2 over 256 bins.
    words = np.concatenate([oracle_lib.philox4x32_10([i, 5, 0, 1], [1, 0]) for i in range(4096)])
    b = words.view(np.uint8)
    counts = np.bincount(b, minlength=256)
    expected = b.size / 256
    chi2 = float(((counts - expected) ** 2 / expected).sum())
    # 255 degrees of freedom: mean 255, sd ~22.6; 6 sd band
    assert 120 < chi2 < 390


def test_counter_and_key_words_all_matter(oracle_lib):
    base = oracle_lib.philox4x32_10([1, 2, 3, 4], [5, 6])
    for i in range(6):
        v = [1, 2, 3, 4, 5, 6]
        v[i] ^= 1
        other = oracle_lib.philox4x32_10(v[:4], v[4:])
        assert not np.array_equal(base, other)
