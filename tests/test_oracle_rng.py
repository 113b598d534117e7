"""Pins for the oracle's counter-based noise (Sec. 1, eq. random_props)."""
import numpy as np

from conftest import read_golden
from oracle import rng


def test_splitmix64_published_stream():
    want = [int(v) for v in read_golden("splitmix64_seed1234567.txt")]
    got = [int(v) for v in rng.splitmix64_stream(1234567, 5)]
    assert got == want


def test_words_are_splitmix_outputs_of_hashed_key():
    # word_i is output i+1 of SplitMix64 started from mix64(key)
    key = rng.stream_key(99, rng.PURPOSE_SAMPLE, 2, 17)
    state0 = int(rng.mix64(np.uint64(key)))
    assert np.array_equal(rng.words(99, rng.PURPOSE_SAMPLE, 2, 17, 8),
                          rng.splitmix64_stream(state0, 8))


def test_isotropy_moments():
    # E|z_i|^2 = 1 exactly per element; E[z_i z_j] = 0 (i != j) and E[z] = 0
    n, m = 256, 400
    for kind in (rng.RADEMACHER, rng.Z2Z2):
        Z = rng.noise_block(kind, 7, rng.PURPOSE_SAMPLE, 0, 0, m, n)
        assert np.allclose(np.abs(Z) ** 2, 1.0, atol=1e-15)
        # mean of z over n*m entries: sd 1/sqrt(n m)
        assert abs(Z.mean()) < 5.0 / np.sqrt(n * m)
        # E[z_i z_j] for i != j over columns: (Z Z^T)_ij / m has sd 1/sqrt(m)
        C = (Z @ Z.T) / m
        off = C[~np.eye(n, dtype=bool)]
        assert np.max(np.abs(off)) < 6.0 / np.sqrt(m)
        assert abs(np.mean(off)) < 5.0 / np.sqrt(m * n * (n - 1) / 2)


def test_z2z2_second_moment_vanishes():
    # E[z^2] = 0 for Z2xZ2 (the Z4 property behind ||offdiag(A)||_F^2)
    z = rng.noise_vector(rng.Z2Z2, 3, rng.PURPOSE_SAMPLE, 1, 5, 200000)
    assert abs(np.mean(z * z)) < 5.0 / np.sqrt(200000)


def test_neighbouring_seeds_do_not_share_vectors():
    a = rng.noise_block(rng.Z2Z2, 2000, rng.PURPOSE_SAMPLE, 0, 0, 8, 32)
    b = rng.noise_block(rng.Z2Z2, 2001, rng.PURPOSE_SAMPLE, 0, 0, 8, 32)
    for i in range(8):
        for j in range(8):
            assert not np.array_equal(a[:, i], b[:, j])


def test_keys_separate_streams():
    a = rng.noise_vector(rng.Z2Z2, 1, rng.PURPOSE_SAMPLE, 0, 0, 64)
    for args in [(1, rng.PURPOSE_SKETCH, 0, 0), (1, rng.PURPOSE_SAMPLE, 1, 0),
                 (1, rng.PURPOSE_SAMPLE, 0, 1), (2, rng.PURPOSE_SAMPLE, 0, 0)]:
        b = rng.noise_vector(rng.Z2Z2, *args, 64)
        assert not np.array_equal(a, b)
    # counter access: element i does not depend on the vector length
    long = rng.noise_vector(rng.Z2Z2, 1, rng.PURPOSE_SAMPLE, 0, 0, 1000)
    assert np.array_equal(long[:64], a)
