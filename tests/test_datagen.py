"""The seeded input generators: determinism and distribution shape."""
import numpy as np

import datagen

MASK = (1 << 64) - 1


def _splitmix_py(seed, c):
    # SplitMix64 (Steele, Lea, Flood 2014) written out independently
    z = (seed + (c + 1) * 0x9E3779B97F4A7C15) & MASK
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK
    return z ^ (z >> 31)


def test_splitmix_published_first_outputs():
    # the first outputs of SplitMix64 started from state 0
    assert datagen.splitmix(0, 0) == 0xE220A8397B1DCDAF
    assert datagen.splitmix(0, 1) == 0x6E789E6AA1B965F4
    for s in [0, 1, 7, 12345]:
        for c in [0, 1, 2, 1000, 2 ** 40]:
            assert datagen.splitmix(s, c) == _splitmix_py(s, c)


def test_uniform_rows_are_addressable_and_thread_invariant():
    a = datagen.uniform_codes(1000, 128, 9, threads=1)
    b = datagen.uniform_codes(1000, 128, 9, threads=8)
    c = datagen.uniform_codes(300, 128, 9, first_row=700)
    assert np.array_equal(a, b) and np.array_equal(a[700:], c)
    assert int(a[3, 1]) == _splitmix_py(9, 3 * 2 + 1)
    bits = np.unpackbits(a.view(np.uint8)).mean()
    assert abs(bits - 0.5) < 0.01


def test_gauss_moments():
    g = np.array([datagen.gauss(2, 3 * i) for i in range(20000)], dtype=np.float64) / 65536.0
    assert abs(g.mean()) < 0.03 and abs(g.std() - 1.0) < 0.03
    assert np.abs(g).max() <= 6.0


def test_clustered_codes_deterministic_and_clustered():
    a = datagen.clustered_codes(400, 128, 4, threads=1)
    b = datagen.clustered_codes(400, 128, 4, threads=8)
    c = datagen.clustered_codes(100, 128, 4, first_row=300)
    assert np.array_equal(a, b) and np.array_equal(a[300:], c)
    # The 128-bit words of the 256-bit stream start with the 128-bit stream
    # (shared means and hyperplanes).
    d = datagen.clustered_codes(400, 256, 4)
    assert np.array_equal(d[:, :2], a)
    # Points of one mixture component sit close: distances between codes are
    # far below the 64 expected for independent uniform 128-bit codes at the
    # low end.
    x = datagen.clustered_codes(3000, 128, 4)
    dd = np.bitwise_count(x[:1] ^ x).sum(axis=1)
    assert np.sort(dd)[1] < 40
    mu, w = datagen.clustered_params(128)
    assert mu.shape == (1000, 128) and w.shape == (128, 128)


def test_request_stream_shape():
    t, sizes, ks = datagen.request_stream(5000, 100.0, (1, 10, 100, 1000))
    assert np.all(np.diff(t) > 0)
    assert sizes.min() >= 1 and sizes.max() <= 4096
    assert abs(np.mean(np.diff(t)) - 0.01) < 0.001
    assert set(np.unique(ks).tolist()) <= {1, 10, 100, 1000}
    # log-uniform sizes: median near sqrt(4097)
    assert 30 < np.median(sizes) < 110
