"""Pins of the oracle's random streams (Philox4x32-10 and the uniform maps)."""
import ctypes as C
import os

import numpy as np
import pytest

import oracle

GOLD = os.path.join(os.path.dirname(__file__), "golden", "philox4x32_10_kat.txt")


def _kat():
    rows = []
    for line in open(GOLD):
        if line.startswith("#") or not line.strip():
            continue
        v = [int(x, 16) for x in line.split()]
        rows.append((v[0:4], v[4:6], v[6:10]))
    return rows


@pytest.mark.parametrize("ctr,key,expect", _kat())
def test_philox_known_answers(ctr, key, expect):
    assert list(oracle.philox4x32_10(ctr, key)) == expect


def test_uniform_maps_are_exact_word_maps():
    # f32: top 24 bits of each word; f64: top 53 bits of two words (first high)
    seed, tag, idx, step = 0xDEADBEEF12345678, 0, 77, 9
    key = [seed & 0xFFFFFFFF, seed >> 32]
    words = np.concatenate([oracle.philox4x32_10([idx, step, b, tag], key) for b in range(4)])
    u32 = oracle.uniforms(seed, tag, idx, step, 0, 16)
    np.testing.assert_array_equal(u32, (words >> 8).astype(np.float64) * 2.0 ** -24)
    u64 = oracle.uniforms(seed, tag, idx, step, 1, 8)
    w = words.astype(np.uint64)
    expect = (((w[0::2] << np.uint64(32)) | w[1::2]) >> np.uint64(11)).astype(np.float64) * 2.0 ** -53
    np.testing.assert_array_equal(u64, expect)
    assert u32.min() >= 0 and u32.max() < 1 and u64.min() >= 0 and u64.max() < 1


def test_uniform_chi_square_and_moments():
    u = np.concatenate([oracle.uniforms(1, 0, i, 3, 0, 1000) for i in range(200)])
    h, _ = np.histogram(u, bins=100, range=(0, 1))
    e = len(u) / 100
    chi2 = ((h - e) ** 2 / e).sum()
    assert chi2 < 160  # 99 dof, p ~ 1e-4 threshold
    assert abs(u.mean() - 0.5) < 5 * np.sqrt(1 / 12 / len(u))
    assert abs(u.var() - 1 / 12) < 0.002


def test_streams_differ_by_every_key_component():
    base = oracle.uniforms(5, 0, 10, 20, 0, 8)
    for args in [(6, 0, 10, 20), (5, 1, 10, 20), (5, 0, 11, 20), (5, 0, 10, 21)]:
        assert not np.array_equal(base, oracle.uniforms(*args, 0, 8))


@pytest.mark.gpu
def test_philox_matches_rocrand_host_generator():
    """rocRAND's Philox4x32-10 host generator (run as a library) must give the
    same blocks for counter {i, 0, 0, 0} and key = seed."""
    try:
        L = C.CDLL("librocrand.so")
    except OSError:
        pytest.skip("librocrand not loadable")
    gen = C.c_void_p()
    if L.rocrand_create_generator_host(C.byref(gen), 404) != 0:
        pytest.skip("no rocRAND host generator")
    seed = 0x0123456789ABCDEF
    L.rocrand_set_seed(gen, C.c_ulonglong(seed))
    buf = np.zeros(64, np.uint32)
    st = L.rocrand_generate(gen, buf.ctypes.data_as(C.c_void_p), C.c_size_t(64))
    L.rocrand_destroy_generator(gen)
    if st != 0:
        pytest.skip("rocRAND host generator unavailable (status %d)" % st)
    key = [seed & 0xFFFFFFFF, seed >> 32]
    ours = np.concatenate([oracle.philox4x32_10([i, 0, 0, 0], key) for i in range(16)])
    np.testing.assert_array_equal(ours, buf)
