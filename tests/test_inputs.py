"""Checks of the seeded input generators (no method arithmetic lives there)."""
import math

import numpy as np

from paper_2505_06021_amd import inputs


def test_kq_map_is_group_addition():
    kappa, kq = inputs.kgrid((3, 3, 1))
    nk = len(kappa)
    for q in range(nk):
        assert sorted(kq[q]) == list(range(nk))          # a permutation for every q
        for k in range(nk):
            d = (kappa[kq[q, k]] - kappa[k] - kappa[q] + 0.5) % 1.0 - 0.5
            assert np.allclose(d, 0.0)
    assert np.array_equal(kq[0], np.arange(nk))


def test_vhalf_hermitian_positive_and_spectrum():
    s = inputs.make_system("v", (2, 2, 1), 2, 3, 24, 4, 1)
    for iq in range(s.nq):
        vh = s.vhalf[iq]
        assert np.abs(vh - vh.conj().T).max() == 0.0
        lam = np.linalg.eigvalsh(vh @ vh)
        assert lam.min() > 0.0
        assert lam.min() >= 1e-2 * (1 - 1e-9)
    g = inputs.make_system("g", (1, 1, 1), 2, 3, 24, 4, 1, is_complex=False, periodic=False)
    lam = np.linalg.eigvalsh(g.vhalf[0] @ g.vhalf[0])
    assert lam.min() >= 1e-2 * (1 - 1e-9) and lam.max() <= 10.0 * (1 + 1e-9)


def test_band_gap_positive():
    s = inputs.make_system("b", (3, 3, 1), 16, 112, 8, 4, 2025)
    for q in range(s.nq):
        d = s.eps_virt[:, None, :] - s.eps_occ[s.kq[q]][:, :, None]
        assert d.min() >= 0.15 - 1e-12


def test_philox_words_deterministic_and_key_sensitive():
    a = inputs.philox_words(11, 9, 2, 3, 0, 1000)
    b = inputs.philox_words(11, 9, 2, 3, 0, 1000)
    c = inputs.philox_words(11, 9, 2, 4, 0, 1000)
    assert np.array_equal(a, b)
    assert np.mean(a == c) < 0.01
    # a shifted window returns the same words: the stream is counter-based
    d = inputs.philox_words(11, 9, 2, 3, 500, 500)
    assert np.array_equal(a[500:], d)
    # bits are balanced
    bits = np.unpackbits(a.view(np.uint8))
    assert abs(bits.mean() - 0.5) < 0.005


def test_philox_round_is_a_bijection_on_samples():
    # distinct counters under one key give distinct outputs (a random function would
    # collide with probability ~ n^2 / 2^129 here)
    w = inputs.philox_words(5, 1, 0, 0, 0, 200000)
    v = w.view(np.dtype((np.void, 16)))
    assert len(np.unique(v)) == len(v)


def test_B_moments_complex_and_real():
    sig = 0.03
    B = inputs.philox_B_rows(123, sig, 9, 1, 2, 112, 384, True, 0, 8)
    assert B.dtype == np.complex128
    x = B.reshape(-1)
    n = x.size
    assert abs(np.mean(x)) < 5 * sig / math.sqrt(n)
    assert abs(np.mean(np.abs(x) ** 2) / sig ** 2 - 1.0) < 5 * math.sqrt(1.0 / n) * 2
    assert abs(np.var(x.real) / (sig ** 2 / 2) - 1.0) < 0.02
    assert abs(np.var(x.imag) / (sig ** 2 / 2) - 1.0) < 0.02
    assert abs(np.mean(x.real * x.imag)) / (sig ** 2 / 2) < 0.02
    R = inputs.philox_B_rows(123, 0.05, 1, 0, 0, 56, 128, False, 0, 8)
    assert R.dtype == np.float64
    assert abs(np.var(R) / 0.05 ** 2 - 1.0) < 0.03
    # fourth moment of a Gaussian
    z = R.reshape(-1) / 0.05
    assert abs(np.mean(z ** 4) - 3.0) < 0.1


def test_B_rows_are_windows_of_the_block():
    blk = inputs.philox_B_block(9, 0.1, 4, 1, 3, 5, 6, 7, True)
    rows = inputs.philox_B_rows(9, 0.1, 4, 1, 3, 6, 7, True, 2, 4)
    assert np.array_equal(blk[2:4], rows)


def test_uniforms_strictly_inside_unit_interval():
    lo = inputs._uniform_pair(np.array([0], dtype=np.uint64), np.array([0], dtype=np.uint64))
    hi = inputs._uniform_pair(np.array([0xFFFFFFFF], dtype=np.uint64),
                              np.array([0xFFFFFFFF], dtype=np.uint64))
    assert 0.0 < lo[0] < 1e-15 and 1.0 - 1e-15 < hi[0] < 1.0


def test_serving_stream_shape():
    jobs = inputs.serving_jobs(256, 4.0, seed=77)
    assert len(jobs) == 256
    t = [j["arrival"] for j in jobs]
    assert all(b > a for a, b in zip(t, t[1:]))
    assert 40.0 < t[-1] < 100.0            # ~64 s at 4 jobs/s
    assert all(200 <= j["naux"] <= 1500 for j in jobs)
    assert all(8 <= j["nw"] <= 16 for j in jobs)
    assert {j["grid"] for j in jobs} == {(1, 1, 1), (2, 2, 1), (3, 3, 1)}
