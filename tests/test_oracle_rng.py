"""Pins for the oracle's Philox4x64-10 generator and vacancy sampler.

The paper (Section 3.2) only asks for iid vacancies with probability p; the
generator is this project's choice.  Pins: numpy's independent Philox4x64-10
implementation, exact threshold semantics, statistics, and stream splitting.
"""

import numpy as np
import pytest

import oracle


def numpy_block(counter, key):
    """Philox4x64-10 block for `counter` from numpy (which pre-increments)."""
    c = sum(int(w) << (64 * i) for i, w in enumerate(counter))
    c = (c - 1) % (1 << 256)
    words = np.array([(c >> (64 * i)) & ((1 << 64) - 1) for i in range(4)], dtype=np.uint64)
    bg = np.random.Philox(counter=words, key=np.array(key, dtype=np.uint64))
    return bg.random_raw(4)


@pytest.mark.parametrize("counter,key", [
    ((0, 0, 0, 0), (0, 0)),
    ((1, 0, 0, 0), (12345, 678)),
    ((0, 7, 0, 0), (2**64 - 1, 3)),
    ((2**64 - 1, 2**63, 5, 9), (0xDEADBEEF, 0xC0FFEE)),
    ((123456789, 42, 0, 0), (202, (1 << 32) | 16)),
])
def test_philox_matches_numpy(counter, key):
    ours = oracle.philox4x64_10(counter, key)
    ref = numpy_block(counter, key)
    assert list(ours) == list(ref)


def test_vacancy_rule_against_numpy_words(glat):
    N, p, seed, first, ns = 3, 0.37, 99, 5, 4
    tag = oracle.stream_tag(glat, N)
    mask = oracle.sample_vacancies(glat, N, p, seed, tag, first, ns)
    G = glat.n_groups
    thr = int(np.floor(p * 2.0 ** 53))
    for s in range(ns):
        for g in range(N * N * G):
            word = int(numpy_block((first + s, g // 4, 0, 0), (seed, tag))[g % 4])
            want = (word >> 11) < thr
            assert bool(mask[s].reshape(-1)[g]) == want


def test_vacancy_extremes(glat, mlat):
    N = 4
    m0 = oracle.sample_vacancies(glat, N, 0.0, 1, oracle.stream_tag(glat, N), 0, 3)
    assert m0.sum() == 0
    m1 = oracle.sample_vacancies(glat, N, 1.0, 1, oracle.stream_tag(glat, N), 0, 3)
    assert m1.all()
    mm = oracle.sample_vacancies(mlat, N, 1.0, 1, oracle.stream_tag(mlat, N), 0, 3)
    assert (mm[..., 0] == 0).all(), "Mo (group 0) is never removed"
    assert (mm[..., 1:] == 1).all()


def test_vacancy_statistics(glat):
    N, p, M = 16, 0.05, 400
    mask = oracle.sample_vacancies(glat, N, p, 202, oracle.stream_tag(glat, N), 0, M)
    n = mask.size
    frac = mask.mean()
    sd = np.sqrt(p * (1 - p) / n)
    assert abs(frac - p) < 5 * sd
    # neighbouring groups are uncorrelated
    flat = mask.reshape(M, -1).astype(np.float64)
    c = np.corrcoef(flat[:, :-1].ravel(), flat[:, 1:].ravel())[0, 1]
    assert abs(c) < 5 / np.sqrt(flat[:, :-1].size)


def test_stream_split_and_tags(glat):
    N = 4
    tag = oracle.stream_tag(glat, N)
    a = oracle.sample_vacancies(glat, N, 0.3, 7, tag, 0, 10)
    b = np.concatenate([oracle.sample_vacancies(glat, N, 0.3, 7, tag, 0, 4),
                        oracle.sample_vacancies(glat, N, 0.3, 7, tag, 4, 6)])
    assert (a == b).all()
    c = oracle.sample_vacancies(glat, N, 0.3, 7, oracle.stream_tag(glat, 8), 0, 10)
    assert (a != c).any(), "different supercell sizes use independent streams"


def test_invalid_probability(glat):
    with pytest.raises(oracle.OracleError):
        oracle.sample_vacancies(glat, 2, 1.5, 0, 0, 0, 1)
