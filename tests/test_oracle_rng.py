"""Pins for the oracle's random draws: Philox4x32-10 and the pair law.

The oracle's generator is pinned to published known-answer vectors; the pair
law (uniform ordered pairs s != t, Section 2.3) is pinned by its closed form
(each vertex has floor or ceil of 2^64/n preimages) and by a chi-square test.
"""
import os

import numpy as np
import pytest
from scipy import stats

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _kat_rows():
    rows = []
    with open(os.path.join(GOLDEN, "philox4x32_10_kat.txt")) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            w = [int(x, 16) for x in line.split()]
            rows.append((w[0:4], w[4:6], tuple(w[6:10])))
    return rows


def test_philox_known_answers(oracle_mod):
    rows = _kat_rows()
    assert len(rows) == 3
    for ctr, key, want in rows:
        assert oracle_mod.philox4x32_10(ctr, key) == want


def test_uniform64_layout(oracle_mod):
    # draw j of sample i is the Philox block at counter (lo i, hi i, j, 0), key = seed
    seed, i, j = 0x0123456789ABCDEF, 0x1122334455667788, 7
    x = oracle_mod.philox4x32_10([i & 0xFFFFFFFF, i >> 32, j, 0], [seed & 0xFFFFFFFF, seed >> 32])
    assert oracle_mod.uniform64(seed, i, j) == x[0] | (x[1] << 32)


def test_uniform64_bits_balanced(oracle_mod):
    # every bit of the 64-bit word is a fair coin over many draws
    words = np.array([oracle_mod.uniform64(5, i, 1) for i in range(20000)], dtype=np.uint64)
    bits = ((words[:, None] >> np.arange(64, dtype=np.uint64)) & np.uint64(1)).astype(np.float64)
    freq = bits.mean(axis=0)
    # 5 sigma of a binomial(20000, 1/2) proportion
    assert np.all(np.abs(freq - 0.5) < 5 * 0.5 / np.sqrt(20000))


def test_pair_distinct_and_in_range(oracle_mod):
    for n in (2, 3, 17, 1000, 2**23 - 1):
        s, t = oracle_mod.pairs(3, 0, 5000, n)
        assert np.all(s != t)
        assert s.min() >= 0 and t.min() >= 0 and s.max() < n and t.max() < n


def test_pair_n2_is_both_orders(oracle_mod):
    s, t = oracle_mod.pairs(1, 0, 4000, 2)
    assert set(zip(s.tolist(), t.tolist())) == {(0, 1), (1, 0)}
    frac = float(np.mean(s == 0))
    assert abs(frac - 0.5) < 5 * 0.5 / np.sqrt(4000)


def test_pair_preimage_closed_form(oracle_mod):
    # s = floor(U * n / 2^64): the preimage of s is [ceil(s 2^64 / n), ceil((s+1) 2^64 / n)),
    # so every vertex gets floor(2^64/n) or ceil(2^64/n) of the 2^64 words.
    for n in (3, 7, 1000, 174015):
        sizes = {((s + 1) * 2**64 + n - 1) // n - (s * 2**64 + n - 1) // n for s in range(min(n, 500))}
        assert sizes <= {2**64 // n, -(-(2**64) // n)}
    # and the oracle's s agrees with that mapping for the first word of draw 0
    n = 12345
    for i in range(200):
        x = oracle_mod.philox4x32_10([i, 0, 0, 0], [9, 0])
        u = x[0] | (x[1] << 32)
        s, _ = oracle_mod.pair(9, i, n)
        assert s * 2**64 <= u * n < (s + 1) * 2**64


def test_pair_chi_square(oracle_mod):
    n = 10
    m = 400_000
    s, t = oracle_mod.pairs(11, 0, m, n)
    cells = np.bincount(s.astype(np.int64) * n + t, minlength=n * n).reshape(n, n)
    assert np.all(np.diag(cells) == 0)
    obs = cells[~np.eye(n, dtype=bool)]
    exp = np.full(obs.size, m / (n * (n - 1)))
    chi2 = float(((obs - exp) ** 2 / exp).sum())
    p = stats.chi2.sf(chi2, obs.size - 1)
    assert p > 1e-4, (chi2, p)


def test_pairs_depend_only_on_index(oracle_mod):
    s1, t1 = oracle_mod.pairs(42, 1000, 100, 999)
    s2, t2 = oracle_mod.pairs(42, 0, 1100, 999)
    assert np.array_equal(s1, s2[1000:]) and np.array_equal(t1, t2[1000:])
    s3, _ = oracle_mod.pairs(43, 1000, 100, 999)
    assert not np.array_equal(s1, s3)


@pytest.mark.parametrize("i", [0, 1, 2**32 - 1, 2**32, 2**40 + 5])
def test_pair_high_sample_indices(oracle_mod, i):
    # the high word of the sample index reaches the counter
    s, t = oracle_mod.pair(1, i, 2**22)
    x = oracle_mod.philox4x32_10([i & 0xFFFFFFFF, i >> 32, 0, 0], [1, 0])
    assert s == ((x[0] | (x[1] << 32)) * 2**22) >> 64
    tt = ((x[2] | (x[3] << 32)) * (2**22 - 1)) >> 64
    assert t == tt + (tt >= s)


def test_philox_against_rocrand_engine(tmp_path, oracle_mod):
    """rocRAND's Philox4x32-10 engine (its open-source header, compiled here
    into tests/rocrand_philox_ref.cpp) emits, for key = seed and the block
    counter in word 0, exactly the oracle's blocks."""
    import shutil
    import subprocess

    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    exe = tmp_path / "philox_ref"
    src = os.path.join(os.path.dirname(__file__), "rocrand_philox_ref.cpp")
    subprocess.check_call([hipcc, "-O1", "-I/opt/rocm/include", src, "-o", str(exe)],
                          stdout=subprocess.DEVNULL, stderr=subprocess.DEVNULL)
    for seed in (0, 1, 0x0123456789ABCDEF, 2**64 - 1):
        out = subprocess.check_output([str(exe), str(seed), "64"], text=True).split()
        words = [int(x) for x in out]
        key = [seed & 0xFFFFFFFF, seed >> 32]
        for k in range(64):
            assert tuple(words[4 * k: 4 * k + 4]) == oracle_mod.philox4x32_10([k, 0, 0, 0], key)
