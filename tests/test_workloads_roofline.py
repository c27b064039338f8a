"""Input-generator determinism/recipe and the paper's byte-model integers."""
import math

import numpy as np

import workloads as W
from paper_2606_26439_amd import roofline as R


def test_generators_are_deterministic():
    a = W.ragged_case(50, dim=64, nq=8)
    b = W.ragged_case(50, dim=64, nq=8)
    for k in a:
        assert np.array_equal(a[k], b[k])
    assert np.array_equal(W.pq_codes(100, seed=2), W.pq_codes(100, seed=2))
    assert np.array_equal(W.candidates(3, 1000, 4, (10, 50))[1], W.candidates(3, 1000, 4, (10, 50))[1])


def test_lognormal_lengths_recipe():
    n = W.doc_lengths(400000, seed=0)
    assert n.min() >= 8 and n.max() <= 180
    # arithmetic-mean-70 reading, clipped: E[Nd] ~= 69.4
    assert abs(n.mean() - 69.4) < 0.2
    assert 0.01 < (n == 180).mean() < 0.025


def test_unit_tokens_are_unit():
    x = W.unit_tokens(100, 128, W.rng(0)).astype(np.float64)
    np.testing.assert_allclose((x * x).sum(1), 1.0, rtol=1e-6)


def test_plain_case_shapes():
    c = W.plain_fp32_case()
    assert c["q"].shape == (32, 128) and c["d"].shape == (4096 * 32, 128)
    assert c["d_off"][-1] == 4096 * 32


def test_candidates_unique_and_in_range():
    off, ids = W.candidates(4, 5000, seed=4, size_range=(1000, 3000))
    for a in range(4):
        seg = ids[off[a]:off[a + 1]]
        assert len(np.unique(seg)) == len(seg)
        assert seg.min() >= 0 and seg.max() < 5000
        assert 1000 <= len(seg) <= 3000


def test_paper_io_table_integers():
    # Sec. 2.3 worked table: Nq=32, Nd=128, d=128, B=10^4, FP16.
    assert R.io_naive(10000, 32, 128, 128) == 655_368_192
    assert R.io_fused(10000, 32, 128, 128) == 328_968_192
    f = R.flops(10000, 32, 128, 128)
    assert round(R.arithmetic_intensity(f, R.io_naive(10000, 32, 128, 128)), 1) == 16.1
    assert round(R.arithmetic_intensity(f, R.io_fused(10000, 32, 128, 128)), 1) == 32.0
    # "2.0x" at Nq = 32 and "3.0x" at Nq = 64
    assert round(R.io_naive(10000, 32, 128, 128) / R.io_fused(10000, 32, 128, 128), 1) == 2.0
    assert round(R.io_naive(10000, 64, 128, 128) / R.io_fused(10000, 64, 128, 128), 1) == 3.0


def test_paper_pq_io_integers():
    # Sec. 4.4 table: B=100K, Nq=32, Nd=128, M=16, K=256.
    dec = R.pq_io_decompress(100000, 32, 128, 128, 16)
    fus = R.pq_io_fused(100000, 32, 128, 16, 256)
    assert dec == 6_758_400_000
    assert fus == 218_124_288
    assert round(dec / fus, 1) == 31.0
    # Sec. 4.3: the table for Nq=32, M=16, K=256 in FP32 is 512 KB.
    assert 32 * 16 * 256 * 4 == 512 * 1024


def test_theorem_one_optimum():
    base = R.io_theorem(1000, 32, 128, 128, BQ=32)
    assert base == (32 * 128 + 1000 * 128 * 128) * 2 + 1000 * 4
    assert R.io_theorem(1000, 32, 128, 128, BQ=16) > base
    assert R.io_theorem(1000, 32, 128, 128, BQ=64) == base
