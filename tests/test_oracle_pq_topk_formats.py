"""Pins of the oracle's PQ, top-k and number-format routines."""
import json
import math
import os

import numpy as np
import pytest
import torch

import oracle
import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------- PQ (Sec. 4)

def test_pq_golden_hand_computed():
    g = json.load(open(os.path.join(GOLDEN, "pq_small.json")))
    cb = np.array(g["codebooks"], np.float64)
    q = np.array(g["q"], np.float64)
    codes = np.array(g["codes"], np.uint8)
    off = np.array(g["doc_offsets"], np.int64)
    assert np.array_equal(oracle.pq_lut_build(q, cb), np.array(g["table"], np.float64))
    assert np.array_equal(oracle.pq_decode(codes, cb), np.array(g["decoded"], np.float64))
    table = oracle.pq_lut_build(q, cb)
    assert np.array_equal(oracle.pq_lut_score(table, codes, off), np.array(g["scores"]))
    assert np.array_equal(oracle.pq_decode_score(q, [0, 1], codes, cb, off), np.array(g["scores"]))


def test_pq_decode_indexing():
    # Centroid values encode (m, k, u) so a wrong index shows up by value.
    M, K, dsub = 4, 16, 3
    cb = np.zeros((M, K, dsub))
    for m in range(M):
        for k in range(K):
            for u in range(dsub):
                cb[m, k, u] = m * 10000 + k * 10 + u
    codes = W.rng(1).integers(0, K, size=(7, M), dtype=np.uint8)
    dec = oracle.pq_decode(codes, cb)
    for t in range(7):
        for m in range(M):
            for u in range(dsub):
                assert dec[t, m * dsub + u] == m * 10000 + int(codes[t, m]) * 10 + u


def test_pq_table_vs_numpy():
    g = W.rng(2)
    M, K, dsub = 4, 8, 4
    cb = g.standard_normal((M, K, dsub))
    q = g.standard_normal((3, M * dsub))
    T = oracle.pq_lut_build(q, cb)
    want = np.einsum("imu,mku->imk", q.reshape(3, M, dsub), cb)
    np.testing.assert_allclose(T, want, rtol=1e-13, atol=1e-14)


def test_pq_integer_lut_is_exact():
    # Small integers: every table entry and every sum is an exact integer, so
    # the LUT route and a pure-integer brute force must agree exactly.
    g = W.rng(3)
    M, K, dsub = 4, 8, 2
    cb = g.integers(-3, 4, size=(M, K, dsub))
    q = g.integers(-3, 4, size=(5, M * dsub))
    lens = [3, 1, 4, 2]
    off = W.offsets_from_lengths(lens)
    codes = g.integers(0, K, size=(off[-1], M), dtype=np.uint8)
    T = oracle.pq_lut_build(q.astype(np.float64), cb.astype(np.float64))
    got = oracle.pq_lut_score(T, codes, off)
    for b in range(len(lens)):
        tot = 0
        for i in range(5):
            best = None
            for j in range(off[b], off[b + 1]):
                v = 0
                for m in range(M):
                    c = int(codes[j, m])
                    v += sum(int(q[i, m * dsub + u]) * int(cb[m, c, u]) for u in range(dsub))
                best = v if best is None else max(best, v)
            tot += best
        assert got[b] == float(tot)


def test_pq_lut_equals_decode_then_score():
    # The ADC identity: sum_m T[i,m,c_m] = q_i . concat_m C[m, c_m] (real arithmetic).
    cb = W.pq_codebooks(M=8, K=256, dsub=16, seed=2).astype(np.float64)
    lens = W.doc_lengths(30, seed=5)
    off = W.offsets_from_lengths(lens)
    codes = W.pq_codes(int(off[-1]), seed=5)
    q = W.unit_tokens(32, 128, W.rng(6))
    T = oracle.pq_lut_build(q, cb)
    lut = oracle.pq_lut_score(T, codes, off)
    dec = oracle.pq_decode_score(q, [0, 32], codes, cb, off)
    np.testing.assert_allclose(lut, dec, rtol=1e-12, atol=1e-12)
    sel = np.array([4, 0, 29, 4], np.int32)
    np.testing.assert_array_equal(oracle.pq_lut_score(T, codes, off, sel), lut[sel])


# ---------------------------------------------------------------- top-k

@pytest.mark.parametrize("n,k,distinct", [(50, 10, None), (200, 100, 7), (5, 8, None),
                                          (0, 3, None), (300, 1, 2)])
def test_topk_vs_python_sort(n, k, distinct):
    s = W.random_scores(n, seed=n + k, n_distinct=distinct).astype(np.float64)
    ids = W.rng(9).permutation(10 * n + 1)[:n].astype(np.int64)
    got_ids, got_s = oracle.topk(s, k, ids)
    order = sorted(range(n), key=lambda i: (-s[i], ids[i]))[:k]
    want_ids = [int(ids[i]) for i in order] + [-1] * (k - min(k, n))
    want_s = [float(s[i]) for i in order] + [-math.inf] * (k - min(k, n))
    assert got_ids.tolist() == want_ids
    assert got_s.tolist() == want_s


def test_topk_default_ids_are_positions():
    s = np.array([1.0, 3.0, 3.0, -math.inf, 2.0])
    ids, vals = oracle.topk(s, 4)
    assert ids.tolist() == [1, 2, 4, 0]
    assert vals.tolist() == [3.0, 3.0, 2.0, 1.0]


# ---------------------------------------------------------------- formats

def _probe_values():
    g = W.rng(21)
    parts = [
        g.standard_normal(20000).astype(np.float32),
        (g.standard_normal(5000) * 1e-5).astype(np.float32),   # f16 subnormal range
        (g.standard_normal(5000) * 3e4).astype(np.float32),    # near f16 max
        np.array([0.0, -0.0, 1.0, -1.0, 65504.0, 65519.0, 2 ** -24, 2 ** -25,
                  3 * 2 ** -25, 1 + 2 ** -11, 1 + 3 * 2 ** -11, 1 + 2 ** -8,
                  1 + 3 * 2 ** -8, 2 ** -126, 2 ** -130], np.float32),
    ]
    return np.concatenate(parts)


def test_f16_rounding_matches_numpy():
    x = _probe_values()
    x = x[np.abs(x) < 65520]
    want = x.astype(np.float16).view(np.uint16)
    assert np.array_equal(oracle.round_f16(x), want)
    np.testing.assert_array_equal(oracle.decode_f16(want), want.view(np.float16).astype(np.float64))


def test_bf16_rounding_matches_torch():
    x = _probe_values()
    want = torch.from_numpy(x).to(torch.bfloat16).view(torch.int16).numpy().view(np.uint16)
    assert np.array_equal(oracle.round_bf16(x), want)
    dec = torch.from_numpy(want.view(np.int16)).view(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(oracle.decode_bf16(want), dec)


def test_e4m3_rounding_matches_torch():
    g = W.rng(22)
    x = np.concatenate([g.standard_normal(20000) * 50, g.standard_normal(5000) * 0.01,
                        [0.0, 448.0, -448.0, 2 ** -9, 2 ** -10, 3 * 2 ** -10, 1.0625,
                         1.1875, 240.0, 232.0]]).astype(np.float32)
    x = x[np.abs(x) <= 448]
    want = torch.from_numpy(x).to(torch.float8_e4m3fn).view(torch.uint8).numpy()
    assert np.array_equal(oracle.round_e4m3(x), want)
    dec = torch.from_numpy(want).view(torch.float8_e4m3fn).to(torch.float64).numpy()
    np.testing.assert_array_equal(oracle.decode_e4m3(want), dec)


def test_e4m3_known_codes_and_saturation():
    x = np.array([1.0, 448.0, 2 ** -9, -2.0, 0.0, 500.0, -1e6], np.float32)
    assert oracle.round_e4m3(x).tolist() == [0x38, 0x7E, 0x01, 0xC0, 0x00, 0x7E, 0xFE]


def test_quant_e4m3_scale_is_minimal_power_of_two():
    g = W.rng(23)
    x = np.concatenate([W.unit_tokens(200, 128, g), np.zeros((1, 128), np.float32),
                        np.full((1, 128), 448.0, np.float32),
                        np.full((1, 128), 448.0 * 2 ** -20 * 1.0000001, np.float32)])
    codes, s = oracle.quant_e4m3(x)
    amax = np.abs(x).max(axis=1).astype(np.float64)
    for t in range(len(x)):
        st = float(s[t])
        m, e = math.frexp(st)
        assert m == 0.5  # power of two
        if amax[t] == 0:
            assert st == 1.0
        else:
            assert amax[t] <= 448.0 * st
            assert amax[t] > 448.0 * st / 2
    assert s[-2] == 1.0 and s[-1] == 2.0 ** -19
    dec = oracle.decode_e4m3(codes) * s[:, None]
    # E4M3 keeps 3 mantissa bits: relative error of a normal value <= 2^-4
    big = np.abs(x) > 2 ** -6 * s[:, None]
    assert np.all(np.abs(dec - x)[big] <= np.abs(x)[big] * 2 ** -4 + 1e-30)


def test_exact_values_dyadic_are_exact():
    v = W.dyadic_unit_vectors(4, 128, 0)
    for dt in ("f32", "bf16", "f16", "fp8"):
        vals, _ = oracle.exact_values(v, dt)
        assert np.array_equal(vals, v.astype(np.float64))
