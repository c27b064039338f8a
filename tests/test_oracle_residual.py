"""Pins of the oracle's residual-compressed document scoring.

A token is a centroid plus a per-dimension quantized residual (the compressed
form of the PLAID/WARP indexes the paper compares with and integrates into);
scoring applies Eq. (1) to the decoded vectors. The pins below fix the bit
layout by hand-computed cases, the arithmetic by an independent numpy brute
force, and the structure by special cases with closed forms.
"""
import json
import os

import numpy as np
import pytest

import oracle
import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _unpack_codes(residuals, dim, nbits):
    """Independent unpacking: little-endian bit stream, nbits-wide fields."""
    bits = np.unpackbits(np.asarray(residuals, np.uint8), axis=1, bitorder="little")
    bits = bits[:, :dim * nbits].reshape(len(residuals), dim, nbits).astype(np.int64)
    return (bits << np.arange(nbits)).sum(axis=2)


def _brute_scores(q, q_off, dec, d_off):
    out = []
    for a in range(len(q_off) - 1):
        qa = q[q_off[a]:q_off[a + 1]]
        for b in range(len(d_off) - 1):
            db = dec[d_off[b]:d_off[b + 1]]
            if len(qa) == 0:
                out.append(0.0)
            elif len(db) == 0:
                out.append(-np.inf)
            else:
                out.append(float((qa @ db.T).max(axis=1).sum()))
    return np.array(out)


@pytest.mark.parametrize("case", range(3))
def test_residual_golden_hand_computed(case):
    g = json.load(open(os.path.join(GOLDEN, "residual_small.json")))["cases"][case]
    args = (np.array(g["ids"], np.int32), np.array(g["residuals"], np.uint8),
            np.array(g["centroids"], np.float64), np.array(g["weights"], np.float64), g["nbits"])
    dec = oracle.residual_decode(*args)
    assert np.array_equal(dec, np.array(g["decoded"], np.float64))
    q = np.array(g["q"], np.float64)
    s = oracle.residual_decode_score(q, [0, len(q)], *args, np.array(g["doc_offsets"]))
    assert np.array_equal(s, np.array(g["scores"]))


@pytest.mark.parametrize("nbits", [1, 2, 4])
def test_residual_matches_numpy_brute_force(nbits):
    g = W.rng(40 + nbits)
    dim, n_c = 32, 11
    lens = g.integers(0, 6, size=9)
    lens[3] = 0  # an empty document
    d_off = W.offsets_from_lengths(lens)
    T = int(d_off[-1])
    cen = g.standard_normal((n_c, dim))
    w = g.standard_normal(1 << nbits)
    ids = g.integers(0, n_c, size=T).astype(np.int32)
    res = g.integers(0, 256, size=(T, dim * nbits // 8), dtype=np.uint8)
    q_off = np.array([0, 3, 3, 7])  # second query empty
    q = g.standard_normal((7, dim))
    codes = _unpack_codes(res, dim, nbits)
    dec_np = cen[ids] + w[codes]
    dec = oracle.residual_decode(ids, res, cen, w, nbits)
    np.testing.assert_allclose(dec, dec_np, rtol=0, atol=0)
    got = oracle.residual_decode_score(q, q_off, ids, res, cen, w, nbits, d_off)
    want = _brute_scores(q, q_off, dec_np, d_off)
    np.testing.assert_allclose(got, want, rtol=1e-12, atol=1e-12)
    # candidate lists select documents by id
    cand_off = np.array([0, 4, 4, 6])
    cand_ids = np.array([8, 3, 0, 8, 1, 2], np.int32)
    got_c = oracle.residual_decode_score(q, q_off, ids, res, cen, w, nbits, d_off, cand_off,
                                         cand_ids)
    dense = want.reshape(3, 9)
    want_c = [dense[a, b] for a in range(3) for b in cand_ids[cand_off[a]:cand_off[a + 1]]]
    np.testing.assert_allclose(got_c, want_c, rtol=1e-12, atol=1e-12)


def test_zero_residual_reduces_to_plain_maxsim_on_centroids():
    g = W.rng(7)
    dim, n_c = 64, 5
    cen = g.standard_normal((n_c, dim))
    d_off = W.offsets_from_lengths([3, 1, 4])
    ids = g.integers(0, n_c, size=8).astype(np.int32)
    res = g.integers(0, 256, size=(8, dim * 2 // 8), dtype=np.uint8)
    q = g.standard_normal((4, dim))
    got = oracle.residual_decode_score(q, [0, 4], ids, res, cen, np.zeros(4), 2, d_off)
    want = oracle.maxsim(q, [0, 4], cen[ids], d_off)
    assert np.array_equal(got, want)


def test_zero_centroids_one_token_closed_form():
    # Nd = 1 and centroid 0: score = (sum_i q_i) . r with r_k = w[code_k].
    g = W.rng(8)
    dim, nbits = 32, 2
    w = np.array([-3.0, -1.0, 0.5, 2.0])
    res = g.integers(0, 256, size=(1, dim * nbits // 8), dtype=np.uint8)
    r = w[_unpack_codes(res, dim, nbits)[0]]
    q = g.standard_normal((5, dim))
    got = oracle.residual_decode_score(q, [0, 5], np.zeros(1, np.int32), res,
                                       np.zeros((1, dim)), w, nbits, [0, 1])
    np.testing.assert_allclose(got, [q.sum(axis=0) @ r], rtol=1e-13)


def test_token_permutation_is_bit_identical():
    g = W.rng(9)
    dim, nbits, n_c = 32, 2, 6
    T = 7
    cen = g.standard_normal((n_c, dim))
    w = g.standard_normal(4)
    ids = g.integers(0, n_c, size=T).astype(np.int32)
    res = g.integers(0, 256, size=(T, 8), dtype=np.uint8)
    q = g.standard_normal((3, dim))
    perm = g.permutation(T)
    a = oracle.residual_decode_score(q, [0, 3], ids, res, cen, w, nbits, [0, T])
    b = oracle.residual_decode_score(q, [0, 3], ids[perm], res[perm], cen, w, nbits, [0, T])
    assert np.array_equal(a, b)


def test_centroid_id_out_of_range_is_rejected():
    with pytest.raises(ValueError):
        oracle.residual_decode(np.array([2], np.int32), np.zeros((1, 8), np.uint8),
                               np.zeros((2, 32)), np.zeros(4), 2)
    with pytest.raises(ValueError):
        oracle.residual_decode(np.array([-1], np.int32), np.zeros((1, 8), np.uint8),
                               np.zeros((2, 32)), np.zeros(4), 2)
