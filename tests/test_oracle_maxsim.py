"""Pins of the FP64 MaxSim oracle against facts that do not come from it.

Eq. (1) of the paper (Background): MaxSim(Q, D) = sum_i max_j q_i . d_j.
"""
import json
import math
import os

import numpy as np
import pytest

import oracle
import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _pack(sets, dim):
    lens = [len(s) for s in sets]
    off = W.offsets_from_lengths(lens)
    rows = [np.asarray(s, np.float64).reshape(-1, dim) for s in sets if len(s)]
    tok = np.concatenate(rows) if rows else np.zeros((0, dim))
    return tok, off


def _numpy_reference(q, q_off, d, d_off):
    """Independent route: one matmul for all similarities, then segment reductions."""
    S = d @ q.T  # [T, total query tokens]
    out = []
    for a in range(len(q_off) - 1):
        for b in range(len(d_off) - 1):
            qs = slice(q_off[a], q_off[a + 1])
            ds = slice(d_off[b], d_off[b + 1])
            blk = S[ds, qs]
            if blk.shape[1] == 0:
                out.append(0.0)
            elif blk.shape[0] == 0:
                out.append(-math.inf)
            else:
                out.append(blk.max(axis=0).sum())
    return np.array(out)


def test_golden_hand_computed():
    g = json.load(open(os.path.join(GOLDEN, "maxsim_small.json")))
    q = np.array(g["q"], np.float64)
    d, d_off = _pack(g["docs"], 2)
    got = oracle.maxsim(q, [0, len(q)], d, d_off)
    want = np.array([float(s) for s in g["scores"]])
    assert np.array_equal(got, want)


@pytest.mark.parametrize("seed", range(6))
def test_brute_force_vs_numpy(seed):
    g = W.rng(100 + seed)
    dim = int(g.integers(1, 9))
    nq_l = g.integers(0, 5, size=3)
    nd_l = g.integers(0, 6, size=int(g.integers(1, 11)))
    q_off = W.offsets_from_lengths(nq_l)
    d_off = W.offsets_from_lengths(nd_l)
    q = g.standard_normal((q_off[-1], dim))
    d = g.standard_normal((d_off[-1], dim))
    got = oracle.maxsim(q, q_off, d, d_off)
    want = _numpy_reference(q, q_off, d, d_off)
    fin = np.isfinite(want)
    assert np.array_equal(np.isfinite(got), fin)
    assert np.array_equal(got[~fin], want[~fin])
    np.testing.assert_allclose(got[fin], want[fin], rtol=1e-12, atol=1e-12)


def test_single_doc_token_closed_form():
    # Nd = 1: every max is the only term, so the score is (sum_i q_i) . d_1.
    g = W.rng(7)
    q = g.standard_normal((5, 16))
    d = g.standard_normal((1, 16))
    got = oracle.maxsim(q, [0, 5], d, [0, 1])[0]
    assert got == pytest.approx(float(q.sum(axis=0) @ d[0]), rel=1e-13)


def test_single_query_token_closed_form():
    # Nq = 1: the score is the largest single dot product.
    g = W.rng(8)
    q = g.standard_normal((1, 12))
    d = g.standard_normal((9, 12))
    got = oracle.maxsim(q, [0, 1], d, [0, 9])[0]
    assert got == max(float(np.dot(q[0], r)) for r in d)


def test_all_dots_negative_pins_minus_inf_init():
    # D = -Q (one doc of Nq tokens) with orthonormal-ish Q: every dot with a
    # non-matching token is ~0 and with the matching one is -1; a doc made of
    # -q_0 only gives -sum_i q_i.q_0 < 0, which an init at 0 would hide.
    q = np.eye(4)[:3]
    d = -q[:1]
    got = oracle.maxsim(q, [0, 3], d, [0, 1])[0]
    assert got == -1.0


def test_query_contained_in_doc_gives_exactly_nq():
    # Dyadic unit vectors: q_i . q_i = 1 exactly and |q_i . x| <= 1 for unit x.
    for seed in range(3):
        q = W.dyadic_unit_vectors(8, 128, seed)
        extra = W.dyadic_unit_vectors(20, 128, seed + 50)
        d = np.concatenate([extra[:10], q, extra[10:]])
        got = oracle.maxsim(q, [0, 8], d, [0, len(d)])[0]
        assert got == 8.0


def test_empty_doc_and_empty_query():
    q = np.ones((2, 4))
    d = np.ones((3, 4))
    assert oracle.maxsim(q, [0, 2], d, [0, 0, 3])[0] == -math.inf
    assert oracle.maxsim(q, [0, 0], d, [0, 3])[0] == 0.0


def test_invariants():
    g = W.rng(11)
    q = W.unit_tokens(6, 32, g)
    d = W.unit_tokens(15, 32, g)
    base = oracle.maxsim(q, [0, 6], d, [0, 15])[0]
    # doc-token permutation: each dot is computed identically -> bit-identical
    perm = g.permutation(15)
    assert oracle.maxsim(q, [0, 6], d[perm], [0, 15])[0] == base
    # duplicating a doc token changes nothing
    dd = np.concatenate([d, d[3:4]])
    assert oracle.maxsim(q, [0, 6], dd, [0, 16])[0] == base
    # appending a token never decreases the score
    de = np.concatenate([d, W.unit_tokens(1, 32, g)])
    assert oracle.maxsim(q, [0, 6], de, [0, 16])[0] >= base
    # scaling Q by a power of two scales every dot exactly
    assert oracle.maxsim(q * 4.0, [0, 6], d, [0, 15])[0] == 4.0 * base
    # unit-norm tokens: every dot <= 1, so score <= Nq
    assert base <= 6.0 + 1e-12
    # query-token permutation only reorders the outer sum
    qp = q[g.permutation(6)]
    assert oracle.maxsim(qp, [0, 6], d, [0, 15])[0] == pytest.approx(base, rel=1e-14)


def test_zero_extension_is_exact():
    # Dimension tiling splits the dot product; zero-extending d adds +0 terms.
    g = W.rng(12)
    q = W.unit_tokens(4, 128, g)
    d = W.unit_tokens(10, 128, g)
    base = oracle.maxsim(q, [0, 4], d, [0, 4, 10])
    for ext in (128, 384, 640):
        qz = np.concatenate([q, np.zeros((4, ext), np.float32)], axis=1)
        dz = np.concatenate([d, np.zeros((10, ext), np.float32)], axis=1)
        assert np.array_equal(oracle.maxsim(qz, [0, 4], dz, [0, 4, 10]), base)


def test_split_dimension_identity():
    # q.d = q[:128].d[:128] + q[128:].d[128:]: with one token per side the
    # score is a single dot, so the split sum must match it.
    g = W.rng(13)
    q = W.unit_tokens(1, 256, g)
    d = W.unit_tokens(1, 256, g)
    full = oracle.maxsim(q, [0, 1], d, [0, 1])[0]
    lo = oracle.maxsim(q[:, :128], [0, 1], d[:, :128], [0, 1])[0]
    hi = oracle.maxsim(q[:, 128:], [0, 1], d[:, 128:], [0, 1])[0]
    assert full == pytest.approx(lo + hi, rel=1e-14, abs=1e-15)


def test_candidates_select_from_dense():
    c = W.ragged_case(40, dim=16, nq=5, n_queries=3, nq_range=(1, 6))
    dense = oracle.maxsim(c["q"], c["q_off"], c["d"], c["d_off"]).reshape(3, 40)
    cand_off, cand_ids = W.candidates(3, 40, seed=4, size_range=(5, 20))
    sc = oracle.maxsim(c["q"], c["q_off"], c["d"], c["d_off"], cand_off, cand_ids)
    for a in range(3):
        ids = cand_ids[cand_off[a]:cand_off[a + 1]]
        assert np.array_equal(sc[cand_off[a]:cand_off[a + 1]], dense[a, ids])


def test_candidate_out_of_range_is_rejected():
    with pytest.raises(ValueError):
        oracle.maxsim(np.ones((1, 4)), [0, 1], np.ones((2, 4)), [0, 2], [0, 1], [5])
