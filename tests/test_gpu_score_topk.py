"""GPU parity of the fused score + top-k call (top-k in the scorer's epilogue,
no score array) through the C ABI.

Its contract is bit-identity with maxsim_score followed by maxsim_topk over
per-query segments, which the other GPU tests pin against the oracle; here
both sides run on the same inputs and every (score, id) of every row must
match bit for bit, across element types, query groupings, candidate lists
(empty, repeated ids), short segments padded with (-inf, -1), empty
documents, ties, and ranges that overflow the workgroups' LDS key slots.
The smaller cases are also checked against the oracle's own top-k.
"""
import numpy as np
import pytest
import torch

import oracle
import paper_2606_26439_amd as M
import workloads as W
from tests._gpu import REL_TOL_DT, dev, device_tokens, o1_scores

pytestmark = pytest.mark.gpu

DTYPES = ["f32", "bf16", "f16", "fp8"]


def _reference(Q, D, k, cand=None):
    """maxsim_score + maxsim_topk over per-query segments."""
    s = M.score(Q, D, cand)
    if cand is not None:
        seg, ids = cand.offsets, cand.doc_ids
    else:
        seg = torch.arange(Q.n_sets + 1, dtype=torch.int64, device="cuda") * D.n_sets
        ids = None
    return M.topk(s, seg, k, ids=ids, n_total=s.numel()), s


def _assert_identical(got, want, what):
    gs, gi = (t.cpu().numpy() for t in got)
    ws, wi = (t.cpu().numpy() for t in want)
    assert gi.shape == wi.shape, what
    for a in range(gi.shape[0]):
        assert gi[a].tolist() == wi[a].tolist(), f"{what}: ids of row {a}"
        assert np.array_equal(gs[a].view(np.uint32), ws[a].view(np.uint32)), \
            f"{what}: scores of row {a}"


def _ragged(n_docs, dim, seed, nq_lens, empty_every=0):
    lens = W.doc_lengths(n_docs, seed)
    if empty_every:
        lens[::empty_every] = 0
    d_off = W.offsets_from_lengths(lens)
    g = W.rng(seed + 1)
    d = W.unit_tokens(int(d_off[-1]), dim, g)
    q_off = W.offsets_from_lengths(nq_lens)
    q = W.unit_tokens(int(q_off[-1]), dim, g)
    return q, q_off, d, d_off


def _check_vs_oracle(got, q, q_off, d, d_off, dtype, k, cand_off=None, cand_ids=None):
    """Each row's ids equal the oracle's top-k of the exact (O1) scores up to
    swaps between near-ties, and each returned score is within the gate of
    the exact score of its id."""
    want = o1_scores(q, q_off, d, d_off, dtype, cand_off, cand_ids)
    gs, gi = (t.cpu().numpy() for t in got)
    n_docs = len(d_off) - 1
    tol = REL_TOL_DT[dtype] * 64
    for a in range(len(q_off) - 1):
        if cand_off is None:
            seg = want[a * n_docs:(a + 1) * n_docs]
            ids = np.arange(n_docs)
        else:
            seg = want[cand_off[a]:cand_off[a + 1]]
            ids = np.asarray(cand_ids[cand_off[a]:cand_off[a + 1]], np.int64)
        wi, ws = oracle.topk(seg, k, ids if cand_off is not None else None)
        real = wi >= 0
        assert np.array_equal(gi[a][~real], wi[~real]), a
        by_id = {}
        for i, s in zip(ids.tolist(), seg.tolist()):
            by_id[i] = max(by_id.get(i, -np.inf), s)
        for j in np.nonzero(real)[0]:
            e = by_id[int(gi[a][j])]
            if np.isfinite(e):
                assert abs(float(gs[a][j]) - e) <= tol, (a, j)
            # rank j of the GPU list is a near-tie of rank j of the oracle list
            if np.isfinite(ws[j]):
                assert abs(e - ws[j]) <= 2 * tol, (a, j, e, ws[j])


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("k", [1, 10, 100])
def test_single_query_bit_identical(dtype, k):
    q, q_off, d, d_off = _ragged(3000, 128, seed=11, nq_lens=[32], empty_every=97)
    Q = device_tokens(q, q_off, dtype)
    D = device_tokens(d, d_off, dtype)
    got = M.score_topk(Q, D, k)
    want, _ = _reference(Q, D, k)
    _assert_identical(got, want, f"{dtype} k={k}")
    _check_vs_oracle(got, q, q_off, d, d_off, dtype, k)


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("dim", [64, 256, 96])
def test_grouped_queries_bit_identical(dtype, dim):
    # uneven query lengths (grouped units share document reads), d beyond one
    # chunk and d not a multiple of the chunk
    q, q_off, d, d_off = _ragged(1500, dim, seed=dim, nq_lens=[32, 5, 17, 9, 32, 1, 12],
                                 empty_every=41)
    Q = device_tokens(q, q_off, dtype)
    D = device_tokens(d, d_off, dtype)
    for k in (3, 100):
        got = M.score_topk(Q, D, k)
        want, _ = _reference(Q, D, k)
        _assert_identical(got, want, f"{dtype} d={dim} k={k}")
    _check_vs_oracle(got, q, q_off, d, d_off, dtype, 100)


@pytest.mark.parametrize("dtype", DTYPES)
def test_candidates_bit_identical(dtype):
    q, q_off, d, d_off = _ragged(4000, 128, seed=5, nq_lens=[32, 8, 64, 20, 3], empty_every=53)
    g = W.rng(9)
    sizes = [700, 0, 2500, 40, 1300]  # an empty list, a list shorter than k
    ids = [g.choice(4000, s, replace=False).astype(np.int32) for s in sizes]
    ids[2][::7] = ids[2][3]  # repeated ids inside one list
    cand_off = W.offsets_from_lengths(sizes)
    cand_ids = np.concatenate(ids).astype(np.int32)
    Q = device_tokens(q, q_off, dtype)
    D = device_tokens(d, d_off, dtype)
    C = M.Candidates(dev(cand_off), dev(cand_ids))
    for k in (1, 100, 1024):
        got = M.score_topk(Q, D, k, cand=C)
        want, _ = _reference(Q, D, k, C)
        _assert_identical(got, want, f"{dtype} candidates k={k}")
    _check_vs_oracle(M.score_topk(Q, D, 100, cand=C), q, q_off, d, d_off, dtype, 100,
                     cand_off, cand_ids)


def test_padding_ties_and_degenerate_queries():
    # fewer docs than k, empty documents (-inf), an empty query (every score
    # 0: a tie broken by id), and two identical documents (an exact tie)
    lens = W.doc_lengths(60, 3)
    lens[::4] = 0
    lens[5] = lens[1]
    d_off = W.offsets_from_lengths(lens)
    d = W.unit_tokens(int(d_off[-1]), 128, W.rng(4))
    d[d_off[5]:d_off[6]] = d[d_off[1]:d_off[2]]
    q_off = W.offsets_from_lengths([32, 0, 7])
    q = W.unit_tokens(int(q_off[-1]), 128, W.rng(5))
    Q = device_tokens(q, q_off, "f16", max_len=32)
    D = device_tokens(d, d_off, "f16")
    for k in (5, 60, 100, 1024):
        got = M.score_topk(Q, D, k)
        want, s = _reference(Q, D, k)
        _assert_identical(got, want, f"degenerate k={k}")
    s = s.cpu().numpy()
    assert s[1] == s[5] and np.isneginf(s[0]) and (s[60:120] == 0).all()
    # no documents at all: every row is padding
    E = device_tokens(np.zeros((0, 128), np.float32), np.zeros(1, np.int64), "f16")
    gs, gi = M.score_topk(Q, E, 10)
    assert (gi.cpu().numpy() == -1).all()
    assert np.isneginf(gs.cpu().numpy()).all()


def test_ranges_beyond_the_lds_key_slots():
    # 1M documents of 1 token, then of 3, and four 32-token queries sharing
    # one unit: with the shipped launch shapes the waves over the one-token
    # half hold more keys than their LDS slots and spill them to the
    # workspace, the others keep theirs in LDS.
    n = 1_000_000
    lens = np.where(np.arange(n) < n // 2, 1, 3)
    d_off = W.offsets_from_lengths(lens)
    T = int(d_off[-1])
    d = W.unit_tokens_gpu(T, 128, seed=77)
    q_off = W.offsets_from_lengths([32, 32, 32, 32])
    q = W.unit_tokens(128, 128, W.rng(78))
    Q = device_tokens(q, q_off, "f16", max_len=32)
    dt, _ = M.quantize(d, "f16")
    del d
    D = M.Tokens(dt, dev(d_off), "f16", None, max_len=3)
    for k in (100, 1000):
        got = M.score_topk(Q, D, k)
        want, _ = _reference(Q, D, k)
        _assert_identical(got, want, f"mixed spill k={k}")
    # one query alone
    Q1 = device_tokens(q[:32], [0, 32], "f16", max_len=32)
    got = M.score_topk(Q1, D, 100)
    want, _ = _reference(Q1, D, 100)
    _assert_identical(got, want, "one query, 1M short docs")
    del dt, D
    torch.cuda.empty_cache()


def test_repeated_calls_reuse_the_workspace():
    q, q_off, d, d_off = _ragged(2000, 128, seed=21, nq_lens=[32, 16])
    Q = device_tokens(q, q_off, "bf16")
    D = device_tokens(d, d_off, "bf16")
    ws = torch.empty(M.score_topk_workspace_bytes(Q, D, 50), dtype=torch.uint8, device="cuda")
    first = M.score_topk(Q, D, 50, workspace=ws)
    first = tuple(t.clone() for t in first)
    ws.fill_(0xA5)  # contents are ignored
    second = M.score_topk(Q, D, 50, workspace=ws)
    _assert_identical(second, first, "second call")
    with pytest.raises(M.MaxSimError):
        M.score_topk(Q, D, 50, workspace=ws[:ws.numel() - 1])
