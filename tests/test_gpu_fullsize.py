"""GPU parity at the benchmark's full sizes, in the launch configurations the
benchmark times (the packaged tuned launch shapes load with the library).

The oracle cannot score a million documents in a test, so each workload is
checked on seeded samples scored one by one in FP64, and the top-100 is
checked against the exact top-100: the GPU's scores are within the O1 gate of
the exact ones, so every document whose exact score can reach the exact
100th lies in {GPU score >= GPU 100th - margin}; the oracle scores that set
exactly and the exact top-100 follows.
"""
import numpy as np
import pytest
import torch

import oracle
import paper_2606_26439_amd as M
import workloads as W
from tests._gpu import (REL_TOL_DT, assert_close_o1, assert_topk_matches_exact, device_tokens,
                        doc_rows, gen_device_tokens)

pytestmark = pytest.mark.gpu

N_DOCS = 1_000_000
K = 100


def _release():
    torch.cuda.synchronize()
    torch.cuda.empty_cache()


def _exact_topk_by_id(gpu_scores, margin, score_fn, k=K):
    """Oracle scores of every document whose GPU score is within `margin` of
    the GPU's k-th best; returns {id: exact score}."""
    kth = float(torch.topk(gpu_scores, k).values[-1])
    cand = torch.nonzero(gpu_scores >= kth - margin).flatten().cpu().numpy()
    assert len(cand) < 20000, len(cand)
    ex = score_fn(cand)
    return dict(zip(cand.tolist(), ex.tolist()))


def test_plain_fp32_4096_docs_every_score():
    # 4,096 docs of 32 tokens, one 32-token query, FP32, seed 0: every score
    # against the oracle, and the top-100 ids.
    c = W.plain_fp32_case()
    Q = device_tokens(c["q"], c["q_off"], "f32", max_len=32)
    D = device_tokens(c["d"], c["d_off"], "f32", max_len=32)
    got = M.score(Q, D)
    want = oracle.maxsim(c["q"].astype(np.float64), c["q_off"], c["d"].astype(np.float64),
                         c["d_off"])
    assert_close_o1(got.cpu().numpy(), want, "plain fp32", "f32")
    seg = torch.tensor([0, len(want)], dtype=torch.int64, device="cuda")
    _, ids = M.topk(got, seg, K)
    exact = dict(enumerate(want.tolist()))
    assert_topk_matches_exact(ids.cpu().numpy()[0], None, exact, K, 1e-5 * 32, "plain fp32")


@pytest.fixture(scope="module")
def ragged_1m():
    lens = W.doc_lengths(N_DOCS, 0)
    d_off = W.offsets_from_lengths(lens)
    T = int(d_off[-1])
    d32 = W.unit_tokens_gpu(T, 128, seed=1000)
    q = W.unit_tokens(32, 128, W.rng(1))
    yield dict(d_off=d_off, T=T, d32=d32, q=q, d_off_dev=torch.from_numpy(d_off).cuda())
    del d32
    _release()


@pytest.mark.parametrize("dtype", ["f32", "bf16", "f16", "fp8"])
def test_ragged_1m_docs_sampled_and_top100(ragged_1m, dtype):
    w = ragged_1m
    qt, qs = M.quantize(torch.from_numpy(w["q"]).cuda(), dtype)
    Q = M.Tokens(qt, torch.tensor([0, 32], device="cuda"), dtype, qs, max_len=32)
    dt, ds = M.quantize(w["d32"], dtype)
    D = M.Tokens(dt, w["d_off_dev"], dtype, ds, max_len=180)
    scores = M.score(Q, D)
    # every document scored directly equals the candidate list of all of
    # them, bit for bit (for FP32 the direct form packs each document's last
    # partial tile with the next document's rows, the candidate form clamps)
    ids_all = torch.arange(N_DOCS, dtype=torch.int32, device="cuda")
    per_doc = M.score(Q, D, M.Candidates(torch.tensor([0, N_DOCS], device="cuda"), ids_all))
    assert torch.equal(scores.view(torch.int32), per_doc.view(torch.int32)), dtype
    del ids_all, per_doc
    qv, _ = oracle.exact_values(w["q"], dtype)

    def o1(docs):
        rows, off = doc_rows(w["d_off"], docs)
        x = w["d32"][torch.from_numpy(rows).cuda()].cpu().numpy()
        dv, _ = oracle.exact_values(x, dtype)
        return oracle.maxsim(qv, [0, 32], dv, off)

    # seeded sample of 3,000 documents, incl. the first and the last
    samp = np.unique(np.concatenate([[0, N_DOCS - 1],
                                     W.rng(17).choice(N_DOCS, 3000, replace=False)]))
    assert_close_o1(scores[torch.from_numpy(samp).cuda()].cpu().numpy(), o1(samp),
                    f"1M {dtype}", dtype)
    # top-100 through the library's top-k against the exact top-100 of O1
    seg = torch.tensor([0, N_DOCS], dtype=torch.int64, device="cuda")
    _, ids = M.topk(scores, seg, K)
    tol = REL_TOL_DT[dtype] * 32
    exact = _exact_topk_by_id(scores, 4 * tol, o1)
    assert_topk_matches_exact(ids.cpu().numpy()[0], None, exact, K, 2 * tol, f"1M {dtype}")
    del dt, ds, D, scores
    _release()


def test_ragged_1m_f16_fused_and_unfused_top100_identical(ragged_1m):
    # The headline comparison at its full size (1M ragged docs, one 32-token
    # query, d = 128, FP16): the unfused comparator that materialises S and
    # the fused scorer select the same top-100 ids, and both equal the exact
    # top-100 of the oracle up to swaps between near-ties.
    w = ragged_1m
    qt, _ = M.quantize(torch.from_numpy(w["q"]).cuda(), "f16")
    Q = M.Tokens(qt, torch.tensor([0, 32], device="cuda"), "f16", None, max_len=32)
    dt, _ = M.quantize(w["d32"], "f16")
    D = M.Tokens(dt, w["d_off_dev"], "f16", None, max_len=180)
    seg = torch.tensor([0, N_DOCS], dtype=torch.int64, device="cuda")
    fused = M.score(Q, D)
    _, ids_f = M.topk(fused, seg, K)
    ws = torch.empty(M.unfused_workspace_bytes(Q, D), dtype=torch.uint8, device="cuda")
    unfused = M.score_unfused(Q, D, workspace=ws)
    del ws
    _, ids_u = M.topk(unfused, seg, K)
    ids_f, ids_u = ids_f.cpu().numpy()[0], ids_u.cpu().numpy()[0]
    assert set(ids_f.tolist()) == set(ids_u.tolist())
    qv, _ = oracle.exact_values(w["q"], "f16")

    def o1(docs):
        rows, off = doc_rows(w["d_off"], docs)
        x = w["d32"][torch.from_numpy(rows).cuda()].cpu().numpy()
        dv, _ = oracle.exact_values(x, "f16")
        return oracle.maxsim(qv, [0, 32], dv, off)

    tol = REL_TOL_DT["f16"] * 32
    exact = _exact_topk_by_id(fused, 4 * tol, o1)
    assert_topk_matches_exact(ids_f, None, exact, K, 2 * tol, "1M f16 fused")
    assert_topk_matches_exact(ids_u, None, exact, K, 2 * tol, "1M f16 unfused")
    # and the scores themselves agree within the gate on a sample
    samp = torch.from_numpy(np.sort(W.rng(23).choice(N_DOCS, 2000, replace=False))).cuda()
    assert_close_o1(unfused[samp].cpu().numpy(), fused[samp].cpu().numpy().astype(np.float64),
                    "unfused vs fused", "f16")
    del dt, D, fused, unfused
    _release()


@pytest.mark.parametrize("dim", [64, 256, 512, 768])
def test_dimension_tiling_500k_docs_sampled(dim):
    B, nd = 500_000, 128
    samp = np.sort(W.rng(11 + dim).choice(B, 64, replace=False))
    rows = (samp[:, None] * nd + np.arange(nd)[None, :]).ravel()
    tok, _, f32 = gen_device_tokens(B * nd, dim, "bf16", seed=3000 + dim, sample_rows=rows)
    q = W.unit_tokens(32, dim, W.rng(1))
    qt, _ = M.quantize(torch.from_numpy(q).cuda(), "bf16")
    Q = M.Tokens(qt, torch.tensor([0, 32], device="cuda"), "bf16", None, max_len=32)
    D = M.Tokens(tok, torch.arange(B + 1, device="cuda", dtype=torch.int64) * nd, "bf16", None,
                 max_len=nd)
    got = M.score(Q, D)[torch.from_numpy(samp).cuda()].cpu().numpy()
    qv, _ = oracle.exact_values(q, "bf16")
    dv, _ = oracle.exact_values(f32, "bf16")
    want = oracle.maxsim(qv, [0, 32], dv, np.arange(len(samp) + 1) * nd)
    assert_close_o1(got, want, f"d={dim}", "bf16")
    del tok, D
    _release()


def test_pq_2m_docs_64_queries_sampled_and_top100():
    n_docs, nq, n_q = 2_000_000, 32, 64
    lens = W.doc_lengths(n_docs, 0)
    d_off = W.offsets_from_lengths(lens)
    T = int(d_off[-1])
    codes = W.pq_codes_gpu(T, 8, 256, seed=2)
    cb = W.pq_codebooks(8, 256, 16, seed=2)
    q = W.unit_tokens(n_q * nq, 128, W.rng(1))
    qt, _ = M.quantize(torch.from_numpy(q).cuda(), "f16")
    Q = M.Tokens(qt, torch.from_numpy(np.arange(n_q + 1, dtype=np.int64) * nq).cuda(), "f16",
                 None, max_len=nq)
    D = M.PQDocs(torch.from_numpy(cb).cuda(), codes, torch.from_numpy(d_off).cuda())
    scores = M.pq_score(Q, D).view(n_q, n_docs)
    qv, _ = oracle.exact_values(q, "f16")
    cb64 = cb.astype(np.float64)

    def o1(a, docs):
        rows, off = doc_rows(d_off, docs)
        c = codes[torch.from_numpy(rows).cuda()].cpu().numpy()
        return oracle.pq_decode_score(qv[a * nq:(a + 1) * nq], [0, nq], c, cb64, off)

    samp = np.sort(W.rng(13).choice(n_docs, 400, replace=False))
    for a in (0, 31, 63):
        got = scores[a, torch.from_numpy(samp).cuda()].cpu().numpy()
        assert_close_o1(got, o1(a, samp), f"pq query {a}", "f32")
    seg = torch.from_numpy(np.arange(n_q + 1, dtype=np.int64) * n_docs).cuda()
    _, ids = M.topk(scores.reshape(-1), seg, K)
    ids = ids.cpu().numpy()
    for a in (0, 63):
        exact = _exact_topk_by_id(scores[a], 2e-3, lambda docs: o1(a, docs))
        assert_topk_matches_exact(ids[a], None, exact, K, 4e-4, f"pq top-100 query {a}")
    del codes, D, scores
    _release()
