"""Serving on the GPU: every request's top-k is the same alone and in a mix
of concurrently batched requests (bit for bit), for exact, PQ and
residual-compressed scoring, and agrees with the FP64 oracle's ranking."""
import numpy as np
import pytest
import torch

import oracle
import paper_2606_26439_amd as M
import workloads as W
from paper_2606_26439_amd import serve as S
from tests._gpu import dev

pytestmark = pytest.mark.gpu

N_POOL = 6000


@pytest.fixture(scope="module")
def pool():
    c = W.ragged_case(N_POOL, dim=128, nq=32)
    tok, _ = M.quantize(dev(c["d"]), "f16")
    d_off = dev(c["d_off"])
    docs = M.Tokens(tok, d_off, "f16", None, max_len=180)
    cb = W.pq_codebooks(8, 256, 16, seed=2)
    codes = W.pq_codes(int(c["d_off"][-1]), seed=2)
    pq = M.PQDocs(dev(cb), dev(codes), d_off)
    T = int(c["d_off"][-1])
    cen = W.residual_centroids(512, 128, seed=5)
    wts = W.residual_weights(2)
    rids = W.residual_ids(T, 512, seed=6)
    rcodes = W.residual_codes(T, 128, 2, seed=6)
    res = M.ResidualDocs(dev(cen), dev(wts), dev(rids), dev(rcodes), d_off, 2)
    return dict(docs=docs, pq=pq, res=res, d=c["d"], d_off=c["d_off"], cb=cb, codes=codes,
                cen=cen, wts=wts, rids=rids, rcodes=rcodes)


def _requests(n, seed=0):
    g = W.rng(seed)
    off, ids = W.candidates(n, N_POOL, seed=seed + 4, size_range=(50, 3000))
    reqs = []
    for i in range(n):
        q = W.unit_tokens(int(g.integers(8, 65)), 128, g)
        reqs.append(S.Request(i, q, ids[off[i]:off[i + 1]].copy(),
                              mode=("exact", "pq", "residual")[(i // 4) % 3]))
    return reqs


def _clone(r):
    return S.Request(r.rid, r.query, r.cand_ids, mode=r.mode)


def test_alone_equals_mixed(pool):
    reqs = _requests(60)
    be = S.GpuBackend(pool["docs"], pool["pq"], k=100, n_slots=3, pool_res=pool["res"])
    mixed = [_clone(r) for r in reqs]
    t0 = 0.0
    arr = W.poisson_arrivals(len(mixed), 20000.0, seed=9)
    import time
    start = time.perf_counter()
    for r, a in zip(mixed, arr):
        r.arrival = start + float(a) + t0
    srv = S.Server(S.Scheduler(128, 100, max_inflight=3), be)
    done = srv.run(mixed)
    assert all(r.status == "done" for r in done)
    assert srv.batches_launched < len(mixed)  # requests really were batched together
    for r in reqs:
        alone = _clone(r)
        S.Server(S.Scheduler(128, 100, max_inflight=1, max_batch_requests=1), be).run([alone])
        m = next(x for x in mixed if x.rid == r.rid)
        assert np.array_equal(alone.top_ids, m.top_ids), r.rid
        assert np.array_equal(alone.top_scores.view(np.uint32), m.top_scores.view(np.uint32)), r.rid


def test_served_topk_matches_oracle(pool):
    reqs = _requests(6, seed=5)
    be = S.GpuBackend(pool["docs"], pool["pq"], k=100, pool_res=pool["res"])
    S.Server(S.Scheduler(128, 100), be).run(reqs)
    dv, _ = oracle.exact_values(pool["d"], "f16")
    for r in reqs:
        qv, _ = oracle.exact_values(r.query, "f16")
        nq = len(qv)
        if r.mode == "pq":
            want = oracle.pq_decode_score(qv, [0, nq], pool["codes"], pool["cb"].astype(np.float64),
                                          pool["d_off"], [0, len(r.cand_ids)], r.cand_ids)
        elif r.mode == "residual":
            want = oracle.residual_decode_score(qv, [0, nq], pool["rids"], pool["rcodes"],
                                                pool["cen"].astype(np.float64),
                                                pool["wts"].astype(np.float64), 2, pool["d_off"],
                                                [0, len(r.cand_ids)], r.cand_ids)
        else:
            want = oracle.maxsim(qv, [0, nq], dv, pool["d_off"], [0, len(r.cand_ids)], r.cand_ids)
        by_id = dict(zip(r.cand_ids.tolist(), want.tolist()))
        k = min(100, len(r.cand_ids))
        kth = np.sort(want)[::-1][k - 1]
        got = [i for i in r.top_ids.tolist() if i >= 0]
        assert len(got) == k
        # every selected doc is within the score tolerance of the oracle's k-th best
        assert all(by_id[i] >= kth - 1e-4 * max(1.0, abs(kth)) for i in got), r.rid
        # and the returned scores match the oracle's scores of those docs
        np.testing.assert_allclose(r.top_scores[:k].astype(np.float64),
                                   [by_id[i] for i in got], rtol=1e-5, atol=1e-5)


def test_full_5m_pool_requests_match_oracle():
    # The serving pool at full size (5M FP16 docs, 88.8 GB, plus the PQ copy);
    # a few requests with small candidate sets so the oracle scores every one.
    from tests._gpu import doc_rows, gen_device_tokens
    n_pool, k = 5_000_000, 100
    lens = W.doc_lengths(n_pool, 0)
    d_off = W.offsets_from_lengths(lens)
    T = int(d_off[-1])
    g = W.rng(21)
    cands = [np.sort(g.choice(n_pool, int(n), replace=False)).astype(np.int32)
             for n in (150, 1200, 2500, 2500)]
    rows_all, _ = doc_rows(d_off, np.unique(np.concatenate(cands)))
    tok, _, f32 = gen_device_tokens(T, 128, "f16", seed=5000, sample_rows=rows_all)
    d_off_dev = dev(d_off)
    docs = M.Tokens(tok, d_off_dev, "f16", None, max_len=int(lens.max()))
    codes = W.pq_codes_gpu(T, 8, 256, seed=2)
    cb = W.pq_codebooks(8, 256, 16, seed=2)
    pq = M.PQDocs(dev(cb), codes, d_off_dev)
    reqs = [S.Request(i, W.unit_tokens(int(g.integers(8, 65)), 128, g), c,
                      mode="pq" if i % 2 else "exact") for i, c in enumerate(cands)]
    be = S.GpuBackend(docs, pq, k=k)
    S.Server(S.Scheduler(128, k), be).run(reqs)
    # position of each pool row inside the gathered FP32 sample
    where = {int(r): i for i, r in enumerate(rows_all)}
    cb64 = cb.astype(np.float64)
    for r in reqs:
        assert r.status == "done", (r.rid, r.status, r.error)
        rows, off = doc_rows(d_off, r.cand_ids)
        qv, _ = oracle.exact_values(r.query, "f16")
        nq = len(qv)
        if r.mode == "pq":
            c = codes[torch.from_numpy(rows).cuda()].cpu().numpy()
            want = oracle.pq_decode_score(qv, [0, nq], c, cb64, off)
        else:
            dv, _ = oracle.exact_values(f32[[where[int(x)] for x in rows]], "f16")
            want = oracle.maxsim(qv, [0, nq], dv, off)
        kk = min(k, len(want))
        ex_ids, ex_s = oracle.topk(want, kk, r.cand_ids.astype(np.int64))
        by_id = dict(zip(r.cand_ids.tolist(), want.tolist()))
        got = r.top_ids[:kk].tolist()
        kth = float(ex_s[kk - 1])
        for i in set(got) ^ set(ex_ids.tolist()):  # only near-ties may differ
            assert abs(by_id[i] - kth) <= 1e-5 * 64, (r.rid, i)
        np.testing.assert_allclose(r.top_scores[:kk].astype(np.float64),
                                   [by_id[i] for i in got], rtol=1e-5, atol=1e-5)
    del tok, docs, codes, pq, be
    torch.cuda.empty_cache()
