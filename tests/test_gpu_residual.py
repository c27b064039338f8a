"""GPU parity of MaxSim over residual-compressed documents (centroid id plus a
per-dimension quantized residual), through the C ABI, against the FP64
oracle's decode-then-score.

Small cases span several 16-token tiles, ragged tails, empty documents and
queries, every residual width (1, 2, 4 bits), every dimension (64, 128, 256)
and every query-block count; the full-size case is the benchmark's workload
(1M documents, 2^17 centroids, 2-bit residuals) checked on sampled documents
and through the exact top-100.
"""
import json

import numpy as np
import pytest
import torch

import oracle
import paper_2606_26439_amd as M
import workloads as W
from tests._gpu import REL_TOL, assert_close_o1, assert_topk_matches_exact, dev, doc_rows

pytestmark = pytest.mark.gpu


def _case(n_docs, dim, nbits, n_c, seed, nq_lens, integer=False):
    g = W.rng(seed)
    lens = W.doc_lengths(n_docs, seed)
    lens[0] = 0
    lens[1] = 1
    lens[2] = 17  # one full tile and a one-row tail
    lens[3] = 16
    d_off = W.offsets_from_lengths(lens)
    T = int(d_off[-1])
    q_off = W.offsets_from_lengths(nq_lens)
    if integer:
        cen = g.integers(-2, 3, size=(n_c, dim)).astype(np.float16)
        w = g.integers(-2, 3, size=1 << nbits).astype(np.float16)
        q = g.integers(-1, 2, size=(int(q_off[-1]), dim)).astype(np.float16)
    else:
        cen = W.residual_centroids(n_c, dim, seed=seed + 5)
        w = W.residual_weights(nbits)
        q = W.unit_tokens(int(q_off[-1]), dim, g).astype(np.float16)
    ids = W.residual_ids(T, n_c, seed=seed + 6)
    res = W.residual_codes(T, dim, nbits, seed=seed + 6)
    return dict(q=q, q_off=q_off, cen=cen, w=w, ids=ids, res=res, d_off=d_off, nbits=nbits)


def _device(c, max_len=None):
    Q = M.Tokens(dev(c["q"]), dev(c["q_off"]), "f16", max_len=max_len)
    D = M.ResidualDocs(dev(c["cen"]), dev(c["w"]), dev(c["ids"]), dev(c["res"]), dev(c["d_off"]),
                       c["nbits"])
    return Q, D


def _oracle(c, cand_off=None, cand_ids=None):
    return oracle.residual_decode_score(c["q"].astype(np.float64), c["q_off"], c["ids"], c["res"],
                                        c["cen"].astype(np.float64), c["w"].astype(np.float64),
                                        c["nbits"], c["d_off"], cand_off, cand_ids)


@pytest.mark.parametrize("nbits", [1, 2, 4])
@pytest.mark.parametrize("dim", [64, 128, 256])
def test_residual_integer_values_are_bit_exact(nbits, dim):
    # small integers: every product and sum is exact in FP32, so any wrong
    # id, bit field or column pairing changes the result
    c = _case(120, dim, nbits, 37, seed=nbits * 7 + dim, nq_lens=[32, 5, 64], integer=True)
    Q, D = _device(c)
    got = M.residual_score(Q, D).cpu().numpy().astype(np.float64)
    assert np.array_equal(got, _oracle(c))


@pytest.mark.parametrize("nbits", [1, 2, 4])
@pytest.mark.parametrize("dim", [64, 128, 256])
def test_residual_matches_decode_then_score(nbits, dim):
    c = _case(300, dim, nbits, 1000, seed=dim + nbits, nq_lens=[32, 7, 64, 1])
    Q, D = _device(c)
    assert_close_o1(M.residual_score(Q, D).cpu().numpy(), _oracle(c), f"residual {dim} {nbits}")


@pytest.mark.parametrize("nq_lens", [[16, 3], [32, 32, 20], [0, 12]])
def test_residual_query_blocks_and_empty_query(nq_lens):
    # max_len 16 / 32 / 12: one, two and one 16-column query blocks; an
    # empty query scores 0 against every document (and -inf never appears)
    c = _case(200, 128, 2, 500, seed=len(nq_lens) + sum(nq_lens), nq_lens=nq_lens)
    Q, D = _device(c)
    got = M.residual_score(Q, D).cpu().numpy()
    want = _oracle(c)
    assert_close_o1(got, want, f"residual nq {nq_lens}")
    if nq_lens[0] == 0:
        assert np.all(got[:200] == 0.0)


def test_residual_candidates():
    c = _case(600, 128, 2, 2000, seed=11, nq_lens=[32, 16, 50])
    cand_off, cand_ids = W.candidates(3, 600, seed=12, size_range=(50, 400))
    Q, D = _device(c)
    got = M.residual_score(Q, D, M.Candidates(dev(cand_off), dev(cand_ids))).cpu().numpy()
    assert_close_o1(got, _oracle(c, cand_off, cand_ids), "residual candidates")


def test_residual_query_longer_than_bound_is_nan():
    # max_len declared 16 but the second query has 20 tokens: its scores are
    # NaN (the bound sizes the kernel's query registers), the first's are exact
    c = _case(100, 128, 2, 64, seed=3, nq_lens=[16, 20])
    Q, D = _device(c, max_len=16)
    got = M.residual_score(Q, D).cpu().numpy()
    want = _oracle(c)
    assert_close_o1(got[:100], want[:100], "residual within bound")
    assert np.all(np.isnan(got[100:]))


def test_residual_zero_weights_equal_plain_fused_path_on_centroids():
    # with every residual value 0 a token is its centroid: the same scores as
    # the plain fused scorer on the gathered centroid rows (two GPU paths)
    c = _case(250, 128, 2, 300, seed=17, nq_lens=[32, 9])
    c["w"] = np.zeros(4, np.float16)
    Q, D = _device(c)
    got = M.residual_score(Q, D).cpu().numpy()
    rows = dev(c["cen"][c["ids"]])
    plain = M.score(Q, M.Tokens(rows, dev(c["d_off"]), "f16")).cpu().numpy()
    assert_close_o1(got, plain.astype(np.float64), "residual vs plain")
    assert_close_o1(got, _oracle(c), "residual zero weights")


@pytest.fixture
def res_pipe(request, tmp_path):
    """Forces the residual scorer's load-pipeline variant for every key the
    test can touch; afterwards restores the packaged tuning."""
    entries = [{"residual": 1, "nbits": nb, "dim": dm, "nqb": q, "cand": c, "pipe": request.param}
               for nb in (1, 2, 4) for dm in (64, 128, 256) for q in (1, 2, 4) for c in (0, 1)]
    path = tmp_path / "res.json"
    path.write_text(json.dumps({"version": 1, "entries": entries}))
    M.load_tune_cache(str(path))
    yield request.param
    # the packaged cache holds no forced entries for these keys: drop them
    entries = [dict(e, pipe=2) for e in entries]
    path.write_text(json.dumps({"version": 1, "entries": entries}))
    M.load_tune_cache(str(path))
    M.load_tune_cache(M.default_tune_cache())


@pytest.mark.parametrize("res_pipe", [0, 1, 2, 3], indirect=True)
@pytest.mark.parametrize("nbits", [1, 2, 4])
def test_residual_every_pipeline_variant(res_pipe, nbits):
    # ragged docs (tiles of 1..16 rows, empty docs) and candidate lists with
    # every ring depth
    c = _case(400, 128, nbits, 300, seed=31 + nbits, nq_lens=[32, 13, 64, 0])
    cand_off, cand_ids = W.candidates(4, 400, seed=32, size_range=(1, 300))
    Q, D = _device(c)
    got = M.residual_score(Q, D).cpu().numpy()
    assert_close_o1(got, _oracle(c), f"residual pipe {res_pipe}")
    got_c = M.residual_score(Q, D, M.Candidates(dev(cand_off), dev(cand_ids))).cpu().numpy()
    assert_close_o1(got_c, _oracle(c, cand_off, cand_ids), f"residual cand pipe {res_pipe}")


def test_residual_autotune_keeps_results_within_tolerance(tmp_path):
    c = _case(3000, 128, 2, 4096, seed=41, nq_lens=[32])
    Q, D = _device(c)
    rep = M.residual_autotune(Q, D, reps=2, cache_path=str(tmp_path / "t.json"))
    assert {t["pipe"] for t in rep["trials"]} == {0, 1, 2, 3}, rep
    assert '"residual":1' in (tmp_path / "t.json").read_text()
    assert_close_o1(M.residual_score(Q, D).cpu().numpy(), _oracle(c), "residual after autotune")
    M.load_tune_cache(M.default_tune_cache())


def test_residual_no_documents_and_workspace_checks():
    c = _case(50, 128, 2, 64, seed=5, nq_lens=[32])
    Q, D = _device(c)
    need = M.residual_workspace_bytes(Q, D)
    assert need == 64 * 32 * 4
    ws = torch.empty(need - 256, dtype=torch.uint8, device="cuda")
    with pytest.raises(M.MaxSimError) as e:
        M.residual_score(Q, D, workspace=ws)
    assert e.value.status == 3
    empty = M.ResidualDocs(D.centroids, D.weights, D.centroid_ids[:0], D.residuals[:0],
                           torch.zeros(1, dtype=torch.int64, device="cuda"), 2)
    assert M.residual_score(Q, empty).numel() == 0


def test_residual_documents_without_tokens():
    # five documents, none with a token (no id or code arrays at all): -inf
    # for a query with tokens, 0 for an empty query
    c = _case(40, 128, 2, 64, seed=13, nq_lens=[32, 0])
    Q, D = _device(c)
    empty = M.ResidualDocs(D.centroids, D.weights, D.centroid_ids[:0], D.residuals[:0],
                           torch.zeros(6, dtype=torch.int64, device="cuda"), 2)
    got = M.residual_score(Q, empty).cpu().numpy()
    assert np.all(np.isneginf(got[:5])) and np.all(got[5:] == 0.0)


def test_residual_validate_flags_bad_centroid_ids():
    c = _case(80, 128, 2, 64, seed=9, nq_lens=[32])
    Q, D = _device(c)
    M.validate(D, Q)  # clean
    D.centroid_ids[5] = 64
    with pytest.raises(M.MaxSimError) as e:
        M.validate(D, Q)
    assert e.value.status == 5 and "centroid ids" in str(e.value)
    D.centroid_ids[5] = -1
    with pytest.raises(M.MaxSimError):
        M.validate(D, Q)


# ------------------------------------------------------- full size

N_DOCS = 1_000_000
N_CENTROIDS = 1 << 17


def test_residual_full_size_sampled_and_top100():
    """The benchmark's workload: 1M ragged docs, one 32-token F16 query,
    d = 128, 2^17 centroids, 2-bit residuals."""
    lens = W.doc_lengths(N_DOCS, 0)
    d_off = W.offsets_from_lengths(lens)
    T = int(d_off[-1])
    cen = W.residual_centroids(N_CENTROIDS, 128, seed=5)
    w = W.residual_weights(2)
    ids = W.residual_ids_gpu(T, N_CENTROIDS, seed=6)
    res = W.residual_codes_gpu(T, 128, 2, seed=6)
    q = W.unit_tokens(32, 128, W.rng(1)).astype(np.float16)
    q_off = np.array([0, 32], np.int64)
    Q = M.Tokens(dev(q), dev(q_off), "f16")
    D = M.ResidualDocs(dev(cen), dev(w), ids, res, dev(d_off), 2)
    got = M.residual_score(Q, D)
    torch.cuda.synchronize()
    gs = got.cpu().numpy()

    def exact(docs):
        docs = np.asarray(docs, np.int64)
        rows, off = doc_rows(d_off, docs)
        r = torch.from_numpy(rows).cuda()
        return oracle.residual_decode_score(q.astype(np.float64), q_off,
                                            ids[r].cpu().numpy(), res[r].cpu().numpy(),
                                            cen.astype(np.float64), w.astype(np.float64), 2, off)

    sample = np.sort(W.rng(77).choice(N_DOCS, size=3000, replace=False))
    sample[:2] = [0, N_DOCS - 1]
    assert_close_o1(gs[sample], exact(sample), "residual 1M sampled")
    # exact top-100: every doc that can reach the exact 100th is within the
    # gate of the GPU's 100th
    margin = 4 * REL_TOL * 32
    kth = float(torch.topk(got, 100).values[-1])
    cand = torch.nonzero(got >= kth - margin).flatten().cpu().numpy()
    assert len(cand) < 20000
    exact_by_id = dict(zip(cand.tolist(), exact(cand).tolist()))
    seg = torch.tensor([0, N_DOCS], dtype=torch.int64, device="cuda")
    _, top_ids = M.topk(got, seg, 100)
    assert_topk_matches_exact(top_ids.cpu().numpy()[0], None, exact_by_id, 100, REL_TOL * 32,
                              "residual 1M top-100")
    del ids, res, got, D
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
