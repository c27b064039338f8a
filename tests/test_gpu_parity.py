"""GPU parity: the HIP path through the C ABI against the FP64 oracle.

Sizes keep the oracle to seconds while spanning several 16-row tiles, ragged
tails, empty documents, every query-token capacity and every d-chunk width.
"""
import json

import numpy as np
import pytest
import torch

import oracle
import paper_2606_26439_amd as M
import workloads as W
from tests._gpu import assert_close_o1, dev, device_tokens, o1_scores

pytestmark = pytest.mark.gpu

DTYPES = ["f32", "bf16", "f16", "fp8"]


def _ragged(n_docs, dim, seed, nq_lens, empty_every=0):
    lens = W.doc_lengths(n_docs, seed)
    if empty_every:
        lens[::empty_every] = 0
    lens[1] = 1
    lens[2] = 17  # one full tile + a one-row tail
    d_off = W.offsets_from_lengths(lens)
    g = W.rng(seed + 1)
    d = W.unit_tokens(int(d_off[-1]), dim, g)
    q_off = W.offsets_from_lengths(nq_lens)
    q = W.unit_tokens(int(q_off[-1]), dim, g)
    return q, q_off, d, d_off


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("dim", [64, 128, 768])
def test_quantize_bit_exact(dtype, dim):
    x = W.unit_tokens(1001, dim, W.rng(dim))
    x[5] = 0.0  # all-zero token: scale 1
    x[7] *= 300.0  # large values
    tok, sc = M.quantize(dev(x), dtype)
    torch.cuda.synchronize()
    _, payload = oracle.exact_values(x, dtype)
    if dtype == "f32":
        assert np.array_equal(tok.cpu().numpy().view(np.uint32), x.view(np.uint32))
    elif dtype in ("bf16", "f16"):
        got = tok.view(torch.int16).cpu().numpy().view(np.uint16)
        assert np.array_equal(got, payload[0])
    else:
        assert np.array_equal(tok.cpu().numpy(), payload[0])
        assert np.array_equal(sc.cpu().numpy(), payload[1])


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("dim", [64, 128, 256, 768])
def test_fused_all_docs(dtype, dim):
    nq_lens = [32, 5, 17] if dim <= 256 else [32, 3]
    q, q_off, d, d_off = _ragged(150, dim, seed=dim + 3, nq_lens=nq_lens, empty_every=37)
    Q = device_tokens(q, q_off, dtype)
    D = device_tokens(d, d_off, dtype)
    got = M.score(Q, D).cpu().numpy()
    want = o1_scores(q, q_off, d, d_off, dtype)
    assert_close_o1(got, want, f"{dtype} d={dim}", dtype)


@pytest.mark.parametrize("nq", [1, 16, 31, 33, 48, 64])
def test_fused_query_capacities(nq):
    q, q_off, d, d_off = _ragged(120, 128, seed=nq, nq_lens=[nq, max(1, nq // 2)])
    Q = device_tokens(q, q_off, "f16")
    D = device_tokens(d, d_off, "f16")
    assert_close_o1(M.score(Q, D).cpu().numpy(), o1_scores(q, q_off, d, d_off, "f16"), f"nq={nq}")


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("dim", [192, 1024])
def test_fused_dimension_edges(dtype, dim):
    # d = 192: three 64-wide chunks (not a multiple of 128); d = 1024: the
    # largest supported width (the query blocks fill the LDS beside the ring)
    q, q_off, d, d_off = _ragged(70, dim, seed=dim + 5, nq_lens=[32, 9], empty_every=31)
    Q = device_tokens(q, q_off, dtype)
    D = device_tokens(d, d_off, dtype)
    got = M.score(Q, D).cpu().numpy()
    want = o1_scores(q, q_off, d, d_off, dtype)
    assert_close_o1(got, want, f"{dtype} d={dim}", dtype)


@pytest.mark.parametrize("dtype", DTYPES)
def test_fused_candidates(dtype):
    q, q_off, d, d_off = _ragged(400, 128, seed=11, nq_lens=[8, 64, 20, 1, 40], empty_every=50)
    cand_off, cand_ids = W.candidates(5, 400, seed=4, size_range=(10, 300))
    # a query with no candidates and a repeated id
    sizes = np.diff(cand_off)
    sizes[3] = 0
    ids = [cand_ids[cand_off[a]:cand_off[a + 1]] for a in range(5)]
    ids[3] = ids[3][:0]
    ids[1] = np.concatenate([ids[1], ids[1][:3]])
    cand_ids = np.concatenate(ids).astype(np.int32)
    cand_off = W.offsets_from_lengths([len(x) for x in ids])
    Q = device_tokens(q, q_off, dtype)
    D = device_tokens(d, d_off, dtype)
    C = M.Candidates(dev(cand_off), dev(cand_ids))
    got = M.score(Q, D, C).cpu().numpy()
    want = o1_scores(q, q_off, d, d_off, dtype, cand_off, cand_ids)
    assert_close_o1(got, want, f"{dtype} candidates", dtype)


@pytest.mark.parametrize("dtype", DTYPES)
def test_query_inside_doc_scores_exactly_nq(dtype):
    # Dyadic unit vectors are exact in every format, q.q = 1 exactly and every
    # other dot is < 1, so a document holding every query token scores Nq.
    nq = 24
    q = W.dyadic_unit_vectors(nq, 128, seed=1)
    docs = []
    for b in range(40):
        other = W.dyadic_unit_vectors(30, 128, seed=100 + b)
        sel = np.random.default_rng(b).permutation(nq)[: (nq if b % 2 == 0 else nq // 2)]
        docs.append(np.concatenate([other[:b % 30], q[sel], other[b % 30:]]))
    d_off = W.offsets_from_lengths([len(x) for x in docs])
    d = np.concatenate(docs)
    Q = device_tokens(q, [0, nq], dtype)
    D = device_tokens(d, d_off, dtype)
    got = M.score(Q, D).cpu().numpy()
    assert np.all(got[0::2] == float(nq)), got[0::2]
    want = o1_scores(q, [0, nq], d, d_off, dtype)
    assert_close_o1(got, want, dtype, dtype)


@pytest.mark.parametrize("unfused", [False, True])
def test_fp8_small_integer_tokens_are_bit_exact(unfused):
    # Components that are small integers (|x| <= 15) convert to E4M3 exactly
    # (the per-token power-of-two scale is 2^-4, and 16 x fits E4M3's 3-bit
    # mantissa), every product is an integer and every partial sum of them
    # stays below 2^15: exact in FP32 whatever the order of the additions or
    # the matrix core's internal precision. So here the FP8 path must equal
    # the oracle bit for bit. The looser FP8 gate on Gaussian data (1e-4
    # relative) therefore covers only the rounding of inexact partial sums
    # inside the matrix core; an indexing or scaling error would fail here.
    g = W.rng(77)
    lens = W.doc_lengths(3000, 77)
    lens[::50] = 0
    d_off = W.offsets_from_lengths(lens)
    d = g.integers(-15, 16, size=(int(d_off[-1]), 128)).astype(np.float32)
    q_off = W.offsets_from_lengths([32, 17])
    q = g.integers(-15, 16, size=(int(q_off[-1]), 128)).astype(np.float32)
    Q = device_tokens(q, q_off, "fp8")
    D = device_tokens(d, d_off, "fp8")
    qv, _ = oracle.exact_values(q, "fp8")
    dv, _ = oracle.exact_values(d, "fp8")
    assert np.array_equal(qv, q) and np.array_equal(dv, d)  # the conversion is exact
    got = (M.score_unfused(Q, D) if unfused else M.score(Q, D)).cpu().numpy().astype(np.float64)
    want = oracle.maxsim(qv, q_off, dv, d_off)
    assert np.array_equal(got, want)


@pytest.mark.parametrize("dtype", ["f32", "bf16", "fp8"])
def test_doc_token_permutation_is_bit_identical(dtype):
    q, q_off, d, d_off = _ragged(60, 128, seed=5, nq_lens=[32])
    g = W.rng(9)
    dp = d.copy()
    for b in range(60):
        s, e = d_off[b], d_off[b + 1]
        dp[s:e] = d[s:e][g.permutation(e - s)]
    Q = device_tokens(q, q_off, dtype)
    a = M.score(Q, device_tokens(d, d_off, dtype)).cpu().numpy()
    b = M.score(Q, device_tokens(dp, d_off, dtype)).cpu().numpy()
    assert np.array_equal(a, b)


@pytest.mark.parametrize("dtype", ["bf16", "f16", "f32"])
def test_zero_extended_dimension_is_bit_identical(dtype):
    # Dimension tiling accumulates the 128-wide chunks into the same FP32
    # registers; zero chunks add exact zeros, so the result cannot change.
    q, q_off, d, d_off = _ragged(80, 128, seed=21, nq_lens=[32, 9])
    base = M.score(device_tokens(q, q_off, dtype), device_tokens(d, d_off, dtype)).cpu().numpy()
    for ext in (128, 384, 640):
        qz = np.concatenate([q, np.zeros((len(q), ext), np.float32)], axis=1)
        dz = np.concatenate([d, np.zeros((len(d), ext), np.float32)], axis=1)
        got = M.score(device_tokens(qz, q_off, dtype), device_tokens(dz, d_off, dtype))
        assert np.array_equal(got.cpu().numpy(), base), ext


def test_scores_do_not_depend_on_launch_shape():
    q, q_off, d, d_off = _ragged(300, 128, seed=31, nq_lens=[32, 7, 64])
    Q = device_tokens(q, q_off, "f16")
    D = device_tokens(d, d_off, "f16")
    ref = M.score(Q, D).cpu().numpy()
    rep = M.autotune(Q, D, reps=2)
    assert len(rep["trials"]) >= 6 and rep["best"]["ms"] > 0
    assert np.array_equal(M.score(Q, D).cpu().numpy(), ref)


_DT_CODE = {"f32": 0, "bf16": 1, "f16": 2, "fp8": 3}


def _force_cfg(tmp_path, dtype, dim, stage, pf, nw, wg_per_cu=0, rows=16):
    entries = [{"dtype": _DT_CODE[dtype], "dim": dim, "nqb": nqb, "pf": pf, "nw": nw,
                "wg_per_cu": wg_per_cu, "stage": stage, "rows": rows} for nqb in (1, 2, 4, 8)]
    path = tmp_path / f"cfg_{dtype}_{dim}_{stage}_{pf}_{nw}_{rows}.json"
    path.write_text(json.dumps({"version": 1, "entries": entries}))
    M.load_tune_cache(str(path))


def _expected_lds(dtype, dim, stage, pf, nw, rows):
    """LDS bytes the library asks for under a forced configuration (4 query
    blocks: the cases below have a 64-token query)."""
    esz = {"f32": 4, "bf16": 2, "f16": 2, "fp8": 1}[dtype]
    q1 = 4 * 16 * dim * esz
    dch = 128 if dim % 128 == 0 else 64
    if (stage and esz <= 2 and dim >= 512 and dim % 256 == 0
            and q1 + nw * pf * 16 * 256 * esz <= 160 * 1024):
        dch = 256  # wide chunks: staged tiles whose ring fits
    rt = 32 if (rows == 32 and stage and dim == dch and dtype == "fp8") else 16
    ring = stage * nw * pf * rt * dch * esz
    if dim == dch:  # query operand in VGPRs
        return ring
    if nw * q1 + ring <= 160 * 1024:  # one LDS copy per wave
        return nw * q1 + ring
    return q1 + ring  # one copy per workgroup


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("dim", [64, 128, 256, 768])
def test_every_launch_configuration_is_bit_identical(tmp_path, dtype, dim):
    # Register-direct and LDS-staged tiles, every prefetch depth and
    # workgroup size, 16- and (FP8) 32-row steps: the same wave-level
    # arithmetic, so the same bits.
    q, q_off, d, d_off = _ragged(90, dim, seed=dim + 61, nq_lens=[32, 7, 64, 16], empty_every=29)
    Q = device_tokens(q, q_off, dtype)
    Q2 = device_tokens(q[q_off[2]:], q_off[2:] - q_off[2], dtype)
    D = device_tokens(d, d_off, dtype)
    want = o1_scores(q, q_off, d, d_off, dtype)
    configs = [(stage, pf, nw, 16) for stage in (0, 1) for pf in (2, 3, 4) for nw in (4, 8)]
    if dtype == "fp8":
        configs += [(1, pf, nw, 32) for pf in (2, 3, 4) for nw in (4, 8)]
    ref = None
    try:
        for stage, pf, nw, rows in configs:
            _force_cfg(tmp_path, dtype, dim, stage, pf, nw, rows=rows)
            if _expected_lds(dtype, dim, stage, pf, nw, rows) > 160 * 1024:
                with pytest.raises(M.MaxSimError):
                    M.score(Q, D)
                continue
            got = M.score(Q, D).cpu().numpy()
            if ref is None:
                ref = got
                assert_close_o1(got, want, f"{dtype} d={dim}", dtype)
            assert np.array_equal(got.view(np.uint32), ref.view(np.uint32)), (stage, pf, nw, rows)
            # the last two queries alone give the same bits
            got2 = M.score(Q2, D).cpu().numpy()
            assert np.array_equal(got2.view(np.uint32), ref[2 * 90:].view(np.uint32)), (
                stage, pf, nw, rows)
    finally:
        _force_cfg(tmp_path, dtype, dim, 0, 2 if dtype == "f32" else 4, 4)
        M.load_tune_cache(M.default_tune_cache())


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("nd_max", [3, 20, 40])
def test_all_documents_equal_candidate_lists_of_all(tmp_path, dtype, nd_max):
    # Every document scored directly and as a candidate list of all documents
    # give the same bits, short and empty documents included. Without
    # candidate lists the FP32 form packs a document's last, partial tile with
    # the next document's first rows (with them it clamps the tile to the
    # document's last row), so for FP32 this pins packed tiles to clamped
    # ones, under every launch shape.
    g = W.rng(71 + nd_max)
    n_docs = 700
    lens = g.integers(0, nd_max + 1, n_docs)
    lens[:3] = 0
    lens[-2:] = 0
    lens[10:16] = [16, 15, 17, 1, 31, 33]  # tile-sized, one short, one over, single rows
    d_off = W.offsets_from_lengths(lens)
    d = W.unit_tokens(int(d_off[-1]), 128, g)
    q_off = W.offsets_from_lengths([32, 7, 0, 64, 20])
    q = W.unit_tokens(int(q_off[-1]), 128, g)
    Q = device_tokens(q, q_off, dtype)
    D = device_tokens(d, d_off, dtype)
    n_q = len(q_off) - 1
    C = M.Candidates(dev(np.arange(n_q + 1, dtype=np.int64) * n_docs),
                     dev(np.tile(np.arange(n_docs, dtype=np.int32), n_q)))
    want = o1_scores(q, q_off, d, d_off, dtype)
    configs = [None]
    if dtype == "f32":
        configs = [(stage, pf, nw) for stage in (0, 1) for pf in (2, 3, 4) for nw in (4, 8)]
    try:
        for cfg in configs:
            if cfg is not None:
                _force_cfg(tmp_path, dtype, 128, *cfg)
                if _expected_lds(dtype, 128, *cfg, 16) > 160 * 1024:
                    with pytest.raises(M.MaxSimError):
                        M.score(Q, D)
                    continue
            dense = M.score(Q, D).cpu().numpy()
            per_doc = M.score(Q, D, C).cpu().numpy()
            assert np.array_equal(dense.view(np.uint32), per_doc.view(np.uint32)), cfg
            assert_close_o1(dense, want, f"{dtype} nd<={nd_max} {cfg}", dtype)
    finally:
        if dtype == "f32":
            _force_cfg(tmp_path, dtype, 128, 0, 2, 4)  # the built-in FP32 shape
        M.load_tune_cache(M.default_tune_cache())


@pytest.mark.parametrize("dtype", ["f32", "f16", "fp8"])
def test_unfused_comparator(dtype):
    q, q_off, d, d_off = _ragged(500, 128, seed=41, nq_lens=[32, 12], empty_every=97)
    Q = device_tokens(q, q_off, dtype)
    D = device_tokens(d, d_off, dtype)
    fused = M.score(Q, D).cpu().numpy()
    unf = M.score_unfused(Q, D).cpu().numpy()
    want = o1_scores(q, q_off, d, d_off, dtype)
    assert_close_o1(unf, want, "unfused", dtype)
    for a in range(2):
        f = fused[a * 500:(a + 1) * 500]
        u = unf[a * 500:(a + 1) * 500]
        assert set(np.argsort(-f, kind="stable")[:100]) == set(np.argsort(-u, kind="stable")[:100])


def test_query_capacity_is_enforced():
    q, q_off, d, d_off = _ragged(10, 128, seed=2, nq_lens=[65])
    with pytest.raises(M.MaxSimError):
        M.score(device_tokens(q, q_off, "f16"), device_tokens(d, d_off, "f16"))
    # a caller that understates max_len gets NaN scores, never an overrun
    Q = device_tokens(q, q_off, "f16", max_len=32)
    got = M.score(Q, device_tokens(d, d_off, "f16")).cpu().numpy()
    assert np.all(np.isnan(got))


@pytest.mark.parametrize("dtype,dim", [("f16", 128), ("fp8", 128), ("bf16", 256), ("f32", 128)])
def test_grouped_queries_share_document_reads(dtype, dim):
    # 13 queries of at most 16 tokens (one empty) against all documents: the
    # kernel scores up to 8 of them per document read (units of 8 + 5)
    nq_lens = [16, 1, 0, 9, 16, 3, 12, 16, 5, 16, 2, 7, 16]
    q, q_off, d, d_off = _ragged(140, dim, seed=dim + 71, nq_lens=nq_lens, empty_every=23)
    Q = device_tokens(q, q_off, dtype, max_len=16)
    D = device_tokens(d, d_off, dtype)
    got = M.score(Q, D).cpu().numpy()
    want = o1_scores(q, q_off, d, d_off, dtype)
    assert_close_o1(got, want, f"grouped {dtype} d={dim}", dtype)
    # each query alone gives the same bits as inside its unit
    for a in (0, 3, 12):
        Qa = device_tokens(q[q_off[a]:q_off[a + 1]], [0, nq_lens[a]], dtype, max_len=16)
        alone = M.score(Qa, D).cpu().numpy()
        assert np.array_equal(alone.view(np.uint32), got[a * 140:(a + 1) * 140].view(np.uint32)), a


@pytest.mark.parametrize("dtype", ["f16", "bf16", "fp8"])
def test_32_token_queries_share_document_reads(dtype):
    # 11 queries of at most 32 tokens at d = 128: units of 4 + 4 + 3 queries
    # (8 query blocks each; one empty query, ragged lengths)
    nq_lens = [32, 17, 0, 32, 5, 31, 32, 16, 1, 32, 24]
    q, q_off, d, d_off = _ragged(150, 128, seed=83, nq_lens=nq_lens, empty_every=19)
    Q = device_tokens(q, q_off, dtype, max_len=32)
    D = device_tokens(d, d_off, dtype)
    got = M.score(Q, D).cpu().numpy()
    want = o1_scores(q, q_off, d, d_off, dtype)
    assert_close_o1(got, want, f"four per unit {dtype}", dtype)
    for a in (0, 2, 7, 10):
        Qa = device_tokens(q[q_off[a]:q_off[a + 1]], [0, nq_lens[a]], dtype, max_len=32)
        alone = M.score(Qa, D).cpu().numpy()
        assert np.array_equal(alone.view(np.uint32), got[a * 150:(a + 1) * 150].view(np.uint32)), a


def test_understated_length_poisons_only_that_query():
    # max_len 16 but query 1 has 20 tokens: its scores are NaN, the others in
    # its unit are exact
    nq_lens = [16, 20, 5, 16]
    q, q_off, d, d_off = _ragged(60, 128, seed=77, nq_lens=nq_lens)
    Q = device_tokens(q, q_off, "f16", max_len=16)
    got = M.score(Q, device_tokens(d, d_off, "f16")).cpu().numpy().reshape(4, 60)
    assert np.all(np.isnan(got[1]))
    want = o1_scores(q, q_off, d, d_off, "f16").reshape(4, 60)
    for a in (0, 2, 3):
        assert_close_o1(got[a], want[a], f"query {a}", "f16")


# ----------------------------------------------------------------- top-k

@pytest.mark.parametrize("k", [1, 7, 100, 1024])
def test_topk_bit_exact(k):
    # the last segment has only 3 distinct scores: its boundary set of equal
    # scores overflows the compaction buffer and takes the exact radix path
    sizes = [0, 5, 100, 1000, 3, 70000, 130, 20000]
    distinct = [None, None, 40, None, None, None, 40, 3]
    off = W.offsets_from_lengths(sizes)
    parts = [W.random_scores(s, seed=i, n_distinct=distinct[i]) for i, s in enumerate(sizes)]
    s = np.concatenate(parts).astype(np.float32)
    s[off[1] + 1] = -np.inf
    s[off[1] + 3] = np.nan
    ids = W.rng(3).permutation(len(s)).astype(np.int32)
    for use_ids in (True, False):
        gs, gi = M.topk(dev(s), dev(off), k, ids=dev(ids) if use_ids else None)
        gs, gi = gs.cpu().numpy(), gi.cpu().numpy()
        for a in range(len(sizes)):
            seg = s[off[a]:off[a + 1]]
            sid = ids[off[a]:off[a + 1]].astype(np.int64) if use_ids else np.arange(len(seg))
            if np.isnan(seg).any():
                # brute force: finite and -inf by (score desc, id asc), NaN last
                order = sorted(range(len(seg)), key=lambda i: (bool(np.isnan(seg[i])),
                               0.0 if np.isnan(seg[i]) else -float(seg[i]), int(sid[i])))[:k]
                want_i = [int(sid[i]) for i in order] + [-1] * (k - len(order))
                assert gi[a].tolist() == want_i, a
                continue
            wi, ws = oracle.topk(seg.astype(np.float64), k, sid if use_ids else None)
            assert gi[a].tolist() == wi.tolist(), a
            assert np.array_equal(gs[a].astype(np.float64), ws), a


# ----------------------------------------------------------------- PQ

def _pq_case(n_docs, M_, K, dsub, seed, nq_lens, integer=False):
    g = W.rng(seed)
    lens = W.doc_lengths(n_docs, seed)
    lens[0] = 0
    d_off = W.offsets_from_lengths(lens)
    codes = g.integers(0, K, size=(int(d_off[-1]), M_), dtype=np.uint8)
    q_off = W.offsets_from_lengths(nq_lens)
    if integer:
        cb = g.integers(-4, 5, size=(M_, K, dsub)).astype(np.float16)
        q = g.integers(-3, 4, size=(int(q_off[-1]), M_ * dsub)).astype(np.float16)
    else:
        cb = (g.standard_normal((M_, K, dsub)) * 0.25).astype(np.float16)
        q = W.unit_tokens(int(q_off[-1]), M_ * dsub, g).astype(np.float16)
    return q, q_off, cb, codes, d_off


def _pq_device(q, q_off, cb, codes, d_off):
    Q = M.Tokens(dev(q), dev(q_off), "f16")
    D = M.PQDocs(dev(cb), dev(codes), dev(d_off))
    return Q, D


PQ_VARIANTS = ["table", "mfma"]


@pytest.fixture
def pq_variant(request, tmp_path):
    """Forces the PQ scorer (table kernel or decode-into-MFMA) for every key
    the test can touch; afterwards restores the automatic choice."""
    v = 0 if request.param == "table" else 1

    def write(variant):
        entries = [{"pq": 1, "M": m, "dsub": ds, "bpq": b, "cand": c, "variant": variant, "nqb": 0}
                   for m in (4, 8, 16) for ds in (4, 8, 16, 32) for b in (1, 2, 4) for c in (0, 1)]
        path = tmp_path / f"pq_{variant}.json"
        path.write_text(json.dumps({"version": 1, "entries": entries}))
        M.load_tune_cache(str(path))

    write(v)
    yield request.param
    write(1)  # variant 1 where it applies, else the table kernel: the default
    M.load_tune_cache(M.default_tune_cache())


@pytest.mark.parametrize("pq_variant", PQ_VARIANTS, indirect=True)
def test_pq_integer_table_is_bit_exact(pq_variant):
    # small integers: every product and sum is exact in FP32 on both kernels
    q, q_off, cb, codes, d_off = _pq_case(200, 8, 256, 16, seed=1, nq_lens=[32, 5], integer=True)
    Q, D = _pq_device(q, q_off, cb, codes, d_off)
    got = M.pq_score(Q, D).cpu().numpy()
    want = oracle.pq_decode_score(q.astype(np.float64), q_off, codes, cb.astype(np.float64), d_off)
    assert np.array_equal(got.astype(np.float64), want)


@pytest.mark.parametrize("pq_variant", PQ_VARIANTS, indirect=True)
@pytest.mark.parametrize("shape", [(8, 256, 16), (16, 256, 8), (4, 64, 32), (8, 256, 32),
                                   (16, 16, 4)])
def test_pq_matches_decode_then_score(pq_variant, shape):
    M_, K, dsub = shape
    q, q_off, cb, codes, d_off = _pq_case(300, M_, K, dsub, seed=M_ + K, nq_lens=[32, 64, 3])
    Q, D = _pq_device(q, q_off, cb, codes, d_off)
    got = M.pq_score(Q, D).cpu().numpy()
    want = oracle.pq_decode_score(q.astype(np.float64), q_off, codes, cb.astype(np.float64), d_off)
    assert_close_o1(got, want, f"pq {shape} {pq_variant}")


@pytest.mark.parametrize("pq_variant", PQ_VARIANTS, indirect=True)
def test_pq_many_queries_grouped(pq_variant):
    # 11 queries of uneven length (one empty) against ragged docs (one
    # empty): the decode kernel packs several queries per wave
    nq_lens = [32, 5, 0, 17, 32, 1, 30, 32, 8, 32, 31]
    q, q_off, cb, codes, d_off = _pq_case(260, 8, 256, 16, seed=23, nq_lens=nq_lens)
    Q, D = _pq_device(q, q_off, cb, codes, d_off)
    got = M.pq_score(Q, D).cpu().numpy()
    want = oracle.pq_decode_score(q.astype(np.float64), q_off, codes, cb.astype(np.float64), d_off)
    assert_close_o1(got, want, f"pq grouped {pq_variant}")


@pytest.mark.parametrize("pq_variant", PQ_VARIANTS, indirect=True)
def test_pq_candidates(pq_variant):
    q, q_off, cb, codes, d_off = _pq_case(500, 8, 256, 16, seed=7, nq_lens=[32, 16, 50])
    cand_off, cand_ids = W.candidates(3, 500, seed=8, size_range=(50, 400))
    Q, D = _pq_device(q, q_off, cb, codes, d_off)
    got = M.pq_score(Q, D, M.Candidates(dev(cand_off), dev(cand_ids))).cpu().numpy()
    want = oracle.pq_decode_score(q.astype(np.float64), q_off, codes, cb.astype(np.float64), d_off,
                                  cand_off, cand_ids)
    assert_close_o1(got, want, f"pq candidates {pq_variant}")


@pytest.mark.parametrize("pq_variant", PQ_VARIANTS, indirect=True)
@pytest.mark.parametrize("nd_max", [3, 40])
def test_pq_all_documents_equal_candidate_lists_of_all(pq_variant, nd_max):
    # Every document scored directly (queries grouped per work item) and as
    # a candidate list of all documents (one query per work item) give the
    # same bits, for short documents and empty ones too: each score's
    # products, maxima and sums run in the same order either way.
    g = W.rng(61 + nd_max)
    n_docs = 3000
    lens = g.integers(0, nd_max + 1, n_docs)
    lens[:5] = 0
    lens[-3:] = 0
    d_off = W.offsets_from_lengths(lens)
    codes = g.integers(0, 256, size=(int(d_off[-1]), 8), dtype=np.uint8)
    cb = (g.standard_normal((8, 256, 16)) * 0.25).astype(np.float16)
    q_off = W.offsets_from_lengths([32, 7, 0, 64, 20])
    q = W.unit_tokens(int(q_off[-1]), 128, g).astype(np.float16)
    Q, D = _pq_device(q, q_off, cb, codes, d_off)
    n_q = len(q_off) - 1
    dense = M.pq_score(Q, D).cpu().numpy()
    c_off = np.arange(n_q + 1, dtype=np.int64) * n_docs
    c_ids = np.tile(np.arange(n_docs, dtype=np.int32), n_q)
    per_doc = M.pq_score(Q, D, M.Candidates(dev(c_off), dev(c_ids))).cpu().numpy()
    assert np.array_equal(dense.view(np.uint32), per_doc.view(np.uint32))
    want = oracle.pq_decode_score(q.astype(np.float64), q_off, codes, cb.astype(np.float64), d_off)
    assert_close_o1(dense, want, f"pq packed nd<={nd_max}")


@pytest.mark.parametrize("q_dtype,cb_dtype", [("f32", "f16"), ("f16", "f32"), ("f32", "f32")])
def test_pq_fp32_queries_and_codebooks(q_dtype, cb_dtype):
    # FP32 inputs go through the table kernel (the decode kernel takes FP16)
    q, q_off, cb, codes, d_off = _pq_case(250, 8, 256, 16, seed=43, nq_lens=[32, 11, 64])
    qx = W.unit_tokens(len(q), 128, W.rng(45)) if q_dtype == "f32" else q
    cbx = (W.rng(44).standard_normal(cb.shape) * 0.25).astype(np.float32) if cb_dtype == "f32" else cb
    Q = M.Tokens(dev(qx), dev(q_off), q_dtype)
    D = M.PQDocs(dev(cbx), dev(codes), dev(d_off))
    got = M.pq_score(Q, D).cpu().numpy()
    want = oracle.pq_decode_score(qx.astype(np.float64), q_off, codes, cbx.astype(np.float64), d_off)
    assert_close_o1(got, want, f"pq q={q_dtype} cb={cb_dtype}")


def test_pq_autotune_keeps_results_within_tolerance(tmp_path):
    q, q_off, cb, codes, d_off = _pq_case(400, 8, 256, 16, seed=29, nq_lens=[32] * 9)
    Q, D = _pq_device(q, q_off, cb, codes, d_off)
    rep = M.pq_autotune(Q, D, reps=2)
    assert {t["variant"] for t in rep["trials"]} == {0, 1}, rep
    assert rep["best"]["ms"] > 0
    got = M.pq_score(Q, D).cpu().numpy()
    want = oracle.pq_decode_score(q.astype(np.float64), q_off, codes, cb.astype(np.float64), d_off)
    assert_close_o1(got, want, "pq after autotune")
    M.load_tune_cache(M.default_tune_cache())
