"""GPU parity over the whole dimension range of the C ABI: d % 16 == 0,
16 <= d <= 1024 (Alg. 1 takes any Q in R^{Nq x d}). Widths that are not a
multiple of the kernel's d-chunk are zero-extended inside the kernel, which
adds exact zeros, so the scores also equal, bit for bit, those of the rows
zero-padded on the host to whole chunks."""
import numpy as np
import pytest

import oracle
import paper_2606_26439_amd as M
import workloads as W
from tests._gpu import assert_close_o1, dev, device_tokens, o1_scores

pytestmark = pytest.mark.gpu

DTYPES = ["f32", "bf16", "f16", "fp8"]
DIMS = [16, 32, 48, 96, 160, 400]


def _case(n_docs, dim, seed, nq_lens, empty_every=0):
    lens = W.doc_lengths(n_docs, seed)
    if empty_every:
        lens[::empty_every] = 0
    lens[1], lens[2] = 1, 17
    d_off = W.offsets_from_lengths(lens)
    g = W.rng(seed + 1)
    d = W.unit_tokens(int(d_off[-1]), dim, g)
    q_off = W.offsets_from_lengths(nq_lens)
    q = W.unit_tokens(int(q_off[-1]), dim, g)
    return q, q_off, d, d_off


def _padded_width(dim):
    """The width the kernel zero-extends d to (whole chunks)."""
    if dim <= 64:
        return 64
    if dim <= 128:
        return 128
    return -(-dim // 64) * 64 if dim % 128 else dim


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("dim", DIMS)
def test_quantize_bit_exact_any_width(dtype, dim):
    x = W.unit_tokens(301, dim, W.rng(dim + 1))
    x[3] = 0.0
    x[4] *= 500.0
    tok, sc = M.quantize(dev(x), dtype)
    _, payload = oracle.exact_values(x, dtype)
    if dtype == "f32":
        assert np.array_equal(tok.cpu().numpy().view(np.uint32), x.view(np.uint32))
    elif dtype in ("bf16", "f16"):
        import torch
        got = tok.view(torch.int16).cpu().numpy().view(np.uint16)
        assert np.array_equal(got, payload[0])
    else:
        assert np.array_equal(tok.cpu().numpy(), payload[0])
        assert np.array_equal(sc.cpu().numpy(), payload[1])


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("dim", DIMS)
def test_fused_any_width_all_docs_and_candidates(dtype, dim):
    q, q_off, d, d_off = _case(130, dim, seed=dim + 7, nq_lens=[32, 5, 64, 17], empty_every=41)
    Q = device_tokens(q, q_off, dtype)
    D = device_tokens(d, d_off, dtype)
    got = M.score(Q, D).cpu().numpy()
    assert_close_o1(got, o1_scores(q, q_off, d, d_off, dtype), f"{dtype} d={dim}", dtype)
    # candidate lists (one query with none, a repeated id)
    cand_off, cand_ids = W.candidates(4, 130, seed=dim, size_range=(5, 90))
    ids = [cand_ids[cand_off[a]:cand_off[a + 1]] for a in range(4)]
    ids[2] = ids[2][:0]
    ids[0] = np.concatenate([ids[0], ids[0][:2]])
    cand_ids = np.concatenate(ids).astype(np.int32)
    cand_off = W.offsets_from_lengths([len(x) for x in ids])
    C = M.Candidates(dev(cand_off), dev(cand_ids))
    gotc = M.score(Q, D, C).cpu().numpy()
    want = o1_scores(q, q_off, d, d_off, dtype, cand_off, cand_ids)
    assert_close_o1(gotc, want, f"{dtype} d={dim} candidates", dtype)


@pytest.mark.parametrize("dtype", ["f32", "bf16", "fp8"])
@pytest.mark.parametrize("dim", DIMS)
def test_in_kernel_zero_extension_equals_host_padding(dtype, dim):
    q, q_off, d, d_off = _case(70, dim, seed=dim + 13, nq_lens=[32, 9])
    pw = _padded_width(dim)
    a = M.score(device_tokens(q, q_off, dtype), device_tokens(d, d_off, dtype)).cpu().numpy()
    qz = np.concatenate([q, np.zeros((len(q), pw - dim), np.float32)], axis=1)
    dz = np.concatenate([d, np.zeros((len(d), pw - dim), np.float32)], axis=1)
    b = M.score(device_tokens(qz, q_off, dtype), device_tokens(dz, d_off, dtype)).cpu().numpy()
    assert np.array_equal(a, b)


@pytest.mark.parametrize("dtype", ["f32", "f16", "fp8"])
@pytest.mark.parametrize("dim", [16, 96, 400])
def test_unfused_any_width(dtype, dim):
    q, q_off, d, d_off = _case(90, dim, seed=dim + 19, nq_lens=[32, 12], empty_every=29)
    Q = device_tokens(q, q_off, dtype)
    D = device_tokens(d, d_off, dtype)
    unf = M.score_unfused(Q, D).cpu().numpy()
    assert_close_o1(unf, o1_scores(q, q_off, d, d_off, dtype), f"unfused {dtype} d={dim}", dtype)
