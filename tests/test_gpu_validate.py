"""Device-side input checks (maxsim_validate / maxsim_validate_pq /
maxsim_check): clean inputs pass, and each planted violation is reported by
name. The corrupted inputs go only to the checking kernels, which read
nothing beyond the declared array sizes."""
import numpy as np
import pytest
import torch

import paper_2606_26439_amd as M
import workloads as W
from tests._gpu import dev, device_tokens

pytestmark = pytest.mark.gpu

EDEVCHECK = 5


def _case(dtype="f16", n_docs=300, nq_lens=(32, 7, 20)):
    lens = W.doc_lengths(n_docs, 3)
    lens[4] = 0
    d_off = W.offsets_from_lengths(lens)
    g = W.rng(4)
    d = W.unit_tokens(int(d_off[-1]), 128, g)
    q_off = W.offsets_from_lengths(list(nq_lens))
    q = W.unit_tokens(int(q_off[-1]), 128, g)
    cand_off, cand_ids = W.candidates(len(nq_lens), n_docs, seed=5, size_range=(20, 200))
    return (device_tokens(q, q_off, dtype, max_len=max(nq_lens)),
            device_tokens(d, d_off, dtype), M.Candidates(dev(cand_off), dev(cand_ids)),
            d_off, cand_off, cand_ids)


def _expect(what, fn):
    with pytest.raises(M.MaxSimError) as ei:
        fn()
    assert ei.value.status == EDEVCHECK, str(ei.value)
    assert what in str(ei.value), str(ei.value)


@pytest.mark.parametrize("dtype", ["f32", "bf16", "f16", "fp8"])
def test_clean_inputs_pass(dtype):
    Q, D, C, *_ = _case(dtype)
    M.validate(D)
    M.validate(D, Q)
    M.validate(D, Q, C)


def test_each_violation_is_named():
    Q, D, C, d_off, cand_off, cand_ids = _case()
    bad = d_off.copy()
    bad[10] = bad[11] + 1  # decreasing
    _expect("document offsets", lambda: M.validate(M.Tokens(D.tokens, dev(bad), "f16", None, 180)))
    bad = d_off.copy()
    bad[-1] -= 1  # last offset != n_tokens
    _expect("document offsets", lambda: M.validate(M.Tokens(D.tokens, dev(bad), "f16", None, 180)))
    short = M.Tokens(Q.tokens, Q.offsets, "f16", None, max_len=16)  # a 32-token query
    _expect("query longer than max_len", lambda: M.validate(D, short))
    ids = cand_ids.copy()
    ids[3] = D.n_sets  # one past the last document
    _expect("candidate ids", lambda: M.validate(D, Q, M.Candidates(dev(cand_off), dev(ids))))
    ids[3] = -1
    _expect("candidate ids", lambda: M.validate(D, Q, M.Candidates(dev(cand_off), dev(ids))))
    co = cand_off.copy()
    co[1] = co[2] + 1
    _expect("candidate offsets", lambda: M.validate(D, Q, M.Candidates(dev(co), dev(cand_ids))))


def test_fp8_scale_must_be_a_power_of_two():
    Q, D, *_ = _case("fp8")
    sc = D.scales.clone()
    sc[7] *= 1.5
    _expect("FP8 scales", lambda: M.validate(M.Tokens(D.tokens, D.offsets, "fp8", sc, 180)))
    sc = D.scales.clone()
    sc[9] = 0.0
    _expect("FP8 scales", lambda: M.validate(M.Tokens(D.tokens, D.offsets, "fp8", sc, 180)))


def test_pq_codes_below_k():
    lens = W.doc_lengths(200, 6)
    d_off = W.offsets_from_lengths(lens)
    codes = W.pq_codes(int(d_off[-1]), 8, 64, seed=6)
    cb = W.pq_codebooks(8, 64, 16, seed=6)
    D = M.PQDocs(dev(cb), dev(codes), dev(d_off))
    M.validate(D)
    codes[123, 5] = 64
    _expect("PQ codes", lambda: M.validate(M.PQDocs(dev(cb), dev(codes), dev(d_off))))
