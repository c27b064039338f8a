"""Shared helpers of the GPU tests (not collected by pytest)."""
import numpy as np
import torch

import oracle
import paper_2606_26439_amd as M

# Kernel-correctness gate against O1 (the exact values the GPU receives):
# FP32 accumulation of exact products, |gpu - O1| <= tol * max(|O1|, 1).
# The f8f6f4 MFMA adds each 32-byte block of products inside the matrix core
# at a precision below an IEEE FP32 add chain (measured up to 1.2e-5 relative
# per score, against <= 1.3e-7 for the other types), so FP8 is gated at 1e-4:
# still 600x inside the 6e-2 precision bound of the FP8 form.
REL_TOL = 1e-5
REL_TOL_DT = {"f32": 1e-5, "bf16": 1e-5, "f16": 1e-5, "fp8": 1e-4}
# Precision-form bounds against O2 (the FP32 values before rounding).
O2_TOL = {"f32": None, "bf16": 2e-2, "f16": 2e-2, "fp8": 6e-2}


def dev(x, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(x))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def device_tokens(x_f32, off, dtype, max_len=None):
    """Upload FP32 tokens and convert them on the device with the library's kernel."""
    x = dev(np.ascontiguousarray(x_f32, np.float32))
    tok, sc = M.quantize(x, dtype)
    return M.Tokens(tok, dev(np.asarray(off, np.int64)), dtype, sc, max_len)


def assert_close_o1(got, want, what="", dtype=None):
    got = np.asarray(got, np.float64)
    want = np.asarray(want, np.float64)
    assert got.shape == want.shape, (got.shape, want.shape)
    inf = ~np.isfinite(want)
    assert np.array_equal(got[inf], want[inf]), f"{what}: non-finite scores differ"
    g, w = got[~inf], want[~inf]
    if g.size:
        err = np.abs(g - w) / np.maximum(np.abs(w), 1.0)
        i = int(np.argmax(err))
        tol = REL_TOL_DT.get(dtype, REL_TOL)
        assert err[i] <= tol, f"{what}: max rel err {err[i]:.3e} at {i}: {g[i]} vs {w[i]}"


def o1_scores(q, q_off, d, d_off, dtype, cand_off=None, cand_ids=None):
    qv, _ = oracle.exact_values(q, dtype)
    dv, _ = oracle.exact_values(d, dtype)
    return oracle.maxsim(qv, q_off, dv, d_off, cand_off, cand_ids)


def gen_device_tokens(n_tokens, dim, dtype, seed, sample_rows=()):
    """Document tokens of `dtype` drawn on the device chunk by chunk (FP32 draw
    from the seeded generator, then the library's conversion), plus the FP32
    source rows `sample_rows` (sorted) for the oracle."""
    import workloads as W
    tok = torch.empty((n_tokens, dim), dtype=M._binding.TORCH_DTYPES[dtype], device="cuda")
    sc = torch.empty(n_tokens, dtype=torch.float32, device="cuda") if dtype == "fp8" else None
    rows = np.asarray(sample_rows, np.int64)
    keep = []
    for s, e, x in W.unit_tokens_gpu_chunks(n_tokens, dim, seed):
        t, c = M.quantize(x, dtype)
        tok[s:e] = t
        if sc is not None:
            sc[s:e] = c
        sel = rows[(rows >= s) & (rows < e)]
        if sel.size:
            keep.append(x[torch.from_numpy(sel - s).cuda()].cpu().numpy())
        del x, t, c
    torch.cuda.synchronize()
    f32 = np.concatenate(keep) if keep else np.zeros((0, dim), np.float32)
    return tok, sc, f32


def doc_rows(d_off, docs):
    """Token row indices of the given documents, and their CSR offsets."""
    docs = np.asarray(docs, np.int64)
    rows = np.concatenate([np.arange(d_off[b], d_off[b + 1]) for b in docs]) if docs.size \
        else np.zeros(0, np.int64)
    lens = d_off[docs + 1] - d_off[docs]
    off = np.zeros(len(docs) + 1, np.int64)
    np.cumsum(lens, out=off[1:])
    return rows, off


def assert_topk_matches_exact(got_ids, got_scores, exact_by_id, k, tol, what=""):
    """R19 (ii): the GPU's top-k ids equal the exact top-k, except that an entry
    may swap with one whose exact score is within `tol` of the exact k-th best
    (a near-tie the kernel's rounding may order either way)."""
    ex = sorted(exact_by_id.items(), key=lambda t: (-t[1], t[0]))
    exact_ids = [i for i, _ in ex[:k]]
    kth = ex[k - 1][1]
    got = [int(i) for i in got_ids[:k]]
    assert len(set(got)) == k, what
    for i in set(got) ^ set(exact_ids):
        assert i in exact_by_id, f"{what}: id {i} was not among the oracle's candidates"
        assert abs(exact_by_id[i] - kth) <= tol, \
            f"{what}: id {i} exact {exact_by_id[i]} vs k-th {kth}"
