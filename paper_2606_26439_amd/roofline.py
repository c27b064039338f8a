"""Analytical byte / FLOP model of MaxSim scoring and the MI355X roofline.

Formulas restate the paper's roofline analysis:

* FLOPs            = B * Nq * Nd * (2d + 1)                      (Eq. flops, Sec. 2.3)
* IO_naive         = Nq*d*e + B*Nd*d*e + 2*B*Nq*Nd*4              (Eq. io_naive)
* IO_fused         = Nq*d*e + B*Nd*d*e + B*Nq*4                   (Eq. io_flash)
* IO(BQ)           = (Nq*d + ceil(Nq/BQ)*B*Nd*d)*e + B*4           (Theorem 1)
* PQ decompress    = B*Nd*(M + 2d) + 2*B*Nq*Nd*4                  (Sec. 4.4 table)
* PQ fused         = Nq*M*K*4 + B*Nd*M + B*Nq*4                   (Sec. 4.4 table)
* PQ table FLOPs   = Nq*M*K*2*dsub                                (Sec. 4.3, Phase 1)

The paper prints two forms of the output term: B*Nq*4 in Eq. io_flash and
its worked table, B*4 in Theorem 1. Both are provided; the measurement code
counts 4 bytes per (query, doc) score, the Theorem 1 form.

For ragged documents the per-document token count is summed instead of
B*Nd, and the measured kernels also read one int64 offset pair per document
(counted separately as index bytes).
"""
from __future__ import annotations

import math

# MI355X published peaks (dense, no sparsity).
HBM_PEAK_BPS = 8.0e12
PEAK_FLOPS = {
    "bf16": 2.5e15,
    "f16": 2.5e15,
    "fp8": 5.0e15,
    "f32": 157.3e12,
    "f64": 78.6e12,
}
ELEM_BYTES = {"f32": 4, "bf16": 2, "f16": 2, "fp8": 1}


def flops(B, Nq, Nd, d):
    """Eq. (flops): dot products plus one max comparison per (i, j) pair."""
    return B * Nq * Nd * (2 * d + 1)


def io_naive(B, Nq, Nd, d, e=2):
    """Eq. (io_naive): read Q, read D, write and read back the FP32 S matrix."""
    return Nq * d * e + B * Nd * d * e + 2 * B * Nq * Nd * 4


def io_fused(B, Nq, Nd, d, e=2):
    """Eq. (io_flash), with the B*Nq*4 output term the paper's table uses."""
    return Nq * d * e + B * Nd * d * e + B * Nq * 4


def io_theorem(B, Nq, Nd, d, BQ, e=2):
    """Theorem 1: D is read once per query block; output B*4 bytes."""
    return (Nq * d + math.ceil(Nq / BQ) * B * Nd * d) * e + B * 4


def arithmetic_intensity(flop, io):
    return flop / io


def pq_io_decompress(B, Nq, Nd, d, M):
    return B * Nd * (M + d * 2) + 2 * B * Nq * Nd * 4


def pq_io_fused(B, Nq, Nd, M, K):
    return Nq * M * K * 4 + B * Nd * M + B * Nq * 4


def pq_table_flops(Nq, M, K, dsub):
    return Nq * M * K * 2 * dsub


# ---------------------------------------------------------------------------
# Algorithmic bytes of the measured kernels (what "achieved GB/s" divides).
# ---------------------------------------------------------------------------

def fused_bytes(n_tokens, n_docs, n_pairs, nq_tokens_total, dim, dtype, with_index=True):
    """Bytes the fused scorer must move at minimum: each doc token once, each
    query token once, FP8 per-token scales, one FP32 score per (query, doc)
    pair and, for ragged CSR, one offset pair per scored document."""
    e = ELEM_BYTES[dtype]
    b = n_tokens * dim * e + nq_tokens_total * dim * e + 4 * n_pairs
    if dtype == "fp8":
        b += 4 * n_tokens + 4 * nq_tokens_total
    if with_index:
        b += 8 * (n_docs + 1)
    return b


def fused_topk_bytes(n_tokens, n_docs, n_queries, nq_tokens_total, dim, dtype, k):
    """Fused scoring with the top-k selected in the scorer: the same reads,
    but the output is k (score, id) pairs per query instead of one score per
    (query, doc) pair."""
    b = fused_bytes(n_tokens, n_docs, 0, nq_tokens_total, dim, dtype)
    return b + 8 * k * n_queries


def unfused_bytes(n_tokens, n_docs, n_pairs, nq, dim, dtype):
    """Fused bytes plus writing and reading back S [T, Nq] in FP32."""
    return fused_bytes(n_tokens, n_docs, n_pairs, nq, dim, dtype) + 2 * n_tokens * nq * 4


def pq_bytes(n_tokens, n_docs, n_queries, M, with_index=True):
    """Fused PQ: codes read once, one FP32 score per (query, doc)."""
    b = n_tokens * M + 4 * n_queries * n_docs
    if with_index:
        b += 8 * (n_docs + 1)
    return b
