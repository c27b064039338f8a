"""Seeded synthetic inputs with the shapes of the paper's workloads.

This module only draws random numbers and packs them; it holds none of the
method's arithmetic (no dot products, no maxima, no number-format rounding).
Both the GPU path's tests/benchmark and the FP64 oracle take their inputs from
here, and it imports neither.

Recipe (all tokens are i.i.d. N(0,1) vectors L2-normalised per token in FP64
and stored as FP32, the "synthetic normalised random data" of the paper's
evaluation):

* document lengths: Nd = rint(X), X ~ lognormal with arithmetic mean 70 and
  sigma 0.5 (so mu = ln 70 - sigma^2 / 2), clipped to [8, 180];
* PQ centroids: N(0, 1/16) (std 0.25) stored as FP16; codes uniform on
  [0, K) per (token, subspace);
* residual-compressed documents: centroids are unit-norm Gaussian vectors
  stored as FP16 (seed 5); each token's centroid id is uniform on
  [0, n_centroids) and each dimension's residual code uniform on
  [0, 2^nbits) (seed 6); the residual value of code c is
  0.02 * Phi^-1((c + 1/2) / 2^nbits), the centre of the c-th
  equal-probability bucket of N(0, 0.02^2), stored as FP16;
* serving: Poisson arrivals (exponential gaps), Nq uniform on {8..64},
  candidate-set size uniform on {1000..100000}, ids drawn without
  replacement from the pool.

CPU generators use numpy's PCG64; the GPU generators (``*_gpu``) use torch's
device generator seeded the same way, in fixed-size chunks, so a run is
reproducible on the same software stack.
"""
from __future__ import annotations

import math
from statistics import NormalDist

import numpy as np

LOGNORMAL_SIGMA = 0.5
LOGNORMAL_MEAN = 70.0
ND_MIN, ND_MAX = 8, 180


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def doc_lengths(n_docs: int, seed: int) -> np.ndarray:
    """Nd per document: rint(lognormal(arith. mean 70, sigma 0.5)) clipped to [8, 180]."""
    mu = math.log(LOGNORMAL_MEAN) - LOGNORMAL_SIGMA ** 2 / 2
    x = rng(seed).lognormal(mean=mu, sigma=LOGNORMAL_SIGMA, size=n_docs)
    return np.clip(np.rint(x), ND_MIN, ND_MAX).astype(np.int64)


def offsets_from_lengths(lengths) -> np.ndarray:
    off = np.zeros(len(lengths) + 1, np.int64)
    np.cumsum(np.asarray(lengths, np.int64), out=off[1:])
    return off


def normalise_rows(x: np.ndarray) -> np.ndarray:
    """Per-token L2 normalisation in FP64, stored as FP32 (input preparation)."""
    x = np.asarray(x, np.float64)
    n = np.sqrt((x * x).sum(axis=1, keepdims=True))
    n[n == 0] = 1.0
    return (x / n).astype(np.float32)


def unit_tokens(n: int, dim: int, gen: np.random.Generator) -> np.ndarray:
    return normalise_rows(gen.standard_normal((n, dim)))


def plain_fp32_case(seed: int = 0, nq: int = 32, dim: int = 128, n_docs: int = 4096,
                    nd: int = 32):
    """Plain FP32 parity workload: one query, fixed-length docs, one seed.

    Q is drawn first, then all document tokens, from the same generator.
    Returns dict(q [nq, dim] f32, q_off, d [n_docs*nd, dim] f32, d_off).
    """
    g = rng(seed)
    q = unit_tokens(nq, dim, g)
    d = unit_tokens(n_docs * nd, dim, g)
    return dict(q=q, q_off=np.array([0, nq], np.int64), d=d,
                d_off=offsets_from_lengths(np.full(n_docs, nd, np.int64)))


def ragged_case(n_docs: int, dim: int = 128, nq: int = 32, seed_docs: int = 0,
                seed_query: int = 1, n_queries: int = 1, nq_range=None, lengths=None):
    """Ragged lognormal-length docs and one or more queries, all on the CPU.

    nq_range=(lo, hi) draws each query's token count uniformly on {lo..hi}.
    """
    lens = doc_lengths(n_docs, seed_docs) if lengths is None else np.asarray(lengths, np.int64)
    d_off = offsets_from_lengths(lens)
    gd = rng(seed_docs + 1000)
    d = unit_tokens(int(d_off[-1]), dim, gd)
    gq = rng(seed_query)
    if nq_range is None:
        qlens = np.full(n_queries, nq, np.int64)
    else:
        qlens = gq.integers(nq_range[0], nq_range[1] + 1, size=n_queries).astype(np.int64)
    q_off = offsets_from_lengths(qlens)
    q = unit_tokens(int(q_off[-1]), dim, gq)
    return dict(q=q, q_off=q_off, d=d, d_off=d_off)


def candidates(n_queries: int, n_pool: int, seed: int, size_range=(1000, 100000)):
    """Per-query candidate ids drawn uniformly without replacement.

    Returns (cand_off int64 [n_queries+1], cand_ids int32 [total]).
    """
    g = rng(seed)
    lo, hi = size_range
    hi = min(hi, n_pool)
    lo = min(lo, hi)
    sizes = g.integers(lo, hi + 1, size=n_queries).astype(np.int64)
    ids = [g.choice(n_pool, size=int(s), replace=False).astype(np.int32) for s in sizes]
    return offsets_from_lengths(sizes), (np.concatenate(ids) if ids else np.zeros(0, np.int32))


def pq_codebooks(M: int = 8, K: int = 256, dsub: int = 16, seed: int = 2) -> np.ndarray:
    """Centroids C[M, K, dsub] ~ N(0, 1/16), stored as FP16."""
    return (rng(seed).standard_normal((M, K, dsub)) * 0.25).astype(np.float16)


def pq_codes(n_tokens: int, M: int = 8, K: int = 256, seed: int = 2) -> np.ndarray:
    """Codes uniform on [0, K) per (token, subspace), uint8 [n_tokens, M]."""
    return rng(seed + 7).integers(0, K, size=(n_tokens, M), dtype=np.uint8)


RESIDUAL_SIGMA = 0.02


def residual_centroids(n_centroids: int, dim: int = 128, seed: int = 5) -> np.ndarray:
    """Centroids [n_centroids, dim]: unit-norm Gaussian rows stored as FP16."""
    return unit_tokens(n_centroids, dim, rng(seed)).astype(np.float16)


def residual_weights(nbits: int) -> np.ndarray:
    """Residual value of each code: bucket centres of N(0, RESIDUAL_SIGMA^2), FP16."""
    n = 1 << nbits
    nd = NormalDist(0.0, RESIDUAL_SIGMA)
    return np.array([nd.inv_cdf((c + 0.5) / n) for c in range(n)]).astype(np.float16)


def residual_ids(n_tokens: int, n_centroids: int, seed: int = 6) -> np.ndarray:
    """Centroid id per token, uniform on [0, n_centroids), int32."""
    return rng(seed).integers(0, n_centroids, size=n_tokens, dtype=np.int64).astype(np.int32)


def residual_codes(n_tokens: int, dim: int, nbits: int, seed: int = 6) -> np.ndarray:
    """Packed residual codes [n_tokens, dim*nbits/8] uint8: uniform bytes, so
    every nbits-wide field is uniform on [0, 2^nbits)."""
    return rng(seed + 11).integers(0, 256, size=(n_tokens, dim * nbits // 8), dtype=np.uint8)


def poisson_arrivals(n: int, qps: float, seed: int = 3) -> np.ndarray:
    """Arrival times (s) of an open-loop Poisson process at rate qps."""
    return np.cumsum(rng(seed).exponential(1.0 / qps, size=n))


def dyadic_unit_vectors(n: int, dim: int, seed: int, nnz: int = 64) -> np.ndarray:
    """Vectors with nnz entries of +-1/8 and zeros elsewhere: ||v||^2 = nnz/64.

    With nnz = 64 they are exactly unit length, and every entry is exactly
    representable in FP32, BF16, FP16 and (with a power-of-two scale) FP8.
    """
    g = rng(seed)
    out = np.zeros((n, dim), np.float32)
    for r in range(n):
        cols = g.choice(dim, size=nnz, replace=False)
        out[r, cols] = np.where(g.integers(0, 2, size=nnz) == 1, 0.125, -0.125)
    return out


def random_scores(n: int, seed: int, n_distinct=None) -> np.ndarray:
    """FP32 score arrays for top-k tests; n_distinct forces many exact ties."""
    g = rng(seed)
    if n_distinct is None:
        return (g.standard_normal(n) * 0.5 + 6.5).astype(np.float32)
    vals = (g.standard_normal(n_distinct) * 0.5 + 6.5).astype(np.float32)
    return vals[g.integers(0, n_distinct, size=n)]


# --------------------------------------------------------------------------
# GPU generators (torch device RNG), for workloads too large to draw on a CPU.
# --------------------------------------------------------------------------

GPU_CHUNK_TOKENS = 1 << 22


def unit_tokens_gpu(n: int, dim: int, seed: int, device="cuda", out=None):
    """n unit-norm Gaussian FP32 tokens on the device, drawn in fixed chunks."""
    import torch
    g = torch.Generator(device=device)
    g.manual_seed(seed)
    if out is None:
        out = torch.empty((n, dim), dtype=torch.float32, device=device)
    for s in range(0, n, GPU_CHUNK_TOKENS):
        e = min(n, s + GPU_CHUNK_TOKENS)
        x = torch.randn((e - s, dim), generator=g, device=device, dtype=torch.float64)
        x /= x.norm(dim=1, keepdim=True).clamp_min(1e-300)
        out[s:e] = x.to(torch.float32)
        del x
    return out


def unit_tokens_gpu_chunks(n: int, dim: int, seed: int, device="cuda"):
    """Yields (start, end, FP32 chunk) covering n unit-norm tokens, drawn in the
    same order and chunking as unit_tokens_gpu (so the values are identical)."""
    import torch
    g = torch.Generator(device=device)
    g.manual_seed(seed)
    for s in range(0, n, GPU_CHUNK_TOKENS):
        e = min(n, s + GPU_CHUNK_TOKENS)
        x = torch.randn((e - s, dim), generator=g, device=device, dtype=torch.float64)
        x /= x.norm(dim=1, keepdim=True).clamp_min(1e-300)
        yield s, e, x.to(torch.float32)
        del x


def pq_codes_gpu(n_tokens: int, M: int, K: int, seed: int, device="cuda"):
    import torch
    g = torch.Generator(device=device)
    g.manual_seed(seed)
    out = torch.empty((n_tokens, M), dtype=torch.uint8, device=device)
    step = GPU_CHUNK_TOKENS * 4
    for s in range(0, n_tokens, step):
        e = min(n_tokens, s + step)
        out[s:e] = torch.randint(0, K, (e - s, M), generator=g, device=device,
                                 dtype=torch.int32).to(torch.uint8)
    return out


def residual_ids_gpu(n_tokens: int, n_centroids: int, seed: int, device="cuda"):
    import torch
    g = torch.Generator(device=device)
    g.manual_seed(seed)
    out = torch.empty(n_tokens, dtype=torch.int32, device=device)
    step = GPU_CHUNK_TOKENS * 4
    for s in range(0, n_tokens, step):
        e = min(n_tokens, s + step)
        out[s:e] = torch.randint(0, n_centroids, (e - s,), generator=g, device=device,
                                 dtype=torch.int32)
    return out


def residual_codes_gpu(n_tokens: int, dim: int, nbits: int, seed: int, device="cuda"):
    import torch
    g = torch.Generator(device=device)
    g.manual_seed(seed + 11)
    rb = dim * nbits // 8
    out = torch.empty((n_tokens, rb), dtype=torch.uint8, device=device)
    step = GPU_CHUNK_TOKENS
    for s in range(0, n_tokens, step):
        e = min(n_tokens, s + step)
        out[s:e] = torch.randint(0, 256, (e - s, rb), generator=g, device=device,
                                 dtype=torch.int32).to(torch.uint8)
    return out
