"""FP64 CPU oracle for the TileMaxSim hot path (arXiv 2606.26439).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg may use this package; the GPU library never does. The C
source ``maxsim_oracle.c`` is compiled with gcc (``build()``) into
``liboracle.so`` and called through ctypes. Nothing here imports the GPU
package, and the GPU package imports nothing from here.

Each wrapper takes numpy arrays and returns numpy arrays; the definitions it
follows are stated in the C source:

* :func:`maxsim`            Eq. (1) over CSR token sets (optionally candidates).
* :func:`pq_decode`         the decompress step of the PQ pipeline (Sec. 4.1).
* :func:`pq_lut_build`      Phase 1 distance table T[i,m,k] (Sec. 4.3).
* :func:`pq_lut_score`      Phase 2 lookup-sum-max-sum (Sec. 4.3).
* :func:`pq_decode_score`   decompress-then-score: decode, then Eq. (1).
* :func:`residual_decode`   centroid + quantized residual decompression.
* :func:`residual_decode_score` decode, then Eq. (1).
* :func:`topk`              (score desc, id asc) selection.
* :func:`round_f16`, :func:`round_bf16`, :func:`round_e4m3`, :func:`quant_e4m3`
  and the matching ``decode_*``: round-to-nearest-even number formats.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "maxsim_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

_d = ctypes.POINTER(ctypes.c_double)
_f = ctypes.POINTER(ctypes.c_float)
_i64 = ctypes.POINTER(ctypes.c_int64)
_i32 = ctypes.POINTER(ctypes.c_int32)
_u8 = ctypes.POINTER(ctypes.c_uint8)
_u16 = ctypes.POINTER(ctypes.c_uint16)


def build() -> str:
    """Compile the oracle with gcc (strict IEEE: no -ffast-math, no FMA contraction)."""
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-ffp-contract=off",
           "-fno-fast-math", _SRC, "-o", _LIB_PATH + ".tmp", "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(_LIB_PATH + ".tmp", _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        build()
    lib = ctypes.CDLL(_LIB_PATH)
    lib.oracle_maxsim.argtypes = [_d, _i64, ctypes.c_int64, _d, _i64, ctypes.c_int64,
                                  ctypes.c_int32, _i64, _i32, _d]
    lib.oracle_maxsim.restype = ctypes.c_int
    lib.oracle_pq_decode.argtypes = [_u8, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32,
                                     ctypes.c_int32, _d, _d]
    lib.oracle_pq_decode.restype = ctypes.c_int
    lib.oracle_pq_lut_build.argtypes = [_d, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32,
                                        ctypes.c_int32, _d, _d]
    lib.oracle_pq_lut_build.restype = None
    lib.oracle_pq_lut_score.argtypes = [_d, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32,
                                        _u8, _i64, ctypes.c_int64, _i32, ctypes.c_int64, _d]
    lib.oracle_pq_lut_score.restype = ctypes.c_int
    lib.oracle_residual_decode.argtypes = [_i32, _u8, ctypes.c_int64, ctypes.c_int32,
                                           ctypes.c_int32, ctypes.c_int32, _d, _d, _d]
    lib.oracle_residual_decode.restype = ctypes.c_int
    lib.oracle_topk.argtypes = [_d, _i64, ctypes.c_int64, ctypes.c_int64, _i64, _d]
    lib.oracle_topk.restype = ctypes.c_int
    for name, bt in (("f16", _u16), ("bf16", _u16), ("e4m3", _u8)):
        fn = getattr(lib, "oracle_round_" + name)
        fn.argtypes = [_f, ctypes.c_int64, bt]
        fn.restype = None
        fn = getattr(lib, "oracle_decode_" + name)
        fn.argtypes = [bt, ctypes.c_int64, _d]
        fn.restype = None
    lib.oracle_quant_e4m3.argtypes = [_f, ctypes.c_int64, ctypes.c_int32, _u8, _f]
    lib.oracle_quant_e4m3.restype = None
    _lib = lib
    return lib


def _p(a, t):
    return a.ctypes.data_as(t) if a is not None else None


def _c(a, dtype):
    return None if a is None else np.ascontiguousarray(a, dtype=dtype)


def maxsim(q_tok, q_off, d_tok, d_off, cand_off=None, cand_ids=None) -> np.ndarray:
    """Eq. (1) in FP64. Returns [n_q * n_docs] (no candidates) or [cand_off[-1]]."""
    lib = _load()
    q_tok = _c(q_tok, np.float64)
    d_tok = _c(d_tok, np.float64)
    q_off = _c(q_off, np.int64)
    d_off = _c(d_off, np.int64)
    dim = q_tok.shape[1]
    assert d_tok.shape[1] == dim
    n_q, n_docs = len(q_off) - 1, len(d_off) - 1
    cand_off = _c(cand_off, np.int64)
    cand_ids = _c(cand_ids, np.int32)
    n_out = n_q * n_docs if cand_off is None else int(cand_off[-1])
    out = np.empty(max(n_out, 1), np.float64)
    rc = lib.oracle_maxsim(_p(q_tok, _d), _p(q_off, _i64), n_q, _p(d_tok, _d), _p(d_off, _i64),
                           n_docs, dim, _p(cand_off, _i64), _p(cand_ids, _i32), _p(out, _d))
    if rc != 0:
        raise ValueError("oracle_maxsim: candidate id out of range")
    return out[:n_out]


def pq_decode(codes, codebooks) -> np.ndarray:
    """codes [T, M] uint8, codebooks [M, K, dsub] -> decoded [T, M*dsub] FP64."""
    lib = _load()
    codes = _c(codes, np.uint8)
    cb = _c(codebooks, np.float64)
    M, K, dsub = cb.shape
    T = codes.shape[0]
    out = np.empty((max(T, 1), M * dsub), np.float64)
    if lib.oracle_pq_decode(_p(codes, _u8), T, M, K, dsub, _p(cb, _d), _p(out, _d)) != 0:
        raise ValueError("oracle_pq_decode: code out of range")
    return out[:T]


def pq_lut_build(q_tok, codebooks) -> np.ndarray:
    """Phase 1: T[i, m, k] for one query's tokens q_tok [nq, M*dsub]."""
    lib = _load()
    q = _c(q_tok, np.float64)
    cb = _c(codebooks, np.float64)
    M, K, dsub = cb.shape
    nq = q.shape[0]
    assert q.shape[1] == M * dsub
    out = np.empty((max(nq, 1), M, K), np.float64)
    lib.oracle_pq_lut_build(_p(q, _d), nq, M, K, dsub, _p(cb, _d), _p(out, _d))
    return out[:nq]


def pq_lut_score(table, codes, d_off, doc_sel=None) -> np.ndarray:
    """Phase 2 for one query: scores of docs doc_sel (default: all docs)."""
    lib = _load()
    table = _c(table, np.float64)
    nq, M, K = table.shape
    codes = _c(codes, np.uint8)
    d_off = _c(d_off, np.int64)
    n_docs = len(d_off) - 1
    doc_sel = _c(doc_sel, np.int32)
    n_sel = n_docs if doc_sel is None else len(doc_sel)
    out = np.empty(max(n_sel, 1), np.float64)
    rc = lib.oracle_pq_lut_score(_p(table, _d), nq, M, K, _p(codes, _u8), _p(d_off, _i64),
                                 n_docs, _p(doc_sel, _i32), n_sel, _p(out, _d))
    if rc != 0:
        raise ValueError("oracle_pq_lut_score: bad code or doc id")
    return out[:n_sel]


def pq_decode_score(q_tok, q_off, codes, codebooks, d_off, cand_off=None, cand_ids=None):
    """Decompress-then-score (Sec. 4.1): decode every doc token, then Eq. (1)."""
    dec = pq_decode(codes, codebooks)
    return maxsim(q_tok, q_off, dec, d_off, cand_off, cand_ids)


def residual_decode(ids, residuals, centroids, weights, nbits: int) -> np.ndarray:
    """ids [T] int32, residuals [T, dim*nbits/8] uint8 (packed codes),
    centroids [n_c, dim], weights [2**nbits] -> decoded [T, dim] FP64."""
    lib = _load()
    ids = _c(ids, np.int32)
    res = _c(residuals, np.uint8)
    cen = _c(centroids, np.float64)
    w = _c(weights, np.float64)
    n_c, dim = cen.shape
    assert nbits in (1, 2, 4, 8) and len(w) == 1 << nbits
    T = len(ids)
    assert res.shape == (T, dim * nbits // 8)
    out = np.empty((max(T, 1), dim), np.float64)
    rc = lib.oracle_residual_decode(_p(ids, _i32), _p(res, _u8), T, dim, nbits, n_c,
                                    _p(cen, _d), _p(w, _d), _p(out, _d))
    if rc != 0:
        raise ValueError("oracle_residual_decode: centroid id out of range")
    return out[:T]


def residual_decode_score(q_tok, q_off, ids, residuals, centroids, weights, nbits, d_off,
                          cand_off=None, cand_ids=None):
    """Decompress-then-score: decode every doc token, then Eq. (1)."""
    dec = residual_decode(ids, residuals, centroids, weights, nbits)
    return maxsim(q_tok, q_off, dec, d_off, cand_off, cand_ids)


def topk(scores, k, ids=None):
    """Returns (ids int64 [k], scores float64 [k]) ordered by (score desc, id asc)."""
    lib = _load()
    s = _c(scores, np.float64)
    ids = _c(ids, np.int64)
    n = len(s)
    out_ids = np.empty(max(k, 1), np.int64)
    out_s = np.empty(max(k, 1), np.float64)
    if lib.oracle_topk(_p(s, _d), _p(ids, _i64), n, k, _p(out_ids, _i64), _p(out_s, _d)) != 0:
        raise MemoryError("oracle_topk")
    return out_ids[:k], out_s[:k]


def _round(name, x, bits_dtype, ptr_t):
    lib = _load()
    x = np.ascontiguousarray(x, dtype=np.float32)
    out = np.empty(x.shape, bits_dtype)
    getattr(lib, "oracle_round_" + name)(_p(x, _f), x.size, _p(out, ptr_t))
    return out


def _decode(name, bits, bits_dtype, ptr_t):
    lib = _load()
    b = np.ascontiguousarray(bits, dtype=bits_dtype)
    out = np.empty(b.shape, np.float64)
    getattr(lib, "oracle_decode_" + name)(_p(b, ptr_t), b.size, _p(out, _d))
    return out


def round_f16(x):
    """FP32 -> binary16 bit patterns (uint16), round to nearest even."""
    return _round("f16", x, np.uint16, _u16)


def round_bf16(x):
    """FP32 -> bfloat16 bit patterns (uint16), round to nearest even."""
    return _round("bf16", x, np.uint16, _u16)


def round_e4m3(x):
    """FP32 -> OCP E4M3FN bit patterns (uint8), round to nearest even, saturating."""
    return _round("e4m3", x, np.uint8, _u8)


def decode_f16(bits):
    return _decode("f16", bits, np.uint16, _u16)


def decode_bf16(bits):
    return _decode("bf16", bits, np.uint16, _u16)


def decode_e4m3(bits):
    return _decode("e4m3", bits, np.uint8, _u8)


def quant_e4m3(x):
    """Per-token power-of-two scale + E4M3FN codes. x [T, d] FP32 -> (codes u8, scales f32)."""
    lib = _load()
    x = np.ascontiguousarray(x, dtype=np.float32)
    T, dim = x.shape
    codes = np.empty((T, dim), np.uint8)
    scales = np.empty(T, np.float32)
    lib.oracle_quant_e4m3(_p(x, _f), T, dim, _p(codes, _u8), _p(scales, _f))
    return codes, scales


def exact_values(x_f32, dtype: str):
    """The exact FP64 values a GPU receives after this oracle's rounding of x.

    dtype in {"f32", "bf16", "f16", "fp8"}; for fp8 the value is code * scale.
    Returns (values FP64 [T, d], encoded payload) where payload is the bit
    pattern array (and scales for fp8).
    """
    x = np.ascontiguousarray(x_f32, dtype=np.float32)
    if dtype == "f32":
        return x.astype(np.float64), (x,)
    if dtype == "f16":
        b = round_f16(x)
        return decode_f16(b), (b,)
    if dtype == "bf16":
        b = round_bf16(x)
        return decode_bf16(b), (b,)
    if dtype == "fp8":
        c, s = quant_e4m3(x)
        return decode_e4m3(c) * s.astype(np.float64)[:, None], (c, s)
    raise ValueError(dtype)
