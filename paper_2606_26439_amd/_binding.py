"""ctypes binding of libmaxsim.so (include/maxsim.h): argument marshalling only.

PyTorch supplies device memory and the current HIP stream; every step of the
scoring path runs in the library's own HIP kernels. There is no fallback: if
the library is missing every call raises.
"""
from __future__ import annotations

import ctypes
import json
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmaxsim.so")

DTYPES = {"f32": 0, "bf16": 1, "f16": 2, "fp8": 3}
TORCH_DTYPES = {"f32": torch.float32, "bf16": torch.bfloat16, "f16": torch.float16,
                "fp8": torch.uint8}
ELEM_BYTES = {"f32": 4, "bf16": 2, "f16": 2, "fp8": 1}
STATUS = {0: "OK", 1: "EINVAL", 2: "EUNSUPPORTED", 3: "EWORKSPACE", 4: "EHIP"}


class MaxSimError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class CSR(ctypes.Structure):
    _fields_ = [("dtype", ctypes.c_int32), ("dim", ctypes.c_int32), ("n_sets", ctypes.c_int64),
                ("n_tokens", ctypes.c_int64), ("max_len", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("tokens", ctypes.c_void_p),
                ("offsets", ctypes.c_void_p), ("scales", ctypes.c_void_p)]


class Cand(ctypes.Structure):
    _fields_ = [("offsets", ctypes.c_void_p), ("doc_ids", ctypes.c_void_p),
                ("n_total", ctypes.c_int64)]


class PQ(ctypes.Structure):
    _fields_ = [("M", ctypes.c_int32), ("K", ctypes.c_int32), ("dsub", ctypes.c_int32),
                ("cb_dtype", ctypes.c_int32), ("codebooks", ctypes.c_void_p),
                ("codes", ctypes.c_void_p), ("offsets", ctypes.c_void_p),
                ("n_docs", ctypes.c_int64), ("n_tokens", ctypes.c_int64)]


class Residual(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int32), ("nbits", ctypes.c_int32),
                ("n_centroids", ctypes.c_int64), ("centroids", ctypes.c_void_p),
                ("weights", ctypes.c_void_p), ("centroid_ids", ctypes.c_void_p),
                ("residuals", ctypes.c_void_p), ("offsets", ctypes.c_void_p),
                ("n_docs", ctypes.c_int64), ("n_tokens", ctypes.c_int64)]


_lib = None
_P = ctypes.POINTER
_vp = ctypes.c_void_p


def lib():
    """The loaded library (loads on first use; torch is imported first so the
    library binds to the HIP runtime torch already loaded)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built; run __graft_entry__.build() "
                           "(or python -m paper_2606_26439_amd.build)")
    L = ctypes.CDLL(LIB_PATH)
    L.maxsim_abi_version.restype = ctypes.c_int
    L.maxsim_last_error.restype = ctypes.c_char_p
    L.maxsim_quantize.argtypes = [_vp, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32, _vp, _vp,
                                  _vp]
    L.maxsim_score_workspace_size.argtypes = [_P(CSR), _P(CSR), _P(Cand)]
    L.maxsim_score_workspace_size.restype = ctypes.c_size_t
    L.maxsim_score.argtypes = [_P(CSR), _P(CSR), _P(Cand), _vp, _vp, ctypes.c_size_t, _vp]
    L.maxsim_score_topk_workspace_size.argtypes = [_P(CSR), _P(CSR), _P(Cand), ctypes.c_int32]
    L.maxsim_score_topk_workspace_size.restype = ctypes.c_size_t
    L.maxsim_score_topk.argtypes = [_P(CSR), _P(CSR), _P(Cand), ctypes.c_int32, _vp, _vp, _vp,
                                    ctypes.c_size_t, _vp]
    L.maxsim_score_topk_noalloc.argtypes = [_P(CSR), _P(CSR), _P(Cand), ctypes.c_int32, _vp,
                                            _vp, _vp]
    L.maxsim_score_unfused_workspace_size.argtypes = [_P(CSR), _P(CSR)]
    L.maxsim_score_unfused_workspace_size.restype = ctypes.c_size_t
    L.maxsim_score_unfused.argtypes = [_P(CSR), _P(CSR), _vp, _vp, ctypes.c_size_t, _vp]
    L.maxsim_pq_score_workspace_size.argtypes = [_P(CSR), _P(PQ), _P(Cand)]
    L.maxsim_pq_score_workspace_size.restype = ctypes.c_size_t
    L.maxsim_pq_score.argtypes = [_P(CSR), _P(PQ), _P(Cand), _vp, _vp, ctypes.c_size_t, _vp]
    L.maxsim_residual_score_workspace_size.argtypes = [_P(CSR), _P(Residual), _P(Cand)]
    L.maxsim_residual_score_workspace_size.restype = ctypes.c_size_t
    L.maxsim_residual_score.argtypes = [_P(CSR), _P(Residual), _P(Cand), _vp, _vp,
                                        ctypes.c_size_t, _vp]
    L.maxsim_topk_workspace_size.argtypes = [ctypes.c_int64, ctypes.c_int32]
    L.maxsim_topk_workspace_size.restype = ctypes.c_size_t
    L.maxsim_topk.argtypes = [_vp, _vp, ctypes.c_int64, ctypes.c_int64, _vp, ctypes.c_int32, _vp,
                              _vp, _vp, ctypes.c_size_t, _vp]
    L.maxsim_autotune.argtypes = [_P(CSR), _P(CSR), _P(Cand), _vp, _vp, ctypes.c_size_t, _vp,
                                  ctypes.c_int32, ctypes.c_char_p, ctypes.c_char_p,
                                  ctypes.c_size_t]
    L.maxsim_pq_autotune.argtypes = [_P(CSR), _P(PQ), _P(Cand), _vp, _vp, ctypes.c_size_t, _vp,
                                     ctypes.c_int32, ctypes.c_char_p, ctypes.c_char_p,
                                     ctypes.c_size_t]
    L.maxsim_residual_autotune.argtypes = [_P(CSR), _P(Residual), _P(Cand), _vp, _vp,
                                           ctypes.c_size_t, _vp, ctypes.c_int32, ctypes.c_char_p,
                                           ctypes.c_char_p, ctypes.c_size_t]
    L.maxsim_validate.argtypes = [_P(CSR), _P(CSR), _P(Cand), _vp, _vp]
    L.maxsim_validate_pq.argtypes = [_P(CSR), _P(PQ), _P(Cand), _vp, _vp]
    L.maxsim_validate_residual.argtypes = [_P(CSR), _P(Residual), _P(Cand), _vp, _vp]
    L.maxsim_check.argtypes = [_vp, _vp]
    L.maxsim_load_tune_cache.argtypes = [ctypes.c_char_p]
    L.maxsim_stream_probe.argtypes = [_vp, ctypes.c_size_t, ctypes.c_int32, _vp, ctypes.c_int64,
                                      _vp]
    L.maxsim_lds_probe.argtypes = [_vp, ctypes.c_size_t, ctypes.c_int32, ctypes.c_int32, _vp,
                                   ctypes.c_int64, _vp]
    for name in ("maxsim_quantize", "maxsim_score", "maxsim_score_topk",
                 "maxsim_score_topk_noalloc", "maxsim_score_unfused",
                 "maxsim_pq_score",
                 "maxsim_topk", "maxsim_autotune", "maxsim_pq_autotune",
                 "maxsim_load_tune_cache", "maxsim_stream_probe", "maxsim_lds_probe",
                 "maxsim_validate",
                 "maxsim_validate_pq", "maxsim_check", "maxsim_residual_score",
                 "maxsim_validate_residual", "maxsim_residual_autotune"):
        getattr(L, name).restype = ctypes.c_int
    _lib = L
    # launch shapes tuned on an MI355X for the shipped key set (missing: defaults)
    tuned = default_tune_cache()
    if os.path.exists(tuned):
        L.maxsim_load_tune_cache(tuned.encode())
    return L


def default_tune_cache() -> str:
    """The tune cache loaded with the library: $MAXSIM_TUNE_CACHE, else the
    packaged tuned.json."""
    return os.environ.get("MAXSIM_TUNE_CACHE", os.path.join(_HERE, "tuned.json"))


def _check(st: int):
    if st != 0:
        raise MaxSimError(st, lib().maxsim_last_error().decode())


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(stream=None):
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


class Tokens:
    """A CSR set of token-vector sets on the device (documents or queries).

    tokens  [n_tokens, dim] tensor of the element type (uint8 codes for fp8)
    offsets [n_sets + 1] int64 tensor
    scales  [n_tokens] float32 (fp8 only)
    max_len host upper bound on tokens per set (computed if None; queries need it)
    """

    def __init__(self, tokens, offsets, dtype: str, scales=None, max_len=None):
        if dtype not in DTYPES:
            raise ValueError(f"dtype must be one of {list(DTYPES)}")
        self.tokens, self.offsets, self.scales, self.dtype = tokens, offsets, scales, dtype
        self.dim = int(tokens.shape[1])
        self.n_sets = int(offsets.numel()) - 1
        self.n_tokens = int(tokens.shape[0])
        if max_len is None:
            max_len = int((offsets[1:] - offsets[:-1]).max().item()) if self.n_sets > 0 else 0
        self.max_len = int(max_len)

    def csr(self) -> CSR:
        return CSR(DTYPES[self.dtype], self.dim, self.n_sets, self.n_tokens, self.max_len, 0,
                   self.tokens.data_ptr() if self.n_tokens else None, self.offsets.data_ptr(),
                   self.scales.data_ptr() if self.scales is not None else None)


class Candidates:
    """Per-query candidate lists: offsets [n_queries + 1] int64, doc_ids int32."""

    def __init__(self, offsets, doc_ids):
        self.offsets, self.doc_ids = offsets, doc_ids
        self.n_total = int(doc_ids.numel())

    def c(self) -> Cand:
        return Cand(self.offsets.data_ptr(), self.doc_ids.data_ptr() if self.n_total else None,
                    self.n_total)


class PQDocs:
    """PQ-compressed documents: codebooks [M, K, dsub] (f16/f32), codes [T, M] uint8."""

    def __init__(self, codebooks, codes, offsets):
        self.codebooks, self.codes, self.offsets = codebooks, codes, offsets
        self.M, self.K, self.dsub = (int(x) for x in codebooks.shape)
        self.n_docs = int(offsets.numel()) - 1
        self.n_tokens = int(codes.shape[0])
        self.cb_dtype = {torch.float16: DTYPES["f16"], torch.float32: DTYPES["f32"]}[codebooks.dtype]

    def pq(self) -> PQ:
        return PQ(self.M, self.K, self.dsub, self.cb_dtype, self.codebooks.data_ptr(),
                  self.codes.data_ptr() if self.n_tokens else None, self.offsets.data_ptr(),
                  self.n_docs, self.n_tokens)


class ResidualDocs:
    """Residual-compressed documents: centroids [n_c, dim] f16, weights
    [2**nbits] f16, centroid_ids [T] int32, residuals [T, dim*nbits/8] uint8
    (packed codes, low bits first), offsets [n_docs + 1] int64."""

    def __init__(self, centroids, weights, centroid_ids, residuals, offsets, nbits: int):
        self.centroids, self.weights = centroids, weights
        self.centroid_ids, self.residuals, self.offsets = centroid_ids, residuals, offsets
        self.nbits = int(nbits)
        self.n_centroids, self.dim = (int(x) for x in centroids.shape)
        self.n_docs = int(offsets.numel()) - 1
        self.n_tokens = int(centroid_ids.numel())

    def res(self) -> Residual:
        return Residual(self.dim, self.nbits, self.n_centroids, self.centroids.data_ptr(),
                        self.weights.data_ptr(),
                        self.centroid_ids.data_ptr() if self.n_tokens else None,
                        self.residuals.data_ptr() if self.n_tokens else None,
                        self.offsets.data_ptr(), self.n_docs, self.n_tokens)


def _n_pairs(q: Tokens, n_docs: int, cand):
    return cand.n_total if cand is not None else q.n_sets * n_docs


def quantize(x, dtype: str, stream=None, out=None, scales=None):
    """FP32 [T, d] -> (tokens of `dtype`, per-token scales for fp8 else None);
    `out` / `scales`: preallocated [T, d] tokens of that type / [T] FP32."""
    T, d = x.shape
    if out is None:
        out = torch.empty((T, d), dtype=TORCH_DTYPES[dtype], device=x.device)
    if out.shape != (T, d) or out.dtype != TORCH_DTYPES[dtype] or not out.is_contiguous():
        raise ValueError("quantize: out must be a contiguous [T, d] tensor of the target type")
    sc = scales
    if dtype == "fp8" and sc is None:
        sc = torch.empty(T, dtype=torch.float32, device=x.device)
    _check(lib().maxsim_quantize(_ptr(x), T, d, DTYPES[dtype], _ptr(out), _ptr(sc),
                                 _stream(stream)))
    return out, sc


def score(q: Tokens, d: Tokens, cand: Candidates = None, out=None, stream=None):
    """Fused MaxSim scores: [n_q * n_docs] (no candidates) or [cand.n_total]."""
    n = _n_pairs(q, d.n_sets, cand)
    if out is None:
        out = torch.empty(max(n, 0), dtype=torch.float32, device=d.offsets.device)
    qc, dc = q.csr(), d.csr()
    cc = cand.c() if cand is not None else None
    _check(lib().maxsim_score(ctypes.byref(qc), ctypes.byref(dc),
                              ctypes.byref(cc) if cc is not None else None, _ptr(out), None, 0,
                              _stream(stream)))
    return out


def score_topk_workspace_bytes(q: Tokens, d: Tokens, k: int, cand: Candidates = None) -> int:
    qc, dc = q.csr(), d.csr()
    cc = cand.c() if cand is not None else None
    return int(lib().maxsim_score_topk_workspace_size(
        ctypes.byref(qc), ctypes.byref(dc), ctypes.byref(cc) if cc is not None else None, k))


def score_topk(q: Tokens, d: Tokens, k: int, cand: Candidates = None, workspace=None,
               out=None, stream=None):
    """Fused scoring with the top-k in the scorer's epilogue (no score array):
    (scores [n_q, k], ids [n_q, k]) by score descending, then id ascending;
    ids are document indices, or candidate ids with candidate lists."""
    dev = d.offsets.device
    if out is None:
        out = (torch.empty((q.n_sets, k), dtype=torch.float32, device=dev),
               torch.empty((q.n_sets, k), dtype=torch.int32, device=dev))
    if workspace is None:
        workspace = torch.empty(max(score_topk_workspace_bytes(q, d, k, cand), 1),
                                dtype=torch.uint8, device=dev)
    qc, dc = q.csr(), d.csr()
    cc = cand.c() if cand is not None else None
    _check(lib().maxsim_score_topk(ctypes.byref(qc), ctypes.byref(dc),
                                   ctypes.byref(cc) if cc is not None else None, k,
                                   _ptr(out[0]), _ptr(out[1]), _ptr(workspace),
                                   workspace.numel(), _stream(stream)))
    return out


# Bytes of the library's fixed per-GPU scratch (include/maxsim.h,
# MAXSIM_NOALLOC_SCRATCH_BYTES): the largest score_topk workspace that
# score_topk_noalloc accepts.
NOALLOC_SCRATCH_BYTES = 64 * 1024 * 1024


def score_topk_noalloc(q: Tokens, d: Tokens, k: int, cand: Candidates = None, out=None,
                       stream=None):
    """score_topk through the entry point that allocates nothing: its
    workspace is the library's fixed per-GPU scratch (calls that overlap on
    one GPU race). Only the outputs are allocated here, when `out` is None."""
    dev = d.offsets.device
    if out is None:
        out = (torch.empty((q.n_sets, k), dtype=torch.float32, device=dev),
               torch.empty((q.n_sets, k), dtype=torch.int32, device=dev))
    qc, dc = q.csr(), d.csr()
    cc = cand.c() if cand is not None else None
    _check(lib().maxsim_score_topk_noalloc(ctypes.byref(qc), ctypes.byref(dc),
                                           ctypes.byref(cc) if cc is not None else None, k,
                                           _ptr(out[0]), _ptr(out[1]), _stream(stream)))
    return out


def unfused_workspace_bytes(q: Tokens, d: Tokens) -> int:
    qc, dc = q.csr(), d.csr()
    return int(lib().maxsim_score_unfused_workspace_size(ctypes.byref(qc), ctypes.byref(dc)))


def score_unfused(q: Tokens, d: Tokens, out=None, workspace=None, stream=None):
    """Unfused comparator: S = D Q^T to HBM, then max/sum from HBM."""
    n = q.n_sets * d.n_sets
    if out is None:
        out = torch.empty(max(n, 0), dtype=torch.float32, device=d.offsets.device)
    need = unfused_workspace_bytes(q, d)
    if workspace is None:
        workspace = torch.empty(max(need, 1), dtype=torch.uint8, device=d.offsets.device)
    qc, dc = q.csr(), d.csr()
    _check(lib().maxsim_score_unfused(ctypes.byref(qc), ctypes.byref(dc), _ptr(out),
                                      _ptr(workspace), workspace.numel(), _stream(stream)))
    return out


def pq_workspace_bytes(q: Tokens, d: PQDocs, cand: Candidates = None) -> int:
    qc, pc = q.csr(), d.pq()
    cc = cand.c() if cand is not None else None
    return int(lib().maxsim_pq_score_workspace_size(
        ctypes.byref(qc), ctypes.byref(pc), ctypes.byref(cc) if cc is not None else None))


def pq_score(q: Tokens, d: PQDocs, cand: Candidates = None, out=None, workspace=None,
             stream=None):
    """Fused PQ scores (table in LDS), same layout as score()."""
    n = _n_pairs(q, d.n_docs, cand)
    if out is None:
        out = torch.empty(max(n, 0), dtype=torch.float32, device=d.offsets.device)
    qc, pc = q.csr(), d.pq()
    cc = cand.c() if cand is not None else None
    ccp = ctypes.byref(cc) if cc is not None else None
    need = int(lib().maxsim_pq_score_workspace_size(ctypes.byref(qc), ctypes.byref(pc), ccp))
    if workspace is None and need > 0:
        workspace = torch.empty(need, dtype=torch.uint8, device=d.offsets.device)
    _check(lib().maxsim_pq_score(ctypes.byref(qc), ctypes.byref(pc), ccp, _ptr(out),
                                 _ptr(workspace), 0 if workspace is None else workspace.numel(),
                                 _stream(stream)))
    return out


def residual_workspace_bytes(q: Tokens, d: ResidualDocs, cand: Candidates = None) -> int:
    qc, rc = q.csr(), d.res()
    cc = cand.c() if cand is not None else None
    return int(lib().maxsim_residual_score_workspace_size(
        ctypes.byref(qc), ctypes.byref(rc), ctypes.byref(cc) if cc is not None else None))


def residual_score(q: Tokens, d: ResidualDocs, cand: Candidates = None, out=None,
                   workspace=None, stream=None):
    """MaxSim over residual-compressed documents, same layout as score()."""
    n = _n_pairs(q, d.n_docs, cand)
    if out is None:
        out = torch.empty(max(n, 0), dtype=torch.float32, device=d.offsets.device)
    qc, rc = q.csr(), d.res()
    cc = cand.c() if cand is not None else None
    ccp = ctypes.byref(cc) if cc is not None else None
    need = int(lib().maxsim_residual_score_workspace_size(ctypes.byref(qc), ctypes.byref(rc), ccp))
    if workspace is None and need > 0:
        workspace = torch.empty(need, dtype=torch.uint8, device=d.offsets.device)
    _check(lib().maxsim_residual_score(ctypes.byref(qc), ctypes.byref(rc), ccp, _ptr(out),
                                       _ptr(workspace),
                                       0 if workspace is None else workspace.numel(),
                                       _stream(stream)))
    return out


def topk_workspace_bytes(n_segments: int, k: int) -> int:
    return int(lib().maxsim_topk_workspace_size(n_segments, k))


def topk(scores, seg_offsets, k: int, ids=None, n_total=None, workspace=None, stream=None,
         out=None):
    """Per-segment top-k by (score desc, id asc): (scores [n_seg, k], ids [n_seg, k]);
    `out`: preallocated contiguous ([n_seg, k] FP32, [n_seg, k] int32)."""
    n_seg = int(seg_offsets.numel()) - 1
    n_total = int(scores.numel()) if n_total is None else int(n_total)
    dev = seg_offsets.device
    if out is None:
        out = (torch.empty((n_seg, k), dtype=torch.float32, device=dev),
               torch.empty((n_seg, k), dtype=torch.int32, device=dev))
    out_s, out_i = out
    if (out_s.shape != (n_seg, k) or out_i.shape != (n_seg, k) or out_s.dtype != torch.float32
            or out_i.dtype != torch.int32 or not out_s.is_contiguous()
            or not out_i.is_contiguous()):
        raise ValueError("topk: out must be contiguous [n_seg, k] float32 and int32 tensors")
    need = topk_workspace_bytes(n_seg, k)
    if workspace is None:
        workspace = torch.empty(max(need, 1), dtype=torch.uint8, device=dev)
    _check(lib().maxsim_topk(_ptr(scores), _ptr(seg_offsets), n_seg, n_total, _ptr(ids), k,
                             _ptr(out_s), _ptr(out_i), _ptr(workspace), workspace.numel(),
                             _stream(stream)))
    return out_s, out_i


def autotune(q: Tokens, d: Tokens, cand: Candidates = None, reps: int = 10,
             cache_path: str = None, stream=None) -> dict:
    """Times every fused launch shape on this problem and keeps the fastest."""
    n = _n_pairs(q, d.n_sets, cand)
    out = torch.empty(max(n, 1), dtype=torch.float32, device=d.offsets.device)
    qc, dc = q.csr(), d.csr()
    cc = cand.c() if cand is not None else None
    buf = ctypes.create_string_buffer(1 << 16)
    _check(lib().maxsim_autotune(ctypes.byref(qc), ctypes.byref(dc),
                                 ctypes.byref(cc) if cc is not None else None, _ptr(out), None, 0,
                                 _stream(stream), reps,
                                 cache_path.encode() if cache_path else None, buf, len(buf)))
    return json.loads(buf.value.decode())


def pq_autotune(q: Tokens, d: PQDocs, cand: Candidates = None, reps: int = 3,
                cache_path: str = None, stream=None) -> dict:
    """Times the table and decode-into-MFMA PQ scorers on this problem and
    keeps the faster for its key."""
    n = _n_pairs(q, d.n_docs, cand)
    out = torch.empty(max(n, 1), dtype=torch.float32, device=d.offsets.device)
    qc, pc = q.csr(), d.pq()
    cc = cand.c() if cand is not None else None
    ccp = ctypes.byref(cc) if cc is not None else None
    need = int(lib().maxsim_pq_score_workspace_size(ctypes.byref(qc), ctypes.byref(pc), ccp))
    # the table kernel's workspace (the decode kernel needs none)
    ws = torch.empty(max(need, n * 4 * 8, 1), dtype=torch.uint8, device=d.offsets.device)
    buf = ctypes.create_string_buffer(1 << 14)
    _check(lib().maxsim_pq_autotune(ctypes.byref(qc), ctypes.byref(pc), ccp, _ptr(out), _ptr(ws),
                                    ws.numel(), _stream(stream), reps,
                                    cache_path.encode() if cache_path else None, buf, len(buf)))
    return json.loads(buf.value.decode())


def residual_autotune(q: Tokens, d: ResidualDocs, cand: Candidates = None, reps: int = 5,
                      cache_path: str = None, stream=None) -> dict:
    """Times the residual scorer's load-pipeline shapes on this problem and
    keeps the fastest for its key."""
    n = _n_pairs(q, d.n_docs, cand)
    out = torch.empty(max(n, 1), dtype=torch.float32, device=d.offsets.device)
    qc, rc = q.csr(), d.res()
    cc = cand.c() if cand is not None else None
    ccp = ctypes.byref(cc) if cc is not None else None
    need = int(lib().maxsim_residual_score_workspace_size(ctypes.byref(qc), ctypes.byref(rc), ccp))
    ws = torch.empty(max(need, 1), dtype=torch.uint8, device=d.offsets.device)
    buf = ctypes.create_string_buffer(1 << 12)
    _check(lib().maxsim_residual_autotune(ctypes.byref(qc), ctypes.byref(rc), ccp, _ptr(out),
                                          _ptr(ws), ws.numel(), _stream(stream), reps,
                                          cache_path.encode() if cache_path else None, buf,
                                          len(buf)))
    return json.loads(buf.value.decode())


def validate(d, q: Tokens = None, cand: Candidates = None, stream=None):
    """Device-side checks of offsets, candidate ids, FP8 scales (Tokens docs),
    PQ codes (PQDocs docs) or centroid ids (ResidualDocs docs); raises MaxSimError (status 5) naming the
    violated rules. Synchronises the stream."""
    flags = torch.empty(1, dtype=torch.int32, device=d.offsets.device)
    qc = q.csr() if q is not None else None
    cc = cand.c() if cand is not None else None
    qp = ctypes.byref(qc) if qc is not None else None
    cp = ctypes.byref(cc) if cc is not None else None
    if isinstance(d, PQDocs):
        pc = d.pq()
        _check(lib().maxsim_validate_pq(qp, ctypes.byref(pc), cp, _ptr(flags), _stream(stream)))
    elif isinstance(d, ResidualDocs):
        rc = d.res()
        _check(lib().maxsim_validate_residual(qp, ctypes.byref(rc), cp, _ptr(flags),
                                              _stream(stream)))
    else:
        dc = d.csr()
        _check(lib().maxsim_validate(qp, ctypes.byref(dc), cp, _ptr(flags), _stream(stream)))
    _check(lib().maxsim_check(_ptr(flags), _stream(stream)))


def stream_probe(buf, variant: int = 0, stream=None):
    """Streams the bytes of `buf` (a device tensor) once; returns the checksum
    tensor (one per wave). Time it with events to get the read ceiling."""
    sink = torch.empty(256 * 8 * 4, dtype=torch.int32, device=buf.device)
    _check(lib().maxsim_stream_probe(_ptr(buf), buf.numel() * buf.element_size(), variant,
                                     _ptr(sink), sink.numel(), _stream(stream)))
    return sink


LDS_PROBE_READS_PER_16B = {0: 128, 1: 32, 2: 32}
LDS_PROBE_READ_BYTES = {0: 4, 1: 16, 2: 16}


def lds_probe(buf, variant: int = 1, table_bytes: int = 131072, stream=None):
    """Streams the bytes of `buf` and gathers from an LDS table for each word
    (maxsim_lds_probe); returns the checksum tensor. Lane-level reads issued:
    buf bytes / 16 * LDS_PROBE_READS_PER_16B[variant]."""
    sink = torch.empty(256 * 16, dtype=torch.int32, device=buf.device)
    _check(lib().maxsim_lds_probe(_ptr(buf), buf.numel() * buf.element_size(), variant,
                                  table_bytes, _ptr(sink), sink.numel(), _stream(stream)))
    return sink


def load_tune_cache(path: str):
    _check(lib().maxsim_load_tune_cache(path.encode()))
