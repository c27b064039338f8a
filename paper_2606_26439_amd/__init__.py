"""MI355X (gfx950) TileMaxSim: fused late-interaction MaxSim scoring.

Hand-written HIP kernels behind the C ABI of ``include/maxsim.h``
(``libmaxsim.so``); this package is the thin ctypes binding plus the serving
loop built on it. PyTorch provides device memory and streams only.

    from paper_2606_26439_amd import Tokens, quantize, score, topk
"""
from ._binding import (DTYPES, ELEM_BYTES, Candidates, MaxSimError, PQDocs,  # noqa: F401
                       ResidualDocs, Tokens, autotune, default_tune_cache, lib,
                       load_tune_cache, pq_autotune, pq_score, pq_workspace_bytes, quantize,
                       residual_autotune,
                       residual_score,
                       residual_workspace_bytes, score, score_topk, score_topk_noalloc,
                       score_topk_workspace_bytes, NOALLOC_SCRATCH_BYTES,
                       score_unfused, stream_probe, lds_probe, topk,
                       topk_workspace_bytes, unfused_workspace_bytes, validate)
