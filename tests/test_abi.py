"""CPU checks of the C-ABI library: it loads, exports every declared entry
point, and rejects invalid host-visible arguments before touching a device."""
import ctypes
import os
import re

import pytest
import torch  # noqa: F401  (binds the library to torch's HIP runtime)

import paper_2606_26439_amd as M
from paper_2606_26439_amd import _binding as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    txt = open(os.path.join(ROOT, "include", "maxsim.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(maxsim_[a-z_]+)\s*\(", txt)))


def test_library_exports_every_declared_symbol():
    names = declared_functions()
    assert len(names) >= 13
    L = M.lib()
    for n in names:
        assert hasattr(L, n), n
    assert L.maxsim_abi_version() == 1


def _csr(dtype=2, dim=128, n_sets=1, n_tokens=4, max_len=4, tokens=16, offsets=16, scales=None):
    return B.CSR(dtype, dim, n_sets, n_tokens, max_len, 0, tokens, offsets, scales)


@pytest.mark.parametrize("q,d,code", [
    (dict(dim=100), dict(dim=100), 2),                # dim not a multiple of 16
    (dict(dim=8), dict(dim=8), 2),                    # dim below 16
    (dict(dim=1040), dict(dim=1040), 2),              # dim above 1024
    (dict(dtype=7), dict(), 1),                       # unknown dtype
    (dict(max_len=65), dict(), 2),                    # too many query tokens
    (dict(), dict(dim=256), 1),                       # dims differ
    (dict(dtype=1), dict(), 1),                       # dtypes differ
    (dict(tokens=8), dict(), 1),                      # misaligned tokens
    (dict(offsets=None), dict(), 1),                  # NULL offsets
    (dict(dtype=3), dict(dtype=3), 1),                # FP8 without scales
    (dict(n_sets=-1), dict(), 1),                     # negative size
])
def test_score_rejects_bad_arguments(q, d, code):
    L = M.lib()
    qc, dc = _csr(**q), _csr(**d)
    st = L.maxsim_score(ctypes.byref(qc), ctypes.byref(dc), None, ctypes.c_void_p(16), None, 0,
                        None)
    assert st == code, L.maxsim_last_error()
    assert L.maxsim_last_error()


def test_topk_and_quantize_validation():
    L = M.lib()
    assert L.maxsim_topk(None, ctypes.c_void_p(8), 1, 10, None, 0, None, None, None, 0, None) == 2
    assert L.maxsim_topk(None, ctypes.c_void_p(8), 1, 10, None, 5, ctypes.c_void_p(8),
                         ctypes.c_void_p(8), None, 0, None) == 1  # NULL scores with n_total > 0
    assert L.maxsim_topk(ctypes.c_void_p(8), ctypes.c_void_p(8), 1, 10, None, 5,
                         ctypes.c_void_p(8), ctypes.c_void_p(8), None, 0, None) == 3  # workspace
    assert L.maxsim_topk_workspace_size(4, 100) > 4 * 100 * 8
    assert L.maxsim_quantize(ctypes.c_void_p(16), 4, 100, 2, ctypes.c_void_p(16), None, None) == 2
    assert L.maxsim_quantize(ctypes.c_void_p(16), 4, 128, 3, ctypes.c_void_p(16), None, None) == 1
    assert L.maxsim_quantize(ctypes.c_void_p(16), 4, 128, 2, ctypes.c_void_p(16),
                             ctypes.c_void_p(16), None) == 1


def test_pq_and_unfused_validation():
    L = M.lib()
    qc = _csr(dim=128)
    pq = B.PQ(8, 256, 16, 2, 16, 16, 16, 10, 100)
    bad = B.PQ(6, 256, 16, 2, 16, 16, 16, 10, 100)
    assert L.maxsim_pq_score(ctypes.byref(qc), ctypes.byref(bad), None, ctypes.c_void_p(16), None,
                             0, None) == 2
    qbf = _csr(dtype=1, dim=128)
    assert L.maxsim_pq_score(ctypes.byref(qbf), ctypes.byref(pq), None, ctypes.c_void_p(16), None,
                             0, None) == 2
    dc = _csr(n_tokens=1000)
    need = L.maxsim_score_unfused_workspace_size(ctypes.byref(qc), ctypes.byref(dc))
    assert need == 1 * 1000 * 16 * 4
    assert L.maxsim_score_unfused(ctypes.byref(qc), ctypes.byref(dc), ctypes.c_void_p(16), None, 0,
                                  None) == 3
    # a size that overflows size_t is reported, never wrapped to a small one
    huge = _csr(n_tokens=1 << 62)
    assert L.maxsim_score_unfused_workspace_size(ctypes.byref(qc), ctypes.byref(huge)) == 2**64 - 1
    assert L.maxsim_score_unfused(ctypes.byref(qc), ctypes.byref(huge), ctypes.c_void_p(16),
                                  ctypes.c_void_p(256), 2**63, None) == 2


def test_missing_tune_cache_is_a_no_op(tmp_path):
    assert M.lib().maxsim_load_tune_cache(str(tmp_path / "none.json").encode()) == 0


def test_validate_rejects_bad_host_arguments():
    L = M.lib()
    dc = _csr()
    # NULL flag word
    assert L.maxsim_validate(None, ctypes.byref(dc), None, None, None) == 1
    assert L.maxsim_check(None, None) == 1
    # candidates without the queries they belong to
    cc = B.Cand(16, 16, 4)
    assert L.maxsim_validate(None, ctypes.byref(dc), ctypes.byref(cc), ctypes.c_void_p(16),
                             None) == 1
    bad = _csr(dim=100)
    assert L.maxsim_validate(None, ctypes.byref(bad), None, ctypes.c_void_p(16), None) == 2
    assert L.maxsim_validate_pq(None, None, None, ctypes.c_void_p(16), None) == 1


def _res(dim=128, nbits=2, n_c=1000, centroids=16, weights=16, ids=16, residuals=16,
         n_docs=10, n_tokens=100):
    return B.Residual(dim, nbits, n_c, centroids, weights, ids, residuals, 16, n_docs, n_tokens)


@pytest.mark.parametrize("q,d,code", [
    (dict(dim=96), dict(dim=96), 2),        # dim not 64, 128 or 256
    (dict(), dict(nbits=3), 2),             # residual width
    (dict(dtype=1), dict(), 2),             # queries must be F16
    (dict(dim=256), dict(), 1),             # dims differ
    (dict(), dict(n_c=0), 1),               # no centroids
    (dict(), dict(residuals=8), 1),         # misaligned residual rows
    (dict(), dict(centroids=None), 1),      # NULL centroids
    (dict(max_len=65), dict(), 2),          # too many query tokens
])
def test_residual_rejects_bad_arguments(q, d, code):
    L = M.lib()
    qc, rc = _csr(**q), _res(**d)
    st = L.maxsim_residual_score(ctypes.byref(qc), ctypes.byref(rc), None, ctypes.c_void_p(16),
                                 ctypes.c_void_p(256), 1 << 30, None)
    assert st == code, L.maxsim_last_error()


def test_residual_workspace_is_the_centroid_table():
    L = M.lib()
    qc = _csr(n_tokens=37, max_len=37)
    rc = _res(n_c=1001)
    need = L.maxsim_residual_score_workspace_size(ctypes.byref(qc), ctypes.byref(rc), None)
    # one query of max_len 37: 64 columns (16 x ceil(37 / 16) rounded up to 4 blocks)
    assert need == (1001 * 64 * 4 + 255) // 256 * 256
    assert L.maxsim_residual_score(ctypes.byref(qc), ctypes.byref(rc), None, ctypes.c_void_p(16),
                                   ctypes.c_void_p(256), need - 1, None) == 3
    assert L.maxsim_validate_residual(None, ctypes.byref(rc), None, None, None) == 1
    assert L.maxsim_validate_residual(None, None, None, ctypes.c_void_p(16), None) == 1


@pytest.mark.parametrize("dim", [16, 32, 48, 96, 160, 400, 1024])
def test_every_multiple_of_16_up_to_1024_is_accepted(dim):
    # no queries: nothing to launch, so the call validates and returns OK on
    # any machine; quantize with no tokens likewise
    L = M.lib()
    for dt in (0, 1, 2, 3):
        qc = _csr(dtype=dt, dim=dim, n_sets=0, n_tokens=0, max_len=32, tokens=None,
                  scales=16 if dt == 3 else None)
        dc = _csr(dtype=dt, dim=dim, scales=16 if dt == 3 else None)
        st = L.maxsim_score(ctypes.byref(qc), ctypes.byref(dc), None, ctypes.c_void_p(16), None,
                            0, None)
        assert st == 0, L.maxsim_last_error()
        st = L.maxsim_score_unfused(ctypes.byref(qc), ctypes.byref(dc), ctypes.c_void_p(16),
                                    None, 0, None)
        assert st == 0, L.maxsim_last_error()
        assert L.maxsim_quantize(ctypes.c_void_p(16), 0, dim, dt, ctypes.c_void_p(16),
                                 ctypes.c_void_p(16) if dt == 3 else None, None) == 0


def test_score_topk_validation():
    L = M.lib()
    qc, dc = _csr(), _csr()
    for k in (0, -3, 1025):
        st = L.maxsim_score_topk(ctypes.byref(qc), ctypes.byref(dc), None, k, ctypes.c_void_p(16),
                                 ctypes.c_void_p(16), None, 0, None)
        assert st == 1, L.maxsim_last_error()
        assert L.maxsim_score_topk_workspace_size(ctypes.byref(qc), ctypes.byref(dc), None, k) == 0
    bad = _csr(dim=100)
    st = L.maxsim_score_topk(ctypes.byref(bad), ctypes.byref(bad), None, 10, ctypes.c_void_p(16),
                             ctypes.c_void_p(16), None, 0, None)
    assert st == 2, L.maxsim_last_error()
    assert L.maxsim_score_topk(None, ctypes.byref(dc), None, 10, None, None, None, 0, None) == 1
