"""The document-end column sums of the grouped fused kernels and of the PQ
decode-into-MFMA kernel run as four DPP row rotations (by 8, 4, 2, 1 lanes)
with adds; the other kernels use an xor butterfly (lane ^ 8, ^ 4, ^ 2, ^ 1).
Both must leave the same FP32 bits in lane 0, whichever way the rotation
turns, so that a query scores the same alone (one block, butterfly) and in
a unit (several blocks, rotations). Simulated here in float32 on the host."""
import numpy as np
import pytest


def _butterfly(a):
    v = a.copy()
    for m in (8, 4, 2, 1):
        v = (v + v[np.arange(16) ^ m]).astype(np.float32)
    return v


def _rotations(a, direction):
    v = a.copy()
    for m in (8, 4, 2, 1):
        v = (v + v[(np.arange(16) + direction * m) % 16]).astype(np.float32)
    return v


@pytest.mark.parametrize("direction", [1, -1])
def test_rotation_sum_matches_butterfly_in_lane0(direction):
    g = np.random.default_rng(7)
    for _ in range(2000):
        a = (g.standard_normal(16) * 10.0 ** g.integers(-3, 4, 16)).astype(np.float32)
        r = _rotations(a, direction)
        b = _butterfly(a)
        assert r[0].view(np.uint32) == b[0].view(np.uint32)
        # every lane of the row holds a full sum (lane 0 is the one stored)
        assert np.allclose(r, np.float32(a.astype(np.float64).sum()), rtol=1e-5, atol=1e-3)


def test_rotation_sum_is_order_sensitive_elsewhere():
    # the equality is a property of lane 0's pairing, not of FP addition in
    # general: a plain left-to-right sum differs for some inputs
    g = np.random.default_rng(3)
    differs = False
    for _ in range(200):
        a = (g.standard_normal(16) * 10.0 ** g.integers(-3, 4, 16)).astype(np.float32)
        seq = np.float32(0)
        for x in a:
            seq = np.float32(seq + x)
        differs |= seq.view(np.uint32) != _butterfly(a)[0].view(np.uint32)
    assert differs
