"""The measured ceilings the kernels are reported against read what they
claim: the LDS gather probe's per-wave checksums equal a host recomputation of
the table entries its documented index pattern selects."""
import numpy as np
import pytest
import torch

import paper_2606_26439_amd as M

pytestmark = pytest.mark.gpu


def _expected(words, variant, slots, n_waves):
    """Per-wave XOR checksums of lds_gather for a buffer of uint32 words."""
    i = np.arange(slots, dtype=np.uint64)
    table = np.stack([(i * 2654435761) & 0xFFFFFFFF, i ^ 0x9e3779b9, i + 7,
                      (~i) & 0xFFFFFFFF], axis=1).astype(np.uint32)
    flat = table.reshape(-1)
    units = words.size // 256  # 1 KiB of words per wave step
    w = words[:units * 256].reshape(units, 64, 4)  # [unit][lane][word]
    lanes = np.arange(64, dtype=np.uint32)[None, :, None]
    reps = 4 if variant == 0 else 1
    acc = np.zeros((units, 64), np.uint32)
    for rep in range(reps):
        x = w ^ np.uint32((0x9e3779b9 * rep) & 0xFFFFFFFF)
        for sft in range(8):
            k = ((x >> np.uint32(4 * sft)) | (x << np.uint32((32 - 4 * sft) % 32))) \
                if sft else x
            if variant == 0:
                v = flat[k & np.uint32(slots * 4 - 1)]
            elif variant == 1:
                e = table[k & np.uint32(slots - 1)]
                v = e[..., 0] ^ e[..., 1] ^ e[..., 2] ^ e[..., 3]
            else:
                idx = ((k & np.uint32(slots - 1)) & ~np.uint32(15)) | (lanes & np.uint32(15))
                e = table[idx]
                v = e[..., 0] ^ e[..., 1] ^ e[..., 2] ^ e[..., 3]
            acc ^= np.bitwise_xor.reduce(v, axis=2)
    per_unit = np.bitwise_xor.reduce(acc, axis=1)
    out = np.zeros(n_waves, np.uint32)
    for wv in range(n_waves):
        lo, hi = units * wv // n_waves, units * (wv + 1) // n_waves
        if hi > lo:
            out[wv] = np.bitwise_xor.reduce(per_unit[lo:hi])
    return out


@pytest.mark.parametrize("variant", [0, 1, 2])
@pytest.mark.parametrize("table_bytes", [65536, 131072])
def test_lds_probe_reads_the_documented_entries(variant, table_bytes):
    g = np.random.default_rng(variant)
    words = g.integers(0, 2 ** 32, size=(3 << 20) // 4 + 64, dtype=np.uint32)  # ragged tail
    buf = torch.from_numpy(words.view(np.uint8).copy()).cuda()
    sink = M.lds_probe(buf, variant, table_bytes).cpu().numpy().view(np.uint32)
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    n_waves = min(sink.size // 16, cus) * 16
    want = _expected(words, variant, table_bytes // 16, n_waves)
    assert np.array_equal(sink[:n_waves], want)
