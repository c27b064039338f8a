"""The row reductions over four lane rows (device_common.h: max_rows4,
sum_rows4) are inline gfx950 assembly (v_permlane16_swap /
v_permlane32_swap), which the compiler's hazard recognizer does not inspect.
Build the kernels that use them (the PQ decode-into-MFMA scorer, the
residual scorer, and one instance of the fused scorer) to gfx950 assembly on
the CPU and check what the assembly relies on: each swap is preceded by 4
wait states (a VALU write of a VGPR the swap reads needs 2; a V_CMPX write of
EXEC needs 4), and the first max or add after it reads both swapped
registers, neither of which is written in between."""
import os
import re
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


SOURCES = {
    # source, minimum number of swaps expected in its assembly
    "pq_mfma": (os.path.join(ROOT, "paper_2606_26439_amd", "csrc", "pq_mfma.hip"), 16),
    "residual": (os.path.join(ROOT, "paper_2606_26439_amd", "csrc", "residual.hip"), 16),
    "fused": (os.path.join(ROOT, "tests", "fused_swap_instance.hip"), 8),
}


@pytest.fixture(scope="module", params=sorted(SOURCES))
def asm(request, tmp_path_factory):
    if not (os.path.exists(HIPCC) or shutil.which("hipcc")):
        pytest.skip("hipcc not available")
    src, n_min = SOURCES[request.param]
    out = tmp_path_factory.mktemp("asm") / (request.param + ".s")
    cmd = [HIPCC, "-O3", "-std=c++17", "--offload-arch=gfx950", "-Xclang", "-target-feature",
           "-Xclang", "-packed-fp32-ops", "-fno-honor-nans", "-I", os.path.join(ROOT, "include"),
           "-x", "hip", "--cuda-device-only", "-S", src, "-o", str(out)]
    subprocess.run(cmd, check=True, capture_output=True)
    return [ln.split(";")[0].strip() for ln in out.read_text().splitlines()], n_min


def _program(lines):
    """Instructions in order, and the instruction index each label names."""
    ins, labels = [], {}
    for ln in lines:
        if not ln or ln.startswith((".", ";")) and not ln.endswith(":"):
            continue
        if ln.endswith(":"):
            labels[ln[:-1]] = len(ins)
        elif not ln.startswith("."):
            ins.append(ln)
    return ins, labels


def _vregs(text):
    """VGPR names an operand text names: v7, or each of v[4:7]."""
    out = set(re.findall(r"\bv\d+\b", text))
    for a, b in re.findall(r"\bv\[(\d+):(\d+)\]", text):
        out |= {f"v{i}" for i in range(int(a), int(b) + 1)}
    return out


def _maxes_after(ins, labels, start, regs, limit=400):
    """Follows every control-flow path from `start` while either swapped
    register still holds its swapped value, and returns the max or add
    instructions that read one of them (the row reduction the swap feeds). A write ends a
    register's life; other reads are not the max and are skipped (on paths
    where the compiler proved the max dead, the registers hold don't-care
    values)."""
    todo, seen, found = [(start, frozenset(regs))], set(), []
    while todo:
        pos, live = todo.pop()
        steps = 0
        while live and pos < len(ins) and steps < limit:
            if (pos, live) in seen:
                break
            seen.add((pos, live))
            steps += 1
            ln = ins[pos]
            if ln.startswith("s_"):
                m = re.match(r"s_(c?branch)\w*\s+(\S+)", ln)
                if m:
                    tgt = labels[m.group(2)]
                    if m.group(1) == "branch":
                        pos = tgt
                        continue
                    todo.append((tgt, live))
                elif ln.startswith(("s_endpgm", "s_setpc")):
                    break
                pos += 1
                continue
            stores = ln.startswith(("global_store", "buffer_store", "ds_write", "flat_store"))
            opnds = (ln.split(None, 1) + [""])[1].split(",")
            dst = set() if stores else _vregs(opnds[0])
            reads = set().union(*(_vregs(o) for o in (opnds if stores else opnds[1:])))
            if ln.startswith(("v_max", "v_add_f32")) and reads & live:
                found.append((ln, reads))
                break
            live = live - dst
            pos += 1
    return found


def test_every_swap_has_its_wait_states_and_a_reduction_of_both_registers(asm):
    lines, n_min = asm
    ins, labels = _program(lines)
    swaps = [i for i, ln in enumerate(ins) if re.match(r"v_permlane(16|32)_swap_b32\b", ln)]
    assert len(swaps) >= n_min, "expected the swap-based row reduction in every kernel instance"
    for i in swaps:
        prev = ins[i - 1]
        m = re.match(r"s_nop\s+(\d+)", prev)
        assert m and int(m.group(1)) >= 3, f"swap at {i} preceded by {prev!r}"
        regs = re.findall(r"\bv\d+\b", ins[i])
        assert len(regs) == 2 and regs[0] != regs[1], ins[i]
        maxes = _maxes_after(ins, labels, i + 1, regs)
        assert maxes, f"no max or add reads the swap {ins[i]!r}"
        for ln, reads in maxes:
            assert set(regs) <= reads, f"the reduction after {ins[i]!r} reads one copy: {ln!r}"
