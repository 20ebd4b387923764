"""Static check of the built library's gfx950 code: no s_barrier may be reached while an LDS
operation issued before it can still be in flight (no s_waitcnt lgkmcnt(0) in between on some
path).  Waves meet at a barrier to hand LDS data to each other; hipcc's code for __syncthreads()
did not always wait for the LDS operations before it (the back edge of a loop ending in LDS
stores reached the loop's barrier with them in flight, and another wave's later LDS increments
could land first and be lost).  The check disassembles libtqp.so (the code objects built here
from this repository's sources), splits every kernel into basic blocks, and propagates "an LDS
operation may be pending" along every control-flow edge."""
import os
import re
import shutil
import subprocess
import tempfile
from collections import defaultdict

import pytest

LLVM = "/opt/rocm/llvm/bin"
SO = os.path.join(os.path.dirname(__file__), "..", "paper_2203_01877_amd", "libtqp.so")

FUNC = re.compile(r"^([0-9a-f]+) <(\S+)>:$")
INSTR = re.compile(r"^\s+(\S+)(.*?)\s*//\s*([0-9A-Fa-f]+):")
TARGET = re.compile(r"<(\S+?)(?:\+0x([0-9a-f]+))?>\s*$")
# LDS-accessing instructions (the cross-lane ds_ operations do not touch LDS memory)
NOT_LDS = ("ds_swizzle", "ds_permute", "ds_bpermute")


def _functions(text):
    """{name: [(addr, mnemonic, operands, target_addr or None)]} from llvm-objdump -d output."""
    funcs, base, cur = {}, {}, None
    for line in text.splitlines():
        m = FUNC.match(line)
        if m:
            cur = m.group(2)
            base[cur] = int(m.group(1), 16)
            funcs[cur] = []
            continue
        if cur is None:
            continue
        m = INSTR.match(line)
        if not m:
            continue
        mnem, ops, addr = m.group(1), m.group(2), int(m.group(3), 16)
        tgt = None
        if mnem.startswith("s_branch") or mnem.startswith("s_cbranch"):
            t = TARGET.search(line)
            if t and t.group(1) in base:
                tgt = base[t.group(1)] + int(t.group(2) or "0", 16)
        funcs[cur].append((addr, mnem, ops, tgt))
    return funcs


def _barriers_with_pending_lds(ins):
    """Addresses of s_barrier instructions some path reaches with an LDS operation not yet waited for."""
    if not ins:
        return []
    addrs = [a for a, _, _, _ in ins]
    index = {a: i for i, a in enumerate(addrs)}
    leaders = {0}
    for i, (_, mnem, _, tgt) in enumerate(ins):
        if tgt is not None and tgt in index:
            leaders.add(index[tgt])
        if mnem.startswith(("s_branch", "s_cbranch", "s_endpgm", "s_setpc")) and i + 1 < len(ins):
            leaders.add(i + 1)
    starts = sorted(leaders)
    blocks = [(s, (starts[k + 1] if k + 1 < len(starts) else len(ins))) for k, s in enumerate(starts)]
    block_of = {s: k for k, (s, _) in enumerate(blocks)}
    succ = defaultdict(list)
    for k, (s, e) in enumerate(blocks):
        _, mnem, _, tgt = ins[e - 1]
        if mnem.startswith("s_endpgm") or mnem.startswith("s_setpc"):
            continue
        if tgt is not None and tgt in index and index[tgt] in block_of:
            succ[k].append(block_of[index[tgt]])
        if not mnem.startswith("s_branch") and k + 1 < len(blocks):
            succ[k].append(k + 1)

    def run(k, pending, found=None):
        s, e = blocks[k]
        for i in range(s, e):
            _, mnem, ops, _ = ins[i]
            if mnem == "s_waitcnt" and "lgkmcnt(0)" in ops:
                pending = False
            elif mnem == "s_barrier":
                if pending and found is not None:
                    found.append(ins[i][0])
            elif mnem.startswith("ds_") and not mnem.startswith(NOT_LDS):
                pending = True
        return pending

    pend_in = [False] * len(blocks)
    work = list(range(len(blocks)))
    while work:
        k = work.pop()
        out = run(k, pend_in[k])
        for j in succ[k]:
            if out and not pend_in[j]:
                pend_in[j] = True
                work.append(j)
    found = []
    for k in range(len(blocks)):
        run(k, pend_in[k], found)
    return found


def test_no_barrier_with_lds_in_flight():
    so = os.path.abspath(SO)
    if not os.path.exists(so):
        pytest.skip("libtqp.so is not built")
    objdump = os.path.join(LLVM, "llvm-objdump")
    if not os.path.exists(objdump):
        pytest.skip("llvm-objdump is not installed")
    with tempfile.TemporaryDirectory() as tmp:
        lib = os.path.join(tmp, "libtqp.so")
        shutil.copy(so, lib)
        # the offload bundles are written next to the copy
        subprocess.run([objdump, "--offloading", lib], cwd=tmp, check=True, capture_output=True, timeout=300)
        objs = sorted(f for f in os.listdir(tmp) if f.endswith("gfx950"))
        assert objs, "no gfx950 code object in libtqp.so"
        bad, kernels = [], 0
        for f in objs:
            text = subprocess.run([objdump, "-d", "--mcpu=gfx950", os.path.join(tmp, f)], check=True,
                                  capture_output=True, text=True, timeout=300).stdout
            for name, ins in _functions(text).items():
                kernels += 1
                for addr in _barriers_with_pending_lds(ins):
                    bad.append("%s at 0x%x" % (name, addr))
    assert kernels > 100
    assert not bad, "s_barrier reached with LDS operations in flight: " + "; ".join(bad[:10])


def test_detector_flags_a_back_edge():
    """The dataflow itself: a loop whose body ends in an LDS store and whose head is a barrier is
    flagged; the same loop with a wait before the back edge is not."""
    base = [(0, "s_mov_b32", " s0, 0", None), (4, "s_barrier", "", None), (8, "ds_add_u32", " v1, v2", None)]
    tail = [(12, "ds_write_b32", " v1, v3", None), (16, "s_cbranch_scc1", " -5", 4), (20, "s_endpgm", "", None)]
    assert _barriers_with_pending_lds(base + tail) == [4]
    waited = [(12, "ds_write_b32", " v1, v3", None), (14, "s_waitcnt", " lgkmcnt(0)", None),
              (16, "s_cbranch_scc1", " -5", 4), (20, "s_endpgm", "", None)]
    assert _barriers_with_pending_lds(base + waited) == []
