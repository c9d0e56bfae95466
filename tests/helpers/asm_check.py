"""Check of the compiled kernels for one code-generation hazard.

In the general kernels the compiler once placed the copy of a value that
lives across an if/else join (a walker's weight, moved to accumulation
registers for the long mode passes) at the top of the join block, before
the instruction that restores the exec mask.  The copy then ran only on the
lanes of one side of the branch, and the others read a register that had
never been written.

This module compiles the kernel sources to gfx950 assembly and lists, per
kernel, every labelled block whose first instructions write vector or
accumulation registers before its first exec-mask instruction, when that
instruction is the restore ``s_or_b64 exec, exec, s[..]``.

A branch arm that the compiler placed out of line has the same shape, and
is correct: its writes run under the arm's exec mask.  Such a block is left
out when every way into it sets that mask: it is reached only by
``s_cbranch_execnz`` straight after ``s_and_saveexec_b64 sX, ..``, or by
falling through ``s_and_saveexec_b64 sX, ..; s_cbranch_execz``, where sX is
the pair the block's restore reads (or it has no fall-through at all, after
``s_endpgm`` or ``s_branch``).  A join block is still reported: it is
entered from an arm's last instruction or by ``s_cbranch_execz``.  A
finding is a place to read, not proof of an error; the current kernels have
none.

    python tests/helpers/asm_check.py        # all kernel sources, ~8 minutes

It is a test of the build, not part of the library.
"""
from __future__ import annotations

import os
import re
import subprocess
import sys
import tempfile
from concurrent.futures import ThreadPoolExecutor
from typing import Dict, List, Tuple

_ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
if _ROOT not in sys.path:
    sys.path.insert(0, _ROOT)
from paper_2608_14544_amd import build as B  # noqa: E402

_LABEL = re.compile(r"^(\.LBB\d+_\d+):")
_FUNC = re.compile(r"^(_Z\w+):")
_RESTORE = re.compile(r"s_or_b64 exec, exec, (s\[\d+:\d+\])")
_VECTOR_WRITE = ("v_", "global_load", "ds_read", "buffer_load", "scratch_load")
_NOT_A_WRITE = ("v_cmp", "v_readlane", "v_readfirstlane")


def _instr(line: str) -> str:
    return line.split(";")[0].strip()


def _prev_instr(lines: List[str], i: int) -> Tuple[int, str]:
    """The nearest instruction before line i (labels and comments skipped)."""
    j = i - 1
    while j >= 0:
        s = _instr(lines[j])
        if s and not s.startswith((".LBB", "_Z")) and not s.endswith(":"):
            return j, s
        j -= 1
    return -1, ""


def _arm_only(lines: List[str], i: int, pair: str, targets: Dict[str, List[int]], label: str) -> bool:
    """True when every entry into the block at line i sets the exec mask
    saved in ``pair`` (see the module notes)."""
    saveexec = "s_and_saveexec_b64 " + pair
    j, s = _prev_instr(lines, i)
    if s.startswith("s_cbranch_execz"):
        if not _prev_instr(lines, j)[1].startswith(saveexec):
            return False
    elif not s.startswith(("s_endpgm", "s_branch", "s_setpc")):
        return False
    for k in targets.get(label, []):
        t = _instr(lines[k])
        if not t.startswith("s_cbranch_execnz") or not _prev_instr(lines, k)[1].startswith(saveexec):
            return False
    return True


def scan(asm: str, functions: str = "kernel") -> Dict[str, List[Tuple[str, List[str]]]]:
    """Findings in one assembly text: {function: [(label, first writes)]},
    for functions whose symbol contains ``functions``."""
    lines = asm.split("\n")
    targets: Dict[str, List[int]] = {}
    for k, line in enumerate(lines):
        t = _instr(line)
        if t.startswith(("s_branch", "s_cbranch")):
            targets.setdefault(t.split()[-1], []).append(k)
    out: Dict[str, List[Tuple[str, List[str]]]] = {}
    func = None
    for i, line in enumerate(lines):
        m = _FUNC.match(line)
        if m:
            func = m.group(1)
            continue
        m = _LABEL.match(line)
        if not m or func is None or functions not in func:
            continue
        writes: List[str] = []
        pair = None
        for j in range(i + 1, min(i + 64, len(lines))):
            s = _instr(lines[j])
            if not s:
                continue
            if s.startswith((".LBB", "_Z", "s_branch", "s_cbranch", "s_endpgm", "s_setpc")):
                break
            if "exec" in s:
                r = _RESTORE.match(s)
                pair = r.group(1) if r else None
                break
            if s.startswith(_VECTOR_WRITE) and not s.startswith(_NOT_A_WRITE):
                writes.append(s)
        if pair and writes and not _arm_only(lines, i, pair, targets, m.group(1)):
            out.setdefault(func, []).append((m.group(1), writes[:4]))
    return out


def device_asm(source: str, out_dir: str) -> str:
    """Compiles one kernel source to gfx950 assembly (device code only)."""
    path = os.path.join(B.CSRC, source)
    out = os.path.join(out_dir, source + ".s")
    cmd = [B.hipcc(), *B.HIP_FLAGS, "-I", B.INCLUDE, "-I", B.CSRC, "-x", "hip", "-S", "--offload-device-only",
           path, "-o", out]
    subprocess.run(cmd, check=True, stdout=subprocess.DEVNULL, stderr=subprocess.DEVNULL)
    with open(out) as f:
        return f.read()


def check(sources=None, jobs: int = 0) -> Dict[str, Dict[str, List[Tuple[str, List[str]]]]]:
    """Compiles the kernel sources and scans them; {source: findings}."""
    sources = sources or [s for s in B.SOURCES if s.endswith(".hip")]
    jobs = jobs or min(len(sources), max(1, os.cpu_count() or 2))
    with tempfile.TemporaryDirectory() as tmp:
        with ThreadPoolExecutor(max_workers=jobs) as ex:
            texts = list(ex.map(lambda s: device_asm(s, tmp), sources))
    return {s: scan(t) for s, t in zip(sources, texts)}


def main(argv) -> int:
    found = check(argv or None)
    n = 0
    for src, per in found.items():
        for func, hits in per.items():
            for label, writes in hits:
                n += 1
                print(f"{src}: {func[:100]} {label}: {writes}")
    print(f"{n} finding(s) in {len(found)} source(s)")
    return 1 if n else 0


if __name__ == "__main__":
    sys.exit(main(sys.argv[1:]))
