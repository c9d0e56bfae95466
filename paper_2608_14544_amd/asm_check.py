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
instruction is the restore ``s_or_b64 exec, exec, s[..]``.  Code that
belongs to a branch arm can have this shape too, so a finding is a place to
read, not proof of an error; the current kernels have none.

    python -m paper_2608_14544_amd.asm_check        # all kernel sources, ~8 minutes
"""
from __future__ import annotations

import os
import re
import subprocess
import sys
import tempfile
from concurrent.futures import ThreadPoolExecutor
from typing import Dict, List, Tuple

from . import build as B

_LABEL = re.compile(r"^(\.LBB\d+_\d+):")
_FUNC = re.compile(r"^(_Z\w+):")
_RESTORE = re.compile(r"s_or_b64 exec, exec, s\[\d+:\d+\]")
_VECTOR_WRITE = ("v_", "global_load", "ds_read", "buffer_load", "scratch_load")
_NOT_A_WRITE = ("v_cmp", "v_readlane", "v_readfirstlane")


def scan(asm: str, functions: str = "kernel") -> Dict[str, List[Tuple[str, List[str]]]]:
    """Findings in one assembly text: {function: [(label, first writes)]},
    for functions whose symbol contains ``functions``."""
    lines = asm.split("\n")
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
        restore = False
        for j in range(i + 1, min(i + 64, len(lines))):
            s = lines[j].split(";")[0].strip()
            if not s:
                continue
            if s.startswith((".LBB", "_Z", "s_branch", "s_cbranch", "s_endpgm", "s_setpc")):
                break
            if "exec" in s:
                restore = bool(_RESTORE.match(s))
                break
            if s.startswith(_VECTOR_WRITE) and not s.startswith(_NOT_A_WRITE):
                writes.append(s)
        if restore and writes:
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
