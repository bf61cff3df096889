"""Build-time check of the compiled gfx950 kernels: no loop that holds a
workgroup barrier may exit lane by lane.

A loop whose exit depends on a per-lane (divergent) condition runs, on the
GPU, until the last lane of a wave leaves it, with the other lanes masked off.
If such a loop holds an ``s_barrier``, a wave reaches the barrier with only
some of its lanes: the barrier (counted per wave) releases while the masked
lanes have not done the work that was to precede it.  The typical source is
an item loop that starts with ``if (tid == 0) slot = atomicAdd(queue, 1)``
and a barrier: ``tid == 0`` is loop-invariant, the compiler folds that branch
into the back edge, and the loop becomes a nest whose inner loop (the
barrier, the item) lanes 1..63 of wave 0 re-enter without thread 0's pop.

The check reads the device assembly that the build keeps (clang's loop
comments name each block's innermost loop header) and reports every loop
that contains ``s_barrier`` and also either masks lanes out of the loop
(``s_andn2_b64 exec, exec, ...``) or branches back to its header while some
lanes are active (``s_cbranch_execnz``).
"""
from __future__ import annotations

import re

_FUNC = re.compile(r"\n(_Z\w+):\s*;.*?\n(.*?)\.Lfunc_end", re.S)
_LABEL = re.compile(r"(\.LBB\d+_\d+|; %bb\.\d+):(.*)")


def divergent_barrier_loops(asm: str) -> list[tuple[str, str]]:
    """(kernel symbol, loop header) of every loop in `asm` that holds a
    barrier and has a lane-by-lane exit."""
    found = []
    for name, body in _FUNC.findall(asm):
        loop = None
        barrier, divergent = set(), set()
        for line in body.split("\n"):
            m = _LABEL.match(line)
            if m:
                comment = m.group(2)
                head = re.search(r"Header=BB(\d+_\d+)", comment)
                if "Loop Header" in comment and m.group(1).startswith(".LBB"):
                    loop = "BB" + m.group(1)[4:]
                else:
                    loop = "BB" + head.group(1) if head else None
                continue
            if loop is None:
                continue
            if "s_barrier" in line:
                barrier.add(loop)
            # lanes masked out of the loop, or a back edge taken while some
            # lanes remain (an execz branch to the header is taken only when
            # no lane is active: not a lane-by-lane exit)
            if re.search(r"s_andn2_b64\s+exec,\s*exec", line) or \
                    re.search(r"s_cbranch_execnz\s+\.L" + loop + r"\b", line):
                divergent.add(loop)
        found += [(name, h) for h in sorted(barrier & divergent)]
    return found


def check_file(path: str) -> list[tuple[str, str]]:
    with open(path) as f:
        return divergent_barrier_loops(f.read())
