"""Scan of AMDGPU assembly for workgroup barriers inside loops whose exit is
taken per lane (an exec-masked exit).

In such a loop some lanes of a wavefront can leave while the others go round
again through ``s_barrier``, which then pairs with a different barrier of the
other wavefronts: the workgroup hangs or reads stale shared data.  Source code
with uniform loops can still compile to this shape when a divergent step sits
at the end of a loop body, so the compiled code is checked, not the source.

The scan uses the loop annotations LLVM writes into ``-S`` output: every block
label (``.LBBx_y:`` or ``; %bb.N:``) carries its innermost loop (``in Loop:
Header=BBx_y``) or marks a loop header, with ``Parent Loop`` lines giving the
nesting.  A loop is flagged when one of its blocks executes ``s_andn2_b64 exec,
exec, ...`` (the lane-wise exit) and the loop or a loop nested in it contains
``s_barrier``.
"""
import re


def split_kernels(text):
    kernels, cur = [], None
    for line in text.split("\n"):
        m = re.match(r"^(_Z\w+):", line)
        if m:
            cur = [m.group(1), []]
            kernels.append(cur)
        elif cur is not None:
            cur[1].append(line)
    return kernels


def flagged_loops(lines):
    blocks, blk = [], None
    for line in lines:
        m = re.match(r"^\.LBB(\d+_\d+):(.*)", line) or re.match(r"^; %bb\.(\d+):(.*)", line)
        if m:
            blk = {"label": "BB" + m.group(1), "loop": None, "parents": [], "header": False, "body": []}
            blocks.append(blk)
            rest = m.group(2)
            mm = re.search(r"in Loop: Header=(BB\d+_\d+)", rest)
            if mm:
                blk["loop"] = mm.group(1)
            mm = re.search(r"Parent Loop (BB\d+_\d+)", rest)
            if mm:
                blk["parents"].append(mm.group(1))
            if "Loop Header" in rest and "in Loop" not in rest:
                blk["header"] = True
            continue
        if blk is None:
            continue
        s = line.strip()
        if s.startswith(";"):
            mm = re.search(r"Parent Loop (BB\d+_\d+)", s)
            if mm:
                blk["parents"].append(mm.group(1))
            if "Loop Header" in s and "in Loop" not in s:
                blk["header"] = True
            continue
        blk["body"].append(s)
    parent = {}
    for b in blocks:
        if b["header"]:
            b["loop"] = b["label"]
            parent[b["label"]] = b["parents"][-1] if b["parents"] else None
    members = {}
    for b in blocks:
        h = b["loop"]
        while h is not None:
            members.setdefault(h, []).append(b)
            h = parent.get(h)
    bad = set()
    for b in blocks:
        if b["loop"] and any(x.startswith("s_andn2_b64 exec, exec") for x in b["body"]):
            if any("s_barrier" in x for bb in members.get(b["loop"], []) for x in bb["body"]):
                bad.add(b["loop"])
    return sorted(bad)


def scan(text):
    """{kernel symbol: [flagged loop headers]} for every kernel with one."""
    out = {}
    for name, lines in split_kernels(text):
        bad = flagged_loops(lines)
        if bad:
            out[name] = bad
    return out
