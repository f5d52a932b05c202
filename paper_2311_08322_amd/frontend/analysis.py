"""Analysis of the definition IR: checks of the language's rules and the
implementation plan the code generator follows (GT4Py paper, Sec. 2.3: the
analysis pipeline lowers the definition IR towards the parallel model).

Rules (errors raised as StencilAnalysisError):
* PARALLEL computations: a variable written in the computation is not read
  at a vertical offset in it, a statement does not read its own target at a
  horizontal offset (self-assignment with a dependency, Sec. 2.2), and an
  API field written in the computation is not read in it.
* FORWARD / BACKWARD computations: a variable written in the computation is
  read at a zero horizontal offset only, and vertically at dk = 0 or at the
  level already computed (dk = -1 going up, +1 going down); the first level
  of the sweep may not read such a previous level (checked per call, the
  level bounds depend on nk).
* Temporaries are read only after an assignment (checked by the parser).

Plan:
* extents: where each variable must be computed (temporaries) or readable
  (API fields), as offsets from the compute domain, found by walking the
  statements backwards from the outputs (which need exactly the domain);
* storage of temporaries: `lds` (written and read only in one PARALLEL
  computation: one level of it lives in LDS), `reg` (only in one sequential
  computation: a register per column, plus the previous level's value when
  the sweep reads it), `hbm` (crosses computations: a 3-D buffer in the
  workspace over its extent);
* per PARALLEL computation, the input fields read at horizontal offsets are
  staged per level in LDS (one box per field and vertical offset);
* per sequential computation, the horizontal region the sweep runs on.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Dict, List, Tuple

from . import ir


class StencilAnalysisError(ValueError):
    pass


ZERO = (0, 0, 0, 0)  # (ilo, ihi, jlo, jhi)
EMPTY = None


def _union(a, b):
    if a is None:
        return b
    if b is None:
        return a
    return (min(a[0], b[0]), max(a[1], b[1]), min(a[2], b[2]), max(a[3], b[3]))


def _shifted(e, off):
    if e is None:
        return None
    return (e[0] + off[0], e[1] + off[0], e[2] + off[1], e[3] + off[1])


@dataclass
class TempInfo:
    name: str
    storage: str = "reg"
    ext: Tuple[int, int, int, int] = ZERO
    comps: set = field(default_factory=set)  # computations writing it
    read_comps: set = field(default_factory=set)


@dataclass
class FieldInfo:
    name: str
    read: bool = False
    written: bool = False
    ext: Tuple[int, int, int, int] = ZERO
    # (computation, block, dk) of every read, for the per-call vertical check
    kreads: List[Tuple[int, int, int]] = field(default_factory=list)


@dataclass
class CompPlan:
    index: int
    order: str
    blocks: Tuple[Tuple[ir.Interval, Tuple[ir.Stmt, ...]], ...]
    writes: List[str] = field(default_factory=list)
    # PARALLEL: extent of each top-level statement (same order as the block's)
    stmt_ext: List[List[Tuple[int, int, int, int]]] = field(default_factory=list)
    # PARALLEL: staged (field, dk) -> box extent
    staged: Dict[Tuple[str, int], Tuple[int, int, int, int]] = field(default_factory=dict)
    # sequential: region of the sweep; variables whose previous level is read
    region: Tuple[int, int, int, int] = ZERO
    kcache: List[str] = field(default_factory=list)
    # sequential: (block, var) pairs reading the previous level
    prev_reads: List[Tuple[int, str]] = field(default_factory=list)


@dataclass
class Plan:
    sdef: ir.StencilDef
    fields: Dict[str, FieldInfo]
    temps: Dict[str, TempInfo]
    comps: List[CompPlan]
    # temporaries read at vertical offsets: (comp, block, name, dk)
    temp_kreads: List[Tuple[int, int, str, int]] = field(default_factory=list)
    # computations fused into one kernel each, in program order
    groups: List[List[int]] = field(default_factory=list)


def _writes(stmts):
    out = []
    for s in stmts:
        out += ir.stmt_accesses(s)[1]
    return out


def _comp_reads(cp):
    out = []
    for _, stmts in cp.blocks:
        for s in stmts:
            out += ir.stmt_accesses(s)[0]
    return out


def _groups(comps, temps):
    """Fusion of computations into kernels, in program order.  A group is a
    run of PARALLEL computations (P), optionally followed by one sweep S
    (FORWARD or BACKWARD) and by more sweeps (S*), every sweep on the
    domain's columns (its region is the domain), so that a workgroup's lanes
    are exactly its tile's columns.  Fused, the run is evaluated level by
    level inside S's sweep, before S's block of that level.  A computation
    joins the group only if that gives the unfused result:
    * P and S read what earlier members wrote at dk = 0 (one level is held),
      at horizontal offsets only if it is a temporary (LDS box of the
      workgroup; API fields written by the run belong to other workgroups
      off the tile), and a later P member reads no API field the run wrote;
    * S* read what earlier members wrote at their own column (any level);
    * no member writes a variable an earlier member reads."""
    groups = []
    n = len(comps)
    i = 0
    while i < n:
        g = [i]
        wr = set(comps[i].writes)
        rd = {a.name for a in _comp_reads(comps[i])}
        role = "P" if comps[i].order == ir.PARALLEL else "S*"
        if role == "S*" and comps[i].region != ZERO:
            groups.append(g)
            i += 1
            continue

        def fits(cp, role):
            if set(cp.writes) & rd:
                return False
            for a in _comp_reads(cp):
                if a.name not in wr:
                    continue
                horiz = (a.offset[0], a.offset[1]) != (0, 0)
                if role in ("P", "S"):
                    if a.offset[2] != 0:
                        return False
                    if a.name not in temps and (horiz or role == "P"):
                        return False
                elif horiz:
                    return False
            return True

        j = i + 1
        while j < n:
            cp = comps[j]
            if cp.order == ir.PARALLEL:
                nxt = "P" if role == "P" else None
            else:
                nxt = "S" if role == "P" else "S*"
                if cp.region != ZERO:
                    nxt = None
            if nxt is None or not fits(cp, nxt):
                break
            g.append(j)
            wr |= set(cp.writes)
            rd |= {a.name for a in _comp_reads(cp)}
            role = nxt
            j += 1
        groups.append(g)
        i = j
    return groups


def analyse(sdef: ir.StencilDef) -> Plan:
    fields = {f: FieldInfo(f) for f in sdef.fields}
    temps: Dict[str, TempInfo] = {}
    comps = []
    for ci, c in enumerate(sdef.computations):
        cp = CompPlan(ci, c.order, c.blocks)
        w = []
        for _, stmts in c.blocks:
            for n in _writes(stmts):
                if n not in w:
                    w.append(n)
        cp.writes = w
        for n in w:
            if n in fields:
                fields[n].written = True
            else:
                temps.setdefault(n, TempInfo(n)).comps.add(ci)
        comps.append(cp)

    # ---- rules and read bookkeeping
    plan = Plan(sdef, fields, temps, comps)
    for cp in comps:
        wset = set(cp.writes)
        for bi, (iv, stmts) in enumerate(cp.blocks):
            def check_stmt(s):
                reads, writes = ir.stmt_accesses(s)
                for a in reads:
                    di, dj, dk = a.offset
                    if a.name in fields:
                        fields[a.name].read = True
                        fields[a.name].kreads.append((cp.index, bi, dk))
                    else:
                        temps[a.name].read_comps.add(cp.index)
                        plan.temp_kreads.append((cp.index, bi, a.name, dk))
                    if cp.order == ir.PARALLEL:
                        if a.name in wset and dk != 0:
                            raise StencilAnalysisError(
                                f"{a.name} is written in a PARALLEL computation and read there at dk = {dk}")
                        if a.name in wset and a.name in fields:
                            raise StencilAnalysisError(
                                f"API field {a.name} is written in a PARALLEL computation and read in it "
                                "(assign a temporary instead)")
                        if a.name in writes and (di, dj) != (0, 0) and isinstance(s, ir.Assign):
                            raise StencilAnalysisError(
                                f"{a.name} = ... reads {a.name} at offset {(di, dj)}: self-assignment with a "
                                "horizontal dependency in a PARALLEL computation")
                    else:
                        if a.name in wset:
                            if (di, dj) != (0, 0):
                                raise StencilAnalysisError(
                                    f"{a.name} is written in a {cp.order} computation and read there at the "
                                    f"horizontal offset {(di, dj)}")
                            allowed = (0, -1) if cp.order == ir.FORWARD else (0, 1)
                            if dk not in allowed:
                                raise StencilAnalysisError(
                                    f"{a.name} is written in a {cp.order} computation and read there at "
                                    f"dk = {dk} (allowed: {allowed})")
                            if dk != 0:
                                if a.name not in cp.kcache:
                                    cp.kcache.append(a.name)
                                if (bi, a.name) not in cp.prev_reads:
                                    cp.prev_reads.append((bi, a.name))
                if isinstance(s, ir.If):
                    for t in s.then + s.orelse:
                        check_stmt(t)
            for s in stmts:
                check_stmt(s)

    # ---- extents: backwards from the outputs
    need: Dict[str, Tuple[int, int, int, int]] = {}
    for f in fields.values():
        if f.written:
            need[f.name] = ZERO

    def walk_back(stmts, cp, exts_out):
        """Reverse pass over one block; records each statement's extent."""
        for s in reversed(stmts):
            _, writes = ir.stmt_accesses(s)
            if cp.order == ir.PARALLEL:
                ext = None
                for wv in writes:
                    ext = _union(ext, need.get(wv))
                if ext is None:
                    ext = ZERO  # dead store: computed on the domain only
                if isinstance(s, ir.Assign):
                    need.pop(s.target, None)
            else:
                ext = cp.region
            exts_out.append(ext)
            reads, _ = ir.stmt_accesses(s)
            for a in reads:
                need[a.name] = _union(need.get(a.name), _shifted(ext, a.offset))
        exts_out.reverse()

    for cp in reversed(comps):
        if cp.order != ir.PARALLEL:
            reg = None
            for wv in cp.writes:
                reg = _union(reg, need.get(wv))
            cp.region = reg if reg is not None else ZERO
            for wv in cp.writes:
                need.pop(wv, None)
        # blocks cover disjoint levels: each starts from the same needs
        start = dict(need)
        merged = dict(need)
        cp.stmt_ext = [None] * len(cp.blocks)
        for bi in reversed(range(len(cp.blocks))):
            need.clear()
            need.update(start)
            exts = []
            walk_back(list(cp.blocks[bi][1]), cp, exts)
            cp.stmt_ext[bi] = exts
            for k, v in need.items():
                merged[k] = _union(merged.get(k), v)
            # a value written in this block is not needed from before it
        need.clear()
        need.update(merged)
        if cp.order == ir.PARALLEL:
            for wv in cp.writes:
                if wv in temps:
                    pass
        for wv in cp.writes:
            if wv in temps:
                t = temps[wv]
                e = None
                for bi, (_, stmts) in enumerate(cp.blocks):
                    for s, ext in zip(stmts, cp.stmt_ext[bi]):
                        if wv in ir.stmt_accesses(s)[1]:
                            e = _union(e, ext)
                t.ext = _union(t.ext, e) if e is not None else t.ext

    for f in fields.values():
        if f.read:
            f.ext = _union(ZERO, need.get(f.name)) if need.get(f.name) is not None else ZERO

    # ---- kernel groups (fusion), then the storage of temporaries
    plan.groups = _groups(comps, set(temps))
    group_of = {}
    for gi, g in enumerate(plan.groups):
        for c in g:
            group_of[c] = gi
    for t in temps.values():
        users = t.comps | t.read_comps
        gs = {group_of[c] for c in users}
        t.storage = "hbm"
        if len(gs) == 1:
            g = plan.groups[gs.pop()]
            prun = [c for c in g if comps[c].order == ir.PARALLEL]
            first_seq = [c for c in g if comps[c].order != ir.PARALLEL][:1]
            if t.comps <= set(prun) and t.read_comps <= set(prun) | set(first_seq):
                t.storage = "lds"
            elif len(t.comps) == 1 and t.read_comps <= t.comps and comps[next(iter(t.comps))].order != ir.PARALLEL:
                t.storage = "reg"
    for t in temps.values():
        if t.storage == "hbm":
            t.ext = _union(t.ext, ZERO)

    # ---- LDS staging of input fields in PARALLEL computations: a (field, dk)
    # read anywhere at a horizontal offset is staged, and then serves all its
    # reads (the box covers every reader's extent and offset)
    for cp in comps:
        if cp.order != ir.PARALLEL:
            continue
        keys = set()
        for _, stmts in cp.blocks:
            for s in stmts:
                for a in ir.stmt_accesses(s)[0]:
                    if a.name in fields and (a.offset[0], a.offset[1]) != (0, 0):
                        keys.add((a.name, a.offset[2]))
        for bi, (_, stmts) in enumerate(cp.blocks):
            for s, ext in zip(stmts, cp.stmt_ext[bi]):
                for a in ir.stmt_accesses(s)[0]:
                    key = (a.name, a.offset[2])
                    if key in keys:
                        cp.staged[key] = _union(cp.staged.get(key), _shifted(ext, a.offset))
    return plan


def vertical_check(plan: Plan, nk: int, kranges: Dict[str, Tuple[int, int]]):
    """Per-call check of the vertical accesses for nk levels: every read of an
    API field stays inside the levels the caller's field provides
    (kranges[name] = (lowest, highest + 1) relative to the domain's level 0),
    every temporary read stays inside [0, nk), sequential blocks do not
    overlap, and a sweep never reads the previous level at its first level."""
    for name, f in plan.fields.items():
        lo, hi = kranges[name]
        for ci, bi, dk in f.kreads:
            a, b = plan.comps[ci].blocks[bi][0].bounds(nk)
            if a < b and (a + dk < lo or b + dk > hi):
                raise StencilAnalysisError(
                    f"{name} is read at levels [{a + dk}, {b + dk}) but provides [{lo}, {hi})")
    for ci, bi, name, dk in plan.temp_kreads:
        a, b = plan.comps[ci].blocks[bi][0].bounds(nk)
        if a < b and (a + dk < 0 or b + dk > nk):
            raise StencilAnalysisError(f"temporary {name} is read at levels [{a + dk}, {b + dk}) outside [0, {nk})")
    for cp in plan.comps:
        spans = sorted(iv.bounds(nk) for iv, _ in cp.blocks)
        spans = [s for s in spans if s[0] < s[1]]
        for (a0, b0), (a1, b1) in zip(spans, spans[1:]):
            if a1 < b0:
                raise StencilAnalysisError(f"computation {cp.index}: intervals overlap for nk = {nk}")
        if cp.order == ir.PARALLEL or not spans:
            continue
        covered = set()
        for a, b in spans:
            covered.update(range(a, b))
        for bi, name in cp.prev_reads:
            a, b = cp.blocks[bi][0].bounds(nk)
            if a >= b:
                continue
            if cp.order == ir.FORWARD and (a - 1) not in covered:
                raise StencilAnalysisError(f"{name}[0,0,-1] is read at level {a}, below the sweep's first level")
            if cp.order == ir.BACKWARD and b not in covered:
                raise StencilAnalysisError(f"{name}[0,0,1] is read at level {b - 1}, above the sweep's first level")
