"""HIP code generation for gfx950 from an analysed stencil (the backend of
the toolchain in the GT4Py paper, Sec. 2.3).

One kernel per computation, launched in program order (Sec. 2.2: the
computations behave as if run one after the other):

* PARALLEL: a workgroup of 256 lanes owns a 64 x 4 tile of the domain and
  marches a block of levels.  Per level, each input field read at a
  horizontal offset is staged in LDS over the box its readers need (one
  coalesced pass), then every statement runs over its own box (the tile
  grown by the extent the analysis found), writing temporaries into their
  LDS boxes, with a barrier between statements.  Outputs are stored inside
  the domain only; temporaries that cross computations also go to their
  workspace buffer.
* FORWARD / BACKWARD: one lane per column of the sweep's region (64 x 4
  lanes per workgroup, rows along i for coalescing), levels visited upwards
  or downwards; a variable written in the sweep lives in a register, and the
  previous level's value in a second one when the sweep reads it.

The generated source also holds the C ABI of ``include/gtscript_abi.h``,
with the argument checks of the plan (field coverage, vertical ranges,
workspace).  Arithmetic is literal: the library is built without
floating-point contraction.
"""
from __future__ import annotations

from . import ir
from .analysis import Plan

GEN_VERSION = 4
TI, TJ = 64, 4
MIN_WGS = 2048


class CodegenError(ValueError):
    pass


def _reads(cp):
    out = []
    for _, stmts in cp.blocks:
        for s in stmts:
            out += ir.stmt_accesses(s)[0]
    return out


def _c(v: float) -> str:
    return f"((real){float(v)!r})"


class _Gen:
    def __init__(self, plan: Plan, dtype: str, fingerprint: str):
        self.p = plan
        self.real = "double" if dtype == "float64" else "float"
        self.dtype = dtype
        self.fp = fingerprint
        self.hbm = [t for t in plan.temps.values() if t.storage == "hbm"]
        # flattened block index per (computation, block)
        self.bidx = {}
        n = 0
        for cp in plan.comps:
            for bi in range(len(cp.blocks)):
                self.bidx[(cp.index, bi)] = n
                n += 1
        self.nblocks = n

    # ------------------------------------------------------------ helpers
    def f_inside(self, name, i, j):
        e = self.p.fields[name].ext
        return f"({i} >= {e[0]} && {i} < A.ni + {e[1]} && {j} >= {e[2]} && {j} < A.nj + {e[3]})"

    def t_inside(self, name, i, j):
        e = self.p.temps[name].ext
        return f"({i} >= {e[0]} && {i} < A.ni + {e[1]} && {j} >= {e[2]} && {j} < A.nj + {e[3]})"

    def gld_field(self, name, i, j, k):
        return (f"gld(A.f_{name}, A.f_{name}_sj, A.f_{name}_sk, {i}, {j}, {k}, "
                f"{self.f_inside(name, i, j)})")

    def gld_temp(self, name, i, j, k):
        return (f"gld(A.t_{name}, A.t_{name}_sj, A.t_{name}_sk, {i}, {j}, {k}, "
                f"{self.t_inside(name, i, j)})")

    # ------------------------------------------------------------ expressions
    def expr(self, e, acc):
        if isinstance(e, ir.Const):
            return _c(e.value)
        if isinstance(e, ir.Scalar):
            return f"A.s_{e.name}"
        if isinstance(e, ir.Access):
            return acc(e)
        if isinstance(e, ir.Unary):
            a = self.expr(e.a, acc)
            return f"(-{a})" if e.op == "-" else f"(!{a})"
        if isinstance(e, ir.Binary):
            return f"({self.expr(e.a, acc)} {e.op} {self.expr(e.b, acc)})"
        if isinstance(e, ir.Compare):
            return f"({self.expr(e.a, acc)} {e.op} {self.expr(e.b, acc)})"
        if isinstance(e, ir.BoolOp):
            op = "&&" if e.op == "and" else "||"
            return f"({self.expr(e.a, acc)} {op} {self.expr(e.b, acc)})"
        if isinstance(e, ir.Ternary):
            return (f"(({self.expr(e.cond, acc)}) ? (real)({self.expr(e.a, acc)}) : "
                    f"(real)({self.expr(e.b, acc)}))")
        if isinstance(e, ir.Builtin):
            fn = {"abs": "fabs", "min": "fmin", "max": "fmax", "sqrt": "sqrt", "exp": "exp",
                  "log": "log"}[e.name]
            args = ", ".join(f"(real)({self.expr(a, acc)})" for a in e.args)
            return f"{fn}({args})"
        raise CodegenError(f"unknown expression {e!r}")

    # ------------------------------------------------------------ level pipeline
    def gldk_field(self, name, i, j, k, valid="true"):
        """Load with the caller's vertical range checked too (prefetches
        reach levels no statement reads there)."""
        return (f"gld(A.f_{name}, A.f_{name}_sj, A.f_{name}_sk, {i}, {j}, {k}, "
                f"({self.f_inside(name, i, j)} && ({k}) >= -A.f_{name}_klo && ({k}) < A.f_{name}_khi && ({valid})))")

    def gldk_temp(self, name, i, j, k, valid="true"):
        return (f"gld(A.t_{name}, A.t_{name}_sj, A.t_{name}_sk, {i}, {j}, {k}, "
                f"({self.t_inside(name, i, j)} && ({k}) >= 0 && ({k}) < A.nk && ({valid})))")

    class _Pipe:
        """Registers of one level loop: for each input read at the lane's own
        column (key (kind, name, dk)) the value of the current level, and the
        staged boxes of the tile's inputs; the next level's are loaded at the
        top of each level, while the current one is computed."""

        def __init__(self, tag):
            self.tag = tag
            self.cols = []    # (kind, name, dk)
            self.boxes = []   # (array, field, dk, ext, width, count)

        def col(self, kind, name, dk):
            key = (kind, name, dk)
            if key not in self.cols:
                self.cols.append(key)
            return f"pc{self.tag}_{kind}_{name}_{'m' if dk < 0 else 'p'}{abs(dk)}"

    def pipe_lines(self, pipe, I, J, kexpr, valid, which, step=0):
        """Loads of every pipelined value for level kexpr into the `which`
        registers (cur / nxt).  For the next level (step = +1 going up, -1
        going down) a value the current level already holds at dk + step is
        copied instead of loaded again."""
        out = []
        for (kind, name, dk) in pipe.cols:
            r = pipe.col(kind, name, dk)
            if step and (kind, name, dk + step) in pipe.cols:
                out.append(f"{r}_{which} = {pipe.col(kind, name, dk + step)}_cur;")
                continue
            ld = (self.gldk_field(name, I, J, f"{kexpr} + ({dk})", valid) if kind == "f"
                  else self.gldk_temp(name, I, J, f"{kexpr} + ({dk})", valid))
            out.append(f"{r}_{which} = {ld};")
        for (arr, f, dk, e, bw, cnt) in pipe.boxes:
            n_it = (cnt + 255) // 256
            for it in range(n_it):
                el = f"(tid + {it * 256})"
                gi, gj = f"(i0 + ({e[0]}) + {el} % {bw})", f"(j0 + ({e[2]}) + {el} / {bw})"
                ld = self.gldk_field(f, gi, gj, f"{kexpr} + ({dk})", f"({valid}) && {el} < {cnt}")
                out.append(f"pb_{arr}_{which}[{it}] = {ld};")
        return out

    def pipe_decls(self, pipe):
        out = []
        for (kind, name, dk) in pipe.cols:
            r = pipe.col(kind, name, dk)
            out.append(f"real {r}_cur = (real)0, {r}_nxt = (real)0;")
        for (arr, f, dk, e, bw, cnt) in pipe.boxes:
            n_it = (cnt + 255) // 256
            out.append(f"real pb_{arr}_cur[{n_it}], pb_{arr}_nxt[{n_it}];")
        return out

    def pipe_rotate(self, pipe):
        out = []
        for (kind, name, dk) in pipe.cols:
            r = pipe.col(kind, name, dk)
            out.append(f"{r}_cur = {r}_nxt;")
        for (arr, f, dk, e, bw, cnt) in pipe.boxes:
            for it in range((cnt + 255) // 256):
                out.append(f"pb_{arr}_cur[{it}] = pb_{arr}_nxt[{it}];")
        return out

    # ------------------------------------------------------------ LDS synchronisation
    class _Sync:
        """Barrier placement inside a tile kernel: a barrier goes before a
        statement that reads LDS data written since the last barrier by
        other lanes, or writes LDS data that other lanes wrote or read since
        then.  Lanes map to box points by the statement's box (ext); the
        same box and a zero offset mean the same lane."""
        MIXED = "mixed"

        def __init__(self):
            self.dirty, self.reads = {}, {}

        def copy(self):
            c = _Gen._Sync()
            c.dirty = dict(self.dirty)
            c.reads = {k: set(v) for k, v in self.reads.items()}
            return c

        def need(self, reads, writes, ext):
            for arr, off in reads:
                d = self.dirty.get(arr)
                if d is not None and (d != ext or off != (0, 0)):
                    return True
            for arr in writes:
                d = self.dirty.get(arr)
                if d is not None and d != ext:
                    return True
                for (e2, off2) in self.reads.get(arr, ()):
                    if e2 != ext or off2 != (0, 0):
                        return True
            return False

        def record(self, reads, writes, ext):
            for arr, off in reads:
                self.reads.setdefault(arr, set()).add((ext, off))
            for arr in writes:
                self.dirty[arr] = ext

        def clear(self):
            self.dirty, self.reads = {}, {}

        @staticmethod
        def merge(states):
            m = _Gen._Sync()
            for st in states:
                for arr, d in st.dirty.items():
                    if arr in m.dirty and m.dirty[arr] != d:
                        m.dirty[arr] = _Gen._Sync.MIXED
                    else:
                        m.dirty.setdefault(arr, d)
                for arr, rs in st.reads.items():
                    m.reads.setdefault(arr, set()).update(rs)
            return m

    # ------------------------------------------------------------ PARALLEL parts
    def _stag(self, ci, f, dk):
        return f"S{ci}_{f}_{'m' if dk < 0 else 'p'}{abs(dk)}"

    def tile_decls(self, pruns, lds_names, pipe):
        """LDS boxes of a tile kernel: the temporaries the run keeps on chip
        and the staged input boxes of every run member (their loads go
        through the level pipeline)."""
        p = self.p
        boxes, lines = {}, []
        for t in lds_names:
            e = p.temps[t].ext
            bw, bh = TI + e[1] - e[0], TJ + e[3] - e[2]
            boxes[("L", t)] = (e, bw)
            lines.append(f"  __shared__ real L_{t}[{bw * bh}];")
        for cp in pruns:
            for (f, dk), e in sorted(cp.staged.items()):
                bw, bh = TI + e[1] - e[0], TJ + e[3] - e[2]
                arr = self._stag(cp.index, f, dk)
                boxes[("S", cp.index, f, dk)] = (e, bw)
                lines.append(f"  __shared__ real {arr}[{bw * bh}];")
                pipe.boxes.append((arr, f, dk, e, bw, bw * bh))
        return boxes, lines

    def _lds_reads(self, s, ci, boxes):
        out = []
        for a in ir.stmt_accesses(s)[0]:
            di, dj, dk = a.offset
            if ("S", ci, a.name, dk) in boxes:
                out.append((self._stag(ci, a.name, dk), (di, dj)))
            elif ("L", a.name) in boxes and dk == 0:
                out.append((f"L_{a.name}", (di, dj)))
        return out

    def _lds_writes(self, s, boxes):
        return [f"L_{w}" for w in ir.stmt_accesses(s)[1] if ("L", w) in boxes]

    def par_level(self, cp, boxes, pipe, sync, written_in_group):
        """The statements of a PARALLEL computation at level k: block chain,
        staging from the pipeline registers, statements with the barriers
        the sync state asks for.  Returns (lines, sync state after)."""
        out = []
        first = True
        ends = []
        for bi, (_, stmts) in enumerate(cp.blocks):
            b = self.bidx[(cp.index, bi)]
            out.append(f"{'if' if first else '} else if'} (k >= A.blo[{b}] && k < A.bhi[{b}]) {{")
            first = False
            st = sync.copy()
            staged_here = sorted({(a.name, a.offset[2]) for s_ in stmts for a in ir.stmt_accesses(s_)[0]
                                  if (a.name, a.offset[2]) in cp.staged})
            staged_arrs = [self._stag(cp.index, f, dk) for f, dk in staged_here]
            if staged_here:
                if st.need([], staged_arrs, "staging"):
                    out.append("  __syncthreads();")
                    st.clear()
                for (f, dk) in staged_here:
                    e, bw = boxes[("S", cp.index, f, dk)]
                    cnt = bw * (TJ + e[3] - e[2])
                    arr = self._stag(cp.index, f, dk)
                    for it in range((cnt + 255) // 256):
                        guard = f"if (tid + {it * 256} < {cnt}) " if (it + 1) * 256 > cnt else ""
                        out.append(f"  {guard}{arr}[tid + {it * 256}] = pb_{arr}_cur[{it}];")
                st.record([], staged_arrs, "staging")
            for s_, ext in zip(stmts, cp.stmt_ext[bi]):
                self._check_if_offsets(s_)
                rd, wr = self._lds_reads(s_, cp.index, boxes), self._lds_writes(s_, boxes)
                if st.need(rd, wr, ext):
                    out.append("  __syncthreads();")
                    st.clear()
                bw, bh = TI + ext[1] - ext[0], TJ + ext[3] - ext[2]
                lane = ext == (0, 0, 0, 0)
                out += [f"  for (int e = tid; e < {bw * bh}; e += 256) {{",
                        f"    const int li = e % {bw}, lj = e / {bw};",
                        f"    const int pi = i0 + ({ext[0]}) + li, pj = j0 + ({ext[2]}) + lj;"]
                acc = self._tile_acc(cp.index, boxes, "pi", "pj", pipe if lane else None, written_in_group)
                out += ["    " + l for l in self.stmt_code(s_, acc, self._par_store(boxes))]
                out.append("  }")
                st.record(rd, wr, ext)
            ends.append(st)
        if not first:
            out.append("} else {")
            ends.append(sync.copy())
            out.append("}")
        return out, _Gen._Sync.merge(ends) if ends else sync

    def _tile_acc(self, ci, boxes, I, J, pipe, written_in_group):
        """Accessor inside a tile kernel at point (I, J, k): staged inputs of
        computation ci and the run's temporaries from LDS; inputs at the
        lane's own column from the pipeline (pipe given only where the point
        is the lane's column); the rest from memory."""
        p = self.p

        def acc(a):
            di, dj, dk = a.offset
            if ("S", ci, a.name, dk) in boxes:
                e, bw = boxes[("S", ci, a.name, dk)]
                return (f"{self._stag(ci, a.name, dk)}[({I} + ({di}) - i0 - ({e[0]})) + "
                        f"({J} + ({dj}) - j0 - ({e[2]})) * {bw}]")
            if ("L", a.name) in boxes and dk == 0:
                e, bw = boxes[("L", a.name)]
                return f"L_{a.name}[({I} + ({di}) - i0 - ({e[0]})) + ({J} + ({dj}) - j0 - ({e[2]})) * {bw}]"
            if pipe is not None and (di, dj) == (0, 0) and a.name not in written_in_group:
                kind = "f" if a.name in p.fields else "t"
                if kind == "f" or p.temps[a.name].storage == "hbm":
                    return pipe.col(kind, a.name, dk) + "_cur"
            if a.name in p.fields:
                return self.gld_field(a.name, f"{I} + ({di})", f"{J} + ({dj})", f"k + ({dk})")
            if p.temps[a.name].storage != "hbm":
                raise CodegenError(f"{a.name} read where it is not held")
            return self.gld_temp(a.name, f"{I} + ({di})", f"{J} + ({dj})", f"k + ({dk})")
        return acc

    def _par_store(self, boxes):
        p = self.p

        def store(name, v):
            out = []
            if name in p.fields:
                out.append(f"if (pi >= 0 && pi < A.ni && pj >= 0 && pj < A.nj) "
                           f"A.f_{name}[(int64_t)pi + (int64_t)pj * A.f_{name}_sj + (int64_t)k * A.f_{name}_sk] = {v};")
            else:
                if ("L", name) in boxes:
                    e, bw = boxes[("L", name)]
                    out.append(f"L_{name}[(pi - i0 - ({e[0]})) + (pj - j0 - ({e[2]})) * {bw}] = {v};")
                if p.temps[name].storage == "hbm":
                    out.append(f"if ({self.t_inside(name, 'pi', 'pj')}) A.t_{name}[(int64_t)pi + "
                               f"(int64_t)pj * A.t_{name}_sj + (int64_t)k * A.t_{name}_sk] = {v};")
            return out
        return store

    def _check_if_offsets(self, s):
        if not isinstance(s, ir.If):
            return
        reads, writes = ir.stmt_accesses(s)
        for a in reads:
            if a.name in writes and (a.offset[0], a.offset[1]) != (0, 0):
                raise CodegenError(f"{a.name} is written inside an if and read there at a horizontal offset")

    def stmt_code(self, s, acc, store):
        if isinstance(s, ir.Assign):
            v = self.expr(s.value, acc)
            return ["{", f"  const real v_ = (real)({v});"] + ["  " + l for l in store(s.target, "v_")] + ["}"]
        out = [f"if ({self.expr(s.cond, acc)}) {{"]
        for t in s.then:
            out += ["  " + l for l in self.stmt_code(t, acc, store)]
        out.append("} else {")
        for t in s.orelse:
            out += ["  " + l for l in self.stmt_code(t, acc, store)]
        out.append("}")
        return out

    # ------------------------------------------------------------ sweeps
    def seq_decls(self, cp):
        out = [f"real cur_{cp.index}_{v} = (real)0;" for v in cp.writes]
        out += [f"real prev_{cp.index}_{v} = (real)0;" for v in cp.kcache]
        return out

    def seq_level(self, cp, outer_acc, pipe, written_in_group):
        """The block chain of a sweep at level k for the lane's column (i, j);
        outer_acc serves values of the fused run (None outside a tile
        kernel), pipe the lane-column inputs."""
        p = self.p
        wset = list(cp.writes)
        c = cp.index
        out = ["bool done = false;"]
        for bi, (_, stmts) in enumerate(cp.blocks):
            b = self.bidx[(c, bi)]
            out.append(f"if (!done && k >= A.blo[{b}] && k < A.bhi[{b}]) {{")
            out.append("  done = true;")
            need_init = []

            def scan(stmts, assigned):
                for s_ in stmts:
                    reads = list(ir.accesses(s_.value)) if isinstance(s_, ir.Assign) else list(ir.accesses(s_.cond))
                    for a in reads:
                        if a.name in wset and a.offset[2] == 0 and a.name not in assigned and a.name not in need_init:
                            need_init.append(a.name)
                    if isinstance(s_, ir.Assign):
                        assigned.add(s_.target)
                    else:
                        t_set, e_set = set(assigned), set(assigned)
                        scan(s_.then, t_set)
                        scan(s_.orelse, e_set)
                        assigned |= (t_set & e_set)
            scan(stmts, set())
            for v in need_init:
                if v in p.fields:
                    out.append(f"  cur_{c}_{v} = {self.gld_field(v, 'i', 'j', 'k')};")
                elif p.temps[v].storage == "hbm":
                    out.append(f"  cur_{c}_{v} = {self.gld_temp(v, 'i', 'j', 'k')};")
                else:
                    raise CodegenError(f"{v} is read at a level before the sweep assigns it there")

            def acc(a):
                di, dj, dk = a.offset
                if a.name in wset:
                    return f"cur_{c}_{a.name}" if dk == 0 else f"prev_{c}_{a.name}"
                if outer_acc is not None:
                    return outer_acc(a)
                if pipe is not None and (di, dj) == (0, 0) and a.name not in written_in_group:
                    kind = "f" if a.name in p.fields else "t"
                    if kind == "f" or p.temps[a.name].storage == "hbm":
                        return pipe.col(kind, a.name, dk) + "_cur"
                if a.name in p.fields:
                    return self.gld_field(a.name, f"i + ({di})", f"j + ({dj})", f"k + ({dk})")
                if p.temps[a.name].storage != "hbm":
                    raise CodegenError(f"{a.name} read outside its computation")
                return self.gld_temp(a.name, f"i + ({di})", f"j + ({dj})", f"k + ({dk})")

            def store(name, v):
                res = [f"cur_{c}_{name} = {v};"]
                if name in p.fields:
                    res.append(f"if (i >= 0 && i < A.ni && j >= 0 && j < A.nj) A.f_{name}[(int64_t)i + "
                               f"(int64_t)j * A.f_{name}_sj + (int64_t)k * A.f_{name}_sk] = {v};")
                elif p.temps[name].storage == "hbm":
                    res.append(f"if ({self.t_inside(name, 'i', 'j')}) A.t_{name}[(int64_t)i + (int64_t)j * "
                               f"A.t_{name}_sj + (int64_t)k * A.t_{name}_sk] = {v};")
                return res

            for s_ in stmts:
                out += ["  " + l for l in self.stmt_code(s_, acc, store)]
            out.append("}")
        if cp.kcache:
            out.append("if (done) {")
            for v in cp.kcache:
                out.append(f"  prev_{c}_{v} = cur_{c}_{v};")
            out.append("}")
        return out

    def level_loop(self, order, lo, hi, body, pipe, I, J, valid_lane="true"):
        """A level loop (upwards or downwards) with its register pipeline:
        the first level's values before the loop, the next level's loaded at
        the top of every level, rotated at its end."""
        up = order != ir.BACKWARD
        k0 = f"({lo})" if up else f"({hi}) - 1"
        out = self.pipe_decls(pipe)
        out += self.pipe_lines(pipe, I, J, k0, f"({lo}) < ({hi}) && ({valid_lane})", "cur")
        out += [f"for (int s = 0; s < ({hi}) - ({lo}); ++s) {{",
                f"  const int k = {f'({lo}) + s' if up else f'({hi}) - 1 - s'};",
                f"  const int kn = {'k + 1' if up else 'k - 1'};"]
        out += ["  " + l for l in self.pipe_lines(pipe, I, J, "kn", f"s + 1 < ({hi}) - ({lo}) && ({valid_lane})", "nxt",
                                                  1 if up else -1)]
        out += ["  " + l for l in body]
        out += ["  " + l for l in self.pipe_rotate(pipe)]
        out.append("}")
        return out

    # ------------------------------------------------------------ kernels
    def group_kernel(self, gi, g):
        p = self.p
        members = [p.comps[c] for c in g]
        prun = [cp for cp in members if cp.order == ir.PARALLEL]
        seqs = [cp for cp in members if cp.order != ir.PARALLEL]
        written = set()
        for cp in members:
            written |= set(cp.writes)
        L = [f"__global__ void __launch_bounds__(256) gts_g{gi}(Args A) {{"]
        if not prun:
            # sweeps only: one lane per column of the region
            r = seqs[0].region
            L += [f"  const int i = (int)blockIdx.x * 64 + (int)(threadIdx.x & 63) + ({r[0]});",
                  f"  const int j = (int)blockIdx.y * 4 + (int)(threadIdx.x >> 6) + ({r[2]});",
                  f"  if (i >= A.ni + ({r[1]}) || j >= A.nj + ({r[3]})) return;"]
            for n, cp in enumerate(seqs):
                L += ["  " + l for l in self.seq_decls(cp)]
                pipe = _Gen._Pipe(f"{gi}_{n}")
                # later sweeps of the group run after this lane finished the earlier ones
                body = self.seq_level(cp, None, pipe, set(cp.writes) | {w for c in seqs[n + 1:] for w in c.writes})
                L += ["  {"] + ["    " + l for l in self.level_loop(cp.order, f"A.clo[{cp.index}]", f"A.chi[{cp.index}]",
                                                                       body, pipe, "i", "j")] + ["  }"]
            L.append("}")
            return "\n".join(L)
        # the run's temporaries held in LDS: those read by the run or the first sweep
        readers = {a.name for cp in prun + seqs[:1] for a in _reads(cp)}
        lds = list(dict.fromkeys(t for cp in prun for t in cp.writes if t in p.temps and t in readers))
        pipe = _Gen._Pipe(f"{gi}")
        boxes, decls = self.tile_decls(prun, lds, pipe)
        L += ["  const int tid = threadIdx.x;",
              f"  const int tiles_i = (A.ni + {TI - 1}) / {TI};",
              f"  const int i0 = (int)(blockIdx.x % tiles_i) * {TI}, j0 = (int)(blockIdx.x / tiles_i) * {TJ};",
              f"  const int i = i0 + (tid & {TI - 1}), j = j0 + tid / {TI};",
              "  const bool act = i < A.ni && j < A.nj;"]
        L += decls
        for cp in seqs:
            L += ["  " + l for l in self.seq_decls(cp)]
        sync = _Gen._Sync()
        body = []
        for cp in prun:
            lines, sync = self.par_level(cp, boxes, pipe, sync, written)
            body += lines
        if seqs:
            S = seqs[0]
            zero = (0, 0, 0, 0)
            rd = [(f"L_{a.name}", (a.offset[0], a.offset[1])) for a in _reads(S)
                  if ("L", a.name) in boxes and a.offset[2] == 0]
            if sync.need(rd, [], zero):
                body.append("__syncthreads();")
                sync.clear()
            inner = self.seq_level(S, self._tile_acc(-1, boxes, "i", "j", pipe, written), pipe, written)
            body += ["if (act) {"] + ["  " + l for l in inner] + ["}"]
        body.append("__syncthreads();")  # the next level overwrites the boxes
        if seqs:
            L += ["  " + l for l in self.level_loop(seqs[0].order, f"A.glo[{gi}]", f"A.ghi[{gi}]", body, pipe,
                                                     "i", "j")]
            for n, cp in enumerate(seqs[1:]):
                p2 = _Gen._Pipe(f"{gi}_{n + 1}")
                # everything earlier members wrote is complete for this column
                # (this lane's sweep, or other lanes before the last barrier)
                inner = self.seq_level(cp, None, p2, set(cp.writes))
                L += ["  if (act) {"] + ["    " + l for l in self.level_loop(cp.order, f"A.clo[{cp.index}]",
                                                                                f"A.chi[{cp.index}]", inner, p2,
                                                                                "i", "j")] + ["  }"]
        else:
            L += ["  const int kbeg = blockIdx.y * A.kchunk, kend = min(kbeg + A.kchunk, A.nk);"]
            L += ["  " + l for l in self.level_loop(ir.FORWARD, "kbeg", "kend", body, pipe, "i", "j")]
        L.append("}")
        return "\n".join(L)

    # ------------------------------------------------------------ host side
    def host(self):
        p = self.p
        sd = p.sdef
        nf, ns = len(sd.fields), len(sd.scalars)
        L = []
        L.append("static int bound(int nk, int none, int v, int dflt) {")
        L.append("  int x = none ? dflt : (v >= 0 ? v : nk + v);")
        L.append("  return x < 0 ? 0 : (x > nk ? nk : x);")
        L.append("}")
        L.append("static size_t r256(size_t b) { return (b + 255) & ~(size_t)255; }")
        # workspace
        L.append("static size_t ws_bytes(int64_t ni, int64_t nj, int64_t nk) {")
        L.append("  size_t b = 0;")
        for t in self.hbm:
            e = t.ext
            L.append(f"  b += r256(sizeof(real) * (size_t)(ni + {e[1] - e[0]}) * (size_t)(nj + {e[3] - e[2]}) * (size_t)nk);")
        L.append("  return b;")
        L.append("}")
        L.append('extern "C" size_t gts_workspace_bytes(const int64_t domain[3]) {')
        L.append("  if (!domain || domain[0] < 0 || domain[1] < 0 || domain[2] < 0) return 0;")
        L.append("  return ws_bytes(domain[0], domain[1], domain[2]);")
        L.append("}")
        sig = f"{sd.name}|{','.join(sd.fields)}|{','.join(sd.scalars)}|{self.dtype}|{self.fp}"
        L.append(f'extern "C" const char* gts_signature(void) {{ return "{sig}"; }}')
        L.append('extern "C" const char* gts_last_error(void) { return g_err; }')
        L.append('extern "C" int gts_run(const gts_field* fields, int nfields, const double* scalars, int nscalars,')
        L.append("                       const int64_t domain[3], void* workspace, size_t workspace_bytes, hipStream_t stream) {")
        L.append("  g_err[0] = 0;")
        L.append(f"  if (nfields != {nf}) return fail(GTS_E_ARG, \"%d fields given, the stencil takes {nf}\", nfields);")
        L.append(f"  if (nscalars != {ns}) return fail(GTS_E_ARG, \"%d scalars given, the stencil takes {ns}\", nscalars);")
        if nf:
            L.append("  if (!fields) return fail(GTS_E_NULL, \"fields is NULL\");")
        if ns:
            L.append("  if (!scalars) return fail(GTS_E_NULL, \"scalars is NULL\");")
        L.append("  if (!domain) return fail(GTS_E_NULL, \"domain is NULL\");")
        L.append("  const int64_t ni = domain[0], nj = domain[1], nk = domain[2];")
        L.append("  if (ni < 0 || nj < 0 || nk < 0 || ni > (1 << 30) || nj > (1 << 30) || nk > (1 << 30))")
        L.append("    return fail(GTS_E_ARG, \"domain out of range\");")
        L.append("  Args A;")
        L.append("  memset(&A, 0, sizeof A);")
        L.append("  A.ni = (int)ni; A.nj = (int)nj; A.nk = (int)nk;")
        # block bounds
        for cp in p.comps:
            for bi, (iv, _) in enumerate(cp.blocks):
                b = self.bidx[(cp.index, bi)]
                s0 = 1 if iv.start is None else 0
                s1 = 1 if iv.end is None else 0
                L.append(f"  A.blo[{b}] = bound((int)nk, {s0}, {iv.start or 0}, 0);")
                L.append(f"  A.bhi[{b}] = bound((int)nk, {s1}, {iv.end or 0}, (int)nk);")
                L.append(f"  if (A.bhi[{b}] < A.blo[{b}]) A.bhi[{b}] = A.blo[{b}];")
        # per computation: overlap check and level range
        for cp in p.comps:
            bs = [self.bidx[(cp.index, bi)] for bi in range(len(cp.blocks))]
            L.append(f"  A.clo[{cp.index}] = (int)nk; A.chi[{cp.index}] = 0;")
            for x in bs:
                L.append(f"  if (A.blo[{x}] < A.bhi[{x}]) {{ A.clo[{cp.index}] = imin(A.clo[{cp.index}], A.blo[{x}]); "
                         f"A.chi[{cp.index}] = imax(A.chi[{cp.index}], A.bhi[{x}]); }}")
            for a in range(len(bs)):
                for b2 in range(a + 1, len(bs)):
                    x, y = bs[a], bs[b2]
                    L.append(f"  if (A.blo[{x}] < A.bhi[{x}] && A.blo[{y}] < A.bhi[{y}] && A.blo[{x}] < A.bhi[{y}] && "
                             f"A.blo[{y}] < A.bhi[{x}]) return fail(GTS_E_LEVELS, \"computation {cp.index}: intervals overlap\");")
            for bi, name in cp.prev_reads:
                x = self.bidx[(cp.index, bi)]
                lvl = f"A.blo[{x}] - 1" if cp.order == ir.FORWARD else f"A.bhi[{x}]"
                cov = " || ".join(f"({lvl} >= A.blo[{y}] && {lvl} < A.bhi[{y}])" for y in bs if y != x) or "false"
                L.append(f"  if (A.blo[{x}] < A.bhi[{x}] && !({cov})) return fail(GTS_E_LEVELS, "
                         f"\"{name}: the sweep reads a level it has not computed\");")
        for ci, bi, name, dk in p.temp_kreads:
            x = self.bidx[(ci, bi)]
            L.append(f"  if (A.blo[{x}] < A.bhi[{x}] && (A.blo[{x}] + ({dk}) < 0 || A.bhi[{x}] + ({dk}) > (int)nk)) "
                     f"return fail(GTS_E_LEVELS, \"temporary {name} read outside its levels\");")
        L.append("  if (ni == 0 || nj == 0 || nk == 0) return GTS_OK;")
        # fields
        for fi, f in enumerate(sd.fields):
            info = p.fields[f]
            e = info.ext if info.read else (0, 0, 0, 0)
            L.append(f"  {{ const gts_field* F = &fields[{fi}];")
            L.append(f"    if (!F->data) return fail(GTS_E_NULL, \"field {f}: data is NULL\");")
            L.append(f"    if (F->stride[0] != 1 || F->lo[0] < 0 || F->lo[1] < 0 || F->lo[2] < 0 || "
                     f"F->stride[1] < F->lo[0] + F->hi[0] || F->stride[2] < F->stride[1] * (F->lo[1] + F->hi[1]))")
            L.append(f"      return fail(GTS_E_STRIDE, \"field {f}: bad strides or extents\");")
            L.append(f"    if (F->lo[0] < {-e[0]} || F->hi[0] < ni + {e[1]} || F->lo[1] < {-e[2]} || F->hi[1] < nj + {e[3]})")
            L.append(f"      return fail(GTS_E_HALO, \"field {f}: needs [%lld, %lld) x [%lld, %lld)\", "
                     f"(long long){e[0]}, (long long)(ni + {e[1]}), (long long){e[2]}, (long long)(nj + {e[3]}));")
            if info.written:
                L.append(f"    if (F->hi[2] < nk) return fail(GTS_E_HALO, \"field {f}: fewer than nk levels\");")
            for ci, bi, dk in info.kreads:
                x = self.bidx[(ci, bi)]
                L.append(f"    if (A.blo[{x}] < A.bhi[{x}] && (A.blo[{x}] + ({dk}) < -F->lo[2] || A.bhi[{x}] + ({dk}) > F->hi[2]))")
                L.append(f"      return fail(GTS_E_HALO, \"field {f}: levels read beyond the field\");")
            L.append(f"    A.f_{f} = (real*)F->data; A.f_{f}_sj = F->stride[1]; A.f_{f}_sk = F->stride[2];")
            L.append(f"    A.f_{f}_klo = F->lo[2]; A.f_{f}_khi = F->hi[2]; }}")
        for si, s in enumerate(sd.scalars):
            L.append(f"  A.s_{s} = (real)scalars[{si}];")
        L.append("  const size_t need = ws_bytes(ni, nj, nk);")
        L.append("  if (need) {")
        L.append("    if (!workspace) return fail(GTS_E_NULL, \"workspace is NULL (%zu bytes needed)\", need);")
        L.append("    if (workspace_bytes < need || ((uintptr_t)workspace & 255))")
        L.append("      return fail(GTS_E_WORKSPACE, \"workspace of %zu bytes (256-byte aligned) needed\", need);")
        L.append("  }")
        L.append("  char* wp = (char*)workspace;")
        for t in self.hbm:
            e = t.ext
            L.append(f"  A.t_{t.name}_sj = ni + {e[1] - e[0]}; A.t_{t.name}_sk = A.t_{t.name}_sj * (nj + {e[3] - e[2]});")
            L.append(f"  A.t_{t.name} = (real*)wp + ({-e[0]}) + ({-e[2]}) * A.t_{t.name}_sj;")
            L.append(f"  wp += r256(sizeof(real) * (size_t)A.t_{t.name}_sk * (size_t)nk);")
        for gi, g in enumerate(p.groups):
            members = [p.comps[c] for c in g]
            prun = [cp for cp in members if cp.order == ir.PARALLEL]
            seqs = [cp for cp in members if cp.order != ir.PARALLEL]
            if prun and not seqs:
                L += ["  {",
                      f"    const int tiles = (int)(((ni + {TI - 1}) / {TI}) * ((nj + {TJ - 1}) / {TJ}));",
                      "    int kc = (int)nk;",
                      f"    while (kc > 1 && (int64_t)tiles * ((nk + kc - 1) / kc) < {MIN_WGS}) kc = (kc + 1) / 2;",
                      "    A.kchunk = kc;",
                      f"    hipLaunchKernelGGL(gts_g{gi}, dim3(tiles, (unsigned)((nk + kc - 1) / kc)), dim3(256), 0, stream, A);",
                      "  }"]
            elif prun:
                sweep = [cp for cp in prun] + seqs[:1]
                L.append(f"  A.glo[{gi}] = (int)nk; A.ghi[{gi}] = 0;")
                for cp in sweep:
                    L.append(f"  if (A.clo[{cp.index}] < A.chi[{cp.index}]) {{ A.glo[{gi}] = imin(A.glo[{gi}], "
                             f"A.clo[{cp.index}]); A.ghi[{gi}] = imax(A.ghi[{gi}], A.chi[{cp.index}]); }}")
                L += [f"  if (A.glo[{gi}] < A.ghi[{gi}] || " + " || ".join(f"A.clo[{cp.index}] < A.chi[{cp.index}]" for cp in seqs) + ") {",
                      f"    const int tiles = (int)(((ni + {TI - 1}) / {TI}) * ((nj + {TJ - 1}) / {TJ}));",
                      f"    hipLaunchKernelGGL(gts_g{gi}, dim3(tiles), dim3(256), 0, stream, A);",
                      "  }"]
            else:
                r = seqs[0].region
                cond = " || ".join(f"A.clo[{cp.index}] < A.chi[{cp.index}]" for cp in seqs)
                L += [f"  if ({cond}) {{",
                      f"    const int64_t W = ni + {r[1] - r[0]}, H = nj + {r[3] - r[2]};",
                      f"    hipLaunchKernelGGL(gts_g{gi}, dim3((unsigned)((W + 63) / 64), (unsigned)((H + 3) / 4)), dim3(256), 0, stream, A);",
                      "  }"]
        L.append("  hipError_t e = hipGetLastError();")
        L.append("  if (e != hipSuccess) return fail(GTS_E_HIP, \"launch: %s\", hipGetErrorString(e));")
        L.append("  return GTS_OK;")
        L.append("}")
        return "\n".join(L)

    def source(self):
        p = self.p
        sd = p.sdef
        head = [f"// generated by the stencil frontend (generator version {GEN_VERSION}) from `{sd.name}`;",
                f"// fingerprint {self.fp}, dtype {self.dtype}.  Do not edit: regenerated from the definition.",
                "#include <hip/hip_runtime.h>",
                "#include <math.h>",
                "#include <stdarg.h>",
                "#include <stdint.h>",
                "#include <stdio.h>",
                "#include <string.h>",
                '#include "gtscript_abi.h"',
                f"typedef {self.real} real;",
                "static thread_local char g_err[512];",
                "static int fail(int code, const char* fmt, ...) {",
                "  va_list ap; va_start(ap, fmt); vsnprintf(g_err, sizeof g_err, fmt, ap); va_end(ap); return code;",
                "}",
                "static inline int imin(int a, int b) { return a < b ? a : b; }",
                "static inline int imax(int a, int b) { return a > b ? a : b; }",
                "__device__ __forceinline__ real gld(const real* p, int64_t sj, int64_t sk, int i, int j, int k, bool ok) {",
                "  return ok ? p[(int64_t)i + (int64_t)j * sj + (int64_t)k * sk] : (real)0;",
                "}",
                "struct Args {"]
        for f in sd.fields:
            head.append(f"  real* f_{f}; int64_t f_{f}_sj, f_{f}_sk, f_{f}_klo, f_{f}_khi;")
        for t in self.hbm:
            head.append(f"  real* t_{t.name}; int64_t t_{t.name}_sj, t_{t.name}_sk;")
        for s in sd.scalars:
            head.append(f"  real s_{s};")
        head += ["  int ni, nj, nk, kchunk;",
                 f"  int blo[{max(1, self.nblocks)}], bhi[{max(1, self.nblocks)}];",
                 f"  int clo[{max(1, len(p.comps))}], chi[{max(1, len(p.comps))}];",
                 f"  int glo[{max(1, len(p.groups))}], ghi[{max(1, len(p.groups))}];",
                 "};"]
        body = [self.group_kernel(gi, g) for gi, g in enumerate(p.groups)]
        return "\n".join(head) + "\n\n" + "\n\n".join(body) + "\n\n" + self.host() + "\n"


def generate(plan: Plan, dtype: str, fingerprint: str) -> str:
    if dtype not in ("float64", "float32"):
        raise CodegenError(f"dtype {dtype} unsupported (float64, float32)")
    return _Gen(plan, dtype, fingerprint).source()
