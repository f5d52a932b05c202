"""Intermediate representations of the stencil frontend.

Definition IR: what the user wrote, after parsing (GT4Py paper, Sec. 2.3:
frontends produce a definition IR; analysis lowers it towards the parallel
model of the implementation).  Trees of frozen dataclasses, so that their
``repr`` is a canonical text: the fingerprint of a stencil hashes that text,
which is why reformatting or comments never change it.

Expressions
  Const(value)                 a number (externals are folded to these)
  Access(name, offset)         a field or temporary at an (i, j, k) offset
  Scalar(name)                 a read-only scalar parameter
  Unary(op, a), Binary(op, a, b), Compare(op, a, b), BoolOp(op, a, b)
  Ternary(cond, a, b)          a if cond else b, per point
  Builtin(name, args)          abs, min, max, sqrt, exp, log
Statements
  Assign(target, value)        per point over the whole iteration space
  If(cond, then, orelse)       per point
Structure
  Interval(start, end)         vertical range; ints count from the bottom,
                               negative ints from the top, None = the end
  Computation(order, blocks)   blocks: [(Interval, [statements])]
  StencilDef(name, fields, scalars, computations)
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import Optional, Tuple, Union

PARALLEL, FORWARD, BACKWARD = "PARALLEL", "FORWARD", "BACKWARD"


@dataclass(frozen=True)
class Const:
    value: float


@dataclass(frozen=True)
class Access:
    name: str
    offset: Tuple[int, int, int] = (0, 0, 0)


@dataclass(frozen=True)
class Scalar:
    name: str


@dataclass(frozen=True)
class Unary:
    op: str  # "-" or "not"
    a: "Expr"


@dataclass(frozen=True)
class Binary:
    op: str  # + - * /
    a: "Expr"
    b: "Expr"


@dataclass(frozen=True)
class Compare:
    op: str  # < <= > >= == !=
    a: "Expr"
    b: "Expr"


@dataclass(frozen=True)
class BoolOp:
    op: str  # and, or
    a: "Expr"
    b: "Expr"


@dataclass(frozen=True)
class Ternary:
    cond: "Expr"
    a: "Expr"
    b: "Expr"


@dataclass(frozen=True)
class Builtin:
    name: str
    args: Tuple["Expr", ...]


Expr = Union[Const, Access, Scalar, Unary, Binary, Compare, BoolOp, Ternary, Builtin]


@dataclass(frozen=True)
class Assign:
    target: str
    value: Expr


@dataclass(frozen=True)
class If:
    cond: Expr
    then: Tuple["Stmt", ...]
    orelse: Tuple["Stmt", ...]


Stmt = Union[Assign, If]


@dataclass(frozen=True)
class Interval:
    start: Optional[int]  # None: 0
    end: Optional[int]    # None: nk

    def bounds(self, nk: int):
        """[lo, hi) in levels for a domain of nk levels."""
        def at(v, default):
            if v is None:
                return default
            return v if v >= 0 else nk + v
        return max(0, at(self.start, 0)), min(nk, at(self.end, nk))


@dataclass(frozen=True)
class Computation:
    order: str
    blocks: Tuple[Tuple[Interval, Tuple[Stmt, ...]], ...]


@dataclass(frozen=True)
class StencilDef:
    name: str
    fields: Tuple[str, ...]   # API fields, in signature order
    scalars: Tuple[str, ...]  # read-only scalar parameters, in signature order
    computations: Tuple[Computation, ...]


# ------------------------------------------------------------------ walkers
def expr_children(e):
    if isinstance(e, (Unary,)):
        return (e.a,)
    if isinstance(e, (Binary, Compare, BoolOp)):
        return (e.a, e.b)
    if isinstance(e, Ternary):
        return (e.cond, e.a, e.b)
    if isinstance(e, Builtin):
        return e.args
    return ()


def accesses(e):
    """Every Access in an expression tree."""
    if isinstance(e, Access):
        yield e
    for c in expr_children(e):
        yield from accesses(c)


def stmt_accesses(s):
    """(reads, writes) of a statement: reads as Access nodes, writes as names."""
    if isinstance(s, Assign):
        return list(accesses(s.value)), [s.target]
    reads = list(accesses(s.cond))
    writes = []
    for t in s.then + s.orelse:
        r, w = stmt_accesses(t)
        reads += r
        writes += w
    return reads, writes
