"""GTScript-like Python functions -> definition IR.

The language is a strict subset of Python syntax, parsed with the standard
``ast`` module (GT4Py paper, Sec. 2.2): a stencil is a function whose
parameters are fields (annotated ``Field``) and read-only scalars (any other
annotation, or keyword-only), and whose body is a sequence of
``with computation(ORDER)`` blocks, each holding ``with interval(start, end)``
blocks (or ``with computation(ORDER), interval(...)`` for a single one).
Inside an interval: assignments to a name and if/else, with the usual
arithmetic, comparisons, boolean operators, conditional expressions and the
builtins abs/min/max/sqrt/exp/log.  ``name[di, dj, dk]`` reads a field or a
temporary at an offset from the point being computed.  A name first seen on
the left of an assignment is a temporary field.  Calls to ``@function``
objects are inlined (arguments substituted, offsets composed); names in the
``externals`` mapping are compile-time constants.
"""
from __future__ import annotations

import ast
import inspect
import textwrap

from . import ir

BUILTINS = {"abs": 1, "min": 2, "max": 2, "sqrt": 1, "exp": 1, "log": 1}
ORDERS = {"PARALLEL": ir.PARALLEL, "FORWARD": ir.FORWARD, "BACKWARD": ir.BACKWARD}


class GTScriptSyntaxError(SyntaxError):
    pass


def _err(node, msg):
    line = getattr(node, "lineno", "?")
    return GTScriptSyntaxError(f"line {line}: {msg}")


def function_ast(fn):
    src = textwrap.dedent(inspect.getsource(fn))
    mod = ast.parse(src)
    fdef = mod.body[0]
    if not isinstance(fdef, ast.FunctionDef):
        raise GTScriptSyntaxError(f"{fn.__name__}: not a function definition")
    return fdef


def _is_field_annotation(a):
    if a is None:
        return False
    if isinstance(a, ast.Name):
        return a.id == "Field"
    if isinstance(a, ast.Subscript):
        return _is_field_annotation(a.value)
    if isinstance(a, ast.Attribute):
        return a.attr == "Field"
    if isinstance(a, ast.Constant) and isinstance(a.value, str):
        return a.value.startswith("Field")
    return False


def _int_of(node):
    if isinstance(node, ast.Constant) and isinstance(node.value, int) and not isinstance(node.value, bool):
        return node.value
    if isinstance(node, ast.UnaryOp) and isinstance(node.op, (ast.USub, ast.UAdd)):
        v = _int_of(node.operand)
        if v is not None:
            return -v if isinstance(node.op, ast.USub) else v
    return None


class _Scope:
    """Name bindings while lowering one stencil or one inlined function."""

    def __init__(self, fields, scalars, externals, functions, temps, binds=None):
        self.fields = fields
        self.scalars = scalars
        self.externals = externals
        self.functions = functions  # name -> Function object (inlined)
        self.temps = temps          # set of temporaries assigned so far (shared)
        self.binds = binds or {}    # function params / locals -> Expr


def _shift(e, off, node):
    if off == (0, 0, 0):
        return e
    if isinstance(e, ir.Access):
        return ir.Access(e.name, tuple(a + b for a, b in zip(e.offset, off)))
    raise _err(node, "an offset applies to a field argument only, not to an expression")


class _Lower:
    def __init__(self, scope: _Scope):
        self.s = scope

    # ---------------------------------------------------------- expressions
    def expr(self, n):
        s = self.s
        if isinstance(n, ast.Constant):
            if isinstance(n.value, bool) or not isinstance(n.value, (int, float)):
                raise _err(n, f"unsupported constant {n.value!r}")
            return ir.Const(float(n.value))
        if isinstance(n, ast.Name):
            return self.name(n.id, n)
        if isinstance(n, ast.Subscript):
            if not isinstance(n.value, ast.Name):
                raise _err(n, "only a name can be indexed")
            idx = n.slice
            elts = idx.elts if isinstance(idx, ast.Tuple) else [idx]
            off = tuple(_int_of(e) for e in elts)
            if len(off) != 3 or any(o is None for o in off):
                raise _err(n, "an offset is three integer constants [di, dj, dk]")
            return _shift(self.name(n.value.id, n), off, n)
        if isinstance(n, ast.UnaryOp):
            a = self.expr(n.operand)
            if isinstance(n.op, ast.USub):
                return ir.Const(-a.value) if isinstance(a, ir.Const) else ir.Unary("-", a)
            if isinstance(n.op, ast.UAdd):
                return a
            if isinstance(n.op, ast.Not):
                return ir.Unary("not", a)
            raise _err(n, "unsupported unary operator")
        if isinstance(n, ast.BinOp):
            ops = {ast.Add: "+", ast.Sub: "-", ast.Mult: "*", ast.Div: "/"}
            if isinstance(n.op, ast.Pow):
                p = _int_of(n.right)
                if p is None or not 1 <= p <= 4:
                    raise _err(n, "only small integer powers (1..4) are supported")
                a = self.expr(n.left)
                r = a
                for _ in range(p - 1):
                    r = ir.Binary("*", r, a)
                return r
            op = ops.get(type(n.op))
            if op is None:
                raise _err(n, "unsupported binary operator")
            return ir.Binary(op, self.expr(n.left), self.expr(n.right))
        if isinstance(n, ast.Compare):
            if len(n.ops) != 1:
                raise _err(n, "chained comparisons are not supported")
            ops = {ast.Lt: "<", ast.LtE: "<=", ast.Gt: ">", ast.GtE: ">=", ast.Eq: "==", ast.NotEq: "!="}
            op = ops.get(type(n.ops[0]))
            if op is None:
                raise _err(n, "unsupported comparison")
            return ir.Compare(op, self.expr(n.left), self.expr(n.comparators[0]))
        if isinstance(n, ast.BoolOp):
            op = "and" if isinstance(n.op, ast.And) else "or"
            vals = [self.expr(v) for v in n.values]
            r = vals[0]
            for v in vals[1:]:
                r = ir.BoolOp(op, r, v)
            return r
        if isinstance(n, ast.IfExp):
            return ir.Ternary(self.expr(n.test), self.expr(n.body), self.expr(n.orelse))
        if isinstance(n, ast.Call):
            if not isinstance(n.func, ast.Name) or n.keywords:
                raise _err(n, "calls are name(args) without keywords")
            fname = n.func.id
            args = [self.expr(a) for a in n.args]
            if fname in s.functions:
                return inline(s.functions[fname], args, s, n)
            if fname in BUILTINS:
                if len(args) != BUILTINS[fname]:
                    raise _err(n, f"{fname} takes {BUILTINS[fname]} argument(s)")
                return ir.Builtin(fname, tuple(args))
            raise _err(n, f"unknown function {fname}")
        raise _err(n, f"unsupported expression {type(n).__name__}")

    def name(self, nm, node):
        s = self.s
        if nm in s.binds:
            return s.binds[nm]
        if nm in s.fields or nm in s.temps:
            return ir.Access(nm)
        if nm in s.scalars:
            return ir.Scalar(nm)
        if nm in s.externals:
            v = s.externals[nm]
            if isinstance(v, bool) or not isinstance(v, (int, float)):
                raise _err(node, f"external {nm} is not a number")
            return ir.Const(float(v))
        raise _err(node, f"undefined name {nm} (not a field, scalar, external or earlier temporary)")

    # ---------------------------------------------------------- statements
    def stmts(self, body):
        out = []
        for st in body:
            if isinstance(st, ast.Expr) and isinstance(st.value, ast.Constant):
                continue  # docstring / string comment
            if isinstance(st, ast.Pass):
                continue
            if isinstance(st, ast.Assign):
                if len(st.targets) != 1 or not isinstance(st.targets[0], ast.Name):
                    raise _err(st, "assign to one plain name (no offsets on the left)")
                t = st.targets[0].id
                if t in self.s.scalars or t in self.s.externals:
                    raise _err(st, f"{t} is read-only")
                value = self.expr(st.value)
                if t not in self.s.fields:
                    self.s.temps.add(t)
                out.append(ir.Assign(t, value))
            elif isinstance(st, ast.AugAssign) and isinstance(st.target, ast.Name):
                ops = {ast.Add: "+", ast.Sub: "-", ast.Mult: "*", ast.Div: "/"}
                op = ops.get(type(st.op))
                if op is None:
                    raise _err(st, "unsupported augmented assignment")
                t = st.target.id
                out.append(ir.Assign(t, ir.Binary(op, self.name(t, st), self.expr(st.value))))
            elif isinstance(st, ast.If):
                cond = self.expr(st.test)
                out.append(ir.If(cond, tuple(self.stmts(st.body)), tuple(self.stmts(st.orelse))))
            else:
                raise _err(st, f"unsupported statement {type(st).__name__} inside an interval")
        return out


def inline(func, args, scope: _Scope, node):
    """Substitute the arguments into a @function body: assignments to its
    locals become bindings, the returned expression is the value."""
    fdef = func.ast
    params = [a.arg for a in fdef.args.args]
    if len(params) != len(args):
        raise _err(node, f"{func.name} takes {len(params)} argument(s), got {len(args)}")
    inner = _Scope(scope.fields, scope.scalars, scope.externals, scope.functions, scope.temps,
                   dict(zip(params, args)))
    low = _Lower(inner)
    for st in fdef.body:
        if isinstance(st, ast.Expr) and isinstance(st.value, ast.Constant):
            continue
        if isinstance(st, ast.Assign) and len(st.targets) == 1 and isinstance(st.targets[0], ast.Name):
            inner.binds[st.targets[0].id] = low.expr(st.value)
        elif isinstance(st, ast.Return) and st.value is not None:
            return low.expr(st.value)
        else:
            raise _err(st, f"{func.name}: a function holds assignments and one return")
    raise _err(node, f"{func.name} returns nothing")


def _parse_interval(call, node):
    if not (isinstance(call, ast.Call) and isinstance(call.func, ast.Name) and call.func.id == "interval"):
        raise _err(node, "expected interval(...)")
    a = call.args
    if len(a) == 1 and isinstance(a[0], ast.Constant) and a[0].value is Ellipsis:
        return ir.Interval(None, None)
    if len(a) != 2:
        raise _err(node, "interval(start, end) or interval(...)")
    bounds = []
    for x in a:
        if isinstance(x, ast.Constant) and x.value is None:
            bounds.append(None)
        else:
            v = _int_of(x)
            if v is None:
                raise _err(node, "interval bounds are integer constants or None")
            bounds.append(v)
    return ir.Interval(*bounds)


def _parse_order(call, node):
    if not (isinstance(call, ast.Call) and isinstance(call.func, ast.Name) and call.func.id == "computation"
            and len(call.args) == 1 and isinstance(call.args[0], ast.Name) and call.args[0].id in ORDERS):
        raise _err(node, "expected computation(PARALLEL | FORWARD | BACKWARD)")
    return ORDERS[call.args[0].id]


def parse_stencil(fn, externals=None, functions=None) -> ir.StencilDef:
    fdef = function_ast(fn)
    externals = dict(externals or {})
    functions = dict(functions or {})
    fields, scalars = [], []
    for a in fdef.args.args:
        (fields if _is_field_annotation(a.annotation) else scalars).append(a.arg)
    for a in fdef.args.kwonlyargs:
        if _is_field_annotation(a.annotation):
            raise _err(fdef, f"field {a.arg} must be positional")
        scalars.append(a.arg)
    if fdef.args.vararg or fdef.args.kwarg:
        raise _err(fdef, "no *args / **kwargs")
    scope = _Scope(set(fields), set(scalars), externals, functions, set())
    low = _Lower(scope)
    comps = []
    for st in fdef.body:
        if isinstance(st, ast.Expr) and isinstance(st.value, ast.Constant):
            continue
        if not isinstance(st, ast.With):
            raise _err(st, "the body is a sequence of `with computation(...)` blocks")
        items = [it.context_expr for it in st.items]
        order = _parse_order(items[0], st)
        if len(items) == 2:
            iv = _parse_interval(items[1], st)
            comps.append(ir.Computation(order, ((iv, tuple(low.stmts(st.body))),)))
        elif len(items) == 1:
            blocks = []
            for sub in st.body:
                if isinstance(sub, ast.Expr) and isinstance(sub.value, ast.Constant):
                    continue
                if not (isinstance(sub, ast.With) and len(sub.items) == 1):
                    raise _err(sub, "a computation holds `with interval(...)` blocks")
                iv = _parse_interval(sub.items[0].context_expr, sub)
                blocks.append((iv, tuple(low.stmts(sub.body))))
            comps.append(ir.Computation(order, tuple(blocks)))
        else:
            raise _err(st, "with computation(ORDER)[, interval(...)]")
    if not comps:
        raise _err(fdef, "a stencil needs at least one computation")
    return ir.StencilDef(fdef.name, tuple(fields), tuple(scalars), tuple(comps))
