"""The stencil frontend without a GPU: parsing into the definition IR,
the language rules, extents and storage of the benchmark stencils, the
fingerprint (unchanged by reformatting, changed by any semantic edit),
inlining and externals, the generated library compiling for gfx950 and its
C ABI refusing bad calls before any device work."""
import ctypes
import textwrap

import pytest

from paper_2311_08322_amd import frontend as F
from paper_2311_08322_amd.frontend import build as B
from paper_2311_08322_amd.frontend import ir
from paper_2311_08322_amd.frontend import stencils as S


def _define(src, externals=None, extra=None):
    """A stencil from source text (exec'd in a fresh namespace)."""
    ns = {"Field": F.Field, "computation": F.computation, "interval": F.interval, "PARALLEL": F.PARALLEL,
          "FORWARD": F.FORWARD, "BACKWARD": F.BACKWARD, "function": F.function}
    ns.update(extra or {})
    import linecache
    fname = f"<stencil-{abs(hash(src))}>"
    linecache.cache[fname] = (len(src), None, src.splitlines(True), fname)
    exec(compile(textwrap.dedent(src), fname, "exec"), ns)
    fn = [v for k, v in ns.items() if callable(v) and getattr(v, "__name__", "") == "st"][0]
    return F.StencilObject(fn, externals)


def test_benchmark_stencil_plans():
    p = S.hdiff.plan
    assert p.fields["u"].ext == (-2, 2, -2, 2) and p.fields["out"].written
    assert {t: v.storage for t, v in p.temps.items()} == {"lap": "lds", "flx": "lds", "fly": "lds"}
    assert p.temps["lap"].ext == (-1, 1, -1, 1)
    assert p.temps["flx"].ext == (-1, 0, 0, 0) and p.temps["fly"].ext == (0, 0, -1, 0)
    v = S.vadv.plan
    assert v.fields["w"].ext == (0, 0, 0, 0)
    # one fused kernel: the coefficient computations run inside the forward
    # sweep (a, c in LDS); cp, dp cross into the backward sweep (memory)
    assert v.groups == [[0, 1, 2, 3]]
    assert {t: x.storage for t, x in v.temps.items()} == {"a": "lds", "c": "lds", "m": "reg", "cp": "hbm",
                                                         "dp": "hbm"}
    assert v.comps[2].order == F.FORWARD and set(v.comps[2].kcache) == {"cp", "dp"}
    assert v.comps[3].kcache == ["out"]
    st = S.step.plan
    assert st.groups == [[0, 1, 2, 3, 4]]
    assert st.temps["h"].storage == "lds" and st.fields["u"].ext == (-2, 2, -2, 2)


def test_inlining_composes_offsets_and_folds_externals():
    st = _define('''
        @function
        def dx(f):
            d = f[1, 0, 0] - f[-1, 0, 0]
            return d * HALF
        def st(u: Field, out: Field):
            with computation(PARALLEL), interval(...):
                out = dx(u[0, 1, 0])
    ''', externals={"HALF": 0.5})
    (c,) = st.definition.computations
    (iv, (stmt,)), = c.blocks
    assert stmt == ir.Assign("out", ir.Binary("*", ir.Binary("-", ir.Access("u", (1, 1, 0)), ir.Access("u", (-1, 1, 0))),
                                              ir.Const(0.5)))
    assert st.plan.fields["u"].ext == (-1, 1, 0, 1)  # extents always include the domain itself


BAD = {
    "self-assignment with an offset": ('''
        def st(u: Field, out: Field):
            with computation(PARALLEL), interval(...):
                t = u
                t = t[1, 0, 0] + 1.0
                out = t
    ''', F.StencilAnalysisError),
    "forward reads ahead": ('''
        def st(u: Field, out: Field):
            with computation(FORWARD), interval(...):
                t = u + t[0, 0, 1]
                out = t
    ''', F.GTScriptSyntaxError),
    "forward reads its own value ahead": ('''
        def st(u: Field, out: Field):
            with computation(PARALLEL), interval(...):
                t = u
            with computation(FORWARD), interval(...):
                t = u + t[0, 0, 1]
                out = t
    ''', F.StencilAnalysisError),
    "backward reads below": ('''
        def st(u: Field, out: Field):
            with computation(PARALLEL), interval(...):
                t = u
            with computation(BACKWARD), interval(...):
                t = u + t[0, 0, -1]
                out = t
    ''', F.StencilAnalysisError),
    "parallel vertical dependency": ('''
        def st(u: Field, out: Field):
            with computation(PARALLEL), interval(...):
                t = u
                out = t[0, 0, 1]
    ''', F.StencilAnalysisError),
    "sweep horizontal dependency": ('''
        def st(u: Field, out: Field):
            with computation(FORWARD), interval(...):
                t = u
                out = t[1, 0, 0]
    ''', F.StencilAnalysisError),
    "output read back in a parallel computation": ('''
        def st(u: Field, out: Field):
            with computation(PARALLEL), interval(...):
                out = u
                v = out * 2.0
    ''', F.StencilAnalysisError),
    "undefined name": ('''
        def st(u: Field, out: Field):
            with computation(PARALLEL), interval(...):
                out = u + nothing
    ''', F.GTScriptSyntaxError),
    "offset not constant": ('''
        def st(u: Field, out: Field, *, n: int):
            with computation(PARALLEL), interval(...):
                out = u[n, 0, 0]
    ''', F.GTScriptSyntaxError),
    "scalar written": ('''
        def st(u: Field, out: Field, *, a: float):
            with computation(PARALLEL), interval(...):
                a = u
                out = u
    ''', F.GTScriptSyntaxError),
    "unknown function": ('''
        def st(u: Field, out: Field):
            with computation(PARALLEL), interval(...):
                out = tanh(u)
    ''', F.GTScriptSyntaxError),
    "statement outside a computation": ('''
        def st(u: Field, out: Field):
            out = u
    ''', F.GTScriptSyntaxError),
}


@pytest.mark.parametrize("case", list(BAD), ids=list(BAD))
def test_language_rules(case):
    src, exc = BAD[case]
    with pytest.raises(exc):
        _define(src)


def test_fingerprint_ignores_formatting_and_tracks_semantics():
    a = _define('''
        def st(u: Field, out: Field, *, c: float):
            with computation(PARALLEL), interval(...):
                out = u - c * (u[1, 0, 0] - u)
    ''')
    b = _define('''
        def st(u   : Field,out:Field, *, c: float):
            # the same stencil, reformatted
            with computation(PARALLEL), interval(...):
                out = (u
                       - c * (u[1,0,0] - u))   # comment
    ''')
    c = _define('''
        def st(u: Field, out: Field, *, c: float):
            with computation(PARALLEL), interval(...):
                out = u + c * (u[1, 0, 0] - u)
    ''')
    assert a.fingerprint() == b.fingerprint()
    assert a.fingerprint() != c.fingerprint()
    assert a.fingerprint("float32") != a.fingerprint("float64")


def test_generated_library_compiles_and_validates():
    """The hdiff library builds for gfx950 (cross-compiled here) and its
    C ABI refuses bad calls before touching the device."""
    L = S.hdiff.build("float64")
    sig = L.gts_signature().decode()
    assert sig.startswith("hdiff|u,out|coeff|float64|")
    dom = (ctypes.c_int64 * 3)(16, 12, 4)
    fl = (B.GtsField * 2)()
    base = 0x7F0000000000
    for n, f in enumerate(fl):
        halo = 2 if n == 0 else 0
        f.data = base + (n << 32)
        f.stride[0], f.stride[1], f.stride[2] = 1, 16 + 2 * halo, (16 + 2 * halo) * (12 + 2 * halo)
        f.lo[0] = f.lo[1] = halo
        f.hi[0], f.hi[1] = 16 + halo, 12 + halo
        f.lo[2], f.hi[2] = 0, 4
    sc = (ctypes.c_double * 1)(0.025)
    assert L.gts_run(fl, 1, sc, 1, dom, None, 0, None) == -2  # GTS_E_ARG
    assert L.gts_run(fl, 2, sc, 0, dom, None, 0, None) == -2
    assert L.gts_run(fl, 2, sc, 1, None, None, 0, None) == -1  # GTS_E_NULL
    fl[0].lo[0] = 1  # halo of u too small
    assert L.gts_run(fl, 2, sc, 1, dom, None, 0, None) == -4  # GTS_E_HALO
    assert b"needs" in L.gts_last_error()
    fl[0].lo[0] = 2
    fl[1].stride[1] = 8  # rows overlap
    assert L.gts_run(fl, 2, sc, 1, dom, None, 0, None) == -3  # GTS_E_STRIDE
    fl[1].stride[1] = 16
    empty = (ctypes.c_int64 * 3)(0, 12, 4)
    assert L.gts_run(fl, 2, sc, 1, empty, None, 0, None) == 0  # nothing to do
    assert L.gts_workspace_bytes(dom) == 0  # every temporary on chip
    V = S.vadv.build("float64")
    assert V.gts_workspace_bytes(dom) == 2 * ((16 * 12 * 4 * 8 + 255) // 256 * 256)  # cp, dp


def test_sweep_first_level_is_refused():
    st = _define('''
        def st(u: Field, out: Field):
            with computation(PARALLEL), interval(...):
                t = u
            with computation(FORWARD):
                with interval(1, None):
                    t = u + t[0, 0, -1]
                    out = t
    ''')
    L = st.build("float64")
    dom = (ctypes.c_int64 * 3)(8, 4, 3)
    fl = (B.GtsField * 2)()
    for n, f in enumerate(fl):
        f.data = 0x7F0000000000 + (n << 32)
        f.stride[0], f.stride[1], f.stride[2] = 1, 8, 32
        f.hi[0], f.hi[1], f.hi[2] = 8, 4, 3
    ws = 0x7F0000000000 + (5 << 32)
    rc = L.gts_run(fl, 2, None, 0, dom, ws, 1 << 20, None)
    assert rc == -6, L.gts_last_error()  # GTS_E_LEVELS: level 0 is not swept


FUSION = {
    "a sweep may read the run's temporaries at a horizontal offset": ("""
        def st(u: Field, out: Field):
            with computation(PARALLEL), interval(...):
                t = u * 2.0
            with computation(FORWARD), interval(...):
                out = t[1, 0, 0]
    """, [[0, 1]], {"t": "lds"}),
    "an API field written by the run and read off-column breaks the group": ("""
        def st(u: Field, v: Field, out: Field):
            with computation(PARALLEL), interval(...):
                v = u * 2.0
            with computation(FORWARD), interval(...):
                out = v[1, 0, 0]
    """, [[0], [1]], {}),
    "a run member reading a vertical neighbour of the run is split off": ("""
        def st(u: Field, out: Field):
            with computation(PARALLEL), interval(...):
                t = u * 2.0
            with computation(PARALLEL), interval(0, -1):
                out = t[0, 0, 1]
    """, [[0], [1]], {"t": "hbm"}),
    "a write after a read of the group breaks it": ("""
        def st(u: Field, w: Field, out: Field):
            with computation(PARALLEL), interval(...):
                out = u * 2.0 + w
            with computation(PARALLEL), interval(...):
                w = u * 0.5
    """, [[0], [1]], {}),
    "a second sweep joins when it reads the first one's column": ("""
        def st(u: Field, out: Field):
            with computation(FORWARD), interval(...):
                t = u * 2.0
            with computation(BACKWARD), interval(1, None):
                out = t[0, 0, -1] + t
    """, [[0, 1]], {"t": "hbm"}),
}


@pytest.mark.parametrize("case", list(FUSION), ids=list(FUSION))
def test_fusion_groups(case):
    src, groups, storage = FUSION[case]
    st = _define(src)
    assert st.plan.groups == groups
    for t, where in storage.items():
        assert st.plan.temps[t].storage == where
