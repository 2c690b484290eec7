"""The ctypes declarations of both native libraries match their C prototypes
(a missing argtypes entry silently passes a pointer as a 32-bit int)."""
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _prototypes(text, prefix):
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    text = re.sub(r"//[^\n]*", "", text)
    out = {}
    for m in re.finditer(r"\b(%s[a-z_0-9]*)\s*\(([^;{)]*)\)\s*[;{]" % prefix, text):
        name, params = m.group(1), m.group(2).strip()
        if not params or params == "void":
            out[name] = 0
        else:
            out[name] = params.count(",") + 1
    return out


def test_oracle_argtypes_match_prototypes():
    from oracle import core
    L = core.lib()
    protos = _prototypes(open(os.path.join(ROOT, "oracle", "gmpea_oracle.c")).read(), "orc_")
    checked = 0
    for name, n in protos.items():
        fn = getattr(L, name, None)
        if fn is None or fn.argtypes is None:
            continue
        assert len(fn.argtypes) == n, (name, len(fn.argtypes), n)
        checked += 1
    assert checked >= 15


def test_library_argtypes_match_header():
    from paper_2509_19821_amd import build as B
    if not os.path.exists(B.LIB):
        B.build()
    from paper_2509_19821_amd import gmpea as G
    L = G.lib()
    protos = _prototypes(open(os.path.join(ROOT, "include", "gmpea.h")).read(), "gmpea_")
    assert set(G.EXPORTS) == set(protos), (set(G.EXPORTS) ^ set(protos))
    for name, n in protos.items():
        fn = getattr(L, name)
        if n == 0:
            continue
        assert fn.argtypes is not None and len(fn.argtypes) == n, (name, fn.argtypes, n)
