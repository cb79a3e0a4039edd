"""The C-ABI library loads and exports every symbol include/pastis.h declares
(no GPU needed: nothing here launches device work)."""

import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "pastis.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(pastis_[a-z0-9_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    import paper_2009_14467_amd as P

    L = P.lib()
    names = _declared()
    assert len(names) >= 8
    for name in names:
        assert hasattr(L, name), name
    assert set(names) <= set(P.exported_names()) | {"pastis_default_params"}


def test_default_params_are_the_papers():
    import ctypes

    import paper_2009_14467_amd as P
    from paper_2009_14467_amd._binding import _Params

    p = _Params()
    P.lib().pastis_default_params(ctypes.byref(p))
    assert (p.k, p.gap_open, p.gap_extend, p.xdrop, p.min_identity_pct, p.min_coverage_pct) == (6, 11, 1, 49, 30, 70)


def test_status_strings():
    import paper_2009_14467_amd as P

    L = P.lib()
    assert L.pastis_status_string(0) == b"ok"
    assert b"alphabet" in L.pastis_status_string(2)
