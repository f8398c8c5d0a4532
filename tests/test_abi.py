"""The C-ABI library: loads without a GPU, exports what the header declares,
and rejects bad arguments on the host before any device call."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_symbols():
    src = open(os.path.join(ROOT, "include", "gpumetad.h")).read()
    return sorted(set(re.findall(r"^(?:int|const char\*)\s+(gm_\w+)\s*\(", src, flags=re.M)))


def test_exports_match_header():
    import paper_2510_06873_amd as P

    syms = header_symbols()
    assert len(syms) >= 19
    lib = P.lib()
    for s in syms:
        assert hasattr(lib, s), s
    assert sorted(P.EXPORTS) == syms


def test_strerror_and_version():
    import paper_2510_06873_amd as P

    lib = P.lib()
    for code in range(0, -9, -1):
        assert lib.gm_strerror(code)
    assert b"gfx950" in lib.gm_version()


def _params(**kw):
    from paper_2510_06873_amd.binding import Params

    return Params(**kw).to_c()


@pytest.mark.parametrize("kw,n", [
    (dict(cv_kind=0), 10), (dict(cv_kind=4), 10), (dict(precision=2), 10), (dict(r_c=0.0), 10),
    (dict(skin=-1.0), 10), (dict(taper=0.0), 10), (dict(taper=5.0), 10), (dict(bond_w=0.0), 10),
    (dict(count_w=-1.0), 10), (dict(cv_kind=1, cn_r0=0.0), 10), (dict(sigma=[0.0]), 10),
    (dict(cv_kind=3, sigma=[1.0, 0.0]), 10), (dict(gamma=0.5), 10), (dict(gamma=10.0, kBT=0.0), 10),
    (dict(hill_capacity=-1), 10), (dict(max_neighbors=5000), 10), ({}, 0), ({}, -3)])
def test_create_rejects_bad_params_on_host(kw, n):
    import paper_2510_06873_amd as P

    lib = P.lib()
    h = C.c_void_p(1)
    p = _params(**kw)
    assert lib.gm_create(C.byref(h), C.byref(p), n, None) == -1
    assert h.value is None


def test_null_context_calls():
    import paper_2510_06873_amd as P

    lib = P.lib()
    assert lib.gm_create(None, None, 10, None) == -1
    for name, args in [("gm_destroy", [None]), ("gm_build_neighbors", [None, None, None]),
                       ("gm_cv_forward", [None, None, None]), ("gm_bias_eval", [None, None, None, None]),
                       ("gm_cv_backward", [None, None, None, None]),
                       ("gm_apply_bias_forces", [None, None, None, None]), ("gm_deposit_hill", [None, None]),
                       ("gm_status", [None, 0]), ("gm_set_stream", [None, None])]:
        assert getattr(lib, name)(*args) == -1, name


def test_header_is_plain_c():
    """The boundary is C: no torch, no C++ types in the public header."""
    src = open(os.path.join(ROOT, "include", "gpumetad.h")).read()
    for bad in ("torch", "std::", "template", "class ", "hipStream_t"):
        assert bad not in src


def test_oracle_and_product_are_independent():
    """Neither side imports or includes the other."""
    pkg = os.path.join(ROOT, "paper_2510_06873_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                txt = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in txt and "from oracle" not in txt and "oracle.c" not in txt, f
    for f in os.listdir(os.path.join(ROOT, "oracle")):
        if f.endswith((".py", ".c", ".h")):
            txt = open(os.path.join(ROOT, "oracle", f)).read()
            assert "paper_2510_06873_amd" not in txt and "gpumetad.h" not in txt, f
