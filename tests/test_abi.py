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
    for code in range(0, -10, -1):
        assert lib.gm_strerror(code)
    assert b"gfx950" in lib.gm_version()


def _params(**kw):
    from paper_2510_06873_amd.binding import Params

    return Params(**kw).to_c()


@pytest.mark.parametrize("kw,n", [
    (dict(cv_kind=0), 10), (dict(cv_kind=5), 10), (dict(precision=2), 10), (dict(r_c=0.0), 10),
    (dict(cv_kind=4, external_dims=3), 10), (dict(cv_kind=4, external_dims=0), 0),
    (dict(cv_kind=4, external_dims=2, sigma=[1.0, 0.0]), 0), (dict(cv_kind=4, period=[-1.0, 0.0]), 0),
    (dict(period=[float("inf"), 0.0]), 10), (dict(cv_kind=4, gamma=0.5), 0), (dict(cv_kind=4), -1),
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


def test_null_batch_calls():
    """Every batch entry point refuses a null batch (and a null output
    handle) on the host."""
    import paper_2510_06873_amd as P

    lib = P.lib()
    one = (C.c_int32 * 1)(0)
    box = (C.c_double * 3)(10.0, 10.0, 10.0)
    assert lib.gm_batch_create(None, None, 1, None, None, None) == -1
    for name, args in [("gm_batch_destroy", [None]), ("gm_batch_update", [None, None, 0, None, None]),
                       ("gm_batch_build", [None, box]), ("gm_batch_build_some", [None, one, 1, box, None]),
                       ("gm_batch_step", [None]), ("gm_batch_deposit", [None]),
                       ("gm_batch_deposit_some", [None, one, 1]), ("gm_batch_values", [None, None, None, None])]:
        assert getattr(lib, name)(*args) == -1, name
    h = C.c_void_p()
    assert lib.gm_batch_create(C.byref(h), None, 1, None, None, None) == -1 and not h.value


def test_small_cv_calls_reject_bad_arguments_on_host():
    """Argument checks of the context-free calls run before any device work."""
    import ctypes as C

    import paper_2510_06873_amd as P

    lib = P.lib()
    box = (C.c_double * 3)(10.0, 10.0, 10.0)
    bad_box = (C.c_double * 3)(10.0, 0.0, 10.0)
    fake = C.c_void_p(1 << 20)  # aligned, never dereferenced: every call below fails its checks first
    assert lib.gm_torsions(fake, 10, fake, -1, box, fake, None) == -1
    assert lib.gm_torsions(fake, 10, fake, (1 << 16) + 1, box, fake, None) == -1
    assert lib.gm_torsions(None, 10, fake, 3, box, fake, None) == -1
    assert lib.gm_torsions(fake, 10, fake, 3, bad_box, fake, None) == -1
    assert lib.gm_torsions(None, 0, None, 0, None, None, None) == 0  # nothing to do
    assert lib.gm_torsion_forces(fake, 10, fake, 3, box, fake, fake, 7, None) == -1  # precision
    assert lib.gm_torsion_forces(fake, 10, fake, 3, box, fake, C.c_void_p((1 << 20) + 16), 1, None) == -1
    assert lib.gm_nearest_distance(fake, 10, 10, fake, 5, box, fake, None, None) == -1  # centre out of range
    assert lib.gm_nearest_distance(fake, 10, -1, fake, 5, box, fake, None, None) == -1
    assert lib.gm_nearest_distance(fake, 10, 0, fake, 0, box, fake, None, None) == -1
    assert lib.gm_nearest_distance_forces(fake, 10, 0, fake, 5, box, None, fake, 0, None) == -1
    lo, hi, nb = (C.c_double * 2)(0.0, 0.0), (C.c_double * 2)(1.0, 1.0), (C.c_int32 * 2)(10, 10)
    assert lib.gm_fes_reweight(fake, fake, 100, 3, lo, hi, nb, 1.0, fake, None) == -1
    assert lib.gm_fes_reweight(fake, fake, 0, 2, lo, hi, nb, 1.0, fake, None) == -1
    assert lib.gm_fes_reweight(fake, fake, 100, 2, lo, hi, nb, 0.0, fake, None) == -1
    assert lib.gm_fes_reweight(fake, fake, 100, 2, hi, lo, nb, 1.0, fake, None) == -1
    big = (C.c_int32 * 2)(1 << 13, 1 << 12)
    assert lib.gm_fes_reweight(fake, fake, 100, 2, lo, hi, big, 1.0, fake, None) == -1
    assert lib.gm_fes_hills(None, lo, hi, nb, fake) == -1
    # the allocation-free variant: the same argument checks, then its scratch limit
    assert lib.gm_fes_reweight_noalloc(fake, fake, 100, 3, lo, hi, nb, 1.0, fake, None) == -1
    assert lib.gm_fes_reweight_noalloc(fake, fake, 0, 2, lo, hi, nb, 1.0, fake, None) == -1
    assert lib.gm_fes_reweight_noalloc(None, fake, 100, 2, lo, hi, nb, 1.0, fake, None) == -1
    assert lib.gm_fes_reweight_noalloc(fake, fake, 100, 2, hi, lo, nb, 1.0, fake, None) == -1
    assert lib.gm_fes_reweight_noalloc(fake, fake, 100, 2, lo, hi, big, 1.0, fake, None) == -9
    over = (C.c_int32 * 2)(257, 256)  # 65,792 bins, just past the 65,536 of the fixed scratch
    assert lib.gm_fes_reweight_noalloc(fake, fake, 100, 2, lo, hi, over, 1.0, fake, None) == -9
    over1 = (C.c_int32 * 1)(65537)
    assert lib.gm_fes_reweight_noalloc(fake, fake, 100, 1, lo, hi, over1, 1.0, fake, None) == -9


def test_lattice_virial_on_host():
    import paper_2510_06873_amd as P

    assert P.binding.lattice_virial([3.0, 4.0, 5.0], [0.5, -2.0, 1.0]) == [-1.5, 8.0, -5.0]
    assert P.binding.lattice_virial([3.0, 4.0, 5.0], [2.0]) == [-6.0]
    import ctypes as C
    out = (C.c_double * 3)()
    assert P.lib().gm_lattice_virial((C.c_double * 3)(1, 1, 1), (C.c_double * 3)(1, 1, 1), 4, out) == -1


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
