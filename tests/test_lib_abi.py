"""Host-side checks of the C-ABI library (no GPU work): it loads, exports
every entry point declared in include/ibm.h, and its host-only calls
validate descriptors and size workspaces."""
import ctypes
import os
import re

import numpy as np
import pytest

import workloads as w

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _lib():
    from paper_1912_11908_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        from paper_1912_11908_amd import build
        build.build()
    return _lib, _lib.load()


def _declared():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            txt = open(os.path.join(ROOT, "include", fn)).read()
            names |= set(re.findall(r"^\s*(?:int|void|const char \*)\s*(ibm_\w+)\s*\(", txt, re.M))
    return names


def test_library_exports_every_declared_symbol():
    lib, L = _lib()
    names = _declared()
    assert len(names) >= 15
    for n in sorted(names):
        assert hasattr(L, n), n
    assert names == set(lib.EXPORTS)


def test_header_layout_matches_binding():
    """The ctypes mirror of ibm_case / ibm_info agrees with the C layout
    (computed by compiling a tiny probe against the header)."""
    import subprocess
    import tempfile
    src = r'''
#include <stddef.h>
#include <stdio.h>
#include "ibm.h"
int main(void) {
  printf("%zu %zu %zu %zu %zu %zu\n", sizeof(ibm_case), offsetof(ibm_case, mach),
         offsetof(ibm_case, n_inner), sizeof(ibm_info), offsetof(ibm_info, cls),
         offsetof(ibm_info, time));
  return 0;
}
'''
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "p.c")
        exe = os.path.join(d, "p")
        open(c, "w").write(src)
        subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), c, "-o", exe])
        got = [int(x) for x in subprocess.check_output([exe]).split()]
    lib, _ = _lib()
    exp = [ctypes.sizeof(lib.IbmCase), lib.IbmCase.mach.offset, lib.IbmCase.n_inner.offset,
           ctypes.sizeof(lib.IbmInfo), lib.IbmInfo.cls.offset, lib.IbmInfo.time.offset]
    assert got == exp


@pytest.mark.parametrize("name", ["C1", "C2", "C3", "C4"])
def test_workspace_bytes_host_only(name):
    import paper_1912_11908_amd as P
    case = w.CASES[name]()
    nb = P.workspace_bytes(case)
    nv = case.ndim + 2
    hz = 3 if case.ndim == 3 else 0
    state = nv * (case.nk + 2 * hz) * (case.nj + 6) * (case.ni + 6) * 8
    assert nb > state            # scratch stage buffers live in the workspace
    assert nb < 6 * state + (64 << 20)
    assert P.workspace_bytes(case, "mixed") == nb


def test_invalid_descriptors_rejected():
    import paper_1912_11908_amd as P
    lib, L = _lib()
    case = w.small_case("cylinder", 32)
    c, keep = P.case_struct(case)
    n = ctypes.c_size_t(0)
    assert L.ibm_workspace_bytes(ctypes.byref(c), ctypes.byref(n)) == 0
    bad = [("ndim", 4), ("ni", 2), ("mach", -1.0), ("scheme", 7), ("precision", 3), ("dt", 0.0),
           ("ib_framework", 2), ("reconstruction", 5), ("wall_pressure", 3)]
    for field, val in bad:
        c2, keep2 = P.case_struct(case)
        setattr(c2, field, val)
        assert L.ibm_workspace_bytes(ctypes.byref(c2), ctypes.byref(n)) == -1, field
    # non-increasing faces
    case2 = w.small_case("cylinder", 32)
    case2.xf = case2.xf.copy()
    case2.xf[5] = case2.xf[4]
    c3, keep3 = P.case_struct(case2)
    assert L.ibm_workspace_bytes(ctypes.byref(c3), ctypes.byref(n)) == -1
    # facet index out of range
    case3 = w.small_case("cylinder", 32)
    case3.facet = case3.facet.copy()
    case3.facet[0, 0] = 10 ** 6
    c4, keep4 = P.case_struct(case3)
    assert L.ibm_workspace_bytes(ctypes.byref(c4), ctypes.byref(n)) == -1
    # eq.7 is 2D only; both IB frameworks exist in 2D and 3D
    tube = w.small_case("tube", 16, nz=4, ntheta=16, nzt=2)
    c5, keep5 = P.case_struct(tube)
    assert L.ibm_workspace_bytes(ctypes.byref(c5), ctypes.byref(n)) == 0
    c5.ib_framework = 1
    assert L.ibm_workspace_bytes(ctypes.byref(c5), ctypes.byref(n)) == 0
    c5.wall_pressure = 1
    assert L.ibm_workspace_bytes(ctypes.byref(c5), ctypes.byref(n)) == -1
    # null output pointer and workspace too small never touch the device
    h = ctypes.c_void_p()
    assert L.ibm_create(ctypes.byref(c), ctypes.c_void_p(1), 16, ctypes.byref(h)) == -5
    del keep, keep2, keep3, keep4, keep5


def test_product_path_has_no_cpu_fallback():
    """The binding loads only libibm.so and never the oracle."""
    src = open(os.path.join(ROOT, "paper_1912_11908_amd", "__init__.py")).read()
    src += open(os.path.join(ROOT, "paper_1912_11908_amd", "_lib.py")).read()
    assert "oracle" not in src.replace("oracle's", "")
    assert "import oracle" not in src


def test_bodies_beyond_the_exact_predicates_rejected():
    """The exact crossing predicates (section 3.2) multiply a facet's edge
    extent by a node-to-vertex distance in 64-bit integers on the 2^24
    lattice: a body and IB region too large for that is refused with
    IBM_EGEOM by the host-only sizing call, before any device work.  A square
    of side 60 in a box of side 64 fits (2 * (64 * 2^24)^2 < 2^62 with
    room); one of side 200 does not."""
    import paper_1912_11908_amd as P
    from workloads.cases import Case
    lib, L = _lib()
    n = ctypes.c_size_t(0)
    for side, want in ((60.0, 0), (200.0, -2)):
        h = side / 2
        v = w.snap(np.array([[-h, -h], [h, -h], [h, h], [-h, h]]))
        s = np.array([[0, 1], [1, 2], [2, 3], [3, 0]], np.int32)
        f = w.uniform_faces(64, -0.55 * side - 2, 0.55 * side + 2)
        case = Case("square", 2, f, f.copy(), np.array([-0.5, 0.5]), ("farfield",) * 4 + ("periodic",) * 2,
                    v, s, 0.3, 100.0, dt=1e-3)
        c, keep = P.case_struct(case)
        assert L.ibm_workspace_bytes(ctypes.byref(c), ctypes.byref(n)) == want, side
        del keep
