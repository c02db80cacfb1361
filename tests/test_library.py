"""The C-ABI library without a GPU: it loads, exports every function that
include/shellhom.h declares, its structs match the ctypes mirror, and its
host-side logic (argument validation, workspace and footprint sizing, status
strings) behaves as the header documents.  No call here launches a kernel."""
import ctypes
import math
import os
import re
from ctypes import byref, c_size_t

import numpy as np
import pytest

from paper_2511_04025_amd import binding as B
from paper_2511_04025_amd import workloads as wl

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "shellhom.h")


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(B.LIB_PATH):
        from paper_2511_04025_amd import build
        build.build(verbose=False)
    return B.lib()


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)  # drop comments
    return sorted(set(re.findall(r"\b(shh_[a-z_0-9]+)\s*\(", text)))


def test_every_declared_function_is_exported(lib):
    names = declared_functions()
    assert len(names) >= 20
    raw = ctypes.CDLL(B.LIB_PATH)
    missing = [nm for nm in names if not hasattr(raw, nm)]
    assert not missing, missing
    # and the binding describes exactly the declared set
    assert sorted(B.EXPORTS) == names


def test_struct_layouts_match_the_header(tmp_path):
    # shh_design: 2 int32, 2 pointers, int32 (+pad), pointer, 4 doubles, int32 (+pad), 3 doubles, int32 (+pad)
    assert ctypes.sizeof(B.ShhDesign) == 112
    assert ctypes.sizeof(B.ShhOpts) == 40
    assert ctypes.sizeof(B.ShhResult) == 36 * 8 + 2 * 8 + 6 * 4 + 6 * 8 + 5 * 8 + 8
    assert B.ShhResult.status.offset == ctypes.sizeof(B.ShhResult) - 8
    assert B.ShhResult.active_nodes.offset == ctypes.sizeof(B.ShhResult) - 4
    # and the C compiler agrees, field by field
    import shutil
    import subprocess
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    src = tmp_path / "layout.c"
    inc = os.path.join(os.path.dirname(B.HERE), "include")
    checks = []
    for struct, cls in (("shh_design", B.ShhDesign), ("shh_opts", B.ShhOpts), ("shh_result", B.ShhResult)):
        checks.append(f'printf("{struct} %zu\\n", sizeof({struct}));')
        for name, _ in cls._fields_:
            checks.append(f'printf("{struct}.{name} %zu\\n", offsetof({struct}, {name}));')
    src.write_text("#include <stdio.h>\n#include <stddef.h>\n#include \"shellhom.h\"\nint main(void) {\n"
                   + "\n".join(checks) + "\nreturn 0;\n}\n")
    exe = tmp_path / "layout"
    subprocess.run([cc, "-I", inc, str(src), "-o", str(exe)], check=True)
    out = dict(line.split() for line in subprocess.run([str(exe)], check=True, capture_output=True,
                                                         text=True).stdout.splitlines())
    for struct, cls in (("shh_design", B.ShhDesign), ("shh_opts", B.ShhOpts), ("shh_result", B.ShhResult)):
        assert int(out[struct]) == ctypes.sizeof(cls), struct
        for name, _ in cls._fields_:
            assert int(out[f"{struct}.{name}"]) == getattr(cls, name).offset, (struct, name)


def test_version_and_status_strings(lib):
    assert lib.shh_version() >= 10000
    codes = [B.SHH_OK, B.SHH_NOT_CONVERGED, B.SHH_INVALID_ARG, B.SHH_WORKSPACE_TOO_SMALL, B.SHH_HIP_ERROR,
             B.SHH_OVER_BUDGET, B.SHH_UNSUPPORTED, B.SHH_BREAKDOWN, B.SHH_NOT_FOUND]
    texts = [lib.shh_strerror(c).decode() for c in codes]
    assert len(set(texts)) == len(codes)
    assert "unknown" in lib.shh_strerror(12345).decode()


def ws_bytes(lib, design, precision="mixed", **kw):
    a = B.DesignArgs(design)
    o = B.make_opts(precision, **kw)
    nb = c_size_t(0)
    rc = lib.shh_workspace_bytes(byref(a.c), byref(o), byref(nb))
    return rc, nb.value


def test_workspace_sizes(lib):
    for n in (2, 24, 64, 128):
        d = wl.shell_128(2000, n=n)
        rc_m, bm = ws_bytes(lib, d, "mixed")
        rc_d, bd = ws_bytes(lib, d, "fp64")
        assert rc_m == B.SHH_OK and rc_d == B.SHH_OK
        assert bd > bm > 0
        if n >= 64:
            # seven FP32 CG vectors, the FP64 accumulator, moduli and D^-1: ~664 B/node;
            # FP64: seven FP64 vectors and moduli: ~1024 B/node
            assert 600 < bm / n ** 3 < 700
            assert 980 < bd / n ** 3 < 1060
    # keeping the field for the adjoint adds F, grad F, d (40 B/voxel)
    d = wl.smooth_shell_96(5000, n=24)
    _, b0 = ws_bytes(lib, d, "mixed")
    _, b1 = ws_bytes(lib, d, "mixed", save_for_backward=True)
    assert b1 - b0 >= 40 * 24 ** 3


def test_stiffness_and_engine_footprints(lib):
    o = B.make_opts("mixed")
    nb = c_size_t(0)
    assert lib.shh_workspace_bytes_stiffness(512, byref(o), byref(nb)) == B.SHH_OK and nb.value > 0
    assert lib.shh_workspace_bytes_stiffness(513, byref(o), byref(nb)) == B.SHH_INVALID_ARG
    assert lib.shh_workspace_bytes_stiffness(1, byref(o), byref(nb)) == B.SHH_INVALID_ARG
    d = wl.shell_128(2001, n=96)
    a = B.DesignArgs(d)
    fp = c_size_t(0)
    assert lib.shh_engine_footprint(byref(a.c), byref(o), byref(fp)) == B.SHH_OK
    _, ws = ws_bytes(lib, d, "mixed")
    # an engine slot is the same layout without the stand-alone call's segment tables
    assert 0.99 * ws <= fp.value <= ws


def _invalid(**change):
    d = wl.small_shell_24()
    return d.with_(**change)


@pytest.mark.parametrize("change", [
    dict(n=1), dict(n=513), dict(K=0), dict(K=7), dict(nu=0.5), dict(nu=-1.0), dict(E=0.0),
    dict(E_void=2.0), dict(E_void=-1e-3), dict(kappa=-1.0), dict(dist_mode=2),
    dict(thickness=None, target_vf=0.0), dict(thickness=None, target_vf=1.0), dict(iso=math.inf),
])
def test_design_validation(lib, change):
    rc, _ = ws_bytes(lib, _invalid(**change))
    assert rc == B.SHH_INVALID_ARG, change


def test_nonfinite_charges_and_bad_options(lib):
    d = wl.small_shell_24()
    pos = d.pos.copy()
    pos[3, 1] = np.nan
    assert ws_bytes(lib, d.with_(pos=pos))[0] == B.SHH_INVALID_ARG
    q = d.q.copy()
    q[0] = np.inf
    assert ws_bytes(lib, d.with_(q=q))[0] == B.SHH_INVALID_ARG
    a = B.DesignArgs(d)
    nb = c_size_t(0)
    for o in (B.ShhOpts(precision=2, rtol=1e-6, max_iter=10), B.ShhOpts(precision=1, rtol=0.0, max_iter=10),
              B.ShhOpts(precision=1, rtol=1.0, max_iter=10), B.ShhOpts(precision=1, rtol=1e-6, max_iter=-1)):
        assert lib.shh_workspace_bytes(byref(a.c), byref(o), byref(nb)) == B.SHH_INVALID_ARG
    # the edge of the accepted range
    assert ws_bytes(lib, d.with_(n=512))[0] == B.SHH_OK
    assert ws_bytes(lib, d.with_(E_void=0.0))[0] == B.SHH_OK


def test_option_defaults():
    o = B.make_opts("mixed")
    assert o.precision == B.PREC_MIXED and o.rtol == 1e-6
    o = B.make_opts("fp64")
    assert o.precision == B.PREC_FP64 and o.rtol == 1e-10


def test_workloads_are_seeded_and_shaped():
    a, b = wl.shell_128(2003), wl.shell_128(2003)
    assert np.array_equal(a.pos, b.pos) and np.array_equal(a.q, b.q)
    assert a.n == 128 and len(a.q) == 48 and abs(a.q.sum()) < 1e-12
    assert 0.05 <= a.target_vf <= 0.15 and a.E_void == 1e-6
    c1 = wl.small_shell_24()
    assert c1.n == 24 and sorted(set(c1.q.tolist())) == [-1.0, 1.0] and c1.q.sum() == 0
    c3 = wl.large_shell_256()
    assert c3.n == 256 and len(c3.q) == 64 and c3.q.sum() == 0
    trace = wl.serving_trace(count=64)
    assert {d.n for d in trace} <= {64, 96, 128}
    assert all(16 <= len(d.q) <= 64 and 0.03 <= d.target_vf <= 0.2 for d in trace)
    t = wl.poisson_arrivals(64, 2.0)
    assert np.all(np.diff(t) >= 0) and t[0] >= 0
    c5 = wl.smooth_shell_96(5000)
    assert c5.n == 96 and c5.kappa == 4 * 96 and len(c5.q) == 32


def test_operator_workspace(lib):
    nb = c_size_t(0)
    for n in (2, 130, 512):
        for prec in (B.PREC_FP64, B.PREC_MIXED):
            assert lib.shh_workspace_bytes_operator(n, prec, byref(nb)) == B.SHH_OK
            # moduli + Jacobi diagonal (~16 B/node) plus fixed-size tables
            if n >= 130:
                assert 15.5 < nb.value / n ** 3 < 17.5
            o = B.make_opts("fp64" if prec == B.PREC_FP64 else "mixed")
            full = c_size_t(0)
            assert lib.shh_workspace_bytes_stiffness(n, byref(o), byref(full)) == B.SHH_OK
            assert nb.value < full.value
    for bad in ((1, B.PREC_FP64), (513, B.PREC_FP64), (64, 2), (64, -1)):
        assert lib.shh_workspace_bytes_operator(bad[0], bad[1], byref(nb)) == B.SHH_INVALID_ARG


def test_multigrid_solver_option(lib):
    # n = m 2^k with k >= 1, m <= 8 and n >= 6 coarsens; others are refused up front
    for n, ok in ((128, True), (96, True), (24, True), (20, True), (6, True), (37, False), (50, False), (4, False), (2, False)):
        d = wl.shell_128(2000, n=n)
        rc, nb = ws_bytes(lib, d, "mixed", solver="mg")
        assert rc == (B.SHH_OK if ok else B.SHH_UNSUPPORTED), n
        if ok:
            _, nj = ws_bytes(lib, d, "mixed")
            # the hierarchy adds its stencils and vectors (~1/8 of the voxel level's per level)
            assert nj < nb < 2 * nj
    # SHH_SOLVER_AUTO takes the multigrid where the grid coarsens and Jacobi elsewhere
    for n in (24, 37, 50, 4):
        d = wl.shell_128(2000, n=n)
        rc_a, na = ws_bytes(lib, d, "mixed", solver="auto")
        rc_m, nm = ws_bytes(lib, d, "mixed", solver="mg")
        _, nj = ws_bytes(lib, d, "mixed", solver="jacobi")
        assert rc_a == B.SHH_OK and na == (nm if rc_m == B.SHH_OK else nj), n
    a = B.DesignArgs(wl.small_shell_24())
    nb = c_size_t(0)
    o = B.ShhOpts(precision=1, rtol=1e-6, max_iter=10, solver=5)
    assert lib.shh_workspace_bytes(byref(a.c), byref(o), byref(nb)) == B.SHH_INVALID_ARG
    # the selective solve works in the multigrid solver's workspace where the
    # grid coarsens, else (and with Jacobi only) in the Jacobi path's, at any n
    for n in (24, 37):
        d = wl.shell_128(2000, n=n)
        _, nsel = ws_bytes(lib, d, "mixed", solver="selective")
        _, nsj = ws_bytes(lib, d, "mixed", solver="selective-jacobi")
        _, nj = ws_bytes(lib, d, "mixed", solver="jacobi")
        rc_m, nm = ws_bytes(lib, d, "mixed", solver="mg")
        assert nsj == nj and nsel == (nm if rc_m == B.SHH_OK else nj), n


def test_field_entry_point_validation(lib):
    # argument checks of shh_homogenize_field that return before any device work
    from ctypes import c_double, c_void_p
    o = B.make_opts("mixed")
    res = B.ShhResult()
    fake = c_void_p(256)  # never dereferenced: every call below fails validation first
    for n, dt, Es, Ev, nu in ((1, 0, 1.0, 0.0, 0.3), (8, 3, 1.0, 0.0, 0.3), (8, 0, 0.0, 0.0, 0.3),
                              (8, 0, 1.0, 2.0, 0.3), (8, 0, 1.0, -1.0, 0.3), (8, 2, 1.0, 0.0, 0.5)):
        rc = lib.shh_homogenize_field(n, fake, dt, c_double(Es), c_double(Ev), c_double(nu), byref(o), fake,
                                      c_size_t(1 << 20), None, byref(res))
        assert rc == B.SHH_INVALID_ARG, (n, dt, Es, Ev, nu)


def test_point_field_workspace_needs_only_charges(lib):
    # the point-field entries read the charges, alpha, K and symmetry mode only:
    # a design without a thickness rule is accepted, and the size grows with
    # the points and with the symmetry images
    d = wl.Design(pos=np.zeros((2, 3)), q=np.array([1.0, -1.0]), n=8, K=3)
    sizes = []
    for npts, sym in ((100, 0), (10000, 0), (100, 2)):
        a = B.DesignArgs(d.with_(symmetry=sym))
        nb = c_size_t(0)
        assert lib.shh_workspace_bytes_points(byref(a.c), npts, byref(nb)) == B.SHH_OK
        sizes.append(nb.value)
    assert sizes[1] > sizes[0] and sizes[2] > sizes[0]
    a = B.DesignArgs(d)
    nb = c_size_t(0)
    assert lib.shh_workspace_bytes_points(byref(a.c), 0, byref(nb)) == B.SHH_INVALID_ARG
