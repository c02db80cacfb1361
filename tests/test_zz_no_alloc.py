"""The no-allocation entry point (shh_homogenize_noalloc, the library's fixed
device scratch) against shh_homogenize with a caller-owned workspace: the
same kernels on the same inputs, so the results must be identical.  Two calls
in a row, the second with a smaller design, so that the second runs on what
the first left in the scratch."""
import numpy as np
import pytest

from paper_2511_04025_amd import workloads as wl

from gpu_helpers import gpu_available

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]


def _same(a, b):
    assert a["status"] == b["status"] == 0, (a["status"], b["status"])
    assert np.array_equal(a["C"], b["C"]), np.abs(a["C"] - b["C"]).max()
    assert a["V"] == b["V"] and a["t"] == b["t"]
    assert np.array_equal(a["iters"], b["iters"]) and np.array_equal(a["rel_res"], b["rel_res"])


def test_noalloc_matches_workspace_path_on_consecutive_calls():
    from paper_2511_04025_amd import api, binding as B
    big = wl.shell_128(2003, n=40)                         # mixed multigrid, 40^3
    small = wl.small_shell_24()                            # FP64 Jacobi, 24^3
    cases = [(big, dict(precision="mixed", rtol=1e-5, solver="mg")),
             (small, dict(precision="fp64", rtol=1e-10, solver="jacobi"))]
    for d, kw in cases:
        need = api.workspace_bytes(d, B.make_opts(kw["precision"], kw["rtol"], solver=kw["solver"]))
        assert need <= B.NOALLOC_SCRATCH_BYTES, need
    first = [api.homogenize_noalloc(d, **kw) for d, kw in cases]
    for (d, kw), got in zip(cases, first):
        _same(got, api.homogenize(d, **kw))
        assert all(v == 0.0 for v in got["ms"].values())
    # again, in the other order: the larger design now follows the smaller one
    for (d, kw), ref in zip(cases[::-1], first[::-1]):
        _same(api.homogenize_noalloc(d, **kw), ref)


def test_noalloc_rejects_designs_larger_than_the_scratch():
    from paper_2511_04025_amd import api, binding as B
    d = wl.shell_128(2000, n=96)
    with pytest.raises(B.ShellhomError) as e:
        api.homogenize_noalloc(d, precision="mixed", rtol=1e-5, solver="mg")
    assert e.value.code == B.SHH_SCRATCH_TOO_SMALL
    # the scratch is still usable afterwards
    s = wl.small_shell_24()
    _same(api.homogenize_noalloc(s, precision="fp64", rtol=1e-10), api.homogenize(s, precision="fp64", rtol=1e-10))
