"""The allocation-free entry point gfdtd_solve_static (a fixed device array
as the workspace) against gfdtd_solve (a caller workspace), through the
C-ABI: the same kernels, so the same bits; two calls in a row, the second
smaller, so that contents left in the array by a larger call cannot leak
into a smaller one; and the size limit."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import torch
    assert torch.cuda.is_available()
    import paper_2304_06586_amd as pkg
    pkg.load_library()
    return pkg


def _same(a, b, label):
    for k in ("trace", "dft", "d", "b"):
        assert np.array_equal(a[k], b[k]), (label, k)
    assert a["status"] == b["status"] == 0, label


@pytest.mark.parametrize("precision", [W.F64, W.F32])
def test_static_workspace_equals_caller_workspace(P, precision):
    big = W.small_case(6001, 1500, 0.3, structure="crystal", seed=11, nprobe=4,
                       precision=precision)
    small = W.small_case(777, 900, -0.35, kind=W.MATTER, structure="slab", seed=12,
                         nprobe=3, precision=precision)
    for label, p in (("first, larger", big), ("second, smaller", small)):
        print(f"no-alloc {label}: nz={p.nz} steps={p.steps} precision={precision}",
              flush=True)
        got = P.gfdtd_solve_static(p)
        want = P.gfdtd_solve(p)
        _same(got, want, label)


def test_interface_workload_and_repeat(P):
    p = W.interface_run(0)
    want = P.gfdtd_solve(p)
    for i in range(2):
        print(f"no-alloc interface call {i}", flush=True)
        _same(P.gfdtd_solve_static(p), want, f"interface call {i}")


def test_oversized_problem_rejected(P):
    p = W.small_case(3_000_000, 10, 0.3, seed=1, nprobe=2)
    need = P.gfdtd_workspace_bytes(p)
    assert need > P.gfdtd.GFDTD_STATIC_WORKSPACE_BYTES
    with pytest.raises(P.GfdtdError) as ei:
        P.gfdtd_solve_static(p)
    assert ei.value.status == P.gfdtd.GFDTD_E_NOMEM
    assert "static workspace" in ei.value.message
