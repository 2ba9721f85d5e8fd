"""Host-side tests of the C-ABI library (no GPU): the shared library loads
and exports every function the header declares, argument validation, the
stability pre-flight against the oracle's amplification matrix, and the
size queries."""
import ctypes
import math
import os
import re

import numpy as np
import pytest

import workloads as W
from oracle import stability as st

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = [os.path.join(ROOT, "include", h) for h in ("gfdtd.h", "gfdtd2d.h")]


@pytest.fixture(scope="module")
def P():
    import paper_2304_06586_amd as pkg
    from paper_2304_06586_amd import gfdtd
    if not os.path.exists(gfdtd.LIB_PATH):
        from paper_2304_06586_amd import build
        build.build()
    pkg.load_library()
    return pkg


def _declared():
    names = set()
    for h in HEADERS:
        src = open(h).read()
        src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
        names |= set(re.findall(r"\b(gfdtd2?d?_[a-z_]+)\s*\(", src))
    return sorted(names)


def test_header_functions_are_exported(P):
    lib = ctypes.CDLL(P.gfdtd.LIB_PATH)
    names = _declared()
    assert len(names) >= 18
    for n in names:
        assert hasattr(lib, n), n


def test_binding_covers_header(P):
    assert set(_declared()) == set(P.gfdtd.EXPORTS)


def test_struct_sizes_match_header(P, tmp_path):
    """The ctypes layouts match the C structs: sizes and field offsets
    printed by a C program compiled against the header (the library
    rejects a smaller struct_size, so a mismatch would show as E_INVALID)."""
    import shutil
    import subprocess
    g = P.gfdtd
    structs = ["gfdtd_problem", "gfdtd_result", "gfdtd_exec", "gfdtd_stats",
               "gfdtd_server_config", "gfdtd_tmm_stack", "gfdtd2d_problem",
               "gfdtd2d_result", "gfdtd2d_exec", "gfdtd2d_stats"]
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "gfdtd.h"',
             '#include "gfdtd2d.h"', "int main(void) {"]
    for name in structs:
        lines.append(f'printf("{name} %zu\\n", sizeof({name}));')
        for f, _ in getattr(g, name)._fields_:
            lines.append(f'printf("{name}.{f} %zu\\n", offsetof({name}, {f}));')
    lines += ["return 0;", "}"]
    src = tmp_path / "sizes.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "sizes"
    cc = shutil.which("gcc") or shutil.which("cc")
    assert cc, "no C compiler"
    subprocess.run([cc, "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)],
                   check=True)
    out = dict(line.split() for line in
               subprocess.run([str(exe)], check=True, capture_output=True,
                              text=True).stdout.splitlines())
    for name in structs:
        t = getattr(g, name)
        assert ctypes.sizeof(t) == int(out[name]), name
        for f, _ in t._fields_:
            assert getattr(t, f).offset == int(out[f"{name}.{f}"]), (name, f)


def test_status_strings(P):
    for s in range(8):
        assert P.gfdtd_status_str(s)


def _ok():
    return W.small_case(200, 100, 0.3, seed=0)


@pytest.mark.parametrize("field,value", [
    ("nz", 7), ("nz", 2**31 - 2**20 + 1), ("courant", 0.0), ("courant", float("nan")), ("beta", 1.0),
    ("beta", -1.5), ("src_cell", 0), ("src_cell", 199), ("kind", 5),
    ("precision", 3), ("abc", 9),
])
def test_invalid_scalars_rejected(P, field, value):
    p = _ok()
    if field == "nz":
        p = p.replace(nz=value, eps_rest=p.eps_rest[:value], mu_rest=p.mu_rest[:value],
                      probes=np.array([0]), src_cell=3)
    else:
        p = p.replace(**{field: value})
    with pytest.raises(P.GfdtdError) as e:
        P.gfdtd_check(p)
    assert e.value.status == P.gfdtd.GFDTD_E_INVALID


def test_invalid_arrays_rejected(P):
    p = _ok()
    bad = p.eps_rest.copy()
    bad[17] = -1.0
    for q in (p.replace(eps_rest=bad), p.replace(probes=np.array([0, 200])),
              p.replace(probes=np.arange(65) % 100)):
        with pytest.raises(P.GfdtdError) as e:
            P.gfdtd_check(q)
        assert e.value.status == P.gfdtd.GFDTD_E_INVALID
    nan = p.mu_rest.copy()
    nan[0] = float("inf")
    with pytest.raises(P.GfdtdError):
        P.gfdtd_check(p.replace(mu_rest=nan))


def test_periodic_ends_and_initial_fields_validated(P):
    """A ring accepts a source at any cell (0..nz-1); a grid with ends
    only at 1..nz-2.  Initial fields must be finite and nz long."""
    ring = _ok().replace(abc=W.ABC_PERIODIC)
    for cell in (0, 199):
        P.gfdtd_check(ring.replace(src_cell=cell))
        with pytest.raises(P.GfdtdError) as e:
            P.gfdtd_check(_ok().replace(src_cell=cell))
        assert e.value.status == P.gfdtd.GFDTD_E_INVALID
    with pytest.raises(P.GfdtdError) as e:
        P.gfdtd_check(ring.replace(src_cell=200))
    assert e.value.status == P.gfdtd.GFDTD_E_INVALID
    d, b = W.random_fields(200, 1)
    P.gfdtd_check(ring.replace(init_d=d, init_b=b))
    P.gfdtd_check(_ok().replace(init_b=b))
    bad = d.copy()
    bad[57] = float("nan")
    for q in (ring.replace(init_d=bad), _ok().replace(init_b=bad)):
        with pytest.raises(P.GfdtdError) as e:
            P.gfdtd_check(q)
        assert e.value.status == P.gfdtd.GFDTD_E_INVALID
    with pytest.raises(ValueError):
        P.gfdtd_check(ring.replace(init_d=d[:-1]))


@pytest.mark.parametrize("kind", [W.MODULATION, W.MATTER])
def test_preflight_matches_oracle_scan(P, kind):
    """The library's pre-flight growth equals the oracle's amplification
    matrix scan (independent code, same Section 5 analysis)."""
    for beta in (0.0, 0.2, -0.3, 0.45, 0.7):
        for eps in (1.0, 2.5, 6.0):
            p = W.Problem(nz=16, steps=1, eps_rest=np.full(16, eps),
                          mu_rest=np.ones(16), beta=beta, kind=kind, src_cell=3,
                          flags=W.FLAG_ALLOW_UNSTABLE)
            g = P.gfdtd_check(p)
            want = st.max_growth(0.5, beta, eps, 1.0, kind, ntheta=512)
            assert abs(g - want) < 1e-9, (beta, eps, g, want)


def test_preflight_rejects_unstable_and_flag_overrides(P):
    p = W.small_case(100, 10, 0.3, seed=1, structure="uniform")
    p = p.replace(eps_rest=np.full(100, 16.0), mu_rest=np.ones(100), beta=0.3)
    with pytest.raises(P.GfdtdError) as e:
        P.gfdtd_check(p)
    assert e.value.status == P.gfdtd.GFDTD_E_UNSTABLE
    g = P.gfdtd_check(p.replace(flags=W.FLAG_ALLOW_UNSTABLE))
    assert g > 1.0


def test_sizes(P):
    p = _ok()
    t, d = P.gfdtd_result_sizes(p, 123)
    assert t == len(p.probes) * 123 and d == len(p.probes) * len(p.omegas)
    a = P.gfdtd_workspace_bytes(p, 100)
    b = P.gfdtd_workspace_bytes(p, 1000)
    assert 0 < a < b
    both = P.gfdtd_batch_workspace_bytes([p, p], [100, 100])
    assert both >= 2 * a - 4096
    with pytest.raises(P.GfdtdError):
        P.gfdtd_workspace_bytes(p, -1)


def test_benchmark_configs_pass_preflight(P):
    """Every benchmark configuration is drawn inside the stable region."""
    P.gfdtd_check(W.interface_run(0))
    P.gfdtd_check(W.slab_run(0, nz=4096, steps=10, slab=512))
    for p in W.crystal_runs(0, count=64):
        P.gfdtd_check(p)
    P.gfdtd_check(W.gradient_run(0, downscaled=True))


def test_time_window_validated_and_in_the_preflight(P):
    """A finite-duration window needs a moving modulation, a finite
    positive background and non-NaN switch times; the background medium
    enters the stability pre-flight."""
    p = W.small_case(200, 100, 0.3, seed=0, structure="uniform")
    p = p.replace(eps_rest=np.full(200, 2.0), mu_rest=np.ones(200))
    P.gfdtd_check(p.replace(window=W.TimeWindow(5.0, float("inf"), 1.0, 1.0)))
    for win in (W.TimeWindow(float("nan"), 9.0, 1.0, 1.0),
                W.TimeWindow(0.0, 9.0, 0.0, 1.0),
                W.TimeWindow(0.0, 9.0, 1.0, float("inf"))):
        with pytest.raises(P.GfdtdError) as e:
            P.gfdtd_check(p.replace(window=win))
        assert e.value.status == P.gfdtd.GFDTD_E_INVALID
    with pytest.raises(P.GfdtdError) as e:
        P.gfdtd_check(W.small_case(200, 100, 0.3, kind=W.MATTER, seed=0)
                      .replace(window=W.TimeWindow(0.0, 9.0, 1.0, 1.0)))
    assert e.value.status == P.gfdtd.GFDTD_E_UNSUPPORTED
    # beta n = 0.3 * 4 > 1 for the background alone: unstable
    with pytest.raises(P.GfdtdError) as e:
        P.gfdtd_check(p.replace(window=W.TimeWindow(0.0, 9.0, 16.0, 1.0)))
    assert e.value.status == P.gfdtd.GFDTD_E_UNSTABLE


def test_tmm_stacks_validated(P):
    """gfdtd_tmm_workspace_bytes validates every stack on the host: layer
    count, |beta| < 1 and |beta| n < 1 in each layer, positive media and
    non-negative widths."""
    import ctypes as C
    g = P.gfdtd
    lib = P.load_library()

    def check(stacks):
        arr, keep = g._tmm_structs(stacks)
        n = C.c_size_t(0)
        return lib.gfdtd_tmm_workspace_bytes(arr, len(stacks), 8, C.byref(n)), n.value

    ok = W.TmmStack(eps=np.array([1.0, 4.0, 1.0]), widths=np.array([10.0]), beta=0.3)
    st, n = check([ok])
    assert st == 0 and n > 0
    bad = [W.TmmStack(eps=np.array([1.0]), widths=np.zeros(0), beta=0.1),
           W.TmmStack(eps=np.array([1.0, 4.0, 1.0]), widths=np.array([-1.0]), beta=0.1),
           W.TmmStack(eps=np.array([1.0, 16.0, 1.0]), widths=np.array([5.0]), beta=0.3),
           W.TmmStack(eps=np.array([1.0, 0.0]), widths=np.zeros(0), beta=0.1),
           W.TmmStack(eps=np.array([1.0, 2.0]), widths=np.zeros(0), beta=1.0)]
    for b in bad:
        st, _ = check([ok, b])
        assert st == g.GFDTD_E_INVALID
        assert "stack 1" in g.load_library().gfdtd_last_error().decode()


@pytest.mark.parametrize("field,value", [
    ("cells_per_lane", 6), ("block_steps", 257), ("block_steps", -1),
    ("tile_waves", 5), ("tile_waves", -1), ("exchange_steps", 17),
    ("exchange_steps", -2),
])
def test_invalid_exec_options_rejected(P, field, value):
    """gfdtd_batch_prepare rejects execution options outside their ranges
    before it touches the device (null workspace and stream here)."""
    g = P.gfdtd
    lib = P.load_library()
    ms, arr, st = g._arrays([_ok()], None)
    e = g._exec_struct()
    setattr(e, field, value)
    h = ctypes.c_void_p(None)
    status = lib.gfdtd_batch_prepare(arr, st.ctypes.data_as(g._PI64), 1, ctypes.byref(e),
                                     None, 0, None, ctypes.byref(h))
    assert status == g.GFDTD_E_INVALID
    assert field.split("_")[0] in lib.gfdtd_last_error().decode()
    assert not h.value
