"""Host-side checks of the C ABI that need no GPU: the library loads, exports
every symbol the header declares, and rejects bad configurations before any
device call."""
import ctypes
import os
import re

import numpy as np
import pytest

import workloads as wk
import paper_2602_14854_amd as pkg
from paper_2602_14854_amd import _native as nat

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "dd_dlra.h")

needs_lib = pytest.mark.skipif(not os.path.exists(pkg.library_path()), reason="HIP library not built")


def declared_functions():
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"\b(dd_dlra_[a-z_]+)\s*\(", txt)))


def test_header_and_binding_agree():
    assert declared_functions() == sorted(nat.EXPORTS)


@needs_lib
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(pkg.library_path())
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_config_struct_layout_matches_header(tmp_path):
    """Compile a host-only C probe against the header and compare the size
    and field offsets of dd_dlra_config with the ctypes mirror."""
    import shutil
    import subprocess
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    fields = [f[0] for f in nat.Config._fields_]
    src = tmp_path / "probe.c"
    body = "\n".join(f'  printf("%s %zu\\n", "{f}", offsetof(dd_dlra_config, {f}));' for f in fields)
    src.write_text("#include <stdio.h>\n#include <stddef.h>\n#include \"dd_dlra.h\"\nint main(void){\n"
                   f'  printf("sizeof %zu\\n", sizeof(dd_dlra_config));\n{body}\n  return 0;\n}}\n')
    exe = tmp_path / "probe"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = dict(line.split() for line in subprocess.run([str(exe)], capture_output=True, text=True,
                                                      check=True).stdout.splitlines())
    assert int(out["sizeof"]) == ctypes.sizeof(nat.Config)
    for f in fields:
        assert int(out[f]) == getattr(nat.Config, f).offset, f


def _cfg(**over):
    wl = wk.make_workload("wc-C1")
    for k, v in over.items():
        setattr(wl, k, v)
    return wl


@needs_lib
def test_workspace_size_scales_with_problem():
    dirs = wk.product_directions(4, 4)
    a = pkg.workspace_size(wk.make_custom(8, 8, 2, 2, dirs, [3] * 4))
    b = pkg.workspace_size(wk.make_custom(16, 16, 2, 2, dirs, [3] * 4))
    c = pkg.workspace_size(wk.make_custom(16, 16, 4, 4, dirs, [3] * 16))
    assert 0 < a < b < c


@needs_lib
def test_mixed_precision_workspace_halves_the_working_arrays():
    """The mixed modes store the K-, L-step and V-hat working arrays (two of
    N x t, three of M x t per subdomain) in FP32; everything else stays FP64."""
    wl = wk.make_custom(32, 32, 2, 2, wk.product_directions(8, 8), [5] * 4)
    f64 = pkg.workspace_size(wl, precision=pkg.DD_PREC_FP64)
    f32 = pkg.workspace_size(wl, precision=pkg.DD_PREC_MIXED_FP32)
    bf16 = pkg.workspace_size(wl, precision=pkg.DD_PREC_MIXED_BF16)
    assert f32 == bf16
    saved = 4 * wl.n_sub * wl.r_int_max * (2 * wl.N + 3 * wl.M)
    assert abs((f64 - f32) - saved) <= 6 * 256


@needs_lib
def test_unknown_precision_rejected():
    with pytest.raises(nat.DDError) as ei:
        pkg.workspace_size(_cfg(), precision=7)
    assert ei.value.status == nat.DD_EINVAL
    assert "precision" in str(ei.value)


@needs_lib
@pytest.mark.parametrize("over,needle", [
    (dict(nx=33), "divisible"),
    (dict(x1=5.0), "square"),
    (dict(dt=0.0), "dt"),
    (dict(r_int_max=3), "r_int_max"),
    (dict(r_int_max=130), "128"),
    (dict(r_fixed=70, r_int_max=128), "64"),
    (dict(rank_mode=7), "rank_mode"),
])
def test_invalid_configs_rejected(over, needle):
    with pytest.raises(nat.DDError) as ei:
        pkg.workspace_size(_cfg(**over))
    assert ei.value.status == nat.DD_EINVAL
    assert needle in str(ei.value)


@needs_lib
@pytest.mark.parametrize("name", ["C4", "C5"])
def test_largest_configurations_accepted(name):
    """The adaptive configurations with stored ranks up to 40 / 64 and
    intermediate ranks up to 80 / 128 fit the engine's capacities (the wide
    launch plan)."""
    wl = wk.make_workload(name)
    n = pkg.workspace_size(wl)
    assert n > wl.n_sub * wl.N * wl.r_max * 8


@needs_lib
def test_rk4_substeps_accepted_in_fp64_only():
    """RK4 substeps take the wide launch plan in FP64; the mixed-precision
    modes refuse them, and an unknown integrator is refused by the binding."""
    assert pkg.workspace_size(_cfg(integrator="rk4")) > pkg.workspace_size(_cfg())
    with pytest.raises(nat.DDError) as ei:
        pkg.workspace_size(_cfg(integrator="rk4"), precision=pkg.DD_PREC_MIXED_FP32)
    assert ei.value.status == nat.DD_EINVAL and "RK4" in str(ei.value)
    with pytest.raises(ValueError):
        pkg.workspace_size(_cfg(integrator="midpoint"))


@needs_lib
def test_negative_cross_section_rejected():
    wl = _cfg()
    wl.sigma_s = wl.sigma_s.copy()
    wl.sigma_s[3] = -1.0
    with pytest.raises(nat.DDError) as ei:
        pkg.workspace_size(wl)
    assert "non-negative" in str(ei.value)


@needs_lib
def test_nonorthonormal_factors_rejected_before_device_use():
    wl = _cfg()
    wl.U0 = [2.0 * u for u in wl.U0]
    with pytest.raises(nat.DDError) as ei:
        pkg.DDDLRA(wl)
    assert ei.value.status == nat.DD_EINVAL and "orthonormal" in str(ei.value)


@needs_lib
def test_nan_factors_rejected_before_device_use():
    wl = _cfg()
    S = [s.copy() for s in wl.S0]
    S[1][0, 0] = np.nan
    wl.S0 = S
    with pytest.raises(nat.DDError) as ei:
        pkg.DDDLRA(wl)
    assert "non-finite" in str(ei.value)


@needs_lib
def test_rank_above_capacity_rejected():
    wl = _cfg()
    rng = np.random.default_rng(0)
    u, s, v = wk.random_factors(wl.N, wl.M, 6, wl.h, wl.w, rng)
    wl.U0 = [u] + wl.U0[1:]
    wl.S0 = [s] + wl.S0[1:]
    wl.V0 = [v] + wl.V0[1:]
    with pytest.raises(nat.DDError) as ei:
        pkg.DDDLRA(wl)
    assert "capacity" in str(ei.value)


def test_bench_refuses_more_than_one_gpu():
    """bench.py measures one GPU: --gpus 2 exits with status 2 and says so,
    before touching any device."""
    import subprocess
    import sys
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in (r.stdout + r.stderr)


def test_capacity_variant_of_the_uneven_rank_workload():
    """C4cap keeps C4's geometry and material layout but caps ranks at the
    engine's capacity: initial ranks in 2..21, r_int_max 42, adaptive."""
    a, b = wk.make_workload("C4"), wk.make_workload("C4cap")
    assert (a.nx, a.px, a.w.shape, a.tol) == (b.nx, b.px, b.w.shape, b.tol)
    assert np.array_equal(a.sigma_s, b.sigma_s)
    assert (b.r_max, b.r_int_max, b.rank_mode) == (21, 42, wk.RANK_ADAPTIVE)
    ranks = [S.shape[0] for S in b.S0]
    assert min(ranks) >= 2 and max(ranks) <= 21 and len(set(ranks)) > 5
    assert (a.r_max, a.r_int_max) == (40, 80)


@pytest.mark.parametrize("name", ["C1", "C2", "wc-C2", "C4cap"])
def test_workloads_are_seeded(name):
    """Every input is generated from its seed: two builds agree bit for bit,
    and another seed gives other initial factors."""
    a, b = wk.make_workload(name), wk.make_workload(name)
    for fa, fb in ((a.U0, b.U0), (a.S0, b.S0), (a.V0, b.V0)):
        assert all(np.array_equal(x, y) for x, y in zip(fa, fb))
    assert np.array_equal(a.sigma_s, b.sigma_s) and np.array_equal(a.Q, b.Q) and np.array_equal(a.w, b.w)
    c = wk.make_workload(name, seed=a.seed + 1)
    assert not all(np.array_equal(x, y) for x, y in zip(a.S0 + a.V0, c.S0 + c.V0))


def test_build_flags_tall_skinny_scratch():
    """The build's resource check: scratch memory of a tall-skinny kernel
    (k_*, kw_*) fails the build, that of a small per-subdomain kernel is
    allowed."""
    from paper_2602_14854_amd import build as b
    rem = ("a.hip:1:1: remark: Function Name: _ZN2dd12k_ang_reduceIdLi4ELi2EEEvNS_3DevEii [-Rpass]\n"
           "a.hip:1:1: remark:     ScratchSize [bytes/lane]: 304 [-Rpass]\n"
           "a.hip:2:1: remark: Function Name: _ZN2dd10sw_aug_svdENS_3DevEii [-Rpass]\n"
           "a.hip:2:1: remark:     ScratchSize [bytes/lane]: 80 [-Rpass]\n"
           "a.hip:3:1: remark: Function Name: _ZN2dd7kw_gemmIddLi0ELi4EEEvNS_3DevE [-Rpass]\n"
           "a.hip:3:1: remark:     ScratchSize [bytes/lane]: 0 [-Rpass]\n")
    rep = b.scratch_report(rem)
    assert [v for _, v in rep] == [304, 80, 0]
    flagged = [k for k, v in rep if v > 0 and b._TS_KERNEL.match(k)]
    assert flagged == ["_ZN2dd12k_ang_reduceIdLi4ELi2EEEvNS_3DevEii"]


@needs_lib
def test_inflow_faces_validated_and_sized():
    """A prescribed inflow on a physical face adds layer slots to the state
    arrays; rank, NULL-free arrays and finiteness are checked."""
    import dataclasses
    wl = _cfg()
    A = np.ones((wl.ny, 1))
    B = (np.asarray(wl.omega_x) >= 0).astype(float)[:, None]
    wi = dataclasses.replace(wl, inflow=[(A, B), None, None, None])
    assert pkg.workspace_size(wi) > pkg.workspace_size(wl)
    big = np.ones((wl.ny, wl.r_fixed + 1))
    with pytest.raises(nat.DDError) as ei:
        pkg.workspace_size(dataclasses.replace(wl, inflow=[(big, np.ones((wl.w.shape[0], wl.r_fixed + 1))),
                                                           None, None, None]))
    assert "inflow rank" in str(ei.value)
    bad = A.copy()
    bad[0, 0] = np.nan
    with pytest.raises(nat.DDError) as ei:
        pkg.workspace_size(dataclasses.replace(wl, inflow=[None, None, (np.ones((wl.nx, 1)), B), None]))
        pkg.workspace_size(dataclasses.replace(wl, inflow=[(bad, B), None, None, None]))
    assert "non-finite inflow" in str(ei.value)
