"""Host-only checks of the C ABI: the library loads, exports every declared symbol,
and the plan (no device work) validates, clamps and sizes correctly."""
import ctypes
import os
import re
import subprocess

import pytest

import oracle as O
from paper_2008_01340_amd import ntt

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ntt.h")


def _declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?\w+\*?\s+\**(ntt_\w+)\s*\(", src, flags=re.M)
    return sorted(set(names))


@pytest.fixture(scope="module")
def lib():
    return ntt.load()


def test_header_declares_the_expected_entry_points():
    names = _declared_functions()
    for want in ["ntt_plan", "ntt_decompose", "ntt_reconstruct", "ntt_rel_error"]:
        assert want in names
    assert sorted(names) == sorted(ntt.EXPORTED)


def test_library_exports_every_declared_symbol(lib):
    for name in _declared_functions():
        assert hasattr(lib, name), name
    out = subprocess.run(["nm", "-D", "--defined-only", ntt.LIB_PATH], capture_output=True,
                         text=True).stdout
    exported = {line.split()[-1] for line in out.splitlines() if line.strip()}
    for name in _declared_functions():
        assert name in exported, name


def test_version_and_status_strings(lib):
    assert "gfx950" in ntt.ntt_version()
    for s in range(7):
        assert lib.ntt_status_string(s).decode()
    assert lib.ntt_status_string(99).decode() == "unknown status"


def test_plan_clamps_ranks_like_the_oracle():
    for dims, ranks in [((2, 3, 4), (1, 5, 5, 1)), ((16, 16, 16), (1, 4, 4, 1)),
                        ((4, 100, 2), (1, 50, 50, 1)), ((3, 3, 3, 3), (1, 9, 9, 9, 1))]:
        p = ntt.Plan(dims, ranks, 10)
        nbytes, eff, comp = p.workspace()
        assert eff == O.effective_ranks(dims, ranks)
        assert comp == pytest.approx(O.compression_ratio(dims, eff), rel=1e-14)
        assert nbytes > 0 and nbytes % 256 == 0


def test_plan_strict_ranks_errors():
    with pytest.raises(ntt.NttError) as e:
        ntt.Plan((2, 3, 4), (1, 5, 5, 1), 10, flags=ntt.NTT_STRICT_RANKS)
    assert e.value.status == ntt.NTT_ERR_RANK_INFEASIBLE
    ntt.Plan((16, 16, 16), (1, 4, 4, 1), 10, flags=ntt.NTT_STRICT_RANKS)


@pytest.mark.parametrize("kw,dims,ranks", [
    ({}, (5,), (1, 1)),                          # d < 2
    ({}, (4, 0, 3), (1, 2, 2, 1)),               # zero mode
    ({}, (4, 5, 3), (2, 2, 2, 1)),               # r_0 != 1
    ({}, (4, 5, 3), (1, 2, 2, 3)),               # r_d != 1
    ({}, (4, 5, 3), (1, 0, 2, 1)),               # zero rank
    ({"max_iters": -1}, (4, 5), (1, 2, 1)),
    ({"check_every": 0}, (4, 5), (1, 2, 1)),
    ({"eps": -1.0}, (4, 5), (1, 2, 1)),
    ({"eps": float("nan")}, (4, 5), (1, 2, 1)),
    ({"tol": -0.1}, (4, 5), (1, 2, 1)),
    ({"precision": 7}, (4, 5), (1, 2, 1)),
    ({}, (64, 64, 64), (1, 40, 40, 1)),          # effective rank above 32
    ({}, (1 << 32, 1 << 32, 4), (1, 1, 1, 1)),   # product overflows
    ({"rank_eps": -0.1}, (4, 5), (1, 2, 1)),
    ({"rank_eps": float("inf")}, (4, 5), (1, 2, 1)),
    ({"rank_eps": 0.1}, (3000, 3000), (1, 8, 1)),  # rank rule: shorter side above 2048
    ({"nmf": "bcd", "precision": 1}, (4, 5), (1, 2, 1)),  # BCD runs in FP32 only
    ({"nmf": "bcd", "tol": 1e-3}, (4, 5), (1, 2, 1)),     # BCD: fixed iteration count
    ({"nmf": "bcd", "delta": 1.0}, (4, 5), (1, 2, 1)),
    ({"nmf": "bcd", "delta": -0.5}, (4, 5), (1, 2, 1)),
    ({"nmf": "bcd", "delta": float("nan")}, (4, 5), (1, 2, 1)),
    ({"nmf": "bcd"}, (5000000, 2), (1, 1, 1)),  # BCD: more rows than its grid takes
    ({"stream_cols": -1}, (4, 5), (1, 2, 1)),
    ({"stream_cols": 64, "precision": 1}, (4, 5), (1, 2, 1)),  # streaming: MU in FP32 only
    ({"stream_cols": 64, "nmf": "bcd"}, (4, 5), (1, 2, 1)),
    ({"stream_cols": 64, "rank_eps": 0.1}, (3000, 4), (1, 2, 1)),  # streamed rule: n_1 > 2048
    ({"stream_cols": 64, "tol": 1e-3}, (4, 5), (1, 2, 1)),
    ({"stream_cols": 64, "flags": 4}, (4, 5), (1, 2, 1)),  # no objective trace
])
def test_plan_rejects_invalid_configs(kw, dims, ranks):
    args = {"max_iters": 10}
    args.update(kw)
    it = args.pop("max_iters")
    with pytest.raises(ntt.NttError) as e:
        ntt.Plan(dims, ranks, it, **args)
    assert e.value.status == ntt.NTT_ERR_INVALID_ARG


def test_plan_null_pointers(lib):
    assert lib.ntt_plan(None, None) == ntt.NTT_ERR_INVALID_ARG
    assert lib.ntt_plan_workspace(None, None, None, None) == ntt.NTT_ERR_INVALID_ARG
    assert "null" in lib.ntt_last_error().decode()
    lib.ntt_plan_destroy(None)  # no-op


def test_decompose_argument_errors_without_device_work(lib):
    p = ntt.Plan((4, 5), (1, 2, 1), 3)
    # null workspace and null tensor are rejected before any HIP call
    st = lib.ntt_decompose(p.handle, None, None, None, None, None, None, None, None)
    assert st == ntt.NTT_ERR_WORKSPACE_TOO_SMALL
    st = lib.ntt_decompose(p.handle, None, ctypes.c_void_p(256), None, None, None, None, None, None)
    assert st == ntt.NTT_ERR_INVALID_ARG
    st = lib.ntt_decompose(p.handle, None, ctypes.c_void_p(257), ctypes.c_void_p(256),
                           ntt._ptrs([256, 512]), None, None, None, None)
    assert st == ntt.NTT_ERR_INVALID_ARG  # misaligned workspace


def test_tt_workspace_and_validation():
    n = ntt.ntt_tt_workspace((4, 5, 6), (1, 2, 3, 1))
    assert n >= 2 * 8 and n % 256 == 0
    for dims, ranks in [((4,), (1, 1)), ((4, 5), (1, 33, 1)), ((4, 5), (2, 2, 1))]:
        with pytest.raises(ntt.NttError):
            ntt.ntt_tt_workspace(dims, ranks)


def test_compression_ratio_entry_point_matches_eq4_pins():
    assert ntt.ntt_compression_ratio((48, 42, 64, 38), (1, 1, 1, 1, 1)) == pytest.approx(25536.0)
    assert ntt.ntt_compression_ratio((100, 260, 3, 85), (1, 1, 1, 1, 1)) == pytest.approx(14799.107142857143)


def test_workspace_scales_with_the_problem():
    small = ntt.Plan((16, 16, 16), (1, 4, 4, 1), 10).workspace()[0]
    big = ntt.Plan((32,) * 5, (1, 8, 8, 8, 8, 1), 10).workspace()[0]
    # the 32^5 sweep holds H_1 (8 x 32^4 floats) in the workspace
    assert big >= 8 * 32 ** 4 * 4
    assert small < big


def test_rank_rule_plan_reports_caps_and_covers_every_rank():
    # with rank_eps > 0 the planned ranks are caps: the query reports them, and the
    # workspace covers the caps' plan plus the Gram, eigenvalues and solver scratch
    dims, ranks = (20, 24, 30, 18), (1, 12, 16, 9, 1)
    given = ntt.Plan(dims, ranks, 10)
    rule = ntt.Plan(dims, ranks, 10, rank_eps=0.05)
    wg, eg, cg = given.workspace()
    wr, er, cr = rule.workspace()
    assert er == eg == [1, 12, 16, 9, 1] and cr == cg
    assert wr >= wg + 8 * (24 * 12) ** 2  # at least the largest Gram (288 x 288 FP64)
    lib = ntt.load()
    cfgs = (ntt.NttConfig * 1)()
    b = ntt.Plan((4, 5), (1, 2, 1), 10, rank_eps=0.1)
    cfgs[0] = b.cfg
    out = ctypes.c_void_p()
    assert lib.ntt_batch_plan(1, cfgs, ctypes.byref(out)) == ntt.NTT_ERR_INVALID_ARG


def test_batch_plan_validation_and_workspace():
    b = ntt.Batch([((4, 5, 6), (1, 2, 3, 1), 1), ((8, 8), (1, 3, 1), 2)], 10)
    single = sum(ntt.Plan(dm, rk, 10).workspace()[0] for dm, rk, _ in b.problems)
    assert b.workspace_bytes >= single
    assert b.eff == [[1, 2, 3, 1], [1, 3, 1]]
    with pytest.raises(ntt.NttError):
        ntt.Batch([((4, 5, 6), (1, 2, 3, 2), 1)], 10)  # r_d != 1
    lib = ntt.load()
    assert lib.ntt_batch_plan(0, None, None) == ntt.NTT_ERR_INVALID_ARG


def test_unknown_nmf_is_rejected_and_batched_bcd_is_planned(lib):
    dims, ranks = ntt._i64([4, 5]), ntt._i64([1, 2, 1])
    cfg = ntt.NttConfig(2, ctypes.cast(dims, ctypes.POINTER(ctypes.c_int64)),
                        ctypes.cast(ranks, ctypes.POINTER(ctypes.c_int64)), 5, 0.0, 10, 1e-12, 0,
                        0, 0, 0, 0.0, 2, 0.9999)
    h = ctypes.c_void_p()
    assert lib.ntt_plan(ctypes.byref(cfg), ctypes.byref(h)) == ntt.NTT_ERR_INVALID_ARG
    assert "nmf" in lib.ntt_last_error().decode()
    cfg.nmf = ntt.NTT_NMF_BCD  # batched mode takes BCD problems
    assert lib.ntt_batch_plan(1, ctypes.byref(cfg), ctypes.byref(h)) == ntt.NTT_OK
    lib.ntt_batch_destroy(h)


def test_bcd_workspace_adds_two_h_buffers():
    dims, ranks = (32, 32, 32), (1, 8, 8, 1)
    mu = ntt.Plan(dims, ranks, 10).workspace()[0]
    bcd = ntt.Plan(dims, ranks, 10, nmf="bcd").workspace()[0]
    assert bcd >= mu + 2 * 8 * 32 * 32 * 4


def test_streamed_plan_adds_staging_and_batch_rejects_it(lib):
    dims, ranks = (32, 32, 32, 32), (1, 8, 8, 8, 1)
    resident = ntt.Plan(dims, ranks, 10).workspace()[0]
    streamed = ntt.Plan(dims, ranks, 10, stream_cols=1000).workspace()[0]
    # staging for a 32 x 1000 block of X and an 8 x 1000 block of H
    assert streamed >= resident + (32 + 8) * 1000 * 4
    d, r = ntt._i64([4, 5]), ntt._i64([1, 2, 1])
    cfg = ntt.NttConfig(2, ctypes.cast(d, ctypes.POINTER(ctypes.c_int64)),
                        ctypes.cast(r, ctypes.POINTER(ctypes.c_int64)), 5, 0.0, 10, 1e-12, 0,
                        0, 0, 0, 0.0, 0, 0.9999, 64)
    h = ctypes.c_void_p()
    assert lib.ntt_batch_plan(1, ctypes.byref(cfg), ctypes.byref(h)) == ntt.NTT_ERR_INVALID_ARG


def test_struct_layouts_match_the_c_header(tmp_path):
    # the binding's ctypes structs against sizeof/offsetof compiled from include/ntt.h
    import shutil
    import subprocess
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("no C compiler")
    inc = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include")
    src = tmp_path / "layout.c"
    src.write_text(
        '#include <stddef.h>\n#include <stdio.h>\n#include "ntt.h"\n'
        "int main(void) {\n"
        '  printf("%zu %zu %zu %zu %zu %zu %zu %zu\\n", sizeof(ntt_config), sizeof(ntt_report),\n'
        "         offsetof(ntt_config, nmf), offsetof(ntt_config, bcd_delta),\n"
        "         offsetof(ntt_config, stream_cols), offsetof(ntt_report, corrections),\n"
        "         sizeof(ntt_request), offsetof(ntt_request, bcd_delta));\n"
        "  return 0;\n}\n")
    exe = tmp_path / "layout"
    subprocess.run([gcc, "-std=c99", "-I" + inc, str(src), "-o", str(exe)], check=True)
    got = [int(v) for v in subprocess.run([str(exe)], check=True, capture_output=True,
                                          text=True).stdout.split()]
    want = [ctypes.sizeof(ntt.NttConfig), ctypes.sizeof(ntt.NttReport),
            ntt.NttConfig.nmf.offset, ntt.NttConfig.bcd_delta.offset,
            ntt.NttConfig.stream_cols.offset, ntt.NttReport.corrections.offset,
            ctypes.sizeof(ntt.NttRequest), ntt.NttRequest.bcd_delta.offset]
    assert got == want
