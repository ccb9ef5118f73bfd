"""CPU checks of the C-ABI boundary: the library loads, exports every entry
point include/coloc.h declares, its structs have the layout the binding
assumes, and the pure admission rule agrees with the oracle's."""
import ctypes
import ctypes as C
import math
import os
import re
import subprocess

import numpy as np
import pytest

import oracle
from paper_2501_16909_amd import coloc

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "coloc.h")


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:ci_status_t|const char\*)\s+(\w+)\s*\(", text, flags=re.M)))


def test_library_exports_every_declared_symbol():
    lib = coloc.load_library()
    names = _declared_functions()
    assert len(names) >= 17
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(coloc.EXPORTS), "binding and header disagree"


def test_struct_layouts_match_header(tmp_path):
    structs = {"ci_device_info_t": coloc.DeviceInfo, "ci_wg_record_t": coloc.WgRecord,
               "ci_stressor_opts_t": coloc.StressorOpts, "ci_stressor_report_t": coloc.StressorReport,
               "ci_victim_desc_t": coloc.VictimDesc, "ci_victim_result_t": coloc.VictimResult,
               "ci_measure_opts_t": coloc.MeasureOpts, "ci_cell_t": coloc.Cell,
               "ci_profile_t": coloc.Profile, "ci_request_t": coloc.Request,
               "ci_policy_t": coloc.Policy, "ci_served_t": coloc.Served,
               "ci_decode_config_t": coloc.DecodeConfig, "ci_decode_layout_t": coloc.DecodeLayout,
               "ci_decode_desc_t": coloc.DecodeDesc, "ci_decode_result_t": coloc.DecodeResult,
               "ci_decode_cell_t": coloc.DecodeCell, "ci_gemv_args_t": coloc.GemvArgs}
    src = tmp_path / "sz.c"
    lines = ['#include <stdio.h>', '#include <stddef.h>', f'#include "{HEADER}"', "int main(void){"]
    for cname, py in structs.items():
        lines.append(f'printf("{cname} %zu\\n", sizeof({cname}));')
        for f, _ in py._fields_:
            lines.append(f'printf("{cname}.{f} %zu\\n", offsetof({cname}, {f}));')
    lines.append('printf("CI_NOALLOC_PART_BYTES %llu\\n", (unsigned long long)CI_NOALLOC_PART_BYTES);')
    lines.append("return 0;}")
    src.write_text("\n".join(lines))
    exe = tmp_path / "sz"
    subprocess.check_call(["gcc", "-o", str(exe), str(src)])
    out = dict(l.rsplit(" ", 1) for l in subprocess.check_output([str(exe)], text=True).splitlines())
    for cname, py in structs.items():
        assert int(out[cname]) == ctypes.sizeof(py), cname
        for f, _ in py._fields_:
            assert int(out[f"{cname}.{f}"]) == getattr(py, f).offset, f"{cname}.{f}"
    assert ctypes.sizeof(coloc.WgRecord) == 48
    assert int(out["CI_NOALLOC_PART_BYTES"]) == coloc.NOALLOC_PART_BYTES


def test_errors_are_reported_without_a_device():
    lib = coloc.load_library()
    assert lib.ci_init(0, None) == 1
    assert b"NULL" in lib.ci_last_error()
    assert lib.stressor_stop(None, None) == 1
    assert lib.ci_shutdown(None) == 0
    size = ctypes.c_size_t()
    assert lib.ci_workspace_size(99, 1.0, None, ctypes.byref(size)) == 1
    assert lib.ci_workspace_size(0, float("nan"), None, ctypes.byref(size)) == 1
    assert lib.ci_workspace_size(0, 1.5, None, ctypes.byref(size)) == 1
    assert lib.ci_workspace_size(0, 1.0, None, ctypes.byref(size)) == 0
    ctrl = 2304                              # control words and the XCD slots' ticket lines
    assert size.value == ctrl + 256 * 1 * 48   # records for one work-group per CU
    assert lib.ci_workspace_size(0, 0.5, None, ctypes.byref(size)) == 0
    assert size.value == ctrl + 128 * 1 * 48   # 8 x round(32 x 0.5) CUs
    assert lib.ci_workspace_size(0, 0.0, None, ctypes.byref(size)) == 0
    assert size.value == ctrl
    # the L2 stressor's default shape is three work-groups per CU
    assert lib.ci_workspace_size(1, 0.25, None, ctypes.byref(size)) == 0
    assert size.value == ctrl + 64 * 3 * 48


def _profiles(read_curves=False):
    # fragile: 3x slowdown under full HBM pressure; hog: exerts full HBM pressure
    p = {
        "gemv": {"sens": {"hbm": [1.0, 1.5, 2.0, 2.5, 3.0]}, "press": {"hbm": 0.2}, "occ": 0.6,
                 "hbm_write_frac": 0.0, "press_hbm_read": 0.15},
        "triad": {"sens": {"hbm": [1.0, 1.1, 1.2, 1.3, 1.4]}, "press": {"hbm": 1.0}, "occ": 0.6,
                  "hbm_write_frac": 1 / 3, "press_hbm_read": 0.9},
        "gemm": {"sens": {"lds": [1.0, 1.0, 1.0, 1.0, 1.0], "hbm": [1.0, 1.2, 1.3, 1.5, 2.0]},
                 "press": {"mfma_bf16": 0.9, "hbm": 0.1}, "occ": 0.3, "hbm_write_frac": 0.5,
                 "press_hbm_read": 0.08},
    }
    if read_curves:
        p["gemv"]["sens_hbm_read"] = [1.0, 1.2, 1.3, 1.4, 1.6]
        p["gemm"]["sens_hbm_read"] = [1.0, 1.05, 1.1, 1.2, 1.25]
    return p


def _oracle_job(p):
    # the library stores curves and pressures as FP32: round the same way
    f32 = lambda v: float(np.float32(v))
    sens = [[f32(v) for v in p["sens"].get(r, [1.0] * 5)] for r in coloc.RESOURCES]
    press = [f32(p["press"].get(r, 0.0)) for r in coloc.RESOURCES]
    job = {"sens": sens, "press": press, "bytes": 1, "occ": f32(p["occ"]),
           "hbm_write_frac": f32(p.get("hbm_write_frac", 1.0)), "press_hbm_read": f32(p.get("press_hbm_read", 0.0))}
    if "sens_hbm_read" in p:
        job["sens_hbm_read"] = [f32(v) for v in p["sens_hbm_read"]]
    return job


def test_predicted_slowdown_matches_oracle():
    """ci_predict_slowdown (host code, no device) against the oracle's
    read/write-aware estimator, over every victim and co-runner multiset of
    up to three, with and without read-only HBM curves, and on random
    profiles."""
    import itertools
    for rc in (False, True):
        profs = _profiles(read_curves=rc)
        kinds = list(profs)
        for v in kinds:
            for nco in range(0, 4):
                for co in itertools.combinations_with_replacement(kinds, nco):
                    got = coloc.predict_slowdown(profs, v, list(co))
                    want = oracle.predicted_slowdown_rw(_oracle_job(profs[v]), [_oracle_job(profs[k]) for k in co])
                    assert got == pytest.approx(want, rel=1e-12, abs=0), (rc, v, co)
    rng = np.random.default_rng(9)
    for _ in range(200):
        profs = {}
        for k in ("gemm", "gemv", "triad"):
            profs[k] = {"sens": {r: sorted(1.0 + 3.0 * rng.random(5)) for r in ("hbm", "l2", "lds")},
                        "press": {r: float(rng.random()) for r in ("hbm", "l2", "lds")}, "occ": 0.5,
                        "hbm_write_frac": float(rng.choice([0.0, 0.1, 1 / 6, 0.5])),
                        "press_hbm_read": float(rng.random())}
            if rng.random() < 0.7:
                profs[k]["sens_hbm_read"] = sorted(1.0 + rng.random(5))
        co = list(rng.choice(list(profs), int(rng.integers(0, 4))))
        got = coloc.predict_slowdown(profs, "gemv", co)
        want = oracle.predicted_slowdown_rw(_oracle_job(profs["gemv"]), [_oracle_job(profs[k]) for k in co])
        assert got == pytest.approx(want, rel=1e-12)


@pytest.mark.parametrize("policy", ["naive", "usher", "sensitivity"])
@pytest.mark.parametrize("bound", [1.2, 1.5, 2.5, math.inf])
@pytest.mark.parametrize("read_curves", [False, True])
def test_admission_matches_oracle(policy, bound, read_curves):
    profs = _profiles(read_curves)
    kinds = list(profs)
    import itertools
    for nrun in range(0, 3):
        for running in itertools.product(kinds, repeat=nrun):
            for cand in kinds:
                got = coloc.admit(policy, profs, list(running), cand, 10, 100, bound=bound, slots=4)
                want = oracle.admit(policy, [_oracle_job(profs[k]) for k in running],
                                    _oracle_job(profs[cand]), 100, bound, 4)
                assert got == want, (policy, bound, running, cand)
    assert not coloc.admit("naive", profs, [], "gemv", 101, 100)
    assert not coloc.admit("naive", profs, ["gemv"] * 4, "gemv", 1, 100, slots=4)
    # an idle device admits whatever fits, under every policy and bound
    greedy = {"triad": dict(profs["triad"], occ=1.0, sens={"hbm": [9.0] * 5})}
    assert coloc.admit(policy, greedy, [], "triad", 10, 100, bound=1.0001)



@pytest.mark.parametrize("policy", ["naive", "usher", "sensitivity"])
@pytest.mark.parametrize("read_curves", [False, True])
def test_admission_with_background_matches_oracle(policy, read_curves):
    """ci_admit with a background load (ci_policy_t.background) against the
    oracle's rule, over running sets of up to two, every candidate, several
    bounds, and background loads that are write-heavy (priced on the triad
    curve), read-mostly (priced on the read-only curve when the victim has
    one) or occupancy-only."""
    import itertools
    profs = _profiles(read_curves)
    kinds = list(profs)
    loads = [{"press": {"hbm": 0.5}, "occ": 0.25, "hbm_write_frac": 1 / 3},
             {"press": {"hbm": 0.75}, "occ": 0.0, "hbm_write_frac": 0.0, "press_hbm_read": 0.6},
             {"press": {"mfma_bf16": 0.4, "lds": 0.3}, "occ": 0.45, "hbm_write_frac": 1.0}]
    checked = refused = 0
    for load in loads:
        bgo = _oracle_job(dict(load, sens={}))
        for bound in (1.2, 1.6, 2.5):
            for nrun in range(0, 3):
                for running in itertools.product(kinds, repeat=nrun):
                    for cand in kinds:
                        got = coloc.admit(policy, profs, list(running), cand, 10, 100, bound=bound, slots=4,
                                          background=load)
                        want = oracle.admit(policy, [_oracle_job(profs[k]) for k in running],
                                            _oracle_job(profs[cand]), 100, bound, 4, background=bgo)
                        assert got == want, (policy, load, bound, running, cand)
                        checked += 1
                        refused += not got
    assert checked == 3 * 3 * 13 * 3
    for load in loads:          # a load profile as a co-runner of ci_predict_slowdown
        bgo = _oracle_job(dict(load, sens={}))
        for v in kinds:
            got = coloc.predict_slowdown(profs, v, ["triad", load])
            want = oracle.predicted_slowdown_rw(_oracle_job(profs[v]), [_oracle_job(profs["triad"]), bgo])
            assert got == pytest.approx(want, rel=1e-12, abs=0), (v, load)
    if policy != "naive":
        assert 0 < refused < checked


def test_serve_run_background_argument_checks():
    """serve_run_background refuses, before touching any device, a missing
    options block or report, a stressor with a fixed pass count, and a NULL
    context."""
    lib = coloc.load_library()
    pol = coloc.Policy(0, 1.5, 1 << 30, 4, None, 0, None)
    rep = coloc.StressorReport()
    opts = coloc.StressorOpts()
    out = (coloc.Served * 1)()
    st = lib.serve_run_background(None, None, 0, C.byref(pol), coloc.RES["hbm"], 1.0, None, None, 0, out,
                                  C.byref(rep))
    assert st == 1 and b"NULL opts" in lib.ci_last_error()
    st = lib.serve_run_background(None, None, 0, C.byref(pol), coloc.RES["hbm"], 1.0, C.byref(opts), None, 0,
                                  out, None)
    assert st == 1
    opts.passes = 1
    st = lib.serve_run_background(None, None, 0, C.byref(pol), coloc.RES["hbm"], 1.0, C.byref(opts), None, 0,
                                  out, C.byref(rep))
    assert st == 1 and b"passes" in lib.ci_last_error()
    opts.passes = 0
    st = lib.serve_run_background(None, None, 0, C.byref(pol), coloc.RES["hbm"], 1.0, C.byref(opts), None, 0,
                                  out, C.byref(rep))
    assert st == 1 and b"serve_run: bad argument" in lib.ci_last_error()

def test_admission_rejects_an_unknown_policy_first():
    """An unknown policy is an argument error whatever the request, also one
    that would not fit."""
    profs = _profiles(False)
    arr = coloc.make_profiles(profs)
    for cand_bytes in (10, 10 ** 6):
        pol = coloc.Policy(7, 1.5, 1 << 40, 4, C.cast(arr, C.POINTER(coloc.Profile)), len(profs))
        out = C.c_int(5)
        st = coloc.load_library().ci_admit(C.byref(pol), None, 0, coloc.VICTIMS["gemv"], cand_bytes, 100,
                                           C.byref(out))
        assert st == 1, cand_bytes


LLAMA8B = dict(hidden=4096, n_q=32, n_kv=8, head_dim=128, ffn=14336, vocab=128256, layers=32, batch=1,
               max_ctx=4096, eps=1e-5, rope_base=500000.0)


def test_decode_layout_sizes_and_alignment():
    """The weight arena holds every tensor once, each 128-byte aligned (Llama
    3.1 8B: 8.03 B parameters, less the 0.53 B input-embedding table the
    step does not read)."""
    lay = coloc.Context.decode_layout(LLAMA8B)
    per_layer = 4096 + 6144 * 4096 + 4096 * 4096 + 4096 + 2 * 14336 * 4096 + 4096 * 14336
    assert lay.layer_stride == per_layer                 # every size already a multiple of 64
    assert lay.weight_elems == 32 * per_layer + 4096 + 128256 * 4096
    assert abs(lay.weight_elems + 128256 * 4096 - 8.03e9) < 0.01e9
    for f in ("g_attn", "w_qkv", "w_o", "g_mlp", "w_gu", "w_down", "layer_stride", "g_final", "w_lm"):
        assert getattr(lay, f) % 64 == 0, f
    assert (lay.g_attn, lay.w_qkv) == (0, 4096)
    assert lay.w_o == lay.w_qkv + 6144 * 4096 and lay.g_mlp == lay.w_o + 4096 * 4096
    assert lay.cache_elems == 32 * 1 * 8 * 4096 * 128
    assert lay.attn_part_bytes == 1 * 32 * 64 * 130 * 4
    small = dict(LLAMA8B, hidden=520, ffn=72, n_q=3, n_kv=1, vocab=7, layers=2, max_ctx=65, batch=3)
    lay = coloc.Context.decode_layout(small)
    assert lay.g_attn == 0 and lay.w_qkv == 576            # 520 rounded up to 64
    assert lay.layer_stride % 64 == 0 and lay.w_lm % 64 == 0
    assert lay.attn_part_bytes == 3 * 3 * 2 * 130 * 4


@pytest.mark.parametrize("bad", [dict(hidden=4100), dict(ffn=0), dict(head_dim=64), dict(n_q=12, n_kv=5),
                                 dict(n_q=34, n_kv=2), dict(layers=0), dict(batch=9), dict(batch=0),
                                 dict(max_ctx=0), dict(rope_base=0.0), dict(eps=-1.0)])
def test_decode_layout_rejects_bad_configs(bad):
    with pytest.raises(coloc.CiError) as ei:
        coloc.Context.decode_layout(dict(LLAMA8B, **bad))
    assert ei.value.status == 1


def test_bootstrap_interval_matches_oracle():
    """The library's bootstrap interval (host code, no device) against the
    oracle's on seeded samples of odd and even sizes."""
    rng = np.random.default_rng(5)
    for na, nc, seed in ((20, 20, 0), (7, 12, 16909), (1, 9, 3), (41, 41, 123456789)):
        a = 100.0 + rng.standard_normal(na)
        c = 150.0 + 5 * rng.standard_normal(nc)
        got = coloc.bootstrap_slowdown(a, c, 1000, seed)
        want = oracle.bootstrap_slowdown_ci(a, c, 1000, seed)
        assert got == pytest.approx(want, rel=1e-12), (na, nc, seed)
    with pytest.raises(coloc.CiError) as ei:
        coloc.bootstrap_slowdown([], [1.0])
    assert ei.value.status == 1

