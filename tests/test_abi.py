"""CPU checks of the C-ABI boundary: the library loads, exports every entry
point include/coloc.h declares, its structs have the layout the binding
assumes, and the pure admission rule agrees with the oracle's."""
import ctypes
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
               "ci_policy_t": coloc.Policy, "ci_served_t": coloc.Served}
    src = tmp_path / "sz.c"
    lines = ['#include <stdio.h>', '#include <stddef.h>', f'#include "{HEADER}"', "int main(void){"]
    for cname, py in structs.items():
        lines.append(f'printf("{cname} %zu\\n", sizeof({cname}));')
        for f, _ in py._fields_:
            lines.append(f'printf("{cname}.{f} %zu\\n", offsetof({cname}, {f}));')
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


def test_errors_are_reported_without_a_device():
    lib = coloc.load_library()
    assert lib.ci_init(0, None) == 1
    assert b"NULL" in lib.ci_last_error()
    assert lib.stressor_stop(None, None) == 1
    assert lib.ci_shutdown(None) == 0
    size = ctypes.c_size_t()
    assert lib.ci_workspace_size(99, None, 256, ctypes.byref(size)) == 1
    assert lib.ci_workspace_size(0, None, 256, ctypes.byref(size)) == 0
    assert size.value == 256 + 256 * 1 * 48   # records for one work-group per CU


def _profiles():
    # fragile: 3x slowdown under full HBM pressure; hog: exerts full HBM pressure
    return {
        "gemv": {"sens": {"hbm": [1.0, 1.5, 2.0, 2.5, 3.0]}, "press": {"hbm": 0.2}, "occ": 0.6},
        "triad": {"sens": {"hbm": [1.0, 1.1, 1.2, 1.3, 1.4]}, "press": {"hbm": 1.0}, "occ": 0.6},
        "gemm": {"sens": {"lds": [1.0, 1.0, 1.0, 1.0, 1.0]}, "press": {"mfma_bf16": 0.9}, "occ": 0.3},
    }


def _oracle_job(p):
    # the library stores curves and pressures as FP32: round the same way
    f32 = lambda v: float(np.float32(v))
    sens = [[f32(v) for v in p["sens"].get(r, [1.0] * 5)] for r in coloc.RESOURCES]
    press = [f32(p["press"].get(r, 0.0)) for r in coloc.RESOURCES]
    return {"sens": sens, "press": press, "bytes": 1, "occ": f32(p["occ"])}


@pytest.mark.parametrize("policy", ["naive", "usher", "sensitivity"])
@pytest.mark.parametrize("bound", [1.2, 1.5, 2.5, math.inf])
def test_admission_matches_oracle(policy, bound):
    profs = _profiles()
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
