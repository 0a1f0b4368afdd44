"""CPU tests of the C ABI boundary: the library loads, exports every function
that include/act.h declares, and rejects bad arguments on the host with
ACT_ERR_INVALID before any device work."""
import ctypes
import os
import subprocess
import math
import re

import pytest

from paper_2607_16629_amd import act as A
from paper_2607_16629_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "act.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(act_[a-z0-9_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(A.LIB_PATH):
        pytest.fail("libact.so is not built (run __graft_entry__.build())")
    return A.load()


def test_header_declares_the_named_calls():
    names = declared_functions()
    for required in ("act_plan", "act_decompose", "act_refine", "act_reconstruct",
                     "act_value_and_grad", "act_correlate"):
        assert required in names


def test_library_exports_every_declared_symbol(lib):
    for name in declared_functions():
        assert hasattr(lib, name), name
    assert set(A.EXPORTS) <= set(declared_functions())


def test_struct_layout_matches_header(tmp_path):
    """Sizes and field offsets of the binding's structs equal the C header's,
    as compiled by gcc from include/act.h."""
    fields = {"act_axis": A._Axis, "act_grid": A._Grid, "act_plan_desc": A._PlanDesc,
              "act_launch_shape": A._LaunchShape, "act_lem_desc": A._LemDesc}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "act.h"', "int main(void) {"]
    for cname, py in fields.items():
        lines.append(f'printf("{cname} %zu\\n", sizeof({cname}));')
        for f, _ in py._fields_:
            lines.append(f'printf("{cname}.{f} %zu\\n", offsetof({cname}, {f}));')
    lines += ["return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    inc = os.path.join(os.path.dirname(__file__), "..", "include")
    subprocess.run(["gcc", "-std=c11", "-I", inc, str(src), "-o", str(exe)], check=True)
    got = dict(l.split() for l in subprocess.run([str(exe)], check=True, capture_output=True,
                                                 text=True).stdout.splitlines())
    for cname, py in fields.items():
        assert int(got[cname]) == ctypes.sizeof(py), cname
        for f, _ in py._fields_:
            assert int(got[f"{cname}.{f}"]) == getattr(py, f).offset, (cname, f)


def _plan_status(lib, desc):
    h = ctypes.c_void_p()
    st = lib.act_plan(ctypes.byref(desc), None, ctypes.byref(h))
    return st, lib.act_last_error().decode()


@pytest.mark.parametrize("mutate,needle", [
    (lambda d: setattr(d.grid, "fs_hz", 0.0), "fs_hz"),
    (lambda d: setattr(d.grid, "n_samples", 0), "n_samples"),
    (lambda d: setattr(d.grid.fc_hz, "count", 0), "fc_hz"),
    (lambda d: setattr(d.grid.c_hz_per_s, "hi", float("nan")), "c_hz_per_s"),
    (lambda d: setattr(d.grid.logdt_ln_s, "hi", -10.0), "logdt_ln_s"),
    (lambda d: setattr(d, "dict", 7), "dict"),
    (lambda d: setattr(d, "prec", 9), "prec"),
    (lambda d: setattr(d, "max_batch", 0), "max_batch"),
    (lambda d: (setattr(d, "prec", A.ACT_PREC_F64), setattr(d, "dict", A.ACT_DICT_TABLE)), "F64"),
])
def test_plan_rejects_bad_descriptors_on_host(lib, mutate, needle):
    desc = A.make_desc(W.eeg_grid(512, 32, 16, 16, 8))
    mutate(desc)
    st, msg = _plan_status(lib, desc)
    assert st == A.ACT_ERR_INVALID
    assert needle in msg


def test_null_arguments_rejected(lib):
    h = ctypes.c_void_p()
    assert lib.act_plan(None, None, ctypes.byref(h)) == A.ACT_ERR_INVALID
    assert lib.act_decompose(None, 1, None, None, None, None, 1, None, None, None, None, None,
                             None, None) == A.ACT_ERR_INVALID
    assert lib.act_refine(None, 1, None, None, 1, None, None, None, None) == A.ACT_ERR_INVALID
    assert lib.act_reconstruct(None, 1, 1, None, None, None, None, None, None) == A.ACT_ERR_INVALID
    assert lib.act_value_and_grad(None, 1, 0, None, None, None, None, None, None) == A.ACT_ERR_INVALID
    assert lib.act_correlate(None, 1, None, 0, 1, None, None) == A.ACT_ERR_INVALID
    assert lib.act_tune(None, 1, None, None, None, 3, None, None, None) == A.ACT_ERR_INVALID
    assert lib.act_plan_query(None, 0) == -1
    flops = ctypes.c_double(0.0)
    assert lib.act_search_flops(None, 1, ctypes.byref(flops)) == A.ACT_ERR_INVALID
    n = ctypes.c_int64(0)
    assert lib.act_search_executed(None, ctypes.byref(flops), ctypes.byref(n)) == A.ACT_ERR_INVALID
    assert lib.act_refine_f32(None, 1, None, None, 1, None, None, None, None) == A.ACT_ERR_INVALID
    assert lib.act_lem_decompose_noalloc(None, None, 1, None, None, None, 1, None, None, None, None,
                                         None) == A.ACT_ERR_INVALID
    # the probes check sizes, alignment and counts before touching a device
    assert lib.act_probe_read(None, 16, 8, None, None) == A.ACT_ERR_INVALID
    assert lib.act_probe_read(ctypes.c_void_p(4096), 15, 8, ctypes.c_void_p(4096), None) == A.ACT_ERR_INVALID
    assert lib.act_probe_read(ctypes.c_void_p(4096), 16, 0, ctypes.c_void_p(4096), None) == A.ACT_ERR_INVALID
    assert lib.act_probe_mfma(A.ACT_PREC_F64, 10, 2, ctypes.c_void_p(4096), ctypes.byref(flops),
                              None) == A.ACT_ERR_INVALID
    assert lib.act_probe_mfma(A.ACT_PREC_BF16, 0, 2, ctypes.c_void_p(4096), ctypes.byref(flops),
                              None) == A.ACT_ERR_INVALID
    lib.act_plan_destroy(None)


def test_status_strings(lib):
    for s, name in enumerate(["ACT_OK", "ACT_ERR_INVALID", "ACT_ERR_NOMEM", "ACT_ERR_HIP",
                              "ACT_ERR_UNSUPPORTED"]):
        assert lib.act_status_string(s).decode() == name


def test_binding_refuses_without_gpu():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    with pytest.raises(RuntimeError):
        A.Plan(W.eeg_grid(512, 4, 4, 4, 2))


def test_noalloc_scratch_size_matches_header():
    """The binding's copy of ACT_LEM_SCRATCH_BYTES equals the header's."""
    m = re.search(r"#define\s+ACT_LEM_SCRATCH_BYTES\s+\((\d+)u\s*<<\s*(\d+)\)", open(HEADER).read())
    assert m is not None
    assert int(m.group(1)) << int(m.group(2)) == A.LEM_SCRATCH_BYTES
