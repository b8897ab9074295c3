"""CPU checks of the C ABI: the library loads, exports every function the
header declares, its structs match the Python binding byte for byte, and
argument validation rejects bad calls before touching a GPU."""
import ctypes
import os
import re
import subprocess
import tempfile

import pytest

import paper_2408_05444_amd as mek

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mek.h")


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\**\s+\**(mek_\w+)\s*\(", text, flags=re.M)))


def test_header_declares_the_boundary():
    names = _declared_functions()
    for want in ["mek_version", "mek_status_string", "mek_plan_create", "mek_plan_destroy",
                 "mek_plan_query", "mek_solve", "mek_solve_batched", "mek_philox_uniform", "mek_select",
                 "mek_residual", "mek_residual_batched", "mek_gram", "mek_solve_multi", "mek_solve_async",
                 "mek_cnn_conv3x3", "mek_cnn_conv3x3_grad_input", "mek_cnn_conv3x3_grad_weight",
                 "mek_cnn_mse_grad", "mek_cnn_adam", "mek_cnn_to_bf16", "mek_cnn_round_bf16",
                 "mek_plan_sparse_widths", "mek_solve_multi_async"]:
        assert want in names


def test_library_exports_every_declared_symbol():
    L = mek.lib()
    for name in _declared_functions():
        assert hasattr(L, name), name
    out = subprocess.run(["nm", "-D", "--defined-only", mek.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = set(re.findall(r"\sT\s(mek_\w+)", out))
    assert set(_declared_functions()) <= exported


def test_version_and_status_strings():
    hdr = open(HEADER).read()
    ver = int(re.search(r"#define MEK_ABI_VERSION (\d+)", hdr).group(1))
    assert mek.mek_version() == ver
    for code in [0, 1, 2, -1, -2, -3, -4, -5, -6, -7]:
        assert mek.mek_status_string(code) != "unknown status"
    assert mek.mek_status_string(99) == "unknown status"


def test_constants_match_header():
    hdr = open(HEADER).read()
    consts = dict((k, int(v.strip("()"))) for k, v in
                  re.findall(r"#define (MEK_[A-Z0-9_]+) \(?(-?\d+)\)?", hdr))
    for k, v in consts.items():
        if hasattr(mek, k):
            assert getattr(mek, k) == v, k


def test_struct_layouts_match_c():
    src = r"""
    #include <stdio.h>
    #include <stddef.h>
    #include "mek.h"
    #define F(T, f) printf(#T "." #f " %zu\n", offsetof(T, f));
    int main(void) {
      printf("mek_plan_opts %zu\nmek_solve_opts %zu\nmek_report %zu\n",
             sizeof(mek_plan_opts), sizeof(mek_solve_opts), sizeof(mek_report));
      F(mek_solve_opts, X_ref) F(mek_solve_opts, max_iters) F(mek_solve_opts, replay_len)
      F(mek_solve_opts, hist_cap) F(mek_solve_opts, inner_iters) F(mek_solve_opts, set_hist)
      F(mek_report, passes) F(mek_report, alpha) F(mek_plan_opts, r_in_lds)
      F(mek_plan_opts, update)
      F(mek_solve_opts, block_rows) F(mek_solve_opts, tau) F(mek_solve_opts, cols_hist)
      return 0;
    }
    """
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "probe.c")
        exe = os.path.join(d, "probe")
        open(c, "w").write(src)
        subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), c, "-o", exe])
        out = subprocess.run([exe], capture_output=True, text=True, check=True).stdout
    vals = dict(line.rsplit(" ", 1) for line in out.strip().splitlines())
    assert int(vals["mek_plan_opts"]) == ctypes.sizeof(mek.mek_plan_opts)
    assert int(vals["mek_solve_opts"]) == ctypes.sizeof(mek.mek_solve_opts)
    assert int(vals["mek_report"]) == ctypes.sizeof(mek.mek_report)
    for key, v in vals.items():
        if "." in key:
            T, f = key.split(".")
            assert getattr(getattr(mek, T), f).offset == int(v), key


def test_host_validation_rejects_before_any_gpu_work():
    L = mek.lib()
    h = ctypes.c_void_p()
    vp = ctypes.c_void_p
    EINVAL = mek.MEK_EINVAL
    assert L.mek_plan_create(None, 1, 1, 1, 1, vp(1), vp(1), None, None) == EINVAL
    assert L.mek_plan_create(ctypes.byref(h), 0, 1, 1, 1, vp(1), vp(1), None, None) == EINVAL
    assert L.mek_plan_create(ctypes.byref(h), 2, 2, 2, -3, vp(1), vp(1), None, None) == EINVAL
    assert L.mek_plan_create(ctypes.byref(h), 2, 2, 2, 2, None, vp(1), None, None) == EINVAL
    bad = mek.mek_plan_opts(7, 0.0, 0, -1)
    assert L.mek_plan_create(ctypes.byref(h), 2, 2, 2, 2, vp(1), vp(1), ctypes.byref(bad), None) == EINVAL
    bad = mek.mek_plan_opts(0, float("nan"), 0, -1)
    assert L.mek_plan_create(ctypes.byref(h), 2, 2, 2, 2, vp(1), vp(1), ctypes.byref(bad), None) == EINVAL
    bad = mek.mek_plan_opts(0, 0.0, 0, -1, 5)
    assert L.mek_plan_create(ctypes.byref(h), 2, 2, 2, 2, vp(1), vp(1), ctypes.byref(bad), None) == EINVAL
    mixed_sparse = mek.mek_plan_opts(mek.MEK_MIXED, 0.0, 0, -1, mek.MEK_UPDATE_SPARSE)
    assert L.mek_plan_create(ctypes.byref(h), 2, 2, 2, 2, vp(1), vp(1), ctypes.byref(mixed_sparse),
                             None) == mek.MEK_EUNSUPPORTED
    w4 = (ctypes.c_int32 * 4)()
    assert L.mek_plan_sparse_widths(None, w4) == EINVAL
    assert L.mek_solve(None, vp(1), None, None, vp(1), None, None) == EINVAL
    assert L.mek_select(9, 10, vp(1), vp(1), 1.0, 0.5, 0, 0, 0, 1, vp(1), None, None, None, None) == EINVAL
    assert L.mek_select(2, 10, vp(1), vp(1), 1.0, 1.5, 0, 0, 0, 1, vp(1), None, None, None, None) == EINVAL
    assert L.mek_select(2, 10, vp(1), vp(1), 0.0, 0.5, 0, 0, 0, 1, vp(1), None, None, None, None) == EINVAL
    assert L.mek_select(2, 0, vp(1), vp(1), 1.0, 0.5, 0, 0, 0, 1, vp(1), None, None, None, None) == EINVAL
    assert L.mek_philox_uniform(0, 0, 0, -1, vp(1), None) == EINVAL
    assert L.mek_philox_uniform(0, 0, -5, 3, vp(1), None) == EINVAL
    assert L.mek_philox_uniform(0, 0, 0, 0, None, None) == mek.MEK_OK
    assert L.mek_residual(0, 1, 1, 1, vp(1), vp(1), vp(1), vp(1), vp(2), None) == EINVAL
    assert L.mek_residual(1, 1, 1, 1, vp(1), vp(1), vp(1), vp(1), vp(1), None) == EINVAL  # R aliases
    assert L.mek_residual_batched(0, 1, 1, 1, 1, vp(8), vp(8), vp(8), vp(8), vp(64), None) == EINVAL
    assert L.mek_solve_multi(0, None, None, None, None, None, None, None, None) == EINVAL
    assert L.mek_solve_async(None, vp(8), None, None, vp(8), vp(8), None) == EINVAL
    assert L.mek_solve_multi_async(0, None, None, None, None, None, None, vp(8), None) == EINVAL
    assert L.mek_cnn_conv3x3(1, 4, 8, 8, 32, vp(2), vp(4), None, 1, vp(8), None, None, None) == EINVAL
    assert L.mek_cnn_conv3x3(1, 3, 8, 8, 32, vp(2), vp(4), None, 1, vp(8), vp(16), None, None) == EINVAL
    assert L.mek_cnn_conv3x3(1, 3, 8, 8, 32, vp(2), vp(4), None, 1, vp(8), None, vp(8), None) == EINVAL
    assert L.mek_cnn_conv3x3_grad_input(0, 32, 8, 8, 3, vp(2), None, vp(4), vp(8), None) == EINVAL
    assert L.mek_cnn_conv3x3_grad_weight(1, 3, 8, 8, 7, vp(2), vp(2), None, vp(4), vp(4), None) == EINVAL
    assert L.mek_cnn_mse_grad(0, vp(8), vp(8), None, ctypes.byref(ctypes.c_double()), None) == EINVAL
    assert L.mek_cnn_adam(4, vp(4), vp(4), vp(4), vp(4), vp(4), 1e-3, 0.9, 0.999, 1e-8, 0, None) == EINVAL
    assert L.mek_cnn_adam(4, vp(4), vp(4), vp(4), vp(4), vp(4), 1e-3, 1.0, 0.999, 1e-8, 1, None) == EINVAL
    assert L.mek_solve_multi(1, None, None, None, None, None, None, None, None) == EINVAL
    # R_1 (bytes 24..32) overlaps C_0..C_1 (bytes 16..32)
    assert L.mek_residual_batched(2, 1, 1, 1, 1, vp(1024), vp(2048), vp(4096), vp(16), vp(24),
                                  None) == EINVAL
    assert L.mek_gram(3, 3, vp(1), 2, vp(2), None) == EINVAL
    assert L.mek_gram(3, 3, vp(1), 0, vp(1), None) == EINVAL
    assert L.mek_residual_split(0, 1, 1, 1, 1, 1, vp(4), vp(4), vp(4), vp(8), vp(64), None) == EINVAL
    assert L.mek_residual_split(4, 1, 1, 1, 1, 1, vp(4), vp(4), vp(4), vp(8), vp(64), None) == EINVAL
    assert L.mek_residual_split(3, 1, 0, 1, 1, 1, vp(4), vp(4), vp(4), vp(8), vp(64), None) == EINVAL
    assert L.mek_residual_noalloc(4097, 1, 512, 1, vp(8), vp(8), vp(8), vp(8), vp(64), None) == EINVAL
    assert L.mek_residual_noalloc(0, 1, 1, 1, vp(8), vp(8), vp(8), vp(8), vp(64), None) == EINVAL
    us = ctypes.c_double()
    assert L.mek_exchange_floor(0, 10, 10, 10, 10, ctypes.byref(us), None) == EINVAL
    assert L.mek_exchange_floor(8, 4, 10, 10, 10, ctypes.byref(us), None) == EINVAL
    assert L.mek_exchange_floor(4, 10, 10, 10, 0, ctypes.byref(us), None) == EINVAL
    assert L.mek_plan_destroy(None) == mek.MEK_OK
