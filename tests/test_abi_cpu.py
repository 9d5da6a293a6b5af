"""Host-side checks of the C ABI that need no GPU.

* libkqr.so loads and exports every function declared in include/kqr.h;
* the ctypes mirrors of kqr_options / kqr_info have the C layout (checked
  against a tiny C program compiled with gcc from the same header);
* argument validation returns KQR_EINVAL before any device work, and valid
  calls without a device return KQR_ENODEVICE.
"""
import ctypes as C
import os
import re
import subprocess
import tempfile

import numpy as np
import pytest

from paper_2510_07929_amd import kqr

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "kqr.h")

pytestmark = pytest.mark.skipif(not os.path.exists(kqr.lib_path()), reason="libkqr.so not built")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(kqr_\w+)\s*\(", text, flags=re.M)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("kqr_fit", "kqr_kernel_apply", "kqr_predict", "kqr_kernel_build",
                     "kqr_rpcholesky", "kqr_woodbury_apply", "kqr_pcg_solve", "kqr_ssn_gradient"):
        assert required in names


def test_library_exports_every_declared_symbol():
    lib = C.CDLL(kqr.lib_path())
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing
    # the binding covers every symbol too
    assert set(declared_functions()) <= set(kqr._SIGS)


def test_struct_layouts_match_c():
    src = r'''
#include <stdio.h>
#include <stddef.h>
#include "kqr.h"
int main(void) {
  printf("%zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu\n", sizeof(kqr_options), sizeof(kqr_info),
         offsetof(kqr_options, pivot_uniforms), offsetof(kqr_options, verbose),
         offsetof(kqr_info, kapply_calls), offsetof(kqr_info, t_total),
         offsetof(kqr_options, z_out), offsetof(kqr_options, v_out),
         offsetof(kqr_options, warm_alpha), offsetof(kqr_options, warm_sigma),
         offsetof(kqr_info, core_retries));
  return 0;
}
'''
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "l.c")
        exe = os.path.join(d, "l")
        open(c, "w").write(src)
        subprocess.run(["gcc", "-I", os.path.dirname(HEADER), c, "-o", exe], check=True)
        out = subprocess.run([exe], capture_output=True, text=True, check=True).stdout.split()
    got = [int(v) for v in out]
    exp = [C.sizeof(kqr.KqrOptions), C.sizeof(kqr.KqrInfo),
           kqr.KqrOptions.pivot_uniforms.offset, kqr.KqrOptions.verbose.offset,
           kqr.KqrInfo.kapply_calls.offset, kqr.KqrInfo.t_total.offset,
           kqr.KqrOptions.z_out.offset, kqr.KqrOptions.v_out.offset,
           kqr.KqrOptions.warm_alpha.offset, kqr.KqrOptions.warm_sigma.offset,
           kqr.KqrInfo.core_retries.offset]
    assert got == exp


def test_default_options_and_status_strings():
    o = kqr.kqr_default_options()
    assert o.tol == 1e-6 and o.admm_tol == 1e-3 and o.admm_max_iter == 100 and o.alm_max_iter == 1000
    assert 0 < o.admm_step < (1 + 5 ** 0.5) / 2
    lib = kqr.lib()
    assert lib.kqr_default_options(None) == kqr.KQR_EINVAL
    for s in (0, 1, -1, -2, -3, -4, -5):
        assert len(kqr.status_string(s)) > 0


def _fake(addr=4096):
    return C.c_void_p(addr)


def test_invalid_arguments_are_rejected_before_device_work():
    lib = kqr.lib()
    P = _fake()
    alpha = _fake()
    beta = C.c_double()
    # n < 2
    assert lib.kqr_fit(P, P, 1, 3, 0.5, 1.0, 0, 1.0, None, alpha, C.byref(beta), None, None) == kqr.KQR_EINVAL
    # tau outside (0, 1)
    assert lib.kqr_fit(P, P, 10, 3, 1.0, 1.0, 0, 1.0, None, alpha, C.byref(beta), None, None) == kqr.KQR_EINVAL
    # lambda <= 0, gamma <= 0, unknown kernel, null pointers
    assert lib.kqr_fit(P, P, 10, 3, 0.5, 0.0, 0, 1.0, None, alpha, C.byref(beta), None, None) == kqr.KQR_EINVAL
    assert lib.kqr_fit(P, P, 10, 3, 0.5, 1.0, 0, -1.0, None, alpha, C.byref(beta), None, None) == kqr.KQR_EINVAL
    assert lib.kqr_fit(P, P, 10, 3, 0.5, 1.0, 7, 1.0, None, alpha, C.byref(beta), None, None) == kqr.KQR_EINVAL
    assert lib.kqr_fit(None, P, 10, 3, 0.5, 1.0, 0, 1.0, None, alpha, C.byref(beta), None, None) == kqr.KQR_EINVAL
    # p above 64
    assert lib.kqr_fit(P, P, 10, 65, 0.5, 1.0, 0, 1.0, None, alpha, C.byref(beta), None, None) == kqr.KQR_EINVAL
    # bad options
    o = kqr.kqr_default_options(admm_step=1.7)
    assert lib.kqr_fit(P, P, 10, 3, 0.5, 1.0, 0, 1.0, C.byref(o), alpha, C.byref(beta), None, None) == kqr.KQR_EINVAL
    assert "admm_step" in kqr.last_error()
    # a warm start needs all three vectors, a finite beta and sigma >= 0
    o = kqr.kqr_default_options()
    o.warm_alpha = 4096
    assert lib.kqr_fit(P, P, 10, 3, 0.5, 1.0, 0, 1.0, C.byref(o), alpha, C.byref(beta), None, None) == kqr.KQR_EINVAL
    assert "warm" in kqr.last_error()
    o.warm_v = o.warm_z = 4096
    o.warm_sigma = -1.0
    assert lib.kqr_fit(P, P, 10, 3, 0.5, 1.0, 0, 1.0, C.byref(o), alpha, C.byref(beta), None, None) == kqr.KQR_EINVAL
    o.warm_sigma, o.warm_beta = 1.0, float("nan")
    assert lib.kqr_fit(P, P, 10, 3, 0.5, 1.0, 0, 1.0, C.byref(o), alpha, C.byref(beta), None, None) == kqr.KQR_EINVAL
    # the breakdown test hook: negative counts rejected, (0, 0) accepted without a device
    assert lib.kqr_test_core_breakdowns(-1, 0) == kqr.KQR_EINVAL
    assert lib.kqr_test_core_breakdowns(0, 0) == kqr.KQR_OK
    # the batched-step test hook: 0 or 1
    assert lib.kqr_test_batch_steps(2) == kqr.KQR_EINVAL
    assert lib.kqr_test_batch_steps(1) == kqr.KQR_OK
    # batch threads: 0 (default) .. 16
    assert lib.kqr_set_batch_threads(17) == kqr.KQR_EINVAL
    assert lib.kqr_set_batch_threads(-1) == kqr.KQR_EINVAL
    assert lib.kqr_set_batch_threads(0) == kqr.KQR_OK
    # kernel apply: m out of range, bad ld, misaligned K
    assert lib.kqr_kernel_apply(P, 10, 3, 0, 1.0, None, 0, 0, P, 17, 17, P, 17, 0, None) == kqr.KQR_EINVAL
    assert lib.kqr_kernel_apply(P, 10, 3, 0, 1.0, P, 0, 12, P, 1, 1, P, 1, 0, None) == kqr.KQR_EINVAL
    assert lib.kqr_kernel_apply(P, 10, 3, 0, 1.0, _fake(4100), 0, 16, P, 1, 1, P, 1, 0, None) == kqr.KQR_EINVAL
    # build: ldk < n
    assert lib.kqr_kernel_build(P, 100, 3, 0, 1.0, 0, P, 64, None) == kqr.KQR_EINVAL
    # rpcholesky: uniforms outside [0, 1)
    u = np.array([0.5, 1.0])
    piv = np.zeros(2, dtype=np.int64)
    r = C.c_int64()
    assert lib.kqr_rpcholesky(P, 10, 3, 0, 1.0, None, 0, 0, 2, u.ctypes.data_as(C.c_void_p), P, 4,
                              piv.ctypes.data_as(C.c_void_p), C.byref(r), None) == kqr.KQR_EINVAL
    # woodbury: rank too large
    assert lib.kqr_woodbury_apply(P, 10, 1024, 1024, 1.0, P, P, P, None) == kqr.KQR_EINVAL
    # kkt residuals: null output, tau outside (0, 1), update without sigma
    out = (C.c_double * 7)()
    assert lib.kqr_kkt_residuals(10, 0.5, 1.0, 0.0, 1.0, 1.0, 0, P, P, P, P, P, None, None) == kqr.KQR_EINVAL
    assert lib.kqr_kkt_residuals(10, 1.5, 1.0, 0.0, 1.0, 1.0, 0, P, P, P, P, P, out, None) == kqr.KQR_EINVAL
    assert lib.kqr_kkt_residuals(10, 0.5, 1.0, 0.0, 0.0, 1.0, 1, P, P, P, P, P, out, None) == kqr.KQR_EINVAL
    # on-the-fly launch shape: strip and workgroup target ranges (host-only; valid calls succeed)
    assert lib.kqr_set_otf_shape(33, 0) == kqr.KQR_EINVAL
    assert lib.kqr_set_otf_shape(4, 100) == kqr.KQR_EINVAL
    assert lib.kqr_set_otf_shape(8, 4096) == kqr.KQR_OK
    assert lib.kqr_set_otf_shape(0, 0) == kqr.KQR_OK
    # allocation-free apply: K required, strides >= 1, n beyond the fixed scratch array
    assert lib.kqr_kernel_apply_static(None, 0, 10, 16, P, 1, P, 1, 0, None) == kqr.KQR_EINVAL
    assert lib.kqr_kernel_apply_static(P, 0, 10, 16, P, 0, P, 1, 0, None) == kqr.KQR_EINVAL
    assert lib.kqr_kernel_apply_static(P, 0, 4_000_000, 4_000_000, P, 1, P, 1, 0, None) == kqr.KQR_EINVAL
    assert "static" in kqr.last_error()
    # tuning file and on-the-fly autotuner: null arguments, bad kernel
    cnt = C.c_int()
    assert lib.kqr_tune_save(None, C.byref(cnt)) == kqr.KQR_EINVAL
    assert lib.kqr_tune_load(b"/nonexistent.json", None) == kqr.KQR_EINVAL
    assert lib.kqr_autotune_otf(P, 100, 3, kqr.KQR_LINEAR, 1.0, 0, 1, None, 0, None) == kqr.KQR_EINVAL


@pytest.mark.skipif(kqr.kqr_device_count() > 0, reason="a device is present")
def test_valid_calls_without_device_report_no_device():
    lib = kqr.lib()
    P = _fake()
    beta = C.c_double()
    assert lib.kqr_fit(P, P, 10, 3, 0.5, 1.0, 0, 1.0, None, P, C.byref(beta), None, None) == kqr.KQR_ENODEVICE
    assert lib.kqr_predict(P, 10, 3, P, 0.0, 1.0, 0, 1.0, P, 5, P, None) == kqr.KQR_ENODEVICE


def test_packed_layout_size():
    # upper triangle of ceil(n/128)^2 tiles of 128 x 128 entries (host-only call)
    lib = kqr.lib()
    for n, kd, esz in ((1, 0, 4), (128, 0, 4), (129, 0, 4), (1000, 1, 2), (50000, 0, 4)):
        nt = -(-n // 128)
        assert lib.kqr_packed_bytes(n, kd) == nt * (nt + 1) // 2 * 128 * 128 * esz
    assert lib.kqr_packed_bytes(0, 0) == -1 and lib.kqr_packed_bytes(10, 5) == -1
    # about half of the full layout at scale
    assert lib.kqr_packed_bytes(50000, 0) / (50000 * 50048 * 4) < 0.51


def test_traffic_summaries_are_tied_to_kernel_sources():
    # bench.py reports a measured HBM traffic figure only while the digest in
    # its rocprofv3 summary matches the K-apply source it was measured on
    from paper_2510_07929_amd import traffic
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    for layout, name in (("rows", "kapply_rows_c1_fp32_traffic.md"), ("packed", "kapply_packed_c1_fp32_traffic.md")):
        dig = traffic.source_digest(traffic.source_for(layout))
        assert len(dig) == 16 and int(dig, 16) >= 0
        got = traffic.read_summary(os.path.join(root, "profiles", name))
        assert got is not None
        val, recorded = got
        assert recorded == dig, f"{name} was measured on another version of the {layout} K-apply"
        assert 1e9 < val < 2e10
