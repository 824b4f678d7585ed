"""The C-ABI library loads, exports every symbol include/qs.h declares, and validates without a GPU."""
import ctypes
import os
import re

import pytest

import paper_2203_16044_amd as qs
from paper_2203_16044_amd import binding as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = set()
    for fn in sorted(os.listdir(os.path.join(ROOT, "include"))):
        if fn.endswith(".h"):
            txt = open(os.path.join(ROOT, "include", fn)).read()
            names |= set(re.findall(r"QS_API\s+[\w\s\*]+?\b(qs_\w+)\s*\(", txt))
    return names


def test_header_declares_the_boundary():
    names = _declared()
    for core in ("qs_alloc", "qs_free", "qs_apply_gate", "qs_apply_diag", "qs_apply_controlled", "qs_fused_swap",
                 "qs_probs"):
        assert core in names


def test_every_declared_symbol_is_exported():
    L = ctypes.CDLL(B.LIB_PATH)
    missing = [n for n in sorted(_declared()) if not hasattr(L, n)]
    assert not missing, missing


def test_binding_covers_every_declared_symbol():
    assert _declared() <= set(B.SIGNATURES)


def test_null_handles_are_rejected_without_device_work():
    L = B.lib()
    one = (ctypes.c_int * 1)(0)
    U = (ctypes.c_double * 8)(*([0.0] * 8))
    assert L.qs_apply_gate(None, one, 1, U) == B.QS_EINVAL
    assert L.qs_apply_diag(None, one, 1, U) == B.QS_EINVAL
    assert L.qs_apply_controlled(None, one, 1, one, 1, U) == B.QS_EINVAL
    assert L.qs_fused_swap(None, 0, 1, 1) == B.QS_EINVAL
    assert L.qs_probs(None, None, None) == B.QS_EINVAL
    assert L.qs_plan_run_renorm(None, None, B.QS_RUN_NORM_LAST) == B.QS_EINVAL
    assert L.qs_plan_run_range_renorm(None, None, 0, 0, B.QS_RUN_NORM_LAST) == B.QS_EINVAL
    assert L.qs_renormalize_pending(None, None) == B.QS_EINVAL
    assert L.qs_free(None) == B.QS_EINVAL
    assert "NULL" in qs.qs_last_error()


@pytest.mark.parametrize("n,dtype", [(0, 0), (41, 0), (4, 2), (4, -1)])
def test_alloc_validates_arguments_first(n, dtype):
    h = ctypes.c_void_p()
    assert B.lib().qs_alloc(ctypes.byref(h), n, dtype, None, None) == B.QS_EINVAL
    assert h.value is None


def test_alloc_rejects_misaligned_buffer():
    h = ctypes.c_void_p()
    assert B.lib().qs_alloc(ctypes.byref(h), 4, 0, ctypes.c_void_p(0x1008), None) == B.QS_EINVAL


def test_tunables_validate():
    with pytest.raises(qs.QSError):
        B.qs_set_tunable("no_such_knob", 1)
    with pytest.raises(qs.QSError):
        B.qs_set_tunable("dense_gpt", 3)
    B.qs_set_tunable("dense_gpt", 1)
    for name, bad, good in (("block_wg_per_cu", 0, 32), ("block_wg_per_cu", 4097, 32), ("block_stage_width", 5, 4),
                            ("plan_beam", 65, 16), ("plan_beam", -1, 16), ("mfma_stage_ops", 9, 3),
                            ("mfma_stage_ops", -1, 3), ("block_async", 2, 0), ("block_lanes", 2, 0),
                            ("stage_pack", 2, 1), ("stage_pack", -1, 1), ("plan_beam_search", 2, 0)):
        with pytest.raises(qs.QSError):
            B.qs_set_tunable(name, bad)
        B.qs_set_tunable(name, good)  # the defaults


def test_tunables_read_back():
    """qs_get_tunable returns what qs_set_tunable stored (and the defaults), and rejects unknown names."""
    assert B.qs_get_tunable("plan_beam") == 16 and B.qs_get_tunable("stage_pack") == 1
    assert B.qs_get_tunable("plan_beam_search") == 0 and B.qs_get_tunable("block_wg_per_cu") == 32
    B.qs_set_tunable("plan_beam", 24)
    try:
        assert B.qs_get_tunable("plan_beam") == 24
    finally:
        B.qs_set_tunable("plan_beam", 16)
    with pytest.raises(qs.QSError):
        B.qs_get_tunable("no_such_knob")


def test_binding_rejects_matrix_shape_mismatch():
    import numpy as np
    with pytest.raises(ValueError):
        B.qs_apply_gate(1, (0, 1), np.eye(2))
    with pytest.raises(ValueError):
        B.qs_apply_diag(1, (0,), np.ones(4))
    with pytest.raises(ValueError):
        B.qs_apply_controlled(1, (0,), (1, 2), np.eye(2))


C_CONSUMER = r"""
#include <stdio.h>
#include <string.h>
#include "qs.h"
int main(void)
{
    qs_state *st = (qs_state *)0;
    if (qs_set_tunable("no_such_tunable", 1) != QS_EINVAL || strstr(qs_last_error(), "no_such_tunable") == NULL)
        return 1;
    if (qs_set_tunable("plan_beam", 16) != QS_OK || qs_last_error()[0] != '\0')
        return 2;
    if (qs_alloc(&st, 0, QS_C128, NULL, NULL) != QS_EINVAL || st != NULL)
        return 3;
    if (qs_free(NULL) != QS_EINVAL)
        return 4;
    puts("c consumer ok");
    return 0;
}
"""


@pytest.mark.parametrize("compiler,std", [("gcc", "-std=c99"), ("g++", "-std=c++17")])
def test_header_is_plain_c_and_links_from_c(tmp_path, compiler, std):
    """A C (or C++) program includes qs.h under strict warnings, links libqs.so and gets status codes and thread-
    local messages from host-only calls: the boundary needs no torch and no C++ on the caller's side."""
    import shutil
    import subprocess
    if shutil.which(compiler) is None:
        pytest.skip(f"{compiler} not installed")
    src = tmp_path / ("consumer.c" if compiler == "gcc" else "consumer.cpp")
    src.write_text(C_CONSUMER)
    exe = tmp_path / "consumer"
    libdir = os.path.dirname(B.LIB_PATH)
    cmd = [compiler, std, "-Wall", "-Wextra", "-Werror", "-pedantic", "-I", os.path.join(ROOT, "include"), str(src),
           "-o", str(exe), B.LIB_PATH, f"-Wl,-rpath,{libdir}"]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=60)
    assert r.returncode == 0 and "c consumer ok" in r.stdout, (r.returncode, r.stdout, r.stderr)


def test_product_path_never_loads_the_oracle():
    """Importing the package and planning a circuit through the library loads nothing from oracle/ (the oracle is
    test infrastructure; the product path has no CPU fallback)."""
    import subprocess
    import sys
    code = ("import sys; import paper_2203_16044_amd as qs; from paper_2203_16044_amd import plan, batch, costmodel; "
            "import circuits as C; c = plan.Circuit.from_ops(12, C.u3_cnot_layers(n=12).ops); "
            "p = plan.Plan(c, 'block', 10, 3); p.pass_gates(); p.close(); c.close(); "
            "bad = [m for m in sys.modules if m == 'oracle' or m.startswith('oracle.')]; "
            "print('loaded:', bad); sys.exit(1 if bad else 0)")
    r = subprocess.run([sys.executable, "-c", code], cwd=ROOT, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
