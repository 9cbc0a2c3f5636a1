"""Host-side checks of the C ABI: the library loads, exports every symbol
that include/lc.h declares, reports statuses, applies its grid-size rule and
rejects invalid arguments before touching the GPU."""
import ctypes as C
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_symbols():
    txt = open(os.path.join(ROOT, "include", "lc.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(lc_[a-z_0-9]+)\s*\(", txt)))


@pytest.fixture(scope="module")
def lib():
    import paper_1106_0463_amd as lc
    return lc.load()


def test_every_declared_symbol_is_exported(lib):
    names = _declared_symbols()
    assert len(names) >= 18
    for n in names:
        assert hasattr(lib, n), n


def test_binding_covers_every_symbol():
    from paper_1106_0463_amd._lib import SIGNATURES
    assert sorted(n for n, _, _ in SIGNATURES) == _declared_symbols()


def test_status_strings(lib):
    for s in range(6):
        assert lib.lc_status_string(s).decode().startswith("LC_")


def _smooth_at_least(L):
    n = max(L, 1)
    while True:
        m = n
        for p in (2, 3):
            while m % p == 0:
                m //= p
        if m in (1, 5):
            return n
        n += 1


@pytest.mark.parametrize("M", [2, 4, 6, 256, 300, 1200, 4 * 257, 4 * 8191, 262144, 4 * 3001, 10**6, 4 * 15625, 4 * 3126])
def test_grid_size_rule(M):
    import paper_1106_0463_amd as lc
    Me = lc.grid_size(M)
    L = Me // 4
    assert Me >= M and Me % 4 == 0
    assert L == _smooth_at_least(max(1, -(-max(M, 4) // 4)))
    n = L
    for p in (2, 3):
        while n % p == 0:
            n //= p
    assert n in (1, 5)


@pytest.mark.parametrize("args", [(0, 256, 32), (200, 256, 32), (8, 255, 32), (8, 256, 0),
                                  (8, 256, 70000), (8, 0, 4)])
def test_plan_rejects_invalid(args):
    import paper_1106_0463_amd as lc
    with pytest.raises(lc.LCError) as ei:
        lc.plan(*args)
    assert ei.value.status == 1


def test_null_arguments_rejected(lib):
    assert lib.lc_plan(8, 256, 32, 0, None) == 1
    assert lib.lc_execute(None, None, None, None) == 1
    assert lib.lc_execute_noalloc(None, None, None, None) == 1
    assert lib.lc_plan_info(None, None) == 1
    assert lib.lc_plan_destroy(None) == 0
    assert "null" in lib.lc_last_error().decode() or lib.lc_last_error().decode() != ""
    assert lib.lc_grid_size(1, C.byref(C.c_int64())) == 1


def test_autotune_rejects_null(lib):
    assert lib.lc_autotune(None, None) == 1


@pytest.mark.parametrize("rule", [dict(q=0), dict(q=7, breaks=(0.0,)), dict(q=8, band=100.0, q_max=4),
                                  dict(q=8, breaks=(1.5,)), dict(q=8, grade_ratio=1.0, grade_levels=2),
                                  dict(q=8, band=-1.0), dict(q=8, breaks=tuple(np.linspace(-0.9, 0.9, 65)))])
def test_adaptive_rule_rejected(rule):
    # the rule is validated before any device work
    import paper_1106_0463_amd as lc
    with pytest.raises(lc.LCError) as ei:
        lc.plan_adaptive(16, 64, **rule)
    assert ei.value.status == 1


def test_adaptive_null_rule(lib):
    h = C.c_void_p()
    assert lib.lc_plan_adaptive(16, 64, None, 0, C.byref(h)) == 1


@pytest.mark.parametrize("args", [(0, 64, 8), (40, 64, 8), (8, 63, 8), (8, 64, 0)])
def test_plan_2d_rejects_invalid(args):
    import paper_1106_0463_amd as lc
    with pytest.raises(lc.LCError) as ei:
        lc.plan_2d(*args)
    assert ei.value.status == 1


def test_execute_2d_rejects_null(lib):
    assert lib.lc_execute_2d(None, None, None, None) == 1


@pytest.mark.parametrize("env", [("LC_MGEMM_STAGES", "64,7"), ("LC_MGEMM_STAGES", "16"), ("LC_MGEMM_KCH", "3"),
                                 ("LC_MGEMM_BLOCK_ROWS", "192")])
def test_gemm_overrides_without_kernel_rejected(monkeypatch, env):
    # a product shape the library holds no kernel for fails at plan time,
    # before any device work
    import paper_1106_0463_amd as lc
    monkeypatch.setenv(*env)
    with pytest.raises(lc.LCError) as ei:
        lc.plan_gemm(512, 1024, 512, "bf16x3")
    assert ei.value.status == 1
