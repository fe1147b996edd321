"""C-ABI checks that need no GPU: the library loads, exports every declared
entry point, and its host-only logic (validation, radix planning) is right."""

import ctypes
import os
import re

import numpy as np
import pytest

from paper_1210_2687_amd import admm as A
from paper_1210_2687_amd import workloads as WL

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared(header):
    text = open(os.path.join(ROOT, "include", header)).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(admm_[a-z0-9_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    L = A.lib()
    headers = sorted(f for f in os.listdir(os.path.join(ROOT, "include")) if f.endswith(".h"))
    assert headers == ["admm_deconv.h", "admm_warmstart.h"]
    names = sorted(set(n for h in headers for n in _declared(h)))
    assert len(names) >= 18
    for name in names:
        assert hasattr(L, name), name
    assert sorted(A.exported_symbols()) == names


@pytest.mark.parametrize("n", [8, 12, 15, 30, 49, 64, 96, 105, 125, 128, 135, 160, 189, 343, 360, 512, 1000, 1024, 2048])
def test_radix_schedule_multiplies_to_n(n):
    r = A.admm_fft_radices(n)
    assert r is not None and int(np.prod(r)) == n
    assert all(x in (2, 3, 4, 5, 7, 8) for x in r)


@pytest.mark.parametrize("n", [11, 13, 22, 1021, 0, -4])
def test_radix_schedule_rejects_non_smooth(n):
    assert A.admm_fft_radices(n) is None


def _prob(**kw):
    H, W, k = kw.pop("H", 32), kw.pop("W", 40), kw.pop("k", 5)
    kern = kw.pop("kernel", WL.kernel_uniform(k))
    mask = kw.pop("mask", WL.valid_mask(H, W, k // 2))
    return A.make_problem(kern, mask, kw.pop("lam", 1e-3), reg=kw.pop("reg", A.ADMM_REG_TV),
                          levels=kw.pop("levels", 0), method=kw.pop("method", None))


def test_validation_accepts_good_problem():
    assert A.admm_validate_problem(_prob()) == A.ADMM_OK
    assert A.admm_validate_problem(_prob(reg=A.ADMM_REG_FRAME, levels=3)) == A.ADMM_OK
    assert A.admm_validate_problem(_prob(reg=A.ADMM_REG_FRAME_SYNTHESIS, levels=2)) == A.ADMM_OK
    for reg, J in ((A.ADMM_REG_TV, 0), (A.ADMM_REG_FRAME, 2)):
        assert A.admm_validate_problem(_prob(reg=reg, levels=J, method=A.ADMM_METHOD_CG)) == A.ADMM_OK


def test_validation_of_methods_and_the_synthesis_formulation():
    # FS-MD needs frame levels; the synthesis formulation has no CG variant here; unknown methods are invalid
    assert A.admm_validate_problem(_prob(reg=A.ADMM_REG_FRAME_SYNTHESIS, levels=0)) == A.ADMM_E_UNSUPPORTED
    assert A.admm_validate_problem(_prob(reg=A.ADMM_REG_FRAME_SYNTHESIS, levels=1,
                                         method=A.ADMM_METHOD_CG)) == A.ADMM_E_UNSUPPORTED
    assert A.admm_validate_problem(_prob(method=7)) == A.ADMM_E_INVALID
    assert A.admm_validate_problem(_prob(reg=3)) == A.ADMM_E_INVALID


@pytest.mark.parametrize("case,status", [
    ("even_kernel", A.ADMM_E_UNSUPPORTED),
    ("kernel_too_big", A.ADMM_E_UNSUPPORTED),
    ("not_smooth", A.ADMM_E_UNSUPPORTED),
    ("too_large", A.ADMM_E_UNSUPPORTED),
    ("zero_sum_tv", A.ADMM_E_SINGULAR),
    ("negative_lambda", A.ADMM_E_INVALID),
    ("bad_levels", A.ADMM_E_UNSUPPORTED),
    ("nan_kernel", A.ADMM_E_INVALID),
])
def test_validation_errors(case, status):
    if case == "even_kernel":
        p = _prob(kernel=np.full((4, 4), 1 / 16.0), mask=np.ones((32, 40), np.uint8))
    elif case == "kernel_too_big":
        p = _prob(H=16, W=16, kernel=np.full((17, 17), 1 / 289.0), mask=np.ones((16, 16), np.uint8))
    elif case == "not_smooth":
        p = _prob(H=33, W=40)
    elif case == "too_large":
        p = _prob(H=32768, W=16)
    elif case == "zero_sum_tv":
        k = np.zeros((3, 3))
        k[1, 0], k[1, 2] = 1.0, -1.0
        p = _prob(kernel=k)
    elif case == "negative_lambda":
        p = _prob(lam=-1.0)
    elif case == "bad_levels":
        p = _prob(reg=A.ADMM_REG_FRAME, levels=0)
    else:
        k = WL.kernel_uniform(3)
        k[0, 0] = np.nan
        p = _prob(kernel=k)
    assert A.admm_validate_problem(p) == status
    assert len(A.admm_last_error()) > 0


def test_frame_coefficient_planes_stay_below_4_gib():
    # the kernels address each plane with 32-bit byte offsets: 16384 x 8192 holds
    # 3J + 1 = 7 frame planes (3.8 GB) at J = 2, not 10 at J = 3; TV's pair of
    # dual planes fits at 16384 x 16384
    assert A.admm_validate_problem(_prob(H=16384, W=8192, reg=A.ADMM_REG_FRAME, levels=2)) == A.ADMM_OK
    assert A.admm_validate_problem(_prob(H=16384, W=8192, reg=A.ADMM_REG_FRAME, levels=3)) == A.ADMM_E_UNSUPPORTED
    assert "4 GiB" in A.admm_last_error()
    assert A.admm_validate_problem(_prob(H=16384, W=16384)) == A.ADMM_OK


def test_zero_sum_kernel_allowed_for_frame():
    k = np.zeros((3, 3))
    k[1, 0], k[1, 2] = 1.0, -1.0
    assert A.admm_validate_problem(_prob(kernel=k, reg=A.ADMM_REG_FRAME, levels=2)) == A.ADMM_OK


def test_plan_rejects_invalid_before_touching_the_device():
    k = np.zeros((3, 3))
    k[1, 0], k[1, 2] = 1.0, -1.0
    with pytest.raises(A.AdmmError) as e:
        A.admm_deconv_plan([_prob(), _prob(kernel=k)], stream=0)
    assert e.value.status == A.ADMM_E_SINGULAR
    assert "problem 1" in str(e.value)
    with pytest.raises(A.AdmmError) as e:
        A.admm_deconv_plan([], stream=0)
    assert e.value.status == A.ADMM_E_INVALID


def test_product_path_has_no_oracle_dependency():
    # the binding and the package must not import the oracle (test infrastructure)
    pkg = os.path.join(ROOT, "paper_1210_2687_amd")
    for fn in os.listdir(pkg):
        if fn.endswith(".py"):
            src = open(os.path.join(pkg, fn)).read()
            assert "import oracle" not in src and "from oracle" not in src, fn


@pytest.mark.parametrize("n", [8, 12, 64, 96, 160, 448, 512, 1000, 1024, 1960, 2048])
def test_schedule_variants_factor_n(n):
    default = A.admm_fft_radices(n)
    assert A.admm_fft_schedule(n, 0) == default
    a = 0
    m = n
    while m % 2 == 0:
        m //= 2
        a += 1
    for v in (1, 2, 3):
        r = A.admm_fft_schedule(n, v)
        assert r is not None and int(np.prod(r)) == n, (n, v, r)
        assert all(x in (2, 3, 4, 5, 7, 8, 16) for x in r)
        assert sorted(x for x in r if x % 2) == sorted(x for x in default if x % 2)   # same odd factors
        if v == 1:
            assert all(x in (2, 3, 4, 5, 7) for x in r)
        if v == 2 and any(x % 2 for x in r):
            assert r[0] % 2 == 1                         # odd radices first
        if v == 3:
            assert r.count(16) == a // 4
    assert A.admm_fft_schedule(n, 4) is None and A.admm_fft_schedule(n, -1) is None
