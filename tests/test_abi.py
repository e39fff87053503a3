"""The C ABI library loads and exports every function declared in include/*.h,
and the product never reaches into the oracle (no GPU needed)."""
import ctypes
import glob
import os
import re

import pytest

from paper_1510_04591_amd import adc

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        txt = open(h).read()
        txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
        names |= set(re.findall(r"\b(adc_[a-z0-9_]+)\s*\(", txt))
    return sorted(names)


def test_header_declares_the_solver():
    names = declared_functions()
    for must in ("adc_create", "adc_destroy", "adc_stedc", "adc_stedc_batched", "adc_secular",
                 "adc_lowner", "adc_cauchy_gemm", "adc_hss_build", "adc_hss_apply", "adc_mlp_train"):
        assert must in names


def test_library_exports_every_declared_symbol():
    if not os.path.exists(adc.LIB_PATH):
        pytest.skip("libadc.so not built")
    lib = ctypes.CDLL(adc.LIB_PATH)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing
    assert set(adc.EXPORTS) <= set(declared_functions())


def test_status_strings_and_defaults():
    if not os.path.exists(adc.LIB_PATH):
        pytest.skip("libadc.so not built")
    assert adc.status_string(0) == "ADC_OK"
    assert "NOCONV" in adc.status_string(adc.ADC_ERR_NOCONV)
    o = adc.opts()
    assert (o.dc_leaf, o.hss_min_k, o.hss_leaf, o.oversample, o.r_cap) == (32, 2048, 128, 16, 100)
    assert o.id_tol == 1e-14 and o.rank_eps == 1e-16
    assert o.hss_levels == -1 and o.hss_min_flops == 2.5e10


def test_product_does_not_use_the_oracle():
    srcs = glob.glob(os.path.join(ROOT, "paper_1510_04591_amd", "**", "*.*"), recursive=True)
    for s in srcs:
        if s.endswith((".py", ".hip", ".hpp", ".cpp", ".h")):
            txt = open(s).read()
            assert not re.search(r"^\s*(from|import)\s+oracle", txt, re.M), s
            assert not re.search(r"\boracle\.", txt), s
