"""CPU checks of the C ABI: the library loads, exports every function include/whmc.h declares,
and its host-only logic (filter coefficient tables) agrees with the oracle.  No GPU calls."""
import ctypes
import os
import re

import numpy as np
import pytest

from oracle import hpe
from paper_1805_03560_amd import whmc

HEADER = os.path.join(os.path.dirname(os.path.dirname(__file__)), "include", "whmc.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:whmc_status|void|int|const char\s*\*)\s*(whmc_\w+)\s*\(", text, re.M)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("whmc_load_gauge", "whmc_apply_H", "whmc_apply_MdagM", "whmc_cg_solve", "whmc_force",
                     "whmc_hmc_trajectory"):
        assert required in names


def test_library_exports_every_declared_symbol():
    L = ctypes.CDLL(whmc.LIB_PATH)
    missing = [n for n in declared_functions() if not hasattr(L, n)]
    assert not missing, missing
    assert whmc.lib().whmc_abi_version() == 1


@pytest.mark.parametrize("k,n", [(0, 5), (1, 19), (2, 29), (2, 60)])
def test_filter_coefficients_match_oracle(k, n):
    b, c, alpha = whmc.filter_coefficients(k, n)
    _, bo, co, ao = hpe.coefficients(k, n)
    assert alpha == pytest.approx(float(ao), rel=1e-15)
    for i in range(n + 1):
        assert b[i] == pytest.approx(float(bo[i]), rel=1e-12, abs=1e-25)
        assert c[i] == pytest.approx(float(co[i]), rel=1e-12, abs=1e-25)


def test_filter_coefficients_reject_bad_input():
    with pytest.raises(whmc.WhmcError):
        whmc.filter_coefficients(-1, 3)
