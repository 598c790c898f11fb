"""C-ABI checks that need no GPU: the library loads, exports every entry
point the header declares, and its own parameter-table builder agrees with
the oracle's independent one."""
import ctypes
import os
import re

import numpy as np
import pytest

from oracle import params
from paper_1607_02904_amd import tersoff

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    txt = open(os.path.join(ROOT, "include", "tersoff.h")).read()
    return sorted(set(re.findall(r"\b(ters_[a-z_]+)\s*\(", txt)))


def test_header_declares_the_binding_exports():
    assert set(_declared()) == set(tersoff.EXPORTS)


def test_library_exports_every_declared_symbol():
    L = tersoff.load_library()
    for name in _declared():
        assert hasattr(L, name), name


def test_version_string():
    assert b"gfx950" in tersoff.load_library().ters_version()


def test_sic_table_matches_oracle_builder():
    ours = tersoff.table_sic()
    ref = params.sic()
    assert ours.shape == ref.shape
    assert np.allclose(ours, ref, rtol=1e-15, atol=0.0)
    # unlike-pair entries really are mixed, like-pair entries are the element's
    assert ours[0, 1, 1, params.IDX["A"]] == pytest.approx(1597.311, rel=1e-6)
    assert ours[0, 0, 0, params.IDX["A"]] == params.SI_C["A"]


@pytest.mark.parametrize("name,elem", [("Si(B)", params.SI_B), ("Si(C)", params.SI_C), ("C", params.CARBON)])
def test_element_tables_match_oracle(name, elem):
    assert np.array_equal(tersoff.table_element(name), params.single(elem))


def test_null_arguments_are_rejected_without_a_device():
    L = tersoff.load_library()
    assert L.ters_table_sic(None) == 1
    assert L.ters_destroy(None) == 1
    assert L.ters_sync(None) == 1
    assert L.ters_set_filter(None, 1) == 1
    assert L.ters_set_force_mode(None, 1) == 1
    out = ctypes.c_void_p()
    assert L.ters_create(None, 0, None) == 1
    assert L.ters_last_error(None) == b"null context"
