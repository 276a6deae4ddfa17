"""The C-ABI library loads and exports every symbol include/fcns.h declares
(no compute call: these run without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fcns.h")
LIB = os.path.join(ROOT, "paper_2002_01392_amd", "libfcns.so")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(fcns_[a-z_]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for n in ("fcns_create", "fcns_destroy", "fcns_fc_extend", "fcns_fc_derivative",
              "fcns_rhs_nonlinear", "fcns_pressure_project", "fcns_set_state",
              "fcns_rk_step", "fcns_get_state", "fcns_last_error"):
        assert n in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libfcns.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    for n in declared_functions():
        assert hasattr(lib, n), n


@pytest.mark.skipif(not os.path.exists(LIB), reason="libfcns.so not built")
def test_binding_signatures_cover_the_header():
    from paper_2002_01392_amd import _lib
    assert set(declared_functions()) == set(_lib.SIGNATURES)


def test_problem_struct_matches_header_field_order():
    from paper_2002_01392_amd._lib import FcnsProblem
    src = open(HEADER).read()
    body = src[src.index("typedef struct {"):src.index("} fcns_problem;")]
    body = re.sub(r"/\*.*?\*/", "", body, flags=re.S)
    names = re.findall(r"([A-Za-z_0-9]+)\s*[,;]", body.replace("*", " "))
    assert [f[0] for f in FcnsProblem._fields_] == names


def test_fc_tables_agree_with_the_independent_oracle_tables():
    # the solver's table generator and the oracle's are separate codes
    # (Gram-Schmidt + Householder least squares vs. QR + normal equations)
    import numpy as np
    from oracle.fc_table import fc_tables
    from paper_2002_01392_amd import fctable
    for d, C in fctable.STANDARD:
        t = fctable.load(d, C)
        Q = t[:d * d].reshape(d, d)
        A = t[d * d:].reshape(C, d)
        Qo, Ao, Mo, _ = fc_tables(d, C)
        assert np.abs(Q - Qo).max() < 1e-15
        assert np.abs(A - Ao).max() <= 1e-15 * np.abs(Ao).max()
        assert np.abs(A @ Q.T - Mo).max() < 1e-14 * np.abs(Mo).max()


@pytest.mark.skipif(not os.path.exists(LIB), reason="libfcns.so not built")
def test_footprint_counts_the_context_buffers():
    # no device needed: the library computes it from the shape
    from paper_2002_01392_amd import problem_bytes
    b = problem_bytes(512, 512, 257, 31, 4)
    nkxp = 260
    S, M = 288 * 512 * nkxp * 16, 257 * 512 * nkxp * 16
    W = 8 * 512 * nkxp * 16          # wall-gradient arrays
    assert 12 * S + 33 * M + W <= b < 12 * S + 33 * M + W + (1 << 22)
    assert problem_bytes(32, 32, 33, 31, 3) < problem_bytes(64, 64, 65, 31, 3)
