"""The C-ABI library loads and exports every entry point of include/dsanls.h;
host-side validation returns the documented status codes (no GPU needed)."""
import ctypes
import os
import re

import pytest

from paper_2009_02845_amd import binding as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _header_functions():
    text = open(os.path.join(ROOT, "include", "dsanls.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(dsanls_[A-Za-z0-9_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    lib = B.load()
    names = _header_functions()
    assert len(names) >= 19
    for name in names:
        assert hasattr(lib, name), name
    # and the binding covers all of them
    assert set(names) == set(B.exported_symbols())


def test_status_strings():
    lib = B.load()
    assert lib.dsanls_status_string(0) == b"ok"
    assert lib.dsanls_status_string(7) == b"unsupported"


def _ws(cfg, mat):
    lib = B.load()
    out = ctypes.c_size_t(0)
    st = lib.dsanls_workspace_bytes(ctypes.byref(cfg), ctypes.byref(mat), ctypes.byref(out))
    return st, out.value


FAKE = 1 << 20   # never dereferenced: workspace sizing only reads sizes


def _dense(ld):
    return B.Matrix(format=B.DENSE, dense=FAKE, ld=ld)


@pytest.mark.parametrize("kw,status", [
    (dict(m=0, n=5, k=2, d=3), 2),
    (dict(m=5, n=5, k=513, d=3), 7),
    (dict(m=5, n=5, k=200, d=3, sweeps=0), 7),
    (dict(m=5, n=5, k=200, d=3, solver="pgd"), 7),
    (dict(m=5, n=5, k=200, d=3), 0),
    (dict(m=5, n=5, k=2, d=6, sketch="subsample"), 2),
    (dict(m=5, n=5, k=2, d=4, sketch="identity"), 2),
    (dict(m=5, n=5, k=2, d=3, alpha=-1.0), 1),
    (dict(m=5, n=5, k=2, d=3, sweeps=0, max_sweeps=0), 1),
])
def test_validation_errors(kw, status):
    cfg = B.make_config(**kw)
    st, _ = _ws(cfg, _dense(kw["n"]))
    assert st == status
    assert B.load().dsanls_last_error()


def test_validation_matrix_errors():
    cfg = B.make_config(m=5, n=6, k=2, d=3)
    assert _ws(cfg, _dense(5))[0] == 1                       # ld < n
    assert _ws(cfg, B.Matrix(format=B.DENSE, dense=None, ld=6))[0] == 1
    csr = B.Matrix(format=B.CSR, rowptr=FAKE, colidx=FAKE, vals=FAKE, nnz=3,
                   t_rowptr=FAKE, t_colidx=FAKE, t_vals=FAKE)
    assert _ws(cfg, csr)[0] == 7                             # Gaussian on CSR
    cfg_s = B.make_config(m=5, n=6, k=2, d=3, sketch="subsample")
    assert _ws(cfg_s, csr)[0] == 0
    csr.t_rowptr = None
    st, with_t = _ws(cfg_s, csr)                             # CSR(M^T) built at init: more workspace
    assert st == 0 and with_t > _ws(cfg_s, B.Matrix(format=B.CSR, rowptr=FAKE, colidx=FAKE, vals=FAKE, nnz=3,
                                                   t_rowptr=FAKE, t_colidx=FAKE, t_vals=FAKE))[1]
    csr.t_rowptr = FAKE
    csr.t_vals = None
    assert _ws(cfg_s, csr)[0] == 1                           # CSR(M^T) given in part


def test_workspace_grows_with_problem():
    small = _ws(B.make_config(m=100, n=80, k=8, d=20), _dense(80))
    big = _ws(B.make_config(m=1000, n=800, k=8, d=200), _dense(800))
    assert small[0] == 0 and big[0] == 0 and big[1] > small[1] > 0


@pytest.mark.parametrize("kw,status", [
    # mu_0 = alpha = 0 only in to-tolerance mode
    (dict(m=5, n=5, k=2, d=3, alpha=0.0, beta=1.0), 1),
    (dict(m=5, n=5, k=2, d=3, alpha=0.0, solver="pgd"), 1),
    (dict(m=5, n=5, k=2, d=3, alpha=0.0, beta=0.0, sweeps=0, max_sweeps=10), 0),
    # a node's share must lie inside the whole matrix
    (dict(m=5, n=5, k=2, d=3, row_offset=3, m_global=7), 2),
    (dict(m=5, n=5, k=2, d=3, row_offset=2, m_global=7), 0),
    (dict(m=5, n=5, k=2, d=3, col_offset=-1), 2),
    (dict(m=5, n=5, k=2, d=3, m_global=4), 2),
    # subsampling draws d of n_global columns; identity needs the whole matrix
    (dict(m=5, n=5, k=2, d=8, d_prime=3, sketch="subsample", col_offset=5, n_global=10), 0),
    (dict(m=5, n=5, k=2, d=11, d_prime=3, sketch="subsample", col_offset=5, n_global=10), 2),
    (dict(m=5, n=5, k=2, d=5, sketch="identity", n_global=10), 7),
])
def test_validation_node_share_and_alpha(kw, status):
    cfg = B.make_config(**kw)
    st, _ = _ws(cfg, _dense(kw["n"]))
    assert st == status, B.load().dsanls_last_error()


def test_status_string_internal():
    assert B.load().dsanls_status_string(8) == b"internal failure"
