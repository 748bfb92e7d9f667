"""Host-side checks of libdf3c that need no GPU: the library loads, exports every
entry point declared in include/df3c.h, and rejects bad arguments before any
device work."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "df3c.h")


def _declared():
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:const\s+)?[A-Za-z_0-9]+\s*\*?\s*(df3c_[A-Za-z_0-9]+)\s*\(",
                                 txt, re.M)))


@pytest.fixture(scope="module")
def lib():
    from paper_2210_03192_amd import df3c
    if not os.path.exists(df3c.LIB_PATH):
        pytest.fail("libdf3c.so is not built (run paper_2210_03192_amd/build.py)")
    return df3c.lib()


def test_header_declares_entry_points():
    names = _declared()
    for n in ("df3c_eval_batch", "df3c_coulomb_J", "df3c_coulomb_J_grad", "df3c_init",
              "df3c_status_string"):
        assert n in names


def test_exports_every_declared_symbol(lib):
    for n in _declared():
        assert hasattr(lib, n), n


def test_status_strings(lib):
    for code in (0, -1, -2, -3, -4):
        assert lib.df3c_status_string(code)
    assert lib.df3c_status_string(-99) == b"unknown status"


def test_eval_batch_rejects_null_arguments(lib):
    # validation happens before any HIP call, so this runs without a GPU
    rc = lib.df3c_eval_batch(None, 1, None, None, 5, None, None, None, None, 0, 0, None)
    assert rc == -1
    rc = lib.df3c_eval_batch(None, 1, None, None, -1, None, None, None, None, 0, 0, None)
    assert rc == -1
    assert lib.df3c_eval_batch(None, 1, None, None, 0, None, None, None, None, 0, 0, None) == 0


def test_coulomb_J_rejects_null_arguments(lib):
    assert lib.df3c_coulomb_J(None, 1, None, None, None, None, None, 0, 0, None) == -1
    assert lib.df3c_coulomb_J_grad(None, 1, None, None, None, None, None, None, 0, 0, None) == -1


def test_workspace_sizes(lib):
    a = lib.df3c_eval_batch_workspace(0)
    b = lib.df3c_eval_batch_workspace(100000)
    assert 0 < a < b


def test_screening_entry_points_reject_bad_arguments(lib):
    # null pointers, a null mask and a negative or NaN threshold are rejected
    # before any HIP call
    assert lib.df3c_screen_pairs(None, 1, None, ctypes.c_double(1e-12), None, None) == -1
    assert lib.df3c_coulomb_J_masked(None, 1, None, None, None, None, None, None, 0, 0, None) == -1
    buf = (ctypes.c_double * 3)()
    assert lib.df3c_screen_pairs(buf, 1, None, ctypes.c_double(-1.0), buf, None) == -1
    assert lib.df3c_screen_pairs(buf, 1, None, ctypes.c_double(float("nan")), buf, None) == -1
    assert lib.df3c_coulomb_J_masked_workspace(None, None) == 0


def test_pure_orbital_options(lib):
    # solid-harmonic orbital shells need workspace for the Cartesian J (or the
    # pulled-back G) on top of the Cartesian sizes; pure flags other than 0
    # and 1 are rejected before any HIP call
    from paper_2210_03192_amd import df3c
    lo = np.array([0, 1, 2, 3], np.int32)
    la = np.array([0], np.int32)
    buf = (ctypes.c_double * 8)()
    p = ctypes.cast(buf, ctypes.c_void_p).value

    def shells(l, pure):
        return df3c._Shells(len(l), l.ctypes.data, p, p, p, p, p, p, pure, None)
    aux = shells(la, 1)
    cart, pure, bad = shells(lo, 0), shells(lo, 1), shells(lo, 2)
    nc = 1 + 3 + 6 + 10
    wc = lib.df3c_coulomb_J_workspace(ctypes.byref(aux), ctypes.byref(cart))
    wp = lib.df3c_coulomb_J_workspace(ctypes.byref(aux), ctypes.byref(pure))
    assert wp >= wc + 8 * nc * nc
    wmc = lib.df3c_coulomb_J_masked_workspace(ctypes.byref(aux), ctypes.byref(cart))
    wmp = lib.df3c_coulomb_J_masked_workspace(ctypes.byref(aux), ctypes.byref(pure))
    assert wmp >= wmc + 8 * nc * nc
    gc = lib.df3c_coulomb_J_grad_workspace(ctypes.byref(aux), ctypes.byref(cart), 1)
    gp = lib.df3c_coulomb_J_grad_workspace(ctypes.byref(aux), ctypes.byref(pure), 1)
    assert gp >= gc + 8 * nc * nc
    assert lib.df3c_coulomb_J(buf, 1, ctypes.byref(aux), ctypes.byref(bad), buf, buf, buf,
                              1 << 40, 0, None) == -2
    assert lib.df3c_coulomb_J_grad(buf, 1, ctypes.byref(aux), ctypes.byref(bad), buf, buf, buf,
                                   buf, 1 << 40, 0, None) == -2
    # batched: pure orbital shells need the molecule ranges to size the
    # Cartesian J of every molecule (two molecules of two shells each here)
    mo = np.array([0, 2, 4], np.int32)
    bc = lib.df3c_coulomb_J_batched_workspace(ctypes.byref(aux), ctypes.byref(cart), 2, None)
    assert bc > 0
    assert lib.df3c_coulomb_J_batched_workspace(ctypes.byref(aux), ctypes.byref(pure), 2,
                                                None) == 0
    bp = lib.df3c_coulomb_J_batched_workspace(ctypes.byref(aux), ctypes.byref(pure), 2,
                                              mo.ctypes.data)
    assert bp >= bc + 8 * ((1 + 3) ** 2 + (6 + 10) ** 2)
    bad_mo = np.array([0, 3, 2], np.int32)
    assert lib.df3c_coulomb_J_batched_workspace(ctypes.byref(aux), ctypes.byref(pure), 2,
                                                bad_mo.ctypes.data) == 0


def test_null_l_host_rejected_before_device_work(lib):
    # the plans are sized from l_host: a basis without it is rejected by every
    # entry point (and its workspace query gives 0) before any HIP call
    from paper_2210_03192_amd import df3c
    la = np.array([0, 1], np.int32)
    buf = (ctypes.c_double * 8)()
    p = ctypes.cast(buf, ctypes.c_void_p).value
    good = df3c._Shells(len(la), la.ctypes.data, p, p, p, p, p, p, 1, None)
    nol = df3c._Shells(len(la), None, p, p, p, p, p, p, 0, None)
    nol_pure = df3c._Shells(len(la), None, p, p, p, p, p, p, 1, None)
    A, O, Op = ctypes.byref(good), ctypes.byref(nol), ctypes.byref(nol_pure)
    big = 1 << 40
    assert lib.df3c_coulomb_J(buf, 1, A, O, buf, buf, buf, big, 0, None) == -1
    assert lib.df3c_coulomb_J_masked(buf, 1, A, O, buf, buf, buf, buf, big, 0, None) == -1
    assert lib.df3c_coulomb_J_grad(buf, 1, A, Op, buf, buf, buf, buf, big, 0, None) == -1
    assert lib.df3c_coulomb_J_grad_masked(buf, 1, A, O, buf, buf, buf, buf, buf, big, 0,
                                          None) == -1
    assert lib.df3c_coulomb_gamma(buf, 1, A, O, buf, buf, buf, big, 0, None) == -1
    assert lib.df3c_coulomb_J_workspace(A, O) == 0
    assert lib.df3c_coulomb_J_masked_workspace(A, O) == 0
    assert lib.df3c_coulomb_J_grad_workspace(A, Op, 1) == 0
    assert lib.df3c_coulomb_J_grad_masked_workspace(A, O, 1) == 0


def test_unknown_flags_rejected(lib):
    # flags beyond each entry point's set are rejected before any HIP call
    from paper_2210_03192_amd import df3c
    la = np.array([0], np.int32)
    buf = (ctypes.c_double * 8)()
    p = ctypes.cast(buf, ctypes.c_void_p).value
    sh = df3c._Shells(1, la.ctypes.data, p, p, p, p, p, p, 1, None)
    S = ctypes.byref(sh)
    big = 1 << 40
    assert lib.df3c_coulomb_J(buf, 1, S, S, buf, buf, buf, big, 8, None) == -1
    assert lib.df3c_coulomb_J_grad(buf, 1, S, S, buf, buf, buf, buf, big, 1, None) == -1
    assert lib.df3c_eval_batch(buf, 1, S, S, 1, buf, buf, buf, buf, big, 2, None) == -1
    assert lib.df3c_workspace_status(None, None) == -1
