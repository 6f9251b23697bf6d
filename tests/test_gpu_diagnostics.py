"""The diagnostic switches of the C ABI on the GPU:
  * TC_CHECK_FINITE=1: a NaN or Inf in any binary64 input is reported as
    TC_ERR_INVALID_ARG before any work, and no output is written; clean
    inputs give bitwise the results of a run without the check;
  * TC_DEBUG_SYNC=1: every launch is followed by a synchronisation; the
    results are bitwise those of a run without it.
"""

import ctypes

import numpy as np
import pytest
import torch

from paper_1504_06289_amd import _lib
from paper_1504_06289_amd import workloads as wl
from tests.gpu_common import dev, host, oracle_setup, say

pytestmark = pytest.mark.gpu


def _setup(orc):
    w = wl.small_products(300, 40, R_N=6, b=6.0, seed=21)
    c, ps = oracle_setup(orc, w)
    return w, c, ps


def _tei_status(tc, c, ps, U, prec):
    """tc_tei_gram through the ABI with a NaN-filled J; returns (status, J)."""
    R_f = U[0].shape[0]
    J = torch.full((R_f, R_f), np.nan, dtype=torch.float64, device="cuda")
    arr = (_lib.TcInstance * 1)(tc.make_instance(c, ps, U, J, None))
    L = _lib.lib()
    nb = L.tc_workspace_bytes(_lib.TC_OP_TEI_GRAM, arr, 1, _lib.PRECISIONS[prec])
    ws = torch.empty(nb, dtype=torch.uint8, device="cuda")
    s = L.tc_tei_gram(arr, 1, _lib.PRECISIONS[prec], ctypes.c_void_p(ws.data_ptr()), nb,
                      ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    return s, host(J)


@pytest.mark.parametrize("prec", ["fp64", "ozaki8"])
def test_check_finite(tc, orc, monkeypatch, prec):
    w, c, ps = _setup(orc)
    cd, pd, Ud = dev(c), [dev(p) for p in ps], [dev(u) for u in w.U]
    monkeypatch.delenv("TC_CHECK_FINITE", raising=False)
    s0, J0 = _tei_status(tc, cd, pd, Ud, prec)
    assert s0 == _lib.TC_OK
    monkeypatch.setenv("TC_CHECK_FINITE", "1")
    s1, J1 = _tei_status(tc, cd, pd, Ud, prec)
    assert s1 == _lib.TC_OK
    np.testing.assert_array_equal(J1, J0)
    # one bad value in each input in turn
    for name, bad in [("U[1]", np.nan), ("p[2]", np.inf), ("c", -np.inf), ("U[0]", np.nan)]:
        cb, pb, Ub = cd.clone(), [p.clone() for p in pd], [u.clone() for u in Ud]
        if name == "c":
            cb[3] = bad
        elif name.startswith("p"):
            pb[int(name[2])][1, 17] = bad
        else:
            Ub[int(name[2])][-1, -1] = bad
        s, J = _tei_status(tc, cb, pb, Ub, prec)
        say(f"   {prec}: {name} = {bad}: status {s}")
        assert s == _lib.TC_ERR_INVALID_ARG, (name, s)
        assert np.isnan(J).all(), name   # nothing written
    # without the switch the same input runs (and its J carries the NaN)
    monkeypatch.delenv("TC_CHECK_FINITE")
    Ub = [u.clone() for u in Ud]
    Ub[0][0, 0] = np.nan
    s, J = _tei_status(tc, cd, pd, Ub, prec)
    assert s == _lib.TC_OK and np.isnan(J).any()


def test_check_finite_backward_and_convolve(tc, orc, monkeypatch):
    w, c, ps = _setup(orc)
    cd, pd, Ud = dev(c), [dev(p) for p in ps], [dev(u) for u in w.U]
    Jb = torch.randn(w.R_f, w.R_f, dtype=torch.float64, device="cuda")
    monkeypatch.setenv("TC_CHECK_FINITE", "1")
    ref = [host(x) for x in tc.tei_gram_backward(cd, pd, Ud, Jb)]
    Jb[2, 5] = np.nan
    with pytest.raises(_lib.TcError) as e:
        tc.tei_gram_backward(cd, pd, Ud, Jb)
    assert e.value.status == _lib.TC_ERR_INVALID_ARG
    W = host(tc.convolve(pd[0], Ud[0]))
    Ub = Ud[0].clone()
    Ub[3, 3] = np.inf
    with pytest.raises(_lib.TcError) as e:
        tc.convolve(pd[0], Ub)
    assert e.value.status == _lib.TC_ERR_INVALID_ARG
    monkeypatch.delenv("TC_CHECK_FINITE")
    np.testing.assert_array_equal(host(tc.convolve(pd[0], Ud[0])), W)
    Jb[2, 5] = 0.0
    assert all(np.isfinite(r).all() for r in ref)


@pytest.mark.parametrize("prec", ["fp64", "ozaki8"])
def test_debug_sync_same_results(tc, orc, monkeypatch, prec):
    w, c, ps = _setup(orc)
    cd, pd, Ud = dev(c), [dev(p) for p in ps], [dev(u) for u in w.U]
    monkeypatch.delenv("TC_DEBUG_SYNC", raising=False)
    J0 = host(tc.tei_gram(cd, pd, Ud, prec=prec))
    monkeypatch.setenv("TC_DEBUG_SYNC", "1")
    J1 = host(tc.tei_gram(cd, pd, Ud, prec=prec))
    Jb = host(tc.tei_gram_batched([(cd, pd, Ud), (cd, pd, Ud)], prec=prec)[1])
    np.testing.assert_array_equal(J1, J0)
    np.testing.assert_array_equal(Jb, J0)
