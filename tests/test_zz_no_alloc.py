"""tc_tei_gram_noalloc (the static-scratch variant of tc_tei_gram) through
the C ABI: two calls in a row, the second on a smaller problem, each against
tc_tei_gram on the same inputs (bitwise: the same plans and kernels) and
against the FP64 oracle (1e-12 for binary64, 1e-7 for the int8 split)."""

import ctypes

import numpy as np
import pytest
import torch

from paper_1504_06289_amd import _lib
from paper_1504_06289_amd import workloads as wl
from tests.gpu_common import (block_columns, column_errors, dev, host, oracle_columns,
                              oracle_setup, say)
from tests.metrics import e_J

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-12, "ozaki8": 1e-7}


def _instances(tc, ws_list):
    """(c, p3, U3) device tuples and the TcInstance array with fresh J outputs."""
    insts, Js = [], []
    arr = (_lib.TcInstance * len(ws_list))()
    for i, (c, ps, U) in enumerate(ws_list):
        cd, pd, Ud = dev(c), [dev(p) for p in ps], [dev(u) for u in U]
        J = torch.full((U[0].shape[0],) * 2, np.nan, dtype=torch.float64, device="cuda")
        arr[i] = tc.make_instance(cd, pd, Ud, J, None)
        insts.append((cd, pd, Ud))
        Js.append(J)
    return insts, arr, Js


def _noalloc(tc, ws_list, prec):
    insts, arr, Js = _instances(tc, ws_list)
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    s = _lib.lib().tc_tei_gram_noalloc(arr, len(ws_list), _lib.PRECISIONS[prec], stream)
    assert s == _lib.TC_OK, _lib.lib().tc_status_string(s)
    return insts, [host(J) for J in Js]


@pytest.mark.parametrize("prec", ["fp64", "ozaki8"])
def test_noalloc_matches_tei_gram_two_calls(tc, orc, prec):
    L = _lib.lib()
    # first call: the 1024-cell workload (R_f = 256, R_N = 30)
    w = wl.config("c2")
    c, ps = oracle_setup(orc, w)
    arr = (_lib.TcInstance * 1)()
    arr[0] = tc.make_instance(dev(c), [dev(p) for p in ps], [dev(u) for u in w.U],
                              torch.empty((1, 1), dtype=torch.float64, device="cuda"), None)
    need = L.tc_workspace_bytes(_lib.TC_OP_TEI_GRAM, arr, 1, _lib.PRECISIONS[prec])
    say(f"noalloc {prec}: 1024 cells, workspace {need / 2**20:.1f} MiB of "
        f"{_lib.TC_NOALLOC_SCRATCH_BYTES / 2**20:.0f}")
    assert need <= _lib.TC_NOALLOC_SCRATCH_BYTES
    insts, (J1,) = _noalloc(tc, [(c, ps, w.U)], prec)
    ref1 = host(tc.tei_gram(*insts[0], prec=prec))
    np.testing.assert_array_equal(J1, ref1)
    S = block_columns(w.R_f, seed=123)
    e_blk, e_cols = column_errors(J1, oracle_columns(orc, "c2", c, ps, w.U, S), S)
    say(f"   first call: bitwise equal to tc_tei_gram; {len(S)} oracle columns {e_cols:.2e}")
    assert e_blk <= TOL[prec] and e_cols <= TOL[prec]

    # second call, smaller: a batch of two small instances (several tiles,
    # ragged tails); the scratch keeps the first call's data
    small = []
    for i, (n, R_f, R_N) in enumerate([(300, 100, 9), ((130, 64, 200), 37, 6)]):
        ws_ = wl.small_products(n, R_f, R_N=R_N, b=6.0, seed=60 + i)
        cs, pss = oracle_setup(orc, ws_)
        small.append((cs, pss, ws_.U))
    insts2, J2 = _noalloc(tc, small, prec)
    ref2 = [host(J) for J in tc.tei_gram_batched(insts2, prec=prec)]
    for (cs, pss, Us), Jn, Jr in zip(small, J2, ref2):
        np.testing.assert_array_equal(Jn, Jr)
        err = e_J(Jn, orc.tei_gram(cs, pss, Us))
        say(f"   second call: bitwise equal to tc_tei_gram; e_J {err:.2e}")
        assert err <= TOL[prec]


def test_noalloc_rejects_beyond_scratch(tc, orc):
    w = wl.config("c5")
    c, ps = oracle_setup(orc, w)
    insts, arr, Js = _instances(tc, [(c, ps, w.U)])
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    s = _lib.lib().tc_tei_gram_noalloc(arr, 1, _lib.TC_FP64, stream)
    assert s == _lib.TC_ERR_WORKSPACE
    assert torch.isnan(Js[0]).all()   # nothing written
