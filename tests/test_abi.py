"""The C-ABI library loads and exports every symbol include/tc.h declares, and
its host-side validation rejects bad arguments before touching the GPU
(CPU only: none of these calls reaches a kernel launch)."""
import ctypes
import os
import re

import pytest

from paper_1504_06289_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "tc.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(tc_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(_lib.LIB_PATH):
        pytest.fail("libtc.so is not built (python -m paper_1504_06289_amd.build)")
    return _lib.lib()


def test_exports_every_declared_symbol(L):
    names = declared_functions()
    assert set(names) == set(_lib.EXPORTS), names
    for name in names:
        assert hasattr(L, name), name


def test_status_strings(L):
    for s in range(5):
        assert L.tc_status_string(s).decode().startswith("TC_")
    assert b"unknown" in L.tc_status_string(99)
    assert L.tc_version() >= 100


def declared_enum(name):
    """{enumerator: value} of the typedef enum `name` in include/tc.h."""
    text = open(os.path.join(ROOT, "include", "tc.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    body = re.search(r"typedef enum \{([^}]*)\}\s*" + name + r"\s*;", text).group(1)
    # the *_RANGE_MIN_/*_RANGE_MAX_ entries only widen the enum to the range of int
    return {k: int(v) for k, v in re.findall(r"(TC_[A-Z0-9_]+)\s*=\s*(\d+)", body)
            if not k.endswith(("_RANGE_MIN_", "_RANGE_MAX_"))}


def test_enum_values_follow_the_interface():
    """The precision and status codes keep the interface's numbering
    (binary64 0, binary32 1, split-bfloat16 with three products 2 and with
    six 3); the int8 splitting is appended after them, so a caller written
    against the first numbering never reaches it by accident."""
    prec = declared_enum("tc_precision")
    assert prec == {"TC_FP64": 0, "TC_FP32": 1, "TC_BF16X3": 2, "TC_BF16X6": 3,
                    "TC_OZAKI_I8": 4}
    for k, v in prec.items():
        assert getattr(_lib, k) == v, k
    assert _lib.PRECISIONS == {"fp64": 0, "fp32": 1, "bf16x3": 2, "bf16x6": 3, "ozaki8": 4}
    status = declared_enum("tc_status")
    assert status == {"TC_OK": 0, "TC_ERR_INVALID_ARG": 1, "TC_ERR_WORKSPACE": 2,
                      "TC_ERR_UNSUPPORTED": 3, "TC_ERR_HIP": 4}
    for k, v in status.items():
        assert getattr(_lib, k) == v, k
    assert declared_enum("tc_algorithm") == {"TC_ALGO_AUTO": 0, "TC_ALGO_DIRECT": 1,
                                             "TC_ALGO_FFT": 2}
    routes = declared_enum("tc_batch_route")
    assert routes == {"TC_BATCH_AUTO": 0, "TC_BATCH_FORK_JOIN": 1, "TC_BATCH_QUEUE": 2,
                      "TC_BATCH_QUEUE_T64": 3, "TC_BATCH_QUEUE_K2": 4, "TC_BATCH_QUEUE_T64_K2": 5}
    assert sorted(_lib.BATCH_ROUTES.values()) == sorted(routes.values())


def _inst(n=64, R_f=8, R_N=4, null=None):
    I = _lib.TcInstance()
    for l in range(3):
        I.n[l] = n
        I.p[l] = 0x1000
        I.U[l] = 0x2000
    I.R_f, I.R_N = R_f, R_N
    I.c = 0x3000
    I.J = 0x4000
    I.G_saved = None
    if null:
        setattr(I, null, None)
    return I


def test_workspace_bytes(L):
    I = _inst(n=100, R_f=10, R_N=3)
    arr = (_lib.TcInstance * 1)(I)
    w = L.tc_workspace_bytes(_lib.TC_OP_TEI_GRAM, arr, 1, _lib.TC_FP64)
    # one instance runs its three modes concurrently: the three modes' Grams,
    # then per mode its W and its FFT scratch (twiddles [N], spectra of U
    # [R_f][N/2+1] and of the kernel [R_N][N/2+1], N = 256 for n = 100), each
    # rounded up to 256 bytes
    up = lambda x: (x + 255) // 256 * 256
    fft = up(16 * 256) + up(16 * 10 * 129) + up(16 * 3 * 129)
    mode = up(8 * 3 * 10 * 100) + fft
    assert w == up(8 * 3 * 3 * 100) + 3 * mode
    # row-scaled precisions add, per mode, the row exponents of U [R_f], p [R_N]
    # and W [R_N][R_f]
    for prec in (_lib.TC_FP32, _lib.TC_BF16X3, _lib.TC_BF16X6):
        assert L.tc_workspace_bytes(_lib.TC_OP_TEI_GRAM, arr, 1, prec) == \
            w + 3 * (up(4 * 10) + up(4 * 3) + up(4 * 3 * 10))
    I.G_saved = 0x5000
    arr = (_lib.TcInstance * 1)(I)
    assert L.tc_workspace_bytes(_lib.TC_OP_TEI_GRAM, arr, 1, _lib.TC_FP64) == 3 * mode
    # the adjoint runs the modes in turn: one W and one mode's scratch, and D
    wb = L.tc_workspace_bytes(_lib.TC_OP_TEI_GRAM_BACKWARD, arr, 1, _lib.TC_FP64)
    assert wb == up(8 * 3 * 10 * 100) + up(8 * 3 * 100) + fft
    # beyond 4096 cells the FFT route is four-step: per mode the twiddles
    # [N], the spectra of the row pairs [P][N] and of the kernel [R_N][N],
    # the inverse scratch [kc][P][N] (N = 16384 for 5000 cells, P = 1,
    # kc = 1) and the rows' exponents [R_f]; with the direct route pinned only
    # W remains
    I = _inst(n=5000, R_f=2, R_N=1)
    I.G_saved = 0x5000
    arr = (_lib.TcInstance * 1)(I)
    assert L.tc_tune_get(5000, 2, 1, _lib.TC_FP64) == _lib.ALGORITHMS["fft"]
    assert L.tc_workspace_bytes(_lib.TC_OP_TEI_GRAM, arr, 1, _lib.TC_FP64) == \
        3 * (up(8 * 2 * 5000) + 4 * up(16 * 16384) + up(4 * 2))
    try:
        L.tc_tune_set(5000, 2, 1, _lib.TC_FP64, _lib.ALGORITHMS["direct"])
        assert L.tc_workspace_bytes(_lib.TC_OP_TEI_GRAM, arr, 1, _lib.TC_FP64) == \
            3 * up(8 * 2 * 5000)
    finally:
        L.tc_tune_set(5000, 2, 1, _lib.TC_FP64, _lib.ALGORITHMS["auto"])
    bad = (_lib.TcInstance * 1)(_inst(n=0))
    assert L.tc_workspace_bytes(_lib.TC_OP_TEI_GRAM, bad, 1, _lib.TC_FP64) == ctypes.c_size_t(-1).value
    assert L.tc_workspace_bytes(7, arr, 1, _lib.TC_FP64) == ctypes.c_size_t(-1).value
    assert L.tc_workspace_bytes(_lib.TC_OP_TEI_GRAM, arr, 1, 42) == ctypes.c_size_t(-1).value


@pytest.mark.parametrize("kw", [dict(n=0), dict(n=70000), dict(R_f=0), dict(R_N=0),
                                dict(R_N=1000), dict(null="c"), dict(null="J")])
def test_tei_gram_rejects_bad_instances(L, kw):
    arr = (_lib.TcInstance * 1)(_inst(**kw))
    s = L.tc_tei_gram(arr, 1, _lib.TC_FP64, None, 0, None)
    assert s == _lib.TC_ERR_INVALID_ARG


def test_tei_gram_rejects_null_mode_pointers(L):
    I = _inst()
    I.U[1] = None
    assert L.tc_tei_gram((_lib.TcInstance * 1)(I), 1, _lib.TC_FP64, None, 0, None) == \
        _lib.TC_ERR_INVALID_ARG
    I = _inst()
    I.p[2] = None
    assert L.tc_tei_gram((_lib.TcInstance * 1)(I), 1, _lib.TC_FP64, None, 0, None) == \
        _lib.TC_ERR_INVALID_ARG
    assert L.tc_tei_gram(None, 1, _lib.TC_FP64, None, 0, None) == _lib.TC_ERR_INVALID_ARG
    arr = (_lib.TcInstance * 1)(_inst())
    assert L.tc_tei_gram(arr, 0, _lib.TC_FP64, None, 0, None) == _lib.TC_ERR_INVALID_ARG
    assert L.tc_tei_gram(arr, 1, 17, None, 0, None) == _lib.TC_ERR_INVALID_ARG


def test_tei_gram_workspace_checked_before_launch(L):
    arr = (_lib.TcInstance * 1)(_inst())
    need = L.tc_workspace_bytes(_lib.TC_OP_TEI_GRAM, arr, 1, _lib.TC_FP64)
    assert need > 0
    assert L.tc_tei_gram(arr, 1, _lib.TC_FP64, None, 0, None) == _lib.TC_ERR_WORKSPACE
    assert L.tc_tei_gram(arr, 1, _lib.TC_FP64, ctypes.c_void_p(0x6000), need - 1, None) == \
        _lib.TC_ERR_WORKSPACE


def test_newton_kernel_rejects(L):
    pd = ctypes.POINTER(ctypes.c_double)
    nul = ctypes.cast(None, pd)
    p = ctypes.c_void_p(0x1000)
    nan = float("nan")
    cases = [(0, 0.1, 4, -1.0, 0.5, p), (64, 0.0, 4, -1.0, 0.5, p), (64, -1.0, 4, -1.0, 0.5, p),
             (64, 0.1, 0, -1.0, 0.5, p), (64, 0.1, 4, nan, 0.5, p), (64, 0.1, 4, -1.0, 0.0, p),
             (64, 0.1, 4, -1.0, float("inf"), p), (64, 0.1, 4, -1.0, 0.5, None),
             (64, 0.1, 4, 800.0, 0.5, p)]  # exp overflows: t_k not finite
    for n, h, R_N, u0, hu, pp in cases:
        assert L.tc_newton_kernel(n, h, R_N, u0, hu, nul, nul, pp, None) == \
            _lib.TC_ERR_INVALID_ARG, (n, h, R_N, u0, hu)


def test_convolve_rejects(L):
    v = ctypes.c_void_p(0x1000)
    assert L.tc_convolve(0, 4, 4, v, v, v, 0, None, 0, None) == _lib.TC_ERR_INVALID_ARG
    assert L.tc_convolve(8, 4, 4, None, v, v, 0, None, 0, None) == _lib.TC_ERR_INVALID_ARG
    assert L.tc_convolve(8, 4, 4, v, v, None, 0, None, 0, None) == _lib.TC_ERR_INVALID_ARG
    assert L.tc_convolve(8, 4, 4, v, v, v, 9, None, 0, None) == _lib.TC_ERR_INVALID_ARG


def test_backward_rejects(L):
    arr = (_lib.TcInstance * 1)(_inst())
    jb = (ctypes.c_void_p * 1)(0x7000)
    du = (ctypes.c_void_p * 3)(0x8000, 0x9000, None)
    assert L.tc_tei_gram_backward(arr, 1, jb, du, _lib.TC_FP64, None, 0, None) == \
        _lib.TC_ERR_INVALID_ARG
    du = (ctypes.c_void_p * 3)(0x8000, 0x9000, 0xa000)
    assert L.tc_tei_gram_backward(arr, 1, jb, du, _lib.TC_FP64, None, 0, None) == \
        _lib.TC_ERR_WORKSPACE
    jb0 = (ctypes.c_void_p * 1)(None)
    assert L.tc_tei_gram_backward(arr, 1, jb0, du, _lib.TC_FP64, None, 0, None) == \
        _lib.TC_ERR_INVALID_ARG


def test_product_path_has_no_fallback():
    """The package never imports the oracle and fails loudly without libtc.so."""
    pkg = os.path.join(ROOT, "paper_1504_06289_amd")
    for f in os.listdir(pkg):
        if f.endswith(".py"):
            src = open(os.path.join(pkg, f)).read()
            assert not re.search(r"^\s*(from\s+oracle|import\s+oracle)", src, flags=re.M), f
            assert "liboracle" not in src, f


def declared_define(name):
    text = open(os.path.join(ROOT, "include", "tc.h")).read()
    return int(re.search(r"#define\s+" + name + r"\s+(\d+)", text).group(1))


def test_op_codes_and_static_scratch_size():
    for name in ("TC_OP_CONVOLVE", "TC_OP_TEI_GRAM", "TC_OP_TEI_GRAM_BACKWARD",
                 "TC_OP_AUTOTUNE", "TC_NOALLOC_SCRATCH_BYTES"):
        assert getattr(_lib, name) == declared_define(name), name
    assert _lib.TC_NOALLOC_SCRATCH_BYTES == 256 << 20


def test_int8_fft_forward_needs_no_binary64_W(L):
    """The int8 FFT route writes the int8 slices of W straight from the
    convolution: its forward plan holds no binary64 W, the direct route's and
    the autotuner's (every route may run) do."""
    I = _inst(n=1024, R_f=64, R_N=6)
    arr = (_lib.TcInstance * 1)(I)
    A = _lib.ALGORITHMS
    up = lambda x: (x + 255) // 256 * 256
    W = up(8 * 6 * 64 * 1024)
    assert L.tc_tune_get(1024, 64, 6, _lib.TC_OZAKI_I8) == A["fft"]
    fft = L.tc_workspace_bytes(_lib.TC_OP_TEI_GRAM, arr, 1, _lib.TC_OZAKI_I8)
    try:
        assert L.tc_tune_set(1024, 64, 6, _lib.TC_OZAKI_I8, A["direct"]) == _lib.TC_OK
        direct = L.tc_workspace_bytes(_lib.TC_OP_TEI_GRAM, arr, 1, _lib.TC_OZAKI_I8)
    finally:
        L.tc_tune_set(1024, 64, 6, _lib.TC_OZAKI_I8, A["auto"])
    assert direct == fft + 3 * W          # one W per concurrent mode
    tune = L.tc_workspace_bytes(_lib.TC_OP_AUTOTUNE, arr, 1, _lib.TC_OZAKI_I8)
    assert tune == (fft - up(8 * 3 * 6 * 64 * 64)) // 3 + up(8 * 3 * 6 * 64 * 64) + W
    # the backward recomputes W on every route
    back = L.tc_workspace_bytes(_lib.TC_OP_TEI_GRAM_BACKWARD, arr, 1, _lib.TC_OZAKI_I8)
    assert back >= W


def test_noalloc_rejects_before_any_device_call(L):
    """tc_tei_gram_noalloc validates like tc_tei_gram and rejects a problem
    beyond its static scratch with TC_ERR_WORKSPACE before touching a device
    (this runs without a GPU)."""
    big = (_lib.TcInstance * 1)(_inst(n=4096, R_f=1024, R_N=32))
    need = L.tc_workspace_bytes(_lib.TC_OP_TEI_GRAM, big, 1, _lib.TC_FP64)
    assert need > _lib.TC_NOALLOC_SCRATCH_BYTES
    assert L.tc_tei_gram_noalloc(big, 1, _lib.TC_FP64, None) == _lib.TC_ERR_WORKSPACE
    for kw in (dict(n=0), dict(R_f=0), dict(null="J"), dict(null="c")):
        bad = (_lib.TcInstance * 1)(_inst(**kw))
        assert L.tc_tei_gram_noalloc(bad, 1, _lib.TC_FP64, None) == _lib.TC_ERR_INVALID_ARG
    ok = (_lib.TcInstance * 1)(_inst())
    assert L.tc_tei_gram_noalloc(ok, 0, _lib.TC_FP64, None) == _lib.TC_ERR_INVALID_ARG
    assert L.tc_tei_gram_noalloc(ok, 1, 42, None) == _lib.TC_ERR_INVALID_ARG
    assert L.tc_tei_gram_noalloc(None, 1, _lib.TC_FP64, None) == _lib.TC_ERR_INVALID_ARG


def test_batch_route_table(L):
    """Built-in batch route (fork-join), per-batch entries, and the argument
    checks."""
    R = _lib.BATCH_ROUTES
    insts = (_lib.TcInstance * 3)(_inst(n=512, R_f=40), _inst(n=1024, R_f=300), _inst(n=64))
    other = (_lib.TcInstance * 3)(_inst(n=512, R_f=41), _inst(n=1024, R_f=300), _inst(n=64))
    assert L.tc_batch_tune_get(insts, 3, _lib.TC_OZAKI_I8) == R["fork_join"]
    assert L.tc_batch_tune_get(insts, 3, _lib.TC_FP64) == R["fork_join"]
    assert L.tc_batch_tune_get(insts, 1, _lib.TC_OZAKI_I8) == R["fork_join"]  # one instance
    try:
        assert L.tc_batch_tune_set(insts, 3, _lib.TC_OZAKI_I8, R["queue_k2"]) == _lib.TC_OK
        assert L.tc_batch_tune_get(insts, 3, _lib.TC_OZAKI_I8) == R["queue_k2"]
        # another batch (one R_f differs) keeps the built-in route
        assert L.tc_batch_tune_get(other, 3, _lib.TC_OZAKI_I8) == R["fork_join"]
        assert L.tc_batch_tune_get(insts, 2, _lib.TC_OZAKI_I8) == R["fork_join"]
    finally:
        assert L.tc_batch_tune_set(insts, 3, _lib.TC_OZAKI_I8, R["auto"]) == _lib.TC_OK
    assert L.tc_batch_tune_get(insts, 3, _lib.TC_OZAKI_I8) == R["fork_join"]
    assert L.tc_batch_tune_set(insts, 3, _lib.TC_FP64, R["queue"]) == _lib.TC_ERR_UNSUPPORTED
    assert L.tc_batch_tune_set(insts, 3, _lib.TC_FP64, 9) == _lib.TC_ERR_INVALID_ARG
    assert L.tc_batch_tune_set(insts, 0, _lib.TC_FP64, 1) == _lib.TC_ERR_INVALID_ARG
    assert L.tc_batch_tune_set(None, 1, _lib.TC_FP64, 1) == _lib.TC_ERR_INVALID_ARG
    bad = (_lib.TcInstance * 1)(_inst(n=0))
    assert L.tc_batch_tune_set(bad, 1, _lib.TC_FP64, 1) == _lib.TC_ERR_INVALID_ARG


def test_int8_batch_workspace_covers_the_queue(L):
    """An int8 batch's workspace covers both routes: the fork-join regions and
    the queue plan (every instance's own regions, the job table and one slab
    of Grams per mode for two K parts)."""
    insts = (_lib.TcInstance * 3)(_inst(n=512, R_f=40), _inst(n=1024, R_f=300), _inst(n=64))
    w8 = L.tc_workspace_bytes(_lib.TC_OP_TEI_GRAM, insts, 3, _lib.TC_OZAKI_I8)
    single = sum(L.tc_workspace_bytes(_lib.TC_OP_TEI_GRAM, (_lib.TcInstance * 1)(insts[i]), 1,
                                      _lib.TC_OZAKI_I8) for i in range(3))
    up = lambda x: (x + 255) // 256 * 256
    slabs = sum(3 * up(8 * I.R_N * I.R_f * I.R_f) for I in insts)
    assert w8 >= single + slabs
    tune = L.tc_workspace_bytes(_lib.TC_OP_AUTOTUNE, insts, 3, _lib.TC_OZAKI_I8)
    assert tune >= w8 + sum(up(8 * I.R_f * I.R_f) for I in insts)


def test_tuning_table(L):
    A = _lib.ALGORITHMS
    # built-in rule: FFT from 256 cells up (four-step beyond 4096), direct below
    assert L.tc_tune_get(128, 8, 20, _lib.TC_FP64) == A["direct"]
    assert L.tc_tune_get(1024, 8, 20, _lib.TC_FP64) == A["fft"]
    assert L.tc_tune_get(5000, 8, 20, _lib.TC_FP64) == A["fft"]
    assert L.tc_tune_get(65536, 8, 20, _lib.TC_FP64) == A["fft"]
    assert L.tc_tune_set(1024, 8, 20, _lib.TC_FP64, A["direct"]) == _lib.TC_OK
    assert L.tc_tune_get(1024, 8, 20, _lib.TC_FP64) == A["direct"]
    assert L.tc_tune_get(1024, 8, 20, _lib.TC_OZAKI_I8) == A["fft"]   # other key untouched
    assert L.tc_tune_set(1024, 8, 20, _lib.TC_FP64, A["auto"]) == _lib.TC_OK
    assert L.tc_tune_get(1024, 8, 20, _lib.TC_FP64) == A["fft"]
    assert L.tc_tune_set(5000, 8, 20, _lib.TC_FP64, A["fft"]) == _lib.TC_OK
    assert L.tc_tune_set(5000, 8, 20, _lib.TC_FP64, A["auto"]) == _lib.TC_OK
    assert L.tc_tune_set(0, 8, 20, _lib.TC_FP64, A["fft"]) == _lib.TC_ERR_INVALID_ARG
    assert L.tc_tune_set(64, 8, 20, _lib.TC_FP64, 9) == _lib.TC_ERR_INVALID_ARG


def test_autotune_rejects(L):
    arr = (_lib.TcInstance * 1)(_inst())
    assert L.tc_autotune(arr, 1, _lib.TC_FP64, None, 0, None, None) == _lib.TC_ERR_WORKSPACE
    assert L.tc_autotune(arr, 0, _lib.TC_FP64, None, 0, None, None) == _lib.TC_ERR_INVALID_ARG
    bad = (_lib.TcInstance * 1)(_inst(null="J"))
    assert L.tc_autotune(bad, 1, _lib.TC_FP64, None, 0, None, None) == _lib.TC_ERR_INVALID_ARG


def test_batch_workspace_is_per_branch(L):
    """A batch is spread over 4 branches, each with its own workspace region
    sized for its largest instance, whose modes run in turn (one mode region)."""
    insts = [_inst(n=64, R_f=8, R_N=4) for _ in range(6)]
    arr = (_lib.TcInstance * 6)(*insts)
    single = L.tc_workspace_bytes(_lib.TC_OP_TEI_GRAM, arr, 1, _lib.TC_FP64)
    six = L.tc_workspace_bytes(_lib.TC_OP_TEI_GRAM, arr, 6, _lib.TC_FP64)
    up = lambda x: (x + 255) // 256 * 256
    grams = up(8 * 3 * 4 * 8 * 8)
    assert (single - grams) % 3 == 0   # a lone instance has three mode regions
    one = grams + (single - grams) // 3
    assert six == 4 * up(one)
    two = L.tc_workspace_bytes(_lib.TC_OP_TEI_GRAM, arr, 2, _lib.TC_FP64)
    assert two == 2 * up(one)


def test_term_classes_rejects_bad_arguments(L):
    v = ctypes.c_void_p(0x1000)
    assert L.tc_term_classes(0, 4, v, v, None) == _lib.TC_ERR_INVALID_ARG
    assert L.tc_term_classes(64, 0, v, v, None) == _lib.TC_ERR_INVALID_ARG
    assert L.tc_term_classes(64, 4, None, v, None) == _lib.TC_ERR_INVALID_ARG
    assert L.tc_term_classes(64, 4, v, None, None) == _lib.TC_ERR_INVALID_ARG


def test_coulomb_workspace_and_rejects(L):
    D = _lib.TcDensity()
    D.R_f, D.R_rho, D.R_N = 10, 3, 4
    for l in range(3):
        D.n[l] = 100
    up = lambda x: (x + 255) // 256 * 256
    # H [3][R_N][R_f][R_rho], W [R_N][R_rho][n], FFT scratch of one mode
    # (twiddles [N], spectra of V [R_rho][N/2+1] and of the kernel [R_N][N/2+1])
    fft = up(16 * 256) + up(16 * 3 * 129) + up(16 * 4 * 129)
    assert L.tc_coulomb_workspace_bytes(ctypes.byref(D), _lib.TC_FP64) == \
        up(8 * 3 * 4 * 10 * 3) + up(8 * 4 * 3 * 100) + fft
    assert L.tc_coulomb_workspace_bytes(None, _lib.TC_FP64) == ctypes.c_size_t(-1).value
    bad = _lib.TcDensity()
    bad.R_f, bad.R_rho, bad.R_N = 10, 0, 4
    for l in range(3):
        bad.n[l] = 100
    assert L.tc_coulomb_workspace_bytes(ctypes.byref(bad), _lib.TC_FP64) == \
        ctypes.c_size_t(-1).value
    # null pointers, then a precision the route does not implement
    assert L.tc_coulomb(ctypes.byref(D), _lib.TC_FP64, None, 0, None) == _lib.TC_ERR_INVALID_ARG
    v = 0x1000
    D.c, D.d, D.Jd = v, v, v
    for l in range(3):
        D.p[l], D.U[l], D.V[l] = v, v, v
    assert L.tc_coulomb(ctypes.byref(D), _lib.TC_OZAKI_I8, None, 0, None) == \
        _lib.TC_ERR_UNSUPPORTED
    assert L.tc_coulomb(ctypes.byref(D), _lib.TC_FP64, None, 0, None) == _lib.TC_ERR_WORKSPACE
    assert L.tc_coulomb(ctypes.byref(D), 42, None, 0, None) == _lib.TC_ERR_INVALID_ARG


def test_density_fit_and_tei_cholesky_reject(L):
    v = ctypes.c_void_p(0x1000)
    R = ctypes.c_int(0)
    assert L.tc_density_fit_workspace_bytes(0, 5, 3) == ctypes.c_size_t(-1).value
    assert L.tc_density_fit_workspace_bytes(10, 5, 11) == ctypes.c_size_t(-1).value
    assert L.tc_density_fit(10, 5, v, 1e-6, 3, v, v, None, ctypes.byref(R), None, None, 0,
                            None) == _lib.TC_ERR_WORKSPACE
    assert L.tc_density_fit(10, 5, None, 1e-6, 3, v, v, None, ctypes.byref(R), None, None, 0,
                            None) == _lib.TC_ERR_INVALID_ARG
    assert L.tc_density_fit(10, 5, v, -1.0, 3, v, v, None, ctypes.byref(R), None, None, 0,
                            None) == _lib.TC_ERR_INVALID_ARG
    vp3 = (ctypes.c_void_p * 3)(0x1000, 0x1000, 0x1000)
    nul3 = (ctypes.c_void_p * 3)(0x1000, None, 0x1000)
    assert L.tc_tei_cholesky_workspace_bytes(10, 4, 3, 11) == ctypes.c_size_t(-1).value
    assert L.tc_tei_cholesky(10, 4, 3, v, vp3, vp3, 1e-6, 5, v, None, ctypes.byref(R), None,
                             None, 0, None) == _lib.TC_ERR_WORKSPACE
    assert L.tc_tei_cholesky(10, 4, 3, v, nul3, vp3, 1e-6, 5, v, None, ctypes.byref(R), None,
                             None, 0, None) == _lib.TC_ERR_INVALID_ARG
    assert L.tc_tei_cholesky(10, 4, 300, v, vp3, vp3, 1e-6, 5, v, None, ctypes.byref(R), None,
                             None, 0, None) == _lib.TC_ERR_INVALID_ARG



def test_lattice_rejects(L):
    v = ctypes.c_void_p(0x1000)
    vp3 = (ctypes.c_void_p * 3)(0x1000, 0x1000, 0x1000)
    nul3 = (ctypes.c_void_p * 3)(0x1000, None, 0x1000)
    Lok = (ctypes.c_int * 3)(3, 4, 2)
    Lbad = (ctypes.c_int * 3)(3, 0, 2)
    Lbig = (ctypes.c_int * 3)(3, 100000, 2)
    for n0, Ls, R_N, p, A in [(0, Lok, 5, vp3, vp3), (5, Lbad, 5, vp3, vp3),
                              (5, Lbig, 5, vp3, vp3), (5, Lok, 0, vp3, vp3),
                              (5, Lok, 5, nul3, vp3), (5, Lok, 5, vp3, nul3)]:
        assert L.tc_lattice_sum(n0, Ls, R_N, p, A, None) == _lib.TC_ERR_INVALID_ARG
    h = (ctypes.c_double * 3)(0.1, 0.1, 0.1)
    hbad = (ctypes.c_double * 3)(0.1, 0.0, 0.1)
    E = ctypes.c_double(0.0)
    assert L.tc_lattice_energy(5, Lok, 5, v, h, vp3, 1.0, ctypes.byref(E), v, 47,
                               None) == _lib.TC_ERR_WORKSPACE
    assert L.tc_lattice_energy(5, Lok, 5, v, hbad, vp3, 1.0, ctypes.byref(E), v, 48,
                               None) == _lib.TC_ERR_INVALID_ARG
    assert L.tc_lattice_energy(5, Lok, 5, None, h, vp3, 1.0, ctypes.byref(E), v, 48,
                               None) == _lib.TC_ERR_INVALID_ARG
    assert L.tc_lattice_energy(5, Lok, 5, v, h, nul3, 1.0, ctypes.byref(E), v, 48,
                               None) == _lib.TC_ERR_INVALID_ARG


def _nuclear_problem(M=2, pos=None, Z=None):
    import numpy as np
    P = _lib.TcNuclear()
    P.R_f, P.R_N, P.M = 16, 4, M
    v = 0x1000
    P.c, P.V = v, v
    for l in range(3):
        P.n[l] = 10
        P.h[l] = 0.1
        P.p[l], P.U[l] = v, v
    Zh = np.ones(M) if Z is None else np.asarray(Z, dtype=np.float64)
    ph = np.zeros((M, 3), dtype=np.int32) if pos is None else np.asarray(pos, dtype=np.int32)
    P.Z, P.pos = Zh.ctypes.data, ph.ctypes.data
    return P, (Zh, ph)


def test_nuclear_workspace_and_rejects(L):
    P, keep = _nuclear_problem()
    need = L.tc_nuclear_workspace_bytes(ctypes.byref(P))
    assert need >= 3 * 2 * 4 * 16 * 16 * 8
    assert L.tc_nuclear(ctypes.byref(P), None, 0, None) == _lib.TC_ERR_WORKSPACE
    for kw in [dict(pos=[[0, 0, 10], [1, 1, 1]]), dict(pos=[[0, -1, 0], [1, 1, 1]]),
               dict(Z=[1.0, float("nan")])]:
        Pb, keep2 = _nuclear_problem(**kw)
        assert L.tc_nuclear_workspace_bytes(ctypes.byref(Pb)) == ctypes.c_size_t(-1).value
        assert L.tc_nuclear(ctypes.byref(Pb), ctypes.c_void_p(0x1000), 1 << 30, None) == \
            _lib.TC_ERR_INVALID_ARG
    Pm, keep3 = _nuclear_problem(M=20000)
    assert L.tc_nuclear(ctypes.byref(Pm), ctypes.c_void_p(0x1000), 1 << 30, None) == \
        _lib.TC_ERR_INVALID_ARG
    P.h[1] = 0.0
    assert L.tc_nuclear(ctypes.byref(P), ctypes.c_void_p(0x1000), 1 << 30, None) == \
        _lib.TC_ERR_INVALID_ARG


def test_canonical_to_tucker_rejects(L):
    n = (ctypes.c_int * 3)(50, 40, 30)
    r = (ctypes.c_int * 3)(5, 6, 7)
    big = (ctypes.c_int * 3)(5, 49, 7)
    over_n = (ctypes.c_int * 3)(5, 6, 31)
    assert L.tc_canonical_to_tucker_workspace_bytes(n, 20, r) > 0
    assert L.tc_canonical_to_tucker_workspace_bytes(n, 20, big) == ctypes.c_size_t(-1).value
    assert L.tc_canonical_to_tucker_workspace_bytes(n, 20, over_n) == ctypes.c_size_t(-1).value
    assert L.tc_canonical_to_tucker_workspace_bytes(n, 4, r) == ctypes.c_size_t(-1).value
    v = ctypes.c_void_p(0x1000)
    vp3 = (ctypes.c_void_p * 3)(0x1000, 0x1000, 0x1000)
    nul3 = (ctypes.c_void_p * 3)(0x1000, None, 0x1000)
    args = lambda **kw: dict(dict(n=n, R=20, c=v, A=vp3, r=r, m_max=1, its=10, eps=0.0, Z=vp3,
                                  beta=v), **kw)

    def call(a, ws=v, ws_bytes=1 << 40):
        return L.tc_canonical_to_tucker(a["n"], a["R"], a["c"], a["A"], a["r"], a["m_max"],
                                        a["its"], a["eps"], a["Z"], a["beta"], None, None, ws,
                                        ws_bytes, None)
    assert call(args(), ws=None, ws_bytes=0) == _lib.TC_ERR_WORKSPACE
    assert call(args(its=0)) == _lib.TC_ERR_INVALID_ARG
    assert call(args(m_max=-1)) == _lib.TC_ERR_INVALID_ARG
    assert call(args(A=nul3)) == _lib.TC_ERR_INVALID_ARG
    assert call(args(eps=float("nan"))) == _lib.TC_ERR_INVALID_ARG
    assert call(args(eps=1.0)) == _lib.TC_ERR_INVALID_ARG
    assert call(args(Z=nul3)) == _lib.TC_ERR_INVALID_ARG
    # a sweep needs r_l <= r_m1 r_m2
    skew = (ctypes.c_int * 3)(1, 2, 7)
    assert call(args(r=skew)) == _lib.TC_ERR_INVALID_ARG
