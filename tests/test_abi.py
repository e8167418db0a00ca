"""CPU-side checks of the C ABI: the library loads, exports every function
include/cqr.h declares, and its host-only entry points behave (no device
work is issued by any call here: argument errors return before any HIP call)."""
import ctypes as C
import os
import re

import pytest

from paper_2405_04237_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = [os.path.join(ROOT, "include", f) for f in os.listdir(os.path.join(ROOT, "include"))
           if f.endswith(".h")]


def declared_functions():
    names = set()
    for h in HEADERS:
        text = open(h).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        for mt in re.finditer(r"^\s*(?:const\s+)?[a-z_0-9]+\s*\*?\s*(cqr_[a-z_0-9]+)\s*\(", text, re.M):
            names.add(mt.group(1))
    return names


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(_lib.LIB_PATH):
        pytest.fail("libcqr.so missing: run __graft_entry__.build() first")
    return _lib.lib()


def test_exports_every_declared_symbol(lib):
    names = declared_functions()
    assert {"cqr_factor", "cqr_factor_ex", "cqr_workspace_bytes", "cqr_get_info"} <= names
    for nm in names:
        assert hasattr(lib, nm), nm
    assert names <= set(_lib.SIGNATURES), names - set(_lib.SIGNATURES)


def test_header_constants_match_binding():
    text = open(os.path.join(ROOT, "include", "cqr.h")).read()
    assert re.search(r"#define CQR_MAX_PANEL (\d+)", text).group(1) == str(_lib.CQR_MAX_PANEL)
    for name, val in [("CQR_ERR_ARG", -1), ("CQR_ERR_HIP", -2), ("CQR_ERR_NOMEM", -3),
                      ("CQR_ERR_WORKSPACE", -4), ("CQR_ERR_UNSUPPORTED", -5)]:
        assert re.search(rf"{name} = {val}\b", text), name
        assert getattr(_lib, name) == val
    for name, val in [("CQR_SCHED_MOD", 0), ("CQR_SCHED_ORIG", 1), ("CQR_SCHED_SCQR3", 2)]:
        assert re.search(rf"{name} = {val}\b", text), name
        assert getattr(_lib, name.replace("CQR_", "")) == val


def test_workspace_and_panel_queries(lib):
    assert _lib.workspace_bytes(4096, 64, 16, _lib.SCHED_MOD) > 0
    assert _lib.workspace_bytes(10, 20, 4, _lib.SCHED_MOD) == 0  # m < n
    assert _lib.workspace_bytes(4096, 64, -1, _lib.SCHED_MOD) == 0
    assert _lib.workspace_bytes(4096, 64, 16, 7) == 0
    # ORIG keeps R1 and R2: more workspace than MOD
    assert (_lib.workspace_bytes(1 << 20, 256, 64, _lib.SCHED_ORIG)
            > _lib.workspace_bytes(1 << 20, 256, 64, _lib.SCHED_MOD))
    # a row count whose natural stride is a multiple of 1024 doubles adds the
    # staging copy (one shifted-stride m x n buffer) to the workspace
    extra = (_lib.workspace_bytes(8192, 96, 32, _lib.SCHED_MOD)
             - _lib.workspace_bytes(8208, 96, 32, _lib.SCHED_MOD))
    assert 8 * 8208 * 96 <= extra < 8 * 8208 * 96 + 512
    for n in (1, 16, 64, 100, 256, 1024):
        for s in (_lib.SCHED_MOD, _lib.SCHED_ORIG):
            b = _lib.default_panel(1 << 20, n, s)
            assert 1 <= b <= min(n, 128)  # the default stays within the LDS Cholesky
    # sCQR3 is one whole-matrix panel (b is ignored) and keeps R1, R2 like ORIG
    assert _lib.default_panel(1 << 20, 100, _lib.SCHED_SCQR3) == 100
    assert (_lib.workspace_bytes(1 << 20, 128, 0, _lib.SCHED_SCQR3)
            == _lib.workspace_bytes(1 << 20, 128, 16, _lib.SCHED_SCQR3)
            == _lib.workspace_bytes(1 << 20, 128, 128, _lib.SCHED_ORIG))
    assert _lib.status_string(0) == "success"
    assert "argument" in _lib.status_string(-1)


FAKE = C.c_void_p(4096)  # never dereferenced: every call below fails validation first


@pytest.mark.parametrize("m,n,b,lda,ptrs,sched,expect", [
    (10, 20, 4, 10, True, 0, _lib.CQR_ERR_ARG),        # m < n
    (100, 0, 4, 100, True, 0, _lib.CQR_ERR_ARG),       # n < 1
    (100, 10, 4, 99, True, 0, _lib.CQR_ERR_ARG),       # lda < m
    (100, 10, -2, 100, True, 0, _lib.CQR_ERR_ARG),     # b < 0
    (100, 10, 4, 100, False, 0, _lib.CQR_ERR_ARG),     # null pointers
    (100, 10, 4, 100, True, 3, _lib.CQR_ERR_ARG),      # bad schedule
    (1000, 300, 290, 1000, True, 0, _lib.CQR_ERR_UNSUPPORTED),  # b > CQR_MAX_PANEL
    (1000, 257, 0, 1000, True, 2, _lib.CQR_ERR_UNSUPPORTED),    # sCQR3 with n > CQR_MAX_PANEL
    (100, 10, -1, 100, True, 2, _lib.CQR_ERR_ARG),              # sCQR3 still rejects b < 0
])
def test_argument_errors(lib, m, n, b, lda, ptrs, sched, expect):
    p = FAKE if ptrs else None
    st = _lib.factor_ex(m, n, b, p, lda, p, p, None, sched, None, None, 0)
    assert st == expect
    if sched == 0:
        assert _lib.factor(m, n, b, p, lda, p, p, None) == expect


def test_misaligned_pointer_rejected(lib):
    odd = C.c_void_p(4096 + 4)
    assert _lib.factor_ex(100, 10, 4, odd, 100, FAKE, FAKE, None, 0, None, None, 0) == _lib.CQR_ERR_ARG


def test_small_workspace_rejected(lib):
    need = _lib.workspace_bytes(100, 10, 4, 0)
    ws = C.c_void_p(1 << 20)
    st = _lib.factor_ex(100, 10, 4, FAKE, 100, FAKE, FAKE, None, 0, FAKE, ws, need - 1)
    assert st == _lib.CQR_ERR_WORKSPACE


def test_batched_plan_argument_errors(lib):
    """cqr_plan_batched validates every shape before touching the device."""
    with pytest.raises(_lib.CqrError) as e:
        _lib.plan_batched([100, 50], [10, 60], None, _lib.SCHED_MOD)   # m < n
    assert e.value.status == _lib.CQR_ERR_ARG
    with pytest.raises(_lib.CqrError) as e:
        _lib.plan_batched([1000], [200], None, _lib.SCHED_MOD)         # n > 128
    assert e.value.status == _lib.CQR_ERR_UNSUPPORTED
    with pytest.raises(_lib.CqrError) as e:
        _lib.plan_batched([1000], [100], [64], _lib.SCHED_MOD)         # b > 32
    assert e.value.status == _lib.CQR_ERR_UNSUPPORTED
    with pytest.raises(_lib.CqrError) as e:
        _lib.plan_batched([1000], [100], None, _lib.SCHED_ORIG)        # MOD only
    assert e.value.status == _lib.CQR_ERR_UNSUPPORTED
    with pytest.raises(_lib.CqrError) as e:
        _lib.plan_batched([1000], [100], [-1], _lib.SCHED_MOD)
    assert e.value.status == _lib.CQR_ERR_ARG
    with pytest.raises(_lib.CqrError) as e:
        _lib.plan_batched([(1 << 33) + 1], [16], None, _lib.SCHED_MOD)  # rows past 2^33
    assert e.value.status == _lib.CQR_ERR_UNSUPPORTED
    assert _lib.lib().cqr_factor_batched(None, FAKE, FAKE, FAKE, FAKE, FAKE, None) == _lib.CQR_ERR_ARG


@pytest.mark.parametrize("args,expect", [
    ((0, 100, 10, FAKE, None, 100, 1000, FAKE, FAKE, FAKE, FAKE), _lib.CQR_ERR_ARG),  # batch < 1
    ((1, 5, 10, FAKE, None, 100, 1000, FAKE, FAKE, FAKE, FAKE), _lib.CQR_ERR_ARG),    # m < n
    ((2, 100, 10, FAKE, None, 100, 999, FAKE, FAKE, FAKE, FAKE), _lib.CQR_ERR_ARG),   # stride < lda n
    ((1, 100, 10, None, None, 100, 1000, FAKE, FAKE, FAKE, FAKE), _lib.CQR_ERR_ARG),  # no Q and no A
    ((1, 100, 10, FAKE, None, 100, 1000, None, FAKE, FAKE, FAKE), _lib.CQR_ERR_ARG),  # no R
    ((1, 1000, 257, FAKE, None, 1000, 257000, FAKE, FAKE, FAKE, FAKE), _lib.CQR_ERR_UNSUPPORTED),
])
def test_backward_argument_errors(lib, args, expect):
    bsz, m, n, q, a, lda, stride, r, dq, dr, da = args
    ws = C.c_void_p(1 << 20)
    st = _lib.backward_batched(bsz, m, n, q, a, lda, stride, r, dq, dr, da, None, ws, 1 << 30)
    assert st == expect


def test_backward_workspace_query(lib):
    assert _lib.backward_workspace_bytes(262144, 128, 1) > 0
    assert _lib.backward_workspace_bytes(32768, 64, 64) > _lib.backward_workspace_bytes(32768, 64, 1)
    assert _lib.backward_workspace_bytes(10, 20, 1) == 0


def test_noalloc_argument_errors(lib):
    """cqr_factor_noalloc validates before it touches the device: the usual
    argument errors, a missing info word, and sizes whose workspace exceeds
    its fixed array."""
    f = _lib.factor_noalloc
    assert f(10, 20, 4, FAKE, 10, FAKE, FAKE, 0, FAKE, None) == _lib.CQR_ERR_ARG     # m < n
    assert f(100, 10, 4, None, 100, FAKE, FAKE, 0, FAKE, None) == _lib.CQR_ERR_ARG   # null A
    assert f(100, 10, 4, FAKE, 100, FAKE, FAKE, 0, None, None) == _lib.CQR_ERR_ARG   # no info
    assert f(100, 10, 4, FAKE, 100, FAKE, FAKE, 9, FAKE, None) == _lib.CQR_ERR_ARG   # schedule
    big = (1 << 22, 1024, 128)
    assert _lib.workspace_bytes(*big, _lib.SCHED_MOD) > _lib.CQR_NOALLOC_SCRATCH_BYTES
    assert f(*big[:3], FAKE, big[0], FAKE, FAKE, 0, FAKE, None) == _lib.CQR_ERR_WORKSPACE
    # the limit is the in-place workspace: an aliasing lda adds no staging room
    m, n, b = 1 << 16, 64, 32
    assert _lib.workspace_bytes(m, n, b, 0) <= _lib.CQR_NOALLOC_SCRATCH_BYTES
    text = open(os.path.join(ROOT, "include", "cqr.h")).read()
    assert re.search(r"#define CQR_NOALLOC_SCRATCH_BYTES \(\(size_t\)128 << 20\)", text)


@pytest.mark.parametrize("ut,pt", [(-1, 0), (5, 0), (0, -1), (0, 5)])
def test_tile_option_errors(lib, ut, pt):
    """Kernel-variant options outside enum cqr_tile are argument errors."""
    st = _lib.factor_ex(100, 10, 4, FAKE, 100, FAKE, FAKE, None, 0, None, None, 0,
                        update_tile=ut, proj_tile=pt)
    assert st == _lib.CQR_ERR_ARG


def test_tile_constants_match_header():
    text = open(os.path.join(ROOT, "include", "cqr.h")).read()
    for name, val in _lib.TILES.items():
        assert re.search(rf"CQR_TILE_{name.upper()} = {val}\b", text), name
