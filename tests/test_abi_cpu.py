"""Host-side checks of the C ABI that need no GPU: the library loads, exports
every entry point declared in include/hlf.h, and rejects host-detectable bad
arguments before touching the device."""

import ctypes
import os
import re

import pytest

from paper_2103_00693_amd import hlf

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            src = open(os.path.join(ROOT, "include", fn)).read()
            src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
            names |= set(re.findall(r"\b(hlf_[a-z0-9_]+)\s*\(", src))
    return names


def test_header_declares_the_binding_names():
    assert declared_symbols() == set(hlf.EXPORTED)


def test_library_exports_every_declared_symbol():
    L = hlf.lib()
    for name in declared_symbols():
        assert hasattr(L, name), name


def test_scalar_helpers():
    L = hlf.lib()
    assert L.hlf_version() >> 16 == 1
    assert [L.hlf_words_for(n) for n in (1, 64, 65, 128, 129, 1024)] == [1, 1, 2, 2, 3, 16]
    assert "ERANGE" in hlf.status_string(hlf.HLF_ERANGE)


def _rec(n, null=None):
    W = (n + 63) // 64
    f = hlf._Factors(n, W, 8, 8, 8, 8, 8, 0)
    if null:
        setattr(f, null, 0)
    return f


@pytest.mark.parametrize("null", ["status", "rank", "pivots", "basis", "shift"])
def test_factor_rejects_null_record_members(null):
    L = hlf.lib()
    f = _rec(10, null)
    assert L.hlf_factor(ctypes.c_void_p(8), ctypes.byref(f), None) == hlf.HLF_EINVAL


def test_host_detected_errors():
    L = hlf.lib()
    good = _rec(10)
    assert L.hlf_factor(None, ctypes.byref(good), None) == hlf.HLF_EINVAL
    bad_n = _rec(10)
    bad_n.n = 0
    assert L.hlf_factor(ctypes.c_void_p(8), ctypes.byref(bad_n), None) == hlf.HLF_EINVAL
    big = _rec(10)
    big.n, big.words = 1025, 17
    assert L.hlf_factor(ctypes.c_void_p(8), ctypes.byref(big), None) == hlf.HLF_EINVAL
    wrong_w = _rec(100)
    wrong_w.words = 1
    assert L.hlf_factor(ctypes.c_void_p(8), ctypes.byref(wrong_w), None) == hlf.HLF_EINVAL
    assert L.hlf_factor_ex(ctypes.c_void_p(8), ctypes.byref(good), 4, None) == hlf.HLF_EINVAL  # unknown flag bit
    assert L.hlf_pack_dense(None, 4, ctypes.c_void_p(8), ctypes.c_void_p(8), None) == hlf.HLF_EINVAL
    assert L.hlf_pack_dense(ctypes.c_void_p(8), 0, ctypes.c_void_p(8), ctypes.c_void_p(8), None) == hlf.HLF_EINVAL
    assert L.hlf_pack_dense(ctypes.c_void_p(8), 1025, ctypes.c_void_p(8), ctypes.c_void_p(8), None) == hlf.HLF_EINVAL
    # word_bits must hold n, or be 64*W
    f20 = _rec(20)
    assert L.hlf_enumerate(ctypes.byref(f20), 0, 4, 8, ctypes.c_void_p(16), None) == hlf.HLF_EINVAL
    assert L.hlf_enumerate(ctypes.byref(f20), 0, 4, 16, ctypes.c_void_p(16), None) == hlf.HLF_EINVAL
    assert L.hlf_enumerate(ctypes.byref(f20), 0, 4, 128, ctypes.c_void_p(16), None) == hlf.HLF_EINVAL
    f100 = _rec(100)
    assert L.hlf_enumerate(ctypes.byref(f100), 0, 4, 64, ctypes.c_void_p(16), None) == hlf.HLF_EINVAL
    assert L.hlf_enumerate(ctypes.byref(f20), 0, 4, 32, None, None) == hlf.HLF_EINVAL
    # count == 0 is a no-op that succeeds without touching the device
    assert L.hlf_enumerate(ctypes.byref(f20), 0, 0, 32, None, None) == hlf.HLF_OK
    assert L.hlf_sample(ctypes.byref(f20), 1, 0, None, None, None) == hlf.HLF_OK
    assert L.hlf_sample(ctypes.byref(f20), 1, 5, None, None, None) == hlf.HLF_EINVAL
    assert L.hlf_enumerate_reduce(ctypes.byref(f20), 0, 4, 0, None, ctypes.c_void_p(8), None, None) == hlf.HLF_EINVAL
    assert L.hlf_enumerate_reduce(ctypes.byref(f20), 0, 4, 4, ctypes.c_void_p(8), ctypes.c_void_p(8), None, None) == hlf.HLF_EINVAL


def test_product_package_does_not_import_the_oracle():
    pkg = os.path.join(ROOT, "paper_2103_00693_amd")
    for dirpath, _, files in os.walk(pkg):
        for fn in files:
            if fn.endswith((".py", ".hip", ".cpp", ".h")):
                src = open(os.path.join(dirpath, fn)).read()
                assert "oracle" not in src.lower(), fn


def test_batch_host_validation():
    L = hlf._batch_lib()
    h = ctypes.c_void_p()
    ns = (ctypes.c_int32 * 3)(4, 0, 9)
    assert L.hlf_batch_create(3, ns, ctypes.byref(h)) == hlf.HLF_EINVAL
    ns2 = (ctypes.c_int32 * 1)(1025)
    assert L.hlf_batch_create(1, ns2, ctypes.byref(h)) == hlf.HLF_EINVAL
    assert L.hlf_batch_create(0, ns2, ctypes.byref(h)) == hlf.HLF_EINVAL
    assert L.hlf_batch_destroy(None) == hlf.HLF_OK
    assert L.hlf_batch_reduce(None, ctypes.c_void_p(8), 10, None, None) == hlf.HLF_EINVAL
    assert L.hlf_batch_graph_launch(None, None) == hlf.HLF_EINVAL


def test_host_detected_errors_of_order_and_verification_calls():
    L = hlf.lib()
    f20 = _rec(20)
    p = ctypes.c_void_p(16)
    # unknown flag bits and the word_bits rule of hlf_enumerate
    assert L.hlf_enumerate_ex(ctypes.byref(f20), 0, 4, 32, 2, p, None) == hlf.HLF_EINVAL
    assert L.hlf_enumerate_ex(ctypes.byref(f20), 0, 4, 16, hlf.HLF_ORDER_COUNTER, p, None) == hlf.HLF_EINVAL
    assert L.hlf_enumerate_ex(ctypes.byref(f20), 0, 4, 32, hlf.HLF_ORDER_COUNTER, None, None) == hlf.HLF_EINVAL
    # count = 0 enqueues nothing
    assert L.hlf_enumerate_ex(ctypes.byref(f20), 0, 0, 32, hlf.HLF_ORDER_COUNTER, None, None) == hlf.HLF_OK
    assert L.hlf_pair_stats(ctypes.byref(f20), None, p, None) == hlf.HLF_EINVAL
    assert L.hlf_pair_stats(ctypes.byref(f20), p, None, None) == hlf.HLF_EINVAL
    bad = _rec(20, "status")
    assert L.hlf_pair_stats(ctypes.byref(bad), p, p, None) == hlf.HLF_EINVAL
    # membership needs the kernel buffer of the record
    assert L.hlf_membership(ctypes.byref(f20), p, 3, p, None) == hlf.HLF_EINVAL
    with_kernel = _rec(20)
    with_kernel.kernel = 8
    assert L.hlf_membership(ctypes.byref(with_kernel), None, 3, p, None) == hlf.HLF_EINVAL
    assert L.hlf_membership(ctypes.byref(with_kernel), p, 3, None, None) == hlf.HLF_EINVAL
    assert L.hlf_membership(ctypes.byref(with_kernel), None, 0, None, None) == hlf.HLF_OK


def test_host_detected_errors_of_solve_dense():
    L = hlf.lib()
    p = ctypes.c_void_p(16)
    f20, f100 = _rec(20), _rec(100)
    # NULL A, n > 64, word size below n or not 16/32/64
    assert L.hlf_solve_dense(None, ctypes.byref(f20), 0, 8, 32, p, None) == hlf.HLF_EINVAL
    assert L.hlf_solve_dense(p, ctypes.byref(f100), 0, 8, 64, p, None) == hlf.HLF_EINVAL
    assert L.hlf_solve_dense(p, ctypes.byref(f20), 0, 8, 16, p, None) == hlf.HLF_EINVAL
    assert L.hlf_solve_dense(p, ctypes.byref(f20), 0, 8, 24, p, None) == hlf.HLF_EINVAL
    # misaligned begin (a multiple of 4 for uint32) or output, NULL output
    assert L.hlf_solve_dense(p, ctypes.byref(f20), 2, 8, 32, p, None) == hlf.HLF_EINVAL
    assert L.hlf_solve_dense(p, ctypes.byref(f20), 0, 8, 32, ctypes.c_void_p(24), None) == hlf.HLF_EINVAL
    assert L.hlf_solve_dense(p, ctypes.byref(f20), 0, 8, 32, None, None) == hlf.HLF_EINVAL
    # a NULL record member
    bad = _rec(20, "basis")
    assert L.hlf_solve_dense(p, ctypes.byref(bad), 0, 8, 32, p, None) == hlf.HLF_EINVAL


def test_server_rejects_bad_configurations_on_the_host():
    from paper_2103_00693_amd import serve

    L = serve._lib()
    h = ctypes.c_void_p()
    for bad in (dict(slots=0), dict(slots=65), dict(hbm_bytes=1000), dict(host_bytes=1000),
                dict(num_samples=0), dict(enum_max_rank=31), dict(cache_entries=-1)):
        cfg = dict(slots=2, hbm_bytes=1 << 24, host_bytes=1 << 24, num_samples=16, enum_max_rank=10,
                   cache_entries=4)
        cfg.update(bad)
        c = serve._Config(cfg["slots"], cfg["hbm_bytes"], cfg["host_bytes"], cfg["num_samples"],
                          cfg["enum_max_rank"], cfg["cache_entries"])
        assert L.hlf_server_create(ctypes.byref(c), ctypes.byref(h)) == hlf.HLF_EINVAL, bad
    assert L.hlf_server_create(None, ctypes.byref(h)) == hlf.HLF_EINVAL
    assert L.hlf_server_submit(None, None, 0) == hlf.HLF_EINVAL
    assert L.hlf_server_destroy(None) == hlf.HLF_OK
    assert L.hlf_server_now(None) == -1
