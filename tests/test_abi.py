"""The C-ABI library loads and exports every entry point include/frntt.h
declares; argument errors that need no device are reported as documented."""
from __future__ import annotations

import ctypes
import os
import re

import pytest

import paper_2604_17808_amd as fr
from paper_2604_17808_amd import frntt as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "frntt.h")


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\**\s*([A-Za-z_][A-Za-z0-9_]*)\s*\(",
                       text, flags=re.M)
    return sorted(set(n for n in names if n not in ("if", "while")))


def test_header_declares_expected_calls():
    names = _declared_functions()
    for must in ("ntt_fwd", "ntt_inv", "ntt_coset", "ntt_coset_inv", "ntt_batch",
                 "frntt_ctx_create", "frntt_server_create", "frntt_tune"):
        assert must in names


def test_library_exports_every_declared_symbol():
    L = fr.lib()
    missing = [n for n in _declared_functions() if not hasattr(L, n)]
    assert not missing, missing
    # the binding knows every declared call, and nothing else
    assert set(B.SIGNATURES) == set(_declared_functions())


def test_strerror_and_sizes():
    L = fr.lib()
    assert L.frntt_strerror(0) == b"ok"
    assert L.frntt_strerror(B.EALIGN).startswith(b"data pointer")
    assert L.frntt_strerror(12345) == b"unknown status"
    assert L.frntt_scratch_bytes(10, 4) == 0            # one pass: in place
    assert L.frntt_scratch_bytes(20, 1) == 32 << 20     # two passes: one copy
    assert L.frntt_scratch_bytes(-1, 1) == 0
    assert L.frntt_prepare(None, 10, 0) == B.EINVAL
    assert L.frntt_table_bytes(None) == 0


def test_argument_errors_without_device():
    L = fr.lib()
    assert L.frntt_ctx_create(None, 0, 20, 0) == B.EINVAL
    h = ctypes.c_void_p()
    assert L.frntt_ctx_create(ctypes.byref(h), 0, 0, 0) == B.ERANGE
    assert L.frntt_ctx_create(ctypes.byref(h), 0, 29, 0) == B.ERANGE
    assert L.frntt_ctx_create(ctypes.byref(h), 0, 20, 1 << 7) == B.EINVAL
    assert not h.value
    assert L.ntt_fwd(None, None, 10, 1, None) == B.EINVAL
    assert L.ntt_transform(None, None, 10, 1, 0, None) == B.EINVAL
    assert L.frntt_set_algo(None, 1) == B.EINVAL
    assert L.frntt_ctx_destroy(None) == B.OK
    assert L.frntt_server_destroy(None) in (B.OK, B.EINVAL)
