"""Host-side checks of the RNS lazy product's boundary: the library's moduli
are the ones the oracle derives from the same rule (consecutive primes below
2^31 - 2^24), and argument errors come back before any device work."""
from __future__ import annotations

import paper_2604_17808_amd as fr
from oracle import rns_lazy as R


def test_library_moduli_match_the_oracle():
    q, p = fr.rns_moduli()
    oq, op = R.moduli()
    assert q == oq and p == op


def test_argument_errors_without_a_device():
    L = fr.lib()
    assert L.frntt_rns_encode(None, None, None, 0, None) == fr.frntt.EINVAL
    assert L.frntt_rns_mul(None, None, None, None, 4, None) == fr.frntt.EINVAL
    assert L.frntt_rns_decode(None, None, None, 4, None) == fr.frntt.EINVAL
    assert L.frntt_mont_mul(None, None, None, None, 4, None) == fr.frntt.EINVAL
    assert L.frntt_rns_moduli(None, None) == fr.frntt.EINVAL


def test_wider_moduli_are_the_largest_primes_below_the_width():
    import sympy
    assert fr.FIELD_377 == sympy.prevprime(1 << 377)
    assert fr.FIELD_753 == sympy.prevprime(1 << 753)
    assert fr.FIELD_377 == R.width_params(377)[0] and fr.FIELD_753 == R.width_params(753)[0]


def test_field_create_argument_errors():
    import ctypes
    L = fr.lib()
    out = ctypes.c_void_p()
    assert L.frntt_rns_field_create(None, None, None, 8) == fr.frntt.EINVAL
    assert L.frntt_rns_field_create(ctypes.byref(out), None, None, 8) == fr.frntt.EINVAL
    assert L.frntt_rns_field_destroy(None) == 0
    assert L.frntt_rns_field_encode(None, None, None, 1, None) == fr.frntt.EINVAL
