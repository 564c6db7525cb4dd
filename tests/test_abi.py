"""The C-ABI library builds for gfx950, loads, and exports every entry point
declared in include/*.h; argument errors are reported without a GPU."""
import ctypes
import glob
import os
import re

import pytest

import paper_2512_18345_amd as P

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        src = open(h).read()
        src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
        names |= set(re.findall(r"\b(ckks_[a-z0-9_]+)\s*\(", src))
    return names


def test_header_declares_the_boundary():
    need = {"ckks_ntt", "ckks_intt", "ckks_modup", "ckks_moddown", "ckks_keyswitch",
            "ckks_hmult", "ckks_hrot", "ckks_rescale"}
    assert need <= _declared()


def test_library_exports_every_declared_symbol():
    lib = P.lib()
    for name in sorted(_declared()):
        assert hasattr(lib, name), name
        assert isinstance(getattr(lib, name), ctypes._CFuncPtr)


def test_binding_mirrors_every_entry_point():
    for name in _declared():
        if name == "ckks_last_error":
            continue
        assert callable(getattr(P, name)), name


def test_invalid_arguments_fail_without_touching_a_device():
    with pytest.raises(P.CkksError) as e:
        P.ckks_ctx_create(20, [1073479681], [1019478017], 1)
    assert e.value.code == -4  # logN out of range
    with pytest.raises(P.CkksError) as e:
        P.ckks_ctx_create(16, [1073479681, 1071513601], [1019478017], 3)  # alpha != k
    assert e.value.code == -1
    assert P.ckks_workspace_bytes(None, 3, 1) == 0
    with pytest.raises(P.CkksError):
        P.ckks_ntt(None, 0, 1, False, 0)


def test_server_and_batch_argument_errors_without_a_device():
    with pytest.raises(P.CkksError) as e:
        P.ckks_server_create([], 1 << 20, 4)
    assert e.value.code == -1
    with pytest.raises(P.CkksError):
        P.ckks_batch_create(None, [])
    for call in (lambda: P.ckks_batch_get_plan(None), lambda: P.ckks_batch_set_plan(None, 0, 1, 1),
                 lambda: P.ckks_batch_tune(None, 3, stream=0), lambda: P.ckks_batch_tune_log(None),
                 lambda: P.ckks_ctx_get_schedule(None), lambda: P.ckks_ctx_set_schedule(None),
                 lambda: P.ckks_ctx_tune(None, 4, stream=0)):
        with pytest.raises(P.CkksError) as e:
            call()
        assert e.value.code == -1
