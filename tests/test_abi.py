"""The C-ABI library loads and exports every function the headers in include/
declare (no compute call: runs without a GPU)."""

import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = [os.path.join(ROOT, "include", h) for h in ("smc.h", "smc_fsv.h")]
LIB = os.path.join(ROOT, "paper_0905_2441_amd", "libsmcgpu.so")


def declared_functions():
    text = "\n".join(open(h).read() for h in HEADERS)
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?(?:int|char\s*\*|void)\s*\**\s*(\w+)\s*\(", text, flags=re.M)
    return sorted(set(names))


def test_header_declares_the_hot_path_calls():
    names = declared_functions()
    for required in ("smc_loglik", "smc_rwmh_move", "smc_reweight", "smc_ess",
                     "smc_resample_systematic", "pt_exchange"):
        assert required in names


def test_library_exports_every_declared_symbol():
    if not os.path.exists(LIB):
        pytest.fail("libsmcgpu.so is not built (run python paper_0905_2441_amd/build.py)")
    lib = ctypes.CDLL(LIB)
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_binding_signature_table_matches_header():
    from paper_0905_2441_amd import _lib
    assert sorted(_lib.SIGNATURES) == declared_functions()


def test_last_error_names_the_rejected_argument():
    """After an argument error the thread's last-error text says what was wrong
    (no GPU call is made: the checks run before any device work)."""
    from paper_0905_2441_amd import _lib
    lib = _lib.load()
    assert lib.smc_create(None, 0) == _lib.SMC_ERR_INVALID_ARG
    assert b"out" in lib.smc_last_error()
    assert lib.smc_rng_words(1, 0, 0, 0, 0, 0, None, None) == _lib.SMC_ERR_INVALID_ARG
    assert b"count" in lib.smc_last_error()
    assert lib.smc_set_slices(None, 4) == _lib.SMC_ERR_INVALID_ARG
    assert b"context" in lib.smc_last_error()


def test_invalid_arguments_are_rejected_before_any_gpu_work():
    """NULL context / arrays return SMC_ERR_INVALID_ARG without touching a device."""
    from paper_0905_2441_amd import _lib
    lib = _lib.load()
    assert lib.smc_loglik(None, None, None, 0, None, 0, 0, None, None) == _lib.SMC_ERR_INVALID_ARG
    assert lib.smc_reweight(None, None, None, 0, 0.0, None, None, None, None) == _lib.SMC_ERR_INVALID_ARG
    assert lib.smc_create(None, 0) == _lib.SMC_ERR_INVALID_ARG
    assert lib.smc_rng_words(1, 0, 0, 0, 0, 0, None, None) == _lib.SMC_ERR_INVALID_ARG
    assert lib.smc_destroy(None) == _lib.SMC_OK
