"""The C-ABI library loads and exports every symbol include/hrom.h declares (CPU only)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    src = open(os.path.join(ROOT, "include", "hrom.h")).read()
    return sorted(set(re.findall(r"^\s*(?:int|int32_t|int64_t|size_t|const char\*)\s+(hrom_\w+)\s*\(", src, re.M)))


def test_header_declares_the_four_calls():
    syms = declared_symbols()
    for s in ("hrom_eval", "hrom_condense", "hrom_update", "hrom_backward"):
        assert s in syms


def test_library_exports_every_declared_symbol():
    from paper_2306_02687_amd import binding
    lib = binding.load()
    missing = [s for s in declared_symbols() if not hasattr(lib, s)]
    assert not missing, missing
    assert set(binding.EXPORTED) == set(declared_symbols())


def test_strerror_and_invalid_arguments_without_gpu():
    """Argument validation happens before any HIP call."""
    from paper_2306_02687_amd import binding
    lib = binding.load()
    assert lib.hrom_strerror(0) == b"ok"
    assert b"invalid" in lib.hrom_strerror(-1)
    h = ctypes.c_void_p()
    # null cluster array / zero points / bad precision are rejected up front
    assert lib.hrom_plan_create(ctypes.byref(h), None, 1, 10, 0, 1) == -1
    arr = (binding._Cluster * 1)()
    arr[0] = binding._Cluster(8, 32, None, None, None, 0, 10)
    assert lib.hrom_plan_create(ctypes.byref(h), arr, 1, 10, 0, 1) == -1
    arr[0] = binding._Cluster(200, 32, 1, 1, 1, 0, 10)
    assert lib.hrom_plan_create(ctypes.byref(h), arr, 1, 10, 0, 1) == -5
    arr[0] = binding._Cluster(8, 32, 1, 1, 1, 0, 10)
    assert lib.hrom_plan_create(ctypes.byref(h), arr, 1, 11, 0, 1) == -1
    assert lib.hrom_plan_create(ctypes.byref(h), arr, 1, 10, 7, 1) == -1
    # the six-component condensation needs the objective split
    assert lib.hrom_plan_create(ctypes.byref(h), arr, 1, 10, 0, 16) == -5
    # J2 plasticity on the mixed path needs the split operands like any mixed plan
    assert lib.hrom_plan_create(ctypes.byref(h), arr, 1, 10, 1, 1 | 8) == -5
    # mixed precision without split operands misses the accuracy contract
    assert lib.hrom_plan_create(ctypes.byref(h), arr, 1, 10, 1, 1) == -5
    assert lib.hrom_plan_create(ctypes.byref(h), arr, 1, 10, 2, 1 | 4) == -5
    # empty inputs: no macro points at all, or a cluster that owns none
    assert lib.hrom_plan_create(ctypes.byref(h), arr, 1, 0, 0, 1) == -1
    arr[0] = binding._Cluster(8, 32, 1, 1, 1, 0, 0)
    assert lib.hrom_plan_create(ctypes.byref(h), arr, 1, 0, 0, 1) == -1
    # cluster slices must tile [0, N) in order
    two = (binding._Cluster * 2)()
    two[0] = binding._Cluster(8, 32, 1, 1, 1, 0, 4)
    two[1] = binding._Cluster(8, 32, 1, 1, 1, 5, 6)
    assert lib.hrom_plan_create(ctypes.byref(h), two, 2, 10, 0, 1) == -1
    two[1] = binding._Cluster(8, 32, 1, 1, 1, 4, 5)     # covers 9 of 10 points
    assert lib.hrom_plan_create(ctypes.byref(h), two, 2, 10, 0, 1) == -1
    assert lib.hrom_newton(None, None, None, None, 1e-10, 4, None, None, None, None, None) == -1
    assert lib.hrom_cauchy(None, None, None, None, None) == -1
    assert lib.hrom_eval(None, None, None, None, None, None, None, None, None, None, None) == -1
    assert lib.hrom_condense(None, None, None, None, None, None) == -1
    assert lib.hrom_update(None, None, 0.0, None, None, None) == -1
    assert lib.hrom_backward(None, None, None, None, None, None, None, None) == -1


def test_missing_library_fails_loudly(tmp_path):
    from paper_2306_02687_amd import binding
    with pytest.raises(binding.HromError):
        binding._lib_saved = binding._lib
        binding._lib = None
        try:
            binding.load(str(tmp_path / "nope.so"))
        finally:
            binding._lib = binding._lib_saved
