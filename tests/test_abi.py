"""The C-ABI library loads and exports what include/rewl.h declares, and its
host-side validation works without a GPU (no compute calls here)."""
import ctypes as C
import os
import re

import pytest

from paper_1402_2328_amd import rewl, workloads

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "rewl.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(rewl_[a-z0-9_]+)\s*\(", text)))


def test_header_and_binding_agree():
    decl = declared_functions()
    assert decl == sorted(rewl.EXPORTS)


def test_library_exports_every_declared_symbol():
    lib = rewl.lib()
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_strerror_names_codes():
    lib = rewl.lib()
    for code in range(-8, 1):
        assert lib.rewl_strerror(code).decode() == rewl.ERRORS[code]


@pytest.mark.parametrize("bad", [dict(L=1), dict(L=65), dict(n_windows=0), dict(walkers_per_window=0),
                                 dict(walkers_per_window=65), dict(flat=(6, 5)), dict(lnf_init=0.0),
                                 dict(overlap=(4, 4)), dict(n_windows=400), dict(schedule=2),
                                 dict(schedule=-1), dict(q=128, model=workloads.POTTS)])
def test_workspace_bytes_rejects_bad_parameters(bad):
    cfg = dict(workloads.ISING_L8)
    cfg.update(bad)
    assert rewl.rewl_workspace_bytes([workloads.rewl_params_of(cfg)]) == 0


def test_workspace_bytes_for_configs():
    for cfg in (workloads.ISING_L8, workloads.ISING_L32, workloads.POTTS_Q10_L20, workloads.POTTS_Q10_L20_FP32C):
        n = rewl.rewl_workspace_bytes([workloads.rewl_params_of(cfg)])
        assert 0 < n < 64 * 2 ** 20
    p = [workloads.rewl_params_of(workloads.ISING_L32)]
    assert rewl.rewl_workspace_bytes(p * 4) > 2 * rewl.rewl_workspace_bytes(p)


def test_mixed_precision_batch_rejected():
    a = dict(workloads.ISING_L8)
    b = dict(workloads.ISING_L8, precision=workloads.FP32C)
    assert rewl.rewl_workspace_bytes([workloads.rewl_params_of(a), workloads.rewl_params_of(b)]) == 0


def test_explicit_windows_validated():
    p = [workloads.rewl_params_of(workloads.ISING_L8)]
    good = [([0, 9, 18, 27], [37, 46, 55, 64])]
    assert rewl.rewl_workspace_bytes(p, good) > 0
    for bad in ([([0, 9, 18, 27], [37, 46, 55, 65])],        # beyond the range
                [([0, 40, 41, 42], [37, 46, 55, 64])],       # no overlap between 0 and 1
                [([0, 9, 9, 27], [37, 46, 55, 64])]):        # not increasing
        assert rewl.rewl_workspace_bytes(p, bad) == 0


def test_reserved_parameter_field_must_be_zero():
    p = workloads.rewl_params_of(workloads.ISING_L8)
    assert rewl.rewl_workspace_bytes([p]) > 0
    p.reserved = 1
    assert rewl.rewl_workspace_bytes([p]) == 0


def test_one_over_t_configs_lay_out():
    cfg = dict(workloads.ISING_L32, schedule=workloads.ONE_OVER_T, walkers_per_window=64)
    assert rewl.rewl_workspace_bytes([workloads.rewl_params_of(cfg)]) > 0


def test_measurement_probe_library_exports_its_entry_points():
    """libalurate.so (the VALU issue-cost and LDS-bandwidth probe behind the
    sweep's roofline) is built beside librewl.so and exports both calls;
    bad arguments are rejected before any GPU work."""
    path = os.path.join(os.path.dirname(rewl.__file__), "libalurate.so")
    lib = C.CDLL(path)
    for name in ("alu_rate", "lds_rate"):
        fn = getattr(lib, name)
        fn.argtypes = [C.c_int32, C.POINTER(C.c_double), C.c_int32]
        fn.restype = C.c_int
        out = (C.c_double * 5)()
        assert fn(0, out, 5) == -1
        assert fn(16, None, 5) == -1
        assert fn(16, out, 1) == -1
