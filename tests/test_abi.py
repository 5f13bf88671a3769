"""C-ABI checks that need no GPU: the library builds for gfx950, loads, exports
every entry point the header declares, and rejects bad arguments on the host."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "afqmc.h")


def _declared():
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"\b(afqmc_[a-z_]+)\s*\(", txt)))


@pytest.fixture(scope="module")
def lib():
    from paper_2505_18519_amd import afqmc as A
    if not os.path.exists(A.LIB_PATH):
        from paper_2505_18519_amd import build
        build.build()
    return A.load_library()


def test_header_declares_the_step_calls():
    names = _declared()
    for n in ["afqmc_overlap", "afqmc_green", "afqmc_force_bias", "afqmc_local_energy",
              "afqmc_metropolis_x", "afqmc_propagate", "afqmc_reorthogonalize"]:
        assert n in names


def test_library_exports_every_declared_symbol(lib):
    from paper_2505_18519_amd import afqmc as A
    for n in _declared():
        assert hasattr(lib, n), n
        assert n in A.EXPORTS, f"binding lacks {n}"


def test_host_side_validation(lib):
    from paper_2505_18519_amd import afqmc as A
    out = ctypes.c_void_p()
    assert lib.afqmc_create(None, 0, None, ctypes.byref(out)) == 1
    import numpy as np
    h = np.zeros((2, 2))
    dp = lambda a: a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    s = A.afqmc_system(200, 4, 8, 4, 2, 1, 0.1, dp(h), dp(h), dp(h), dp(h), 0.01, 10, 0, 0, 0.5, 0)
    assert lib.afqmc_create(ctypes.byref(s), 0, None, ctypes.byref(out)) == 2   # M > 160
    for M, N, P in ((64, 41, 2), (8, 9, 2), (0, 1, 2), (8, 2, 65), (8, 2, 0)):  # N > 40, N > M, ...
        s = A.afqmc_system(M, N, 8, 4, P, 1, 0.1, dp(h), dp(h), dp(h), dp(h), 0.01, 10, 0, 0, 0.5, 0)
        assert lib.afqmc_create(ctypes.byref(s), 0, None, ctypes.byref(out)) == 2, (M, N, P)
        assert not out.value
    s = A.afqmc_system(8, 2, 8, 4, 2, 7, 0.1, dp(h), dp(h), dp(h), dp(h), 0.01, 10, 0, 0, 0.5, 0)
    assert lib.afqmc_create(ctypes.byref(s), 0, None, ctypes.byref(out)) == 1   # hidden kind
    s = A.afqmc_system(8, 2, 8, 4, 2, 1, 0.1, dp(h), dp(h), dp(h), dp(h), 0.01, 10, 0, 0, 0.5, 4)
    assert lib.afqmc_create(ctypes.byref(s), 0, None, ctypes.byref(out)) == 1   # precision
    assert lib.afqmc_destroy(None) == 1
    assert lib.afqmc_green(None, 1, None, None, None, None) == 1


def test_binding_rejects_host_tensors():
    import torch
    from paper_2505_18519_amd import afqmc as A
    with pytest.raises(ValueError):
        A._ptr(torch.zeros(4, dtype=torch.float64), torch.float64, 4, "x")


def test_binding_constants_match_the_header():
    """Every AFQMC_* enumerator of include/afqmc.h has the binding constant of
    the same name (prefix dropped) and value."""
    import re
    from paper_2505_18519_amd import afqmc as A
    text = open(HEADER).read()
    found = dict((k, int(v)) for k, v in re.findall(r"\bAFQMC_([A-Z0-9_]+)\s*=\s*(\d+)", text))
    checked = 0
    for name, value in found.items():
        if name in ("OK",) or name.startswith("E_"):
            continue
        assert hasattr(A, name), name
        assert getattr(A, name) == value, (name, getattr(A, name), value)
        checked += 1
    assert checked >= 18
    defines = dict((k, int(v, 0)) for k, v in
                   re.findall(r"#define AFQMC_([A-Z0-9_]+) (0x[0-9a-fA-F]+|\d+)", text))
    for name in ("MLP_HIDDEN", "INIT_STEP", "MEASURE_STEP"):
        assert getattr(A, name) == defines[name], name
    m = re.search(r"#define AFQMC_STATIC_SCRATCH_BYTES \((\d+)u << (\d+)\)", text)
    assert m and A.STATIC_SCRATCH_BYTES == int(m.group(1)) << int(m.group(2))
