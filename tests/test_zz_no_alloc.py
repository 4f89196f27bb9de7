"""The allocation-free ground state (tdse_ground_state_noalloc, static device
workspace) against tdse_ground_state through the C-ABI: bitwise the same
state and energy, on two calls in a row (the second on a smaller grid, so
the workspace holds the first call's larger tables), and the regular
entry point still agrees afterwards."""
import ctypes

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _call(lib, name, p, n, psi):
    fn = getattr(lib.load(), name)
    e = ctypes.c_double()
    st = fn(ctypes.byref(p), n, 1.0, 20000, 1e-13, ctypes.c_void_p(psi.data_ptr()),
            ctypes.byref(e), None)
    assert st == 0, lib.load().tdse_last_error().decode()
    return e.value


def test_noalloc_ground_state_matches_allocating_entry_point(lib):
    import torch

    dev = torch.device("cuda:0")
    for n, dx, a in [(12000, 0.2, 1.1891671), (700, 0.3, 0.9), (16384, 0.15, 1.19)]:
        p = lib.make_params(dx, 0.05, a, 0)
        ref = torch.full((2 * n,), np.nan, dtype=torch.float64, device=dev)
        got = torch.full((2 * n,), np.nan, dtype=torch.float64, device=dev)
        e_ref = _call(lib, "tdse_ground_state", p, n, ref)
        e_got = _call(lib, "tdse_ground_state_noalloc", p, n, got)
        torch.cuda.synchronize()
        print(f"  n={n}: E {e_got:.15f} (allocating {e_ref:.15f})", flush=True)
        assert e_got == e_ref
        assert torch.equal(got, ref)
    # sizes beyond the supported range are refused before any launch
    p = lib.make_params(0.2, 0.05, 1.2, 0)
    big = torch.zeros(2 * 20000, dtype=torch.float64, device=dev)
    fn = lib.load().tdse_ground_state_noalloc
    e = ctypes.c_double()
    assert fn(ctypes.byref(p), 20000, 1.0, 100, 1e-13, ctypes.c_void_p(big.data_ptr()),
              ctypes.byref(e), None) == lib.TDSE_E_UNSUPPORTED
    assert "out of range" in lib.load().tdse_last_error().decode()
