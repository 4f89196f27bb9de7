"""The input interface on the GPU (tdse_resample_field): coarse driver
samples interpolated to the TDSE step by Fourier zero-padding, against the
oracle's rfft + direct trigonometric sum, for even and odd M (the split
Nyquist bin), M' = M (no padding), windows shorter than the padded period,
and a batch whose last row block is ragged."""
import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("batch,M,dtc,dt,nt", [
    (16, 400, 0.4, 0.05, 3199),      # r = 8, the whole padded period
    (13, 75, 0.3, 0.1, 224),         # odd M, r = 3, ragged row block
    (5, 90, 0.3, 0.3, 89),           # M' = M: the samples themselves
    (9, 128, 0.7, 0.07, 700),        # r = 10, first 701 of 1280 fine samples
    (3, 2000, 1.0, 0.04, 49999),     # a long record, M' = 50000
])
def test_resample_matches_oracle(lib, batch, M, dtc, dt, nt):
    import torch

    dev = torch.device("cuda:0")
    x = np.random.default_rng(M + batch).standard_normal((batch, M))
    from paper_2507_04115_amd.driver import resample_field

    fine = resample_field(torch.tensor(x, device=dev), dtc, dt, nt)
    assert fine.is_cuda and fine.is_contiguous() and fine.shape == (batch, nt + 1)
    ref = oracle.resample_field(x, dtc, dt, nt)
    err = np.max(np.abs(fine.cpu().numpy() - ref)) / np.max(np.abs(ref))
    print(f"  batch={batch} M={M} M'={round(M * dtc / dt)} nt={nt}: max rel {err:.2e}", flush=True)
    assert err < 1e-12
    # the coarse samples come back where the fine grid meets the coarse one
    r = round(dtc / dt)
    if abs(dtc / dt - r) < 1e-12:
        got = fine.cpu().numpy()[:, ::r]
        m = min(M, got.shape[1])
        assert np.max(np.abs(got[:, :m] - x[:, :m])) < 1e-12 * np.max(np.abs(x))


def test_resample_binding_rejects_short_buffers(lib):
    import torch

    dev = torch.device("cuda:0")
    x = torch.zeros(4, 64, dtype=torch.float64, device=dev)
    with pytest.raises(ValueError):
        lib.tdse_resample_field(x, 0.3, 0.1, 100, e_fine=torch.empty(4 * 101 - 1, dtype=torch.float64,
                                                                       device=dev))
    with pytest.raises(lib.TDSEError):
        lib.tdse_resample_field(x, 0.3, 0.07, 100)
