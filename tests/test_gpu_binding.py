"""The binding rejects buffers that are too small, on the wrong device or of
the wrong type with a ValueError/TypeError before anything reaches the
library: a short buffer would make the persistent kernels read or write past
its end."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def test_short_buffers_raise_before_any_launch(lib):
    import torch

    dev = torch.device("cuda:0")
    ns = [256, 300]
    nt = 20
    p = lib.make_params(0.2, 0.05, 1.2, nt)
    plan = lib.Plan(p, ns, adjoint_k=8)
    good = torch.zeros(len(ns), nt + 1, dtype=torch.float64, device=dev)
    short = torch.zeros(len(ns) * (nt + 1) - 1, dtype=torch.float64, device=dev)
    psi_short = torch.zeros(sum(ns) - 1, dtype=torch.complex128, device=dev)
    psi_short_f = torch.zeros(2 * sum(ns) - 2, dtype=torch.float64, device=dev)
    st_short = torch.zeros(len(ns) - 1, dtype=torch.int32, device=dev)
    acc = torch.empty_like(good)
    cases = [
        dict(E=short, psi0=None, accel=acc),
        dict(E=good, psi0=None, accel=short),
        dict(E=good, psi0=None, accel=acc, xexp=short),
        dict(E=good, psi0=None, accel=acc, norm=short),
        dict(E=good, psi0=psi_short, accel=acc),
        dict(E=good, psi0=psi_short_f, accel=acc),
        dict(E=good, psi0=None, accel=acc, psi_final=psi_short),
        dict(E=good, psi0=None, accel=acc, sys_status=st_short),
    ]
    for kw in cases:
        with pytest.raises(ValueError):
            lib.tdse_propagate_batch(plan, **kw)
    with pytest.raises(ValueError):
        lib.tdse_adjoint_batch(plan, good, None, short, acc)
    with pytest.raises(ValueError):
        lib.tdse_adjoint_batch(plan, good, None, good, short)
    with pytest.raises(ValueError):
        lib.tdse_adjoint_batch(plan, good, psi_short, good, acc)
    with pytest.raises(TypeError):
        lib.tdse_propagate_batch(plan, good.float(), None, acc)
    # nothing was launched with the bad buffers: a good call still works
    st = torch.full((len(ns),), -1, dtype=torch.int32, device=dev)
    lib.tdse_propagate_batch(plan, good, None, acc, None, None, None, st)
    torch.cuda.synchronize()
    assert np.all(st.cpu().numpy() == 0)
    assert np.all(np.isfinite(acc.cpu().numpy()))
    plan.close()
