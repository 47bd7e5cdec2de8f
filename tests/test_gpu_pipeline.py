"""GPU parity: the host<->device transfer pipeline (transfers reported
separately in the paper, Table 3) gives, for every host-resident system,
the same factors and solution as the device-resident call, and the oracle's."""
from __future__ import annotations

import numpy as np
import pytest
import torch

import oracle
from paper_1907_05767_amd import ebv, inputs
from tests.gpu_util import case, dev, fwd_err, host

pytestmark = pytest.mark.gpu


def _pinned(a: np.ndarray, dtype=torch.float64) -> torch.Tensor:
    return torch.from_numpy(np.ascontiguousarray(a)).to(dtype).pin_memory()


@pytest.mark.parametrize("count", [1, 2, 5])
def test_pipeline_factor_solve(count):
    case(f"pipeline factor+solve count={count}")
    n, nrhs = 300, 3
    As = [inputs.dense(n, 0.5, 700 + s) for s in range(count)]
    Bs = [inputs.rhs(n, nrhs, 700 + s) for s in range(count)]
    ah = [_pinned(a) for a in As]
    bh = [_pinned(b) for b in Bs]
    info = torch.full((count,), 9, dtype=torch.int32, device="cuda")
    p = ebv.Pipeline(n, nrhs)
    p.run(ah, bh, info)
    p.synchronize()
    torch.cuda.synchronize()
    assert int(info.abs().max().item()) == 0
    for s in range(count):
        X_ref, LU_ref, _ = oracle.solve(As[s], Bs[s])
        assert fwd_err(bh[s].numpy(), X_ref) <= 1e-12
        # the device-resident call on the same system: same kernels, same bits
        ta, tb = dev(As[s]), dev(Bs[s])
        ebv.lu_factor_solve_(ta, tb)
        torch.cuda.synchronize()
        assert np.array_equal(bh[s].numpy(), host(tb))


def test_pipeline_factor_only_and_float():
    case("pipeline factor only; float")
    n = 200
    As = [inputs.dense(n, 0.5, 720 + s) for s in range(3)]
    ah = [_pinned(a) for a in As]
    p = ebv.Pipeline(n, 0)
    info = torch.zeros(3, dtype=torch.int32, device="cuda")
    p.run(ah, [], info)
    p.synchronize()
    assert int(info.abs().max().item()) == 0
    for s in range(3):
        LU_ref, _ = oracle.lu_factor(As[s])
        assert np.max(np.abs(ah[s].numpy() - LU_ref)) <= 1e-12
    # float systems through the same pipeline
    B = [inputs.rhs(n, 2, 730 + s) for s in range(3)]
    ah32 = [_pinned(a, torch.float32) for a in As]
    bh32 = [_pinned(b, torch.float32) for b in B]
    p32 = ebv.Pipeline(n, 2, torch.float32)
    p32.run(ah32, bh32)
    p32.synchronize()
    for s in range(3):
        X_ref, _, _ = oracle.solve(As[s], B[s])
        assert fwd_err(bh32[s].numpy(), X_ref) <= 1e-4
