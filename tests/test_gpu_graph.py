"""The ragged batch (plain FP64 and mixed precision) captured into a HIP
graph and replayed: every replay against the eager result and the oracle.

The batched entry point enqueues a fill kernel and one persistent kernel (no
memset, no synchronization), so it can be captured.  Inputs are restored
eagerly between replays (the plain factor works in place), with the eager
work and a synchronization between replays."""
from __future__ import annotations

import numpy as np
import pytest
import torch

import oracle
from paper_1907_05767_amd import ebv, inputs
from tests.gpu_util import case, dev, fwd_err, host

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("mixed", [False, True])
def test_batched_graph_replays(mixed):
    case(f"ragged batch hipGraph capture mixed={mixed}")
    ns, offA, A, offB, B = inputs.ragged(300, 1, 300, 0.5, 21)
    _, X_ref, _ = oracle.factor_solve_batched(ns, offA, A, offB, B)
    rb = ebv.RaggedBatch(ns, offA, offB)
    a0, b0 = dev(A), dev(B)
    tA, tB = a0.clone(), b0.clone()
    info = torch.zeros(rb.count, dtype=torch.int32, device="cuda")
    iters = torch.zeros(rb.count, dtype=torch.int32, device="cuda")
    ws = ebv.workspace(ebv.OP_BATCHED_MIXED if mixed else ebv.OP_BATCHED, ebv.F64, rb.totA, rb.totB, rb.count)
    # eager reference run (also warms up the library's device query)
    ebv.factor_solve_batched_(rb, tA, tB, mixed=mixed, info=info, iters=iters, ws=ws)
    torch.cuda.synchronize()
    eager_X, eager_LU = tB.clone(), tA.clone()
    assert fwd_err(host(eager_X), X_ref) <= 1e-12
    g = torch.cuda.CUDAGraph()
    tA.copy_(a0)
    tB.copy_(b0)
    torch.cuda.synchronize()
    with torch.cuda.graph(g):
        ebv.factor_solve_batched_(rb, tA, tB, mixed=mixed, info=info, iters=iters, ws=ws)
    torch.cuda.synchronize()
    for rep in range(4):
        tA.copy_(a0)
        tB.copy_(b0)
        info.fill_(-7)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert np.all(host(info) == 0), rep
        assert torch.equal(tB, eager_X), rep  # the same kernels on the same data: identical bits
        if not mixed:
            assert torch.equal(tA, eager_LU), rep
        else:
            assert torch.equal(tA, a0), rep  # A untouched
        # eager work between replays
        _ = (tB * 2.0).sum().item()
    Xh = host(tB)
    for k in range(len(ns)):
        b = slice(offB[k], offB[k] + int(ns[k]))
        assert fwd_err(Xh[b], X_ref[b]) <= 1e-12, k
