"""lbm_reduce_noalloc (the reductions with partials in a fixed library array,
no context, no allocation) against lbm_reduce_async, the entry point it is a
variant of: the 8 FP64 values agree bit for bit, on two calls in a row, the
second with a smaller field, with and without a reference field; and a call
changes no device allocation."""
import sys

import numpy as np
import pytest

from paper_1603_09577_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

KEYS = ("sum", "sumsq", "sum_d2", "sum_ref2", "min", "max", "nonfinite", "sum_absd")


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def test_noalloc_equals_reduce_async_two_calls():
    from paper_1603_09577_amd import lbm
    cases = ((300, 211), (77, 29))          # the second call has the smaller field
    outs = []
    for i, (nx, ny) in enumerate(cases):
        say(f"[gpu no-alloc] call {i}: {nx}x{ny}")
        sim = lbm.Lbm(W.spec_nonlinear_2d(nx, ny)).init(W.noise_field((ny, nx), 40 + i))
        sim.step(5)
        phi = sim.phi()
        if i == 1:
            phi.view(-1)[3] = float("nan")  # a non-finite value is counted, not summed
        ref = torch.tensor(W.noise_field((ny, nx), 50 + i), dtype=torch.float64, device="cuda")
        for r in (None, ref):
            want = sim.reduce_async(phi, r)
            got = lbm.reduce_noalloc(phi, r)
            torch.cuda.synchronize()
            assert torch.equal(got, want), (i, r is None, got.tolist(), want.tolist())
            p = phi.cpu().numpy().reshape(-1)
            fin = np.isfinite(p)
            assert got[6].item() == float((~fin).sum())
            assert abs(got[0].item() - p[fin].sum()) <= 1e-13 * abs(p[fin].sum())
            assert got[4].item() == p[fin].min() and got[5].item() == p[fin].max()
            outs.append(got.clone())


def test_noalloc_allocates_nothing_and_rejects():
    from paper_1603_09577_amd import lbm
    phi = torch.rand(1 << 20, dtype=torch.float64, device="cuda")
    out = torch.empty(8, dtype=torch.float64, device="cuda")
    sizes = (1 << 20, 1000, 1, 0)
    want = [phi[:n].sum().item() for n in sizes]    # torch's own work, before the measured window
    lbm.reduce_noalloc(phi, out=out)          # resolves the array's address once
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    got = []
    for n in sizes:
        lbm.reduce_noalloc(phi, out=out, n=n)
        torch.cuda.synchronize()
        got.append(out.tolist())
    assert torch.cuda.mem_get_info()[0] == free0
    for n, w, g in zip(sizes, want, got):
        if n == 0:
            assert g == [0.0, 0.0, 0.0, 0.0, float("inf"), float("-inf"), 0.0, 0.0]
        else:
            assert abs(g[0] - w) <= 1e-12 * max(1.0, w), (n, g[0], w)
    with pytest.raises(lbm.LbmError) as ei:
        lbm.reduce_noalloc(phi, out=out, n=1 << 31)
    assert ei.value.code == lbm.LBM_E_INVALID
