"""The allocation-free PML/TVaR entry point (ara_risk_measures_noalloc) against
ara_risk_measures through the C ABI: identical results on two calls in a row,
the second on a smaller YLT, no device memory taken by the context, and the
argument checks."""
import numpy as np
import pytest

import oracle
import paper_1310_2274_amd as P
from gpu_helpers import torch_cuda

pytestmark = pytest.mark.gpu


def _ylt(torch, n, seed):
    rng = np.random.default_rng(seed)
    y = rng.lognormal(12, 2, n).astype(np.float32)
    y[rng.random(n) < 0.1] = 0.0                  # years below the aggregate retention
    y[rng.random(n) < 0.02] = np.float32(4e6)     # ties at an aggregate limit
    return y, torch.from_numpy(y).cuda()


def test_noalloc_matches_risk_measures_on_two_calls():
    torch = torch_cuda()
    with P.Engine(0) as eng:
        before = P.lib().ara_bytes_in_use(eng.ctx)
        cases = ((1_000_003, (10.0, 50.0, 100.0, 250.0, 1000.0, 1.0), 1), (4_099, (2.0, 10.0, 250.0), 2))
        results = []
        for n, rps, seed in cases:
            y, yd = _ylt(torch, n, seed)
            out = torch.full((2 * len(rps),), float("nan"), dtype=torch.float64, device="cuda")
            P.ara_risk_measures_noalloc(eng.ctx, yd, out, rps)
            torch.cuda.synchronize()
            results.append((y, yd, rps, out.cpu().numpy()))
        # the context took no device memory for these calls
        assert P.lib().ara_bytes_in_use(eng.ctx) == before
        for y, yd, rps, o in results:
            pml, tvar = P.ara_risk_measures(eng.ctx, yd, rps)
            assert np.array_equal(o[0::2], pml) and np.array_equal(o[1::2], tvar)
            po, to = oracle.risk_measures(y.astype(np.float64), rps)
            assert np.array_equal(pml, po)
            assert np.allclose(tvar, to, rtol=1e-12, atol=0)


def test_noalloc_second_context_same_device_and_errors():
    torch = torch_cuda()
    y, yd = _ylt(torch, 10_000, 3)
    rps = (10.0, 100.0)
    with P.Engine(0) as e1, P.Engine(0) as e2:
        o1 = torch.empty(4, dtype=torch.float64, device="cuda")
        o2 = torch.empty(4, dtype=torch.float64, device="cuda")
        P.ara_risk_measures_noalloc(e1.ctx, yd, o1, rps)
        torch.cuda.synchronize()
        P.ara_risk_measures_noalloc(e2.ctx, yd, o2, rps)
        torch.cuda.synchronize()
        assert torch.equal(o1, o2)
        out = torch.full((34,), -1.0, dtype=torch.float64, device="cuda")
        with pytest.raises(P.AraError) as ei:           # beyond the scratch's 16 return periods
            P.ara_risk_measures_noalloc(e1.ctx, yd, out, [10.0] * 17)
        assert ei.value.status == P.ARA_E_INVAL and "16" in ei.value.message
        with pytest.raises(P.AraError) as ei:           # host YLT
            P.ara_risk_measures_noalloc(e1.ctx, y, out, rps, n_trials=y.size)
        assert ei.value.status == P.ARA_E_INVAL
        with pytest.raises(P.AraError) as ei:           # floor(N / RP) < 1
            P.ara_risk_measures_noalloc(e1.ctx, yd, out, (20_000.0,))
        assert ei.value.status == P.ARA_E_RANGE
        torch.cuda.synchronize()
        assert bool((out == -1.0).all())                # nothing written on a refused call
        # still usable after the refusals
        P.ara_risk_measures_noalloc(e1.ctx, yd, o1, rps)
        torch.cuda.synchronize()
        assert torch.equal(o1, o2)
