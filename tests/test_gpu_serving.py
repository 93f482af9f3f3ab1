"""GPU tests of continuous-batching pricing: every result is the same alone and
in the mix, admission follows the memory budget, results match the oracle."""
import numpy as np
import pytest

import oracle
import paper_1310_2274_amd as P
from paper_1310_2274_amd import serving, synth
from gpu_helpers import assert_ylt_close, torch_cuda

pytestmark = pytest.mark.gpu

N, K, C = 20000, 200, 20000


@pytest.fixture(scope="module")
def setup():
    torch = torch_cuda()
    yet = synth.make_yet(N, K, C, seed=77)
    eng = P.Engine(0)
    yh = eng.load_yet(yet, C)
    rng = np.random.default_rng(5)
    layers = [synth.random_layer(rng, C, K, 12, 500, 3000, program_id=i % 3) for i in range(6)]
    yield torch, eng, yh, yet, layers
    eng.close()


def alone(torch, eng, yh, layer, seed, mode):
    desc = eng.load_layer(layer, C)
    out = torch.empty(N, device="cuda")
    P.ara_run_layer_ex(eng.ctx, yh, desc, mode, seed, 0, N, out)
    torch.cuda.synchronize()
    return out.cpu().numpy()


@pytest.mark.parametrize("mode", [P.MODE_PLAIN, P.MODE_MEAN])
def test_results_equal_alone_and_in_the_mix(setup, mode):
    torch, eng, yh, yet, layers = setup
    srv = serving.PricingServer(eng, yh, N, K, C, mode, hbm_budget_bytes=8 << 30, tile=3000)
    reqs = [serving.Request(i, lay, seed=100 + i) for i, lay in enumerate(layers)]
    # requests arrive while others are on the GPU: one joins every other tick
    pending = list(reqs)
    overlap = 0
    while pending or srv.waiting or srv.active:
        if pending and (srv.ticks % 2 == 0 or not (srv.active or srv.waiting)):
            srv.submit(pending.pop(0))
        srv.tick()
        overlap = max(overlap, len(srv.active))
    done = srv.finished
    assert len(done) == len(reqs)
    assert len({r.start for r in done}) == len(reqs) and overlap > 1
    for r in done:
        y_alone = alone(torch, eng, yh, r.layer, r.seed, mode)
        assert np.array_equal(r.ylt.cpu().numpy(), y_alone), f"request {r.req_id}"
        pml, tvar = P.ara_risk_measures(eng.ctx, y_alone, P.DEFAULT_RETURN_PERIODS)
        assert np.array_equal(pml, r.pml) and np.array_equal(tvar, r.tvar)
    # and through the open-loop driver
    srv2 = serving.PricingServer(eng, yh, N, K, C, mode, hbm_budget_bytes=8 << 30, tile=3000)
    reqs2 = [serving.Request(i, lay, seed=100 + i, arrival=0.001 * i) for i, lay in enumerate(layers)]
    done2 = srv2.run_open_loop(reqs2, keep_ylt=True)
    for r2 in done2:
        assert np.array_equal(r2.ylt.cpu().numpy(), next(r for r in done if r.req_id == r2.req_id).ylt.cpu().numpy())
    stats = serving.latency_stats(done2)
    assert stats["p99_s"] >= stats["p50_s"] > 0


def test_admission_waits_for_memory(setup):
    torch, eng, yh, yet, layers = setup
    need = [serving.request_bytes(l, C, N, P.MODE_PLAIN) for l in layers[:4]]
    budget = max(need) + 1                          # the largest request alone just fits
    srv = serving.PricingServer(eng, yh, N, K, C, P.MODE_PLAIN, hbm_budget_bytes=budget, tile=5000)
    reqs = [serving.Request(i, lay, seed=7 + i, arrival=0.0) for i, lay in enumerate(layers[:4])]
    peak = 0
    for r in reqs:
        srv.submit(r)
    while srv.waiting or srv.active:
        srv.tick()
        peak = max(peak, len(srv.active))
        assert srv.used <= budget
    assert peak >= 1 and srv.refusals > 0 and len(srv.finished) == 4
    # a request larger than the whole budget is refused outright
    tiny = serving.PricingServer(eng, yh, N, K, C, P.MODE_PLAIN, hbm_budget_bytes=min(need) // 2, tile=5000)
    tiny.submit(serving.Request(9, layers[0], seed=1))
    with pytest.raises(P.AraError) as ex:
        tiny.tick()
    assert ex.value.status == P.ARA_E_BUDGET


def test_served_request_matches_oracle(setup):
    torch, eng, yh, yet, layers = setup
    srv = serving.PricingServer(eng, yh, N, K, C, P.MODE_PLAIN, hbm_budget_bytes=8 << 30, tile=7000)
    r = serving.Request(0, layers[2], seed=31337, arrival=0.0)
    srv.run_open_loop([r], keep_ylt=True)
    trials = np.array([0, 1, 6999, 7000, 13999, N - 1])
    yo, g, _ = oracle.run_layer(layers[2], yet[trials], trials, C, 31337)
    assert_ylt_close(r.ylt.cpu().numpy()[trials].astype(np.float64), yo, g, "served request")


def test_cancel_and_deadline(setup):
    # a request cancelled while on the GPU and one past its deadline before
    # admission leave with no result and their memory released; the others'
    # results are unchanged
    torch, eng, yh, yet, layers = setup
    srv = serving.PricingServer(eng, yh, N, K, C, P.MODE_PLAIN, hbm_budget_bytes=8 << 30, tile=3000)
    reqs = [serving.Request(i, lay, seed=300 + i) for i, lay in enumerate(layers[:4])]
    reqs[3].deadline = 0.0
    for r in reqs:
        srv.submit(r)
    srv.tick()
    srv.tick()
    assert reqs[1].status == "active" and reqs[3].status == "timed_out"
    assert srv.cancel(1) and not srv.cancel(1) and not srv.cancel(99)
    while srv.waiting or srv.active:
        srv.tick()
    assert {r.req_id: r.status for r in srv.finished + srv.dropped} == \
        {0: "done", 1: "cancelled", 2: "done", 3: "timed_out"}
    assert srv.used == 0 and reqs[1].ylt is None and reqs[1].pml is None
    for r in srv.finished:
        assert np.array_equal(r.ylt.cpu().numpy(), alone(torch, eng, yh, r.layer, r.seed, P.MODE_PLAIN))
