"""GPU tests of the per-occurrence outputs: the year event loss table (each
occurrence's loss net of XELT and occurrence terms, section 2.4's
per-occurrence view) and the occurrence exceedance (largest occurrence loss
per trial, OEP) with its PML/TVaR, against the FP64 oracle."""
import numpy as np
import pytest

import oracle
import paper_1310_2274_amd as P
from paper_1310_2274_amd import synth
from gpu_helpers import ABS_TOL, REL_TOL, assert_ylt_close, torch_cuda

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def eng():
    torch_cuda()
    e = P.Engine(0)
    yield e
    e.close()


def run_yelt(eng, yh, desc, mode, seed, t0, t1, n_occ):
    torch = torch_cuda()
    y = torch.empty(t1 - t0, device="cuda")
    om = torch.empty(t1 - t0, device="cuda")
    ye = torch.full((n_occ,), -7.0, device="cuda")
    P.ara_run_layer_yelt(eng.ctx, yh, desc, mode, seed, t0, t1, y, ye, om)
    y2 = torch.empty(t1 - t0, device="cuda")
    om2 = torch.empty(t1 - t0, device="cuda")
    P.ara_run_layer_ex(eng.ctx, yh, desc, mode, seed, t0, t1, y2, om2)
    torch.cuda.synchronize()
    # asking for the YELT changes nothing else
    assert torch.equal(y, y2) and torch.equal(om, om2)
    return y.cpu().numpy().astype(np.float64), om.cpu().numpy().astype(np.float64), ye.cpu().numpy().astype(np.float64)


@pytest.mark.parametrize("mode", [P.MODE_MEAN, P.MODE_PLAIN])
@pytest.mark.parametrize("N,K,C,J,lo,hi,t0,t1", [
    (1000, 100, 10000, 2, 2000, 2000, 0, 1000),       # the tiny workload's shape
    (130, 63, 400, 3, 50, 150, 17, 101),               # ragged chunk, a trial sub-range
    (33, 130, 200, 40, 30, 120, 0, 33),                # several drain rounds per slot
])
def test_yelt_fixed_length_vs_oracle(eng, mode, N, K, C, J, lo, hi, t0, t1):
    wl = synth.custom(N, K, C, J, lo, hi, seed=N + J)
    lay = wl.layers[0]
    yh = eng.load_yet(wl.yet(), C)
    desc = eng.load_layer(lay, C)
    y, om, ye = run_yelt(eng, yh, desc, mode, 77, t0, t1, (t1 - t0) * K)
    trials = np.arange(t0, t1)
    yo, g, omo, yeo = oracle.run_layer(lay, wl.yet()[trials], trials, C, 77, mode=mode, yelt=True)
    assert_ylt_close(y, yo, g, "YLT")
    assert_ylt_close(om, omo, g, "max occurrence")
    ye = ye.reshape(t1 - t0, K)
    tol = (REL_TOL * g + ABS_TOL)[:, None]
    assert np.all(np.abs(ye - yeo) <= tol), np.max(np.abs(ye - yeo) - tol)
    # the YELT is what the year loss is made of: aggregate terms on its sum, its maximum
    S = ye.sum(axis=1)
    Y = np.minimum(np.maximum(S - np.float32(lay.agg_retention), 0.0), np.float32(lay.agg_limit))
    assert np.all(np.abs(Y - y) <= REL_TOL * g + ABS_TOL)
    assert np.array_equal(ye.max(axis=1), om)


def test_yelt_variable_length_trials(eng):
    rng = np.random.default_rng(21)
    N, C = 80, 300
    lens = rng.integers(0, 150, N)
    lens[[0, 7, 79]] = 0
    offs = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
    ev = rng.integers(0, C, offs[-1], dtype=np.int32)
    wl = synth.custom(N, 1, C, 6, 40, 120, seed=22)
    yh = eng.load_yet(ev, C, trial_offsets=offs)
    desc = eng.load_layer(wl.layers[0], C)
    t0, t1 = 5, 70
    for mode in (P.MODE_MEAN, P.MODE_PLAIN):
        y, om, ye = run_yelt(eng, yh, desc, mode, 9, t0, t1, int(offs[t1] - offs[t0]))
        for i in range(t0, t1):
            seg = ye[offs[i] - offs[t0]:offs[i + 1] - offs[t0]]
            if lens[i] == 0:
                assert y[i - t0] == 0.0 and om[i - t0] == 0.0
                continue
            yo, g, omo, yeo = oracle.run_layer(wl.layers[0], ev[offs[i]:offs[i + 1]].reshape(1, -1), [i], C, 9,
                                               mode=mode, yelt=True)
            assert_ylt_close(y[i - t0:i - t0 + 1], yo, g, f"trial {i}")
            assert np.all(np.abs(seg - yeo[0]) <= REL_TOL * g[0] + ABS_TOL), f"trial {i}"


def test_yelt_host_output_and_errors(eng):
    wl = synth.custom(64, 40, 500, 4, 50, 150, seed=3)
    yh = eng.load_yet(wl.yet(), wl.catalog_size)
    desc = eng.load_layer(wl.layers[0], wl.catalog_size)
    y = np.empty(64, dtype=np.float32)
    ye = np.empty(64 * 40, dtype=np.float32)
    P.ara_run_layer_yelt(eng.ctx, yh, desc, P.MODE_PLAIN, 1, 0, 64, y, ye)     # host buffers: synchronous
    yo, g, omo, yeo = oracle.run_layer(wl.layers[0], wl.yet(), np.arange(64), wl.catalog_size, 1, yelt=True)
    assert np.all(np.abs(ye.reshape(64, 40) - yeo) <= (REL_TOL * g + ABS_TOL)[:, None])
    with pytest.raises(P.AraError):
        P.ara_run_layer_yelt(eng.ctx, yh, desc, P.MODE_PLAIN, 1, 0, 64, y, None)


def test_occurrence_exceedance_risk_measures(eng):
    # OEP: PML/TVaR of the largest occurrence loss per trial, beside the AEP of the YLT
    torch = torch_cuda()
    wl = synth.custom(4000, 200, 5000, 5, 500, 1500, seed=31)
    yh = eng.load_yet(wl.yet(), wl.catalog_size)
    desc = eng.load_layer(wl.layers[0], wl.catalog_size)
    y = torch.empty(4000, device="cuda")
    om = torch.empty(4000, device="cuda")
    P.ara_run_layer_ex(eng.ctx, yh, desc, P.MODE_PLAIN, 5, 0, 4000, y, om)
    rps = [10, 50, 100, 250]
    pml, tvar = P.ara_risk_measures(eng.ctx, om, rps)
    yo, g, omo = oracle.run_layer(wl.layers[0], wl.yet(), np.arange(4000), wl.catalog_size, 5)
    po, to = oracle.risk_measures(omo, rps)
    # each order statistic moves by at most the largest per-trial error
    err = float(np.max(REL_TOL * g + ABS_TOL))
    assert np.all(np.abs(np.asarray(pml) - po) <= err) and np.all(np.abs(np.asarray(tvar) - to) <= err)
    assert np.all(np.asarray(pml) > 0)


# ------------------------------------------------------------ F1: aggregate increments per occurrence
def _w1_layer_gpu(eng, over):
    from conftest import golden
    w = golden("w1_terms.json")
    elts = []
    for e in w["elts"]:
        m = np.array(e["mean"], dtype=float)
        elts.append(synth.ELT(np.array(e["event_id"], dtype=np.int32), m, np.zeros_like(m), None, m * 4,
                              e["deductible"], e["limit"], e["share"]))
    t = dict(w["layer"])
    t.update(over)
    return w, synth.Layer(elts, t["occ_retention"], t["occ_limit"], t["agg_retention"], t["agg_limit"])


def test_increments_hand_worked(eng):
    # the hand-worked excess-of-loss fixture: YELT and its aggregate
    # increments, e.g. (0, 0, 400) for trial (a, b, c) but (200, 200, 0) for
    # (c, b, a) -- the same year loss, a different per-occurrence split
    from conftest import golden
    w = golden("w1_terms.json")
    for case in w["cases"]:
        _, lay = _w1_layer_gpu(eng, case["override"])
        yh = eng.load_yet(np.array([case["trial"]], dtype=np.int32), w["catalog_size"])
        desc = eng.load_layer(lay, w["catalog_size"])
        for mode in (P.MODE_MEAN, P.MODE_PLAIN):
            y = np.empty(1, dtype=np.float32)
            ye = np.empty(3, dtype=np.float32)
            P.ara_run_layer_yelt(eng.ctx, yh, desc, mode, 1, 0, 1, y, ye)
            inc = P.ara_yelt_increments(eng.ctx, yh, 0, 1, lay.agg_retention, lay.agg_limit, ye)
            assert y[0] == case["Y"] and list(ye) == case["yelt"]
            assert list(inc) == case["increments"], (case, list(inc))
        P.ara_free_yet(eng.ctx, yh)


@pytest.mark.parametrize("fixed", [True, False])
def test_increments_vs_oracle(eng, fixed):
    torch = torch_cuda()
    if fixed:
        wl = synth.tiny()
        lay = wl.layers[0]
        C, N = wl.catalog_size, wl.n_trials
        ev = wl.yet()
        yh = eng.load_yet(ev, C)
        offs = np.arange(N + 1, dtype=np.int64) * wl.events_per_trial
    else:
        rng = np.random.default_rng(41)
        N, C = 150, 400
        lens = rng.integers(0, 200, N)
        lens[[0, 3, 149]] = 0
        lens[10] = 130                                          # more than two chunks of 64
        offs = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
        ev = rng.integers(0, C, offs[-1], dtype=np.int32)
        wl = synth.custom(N, 1, C, 6, 60, 160, seed=42)
        lay = wl.layers[0]
        yh = eng.load_yet(ev, C, trial_offsets=offs)
    desc = eng.load_layer(lay, C)
    t0, t1 = (0, N) if fixed else (2, 140)
    n_occ = int(offs[t1] - offs[t0])
    y, om, ye = run_yelt(eng, yh, desc, P.MODE_PLAIN, 5, t0, t1, n_occ)
    inc_dev = P.ara_yelt_increments(eng.ctx, yh, t0, t1, lay.agg_retention, lay.agg_limit,
                                    torch.from_numpy(ye.astype(np.float32)).cuda())
    torch.cuda.synchronize()
    inc = inc_dev.cpu().numpy().astype(np.float64)
    inc_host = P.ara_yelt_increments(eng.ctx, yh, t0, t1, lay.agg_retention, lay.agg_limit, ye.astype(np.float32))
    assert np.array_equal(inc_host.astype(np.float64), inc)       # host and device buffers agree
    for i in range(t0, t1):
        lo, hi = int(offs[i] - offs[t0]), int(offs[i + 1] - offs[t0])
        if hi == lo:
            continue
        row = ev[offs[i]:offs[i + 1]].reshape(1, -1) if not fixed else ev[i:i + 1]
        yo, g, _, yeo = oracle.run_layer(lay, row, [i], C, 5, yelt=True)
        inco = oracle.yelt_increments(yeo, lay.agg_retention, lay.agg_limit)[0]
        # each running sum moves by at most the trial's YELT error, each A_k too
        tol = 2 * (REL_TOL * g[0] + ABS_TOL) + 1e-6 * abs(yo[0])
        assert np.all(np.abs(inc[lo:hi] - inco) <= tol), f"trial {i}"
        # the increments telescope to the year loss
        assert abs(inc[lo:hi].sum() - y[i - t0]) <= 1e-6 * max(1.0, y[i - t0]) + 1e-3
    # increments are order-dependent: with the trial's events reversed the
    # year loss stays (within rounding) but the split moves
    if fixed:
        assert np.any(inc != 0)


def test_increments_errors(eng):
    wl = synth.custom(8, 4, 50, 1, 5, 10, seed=3)
    yh = eng.load_yet(wl.yet(), 50)
    ye = np.zeros(32, dtype=np.float32)
    with pytest.raises(P.AraError) as e:
        P.ara_yelt_increments(eng.ctx, yh, 0, 9, 0.0, 1.0, ye)
    assert e.value.status == P.ARA_E_RANGE
    with pytest.raises(P.AraError) as e:
        P.ara_yelt_increments(eng.ctx, yh, 0, 8, -1.0, 1.0, ye)
    assert e.value.status == P.ARA_E_INVAL
