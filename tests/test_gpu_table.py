"""GPU tests of the table mode: section 3.3's inverse Beta read from a
per-entry table (seventeen FP32 Hermite knots per side of t_s around the
leading-term asymptote, built in FP64), the third sampling form beside the
exact solve and the surrogate.  Against the FP64 oracle its per-draw error is
bounded (relative 2e-4, absolute 2e-5 in x); every term and clamp of the method
is 1-Lipschitz, so a trial's year loss moves by at most 2e-4 of its gross."""
import math

import numpy as np
import pytest

import oracle
import paper_1310_2274_amd as P
from paper_1310_2274_amd import synth
from gpu_helpers import ABS_TOL, gpu_ylt, oracle_ylt, torch_cuda

pytestmark = pytest.mark.gpu

TAB_REL = 2e-4        # per-draw relative error bound of the tabulated inverse
TAB_ABS = 2e-5        # per-draw absolute error bound in x (the loss over max_l)


@pytest.fixture(scope="module")
def eng():
    torch_cuda()
    e = P.Engine(0)
    yield e
    e.close()


def _grid(n, lo, hi, seed):
    rng = np.random.default_rng(seed)
    a = np.exp(rng.uniform(math.log(lo), math.log(hi), n))
    b = np.exp(rng.uniform(math.log(lo), math.log(hi), n))
    u = (2 * rng.integers(0, 2 ** 23, n) + 1) * 2.0 ** -24
    return a, b, u


def _assert_table_close(y, yo, g, what):
    tol = TAB_REL * g + ABS_TOL
    err = np.abs(np.asarray(y, np.float64) - yo)
    assert np.all(err <= tol), (what, int(np.sum(err > tol)), float(np.max(err - tol)))


@pytest.mark.parametrize("lo,hi,seed", [(0.2, 50.0, 1), (1e-3, 40.0, 2)])
def test_table_inverse_per_draw_accuracy(eng, lo, hi, seed):
    a, b, u = _grid(20000, lo, hi, seed)
    a[:3], b[:3], u[:3] = [1, 1, 2], [3, 1, 1], [0.5, 0.3, 0.25]      # closed forms below
    x = P.ara_beta_quantile_table(eng.ctx, a, b, u)
    xo = oracle.beta_inc_inv_vec(u, a, b, threads=0)
    assert x[0] == pytest.approx(1 - 0.5 ** (1 / 3), rel=TAB_REL)
    assert x[1] == pytest.approx(0.3, rel=TAB_REL)
    assert x[2] == pytest.approx(0.5, rel=TAB_REL)
    assert np.all(np.abs(x - xo) <= TAB_ABS), np.max(np.abs(x - xo))
    visible = xo > 1e-30
    rel = np.abs(x[visible] - xo[visible]) / xo[visible]
    assert np.all(rel <= TAB_REL), rel.max()
    assert np.all((x >= 0) & (x <= 1))


def test_table_inverse_paper_scale_parameters(eng):
    rng = np.random.default_rng(4)
    n = 20000
    mu = rng.lognormal(10, 1.5, n)
    sd = mu * rng.uniform(0.5, 1.5, n)
    mx = mu * rng.uniform(3, 10, n)
    ab = np.array([oracle.beta_params(m, s, x)[:2] for m, s, x in zip(mu, sd, mx)])
    u = (2 * rng.integers(0, 2 ** 23, n) + 1) * 2.0 ** -24
    x = P.ara_beta_quantile_table(eng.ctx, ab[:, 0], ab[:, 1], u)
    xo = oracle.beta_inc_inv_vec(u, ab[:, 0], ab[:, 1])
    visible = xo > 1e-30
    rel = np.abs(x[visible] - xo[visible]) / xo[visible]
    assert rel.max() <= 1e-4 and np.quantile(rel, 0.99) <= 3e-5, (rel.max(), np.quantile(rel, 0.99))


def test_table_mode_tiny_workload_vs_oracle(eng):
    wl = synth.tiny()
    y, om, _ = gpu_ylt(eng, wl, P.MODE_TABLE, wl.seed, with_omax=True)
    yo, g, omo = oracle_ylt(wl, np.arange(wl.n_trials), oracle.MODE_PLAIN, wl.seed)
    _assert_table_close(y, yo, g, "table YLT")
    _assert_table_close(om, omo, g, "table max occurrence")
    # the same draws as the exact path: the two agree within the table's bound
    yp, _ = gpu_ylt(eng, wl, P.MODE_PLAIN, wl.seed)
    _assert_table_close(y, yp, g, "table vs plain")


@pytest.mark.parametrize("N,K,C,J,lo,hi,sc", [
    (67, 1, 50, 1, 10, 30, 0.0),          # one event per trial
    (130, 63, 400, 3, 50, 150, 0.6),      # ragged chunk, correlated std
    (33, 130, 200, 40, 30, 120, 0.0),     # many XELTs per event
])
def test_table_mode_ragged_shapes(eng, N, K, C, J, lo, hi, sc):
    wl = synth.custom(N, K, C, J, lo, hi, seed=N + K, sigma_c_frac=sc)
    y, _ = gpu_ylt(eng, wl, P.MODE_TABLE, 11)
    yo, g, _ = oracle_ylt(wl, np.arange(N), oracle.MODE_PLAIN, 11)
    _assert_table_close(y, yo, g, f"table {N}x{K}")


def test_table_mode_degenerate_and_infinite_terms(eng):
    wl = synth.custom(64, 40, 200, 4, 40, 80, seed=5)
    lay = wl.layers[0]
    lay.elts[0].sigma_i[::3] = 0.0                      # sigma = 0: the loss is the mean
    lay.elts[1].limit = math.inf
    lay.elts[2].share = 0.0
    lay.occ_limit = math.inf
    lay.agg_limit = math.inf
    y, _ = gpu_ylt(eng, wl, P.MODE_TABLE, 3)
    yo, g, _ = oracle_ylt(wl, np.arange(64), oracle.MODE_PLAIN, 3)
    _assert_table_close(y, yo, g, "table degenerate/inf")


def test_table_mode_tiles_prepared_and_deterministic(eng):
    torch = torch_cuda()
    wl = synth.portfolio(n_layers=2, n_trials=1500)
    yh = eng.load_yet(wl.yet(), wl.catalog_size)
    hs = [P.ara_prepare_layer(eng.ctx, eng.load_layer(l, wl.catalog_size), P.MODE_TABLE) for l in wl.layers]
    ref = None
    for wpb in (1, 2, 4, 8):
        P.ara_set_trial_tile(eng.ctx, P.MODE_TABLE, wpb)
        outs = [torch.empty(wl.n_trials, device="cuda") for _ in hs]
        P.ara_run_prepared(eng.ctx, yh, hs, [5, 6], 0, wl.n_trials, outs)
        torch.cuda.synchronize()
        got = torch.stack(outs).cpu().numpy()
        if ref is None:
            ref = got
        assert np.array_equal(got, ref), wpb
    single = torch.empty(wl.n_trials, device="cuda")
    P.ara_run_layer_ex(eng.ctx, yh, eng.load_layer(wl.layers[1], wl.catalog_size), P.MODE_TABLE, 6, 0,
                       wl.n_trials, single)
    torch.cuda.synchronize()
    assert np.array_equal(single.cpu().numpy(), ref[1])
    for h in hs:
        P.ara_free_layer(eng.ctx, h)
    P.ara_set_trial_tile(eng.ctx, P.MODE_TABLE, 1)


def test_table_mode_yelt_and_occurrence_outputs(eng):
    # the per-occurrence outputs of the table mode: each occurrence's loss net of
    # XELT and occurrence terms, and the largest per trial
    torch = torch_cuda()
    wl = synth.custom(130, 63, 400, 3, 50, 150, seed=19)
    lay = wl.layers[0]
    yh = eng.load_yet(wl.yet(), wl.catalog_size)
    desc = eng.load_layer(lay, wl.catalog_size)
    t0, t1 = 17, 101
    y = torch.empty(t1 - t0, device="cuda")
    om = torch.empty(t1 - t0, device="cuda")
    ye = torch.full(((t1 - t0) * 63,), -7.0, device="cuda")
    P.ara_run_layer_yelt(eng.ctx, yh, desc, P.MODE_TABLE, 23, t0, t1, y, ye, om)
    torch.cuda.synchronize()
    trials = np.arange(t0, t1)
    yo, g, omo, yeo = oracle.run_layer(lay, wl.yet()[trials], trials, wl.catalog_size, 23, yelt=True)
    _assert_table_close(y.cpu().numpy(), yo, g, "table YLT")
    _assert_table_close(om.cpu().numpy(), omo, g, "table max occurrence")
    ye = ye.cpu().numpy().astype(np.float64).reshape(t1 - t0, 63)
    assert np.all(np.abs(ye - yeo) <= (TAB_REL * g + ABS_TOL)[:, None])
    assert np.array_equal(ye.max(axis=1), om.cpu().numpy().astype(np.float64))
