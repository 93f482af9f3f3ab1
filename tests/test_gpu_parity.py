"""GPU parity: the HIP path through the C ABI against the FP64 oracle on the
same seeded inputs (section 2.2 Algorithm 1, sections 3.1-3.3, section 2.4)."""
import math

import numpy as np
import pytest

import oracle
import paper_1310_2274_amd as P
from paper_1310_2274_amd import synth
from gpu_helpers import assert_ylt_close, gpu_ylt, oracle_ylt, torch_cuda

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def eng():
    torch_cuda()
    e = P.Engine(0)
    yield e
    e.close()


# ------------------------------------------------------------ A3: uniforms
def test_philox_uniforms_bit_exact(eng):
    rng = np.random.default_rng(1)
    n = 4096
    ctr = rng.integers(0, 2 ** 32, size=(n, 4), dtype=np.uint64).astype(np.uint32)
    ctr[:8] = [[0, 0, 0, 0], [0xFFFFFFFF] * 4, [1, 2, 3, 4], [5, 0, 0, 0], [0, 5, 0, 0], [0, 0, 5, 0],
               [0, 0, 0, 5], [7, 7, 7, 7]]
    for key in [(0, 0), (1310, 3), (0xFFFFFFFF, 0xFFFFFFFF), (1310, 0xFFFFFFFF)]:
        got = P.ara_philox_uniforms(eng.ctx, ctr, *key)
        want = np.array([oracle.uniform(oracle.philox4x32_10(c, key)[0]) for c in ctr], dtype=np.float64)
        assert np.array_equal(got.astype(np.float64), want)


def test_uniforms_match_the_oracle_streams(eng):
    # the exact counters the layer kernel uses: (trial, slot, j, 0) under (seed, program)
    ctr = np.array([[t, s, j, 0] for t in (0, 5, 799999) for s in (0, 1, 999) for j in (0, 15, 63)], dtype=np.uint32)
    got = P.ara_philox_uniforms(eng.ctx, ctr, 1310, 7)
    want = [oracle.u_indep(1310, 7, int(c[0]), int(c[1]), int(c[2])) for c in ctr]
    assert np.array_equal(got.astype(np.float64), np.array(want))
    ctr = np.array([[t, s, 0xFFFFFFFF, 1] for t in (0, 9) for s in (0, 3)], dtype=np.uint32)
    got = P.ara_philox_uniforms(eng.ctx, ctr, 1310, 0xFFFFFFFF)
    assert np.array_equal(got.astype(np.float64), [oracle.u_corr(1310, int(c[0]), int(c[1])) for c in ctr])


# ------------------------------------------------------------ A5/A6: inverse Beta
def _grid(n, lo, hi, seed):
    rng = np.random.default_rng(seed)
    a = np.exp(rng.uniform(math.log(lo), math.log(hi), n))
    b = np.exp(rng.uniform(math.log(lo), math.log(hi), n))
    u = (2 * rng.integers(0, 2 ** 23, n) + 1) * 2.0 ** -24
    return a, b, u


@pytest.mark.parametrize("lo,hi,seed", [(0.2, 50.0, 1), (1e-3, 40.0, 2), (3e-6, 35.0, 3)])
def test_beta_quantile_vs_oracle(eng, lo, hi, seed):
    a, b, u = _grid(20000, lo, hi, seed)
    # and the closed-form corners
    a[:4], b[:4], u[:4] = [1, 1, 0.5, 2], [3, 1, 0.5, 1], [0.5, 0.3, 0.3, 0.25]
    x = P.ara_beta_quantile(eng.ctx, a, b, u)
    xo = oracle.beta_inc_inv_vec(u, a, b, threads=0)
    assert x[0] == pytest.approx(1 - 0.5 ** (1 / 3), rel=1e-12)
    assert x[1] == pytest.approx(0.3, rel=1e-12)
    assert x[2] == pytest.approx(math.sin(math.pi * 0.3 / 2) ** 2, rel=1e-12)
    assert x[3] == pytest.approx(0.5, rel=1e-12)
    visible = xo > 1e-30                 # below this the loss is 0 in FP32 on both sides
    rel = np.abs(x[visible] - xo[visible]) / xo[visible]
    assert np.all(rel <= 1e-8), (rel.max(), np.argmax(rel))
    assert np.all(x[~visible] <= 1e-28)


def test_beta_quantile_paper_scale_parameters(eng):
    # (alpha, beta) from the section 3.3 moment matching of LogNormal losses
    rng = np.random.default_rng(4)
    n = 20000
    mu = rng.lognormal(10, 1.5, n)
    sd = mu * rng.uniform(0.5, 1.5, n)
    mx = mu * rng.uniform(3, 10, n)
    ab = np.array([oracle.beta_params(m, s, x)[:2] for m, s, x in zip(mu, sd, mx)])
    u = (2 * rng.integers(0, 2 ** 23, n) + 1) * 2.0 ** -24
    x = P.ara_beta_quantile(eng.ctx, ab[:, 0], ab[:, 1], u)
    xo = oracle.beta_inc_inv_vec(u, ab[:, 0], ab[:, 1])
    visible = xo > 1e-30
    assert np.max(np.abs(x[visible] - xo[visible]) / xo[visible]) <= 1e-8


@pytest.mark.parametrize("lo,hi,seed", [(1e-3, 40.0, 5), (0.2, 50.0, 6), (3e-6, 35.0, 7), (0.1, 0.3, 8),
                                         (1e-5, 2e-3, 9), (0.005, 0.2, 10)])
def test_layer_inverse_per_draw_accuracy(eng, lo, hi, seed):
    # the inverse exactly as the plain layer kernel applies it: the
    # continued-fraction FP32 solve where min(a, b) >= 0.2, the series form on
    # the small side below that (two tiny shapes included: (1e-5, 2e-3)); FP32
    # either way, within 1e-5 relative of the FP64 oracle
    a, b, u = _grid(40000, lo, hi, seed)
    x = P.ara_beta_quantile_layer(eng.ctx, a, b, u)
    xo = oracle.beta_inc_inv_vec(u, a, b, threads=0)
    visible = xo > 1e-30
    rel = np.abs(x - xo) / np.maximum(xo, 1e-300)
    small = np.minimum(a, b) < 0.2
    for sel in (~small, small):
        if np.any(visible & sel):
            assert np.all(rel[visible & sel] <= 1e-5), rel[visible & sel].max()
            assert np.quantile(rel[visible & sel], 0.99) <= 3e-6
    assert np.all(x[~visible] <= 1e-28)


@pytest.mark.parametrize("side", ["upper", "lower"])
def test_layer_inverse_off_grid_tails(eng, side):
    # Correlated draws (section 3.2) give z = Phi(v) anywhere in (0, 1), not on
    # the 2^-24 grid, and as close to 1 as 1 - 1e-13.  The layer's inverse must
    # keep the tail's relative accuracy: with a large leading shape the
    # quantile of a tail probability p is far from 0 or 1, so an error in p
    # shows up in x (rounding z near 1 to FP32 would move p by up to 100%).
    ks = np.arange(6, 14)
    rng = np.random.default_rng(17)
    n = 4000
    k = rng.choice(ks, n)
    tail = 10.0 ** (-k) * rng.uniform(1.0, 9.0, n)
    big = np.exp(rng.uniform(math.log(5.0), math.log(35.0), n))
    small = np.exp(rng.uniform(math.log(0.3), math.log(3.0), n))
    small[::4] = np.exp(rng.uniform(math.log(1e-3), math.log(0.14), n // 4))   # the series form too
    if side == "upper":
        a, b, u = small, big, 1.0 - tail
    else:
        a, b, u = big, small, tail
    x = P.ara_beta_quantile_layer(eng.ctx, a, b, u)
    xo = oracle.beta_inc_inv_vec(u, a, b, threads=0)
    dist = np.minimum(xo, 1.0 - xo)          # distance from the nearer end of [0, 1]
    err = np.abs(x - xo)
    # FP32 solve, either form: 1e-5 of that distance, or FP32's spacing next to 1
    assert np.all(err <= 1e-5 * dist + 1.2e-7), (err / (dist + 1e-30)).max()
    assert np.any(np.minimum(a, b) < 0.2) and np.any(np.minimum(a, b) >= 0.2)
    assert np.median(dist) > 1e-3            # the cases exercise quantiles away from the ends


def test_clamped_entries_beta_params_match_oracle(eng):
    # Section 3.3's moment matching with the std bound: entries whose std
    # exceeds c * sigma_beta_max (c = 0.999) are clamped to it.  The device's
    # FP64 alpha, beta against the oracle's, clamped or not.
    rng = np.random.default_rng(23)
    n = 3000
    mu = rng.lognormal(10, 1.5, n)
    mx = mu * rng.uniform(1.05, 10, n)
    mub = mu / mx
    sbmax = np.sqrt(mub * (1 - mub)) * mx
    sd = sbmax * rng.uniform(0.05, 3.0, n)                 # about two thirds are clamped
    sd[:5] = sbmax[:5] * np.array([0.999, 0.99899, 0.99901, 1.0, 100.0])
    sd[5] = 0.0                                            # degenerate entry
    elt = synth.ELT(np.arange(n, dtype=np.int32), mu, sd, None, mx, 0.0, math.inf, 1.0)
    h = P.ara_load_elts(eng.ctx, n, [elt])[0]
    a, b = P.ara_elt_params(eng.ctx, h, n)
    ref = np.array([oracle.beta_params(m, s, x)[:2] if s > 0 else (0.0, 0.0) for m, s, x in zip(mu, sd, mx)])
    clamped = sd > 0.999 * sbmax
    assert 1000 < clamped.sum() < n
    # nu = (sigma_max / sigma_beta)^2 - 1 cancels near the bound (nu = 0.002 on
    # clamped entries), so a few FP64 roundings of the ratio (the device may fuse
    # the square and the subtraction) become 8 eps (1 + nu) / nu relative in nu
    nu_i = ref[:, 0] + ref[:, 1]
    rtol = 8 * 2.0 ** -53 * (2 + 1 / np.maximum(nu_i, 1e-300))
    assert np.all(np.abs(a - ref[:, 0]) <= rtol * ref[:, 0])
    assert np.all(np.abs(b - ref[:, 1]) <= rtol * ref[:, 1])
    nu = 1 / 0.999 ** 2 - 1
    np.testing.assert_allclose(a[clamped], mub[clamped] * nu, rtol=1e-12)
    P.ara_free_elts(eng.ctx, [h])


def test_normal_quantile_vs_oracle_and_tables(eng):
    # the FP64 Phi^-1 of the correlated draws (section 3.2): tabulated points,
    # both region boundaries of the rational approximations, the ends of the
    # 2^-24 grid, and random grid points
    from scipy.special import ndtri
    from conftest import golden
    pts = golden("normal_points.json")["points"]
    p = np.array([q["p"] for q in pts])
    x = P.ara_normal_quantile(eng.ctx, p)
    for q, v in zip(pts, x):
        assert v == pytest.approx(q["x"], rel=1e-14, abs=1e-15)
    rng = np.random.default_rng(8)
    grid = (2 * rng.integers(0, 2 ** 23, 5000) + 1) * 2.0 ** -24
    edges = np.array([2.0 ** -24, 1 - 2.0 ** -24, 0.075, 0.925, 0.0749999, 0.9250001, math.exp(-25.0),
                      math.exp(-25.0) * 1.0001, 1e-300, 0.5])
    p = np.concatenate([grid, edges])
    x = P.ara_normal_quantile(eng.ctx, p)
    xo = np.array([oracle.norm_quantile(v) for v in p])
    assert np.allclose(x, xo, rtol=1e-14, atol=1e-15)
    assert np.allclose(x, ndtri(p), rtol=1e-13, atol=1e-14)
    with pytest.raises(P.AraError):
        P.ara_normal_quantile(eng.ctx, np.array([0.0]))


def test_beta_quantile_rejects_bad_input(eng):
    with pytest.raises(P.AraError) as e:
        P.ara_beta_quantile(eng.ctx, np.array([1.0]), np.array([-1.0]), np.array([0.5]))
    assert e.value.status == P.ARA_E_INVAL
    with pytest.raises(P.AraError):
        P.ara_beta_quantile(eng.ctx, np.array([1.0]), np.array([1.0]), np.array([1.0]))


# ------------------------------------------------------------ A1-A10: whole layer
@pytest.mark.parametrize("mode", [oracle.MODE_MEAN, oracle.MODE_PLAIN])
def test_tiny_workload_full_ylt(eng, mode):
    wl = synth.tiny()
    y, om, _ = gpu_ylt(eng, wl, mode, wl.seed, with_omax=True)
    yo, g, omo = oracle_ylt(wl, np.arange(wl.n_trials), mode, wl.seed)
    worst = assert_ylt_close(y, yo, g, f"tiny mode {mode}")
    assert_ylt_close(om, omo, g, "max occurrence")
    assert np.all(y >= 0) and np.all(y <= wl.layers[0].agg_limit * (1 + 1e-6))
    print(f"tiny mode={mode}: worst |dY|/G = {worst:.3e}")


@pytest.mark.parametrize("N,K,C,J,lo,hi,sc", [
    (67, 1, 50, 1, 10, 30, 0.0),          # one event per trial
    (130, 63, 400, 3, 50, 150, 0.0),      # chunk of 63 slots
    (65, 65, 300, 17, 20, 60, 0.0),       # ragged chunk, > 16 draws per slot possible
    (33, 130, 200, 40, 30, 120, 0.0),     # 40 XELTs: several drain rounds per slot
    (40, 70, 120, 64, 40, 90, 0.0),       # 64 XELTs, dense hits
    (50, 90, 500, 5, 100, 300, 0.6),      # correlated std (section 3.2 five steps)
    (400, 700, 40000, 2, 800, 1200, 0.0), # sparse (0.05 draws per occurrence): short FP32 lists go to the ring
    (300, 500, 30000, 2, 600, 900, 0.5),  # sparse and correlated: they stay in the chunk
])
def test_ragged_shapes(eng, N, K, C, J, lo, hi, sc):
    wl = synth.custom(N, K, C, J, lo, hi, seed=N * 7 + J, sigma_c_frac=sc)
    for mode in (oracle.MODE_MEAN, oracle.MODE_PLAIN):
        y, om, _ = gpu_ylt(eng, wl, mode, 99, with_omax=True)
        yo, g, omo = oracle_ylt(wl, np.arange(N), mode, 99)
        assert_ylt_close(y, yo, g, f"N={N} K={K} J={J} mode={mode}")
        assert_ylt_close(om, omo, g, "max occurrence")


def test_degenerate_and_infinite_terms(eng):
    wl = synth.custom(64, 40, 200, 4, 40, 80, seed=5)
    lay = wl.layers[0]
    lay.elts[0].sigma_i[::3] = 0.0                      # sigma = 0: loss is the mean
    lay.elts[1].limit = math.inf
    lay.elts[2].share = 0.0
    lay.elts[3].share = 1.0
    lay.occ_limit = math.inf
    lay.agg_limit = math.inf
    y, _ = gpu_ylt(eng, wl, oracle.MODE_PLAIN, 3)
    yo, g, _ = oracle_ylt(wl, np.arange(64), oracle.MODE_PLAIN, 3)
    assert_ylt_close(y, yo, g, "degenerate/inf")


def _band_elt(rng, C, n, sigma_c_frac=0.0):
    # entries with the smaller shape in [0.05, 0.15): just below the
    # small-shape threshold, so every draw goes through the deferred ring
    ids = np.sort(rng.choice(C, size=n, replace=False)).astype(np.int32)
    s = np.exp(rng.uniform(math.log(0.05), math.log(0.15), n))
    big = np.exp(rng.uniform(math.log(0.15), math.log(30.0), n))
    swap = rng.random(n) < 0.5
    a, b = np.where(swap, big, s), np.where(swap, s, big)
    mx = rng.lognormal(11.0, 1.0, n)
    mu = mx * a / (a + b)
    sd = mx * np.sqrt(a * b / ((a + b) ** 2 * (a + b + 1.0)))
    sc = None
    if sigma_c_frac > 0.0:
        frac = rng.uniform(0.0, sigma_c_frac, n)
        sc, sd = sd * frac, sd * (1.0 - frac)
    return synth.ELT(ids, mu, sd, sc, mx, 0.0, math.inf, float(rng.uniform(0.5, 1.0)))


@pytest.mark.parametrize("sigma_c_frac", [0.0, 0.5])
def test_band_shapes_layer_vs_oracle(eng, sigma_c_frac):
    # Every entry a small shape: all draws take the deferred ring and the series
    # form (or the continued fraction on the large side), the ring flushes full
    # waves many times per trial and the pending ring holds most chunks
    # (correlated or not).
    rng = np.random.default_rng(41)
    N, K, C = 200, 300, 600
    wl = synth.custom(N, K, C, 4, 300, 500, seed=41)
    lay = wl.layers[0]
    lay.elts = [_band_elt(rng, C, int(rng.integers(300, 500)), sigma_c_frac) for _ in range(4)]
    lay.occ_retention, lay.occ_limit, lay.agg_retention, lay.agg_limit = 0.0, math.inf, 0.0, math.inf
    h = P.ara_load_elts(eng.ctx, C, lay.elts[:1])[0]
    a, b = P.ara_elt_params(eng.ctx, h, lay.elts[0].n)
    P.ara_free_elts(eng.ctx, [h])
    assert 0.049 < np.min(np.minimum(a, b)) and np.max(np.minimum(a, b)) < 0.151
    y, om, _ = gpu_ylt(eng, wl, oracle.MODE_PLAIN, 17, with_omax=True)
    yo, g, omo = oracle_ylt(wl, np.arange(N), oracle.MODE_PLAIN, 17)
    assert_ylt_close(y, yo, g, f"band shapes, sigma_c_frac={sigma_c_frac}")
    assert_ylt_close(om, omo, g, "max occurrence")
    assert np.mean(y > 0) > 0.2


def test_variable_length_trials_and_empty_trials(eng):
    torch = torch_cuda()
    rng = np.random.default_rng(11)
    N, C = 97, 300
    lens = rng.integers(0, 150, N)
    lens[[0, 5, 96]] = 0
    offs = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
    ev = rng.integers(0, C, offs[-1], dtype=np.int32)
    wl = synth.custom(N, 1, C, 6, 40, 120, seed=12)
    yh = eng.load_yet(ev, C, trial_offsets=offs)
    desc = eng.load_layer(wl.layers[0], C)
    out = torch.empty(N, device="cuda")
    P.ara_run_layer(eng.ctx, yh, desc, P.MODE_PLAIN, 5, out)
    y = out.cpu().numpy().astype(np.float64)
    for i in range(N):
        row = ev[offs[i]:offs[i + 1]].reshape(1, -1)
        if row.shape[1] == 0:
            assert y[i] == 0.0
            continue
        yo, g, _ = oracle.run_layer(wl.layers[0], row, [i], C, 5)
        assert_ylt_close(y[i:i + 1], yo, g, f"trial {i}")


def test_huge_elts_and_catalog(eng):
    # ELTs of up to 2M entries over a 3M-event catalog (the direct-access
    # tables of section 4.1 scale with the catalog; the mean mode's catalog
    # no longer fits its LDS slices and reads the table through L2)
    wl = synth.custom(600, 1000, 3_000_000, 2, 1_500_000, 2_000_000, seed=44)
    assert max(e.n for e in wl.layers[0].elts) >= 1_500_000
    yh = eng.load_yet(wl.yet(), wl.catalog_size)
    rng = np.random.default_rng(45)
    trials = np.unique(np.concatenate([[0, 599], rng.integers(0, 600, 30)]))
    for mode in (oracle.MODE_MEAN, oracle.MODE_PLAIN):
        y, om, _ = gpu_ylt(eng, wl, mode, 13, yet_handle=yh, with_omax=True)
        yo, g, omo = oracle_ylt(wl, trials, mode, 13)
        assert_ylt_close(y[trials], yo, g, f"huge ELTs mode={mode}")
        assert_ylt_close(om[trials], omo, g, "max occurrence")


# ------------------------------------------------------------ paper scale (sampled)
def test_paper_scale_sampled_trials(eng):
    torch = torch_cuda()
    wl = synth.paper_scale()
    yh = eng.load_yet(wl.yet(), wl.catalog_size)
    y, desc = gpu_ylt(eng, wl, oracle.MODE_PLAIN, wl.seed, yet_handle=yh)
    rng = np.random.default_rng(2024)
    trials = np.unique(np.concatenate([[0, 1, 63, 64, wl.n_trials - 1], rng.integers(0, wl.n_trials, 40)]))
    yo, g, _ = oracle_ylt(wl, trials, oracle.MODE_PLAIN, wl.seed, threads=0)
    worst = assert_ylt_close(y[trials], yo, g, "paper scale")
    print(f"paper scale: worst |dY|/G = {worst:.3e} over {trials.size} trials")
    # both aggregate clamps bind at this scale (retention often, limit rarely)
    assert 0.01 < np.mean(y == 0) < 0.5
    assert 0 < np.sum(y == np.float32(wl.layers[0].agg_limit)) < 0.004 * y.size
    # risk measures of the GPU YLT: exact order statistic, FP64 tail mean
    rps = [10, 50, 100, 250]
    pml, tvar = P.ara_risk_measures(eng.ctx, torch.from_numpy(y.astype(np.float32)).cuda(), rps)
    po, to = oracle.risk_measures(y.astype(np.float32).astype(np.float64), rps)
    assert np.array_equal(pml, po)
    np.testing.assert_allclose(tvar, to, rtol=1e-12)
    P.ara_free_yet(eng.ctx, yh)


def test_mean_mode_paper_scale_sampled(eng):
    wl = synth.paper_scale(n_trials=100_000)
    y, _ = gpu_ylt(eng, wl, oracle.MODE_MEAN, wl.seed)
    trials = np.arange(0, wl.n_trials, 997)
    yo, g, _ = oracle_ylt(wl, trials, oracle.MODE_MEAN, wl.seed)
    assert_ylt_close(y[trials], yo, g, "mean mode")


# ------------------------------------------------------------ A11: PML / TVaR
@pytest.mark.parametrize("n", [1, 10, 1000, 65537, 1_000_000])
def test_risk_measures_vs_oracle(eng, n):
    rng = np.random.default_rng(n)
    y = rng.lognormal(10, 2, n).astype(np.float32)
    if n > 100:
        y[rng.integers(0, n, n // 10)] = 0.0            # ties at zero
        y[rng.integers(0, n, n // 50)] = y[7]           # ties at an interior value
    rps = [rp for rp in (1, 2, 10, 50, 100, 250, 1000) if math.floor(n / rp) >= 1]
    pml, tvar = P.ara_risk_measures(eng.ctx, y, rps)
    po, to = oracle.risk_measures(y.astype(np.float64), rps)
    assert np.array_equal(pml, po)
    np.testing.assert_allclose(tvar, to, rtol=1e-12)


def test_risk_measures_hand_worked(eng):
    from conftest import golden
    w = golden("w2_risk.json")
    pml, tvar = P.ara_risk_measures(eng.ctx, np.array(w["ylt"], dtype=np.float32), [c["rp"] for c in w["cases"]])
    for c, p, t in zip(w["cases"], pml, tvar):
        assert p == c["pml"] and t == c["tvar"]


def test_risk_measures_errors(eng):
    with pytest.raises(P.AraError) as e:
        P.ara_risk_measures(eng.ctx, np.ones(10, dtype=np.float32), [11])
    assert e.value.status == P.ARA_E_RANGE


# ------------------------------------------------------------ determinism and batching
def test_deterministic_and_range_invariant(eng):
    torch = torch_cuda()
    wl = synth.custom(1000, 200, 2000, 8, 100, 400, seed=41)
    yh = eng.load_yet(wl.yet(), wl.catalog_size)
    y1, desc = gpu_ylt(eng, wl, P.MODE_PLAIN, 9, yet_handle=yh)
    y2, _ = gpu_ylt(eng, wl, P.MODE_PLAIN, 9, yet_handle=yh)
    assert np.array_equal(y1, y2)
    parts = []
    for t0, t1 in [(0, 1), (1, 333), (333, 334), (334, 1000)]:
        yp, _ = gpu_ylt(eng, wl, P.MODE_PLAIN, 9, yet_handle=yh, t0=t0, t1=t1)
        parts.append(yp)
    assert np.array_equal(np.concatenate(parts), y1)
    # on another stream
    s = torch.cuda.Stream()
    out = torch.empty(wl.n_trials, device="cuda")
    with torch.cuda.stream(s):
        P.ara_run_layer(eng.ctx, yh, desc, P.MODE_PLAIN, 9, out, stream=s)
    s.synchronize()
    assert np.array_equal(out.cpu().numpy().astype(np.float64), y1)
    # host output buffer
    host = np.empty(wl.n_trials, dtype=np.float32)
    P.ara_run_layer(eng.ctx, yh, desc, P.MODE_PLAIN, 9, host)
    assert np.array_equal(host.astype(np.float64), y1)


def test_batched_layers_equal_single_runs(eng):
    torch = torch_cuda()
    wl = synth.portfolio(n_layers=6, n_trials=3000)
    wl.catalog_size = 100_000
    yh = eng.load_yet(wl.yet(), wl.catalog_size)
    descs = [eng.load_layer(l, wl.catalog_size) for l in wl.layers]
    for mode in (P.MODE_MEAN, P.MODE_PLAIN):
        outs = [torch.empty(wl.n_trials, device="cuda") for _ in descs]
        P.ara_run_layers(eng.ctx, yh, descs, mode, 17, outs)
        torch.cuda.synchronize()
        for d, o in zip(descs, outs):
            single = torch.empty(wl.n_trials, device="cuda")
            P.ara_run_layer(eng.ctx, yh, d, mode, 17, single)
            torch.cuda.synchronize()
            assert torch.equal(single, o)
    # and the batch matches the oracle on a few trials of each layer
    trials = np.array([0, 1, 1777, 2999])
    outs = [torch.empty(wl.n_trials, device="cuda") for _ in descs]
    P.ara_run_layers(eng.ctx, yh, descs, P.MODE_PLAIN, 17, outs)
    torch.cuda.synchronize()
    for l, o in enumerate(outs):
        yo, g, _ = oracle.run_layer(wl.layers[l], wl.yet_rows(trials), trials, wl.catalog_size, 17)
        assert_ylt_close(o.cpu().numpy()[trials].astype(np.float64), yo, g, f"batch layer {l}")


# ------------------------------------------------------------ validation and budget
def test_load_validation_errors(eng):
    good = synth.custom(4, 4, 50, 1, 5, 10, seed=3).layers[0].elts[0]

    def bad(**kw):
        e = synth.ELT(good.event_id.copy(), good.mean.copy(), good.sigma_i.copy(), None, good.max_loss.copy(),
                      good.deductible, good.limit, good.share)
        for k, v in kw.items():
            if k in ("mean", "max_loss", "sigma_i", "event_id"):
                getattr(e, k)[0] = v
            else:
                setattr(e, k, v)
        return e

    cases = [(bad(mean=-1.0), P.ARA_E_INVAL), (bad(max_loss=1.0), P.ARA_E_INVAL), (bad(share=1.5), P.ARA_E_INVAL),
             (bad(sigma_i=math.nan), P.ARA_E_INVAL), (bad(event_id=50), P.ARA_E_RANGE),
             (bad(event_id=int(good.event_id[1])), P.ARA_E_INVAL), (bad(limit=0.0), P.ARA_E_INVAL)]
    for e, status in cases:
        with pytest.raises(P.AraError) as ex:
            P.ara_load_elts(eng.ctx, 50, [e])
        assert ex.value.status == status
    with pytest.raises(P.AraError) as ex:
        P.ara_load_yet(eng.ctx, np.array([[0, 1], [2, 50]], dtype=np.int32), 50)
    assert ex.value.status == P.ARA_E_RANGE
    h = P.ara_load_elts(eng.ctx, 50, [good])
    yh = P.ara_load_yet(eng.ctx, np.zeros((3, 3), dtype=np.int32), 60)
    with pytest.raises(P.AraError):     # catalog mismatch
        P.ara_run_layer(eng.ctx, yh, P.layer_desc(h, 0, 1, 0, 1), P.MODE_PLAIN, 1, np.empty(3, np.float32))
    with pytest.raises(P.AraError) as ex:
        P.ara_run_layer(eng.ctx, 12345, P.layer_desc(h, 0, 1, 0, 1), P.MODE_PLAIN, 1, np.empty(3, np.float32))
    assert ex.value.status == P.ARA_E_STATE


def test_hbm_budget_refusal():
    torch_cuda()
    with P.Engine(0, hbm_budget_bytes=8 << 20) as e:
        with pytest.raises(P.AraError) as ex:
            P.ara_load_yet(e.ctx, np.zeros((4096, 1024), dtype=np.int32), 10)   # 16 MB > 8 MB
        assert ex.value.status == P.ARA_E_BUDGET
        assert P.ara_bytes_in_use(e.ctx) < (8 << 20)
        h = P.ara_load_yet(e.ctx, np.zeros((16, 16), dtype=np.int32), 10)
        assert h >= 0


def test_refused_xelt_load_changes_nothing():
    # five XELTs over a 600,000-event catalog (2.4 MB of index each) against an
    # 8 MB budget: the fourth is refused, and the three loaded before it go too
    torch_cuda()
    C = 600_000
    rng = np.random.default_rng(8)
    elts = []
    for k in range(5):
        ids = np.sort(rng.choice(C, 1000, replace=False)).astype(np.int32)
        mu = rng.lognormal(10, 1, 1000)
        elts.append(synth.ELT(ids, mu, 0.5 * mu, None, 5 * mu, 0.0, math.inf, 1.0))
    with P.Engine(0, hbm_budget_bytes=8 << 20) as e:
        with pytest.raises(P.AraError) as ex:
            P.ara_load_elts(e.ctx, C, elts)
        assert ex.value.status == P.ARA_E_BUDGET
        # the three XELTs loaded before the refusal were released (their blocks
        # stay pooled for reuse): three fit again, a fourth still does not
        hs = P.ara_load_elts(e.ctx, C, elts[:3])
        with pytest.raises(P.AraError):
            P.ara_load_elts(e.ctx, C, elts[3:4])
        # and the XELTs that did load hold the right parameters
        a, b = P.ara_elt_params(e.ctx, hs[2], 1000)
        ao, bo = np.array([oracle.beta_params(m, s_, x)[:2] for m, s_, x in
                           zip(elts[2].mean, elts[2].sigma_i, elts[2].max_loss)]).T
        np.testing.assert_allclose(a, ao, rtol=1e-12)
        np.testing.assert_allclose(b, bo, rtol=1e-12)


def test_trial_tile_does_not_change_results_and_autotune(eng):
    torch = torch_cuda()
    wl = synth.portfolio(n_layers=3, n_trials=2000)
    yh = eng.load_yet(wl.yet(), wl.catalog_size)
    for mode in (P.MODE_MEAN, P.MODE_PLAIN):
        hs = [P.ara_prepare_layer(eng.ctx, eng.load_layer(l, wl.catalog_size), mode) for l in wl.layers]
        ref = None
        for wpb in (1, 2, 4, 8):
            P.ara_set_trial_tile(eng.ctx, mode, wpb)
            outs = [torch.empty(wl.n_trials, device="cuda") for _ in hs]
            P.ara_run_prepared(eng.ctx, yh, hs, [5, 6, 7], 0, wl.n_trials, outs)
            torch.cuda.synchronize()
            got = torch.stack(outs).cpu().numpy()
            if ref is None:
                ref = got
            assert np.array_equal(got, ref), (mode, wpb)
        best, ms = P.ara_autotune(eng.ctx, yh, hs, 2000)
        assert best in (1, 2, 4, 8) and np.isfinite(ms).all()
        # prepared runs equal the one-shot call
        single = torch.empty(wl.n_trials, device="cuda")
        P.ara_run_layer_ex(eng.ctx, yh, eng.load_layer(wl.layers[1], wl.catalog_size), mode, 6, 0, wl.n_trials, single)
        torch.cuda.synchronize()
        assert np.array_equal(single.cpu().numpy(), ref[1])
        for h in hs:
            P.ara_free_layer(eng.ctx, h)
        P.ara_set_trial_tile(eng.ctx, mode, 4)


def _fixed_shape_elt(rng, C, n, a, b, q_lo, q_hi, sigma_c_frac=0.0, degenerate=None):
    # every entry the same Beta(a, b) with max loss 1e6, so the XELT's
    # retention and limit sit at the z quantiles q_lo and q_hi of every entry:
    # the draws below q_lo net to 0 and those above q_hi to the limit without
    # a solve, the ones between are solved
    from scipy.special import betaincinv
    ids = np.sort(rng.choice(C, size=n, replace=False)).astype(np.int32)
    mx = np.full(n, 1e6)
    mu = mx * a / (a + b)
    sd = mx * math.sqrt(a * b / ((a + b) ** 2 * (a + b + 1.0)))
    sd = np.full(n, sd)
    if degenerate is not None:              # sigma = 0: the loss is the mean
        sd = np.zeros(n)
        mu = np.full(n, degenerate)
    sc = None
    if sigma_c_frac > 0.0:
        sc, sd = sd * sigma_c_frac, sd * (1.0 - sigma_c_frac)
    ded = 1e6 * float(betaincinv(a, b, q_lo)) if q_lo > 0.0 else 0.0
    top = 1e6 * float(betaincinv(a, b, q_hi)) if q_hi < 1.0 else math.inf
    return synth.ELT(ids, mu, sd, sc, mx, ded, top - ded, 0.75)


@pytest.mark.parametrize("mode,sigma_c_frac", [("plain", 0.0), ("plain", 0.4), ("table", 0.0), ("table", 0.4)])
def test_fixed_term_draws_vs_oracle(eng, mode, sigma_c_frac):
    # XELT terms at entry quantiles: in the plain mode a draw whose loss lies
    # within the retention or beyond retention + limit takes its term without
    # the inverse (term_thresholds); the year and occurrence losses must match
    # the oracle, which solves every draw, trial by trial.  Small shapes (the
    # deferred ring) and degenerate entries below, inside and above the terms
    # are included.
    rng = np.random.default_rng(43)
    N, K, C = 300, 400, 900
    wl = synth.custom(N, K, C, 7, 300, 600, seed=43)
    lay = wl.layers[0]
    lay.elts = [
        _fixed_shape_elt(rng, C, 500, 2.0, 5.0, 0.5, 0.9, sigma_c_frac),
        _fixed_shape_elt(rng, C, 400, 0.7, 3.0, 0.3, 0.99, sigma_c_frac),
        _fixed_shape_elt(rng, C, 400, 4.0, 1.5, 0.0, 0.6, sigma_c_frac),
        _fixed_shape_elt(rng, C, 300, 0.1, 2.0, 0.8, 0.97, sigma_c_frac),       # small shape
        _fixed_shape_elt(rng, C, 300, 2.0, 5.0, 0.5, 0.9, degenerate=1e5),      # mean within the retention
        _fixed_shape_elt(rng, C, 300, 2.0, 5.0, 0.1, 0.2, degenerate=4e5),      # mean beyond retention + limit
        _fixed_shape_elt(rng, C, 300, 2.0, 5.0, 0.2, 0.9, degenerate=3e5),      # mean between
    ]
    lay.occ_retention, lay.occ_limit, lay.agg_retention, lay.agg_limit = 0.0, math.inf, 0.0, math.inf
    y, om, _ = gpu_ylt(eng, wl, P.MODE_PLAIN if mode == "plain" else P.MODE_TABLE, 19, with_omax=True)
    yo, g, omo = oracle_ylt(wl, np.arange(N), oracle.MODE_PLAIN, 19)
    if mode == "plain":
        assert_ylt_close(y, yo, g, f"fixed-term draws, sigma_c_frac={sigma_c_frac}")
        assert_ylt_close(om, omo, g, "max occurrence")
    else:
        # the tabulated inverse is within 2e-4 relative per draw (its own tests),
        # and every term is 1-Lipschitz: a year or occurrence loss moves by at
        # most 2e-4 of the trial's gross
        tol = 2e-4 * g + 1e-3
        assert np.all(np.abs(y - yo) <= tol) and np.all(np.abs(om - omo) <= tol)
    assert np.all(y > 0)
