"""Pins of the FP64 oracle against values and facts fixed outside it.

Each test checks the oracle against something other than itself: published
known-answer vectors, tabulated percentage points, closed forms, symmetries,
independent library routines (scipy, mpmath), hand-worked examples
(tests/golden) and statistical identities of the method.
"""
import math

import numpy as np
import pytest
import scipy.special as sp
import scipy.stats as st

from conftest import golden
from paper_1310_2274_amd import synth

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")


# ------------------------------------------------------------ Philox (A3)
def test_philox_known_answers(orc):
    for v in golden("philox_kat.json")["vectors"]:
        ctr = [int(x, 16) for x in v["ctr"]]
        key = [int(x, 16) for x in v["key"]]
        assert orc.philox4x32_10(ctr, key) == tuple(int(x, 16) for x in v["out"])


def test_uniform_grid_and_ends(orc):
    assert orc.uniform(0) == 2.0 ** -24
    assert orc.uniform(0xFFFFFFFF) == 1.0 - 2.0 ** -24
    assert orc.uniform(1 << 31) == 0.5 + 2.0 ** -24
    for w in (0, 12345, 1 << 31, 0xFFFFFFFF):   # exactly representable in FP32
        u = orc.uniform(w)
        assert float(np.float32(u)) == u


def test_uniform_stream_chi_square(orc):
    n = 40000
    u = np.array([orc.u_indep(1310, 3, t // 50, t % 50, 7) for t in range(n)])
    counts, _ = np.histogram(u, bins=40, range=(0, 1))
    chi2 = ((counts - n / 40) ** 2 / (n / 40)).sum()
    assert st.chi2.sf(chi2, 39) > 1e-4
    # the correlated stream is shared across programs and ELTs, the independent one is not
    assert orc.u_corr(1310, 5, 9) == orc.u_corr(1310, 5, 9)
    assert orc.u_indep(1310, 0, 5, 9, 0) != orc.u_indep(1310, 1, 5, 9, 0)
    assert orc.u_indep(1310, 0, 5, 9, 0) != orc.u_indep(1310, 0, 5, 9, 1)
    assert orc.u_indep(1310, 0, 5, 9, 0) != orc.u_indep(1310, 0, 9, 5, 0)


# ------------------------------------------------------------ normal (A4)
def test_normal_quantile_tabulated(orc):
    for p in golden("normal_points.json")["points"]:
        assert orc.norm_quantile(p["p"]) == pytest.approx(p["x"], rel=1e-15, abs=1e-300)


def test_normal_quantile_vs_library_and_roundtrip(orc):
    ps = np.concatenate([np.logspace(-300, -1, 200), np.linspace(0.01, 0.99, 99),
                         1 - np.logspace(-16, -2, 50)])
    for p in ps:
        x = orc.norm_quantile(p)
        assert x == pytest.approx(float(sp.ndtri(p)), rel=2e-14, abs=1e-15)
        if 1e-300 < p < 1 - 1e-12:
            assert orc.norm_cdf(x) == pytest.approx(p, rel=1e-13)
    assert orc.norm_cdf(0.0) == 0.5
    for m in (0, 1, 1000, 2 ** 20, 2 ** 22 - 1):        # symmetry on the uniform grid (1-u exact)
        u = (2 * m + 1) * 2.0 ** -24
        assert orc.norm_quantile(1 - u) == pytest.approx(-orc.norm_quantile(u), rel=1e-14)


def test_combine_extreme_cases_and_marginal(orc):
    # section 3.2: the two extreme cases sigma_C = 0 and sigma_I = 0
    assert orc.combine(0.3, 0.8, 2.0, 0.0) == 0.3
    assert orc.combine(0.3, 0.8, 0.0, 2.0) == 0.8
    # the normalised combination is N(0,1), so z is uniform
    rng = np.random.default_rng(0)
    ui, uc = rng.random(20000), rng.random(20000)
    z = np.array([orc.combine(a, b, 1.0, 2.5) for a, b in zip(ui, uc)])
    assert st.kstest(z, "uniform").pvalue > 1e-3
    # and it is increasing in each uniform
    assert orc.combine(0.4, 0.5, 1.0, 1.0) < orc.combine(0.41, 0.5, 1.0, 1.0)
    assert orc.combine(0.4, 0.5, 1.0, 1.0) < orc.combine(0.4, 0.51, 1.0, 1.0)


# ------------------------------------------------------------ Beta parameters (A5)
def test_beta_params_worked_example(orc):
    w = golden("w3_beta.json")
    a, b, mub, deg = orc.beta_params(w["mean"], w["sigma"], w["max_loss"])
    assert not deg
    assert a == pytest.approx(w["alpha"], rel=1e-14)
    assert b == pytest.approx(w["beta"], rel=1e-14)
    assert mub == 0.25


def test_beta_params_match_moments(orc):
    # Beta(a,b) has mean a/(a+b) and variance ab/((a+b)^2(a+b+1)): the scaled
    # Beta reproduces the mean exactly and the std whenever it is not clamped.
    rng = np.random.default_rng(1)
    for _ in range(500):
        mx = 10 ** rng.uniform(0, 7)
        mu = mx * rng.uniform(1e-4, 0.999)
        sbmax = math.sqrt((mu / mx) * (1 - mu / mx)) * mx
        sd = sbmax * rng.uniform(0.01, 0.998)
        a, b, _, deg = orc.beta_params(mu, sd, mx)
        assert not deg
        assert mx * a / (a + b) == pytest.approx(mu, rel=1e-12)
        var = a * b / ((a + b) ** 2 * (a + b + 1))
        assert mx * math.sqrt(var) == pytest.approx(sd, rel=1e-10)


def test_beta_params_clamp_and_degenerate(orc):
    mu, mx = 10.0, 100.0
    sbmax = math.sqrt(0.1 * 0.9) * mx
    a, b, _, _ = orc.beta_params(mu, 5 * sbmax, mx)
    nu = 1 / 0.999 ** 2 - 1
    assert a == pytest.approx(0.1 * nu, rel=1e-12) and b == pytest.approx(0.9 * nu, rel=1e-12)
    assert a > 0 and b > 0
    _, _, mub, deg = orc.beta_params(mu, 0.0, mx)
    assert deg and mub == 0.1


# ------------------------------------------------------------ inverse Beta (A6)
def test_inverse_beta_worked_example(orc):
    w = golden("w3_beta.json")
    x = orc.beta_inc_inv(w["z"], w["alpha"], w["beta"])
    assert x == pytest.approx(w["x"], rel=1e-15)
    assert w["max_loss"] * x == pytest.approx(w["loss"], rel=1e-15)


@pytest.mark.parametrize("pure", [False, True])
def test_inverse_beta_closed_forms(orc, pure):
    zs = [2.0 ** -24, 1e-5, 0.01, 0.3, 0.5, 0.77, 0.999, 1 - 2.0 ** -24]
    for z in zs:
        for b in (0.05, 0.7, 3.0, 31.5):       # a = 1: 1 - (1-z)^(1/b)
            assert orc.beta_inc_inv(z, 1.0, b, pure) == pytest.approx(-math.expm1(math.log1p(-z) / b), rel=1e-13)
        for a in (0.05, 0.7, 3.0, 31.5):       # b = 1: z^(1/a)
            assert orc.beta_inc_inv(z, a, 1.0, pure) == pytest.approx(z ** (1 / a), rel=1e-13)
        assert orc.beta_inc_inv(z, 1.0, 1.0, pure) == pytest.approx(z, rel=1e-14)
        # arcsine law: a = b = 1/2 gives sin^2(pi z / 2)
        assert orc.beta_inc_inv(z, 0.5, 0.5, pure) == pytest.approx(math.sin(math.pi * z / 2) ** 2, rel=1e-12)
    assert orc.beta_inc_inv(0.3, 0.5, 0.5) == pytest.approx(0.2061073738537634, rel=1e-14)


def test_inverse_beta_symmetry(orc):
    rng = np.random.default_rng(2)
    for _ in range(300):
        a, b = np.exp(rng.uniform(np.log(0.05), np.log(40), 2))
        z = (2 * rng.integers(0, 2 ** 23) + 1) * 2.0 ** -24
        x = orc.beta_inc_inv(z, a, b)
        y = orc.beta_inc_inv(1 - z, b, a)
        assert x == pytest.approx(1 - y, rel=1e-11, abs=1e-13)


def test_inverse_beta_vs_scipy_stratified(orc):
    rng = np.random.default_rng(3)
    n = 20000
    a = np.exp(rng.uniform(np.log(1e-3), np.log(50), n))
    b = np.exp(rng.uniform(np.log(1e-3), np.log(50), n))
    u = (2 * rng.integers(0, 2 ** 23, n) + 1) * 2.0 ** -24
    x = orc.beta_inc_inv_vec(u, a, b, threads=4)
    xs = sp.betaincinv(a, b, u)
    ok = xs > 1e-280                       # both sides underflow below this
    rel = np.abs(x[ok] - xs[ok]) / xs[ok]
    # loose where a small shape parameter makes the quantile ill-conditioned
    # (relative error scales like 1/min(a, b) there), tight elsewhere
    assert np.quantile(rel, 0.9) < 1e-13
    assert np.quantile(rel, 0.99) < 1e-11
    assert np.all(rel < 1e-6)
    assert np.all(x[~ok] < 1e-270)


def test_inverse_beta_bisection_agrees_with_newton(orc):
    rng = np.random.default_rng(4)
    n = 5000
    a = np.exp(rng.uniform(np.log(3e-6), np.log(40), n))
    b = np.exp(rng.uniform(np.log(6e-6), np.log(40), n))
    u = (2 * rng.integers(0, 2 ** 23, n) + 1) * 2.0 ** -24
    x0 = orc.beta_inc_inv_vec(u, a, b, threads=4)
    x1 = orc.beta_inc_inv_vec(u, a, b, pure_bisection=True, threads=4)
    big = np.maximum(x0, x1) > 1e-300
    rel = np.abs(x0 - x1)[big] / np.maximum(x0, x1)[big]
    assert np.quantile(rel, 0.999) < 1e-12


def test_incomplete_beta_vs_mpmath(orc):
    mp = pytest.importorskip("mpmath")
    mp.mp.dps = 30
    rng = np.random.default_rng(5)
    for _ in range(200):
        a, b = np.exp(rng.uniform(np.log(0.01), np.log(50), 2))
        x = rng.uniform(0.001, 0.999)
        ref = float(mp.betainc(a, b, 0, x, regularized=True))
        assert orc.beta_inc(x, a, b) == pytest.approx(ref, rel=1e-12, abs=1e-300)
        # and the quantile is a root of the mpmath CDF to within its conditioning
        u = (2 * int(rng.integers(0, 2 ** 23)) + 1) * 2.0 ** -24
        q = orc.beta_inc_inv(u, a, b)
        if 1e-200 < q < 1 - 1e-12:
            resid = float(mp.betainc(a, b, 0, q, regularized=True)) - u
            dens = float(mp.exp((a - 1) * mp.log(q) + (b - 1) * mp.log(1 - q) - mp.log(mp.beta(a, b))))
            assert abs(resid) <= 1e-13 * max(u, 1e-300) + 4e-16 * dens * q + 1e-300


def test_scaled_beta_mean_by_quadrature(orc):
    # E[max * Q(U)] = mu: the mean of the sampled loss is the XELT's mean loss
    # (quadrature in u of the oracle's quantile against the closed-form mean)
    from scipy.integrate import quad
    for mu, sd, mx in [(25.0, 19.364916731037084, 100.0), (3e4, 2.5e4, 2e5), (7e3, 9e3, 5e4),
                       (500.0, 2000.0, 3000.0)]:
        a, b, mub, _ = orc.beta_params(mu, sd, mx)
        m1, _ = quad(lambda u: orc.beta_inc_inv(u, a, b), 0, 1, limit=400, epsabs=1e-13, epsrel=1e-11)
        m2, _ = quad(lambda u: orc.beta_inc_inv(u, a, b) ** 2, 0, 1, limit=400, epsabs=1e-13, epsrel=1e-11)
        assert mx * m1 == pytest.approx(mu, rel=1e-7)
        assert mx * math.sqrt(m2 - m1 * m1) == pytest.approx(min(sd, 0.999 * math.sqrt(mub * (1 - mub)) * mx), rel=1e-5)


# ------------------------------------------------------------ terms (A7-A9) and Algorithm 1
def _w1_layer(over):
    w = golden("w1_terms.json")
    elts = []
    for e in w["elts"]:
        m = np.array(e["mean"], dtype=float)
        elts.append(synth.ELT(np.array(e["event_id"], dtype=np.int32), m, np.zeros_like(m), None,
                              m * 4, e["deductible"], e["limit"], e["share"]))
    t = dict(w["layer"])
    t.update(over)
    return w, synth.Layer(elts, t["occ_retention"], t["occ_limit"], t["agg_retention"], t["agg_limit"])


@pytest.mark.parametrize("mode", [0, 1])
def test_terms_hand_worked(orc, mode):
    w = golden("w1_terms.json")
    for case in w["cases"]:
        _, lay = _w1_layer(case["override"])
        rows = np.array([case["trial"]], dtype=np.int32)
        y, g, om, ye = orc.run_layer(lay, rows, [0], w["catalog_size"], seed=1, mode=mode, yelt=True)
        assert y[0] == case["Y"]
        assert g[0] == case["gross"]                            # the scale of every per-trial tolerance
        assert om[0] == case["max_occ"]
        assert list(ye[0]) == case["yelt"]                      # per-occurrence losses (YELT)
        inc = orc.yelt_increments(ye, lay.agg_retention, lay.agg_limit)
        assert list(inc[0]) == case["increments"]               # aggregate increments, order-dependent
        assert math.fsum(inc[0]) == case["Y"]                   # and they telescope to the year loss


def test_risk_measures_hand_worked(orc):
    w = golden("w2_risk.json")
    pml, tvar = orc.risk_measures(np.array(w["ylt"], dtype=float), [c["rp"] for c in w["cases"]])
    for c, p, t in zip(w["cases"], pml, tvar):
        assert p == c["pml"] and t == c["tvar"]
    with pytest.raises(ValueError):
        orc.risk_measures(np.array(w["ylt"], dtype=float), [11])


def test_risk_measures_properties(orc):
    rng = np.random.default_rng(6)
    y = rng.lognormal(0, 2, 5000)
    rps = [2, 10, 50, 100, 250, 1000]
    pml, tvar = orc.risk_measures(y, rps)
    assert np.all(tvar >= pml)
    assert np.all(np.diff(pml) >= 0) and np.all(np.diff(tvar) >= 0)
    # independent of the order of the YLT, and ties do not matter
    p2, t2 = orc.risk_measures(rng.permutation(y), rps)
    assert np.array_equal(pml, p2) and np.array_equal(tvar, t2)
    z = np.repeat([1.0, 2.0, 3.0], 100)
    p3, t3 = orc.risk_measures(z, [3, 2])
    assert list(p3) == [3.0, 2.0]
    assert t3[0] == 3.0 and t3[1] == pytest.approx(400.0 / 150.0, rel=1e-15)


def _small(orc, sigma_c=0.0, terms="binding", N=64, K=30, C=300, J=3, seed=11):
    wl = synth.custom(N, K, C, J, 40, 120, seed=seed, sigma_c_frac=sigma_c, terms=terms)
    return wl, wl.layers[0], wl.yet()


def test_invariants_bounds(orc):
    wl, lay, yet = _small(orc)
    y, g, om = orc.run_layer(lay, yet, np.arange(wl.n_trials), wl.catalog_size, seed=5)
    assert np.all(y >= 0) and np.all(y <= lay.agg_limit)
    assert np.all(om <= lay.occ_limit)
    assert np.all(y <= g + 1e-9)
    assert np.any(y > 0)


@pytest.mark.parametrize("field,direction", [("agg_retention", -1), ("occ_retention", -1),
                                             ("agg_limit", +1), ("occ_limit", +1)])
def test_invariants_monotone_layer_terms(orc, field, direction):
    wl, lay, yet = _small(orc)
    tid = np.arange(wl.n_trials)
    y0, _, _ = orc.run_layer(lay, yet, tid, wl.catalog_size, seed=5)
    setattr(lay, field, getattr(lay, field) * 1.3 + 1000.0)
    y1, _, _ = orc.run_layer(lay, yet, tid, wl.catalog_size, seed=5)
    assert np.all(direction * (y1 - y0) >= -1e-9)
    assert np.any(y1 != y0)


@pytest.mark.parametrize("field,direction", [("deductible", -1), ("limit", +1), ("share", +1)])
def test_invariants_monotone_elt_terms(orc, field, direction):
    wl, lay, yet = _small(orc)
    tid = np.arange(wl.n_trials)
    y0, _, _ = orc.run_layer(lay, yet, tid, wl.catalog_size, seed=5)
    e = lay.elts[1]
    setattr(e, field, min(1.0, getattr(e, field) * 1.5) if field == "share" else getattr(e, field) * 1.5 + 1e4)
    y1, _, _ = orc.run_layer(lay, yet, tid, wl.catalog_size, seed=5)
    assert np.all(direction * (y1 - y0) >= -1e-9)


def test_mean_mode_independent_of_event_order(orc):
    wl, lay, yet = _small(orc)
    tid = np.arange(wl.n_trials)
    rng = np.random.default_rng(8)
    perm = np.array([rng.permutation(r) for r in yet])
    y0, _, _ = orc.run_layer(lay, yet, tid, wl.catalog_size, seed=5, mode=orc.MODE_MEAN)
    y1, _, _ = orc.run_layer(lay, perm, tid, wl.catalog_size, seed=5, mode=orc.MODE_MEAN)
    np.testing.assert_allclose(y0, y1, rtol=1e-13)


def test_zero_sigma_reduces_to_mean_mode(orc):
    # sigma -> 0: secondary uncertainty vanishes and the primary-uncertainty
    # (mean loss) analysis is recovered exactly
    wl, lay, yet = _small(orc)
    for e in lay.elts:
        e.sigma_i = np.zeros_like(e.sigma_i)
    tid = np.arange(wl.n_trials)
    y0, _, _ = orc.run_layer(lay, yet, tid, wl.catalog_size, seed=5, mode=orc.MODE_MEAN)
    y1, _, _ = orc.run_layer(lay, yet, tid, wl.catalog_size, seed=5, mode=orc.MODE_PLAIN)
    np.testing.assert_array_equal(y0, y1)


def test_expected_year_loss_closed_form(orc):
    # With pass-through terms, E[Y] = (K/C) * sum_j sum_e mu_j(e): every event
    # is uniform over the catalog and the sampled loss has mean mu.
    wl = synth.custom(4000, 20, 500, 2, 60, 120, seed=21, terms="none")
    lay = wl.layers[0]
    for e in lay.elts:       # keep the loss distributions moderate for a tight CLT bound
        e.mean = np.full(e.n, 1000.0)
        e.sigma_i = np.full(e.n, 400.0)
        e.max_loss = np.full(e.n, 5000.0)
    y, _, _ = orc.run_layer(lay, wl.yet(), np.arange(wl.n_trials), wl.catalog_size, seed=9, threads=4)
    expect = wl.events_per_trial / wl.catalog_size * sum(float(e.mean.sum()) for e in lay.elts)
    se = y.std(ddof=1) / math.sqrt(y.size)
    assert abs(y.mean() - expect) < 4.5 * se


def test_event_outside_catalog_is_an_error(orc):
    wl, lay, yet = _small(orc)
    bad = yet[:2].copy()
    bad[1, 3] = wl.catalog_size
    with pytest.raises(ValueError):
        orc.run_layer(lay, bad, [0, 1], wl.catalog_size, seed=5)


def test_pipeline_brute_force_tiny(orc):
    """Algorithm 1 written out independently for N<=8, K<=3, J<=2 with the
    quantile from mpmath (not the oracle's continued fraction)."""
    mp = pytest.importorskip("mpmath")
    mp.mp.dps = 30
    wl = synth.custom(8, 3, 20, 2, 6, 12, seed=31, sigma_c_frac=0.6)
    lay = wl.layers[0]
    yet = wl.yet()
    y, g, _ = orc.run_layer(lay, yet, np.arange(8), wl.catalog_size, seed=77)

    def quantile(z, a, b):
        f = lambda x: mp.betainc(a, b, 0, x, regularized=True) - z
        lo, hi = mp.mpf(0), mp.mpf(1)
        for _ in range(200):                 # plain bisection in 30-digit arithmetic
            mid = (lo + hi) / 2
            if f(mid) < 0:
                lo = mid
            else:
                hi = mid
        return hi

    for i in range(8):
        S = mp.mpf(0)
        for k in range(3):
            e = int(yet[i, k])
            c = mp.mpf(0)
            for j, X in enumerate(lay.elts):
                hit = np.nonzero(X.event_id == e)[0]
                if hit.size == 0:
                    continue
                r = int(hit[0])
                mu, si, mx = X.mean[r], X.sigma_i[r], X.max_loss[r]
                sc = 0.0 if X.sigma_c is None else X.sigma_c[r]
                ui = orc.u_indep(77, 0, i, k, j)
                uc = orc.u_corr(77, i, k)
                s = si + sc
                if sc == 0:
                    z = mp.mpf(ui)
                elif si == 0:
                    z = mp.mpf(uc)
                else:
                    vi = mp.sqrt(2) * mp.erfinv(2 * mp.mpf(ui) - 1)
                    vc = mp.sqrt(2) * mp.erfinv(2 * mp.mpf(uc) - 1)
                    wi, wc = mp.mpf(si) / s, mp.mpf(sc) / s
                    v = (vi * wi + vc * wc) / mp.sqrt(wi ** 2 + wc ** 2)
                    z = mp.ncdf(v)
                mub = mp.mpf(mu) / mx
                sbmax = mp.sqrt(mub * (1 - mub))
                sb = min(mp.mpf(s) / mx, mp.mpf("0.999") * sbmax)
                nu = (sbmax / sb) ** 2 - 1
                loss = mx * quantile(z, mub * nu, (1 - mub) * nu)
                c += X.share * min(max(loss - X.deductible, 0), X.limit)
            S += min(max(c - lay.occ_retention, 0), lay.occ_limit)
        Y = min(max(S - lay.agg_retention, 0), lay.agg_limit)
        assert y[i] == pytest.approx(float(Y), rel=1e-10, abs=1e-6)


def test_workload_clamps_bind(orc):
    """The tiny workload's terms are sized so that each clamp binds on a
    fraction of its items (occurrence retention/limit per event, aggregate
    retention/limit per trial)."""
    wl = synth.tiny()
    lay = wl.layers[0]
    y, g, om = orc.run_layer(lay, wl.yet(), np.arange(wl.n_trials), wl.catalog_size, seed=wl.seed, threads=4)
    assert 0.01 < np.mean(y == 0) < 0.99                 # aggregate retention binds
    assert 0.01 < np.mean(y == lay.agg_limit) < 0.99     # aggregate limit binds
    assert np.mean(om == lay.occ_limit) > 0.01           # occurrence limit binds
