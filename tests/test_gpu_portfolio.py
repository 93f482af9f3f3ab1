"""GPU tests of a correlated multi-program portfolio (sections 2.1, 3.1, 3.2):
layers of several programs drawing on shared ELTs whose entries carry a
correlated std, program and portfolio totals, and their PML/TVaR."""
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


def test_correlated_portfolio_layers_totals_and_measures(eng):
    torch = torch_cuda()
    wl = synth.correlated_portfolio(n_programs=4, layers_per_program=2, n_trials=3000)
    N, C = wl.n_trials, wl.catalog_size
    yh = eng.load_yet(wl.yet(), C)
    descs = [eng.load_layer(l, C) for l in wl.layers]
    outs = [torch.empty(N, device="cuda") for _ in descs]
    P.ara_run_layers(eng.ctx, yh, descs, P.MODE_PLAIN, wl.seed, outs)
    torch.cuda.synchronize()
    ys, yos, gs = [], [], []
    trials = np.arange(N)
    for l, lay in enumerate(wl.layers):
        assert any(e.sigma_c is not None for e in lay.elts)
        y = outs[l].cpu().numpy().astype(np.float64)
        yo, g, _ = oracle.run_layer(lay, wl.yet(), trials, C, wl.seed)
        assert_ylt_close(y, yo, g, f"layer {l} (program {lay.program_id})")
        ys.append(y)
        yos.append(yo)
        gs.append(g)
    # program totals and the portfolio total: FP64 sums in the order given
    progs = sorted({l.program_id for l in wl.layers})
    prog_tot = {}
    for p in progs:
        idx = [l for l, lay in enumerate(wl.layers) if lay.program_id == p]
        out = torch.empty(N, device="cuda")
        P.ara_sum_ylts(eng.ctx, [outs[l] for l in idx], out)
        expect = np.zeros(N)
        for l in idx:
            expect += ys[l]
        assert np.array_equal(out.cpu().numpy(), expect.astype(np.float32))
        prog_tot[p] = out
    total = torch.empty(N, device="cuda")
    P.ara_sum_ylts(eng.ctx, [prog_tot[p] for p in progs], total)
    torch.cuda.synchronize()
    # portfolio PML/TVaR against the oracle's total, within the sum of the per-layer bounds
    rps = [10, 50, 100]
    pml, tvar = P.ara_risk_measures(eng.ctx, total, rps)
    po, to = oracle.risk_measures(np.sum(yos, axis=0), rps)
    bound = float(np.max(np.sum([REL_TOL * g + ABS_TOL for g in gs], axis=0))) * (1 + 1e-6) + 1e-2
    assert np.all(np.abs(np.asarray(pml) - po) <= bound) and np.all(np.abs(np.asarray(tvar) - to) <= bound)
    # a program's marginal contribution: the portfolio total without it
    rest = torch.empty(N, device="cuda")
    P.ara_sum_ylts(eng.ctx, [prog_tot[p] for p in progs[1:]], rest)
    pr, _ = P.ara_risk_measures(eng.ctx, rest, rps)
    assert np.all(np.asarray(pr) <= np.asarray(pml) + bound)


def test_correlated_uniform_is_shared_across_programs(eng):
    # section 3.1: z_(E) is one per event occurrence, the same for every program;
    # z_(Prog,E) is per program.  With only the correlated std, two programs
    # holding the same ELT under the same terms see the same losses.
    torch = torch_cuda()
    wl = synth.custom(512, 60, 400, 1, 150, 150, seed=41, sigma_c_frac=0.6)
    e = wl.layers[0].elts[0]
    base = dict(occ_retention=wl.layers[0].occ_retention, occ_limit=wl.layers[0].occ_limit,
                agg_retention=wl.layers[0].agg_retention, agg_limit=wl.layers[0].agg_limit)
    yh = eng.load_yet(wl.yet(), wl.catalog_size)

    def run(elt, prog):
        lay = synth.Layer([elt], program_id=prog, **base)
        out = torch.empty(wl.n_trials, device="cuda")
        P.ara_run_layer(eng.ctx, yh, eng.load_layer(lay, wl.catalog_size), P.MODE_PLAIN, 3, out)
        torch.cuda.synchronize()
        return out.cpu().numpy()

    sd = e.sigma_i + e.sigma_c
    only_c = synth.ELT(e.event_id, e.mean, np.zeros_like(sd), sd, e.max_loss, e.deductible, e.limit, e.share)
    only_i = synth.ELT(e.event_id, e.mean, sd, None, e.max_loss, e.deductible, e.limit, e.share)
    a, b = run(only_c, 0), run(only_c, 7)
    assert np.array_equal(a, b)
    c, d = run(only_i, 0), run(only_i, 7)
    assert not np.array_equal(c, d)
    # and both match the oracle's streams
    yo, g, _ = oracle.run_layer(synth.Layer([only_c], program_id=7, **base), wl.yet(), np.arange(wl.n_trials),
                                wl.catalog_size, 3)
    assert_ylt_close(b.astype(np.float64), yo, g, "correlated only")
