"""GPU tests of the layer-table layouts and of variable-length trials (the
paper's data ranges, section 2.1: trials of ~800-1,500 occurrences, XELTs of
up to millions of entries; section 4.1: direct-access against compact
tables): the hashed layer table gives bit-identical year losses to the direct
one in every mode, and both match the FP64 oracle."""
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


def _both_layouts(eng, wl, mode, seed, yh, with_omax=False):
    P.ara_set_table_kind(eng.ctx, P.TABLE_HASHED)
    try:
        yh_, omh, _ = gpu_ylt(eng, wl, mode, seed, yet_handle=yh, with_omax=True)
    finally:
        P.ara_set_table_kind(eng.ctx, P.TABLE_DIRECT)
    yd, omd, _ = gpu_ylt(eng, wl, mode, seed, yet_handle=yh, with_omax=True)
    return yh_, omh, yd, omd


@pytest.mark.parametrize("case", ["tiny", "ragged", "correlated", "huge_elts", "sparse_catalog"])
@pytest.mark.parametrize("mode", [oracle.MODE_PLAIN, P.MODE_TABLE])
def test_hashed_table_equals_direct_and_oracle(eng, case, mode):
    if case == "tiny":
        wl = synth.tiny()
    elif case == "ragged":
        wl = synth.custom(130, 63, 400, 3, 50, 150, seed=17)
    elif case == "correlated":
        wl = synth.custom(130, 63, 400, 40, 30, 120, seed=18, sigma_c_frac=0.6)
    elif case == "huge_elts":
        # XELTs of up to 2M entries over a 3M-event catalog: nearly every event is held
        wl = synth.custom(300, 1000, 3_000_000, 2, 1_500_000, 2_000_000, seed=44)
    else:
        # a 20M-event catalog covered ~5% by the layer: the hashed table is ~1/8 of the direct one
        wl = synth.sparse_catalog(n_trials=500)
    yh = eng.load_yet(wl.yet(), wl.catalog_size)
    yh_, omh, yd, omd = _both_layouts(eng, wl, mode, 21, yh)
    assert np.array_equal(yh_, yd) and np.array_equal(omh, omd)
    rng = np.random.default_rng(5)
    trials = np.unique(np.concatenate([[0, wl.n_trials - 1], rng.integers(0, wl.n_trials, 40)]))
    yo, g, omo = oracle_ylt(wl, trials, oracle.MODE_PLAIN, 21)
    if mode == oracle.MODE_PLAIN:
        assert_ylt_close(yd[trials], yo, g, f"{case} direct")
        assert_ylt_close(omd[trials], omo, g, f"{case} max occurrence")
    else:
        # the tabulated inverse is within 2e-4 of the FP64 quantile per draw
        assert np.all(np.abs(yd[trials] - yo) <= 2e-4 * g + 1e-3)
    P.ara_free_yet(eng.ctx, yh)


def test_hashed_prepared_batch_and_surrogate(eng):
    # prepared layers (the batch and serving path) and the surrogate kernel read the same tables
    torch = torch_cuda()
    wl = synth.custom(200, 120, 3000, 6, 200, 900, seed=19)
    yh = eng.load_yet(wl.yet(), wl.catalog_size)
    rng = np.random.default_rng(3)
    params = np.concatenate([rng.uniform(-0.3, 0.3, 192), rng.uniform(-0.1, 0.1, 64), rng.uniform(-0.2, 0.2, 4096),
                             rng.uniform(-0.1, 0.1, 64), rng.uniform(-0.05, 0.05, 64), [0.01]]).astype(np.float32)
    P.ara_surrogate_import(eng.ctx, params, mask=np.zeros(P.SUR_CELLS, dtype=np.uint8))
    outs = {}
    for kind in (P.TABLE_DIRECT, P.TABLE_HASHED):
        P.ara_set_table_kind(eng.ctx, kind)
        desc = eng.load_layer(wl.layers[0], wl.catalog_size)
        for mode in (P.MODE_PLAIN, P.MODE_SURROGATE):
            h = P.ara_prepare_layer(eng.ctx, desc, mode)
            out = torch.empty(wl.n_trials, device="cuda")
            P.ara_run_prepared(eng.ctx, yh, [h], [7], 0, wl.n_trials, [out])
            torch.cuda.synchronize()
            outs[(kind, mode)] = out.cpu().numpy()
            P.ara_free_layer(eng.ctx, h)
    P.ara_set_table_kind(eng.ctx, P.TABLE_DIRECT)
    for mode in (P.MODE_PLAIN, P.MODE_SURROGATE):
        assert np.array_equal(outs[(P.TABLE_DIRECT, mode)], outs[(P.TABLE_HASHED, mode)])
    with pytest.raises(P.AraError):
        P.ara_set_table_kind(eng.ctx, 2)
    P.ara_free_yet(eng.ctx, yh)


def _uncovered_event(layer, C):
    held = np.zeros(C, dtype=bool)
    for e in layer.elts:
        held[e.event_id] = True
    free = np.nonzero(~held)[0]
    assert free.size > 0
    return int(free[0])


def test_variable_length_trials_800_to_1500(eng):
    # Trials of U{800..1,500} occurrences (CSR) over the paper-scale layer.
    # The oracle takes them padded to the longest trial with an event that no
    # XELT of the layer holds: such an event draws nothing and adds a zero
    # occurrence loss, and padding at the end leaves every real slot's
    # counter (and so its random number) unchanged.
    torch = torch_cuda()
    wl, ev, offs = synth.paper_variable(n_trials=3000)
    lay = wl.layers[0]
    C = wl.catalog_size
    yh = eng.load_yet(ev, C, trial_offsets=offs)
    desc = eng.load_layer(lay, C)
    out = torch.empty(wl.n_trials, device="cuda")
    om = torch.empty(wl.n_trials, device="cuda")
    P.ara_run_layer_ex(eng.ctx, yh, desc, P.MODE_PLAIN, wl.seed, 0, wl.n_trials, out, om)
    torch.cuda.synchronize()
    y = out.cpu().numpy().astype(np.float64)
    lens = np.diff(offs)
    assert lens.min() >= 800 and lens.max() <= 1500
    pad = _uncovered_event(lay, C)
    rows = np.full((wl.n_trials, int(lens.max())), pad, dtype=np.int32)
    for i in range(wl.n_trials):
        rows[i, :lens[i]] = ev[offs[i]:offs[i + 1]]
    yo, g, omo = oracle.run_layer(lay, rows, np.arange(wl.n_trials), C, wl.seed, threads=0)
    worst = assert_ylt_close(y, yo, g, "variable-length trials")
    assert_ylt_close(om.cpu().numpy().astype(np.float64), omo, g, "max occurrence")
    assert 0.01 < np.mean(y == 0) < 0.6                  # the aggregate retention binds
    print(f"variable-length trials: worst |dY|/G = {worst:.3e}")
    # the hashed table over the same trials gives the same year losses
    P.ara_set_table_kind(eng.ctx, P.TABLE_HASHED)
    try:
        out2 = torch.empty(wl.n_trials, device="cuda")
        P.ara_run_layer(eng.ctx, yh, desc, P.MODE_PLAIN, wl.seed, out2)
        torch.cuda.synchronize()
    finally:
        P.ara_set_table_kind(eng.ctx, P.TABLE_DIRECT)
    assert np.array_equal(out2.cpu().numpy(), out.cpu().numpy())
    P.ara_free_yet(eng.ctx, yh)
