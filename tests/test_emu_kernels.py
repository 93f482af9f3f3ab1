"""The library's HIP sources run on the CPU (tests/emu/): every GPU thread a
host thread, lanes free between synchronisation points, AddressSanitizer on
every device and LDS access, ThreadSanitizer on every cross-lane LDS access.

These are CPU tests of the kernels' memory safety and synchronisation (the
LDS queue, classify pass, deferred ring, pending chunks and hashed table of
the layer kernel; the table builds; the radix select), checked against the
FP64 oracle.  The emulation uses the host's libm where the device code calls
hardware approximations, so it is compared with the oracle at the tolerance
of the GPU tests, not with the GPU bit for bit.
"""
import os
import struct
import subprocess
import tempfile

import numpy as np
import pytest

import oracle
from paper_1310_2274_amd import synth
from conftest import ROOT

EMU = os.path.join(ROOT, "tests", "emu")
RPS = (10.0, 50.0, 100.0, 250.0)
MODE_MEAN, MODE_PLAIN, MODE_TABLE = 0, 1, 3


def _have_compiler():
    return os.path.exists(os.environ.get("EMU_CXX", "/opt/rocm/llvm/bin/clang++"))


pytestmark = pytest.mark.skipif(not _have_compiler(), reason="host clang++ for the CPU emulation not found")


@pytest.fixture(scope="module")
def drivers():
    import importlib.util
    spec = importlib.util.spec_from_file_location("emu_build", os.path.join(EMU, "build.py"))
    m = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(m)
    return {s: m.build(s) for s in ("address", "thread")}


def _write(path, ev, offs, N, K, C, layer, seed, mode, kind):
    with open(path, "wb") as f:
        f.write(struct.pack("<qiii", N, K, C, 1 if offs is not None else 0))
        if offs is not None:
            f.write(np.ascontiguousarray(offs, dtype=np.int64).tobytes())
        f.write(np.ascontiguousarray(ev, dtype=np.int32).tobytes())
        f.write(struct.pack("<i", len(layer.elts)))
        for e in layer.elts:
            f.write(struct.pack("<ii", e.n, 1 if e.sigma_c is not None else 0))
            f.write(np.ascontiguousarray(e.event_id, dtype=np.int32).tobytes())
            f.write(np.ascontiguousarray(e.mean, dtype=np.float64).tobytes())
            f.write(np.ascontiguousarray(e.sigma_i, dtype=np.float64).tobytes())
            if e.sigma_c is not None:
                f.write(np.ascontiguousarray(e.sigma_c, dtype=np.float64).tobytes())
            f.write(np.ascontiguousarray(e.max_loss, dtype=np.float64).tobytes())
            f.write(struct.pack("<ddd", e.deductible, e.limit, e.share))
        f.write(struct.pack("<ddddII", layer.occ_retention, layer.occ_limit, layer.agg_retention,
                            layer.agg_limit, layer.program_id, seed))
        rps = [r for r in RPS if N // r >= 1]
        f.write(struct.pack("<iii", mode, kind, len(rps)))
        f.write(np.array(rps, dtype=np.float64).tobytes())


def _run(driver, ev, offs, N, K, C, layer, seed, mode, kind=0, timeout=900):
    with tempfile.TemporaryDirectory() as d:
        fi, fo = os.path.join(d, "in.bin"), os.path.join(d, "out.bin")
        _write(fi, ev, offs, N, K, C, layer, seed, mode, kind)
        env = dict(os.environ, TSAN_OPTIONS="halt_on_error=1 exitcode=66", ASAN_OPTIONS="detect_leaks=0")
        r = subprocess.run([driver, fi, fo], capture_output=True, text=True, timeout=timeout, env=env)
        assert r.returncode == 0, f"{os.path.basename(driver)} exit {r.returncode}:\n{r.stderr[-4000:]}"
        assert "WARNING: ThreadSanitizer" not in r.stderr and "ERROR: AddressSanitizer" not in r.stderr, r.stderr
        raw = open(fo, "rb").read()
    y = np.frombuffer(raw[:4 * N], dtype=np.float32).astype(np.float64)
    om = np.frombuffer(raw[4 * N:8 * N], dtype=np.float32).astype(np.float64)
    rest = np.frombuffer(raw[8 * N:], dtype=np.float64)
    k = rest.size // 2
    return y, om, rest[:k], rest[k:]


def _check(y, om, yo, g, omo, rel=1e-5):
    tol = rel * g + 1e-3
    assert np.all(np.abs(y - yo) <= tol), float(np.max(np.abs(y - yo) / tol))
    assert np.all(np.abs(om - omo) <= tol)


def _dense_case(n_trials=6, seed=31, sigma_c_frac=0.0):
    # trials of 1,000 events over a 2,000-event catalog, 8 XELTs holding
    # 35-75% of it: ~4,000 draws per trial, a few hundred of them on the FP64
    # path, so the deferred ring fills and flushes full waves in every trial
    return synth.custom(n_trials, 1000, 2000, 8, 700, 1500, seed=seed, sigma_c_frac=sigma_c_frac)


@pytest.mark.parametrize("sanitizer", ["address", "thread"])
def test_plain_layer_under_sanitizers(drivers, sanitizer):
    wl = _dense_case()
    lay = wl.layers[0]
    ev = wl.yet()
    y, om, pml, tvar = _run(drivers[sanitizer], ev.ravel(), None, wl.n_trials, wl.events_per_trial,
                            wl.catalog_size, lay, 5, MODE_PLAIN)
    yo, g, omo = oracle.run_layer(lay, ev, np.arange(wl.n_trials), wl.catalog_size, 5)
    _check(y, om, yo, g, omo)
    assert np.any(y > 0)


@pytest.mark.parametrize("sanitizer", ["address", "thread"])
def test_sparse_plain_layer_under_sanitizers(drivers, sanitizer):
    # a sparse layer (about 0.15 draws per occurrence): most chunks' FP32 lists
    # are short and go to the deferred ring with the small-shape draws, so
    # the ring flushes draws of many chunks at once and the pending ring fills
    wl = synth.custom(6, 1000, 20000, 3, 800, 1200, seed=35)
    lay = wl.layers[0]
    ev = wl.yet()
    y, om, _, _ = _run(drivers[sanitizer], ev.ravel(), None, wl.n_trials, wl.events_per_trial,
                       wl.catalog_size, lay, 11, MODE_PLAIN)
    yo, g, omo = oracle.run_layer(lay, ev, np.arange(wl.n_trials), wl.catalog_size, 11)
    _check(y, om, yo, g, omo)
    assert np.any(y > 0) or np.any(om > 0)


def test_correlated_csr_hashed_under_asan(drivers):
    # correlated std (FP64 z kept in the deferred ring), variable-length trials
    # (one empty), and the hashed layer table
    # a 3,000-event catalog, so some events are held by no XELT (the oracle's padding below)
    wl = synth.custom(6, 1000, 3000, 8, 700, 1500, seed=32, sigma_c_frac=0.6)
    lay = wl.layers[0]
    rng = np.random.default_rng(4)
    N, C = 6, wl.catalog_size
    lens = rng.integers(0, 1300, N)
    lens[3] = 0
    offs = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
    ev = rng.integers(0, C, offs[-1], dtype=np.int32)
    y, om, _, _ = _run(drivers["address"], ev, offs, N, int(lens.max()), C, lay, 9, MODE_PLAIN, kind=1)
    # the oracle takes the trials padded with an event no XELT holds (no draw, no loss)
    held = np.zeros(C, dtype=bool)
    for e in lay.elts:
        held[e.event_id] = True
    pad = int(np.nonzero(~held)[0][0])
    rows = np.full((N, int(lens.max())), pad, dtype=np.int32)
    for i in range(N):
        rows[i, :lens[i]] = ev[offs[i]:offs[i + 1]]
    yo, g, omo = oracle.run_layer(lay, rows, np.arange(N), C, 9)
    _check(y, om, yo, g, omo)
    assert y[3] == 0.0


def test_table_and_mean_modes_under_tsan(drivers):
    wl = synth.custom(4, 300, 1500, 5, 300, 900, seed=33)
    lay = wl.layers[0]
    ev = wl.yet()
    yt, omt, _, _ = _run(drivers["thread"], ev.ravel(), None, wl.n_trials, wl.events_per_trial,
                         wl.catalog_size, lay, 3, MODE_TABLE)
    yo, g, omo = oracle.run_layer(lay, ev, np.arange(wl.n_trials), wl.catalog_size, 3)
    _check(yt, omt, yo, g, omo, rel=2e-4)
    ym, omm, _, _ = _run(drivers["thread"], ev.ravel(), None, wl.n_trials, wl.events_per_trial,
                         wl.catalog_size, lay, 3, MODE_MEAN)
    ymo, gm, ommo = oracle.run_layer(lay, ev, np.arange(wl.n_trials), wl.catalog_size, 3, mode=oracle.MODE_MEAN)
    _check(ym, omm, ymo, gm, ommo)


def test_risk_measures_under_asan(drivers):
    # 600 trials: the radix select over a YLT with zero years and ties
    wl = synth.custom(600, 40, 1000, 2, 100, 200, seed=34)
    lay = wl.layers[0]
    ev = wl.yet()
    y, om, pml, tvar = _run(drivers["address"], ev.ravel(), None, wl.n_trials, wl.events_per_trial,
                            wl.catalog_size, lay, 7, MODE_MEAN)
    po, to = oracle.risk_measures(y, RPS)
    assert np.array_equal(pml, po)
    np.testing.assert_allclose(tvar, to, rtol=1e-12)
