"""Shared helpers of the GPU parity tests: run a workload through the C ABI and
compare with the FP64 oracle on the same seeded inputs."""
import numpy as np

import oracle
import paper_1310_2274_amd as P

# |Y_gpu - Y_oracle| <= REL_TOL * G_i + ABS_TOL per trial, with G_i the trial's
# share-weighted gross loss (sum over its draws of share * loss).  Every term
# and clamp of the method is 1-Lipschitz in the loss, so G_i bounds how far an
# error in any draw can move the year loss; relative to Y itself the check
# would be ill-posed where the retentions make Y much smaller than G.
REL_TOL = 1e-5
ABS_TOL = 1e-3


def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU test without a GPU"
    return torch


def gpu_ylt(eng, wl, mode, seed, layer=0, yet_handle=None, with_omax=False, t0=0, t1=None):
    torch = torch_cuda()
    if yet_handle is None:
        yet_handle = eng.load_yet(wl.yet(), wl.catalog_size)
    desc = eng.load_layer(wl.layers[layer], wl.catalog_size)
    t1 = wl.n_trials if t1 is None else t1
    out = torch.empty(t1 - t0, dtype=torch.float32, device="cuda")
    om = torch.empty(t1 - t0, dtype=torch.float32, device="cuda") if with_omax else None
    P.ara_run_layer_ex(eng.ctx, yet_handle, desc, mode, seed, t0, t1, out, om)
    torch.cuda.synchronize()
    res = out.cpu().numpy().astype(np.float64)
    if with_omax:
        return res, om.cpu().numpy().astype(np.float64), desc
    return res, desc


def oracle_ylt(wl, trials, mode, seed, layer=0, threads=0):
    trials = np.asarray(trials, dtype=np.int64)
    rows = wl.yet_rows(trials)
    return oracle.run_layer(wl.layers[layer], rows, trials, wl.catalog_size, seed, mode=mode, threads=threads)


def assert_ylt_close(y_gpu, y_orc, gross, what=""):
    y_gpu = np.asarray(y_gpu, dtype=np.float64)
    tol = REL_TOL * gross + ABS_TOL
    err = np.abs(y_gpu - y_orc)
    bad = np.nonzero(err > tol)[0]
    assert bad.size == 0, (f"{what}: {bad.size} trials outside tolerance; worst trial {bad[np.argmax(err[bad])]} "
                           f"gpu={y_gpu[bad[0]]!r} oracle={y_orc[bad[0]]!r} gross={gross[bad[0]]!r}")
    return float(np.max(err / np.maximum(gross, 1.0))) if err.size else 0.0
