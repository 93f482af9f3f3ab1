"""MI355X (gfx950) aggregate risk analysis with secondary uncertainty.

Thin ctypes binding over ``libara.so`` (built from ``csrc/`` by ``_build.py``);
the functions carry the names of the C ABI in ``include/ara.h`` and only
marshal arguments: every step of the simulation runs in the library's HIP
kernels.  Arrays may be numpy arrays (host) or torch tensors (host or
device); torch supplies device memory and streams.

If the library is not built, :func:`lib` raises: there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import math
import os
from dataclasses import dataclass
from typing import Iterable, List, Optional, Sequence

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libara.so")

ARA_OK, ARA_E_INVAL, ARA_E_RANGE, ARA_E_NOMEM, ARA_E_BUDGET, ARA_E_DEVICE, ARA_E_STATE = 0, -1, -2, -3, -4, -5, -6
MODE_MEAN, MODE_PLAIN, MODE_SURROGATE, MODE_TABLE = 0, 1, 2, 3
TABLE_DIRECT, TABLE_HASHED = 0, 1
STATUS_NAMES = {0: "ARA_OK", -1: "ARA_E_INVAL", -2: "ARA_E_RANGE", -3: "ARA_E_NOMEM", -4: "ARA_E_BUDGET",
                -5: "ARA_E_DEVICE", -6: "ARA_E_STATE"}
DEFAULT_RETURN_PERIODS = (10.0, 50.0, 100.0, 250.0)


class AraError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")
        self.status = status
        self.message = message


class EltDesc(C.Structure):
    _fields_ = [("n_entries", C.c_int32), ("event_id", C.c_void_p), ("mean", C.c_void_p),
                ("sigma_i", C.c_void_p), ("sigma_c", C.c_void_p), ("max_loss", C.c_void_p),
                ("deductible", C.c_double), ("limit", C.c_double), ("share", C.c_double)]


class LayerDesc(C.Structure):
    _fields_ = [("n_elts", C.c_int32), ("elt_handles", C.POINTER(C.c_int32)),
                ("occ_retention", C.c_double), ("occ_limit", C.c_double),
                ("agg_retention", C.c_double), ("agg_limit", C.c_double), ("program_id", C.c_uint32)]


_lib = None


def lib() -> C.CDLL:
    """The loaded HIP library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_1310_2274_amd._build.build()")
        L = C.CDLL(LIB_PATH)
        vp, i32, i64, u32, u64, d = C.c_void_p, C.c_int32, C.c_int64, C.c_uint32, C.c_uint64, C.c_double
        sig = {
            "ara_create": (i32, [C.c_int, u64, C.POINTER(vp)]),
            "ara_destroy": (None, [vp]),
            "ara_last_error": (C.c_char_p, [vp]),
            "ara_bytes_in_use": (u64, [vp]),
            "ara_load_yet": (i32, [vp, vp, vp, i64, i32, i32, C.POINTER(i32)]),
            "ara_free_yet": (i32, [vp, i32]),
            "ara_load_elts": (i32, [vp, i32, C.POINTER(EltDesc), i32, C.POINTER(i32)]),
            "ara_free_elts": (i32, [vp, C.POINTER(i32), i32]),
            "ara_run_layer": (i32, [vp, i32, C.POINTER(LayerDesc), C.c_int, u32, vp, vp]),
            "ara_run_layer_ex": (i32, [vp, i32, C.POINTER(LayerDesc), C.c_int, u32, i64, i64, vp, vp, vp]),
            "ara_run_layer_yelt": (i32, [vp, i32, C.POINTER(LayerDesc), C.c_int, u32, i64, i64, vp, vp, vp, vp]),
            "ara_run_layers": (i32, [vp, i32, C.POINTER(LayerDesc), i32, C.c_int, u32, C.POINTER(vp), vp]),
            "ara_risk_measures": (i32, [vp, vp, i64, vp, i32, vp, vp, vp]),
            "ara_risk_measures_noalloc": (i32, [vp, vp, i64, vp, i32, vp, vp]),
            "ara_sum_ylts": (i32, [vp, C.POINTER(vp), i32, i64, vp, vp]),
            "ara_normal_quantile": (i32, [vp, vp, i64, vp]),
            "ara_philox_uniforms": (i32, [vp, vp, i64, u32, u32, vp, vp]),
            "ara_set_profiling": (i32, [vp, i32]),
            "ara_prepare_layer": (i32, [vp, C.POINTER(LayerDesc), C.c_int, C.POINTER(i32)]),
            "ara_set_trial_tile": (i32, [vp, C.c_int, i32]),
            "ara_set_table_kind": (i32, [vp, i32]),
            "ara_autotune": (i32, [vp, i32, C.POINTER(i32), i32, i64, C.POINTER(i32), vp]),
            "ara_free_layer": (i32, [vp, i32]),
            "ara_run_prepared": (i32, [vp, i32, C.POINTER(i32), i32, C.POINTER(u32), i64, i64, C.POINTER(vp),
                                       C.POINTER(vp), vp]),
            "ara_surrogate_train": (i32, [vp, i64, i32, i32, d, u32, vp]),
            "ara_surrogate_calibrate": (i32, [vp, i64, u32, d, vp, vp, vp]),
            "ara_surrogate_grad": (i32, [vp, vp, i32, vp, vp]),
            "ara_surrogate_tuples": (i32, [vp, i64, u32, vp]),
            "ara_surrogate_export": (i32, [vp, vp, vp, vp, vp, vp, vp]),
            "ara_surrogate_import": (i32, [vp, vp, vp, vp, i64, vp, vp]),
            "ara_surrogate_eval": (i32, [vp, vp, vp, vp, i64, vp, vp]),
            "ara_last_kernel_ms": (i32, [vp, C.POINTER(C.c_double)]),
            "ara_beta_quantile": (i32, [vp, vp, vp, vp, i64, vp, vp]),
            "ara_beta_quantile_layer": (i32, [vp, vp, vp, vp, i64, vp, vp]),
            "ara_beta_quantile_table": (i32, [vp, vp, vp, vp, i64, vp, vp]),
            "ara_yelt_increments": (i32, [vp, i32, i64, i64, d, d, vp, vp, vp]),
            "ara_elt_params": (i32, [vp, i32, vp, vp]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _ptr(x) -> Optional[int]:
    """Raw address of a numpy array or torch tensor (contiguous), or None."""
    if x is None:
        return None
    if hasattr(x, "data_ptr"):
        if not x.is_contiguous():
            raise ValueError("tensor must be contiguous")
        return x.data_ptr()
    if isinstance(x, np.ndarray):
        if not x.flags["C_CONTIGUOUS"]:
            raise ValueError("array must be C-contiguous")
        return x.ctypes.data
    raise TypeError(f"unsupported buffer type {type(x)}")


def _stream(stream, *bufs) -> Optional[int]:
    """hipStream_t for a call: the given stream, else torch's current stream
    when any buffer is a CUDA tensor (so torch work queued afterwards sees the
    result), else NULL (the null stream)."""
    if stream is None:
        for b in bufs:
            if getattr(b, "is_cuda", False):
                import torch
                return torch.cuda.current_stream(b.device).cuda_stream
        return None
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream)


def _check(ctx, status):
    if status != ARA_OK:
        msg = lib().ara_last_error(ctx)
        raise AraError(status, msg.decode() if msg else "")


# ---------------------------------------------------------------- C ABI names
def ara_create(device: int = 0, hbm_budget_bytes: int = 0):
    h = C.c_void_p()
    st = lib().ara_create(int(device), int(hbm_budget_bytes), C.byref(h))
    if st != ARA_OK:
        raise AraError(st, "ara_create failed")
    return h


def ara_destroy(ctx) -> None:
    lib().ara_destroy(ctx)


def ara_last_error(ctx) -> str:
    m = lib().ara_last_error(ctx)
    return m.decode() if m else ""


def ara_bytes_in_use(ctx) -> int:
    return int(lib().ara_bytes_in_use(ctx))


def ara_load_yet(ctx, event_ids, catalog_size: int, n_trials: Optional[int] = None,
                 events_per_trial: Optional[int] = None, trial_offsets=None) -> int:
    """event_ids: int32 [N, K] (fixed length) or flat int32 with trial_offsets int64 [N+1]."""
    if trial_offsets is not None:
        offs = np.ascontiguousarray(trial_offsets, dtype=np.int64)
        n_trials = offs.shape[0] - 1
        events_per_trial = 0
    else:
        offs = None
        if n_trials is None:
            n_trials, events_per_trial = int(event_ids.shape[0]), int(event_ids.shape[1])
    if isinstance(event_ids, np.ndarray):
        event_ids = np.ascontiguousarray(event_ids, dtype=np.int32)
    h = C.c_int32()
    _check(ctx, lib().ara_load_yet(ctx, _ptr(event_ids), None if offs is None else offs.ctypes.data,
                                   int(n_trials), int(events_per_trial), int(catalog_size), C.byref(h)))
    return h.value


def ara_free_yet(ctx, yet_handle: int) -> None:
    _check(ctx, lib().ara_free_yet(ctx, int(yet_handle)))


def ara_load_elts(ctx, catalog_size: int, elts: Sequence) -> List[int]:
    """elts: objects with event_id, mean, sigma_i, sigma_c (or None), max_loss,
    deductible, limit, share (see ``synth.ELT``)."""
    n = len(elts)
    keep = []
    descs = (EltDesc * max(1, n))()
    for j, e in enumerate(elts):
        arrs = [np.ascontiguousarray(e.event_id, dtype=np.int32), np.ascontiguousarray(e.mean, dtype=np.float64),
                np.ascontiguousarray(e.sigma_i, dtype=np.float64),
                None if e.sigma_c is None else np.ascontiguousarray(e.sigma_c, dtype=np.float64),
                np.ascontiguousarray(e.max_loss, dtype=np.float64)]
        keep.append(arrs)
        descs[j] = EltDesc(int(arrs[0].shape[0]), arrs[0].ctypes.data, arrs[1].ctypes.data, arrs[2].ctypes.data,
                           None if arrs[3] is None else arrs[3].ctypes.data, arrs[4].ctypes.data,
                           float(e.deductible), float(e.limit), float(e.share))
    handles = (C.c_int32 * max(1, n))()
    _check(ctx, lib().ara_load_elts(ctx, int(catalog_size), descs, n, handles))
    return [int(handles[j]) for j in range(n)]


def ara_free_elts(ctx, handles: Sequence[int]) -> None:
    arr = (C.c_int32 * max(1, len(handles)))(*handles)
    _check(ctx, lib().ara_free_elts(ctx, arr, len(handles)))


def layer_desc(handles: Sequence[int], occ_retention: float, occ_limit: float, agg_retention: float,
               agg_limit: float, program_id: int = 0):
    """Build an ara_layer_desc (the returned object keeps its handle array alive)."""
    arr = (C.c_int32 * len(handles))(*handles)
    d = LayerDesc(len(handles), arr, float(occ_retention), float(occ_limit), float(agg_retention),
                  float(agg_limit), int(program_id) & 0xFFFFFFFF)
    d._keep = arr
    return d


def ara_run_layer(ctx, yet_handle: int, layer: LayerDesc, mode: int, seed: int, ylt_out, stream=None) -> None:
    _check(ctx, lib().ara_run_layer(ctx, int(yet_handle), C.byref(layer), int(mode), int(seed) & 0xFFFFFFFF,
                                    _ptr(ylt_out), _stream(stream, ylt_out)))


def ara_run_layer_ex(ctx, yet_handle: int, layer: LayerDesc, mode: int, seed: int, trial_begin: int,
                     trial_end: int, ylt_out, max_occ_out=None, stream=None) -> None:
    _check(ctx, lib().ara_run_layer_ex(ctx, int(yet_handle), C.byref(layer), int(mode), int(seed) & 0xFFFFFFFF,
                                       int(trial_begin), int(trial_end), _ptr(ylt_out), _ptr(max_occ_out),
                                       _stream(stream, ylt_out, max_occ_out)))


def ara_run_layer_yelt(ctx, yet_handle: int, layer: LayerDesc, mode: int, seed: int, trial_begin: int,
                       trial_end: int, ylt_out, yelt_out, max_occ_out=None, stream=None) -> None:
    """Year losses plus the per-occurrence losses (YELT) in the YET's layout."""
    _check(ctx, lib().ara_run_layer_yelt(ctx, int(yet_handle), C.byref(layer), int(mode), int(seed) & 0xFFFFFFFF,
                                         int(trial_begin), int(trial_end), _ptr(ylt_out), _ptr(max_occ_out),
                                         _ptr(yelt_out), _stream(stream, ylt_out, max_occ_out, yelt_out)))


def ara_yelt_increments(ctx, yet_handle: int, trial_begin: int, trial_end: int, agg_retention: float,
                        agg_limit: float, yelt, inc_out=None, stream=None):
    """Per-occurrence aggregate increments A_k - A_{k-1} of a YELT (same layout)."""
    if isinstance(yelt, np.ndarray):
        yelt = np.ascontiguousarray(yelt, dtype=np.float32)
        if inc_out is None:
            inc_out = np.empty_like(yelt)
    elif inc_out is None:
        inc_out = yelt.new_empty(yelt.shape)
    _check(ctx, lib().ara_yelt_increments(ctx, int(yet_handle), int(trial_begin), int(trial_end),
                                          float(agg_retention), float(agg_limit), _ptr(yelt), _ptr(inc_out),
                                          _stream(stream, yelt, inc_out)))
    return inc_out


def ara_elt_params(ctx, elt_handle: int, n_entries: int):
    """(alpha, beta) of each entry of a loaded XELT, as the device derived them (0, 0 if degenerate)."""
    a = np.empty(int(n_entries))
    b = np.empty(int(n_entries))
    _check(ctx, lib().ara_elt_params(ctx, int(elt_handle), a.ctypes.data, b.ctypes.data))
    return a, b


def ara_normal_quantile(ctx, p) -> np.ndarray:
    """Phi^-1(p) on the device, as the correlated draws compute it (FP64, host arrays)."""
    p = np.ascontiguousarray(p, dtype=np.float64)
    x = np.empty_like(p)
    _check(ctx, lib().ara_normal_quantile(ctx, p.ctypes.data, int(p.size), x.ctypes.data))
    return x


def ara_sum_ylts(ctx, ylts, out, n_trials: Optional[int] = None, stream=None) -> None:
    """out[i] = sum of ylts[l][i] (FP64 accumulation); device tensors or raw device addresses."""
    n = len(ylts)
    arr = (C.c_void_p * n)(*[v if isinstance(v, int) else v.data_ptr() for v in ylts])
    nt = int(n_trials if n_trials is not None else out.shape[0])
    _check(ctx, lib().ara_sum_ylts(ctx, arr, n, nt, _ptr(out), _stream(stream, out, *[v for v in ylts if not isinstance(v, int)])))


def ara_run_layers(ctx, yet_handle: int, layers: Sequence[LayerDesc], mode: int, seed: int, ylt_outs,
                   stream=None) -> None:
    n = len(layers)
    arr = (LayerDesc * n)(*layers)
    outs = (C.c_void_p * n)(*[_ptr(o) for o in ylt_outs])
    _check(ctx, lib().ara_run_layers(ctx, int(yet_handle), arr, n, int(mode), int(seed) & 0xFFFFFFFF, outs,
                                     _stream(stream, *ylt_outs)))


def ara_prepare_layer(ctx, layer: LayerDesc, mode: int) -> int:
    h = C.c_int32()
    _check(ctx, lib().ara_prepare_layer(ctx, C.byref(layer), int(mode), C.byref(h)))
    return h.value


def ara_set_trial_tile(ctx, mode: int, wpb: int) -> None:
    _check(ctx, lib().ara_set_trial_tile(ctx, int(mode), int(wpb)))


def ara_autotune(ctx, yet_handle: int, layer_handles: Sequence[int], n_trials: int):
    """Pick the fastest trial tile for these prepared layers; returns (best, ms per candidate 1/2/4/8)."""
    n = len(layer_handles)
    hs = (C.c_int32 * n)(*layer_handles)
    best = C.c_int32()
    ms = np.full(4, np.nan, dtype=np.float32)
    _check(ctx, lib().ara_autotune(ctx, int(yet_handle), hs, n, int(n_trials), C.byref(best), ms.ctypes.data))
    return best.value, ms


def ara_free_layer(ctx, handle: int) -> None:
    _check(ctx, lib().ara_free_layer(ctx, int(handle)))


def ara_run_prepared(ctx, yet_handle: int, layer_handles: Sequence[int], seeds: Sequence[int], trial_begin: int,
                     trial_end: int, ylt_ptrs: Sequence[int], max_occ_ptrs=None, stream=None) -> None:
    """ylt_ptrs / max_occ_ptrs: raw device addresses (ints) or tensors, one per layer."""
    n = len(layer_handles)
    hs = (C.c_int32 * n)(*layer_handles)
    sd = (C.c_uint32 * n)(*[int(v) & 0xFFFFFFFF for v in seeds])
    to_addr = lambda v: v if isinstance(v, int) else _ptr(v)
    outs = (C.c_void_p * n)(*[to_addr(v) for v in ylt_ptrs])
    om = None if max_occ_ptrs is None else (C.c_void_p * n)(*[None if v is None else to_addr(v) for v in max_occ_ptrs])
    bufs = [v for v in ylt_ptrs if not isinstance(v, int)]
    _check(ctx, lib().ara_run_prepared(ctx, int(yet_handle), hs, n, sd, int(trial_begin), int(trial_end), outs, om,
                                       _stream(stream, *bufs)))


def ara_risk_measures(ctx, ylt, return_periods: Iterable[float] = DEFAULT_RETURN_PERIODS, n_trials=None,
                      stream=None):
    rps = np.ascontiguousarray(list(return_periods), dtype=np.float64)
    n = int(n_trials if n_trials is not None else (ylt.numel() if hasattr(ylt, "numel") else ylt.size))
    pml = np.empty(rps.shape[0])
    tvar = np.empty(rps.shape[0])
    if isinstance(ylt, np.ndarray):
        ylt = np.ascontiguousarray(ylt, dtype=np.float32)
    _check(ctx, lib().ara_risk_measures(ctx, _ptr(ylt), n, rps.ctypes.data, rps.shape[0], pml.ctypes.data,
                                        tvar.ctypes.data, _stream(stream, ylt)))
    return pml, tvar


def ara_risk_measures_noalloc(ctx, ylt, out, return_periods: Iterable[float] = DEFAULT_RETURN_PERIODS,
                              n_trials=None, stream=None):
    """PML/TVaR into the device tensor ``out`` (2 * len(return_periods) doubles:
    PML, TVaR per return period) with no allocation and no synchronisation."""
    rps = np.ascontiguousarray(list(return_periods), dtype=np.float64)
    n = int(n_trials if n_trials is not None else ylt.numel())
    _check(ctx, lib().ara_risk_measures_noalloc(ctx, _ptr(ylt), n, rps.ctypes.data, rps.shape[0], _ptr(out),
                                                _stream(stream, ylt, out)))


def ara_set_table_kind(ctx, kind: int) -> None:
    """Layer-table layout for later runs and prepared layers (TABLE_DIRECT or TABLE_HASHED)."""
    _check(ctx, lib().ara_set_table_kind(ctx, int(kind)))


def ara_set_profiling(ctx, enabled: bool) -> None:
    _check(ctx, lib().ara_set_profiling(ctx, int(bool(enabled))))


def ara_last_kernel_ms(ctx) -> float:
    ms = C.c_double()
    _check(ctx, lib().ara_last_kernel_ms(ctx, C.byref(ms)))
    return ms.value


SUR_PARAMS = 4481
SUR_CELLS = 4096


def ara_surrogate_train(ctx, n_tuples: int, epochs: int, batch: int = 4096, lr: float = 3e-3, seed: int = 1):
    losses = np.zeros(max(1, epochs))
    _check(ctx, lib().ara_surrogate_train(ctx, int(n_tuples), int(epochs), int(batch), float(lr),
                                          int(seed) & 0xFFFFFFFF, losses.ctypes.data))
    return losses[:epochs]


def ara_surrogate_calibrate(ctx, n_val: int, seed: int = 2, tol: float = 1e-3):
    cmax = np.zeros(SUR_CELLS, dtype=np.float32)
    cbias = np.zeros(SUR_CELLS, dtype=np.float32)
    nm = C.c_int32()
    _check(ctx, lib().ara_surrogate_calibrate(ctx, int(n_val), int(seed) & 0xFFFFFFFF, float(tol),
                                              cmax.ctypes.data, cbias.ctypes.data, C.byref(nm)))
    return cmax, cbias, nm.value


def ara_surrogate_grad(ctx, tuples):
    t = np.ascontiguousarray(tuples, dtype=np.float32)
    g = np.zeros(SUR_PARAMS, dtype=np.float32)
    loss = C.c_double()
    _check(ctx, lib().ara_surrogate_grad(ctx, t.ctypes.data, int(t.shape[0]), g.ctypes.data, C.byref(loss)))
    return g, loss.value


def ara_surrogate_tuples(ctx, n: int, seed: int):
    out = np.zeros((int(n), 5), dtype=np.float32)
    _check(ctx, lib().ara_surrogate_tuples(ctx, int(n), int(seed) & 0xFFFFFFFF, out.ctypes.data))
    return out


def ara_surrogate_export(ctx):
    P = np.zeros(SUR_PARAMS, dtype=np.float32)
    m = np.zeros(SUR_PARAMS, dtype=np.float32)
    v = np.zeros(SUR_PARAMS, dtype=np.float32)
    step = C.c_int64()
    mask = np.zeros(SUR_CELLS, dtype=np.uint8)
    bias = np.zeros(SUR_CELLS, dtype=np.float32)
    _check(ctx, lib().ara_surrogate_export(ctx, P.ctypes.data, m.ctypes.data, v.ctypes.data, C.byref(step),
                                           mask.ctypes.data, bias.ctypes.data))
    return {"params": P, "adam_m": m, "adam_v": v, "step": step.value, "mask": mask, "bias": bias}


def ara_surrogate_import(ctx, params, adam_m=None, adam_v=None, step: int = 1, mask=None, bias=None):
    P = np.ascontiguousarray(params, dtype=np.float32)
    m = None if adam_m is None else np.ascontiguousarray(adam_m, dtype=np.float32)
    v = None if adam_v is None else np.ascontiguousarray(adam_v, dtype=np.float32)
    k = None if mask is None else np.ascontiguousarray(mask, dtype=np.uint8)
    bb = None if bias is None else np.ascontiguousarray(bias, dtype=np.float32)
    _check(ctx, lib().ara_surrogate_import(ctx, P.ctypes.data, None if m is None else m.ctypes.data,
                                           None if v is None else v.ctypes.data, int(step),
                                           None if k is None else k.ctypes.data,
                                           None if bb is None else bb.ctypes.data))


def ara_surrogate_eval(ctx, a, b, u):
    a, b, u = (np.ascontiguousarray(np.broadcast_to(t, np.broadcast(a, b, u).shape), dtype=np.float64)
               for t in (np.asarray(a, np.float64), np.asarray(b, np.float64), np.asarray(u, np.float64)))
    x = np.zeros(u.shape[0])
    used = np.zeros(u.shape[0], dtype=np.int32)
    _check(ctx, lib().ara_surrogate_eval(ctx, a.ctypes.data, b.ctypes.data, u.ctypes.data, int(u.shape[0]),
                                         x.ctypes.data, used.ctypes.data))
    return x, used


def save_surrogate(ctx, path: str) -> None:
    """Checkpoint the surrogate (weights, Adam state, region table) as .npz."""
    st = ara_surrogate_export(ctx)
    np.savez(path, **{k: np.asarray(v) for k, v in st.items()})


def load_surrogate(ctx, path: str) -> None:
    with np.load(path, allow_pickle=False) as z:
        ara_surrogate_import(ctx, z["params"], z["adam_m"], z["adam_v"], int(z["step"]), z["mask"],
                             z["bias"] if "bias" in z.files else None)


def ara_philox_uniforms(ctx, ctr, key0: int, key1: int, out=None, stream=None):
    ctr = np.ascontiguousarray(ctr, dtype=np.uint32) if isinstance(ctr, np.ndarray) else ctr
    n = (ctr.shape[0] if ctr.ndim == 2 else ctr.shape[0] // 4)
    if out is None:
        out = np.empty(n, dtype=np.float32)
    _check(ctx, lib().ara_philox_uniforms(ctx, _ptr(ctr), int(n), int(key0) & 0xFFFFFFFF,
                                          int(key1) & 0xFFFFFFFF, _ptr(out), _stream(stream, ctr, out)))
    return out


def ara_beta_quantile_layer(ctx, a, b, u, out=None, stream=None):
    """The per-draw inverse as the plain layer kernel applies it."""
    return ara_beta_quantile(ctx, a, b, u, out, stream, _layer=True)


def ara_beta_quantile_table(ctx, a, b, u, out=None, stream=None):
    """The per-draw inverse of the table mode (per-entry tabulated inverse)."""
    return ara_beta_quantile(ctx, a, b, u, out, stream, _layer="table")


def ara_beta_quantile(ctx, a, b, u, out=None, stream=None, _layer=False):
    if isinstance(a, np.ndarray) or np.isscalar(a):
        a, b, u = np.broadcast_arrays(np.asarray(a, np.float64), np.asarray(b, np.float64), np.asarray(u, np.float64))
        a, b, u = (np.ascontiguousarray(v) for v in (a, b, u))
    n = int(u.shape[0])
    if out is None:
        out = np.empty(n, dtype=np.float64)
    fn = (lib().ara_beta_quantile_table if _layer == "table" else
          lib().ara_beta_quantile_layer if _layer else lib().ara_beta_quantile)
    _check(ctx, fn(ctx, _ptr(a), _ptr(b), _ptr(u), n, _ptr(out), _stream(stream, a, b, u, out)))
    return out


# ---------------------------------------------------------------- convenience
class Engine:
    """A context with loaded YETs/XELTs for synthetic workloads (``synth``)."""

    def __init__(self, device: int = 0, hbm_budget_bytes: int = 0):
        self.ctx = ara_create(device, hbm_budget_bytes)
        self.device = device

    def close(self):
        if self.ctx is not None:
            ara_destroy(self.ctx)
            self.ctx = None

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def load_yet(self, yet, catalog_size: int, trial_offsets=None) -> int:
        if trial_offsets is not None:
            return ara_load_yet(self.ctx, yet, catalog_size, trial_offsets=trial_offsets)
        return ara_load_yet(self.ctx, yet, catalog_size)

    def load_layer(self, layer, catalog_size: int, program_id: Optional[int] = None):
        handles = ara_load_elts(self.ctx, catalog_size, layer.elts)
        prog = layer.program_id if program_id is None else program_id
        return layer_desc(handles, layer.occ_retention, layer.occ_limit, layer.agg_retention, layer.agg_limit, prog)

    def run_layer(self, yet_h: int, desc, mode: int, seed: int, out, stream=None):
        ara_run_layer(self.ctx, yet_h, desc, mode, seed, out, stream)
        return out

    def risk_measures(self, ylt, rps=DEFAULT_RETURN_PERIODS, stream=None):
        return ara_risk_measures(self.ctx, ylt, rps, stream=stream)
