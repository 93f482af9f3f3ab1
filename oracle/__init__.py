"""FP64 CPU oracle for aggregate risk analysis with secondary uncertainty.

TEST INFRASTRUCTURE: only the tests, the smoke check and the benchmark's CPU
baseline leg import this package.  The product path (the HIP library and its
Python binding) never imports, loads or calls it, and the two share no code.

The arithmetic lives in ``ara_oracle.c`` (plain C, FP64, OpenMP over trials),
built with gcc by :func:`build`.  This module marshals arguments and adds the
risk measures of section 2.4, written directly from their definition:
k = floor(N / RP); PML is the k-th largest year loss, TVaR the mean of the
k largest (full sort, exactly rounded sum).
"""
from __future__ import annotations

import ctypes as C
import math
import os
import subprocess
from typing import Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "ara_oracle.c")
LIB = os.path.join(HERE, "libara_oracle.so")

MODE_MEAN = 0
MODE_PLAIN = 1
SIGMA_CLAMP = 0.999      # "a value very close to sigma_beta_max" (section 3.3)


def build(force: bool = True) -> str:
    if force or not os.path.exists(LIB):
        tmp = LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11",
                               "-Wall", "-Wextra", "-o", tmp, SRC, "-lm"])
        os.replace(tmp, LIB)
    return LIB


class _Elt(C.Structure):
    _fields_ = [("n", C.c_int32), ("event_id", C.c_void_p), ("mean", C.c_void_p),
                ("sigma_i", C.c_void_p), ("sigma_c", C.c_void_p), ("max_loss", C.c_void_p),
                ("deductible", C.c_double), ("limit", C.c_double), ("share", C.c_double)]


class _Terms(C.Structure):
    _fields_ = [("occ_retention", C.c_double), ("occ_limit", C.c_double),
                ("agg_retention", C.c_double), ("agg_limit", C.c_double)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        L = C.CDLL(LIB)
        L.orc_philox4x32_10.argtypes = [C.POINTER(C.c_uint32)] * 3
        L.orc_uniform.restype = C.c_double
        L.orc_uniform.argtypes = [C.c_uint32]
        L.orc_u_indep.restype = C.c_double
        L.orc_u_indep.argtypes = [C.c_uint32] * 5
        L.orc_u_corr.restype = C.c_double
        L.orc_u_corr.argtypes = [C.c_uint32] * 3
        L.orc_norm_quantile.restype = C.c_double
        L.orc_norm_quantile.argtypes = [C.c_double]
        L.orc_norm_cdf.restype = C.c_double
        L.orc_norm_cdf.argtypes = [C.c_double]
        L.orc_combine.restype = C.c_double
        L.orc_combine.argtypes = [C.c_double] * 4
        L.orc_beta_params.restype = C.c_int
        L.orc_beta_params.argtypes = [C.c_double] * 4 + [C.POINTER(C.c_double)] * 3
        L.orc_log_beta.restype = C.c_double
        L.orc_log_beta.argtypes = [C.c_double, C.c_double]
        L.orc_beta_inc.restype = C.c_double
        L.orc_beta_inc.argtypes = [C.c_double] * 3
        L.orc_beta_inc_inv.restype = C.c_double
        L.orc_beta_inc_inv.argtypes = [C.c_double] * 3 + [C.c_int, C.POINTER(C.c_int)]
        L.orc_beta_inc_inv_vec.restype = None
        L.orc_beta_inc_inv_vec.argtypes = [C.c_void_p] * 3 + [C.c_int64, C.c_int32, C.c_void_p, C.c_int32]
        L.orc_run_layer.restype = C.c_int
        L.orc_run_layer.argtypes = [C.c_void_p, C.c_void_p, C.c_int64, C.c_int32, C.c_int32,
                                    C.POINTER(_Elt), C.c_int32, C.POINTER(_Terms), C.c_uint32,
                                    C.c_uint32, C.c_int32, C.c_double, C.c_void_p, C.c_void_p,
                                    C.c_void_p, C.c_void_p, C.c_int32]
        L.orc_max_threads.restype = C.c_int
        _lib = L
    return _lib


# ---------------------------------------------------------------- primitives
def philox4x32_10(ctr: Sequence[int], key: Sequence[int]) -> tuple:
    c = (C.c_uint32 * 4)(*[int(v) & 0xFFFFFFFF for v in ctr])
    k = (C.c_uint32 * 2)(*[int(v) & 0xFFFFFFFF for v in key])
    o = (C.c_uint32 * 4)()
    lib().orc_philox4x32_10(c, k, o)
    return tuple(int(v) for v in o)


def uniform(w: int) -> float:
    return lib().orc_uniform(int(w) & 0xFFFFFFFF)


def u_indep(seed, program, trial, slot, elt) -> float:
    return lib().orc_u_indep(seed, program, trial, slot, elt)


def u_corr(seed, trial, slot) -> float:
    return lib().orc_u_corr(seed, trial, slot)


def norm_quantile(p: float) -> float:
    return lib().orc_norm_quantile(float(p))


def norm_cdf(v: float) -> float:
    return lib().orc_norm_cdf(float(v))


def combine(u_i, u_c, sigma_i, sigma_c) -> float:
    return lib().orc_combine(float(u_i), float(u_c), float(sigma_i), float(sigma_c))


def beta_params(mean, sigma, max_loss, clamp_c=SIGMA_CLAMP):
    a, b, m = C.c_double(), C.c_double(), C.c_double()
    deg = lib().orc_beta_params(float(mean), float(sigma), float(max_loss), float(clamp_c),
                                C.byref(a), C.byref(b), C.byref(m))
    return a.value, b.value, m.value, bool(deg)


def log_beta(a, b) -> float:
    return lib().orc_log_beta(float(a), float(b))


def beta_inc(x, a, b) -> float:
    return lib().orc_beta_inc(float(x), float(a), float(b))


def beta_inc_inv(u, a, b, pure_bisection: bool = False, return_iters: bool = False):
    it = C.c_int(0)
    x = lib().orc_beta_inc_inv(float(u), float(a), float(b), int(pure_bisection), C.byref(it))
    return (x, it.value) if return_iters else x


def beta_inc_inv_vec(u, a, b, pure_bisection=False, threads=0) -> np.ndarray:
    u = np.ascontiguousarray(u, dtype=np.float64)
    a = np.ascontiguousarray(np.broadcast_to(a, u.shape), dtype=np.float64)
    b = np.ascontiguousarray(np.broadcast_to(b, u.shape), dtype=np.float64)
    out = np.empty_like(u)
    lib().orc_beta_inc_inv_vec(u.ctypes.data, a.ctypes.data, b.ctypes.data, u.size,
                               int(pure_bisection), out.ctypes.data, int(threads))
    return out


def max_threads() -> int:
    return lib().orc_max_threads()


# ---------------------------------------------------------------- Algorithm 1
def run_layer(layer, yet_rows: np.ndarray, trial_ids: Sequence[int], catalog_size: int,
              seed: int, mode: int = MODE_PLAIN, threads: int = 0,
              clamp_c: float = SIGMA_CLAMP, program_id: Optional[int] = None, yelt: bool = False):
    """Year losses of ``layer`` for the given trials (FP64).

    Returns (ylt, gross, max_occ), each float64 [n_rows], and with yelt=True
    also the per-occurrence losses net of XELT and occurrence terms,
    float64 [n_rows][K].
    """
    yet_rows = np.ascontiguousarray(yet_rows, dtype=np.int32)
    tid = np.ascontiguousarray(trial_ids, dtype=np.int64)
    n_rows, K = yet_rows.shape
    assert tid.shape[0] == n_rows
    keep = []
    elts = (_Elt * max(1, len(layer.elts)))()
    for j, e in enumerate(layer.elts):
        arrs = [np.ascontiguousarray(e.event_id, dtype=np.int32),
                np.ascontiguousarray(e.mean, dtype=np.float64),
                np.ascontiguousarray(e.sigma_i, dtype=np.float64),
                None if e.sigma_c is None else np.ascontiguousarray(e.sigma_c, dtype=np.float64),
                np.ascontiguousarray(e.max_loss, dtype=np.float64)]
        keep.append(arrs)
        elts[j] = _Elt(e.n, arrs[0].ctypes.data, arrs[1].ctypes.data, arrs[2].ctypes.data,
                       None if arrs[3] is None else arrs[3].ctypes.data, arrs[4].ctypes.data,
                       float(e.deductible), float(e.limit), float(e.share))
    terms = _Terms(layer.occ_retention, layer.occ_limit, layer.agg_retention, layer.agg_limit)
    ylt = np.empty(n_rows)
    gross = np.empty(n_rows)
    omax = np.empty(n_rows)
    ye = np.zeros((n_rows, K)) if yelt else None
    prog = layer.program_id if program_id is None else program_id
    rc = lib().orc_run_layer(yet_rows.ctypes.data, tid.ctypes.data, n_rows, K, catalog_size,
                             elts, len(layer.elts), C.byref(terms), int(seed) & 0xFFFFFFFF,
                             int(prog) & 0xFFFFFFFF, int(mode), float(clamp_c),
                             ylt.ctypes.data, gross.ctypes.data, omax.ctypes.data,
                             None if ye is None else ye.ctypes.data, int(threads))
    if rc != 0:
        raise ValueError("event id outside the catalog")
    return (ylt, gross, omax, ye) if yelt else (ylt, gross, omax)


# ---------------------------------------------------------------- section 2.3
def yelt_increments(yelt: np.ndarray, agg_retention: float, agg_limit: float, lengths=None) -> np.ndarray:
    """Per-occurrence aggregate increments, from the definition: for each trial
    (row), S_k = sum of its occurrence losses o_0..o_k, A_k =
    min(max(S_k - AggR, 0), AggL) and the increment of occurrence k is
    A_k - A_{k-1} with A_{-1} = 0 (the aggregate terms act on the running sum,
    section 2.3).  ``lengths`` (optional) limits row i to its first lengths[i]
    occurrences; the rest of the row is left 0."""
    yelt = np.asarray(yelt, dtype=np.float64)
    out = np.zeros_like(yelt)
    for i in range(yelt.shape[0]):
        n = yelt.shape[1] if lengths is None else int(lengths[i])
        a_prev, s = 0.0, 0.0
        for k in range(n):
            s += yelt[i, k]
            a = min(max(s - agg_retention, 0.0), agg_limit)
            out[i, k] = a - a_prev
            a_prev = a
    return out


# ---------------------------------------------------------------- section 2.4
def risk_measures(ylt: np.ndarray, return_periods: Sequence[float]):
    """PML and TVaR at each return period RP, from the definition:
    k = floor(N/RP) (k >= 1 required); PML = k-th largest year loss;
    TVaR = mean of the k largest year losses."""
    y = np.sort(np.asarray(ylt, dtype=np.float64))[::-1]
    n = y.shape[0]
    pml, tvar = [], []
    for rp in return_periods:
        k = int(math.floor(n / float(rp)))
        if k < 1:
            raise ValueError("return period longer than the number of trials")
        pml.append(float(y[k - 1]))
        tvar.append(math.fsum(y[:k].tolist()) / k)
    return np.array(pml), np.array(tvar)
