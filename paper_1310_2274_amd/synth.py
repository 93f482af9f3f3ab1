"""Seeded synthetic inputs shaped like the paper's workloads.

This module only draws input tables; it holds none of the method's
arithmetic (no uniforms, quantiles, terms or sums of the simulation).  Both
the HIP path and the FP64 oracle receive the arrays it returns.

The paper's own data (a proprietary Year Event Table, extended event loss
tables for "a million locations", a reinsurance portfolio) is not public,
so every table here is synthetic, with the shapes the paper gives in
section 2.1 (trials of ~1,000 event occurrences, layers of 3-30 XELTs of
10k-30k entries, 1-10 programs) and the recipe stated next to each
function.

Recipe (master seed 1310, numpy PCG64 sub-streams derived per table):

* YET: i.i.d. uniform event IDs in [0, C), drawn with replacement, a fixed
  K events per trial.  Array order is time order (section 2.1 orders each
  trial by time stamp; the stamps themselves are never used).
* ELT j: n_j distinct event IDs (sampled without replacement), mean loss
  mu ~ LogNormal(10, 1.5), independent std sigma_I = mu * U(0.5, 1.5),
  correlated std sigma_C = 0, max exposure = mu * U(3, 10).
* Per-ELT terms: deductible U(0,1)*L0, limit U(5,50)*L0, share U(0.5,1),
  where L0 = e^10 is the median mean loss.
* Layer terms are sized from E = K * sum(n_j) / C, the expected number of
  (event, ELT) hits per trial, so that every clamp binds on a fraction of
  trials (values per workload below).  At paper scale the trial's cumulative
  occurrence loss S lies in about [1.07, 1.31] * E * L0 (oracle, 4,000
  trials: 10% quantile 1.126, 99.9% quantile 1.289), so the aggregate
  retention 1.12 * E * L0 zeroes about 8% of trials and the limit
  0.17 * E * L0 caps about 0.1% -- beyond the 250-year return period, so the
  PML/TVaR at 10-250 years are not all pinned to the limit.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Optional, Sequence

import numpy as np

L0 = math.exp(10.0)          # median of the LogNormal(10, 1.5) mean loss
MASTER_SEED = 1310
YET_BLOCK = 65536            # trials per independently seeded YET block


@dataclass
class ELT:
    """One extended event loss table (section 2.1) plus its financial terms I."""
    event_id: np.ndarray      # int32 [n], distinct, in [0, C)
    mean: np.ndarray          # float64 [n], mu_l > 0
    sigma_i: np.ndarray       # float64 [n], independent std
    sigma_c: Optional[np.ndarray]  # float64 [n] or None (= all zero)
    max_loss: np.ndarray      # float64 [n], max_l > mu_l
    deductible: float = 0.0
    limit: float = math.inf
    share: float = 1.0

    @property
    def n(self) -> int:
        return int(self.event_id.shape[0])


@dataclass
class Layer:
    """A layer: a set of XELTs plus occurrence/aggregate terms (section 2.1)."""
    elts: List[ELT]
    occ_retention: float
    occ_limit: float
    agg_retention: float
    agg_limit: float
    program_id: int = 0

    def expected_hits(self, events_per_trial: int, catalog_size: int) -> float:
        return events_per_trial * sum(e.n for e in self.elts) / catalog_size


@dataclass
class Workload:
    name: str
    n_trials: int
    events_per_trial: int
    catalog_size: int
    layers: List[Layer]
    seed: int = MASTER_SEED          # RNG key word of the simulation
    yet_seed: int = MASTER_SEED
    notes: str = ""
    _yet: Optional[np.ndarray] = field(default=None, repr=False)

    @property
    def trial_events(self) -> int:
        return self.n_trials * self.events_per_trial

    def yet(self) -> np.ndarray:
        """The whole YET, int32 [N, K] (generated once, cached)."""
        if self._yet is None:
            self._yet = make_yet(self.n_trials, self.events_per_trial,
                                 self.catalog_size, self.yet_seed)
        return self._yet

    def yet_rows(self, trials: Sequence[int]) -> np.ndarray:
        """Rows of the YET for selected trials, without drawing the rest."""
        if self._yet is not None:
            return self._yet[np.asarray(trials, dtype=np.int64)]
        return make_yet_rows(trials, self.n_trials, self.events_per_trial,
                             self.catalog_size, self.yet_seed)


def _rng(*key: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence(key[0], spawn_key=tuple(key[1:]))))


def _yet_block(seed: int, b: int, rows: int, K: int, C: int) -> np.ndarray:
    return _rng(seed, 1, b).integers(0, C, size=(rows, K), dtype=np.int32)


def make_yet(N: int, K: int, C: int, seed: int = MASTER_SEED) -> np.ndarray:
    out = np.empty((N, K), dtype=np.int32)
    for b in range((N + YET_BLOCK - 1) // YET_BLOCK):
        lo, hi = b * YET_BLOCK, min(N, (b + 1) * YET_BLOCK)
        out[lo:hi] = _yet_block(seed, b, YET_BLOCK, K, C)[: hi - lo]
    return out


def make_yet_rows(trials: Sequence[int], N: int, K: int, C: int, seed: int = MASTER_SEED) -> np.ndarray:
    trials = np.asarray(trials, dtype=np.int64)
    out = np.empty((trials.shape[0], K), dtype=np.int32)
    for b in np.unique(trials // YET_BLOCK):
        blk = _yet_block(seed, int(b), YET_BLOCK, K, C)
        sel = np.nonzero(trials // YET_BLOCK == b)[0]
        out[sel] = blk[trials[sel] - b * YET_BLOCK]
    return out


def make_elt(rng: np.random.Generator, C: int, n: int, sigma_c_frac: float = 0.0) -> ELT:
    ids = np.sort(rng.choice(C, size=n, replace=False)).astype(np.int32)
    mu = rng.lognormal(10.0, 1.5, size=n)
    sd = mu * rng.uniform(0.5, 1.5, size=n)
    mx = mu * rng.uniform(3.0, 10.0, size=n)
    sc = None
    if sigma_c_frac > 0.0:
        # split the std into an independent and a correlated part
        frac = rng.uniform(0.0, sigma_c_frac, size=n)
        sc = sd * frac
        sd = sd * (1.0 - frac)
    return ELT(event_id=ids, mean=mu, sigma_i=sd, sigma_c=sc, max_loss=mx,
               deductible=float(rng.uniform(0.0, 1.0) * L0),
               limit=float(rng.uniform(5.0, 50.0) * L0),
               share=float(rng.uniform(0.5, 1.0)))


def _elts(rng, C, count, lo, hi, sigma_c_frac=0.0):
    return [make_elt(rng, C, int(rng.integers(lo, hi + 1)), sigma_c_frac) for _ in range(count)]


def tiny(seed: int = MASTER_SEED) -> Workload:
    """1,000 trials x 100 events over a 10,000-event catalog; one layer of two
    ELTs with 2,000 entries each."""
    N, K, C = 1000, 100, 10000
    rng = _rng(seed, 2, 0)
    elts = [make_elt(rng, C, 2000) for _ in range(2)]
    E = K * sum(e.n for e in elts) / C
    lay = Layer(elts, occ_retention=L0, occ_limit=20 * L0,
                agg_retention=0.5 * E * L0, agg_limit=1.5 * E * L0)
    return Workload("tiny_1000x100_2elt", N, K, C, [lay], seed=seed, yet_seed=seed)


def paper_scale(n_trials: int = 800_000, seed: int = MASTER_SEED, sigma_c_frac: float = 0.0) -> Workload:
    """800,000 trials x 1,000 events over a 100,000-event catalog; one layer of
    16 ELTs with 20,000-50,000 entries each.  ``n_trials`` shrinks the YET
    only (same tables, same first trials).  ``sigma_c_frac`` > 0 moves a
    U(0, sigma_c_frac) share of each entry's std into the correlated part."""
    K, C = 1000, 100_000
    rng = _rng(seed, 2, 1)
    elts = _elts(rng, C, 16, 20_000, 50_000, sigma_c_frac)
    E = K * sum(e.n for e in elts) / C
    lay = Layer(elts, occ_retention=L0, occ_limit=20 * L0,
                agg_retention=1.12 * E * L0, agg_limit=0.17 * E * L0)
    return Workload(f"paper_{n_trials}x1000_16elt", n_trials, K, C, [lay], seed=seed, yet_seed=seed)


def random_layer(rng: np.random.Generator, C: int, K: int, max_elts: int, lo: int, hi: int,
                 program_id: int = 0) -> Layer:
    """A layer with a log-uniform ELT count in [1, max_elts] and randomised XL terms."""
    J = int(round(math.exp(rng.uniform(0.0, math.log(max_elts)))))
    elts = _elts(rng, C, max(1, J), lo, hi)
    E = K * sum(e.n for e in elts) / C
    return Layer(elts,
                 occ_retention=float(rng.uniform(0.5, 2.0) * L0),
                 occ_limit=float(rng.uniform(10.0, 40.0) * L0),
                 agg_retention=float(rng.uniform(0.5, 1.1) * E * L0),
                 agg_limit=float(rng.uniform(0.05, 1.0) * E * L0),
                 program_id=program_id)


def portfolio(n_layers: int = 64, n_trials: int = 200_000, seed: int = MASTER_SEED) -> Workload:
    """200,000 trials x 1,000 events over a 100,000-event catalog; 64 layers with
    log-uniform 1-40 ELTs of 5,000-50,000 entries and random XL terms."""
    K, C = 1000, 100_000
    rng = _rng(seed, 2, 3)
    layers = [random_layer(rng, C, K, 40, 5_000, 50_000, program_id=i % 10) for i in range(n_layers)]
    return Workload(f"portfolio_{n_layers}L_{n_trials}x1000", n_trials, K, C, layers, seed=seed, yet_seed=seed)


def correlated_portfolio(n_programs: int = 10, layers_per_program: int = 2, n_trials: int = 200_000,
                         sigma_c_frac: float = 0.6, seed: int = MASTER_SEED) -> Workload:
    """A portfolio of ``n_programs`` programs (section 2.1: up to 10), each of
    ``layers_per_program`` layers, over one YET of n_trials x 1,000 events and
    a 100,000-event catalog.  Every layer draws from the same pool of 24 ELTs
    (1-12 of them, log-uniform), so programs cover the same events; each entry
    carries a correlated std (a U(0, sigma_c_frac) share of its std), whose
    uniform z_(E) is shared by every program (section 3.1)."""
    K, C = 1000, 100_000
    rng = _rng(seed, 2, 6)
    pool = _elts(rng, C, 24, 10_000, 40_000, sigma_c_frac)
    layers = []
    for p in range(n_programs):
        for _ in range(layers_per_program):
            J = int(round(math.exp(rng.uniform(0.0, math.log(12)))))
            pick = sorted(rng.choice(len(pool), size=max(1, J), replace=False).tolist())
            elts = [pool[i] for i in pick]
            E = K * sum(e.n for e in elts) / C
            layers.append(Layer(elts,
                                occ_retention=float(rng.uniform(0.5, 2.0) * L0),
                                occ_limit=float(rng.uniform(10.0, 40.0) * L0),
                                agg_retention=float(rng.uniform(0.5, 1.1) * E * L0),
                                agg_limit=float(rng.uniform(0.05, 1.0) * E * L0),
                                program_id=p))
    return Workload(f"correlated_{n_programs}P_{n_trials}x1000", n_trials, K, C, layers, seed=seed, yet_seed=seed)


def variable_length_yet(N: int, kmin: int, kmax: int, C: int, seed: int = MASTER_SEED):
    """A YET of trials with U{kmin..kmax} events each (section 2.1: ~800-1,500
    occurrences per trial), ids uniform in [0, C), in CSR form: (event ids
    int32 [total], trial offsets int64 [N+1]).  Drawn in blocks of YET_BLOCK
    trials like the fixed-length YET."""
    lens = _rng(seed, 7, N, kmin, kmax).integers(kmin, kmax + 1, size=N)
    offs = np.zeros(N + 1, dtype=np.int64)
    np.cumsum(lens, out=offs[1:])
    ev = np.empty(int(offs[-1]), dtype=np.int32)
    for b in range((N + YET_BLOCK - 1) // YET_BLOCK):
        lo, hi = b * YET_BLOCK, min(N, (b + 1) * YET_BLOCK)
        ev[offs[lo]:offs[hi]] = _rng(seed, 8, b).integers(0, C, size=int(offs[hi] - offs[lo]), dtype=np.int32)
    return ev, offs


def paper_variable(n_trials: int = 800_000, kmin: int = 800, kmax: int = 1500, seed: int = MASTER_SEED):
    """The paper-scale layer (the same 16 ELTs as :func:`paper_scale`) over a
    YET of variable-length trials, U{kmin..kmax} events each, in CSR form.
    The aggregate terms are sized from the mean trial length.  Returns
    (workload, event ids, trial offsets); the workload's events_per_trial is
    the longest trial."""
    base = paper_scale(n_trials, seed)
    lay = base.layers[0]
    kmean = 0.5 * (kmin + kmax)
    E = kmean * sum(e.n for e in lay.elts) / base.catalog_size
    lay.agg_retention = 1.12 * E * L0
    lay.agg_limit = 0.17 * E * L0
    ev, offs = variable_length_yet(n_trials, kmin, kmax, base.catalog_size, seed)
    wl = Workload(f"paper_csr_{n_trials}x{kmin}-{kmax}_16elt", n_trials, kmax, base.catalog_size, [lay],
                  seed=seed, yet_seed=seed)
    return wl, ev, offs


def sparse_catalog(n_trials: int = 200_000, C: int = 20_000_000, n_elts: int = 16, lo: int = 20_000,
                   hi: int = 60_000, seed: int = MASTER_SEED) -> Workload:
    """A large catalog that the layer's XELTs cover only sparsely: n_trials x
    1,000 events over a 20,000,000-event catalog, one layer of 16 ELTs with
    20,000-60,000 entries (about 5% of the catalog), terms as at paper scale."""
    K = 1000
    rng = _rng(seed, 2, 7)
    elts = _elts(rng, C, n_elts, lo, hi)
    E = K * sum(e.n for e in elts) / C
    lay = Layer(elts, occ_retention=L0, occ_limit=20 * L0,
                agg_retention=0.5 * E * L0, agg_limit=1.5 * E * L0)
    return Workload(f"sparse_{n_trials}x1000_C{C}", n_trials, K, C, [lay], seed=seed, yet_seed=seed)


def serving_yet(n_trials: int = 1_000_000, seed: int = MASTER_SEED) -> Workload:
    """Resident YET for ad-hoc pricing: 1,000,000 trials x 1,000 events over a
    200,000-event catalog (requests come from :func:`pricing_request`)."""
    return Workload(f"serving_{n_trials}x1000", n_trials, 1000, 200_000, [], seed=seed, yet_seed=seed)


def pricing_request(req_seed: int, C: int = 200_000, K: int = 1000) -> Layer:
    """One ad-hoc pricing request: a layer of log-uniform 1-32 ELTs with
    10,000-60,000 entries each, lognormal losses and random XL terms."""
    rng = _rng(MASTER_SEED, 4, req_seed)
    return random_layer(rng, C, K, 32, 10_000, 60_000, program_id=int(req_seed % 10))


def custom(N: int, K: int, C: int, n_elts: int, lo: int, hi: int, seed: int = 7,
           sigma_c_frac: float = 0.0, terms: str = "binding") -> Workload:
    """Small workloads for tests: ``terms`` is 'binding' (every clamp can bind)
    or 'none' (pass-through terms)."""
    rng = _rng(seed, 5, N, K, C, n_elts)
    elts = _elts(rng, C, n_elts, lo, hi, sigma_c_frac)
    E = K * sum(e.n for e in elts) / C
    if terms == "none":
        for e in elts:
            e.deductible, e.limit, e.share = 0.0, math.inf, 1.0
        lay = Layer(elts, 0.0, math.inf, 0.0, math.inf)
    else:
        lay = Layer(elts, occ_retention=L0, occ_limit=20 * L0,
                    agg_retention=0.5 * E * L0, agg_limit=1.5 * E * L0)
    return Workload(f"custom_{N}x{K}_{n_elts}elt", N, K, C, [lay], seed=seed, yet_seed=seed)


WORKLOADS = {
    "tiny": tiny,
    "paper": paper_scale,
    "portfolio": portfolio,
}
