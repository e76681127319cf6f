"""Seeded synthetic workloads: the event sets and request traces that the tests
and the benchmark feed both to the HIP library and to the oracle.

This module holds none of the shower's arithmetic.  An event is fully named by
(seed, event id, sqrt(s), t_C, record capacity); every random number *inside*
an event is drawn by each implementation from its own Philox generator, keyed
by that name.  What is drawn here is only the input mix: per-event
centre-of-mass energies and cutoffs for the mixed batch, and the request trace
for serving.  NumPy's PCG64 is used for that, with fixed seeds.

The workloads follow the paper's LEP setup (Section 3: e+e- -> q qbar at
91.2 GeV, alpha_s(M_Z) = 0.118, t_C = 1 GeV^2, up to 10^6 events) and extend it
to uneven shower lengths (mixed energies and cutoffs), serving traffic and a
long-shower stress case.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


@dataclass(frozen=True)
class Workload:
    name: str
    n_events: int
    seed: int = 1
    first_event: int = 0
    ecm: float = 91.2          # GeV (used when per-event arrays are not drawn)
    tcut: float = 1.0          # GeV^2
    cap: int = 64              # partons per event record
    mixed: bool = False        # draw per-event sqrt(s), t_C
    form: str = "plain"
    description: str = ""

    def per_event(self, first: int = 0, count: int | None = None):
        """Per-event (sqrt(s), t_C) arrays, or (None, None) for a fixed point."""
        if not self.mixed:
            return None, None
        return mixed_energies(self.seed, self.n_events, first, count)


def mixed_energies(seed: int, n_events: int, first: int = 0, count: int | None = None):
    """sqrt(s) log-uniform in [10, 500] GeV and t_C uniform in [0.5, 4] GeV^2.

    The arrays for the whole batch are a fixed function of (seed, n_events);
    a slice [first, first+count) of the same batch is returned on request.
    """
    count = n_events - first if count is None else count
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([0x5EED, seed, n_events])))
    u = rng.random(n_events)
    v = rng.random(n_events)
    ecm = 10.0 * np.power(50.0, u)
    tcut = 0.5 + 3.5 * v
    return (np.ascontiguousarray(ecm[first:first + count]),
            np.ascontiguousarray(tcut[first:first + count]))


LEP_SMALL = Workload("lep_91.2GeV_tc1_1e3", 1_000, description="10^3 LEP events, cap 64 (oracle-sized)")
LEP = Workload("lep_91.2GeV_tc1_1e6", 1_000_000, description="10^6 LEP events at 91.2 GeV, t_C = 1 GeV^2, cap 64")
MIXED = Workload("mixed_10-500GeV_tc0.5-4_1e7", 10_000_000, cap=128, mixed=True, form="persistent",
                 description="10^7 events, sqrt(s) log-uniform [10,500] GeV, t_C uniform [0.5,4] GeV^2, cap 128")
STRESS = Workload("stress_500GeV_tc0.25_1e6", 1_000_000, ecm=500.0, tcut=0.25, cap=256,
                  description="10^6 events at 500 GeV, t_C = 0.25 GeV^2, cap 256")

WORKLOADS = {w.name: w for w in (LEP_SMALL, LEP, MIXED, STRESS)}


@dataclass
class Request:
    index: int
    arrival_s: float
    n_events: int
    ecm: float
    tcut: float
    seed: int
    cap: int = 128


@dataclass
class Trace:
    rate_hz: float
    requests: list = field(default_factory=list)

    @property
    def total_events(self) -> int:
        return sum(r.n_events for r in self.requests)


SERVING_ENERGIES = (10.0, 35.0, 91.2, 200.0, 500.0)
SERVING_CUTOFFS = (0.5, 1.0, 2.0)


def serving_trace(n_requests: int, rate_hz: float = 200.0, master_seed: int = 2026,
                  min_log10_n: float = 2.0, max_log10_n: float = 5.0) -> Trace:
    """Poisson arrivals at ``rate_hz``; N = 10^U with U uniform in
    [min_log10_n, max_log10_n]; sqrt(s) uniform over SERVING_ENERGIES;
    t_C uniform over SERVING_CUTOFFS; the request's Philox seed is
    1000 + its index in the trace."""
    rng = np.random.Generator(np.random.PCG64(master_seed))
    gaps = rng.exponential(1.0 / rate_hz, n_requests)
    arrivals = np.cumsum(gaps) - gaps[0]
    logn = rng.uniform(min_log10_n, max_log10_n, n_requests)
    ns = np.floor(np.power(10.0, logn)).astype(np.int64)
    ie = rng.integers(0, len(SERVING_ENERGIES), n_requests)
    it = rng.integers(0, len(SERVING_CUTOFFS), n_requests)
    reqs = [Request(index=i, arrival_s=float(arrivals[i]), n_events=int(ns[i]),
                    ecm=SERVING_ENERGIES[ie[i]], tcut=SERVING_CUTOFFS[it[i]], seed=1000 + i)
            for i in range(n_requests)]
    return Trace(rate_hz=rate_hz, requests=reqs)
