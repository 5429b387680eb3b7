"""The synthetic workloads (fixed seeds) used by the tests, the smoke check and the bench.

  small fit  : 1 000 tracks, 10 layers r = 4..40 cm, no material
  full fit   : 2 000 000 tracks, 17 layers r = 4..100 cm, 0.02 X0 per layer, 5% missing hits, >= 6 hits
  build      : events of U{5 000..20 000} tracks + 20% noise hits per layer, 64 phi x 16 eta bins, N = 6
  batched    : 64 events of log-uniform [1 000, 50 000] tracks, same detector and noise
All: pT ~ U[0.5, 10] GeV, eta ~ U[-1, 1], phi uniform, charge +-1, Bz = 3.8 T,
sigma_rphi = 0.01 cm, sigma_z = 0.1 cm, vertex at the origin.
"""
from __future__ import annotations

from . import synth as S

SEED_SMALL_FIT = S.BASE_SEED + 0
SEED_FULL_FIT = S.BASE_SEED + 1
SEED_BUILD = S.BASE_SEED + 2
SEED_BATCHED = S.BASE_SEED + 3


def small_fit(n=1000):
    return S.make_fit_problem(n, S.detector_small(), SEED_SMALL_FIT)


def fit_workload(det=None, n=2_000_000):
    det = det or S.detector_full()
    return S.make_fit_problem(n, det, SEED_FULL_FIT, p_miss=0.05, min_hits=6)


def build_workload(n_events=16, det=None):
    det = det or S.detector_full()
    sizes = S.uniform_event_sizes(SEED_BUILD, n_events)
    return S.make_build_problem(sizes, det, SEED_BUILD + 1000, p_miss=0.05, noise_frac=0.2)


def batched_workload(n_events=64, det=None):
    det = det or S.detector_full()
    sizes = S.loguniform_event_sizes(SEED_BATCHED, n_events)
    return S.make_build_problem(sizes, det, SEED_BATCHED + 1000, p_miss=0.05, noise_frac=0.2)
