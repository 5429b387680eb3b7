"""Physics judge of track building: efficiency and fake rate (host side, untimed).

Paper, Sec. 3.2: a candidate matching fewer than 7 hits of a simulated track
counts as neither a success nor a fake.  The fraction of a candidate's hits
that must come from the matched track is not stated; 75% is used here.
"""
from __future__ import annotations

import numpy as np


def efficiency(best_hits, seed_track, seed_event, hit_track, track_nhits, min_match=7, frac=0.75):
    """best_hits: (S, L) global hit indices of each seed's best candidate (-1 = none).

    A seed's simulated track counts if it has >= min_match hits; it is found if
    the seed's best candidate has >= min_match hits from that track and they are
    >= frac of the candidate's hits.  A best candidate is a fake if its most
    frequent sim track contributes >= min_match hits but < frac of its hits, or
    if it is matched to no track with >= min_match hits while having >=
    min_match hits itself; otherwise (fewer than min_match matched) neither.
    Returns dict(eff, fake_rate, n_eligible, n_found, n_fake, n_judged).
    """
    S = best_hits.shape[0]
    n_elig = n_found = n_fake = n_judged = 0
    for s in range(S):
        h = best_hits[s]
        h = h[h >= 0]
        trk = hit_track[h] if h.size else np.zeros(0, dtype=np.int64)
        own = seed_track[s]
        ntrue = track_nhits[seed_event[s]][own]
        nm_own = int((trk == own).sum())
        ok_own = nm_own >= min_match and nm_own >= frac * h.size
        if ntrue >= min_match:
            n_elig += 1
            n_found += int(ok_own)
        # fake / neither classification by the candidate's dominant sim track
        real = trk[trk >= 0]
        if real.size:
            vals, cnt = np.unique(real, return_counts=True)
            nm = int(cnt.max())
        else:
            nm = 0
        if nm >= min_match:
            n_judged += 1
            if nm < frac * h.size:
                n_fake += 1
    return dict(eff=n_found / max(n_elig, 1), fake_rate=n_fake / max(n_judged, 1), n_eligible=n_elig,
                n_found=n_found, n_fake=n_fake, n_judged=n_judged)


def judge_problem(prob, best_hits):
    seed_event = np.repeat(np.arange(prob.n_events), np.diff(prob.seed_offsets))
    return efficiency(best_hits, prob.seed_track, seed_event, prob.hit_track, prob.track_nhits)
