"""Physics judge of track building: efficiency and fake rate (host side, untimed).

Sec. 3.2 scores a candidate only when one simulated track supplies at least
seven of its hits; a candidate short of that is left out of both the
efficiency and the fake count.  The share of the candidate's hits that must
come from the matched track is not given there; 75% is used here.
"""
from __future__ import annotations

import numpy as np


def efficiency(best_hits, seed_track, seed_event, hit_track, track_nhits, min_match=7, frac=0.75):
    """best_hits: (S, L) global hit indices of each seed's best candidate (-1 = none).

    A seed's simulated track counts if it has >= min_match hits; it is found if
    the seed's best candidate has >= min_match hits from that track and they are
    >= frac of the candidate's hits.  A best candidate is a fake if its most
    frequent sim track contributes >= min_match hits but < frac of its hits;
    candidates whose most frequent track contributes fewer than min_match hits
    are neither found nor fake.
    Returns dict(eff, fake_rate, n_eligible, n_found, n_fake, n_judged).
    """
    best_hits = np.asarray(best_hits)
    S = best_hits.shape[0]
    if S == 0:
        return dict(eff=0.0, fake_rate=0.0, n_eligible=0, n_found=0, n_fake=0, n_judged=0)
    valid = best_hits >= 0
    trk = np.where(valid, np.asarray(hit_track)[np.where(valid, best_hits, 0)], -1)  # (S, L), -1 = none/noise
    own = np.asarray(seed_track)
    ev = np.asarray(seed_event)
    sizes = np.array([len(t) for t in track_nhits], dtype=np.int64)
    start = np.concatenate([[0], np.cumsum(sizes)[:-1]])
    ntrue = np.concatenate([np.asarray(t) for t in track_nhits])[start[ev] + own]
    nh = valid.sum(axis=1)
    nm_own = ((trk == own[:, None]) & valid).sum(axis=1)
    found = (nm_own >= min_match) & (nm_own >= frac * nh)
    elig = ntrue >= min_match
    # hits of each candidate's most frequent sim track (noise excluded)
    nm = np.zeros(S, dtype=np.int64)
    for j in range(trk.shape[1]):
        cj = ((trk == trk[:, j:j + 1]) & (trk[:, j:j + 1] >= 0)).sum(axis=1)
        nm = np.maximum(nm, cj)
    judged = nm >= min_match
    fake = judged & (nm < frac * nh)
    n_elig, n_found = int(elig.sum()), int((elig & found).sum())
    n_judged, n_fake = int(judged.sum()), int(fake.sum())
    return dict(eff=n_found / max(n_elig, 1), fake_rate=n_fake / max(n_judged, 1), n_eligible=n_elig,
                n_found=n_found, n_fake=n_fake, n_judged=n_judged)


def judge_problem(prob, best_hits):
    seed_event = np.repeat(np.arange(prob.n_events), np.diff(prob.seed_offsets))
    return efficiency(best_hits, prob.seed_track, seed_event, prob.hit_track, prob.track_nhits)
