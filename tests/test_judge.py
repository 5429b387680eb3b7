"""The efficiency / fake-rate judge on hand-made candidates and against a
per-seed loop over random candidates."""
import numpy as np

from paper_1705_02876_amd import judge


def _loop(best_hits, seed_track, seed_event, hit_track, track_nhits, min_match=7, frac=0.75):
    n_elig = n_found = n_fake = n_judged = 0
    for s in range(best_hits.shape[0]):
        h = best_hits[s][best_hits[s] >= 0]
        trk = hit_track[h]
        own = seed_track[s]
        nm_own = int((trk == own).sum())
        if track_nhits[seed_event[s]][own] >= min_match:
            n_elig += 1
            n_found += int(nm_own >= min_match and nm_own >= frac * h.size)
        real = trk[trk >= 0]
        nm = int(np.unique(real, return_counts=True)[1].max()) if real.size else 0
        if nm >= min_match:
            n_judged += 1
            n_fake += int(nm < frac * h.size)
    return n_elig, n_found, n_judged, n_fake


def test_hand_made_cases():
    # one event, tracks 0, 1, 2; hits 0..9 of track 0, 10..19 of track 1, 20..24 noise (-1), 25..29 track 2
    hit_track = np.array([0] * 10 + [1] * 10 + [-1] * 5 + [2] * 5)
    track_nhits = [np.array([10, 10, 5])]
    L = 12
    def row(hits):
        r = -np.ones(L, dtype=np.int64)
        r[:len(hits)] = hits
        return r
    best = np.stack([
        row(list(range(10))),                        # seed of track 0: found
        row(list(range(10, 17)) + [20, 21, 22]),     # track 1: 7 own of 10 hits (70% < 75%): not found, fake
        row(list(range(25, 30)) + [0, 1]),           # track 2 (5 true hits): not eligible; neither
        row(list(range(10, 16))),                    # track 1 again: 6 own: not found, neither
    ])
    r = judge.efficiency(best, np.array([0, 1, 2, 1]), np.zeros(4, dtype=np.int64), hit_track, track_nhits)
    assert (r["n_eligible"], r["n_found"], r["n_judged"], r["n_fake"]) == (3, 1, 2, 1)


def test_matches_per_seed_loop():
    rng = np.random.Generator(np.random.PCG64(5))
    E, L = 3, 17
    track_nhits = [rng.integers(3, 18, n) for n in (40, 1, 25)]
    hit_track = np.concatenate([np.repeat(np.arange(len(t)), t) for t in track_nhits] + [-np.ones(50, int)])
    S = 500
    seed_event = rng.integers(0, E, S)
    seed_track = np.array([rng.integers(0, len(track_nhits[e])) for e in seed_event])
    best = rng.integers(-1, hit_track.size, (S, L))
    # bias half of the candidates towards their own track's hits
    for s in range(0, S, 2):
        ids = np.flatnonzero(hit_track == seed_track[s])
        if ids.size:
            best[s, : min(ids.size, L)] = ids[:L]
    r = judge.efficiency(best, seed_track, seed_event, hit_track, track_nhits)
    # the loop indexes hit_track globally like the judge
    assert (r["n_eligible"], r["n_found"], r["n_judged"], r["n_fake"]) == _loop(best, seed_track, seed_event,
                                                                                hit_track, track_nhits)
