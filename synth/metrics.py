"""Truth matching and rates for reconstructed tracks (host-side evaluation, not the method).

A *leg* is a maximal run of one particle's plane crossings inside one sector along which the
row index is monotonic (the generator assigns leg ids); a leg is *findable* with at least
``n_min`` clusters.  A track is labelled with the leg that contributes most of its hits
(ties: lowest leg id) and is *good* if that fraction is at least ``purity``.

efficiency = findable legs matched by >= 1 good track / findable legs
clone rate = (good tracks - distinct legs they match) / good tracks
fake rate  = tracks that are not good / all tracks
"""
from __future__ import annotations

import numpy as np


def match(leg: np.ndarray, trk_off: np.ndarray, trk_hits: np.ndarray, n_min: int = 10,
          purity: float = 0.9) -> dict:
    leg = np.asarray(leg)
    trk_off = np.asarray(trk_off, dtype=np.int64)
    trk_hits = np.asarray(trk_hits, dtype=np.int64)
    n_tracks = len(trk_off) - 1
    sig = leg >= 0
    legs, counts = np.unique(leg[sig], return_counts=True)
    findable = set(legs[counts >= n_min].tolist())
    good = 0
    matched = set()
    labels = np.full(n_tracks, -1, dtype=np.int64)
    for t in range(n_tracks):
        hl = leg[trk_hits[trk_off[t]:trk_off[t + 1]]]
        if hl.size == 0:
            continue
        v, c = np.unique(hl, return_counts=True)
        # most frequent, ties -> lowest leg id (np.unique sorts ascending; argmax picks first)
        best = int(np.argmax(c))
        lab = int(v[best])
        labels[t] = lab
        if lab >= 0 and c[best] >= purity * hl.size:
            good += 1
            matched.add(lab)
    eff_num = len(findable & matched)
    return dict(
        n_tracks=n_tracks, n_good=good, n_findable=len(findable), n_matched_findable=eff_num,
        efficiency=eff_num / max(1, len(findable)),
        clone_rate=(good - len(matched)) / max(1, good),
        fake_rate=(n_tracks - good) / max(1, n_tracks),
        labels=labels,
    )


def triplet_labels(leg: np.ndarray, crossing: np.ndarray, d: np.ndarray, m: np.ndarray, u: np.ndarray) -> np.ndarray:
    """1 iff d, m, u are consecutive crossings of the same leg (in either direction)."""
    ld, lm, lu = leg[d], leg[m], leg[u]
    cd, cm, cu = crossing[d], crossing[m], crossing[u]
    same = (lm >= 0) & (ld == lm) & (lu == lm)
    consec = ((cd == cm - 1) & (cu == cm + 1)) | ((cd == cm + 1) & (cu == cm - 1))
    return (same & consec).astype(np.uint8)
