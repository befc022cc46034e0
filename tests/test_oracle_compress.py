"""Pins of the compression oracle (Sec. 4, steps 2-4) against what the definitions fix: brute
force over every representable value (dynamic precision), the exact helix of noise-free tracks
(residuals to the extrapolated track), the sorted order of the other clusters, decoding, the
range-ANS length bound and exhaustive optimal prefix codes (Huffman)."""
import dataclasses
import itertools
import math

import numpy as np
import pytest

import oracle
import synth
from oracle import compress as oc

P = synth.TRACKER_PARAMS


def _nearest_with_bits(v: int, n: int) -> int:
    """Brute force: the value with at most n + 1 significant bits nearest to v (ties upwards)."""
    if v == 0:
        return 0
    cands = {0}
    for p in range(0, 34):
        for m in range(1 << n, 1 << (n + 1)):
            if p <= n:
                cands.add(m >> (n - p) if p < n else m)
            else:
                cands.add(m << (p - n))
    best = None
    for c in sorted(cands):
        d = abs(c - v)
        if best is None or d < abs(best - v) or (d == abs(best - v) and c > best):
            best = c
    return best


@pytest.mark.parametrize("n", [3, 4])
def test_dynamic_precision_is_the_nearest_value_with_n_bits_after_the_leading_one(n):
    rng = np.random.default_rng(n)
    vals = list(range(0, 300)) + [int(v) for v in rng.integers(0, 65536, 400)] + [65535, 2 ** 20 + 12345]
    for v in vals:
        r = oc.dynprec(v, n)
        assert r == _nearest_with_bits(v, n), (v, r)
        c = oc.dynprec_code(r, n)
        assert oc.dynprec_decode(c, n) == r and c < 32 << (n + 1)
    assert oc.dynprec(0b101101, 3) == 0b101100 and oc.dynprec(0b111110, 3) == 0b1000000  # carry lengthens
    assert oc.dynprec(15, 3) == 15 and oc.dynprec(16, 3) == 16 and oc.dynprec(17, 3) == 18  # half up


def test_quantisation_and_zigzag():
    assert oc.quantise([0.0, 0.00375, 0.01125, -0.00375, 1.0], oc.INV_QY).tolist() == \
        [0, int(np.rint(np.float64(np.float32(0.00375)) * oc.INV_QY)), 2, 0, 133]
    v = np.arange(-1000, 1000)
    assert np.array_equal(oc.unzigzag(oc.zigzag(v)), v) and oc.zigzag(v).min() == 0
    assert oc.zigzag([0, -1, 1, -2]).tolist() == [0, 1, 2, 3]


def oracle_tracks(o, geom, ev):
    """The oracle's tracks in the tracker's output form (CSR hits in ascending rows, reference row
    = the innermost hit's, FP32 state there)."""
    t = oracle.tracks_for_flags(o, geom, ev.sector)
    return {"hit_offset": t["off"], "n_hits": t["nh"], "hit_ids": t["hits"], "sector": t["sector"],
            "row_ref": np.array([ev.row[t["hits"][a]] for a in t["off"]], dtype=np.int32),
            "x_ref": t["x_ref"], "state": t["state"]}


def _truth_tracks(ev, geom):
    """One track per leg with >= 10 clusters, state = the generator's exact state at its first
    (innermost) crossing, hits in ascending rows."""
    legs, counts = np.unique(ev.leg[ev.leg >= 0], return_counts=True)
    offs, nh, ids, sec, rref, xref, st = [], [], [], [], [], [], []
    o = 0
    for lg, c in zip(legs, counts):
        if c < 10:
            continue
        h = np.nonzero(ev.leg == lg)[0]
        h = h[np.argsort(ev.row[h])]
        i = h[0]
        ph, t, q = ev.exact["phi_loc"][i], ev.exact["dzds"][i], ev.exact["qpt"][i]
        s = math.sin(ph)
        if math.cos(ph) < 0:
            s, t, q = -s, -t, -q
        offs.append(o)
        nh.append(len(h))
        ids.append(h)
        sec.append(int(ev.sector[i]))
        rref.append(int(ev.row[i]))
        xref.append(float(geom["row_x"][ev.row[i]]))
        st.append([ev.exact["y_true"][i], ev.exact["z_true"][i], s, t, q])
        o += len(h)
    return {"hit_offset": np.array(offs), "n_hits": np.array(nh), "hit_ids": np.concatenate(ids),
            "sector": np.array(sec), "row_ref": np.array(rref), "x_ref": np.array(xref, dtype=np.float32),
            "state": np.array(st, dtype=np.float32)}


@pytest.mark.parametrize("seed", [21, 22])
def test_noise_free_residuals_to_the_exact_helix_vanish(seed):
    """sigma = 0 clusters and tracks carrying the generator's exact state: the extrapolated track
    passes through every cluster, so every residual is 0 or, at a rounding boundary, +-1."""
    w = dataclasses.replace(synth.sector_event(seed), pt_lo=0.5, sigma_y=0.0, sigma_z=0.0, eff=1.0,
                            noise_frac=0.0, phi_inset_deg=3.0)
    ev = synth.generate(w, want_exact=True)
    geom = synth.geometry(w)
    trk = _truth_tracks(ev, geom)
    q, sy, sz = synth.cluster_properties(ev)
    c = oc.compress(ev.y, ev.z, ev.row, ev.sector, q, sy, sz, geom, synth.BZ, trk)
    ry, rz = oc.unzigzag(c["streams"]["a_ry"]), oc.unzigzag(c["streams"]["a_rz"])
    assert c["n_attached"] == int(trk["n_hits"].sum()) and c["pred_fail"] == 0
    assert np.abs(ry).max() <= 1 and np.abs(rz).max() <= 1
    assert np.mean(ry == 0) > 0.99 and np.mean(rz == 0) > 0.99
    drow = oc.unzigzag(c["streams"]["a_drow"])
    assert np.all(drow >= 0) and np.all(drow[np.concatenate([[0], np.cumsum(trk["n_hits"])[:-1]])] == 0)


def test_round_trip_sorted_rows_and_entropy_reduction():
    """The oracle's own tracks on a one-sector event: decoding gives back every cluster's
    quantised position and dynamic-precision properties; the other clusters are stored in
    ascending (zq, yq) per row; residuals carry far less entropy than positions."""
    w = synth.SECTOR_EVENT
    ev = synth.generate(w)
    geom = synth.geometry(w)
    o = oracle.track(ev.y, ev.z, ev.row, ev.sector, geom, P, synth.BZ)
    trk = oracle_tracks(o, geom, ev)
    q, sy, sz = synth.cluster_properties(ev)
    c = oc.compress(ev.y, ev.z, ev.row, ev.sector, q, sy, sz, geom, synth.BZ, trk)
    assert c["n_attached"] + c["n_unattached"] + c["n_skipped"] == ev.n
    order = c["order"]
    assert np.array_equal(np.sort(order), np.arange(ev.n))
    d = oc.decompress(c["streams"], c["escapes"], trk, geom, synth.BZ)
    assert np.array_equal(d["sector"], ev.sector[order]) and np.array_equal(d["row"], ev.row[order])
    assert np.array_equal(d["yq"], c["yq"][order]) and np.array_equal(d["zq"], c["zq"][order])
    for k, v, n in (("q", q, 4), ("sy", sy, 3), ("sz", sz, 3)):
        assert np.array_equal(d[k], [oc.dynprec(int(x), n) for x in v[order]]), k
    u = order[c["n_attached"]:]
    key = ev.sector[u].astype(np.int64) * 1000 + ev.row[u]
    assert np.all(np.diff(key) >= 0)
    same = np.diff(key) == 0
    zq, yq = c["zq"][u], c["yq"][u]
    assert np.all((np.diff(zq) > 0) | ((np.diff(zq) == 0) & (np.diff(yq) >= 0)) | ~same)
    cnt = np.bincount(c["streams"]["a_ry"], minlength=oc.ALPHABET)
    raw = np.bincount(np.clip(c["yq"][order[:c["n_attached"]]] - c["yq"].min(), 0, None))
    assert oc.entropy_bits(cnt) < 0.6 * oc.entropy_bits(raw)


@pytest.mark.parametrize("dist", ["geometric", "uniform", "single", "two"])
@pytest.mark.parametrize("n", [0, 1, 4095, 4096, 4097, 20000])
def test_range_ans_round_trip_and_length_bound(dist, n):
    rng = np.random.default_rng(n + len(dist))
    if dist == "geometric":
        s = np.minimum(rng.geometric(0.15, n) - 1, oc.ESC)
    elif dist == "uniform":
        s = rng.integers(0, oc.ALPHABET, n)
    elif dist == "single":
        s = np.full(n, 7)
    else:
        s = rng.choice([3, 4000], n, p=[0.999, 0.001])
    s = s.astype(np.uint16)
    cnt = np.bincount(s, minlength=oc.ALPHABET)
    f = oc.ans_freqs(cnt)
    if n:
        assert f.sum() == 1 << oc.PROB_BITS and np.all(f[cnt > 0] >= 1) and np.all(f[cnt == 0] == 0)
    freq, words, per = oc.ans_encode(s, f)
    assert len(per) == -(-n // oc.BLOCK) and words.size == per.sum()
    assert np.array_equal(oc.ans_decode(words, per, n, freq), s)
    # state algebra: the state starts at 2^23 and ends in [2^23, 2^31) flushed as 32 bits, and one
    # coding step exceeds x 2^P / f by less than f / x <= 2^-9 relative, so the length is the ideal
    # code length plus 24..32 bits per block, within 2^-9 / ln 2 bits per symbol
    ideal = oc.ideal_ans_bits(s, freq)
    bits = 8 * words.size
    nb = len(per)
    slack = n * 2.0 ** -9 / math.log(2) + 1e-9
    assert ideal + 24 * nb - slack <= bits <= ideal + 32 * nb + slack, (bits, ideal, nb)


def _best_prefix_cost(counts):
    """Exhaustive: smallest sum(count * length) over complete prefix codes (Kraft sum 1)."""
    k = len(counts)
    best = None
    for lens in itertools.product(range(1, k), repeat=k):
        if abs(sum(2.0 ** -l for l in lens) - 1.0) < 1e-12:
            c = sum(a * b for a, b in zip(counts, lens))
            best = c if best is None else min(best, c)
    return best


@pytest.mark.parametrize("counts", [[5, 1], [1, 1, 1], [10, 3, 3, 1], [7, 7, 7, 7, 1], [40, 20, 10, 5, 3, 2],
                                    [1, 2, 3, 4, 5, 6]])
def test_huffman_lengths_are_optimal(counts):
    full = np.zeros(16, dtype=np.uint32)
    full[[1, 3, 5, 8, 11, 15][:len(counts)]] = counts
    bits, ln = oc.huffman_bits(full)
    assert bits == _best_prefix_cost(counts)
    assert oc.code_lengths_are_prefix_free(ln)
    ent = oc.entropy_bits(full)
    assert ent <= bits < ent + sum(counts)
