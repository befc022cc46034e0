"""Pins of the oracle's grid, neighbour finder, cleaning, start hits, selection, and of the
whole chain on noise-free input."""
import dataclasses
import math

import numpy as np
import pytest

import oracle
import synth

P = synth.TRACKER_PARAMS


def geom(z_max=250.0, n_sectors=1):
    return dict(n_rows=synth.N_ROWS, row_x=synth.row_x(), tan_half=synth.tan_half(), n_sectors=n_sectors,
                z_min=0.0, z_max=z_max)


def brute_force_neighbours(y, z, row, prm):
    """Every (d, m, u) triplet, no grid: same window, cut and (D, id_u, id_d) order."""
    rx = synth.row_x().astype(np.float64)
    n = len(y)
    up = np.full(n, -1)
    dn = np.full(n, -1)
    vy = 1.5 * prm["sigma_y"] ** 2
    vz = 1.5 * prm["sigma_z"] ** 2
    for m in range(n):
        r = int(row[m])
        if r == 0 or r == synth.N_ROWS - 1:
            continue
        xm, xu, xd = rx[r], rx[r + 1], rx[r - 1]
        best = None
        for u in range(n):
            if row[u] != r + 1:
                continue
            if abs(float(y[u]) - float(y[m])) > prm["win_y"] * (xu - xm) or abs(float(z[u]) - float(z[m])) > prm["win_z"] * (xu - xm):
                continue
            for d in range(n):
                if row[d] != r - 1:
                    continue
                if abs(float(y[d]) - float(y[m])) > prm["win_y"] * (xm - xd) or abs(float(z[d]) - float(z[m])) > prm["win_z"] * (xm - xd):
                    continue
                w = (xm - xd) / (xu - xd)
                py = float(y[d]) + (float(y[u]) - float(y[d])) * w
                pz = float(z[d]) + (float(z[u]) - float(z[d])) * w
                D = (float(y[m]) - py) ** 2 / vy + (float(z[m]) - pz) ** 2 / vz
                if D > prm["nb_chi2_max"]:
                    continue
                key = (D, u, d)
                if best is None or key < best:
                    best = key
        if best is not None:
            up[m], dn[m] = best[1], best[2]
    return up, dn


@pytest.mark.parametrize("seed", range(6))
def test_neighbours_equal_exhaustive_triplets(seed):
    rng = np.random.default_rng(seed)
    rows = np.arange(10, 15)  # five rows
    n_per = rng.integers(3, 21, size=5)
    y, z, row = [], [], []
    for r, k in zip(rows, n_per):
        y += list(rng.uniform(-3, 3, size=k))
        z += list(rng.uniform(20, 26, size=k))
        row += [r] * k
    # hand-built exact ties: duplicated clusters (identical D, broken by id)
    for _ in range(4):
        i = rng.integers(0, len(y))
        y.append(y[i]); z.append(z[i]); row.append(row[i])
    y = np.array(y, dtype=np.float32); z = np.array(z, dtype=np.float32); row = np.array(row, dtype=np.uint8)
    perm = rng.permutation(len(y))
    y, z, row = y[perm], z[perm], row[perm]
    sector = np.zeros_like(row)
    for bins in ((8.0, 8.0), (0.7, 1.3)):
        prm = dict(P, bin_y=bins[0], bin_z=bins[1])
        res = oracle.track(y, z, row, sector, geom(), prm, synth.BZ, stages=oracle.STAGE_GRID | oracle.STAGE_NEIGHBOURS)
        bu, bd = brute_force_neighbours(y, z, row, prm)
        assert np.array_equal(res["up"], bu) and np.array_equal(res["dn"], bd)
    assert (bu >= 0).sum() > 0


def test_exact_tie_broken_by_lowest_ids():
    rx = synth.row_x()
    # middle hit, two identical upper candidates (ids 1, 3) and two identical lower ones (ids 2, 4)
    y = np.array([0.0, 0.05, -0.05, 0.05, -0.05], dtype=np.float32)
    z = np.array([50.0, 50.0, 50.0, 50.0, 50.0], dtype=np.float32)
    row = np.array([20, 21, 19, 21, 19], dtype=np.uint8)
    res = oracle.track(y, z, row, np.zeros(5, np.uint8), geom(), P, synth.BZ, stages=3)
    assert res["up"][0] == 1 and res["dn"][0] == 2
    assert res["nb_flag"][0] & oracle.F_ARGMIN


@pytest.fixture(scope="module")
def pbpb_small():
    w = synth.scaled(synth.PBPB_EVENT, 0.15)
    ev = synth.generate(w)
    return w, ev


def test_results_do_not_depend_on_bin_size(pbpb_small):
    w, ev = pbpb_small
    outs = []
    for by, bz in ((8.0, 8.0), (2.5, 3.0), (40.0, 120.0)):
        prm = dict(P, bin_y=by, bin_z=bz)
        outs.append(oracle.track(ev.y, ev.z, ev.row, ev.sector, synth.geometry(w), prm, synth.BZ, n_threads=4))
    a = outs[0]
    for b in outs[1:]:
        for k in ("up", "dn", "up_c", "dn_c", "start_id", "tl_nhits", "tl_hits", "trk_off", "trk_hits", "hit_key"):
            assert np.array_equal(a[k], b[k]), k
        assert np.array_equal(a["tl_state"], b["tl_state"])


def test_grid_is_sorted_by_sector_row_bin_id(pbpb_small):
    w, ev = pbpb_small
    res = oracle.track(ev.y, ev.z, ev.row, ev.sector, synth.geometry(w), P, synth.BZ, stages=oracle.STAGE_GRID)
    sid = res["sorted_id"]
    assert res["n_valid"] == ev.n and np.array_equal(np.sort(sid), np.arange(ev.n))
    rs = ev.sector[sid].astype(np.int64) * synth.N_ROWS + ev.row[sid]
    assert np.all(np.diff(rs) >= 0)
    assert np.array_equal(res["row_off"][rs], np.searchsorted(rs, rs, side="left"))
    # bin of each sorted hit from the CSR offsets, then ids ascending inside each bin
    b = np.searchsorted(res["bin_off"], np.arange(ev.n), side="right") - 1
    assert np.all(np.diff(b) >= 0)
    same = np.diff(b) == 0
    assert np.all(np.diff(sid.astype(np.int64))[same] > 0)
    # the bin of a hit matches the FP32 bin-index definition
    ny = np.maximum(1, np.ceil(2.0 * (synth.row_x() * synth.tan_half()).astype(np.float64) / P["bin_y"]).astype(np.int64))
    nz = int(max(1, math.ceil(w.z_max / P["bin_z"])))
    r = ev.row[sid]
    ymin = -(synth.row_x()[r] * synth.tan_half())
    vy = (ev.y[sid] - ymin) * np.float32(1.0 / P["bin_y"])
    vz = (ev.z[sid] - np.float32(0.0)) * np.float32(1.0 / P["bin_z"])
    iy = np.where(vy > 0, np.minimum(vy, ny[r] - 1), 0).astype(np.int64)
    iy = np.where(vy >= ny[r], ny[r] - 1, iy)
    iz = np.where(vz > 0, np.minimum(vz, nz - 1), 0).astype(np.int64)
    iz = np.where(vz >= nz, nz - 1, iz)
    assert np.array_equal(b - res["bin_base"][rs], iz * ny[r] + iy)


def test_cleaning_starts_selection_invariants(pbpb_small):
    w, ev = pbpb_small
    res = oracle.track(ev.y, ev.z, ev.row, ev.sector, synth.geometry(w), P, synth.BZ, n_threads=4)
    up, dn, uc, dc = res["up"], res["dn"], res["up_c"], res["dn_c"]
    n = ev.n
    # cleaning keeps exactly the reciprocal links
    for h in range(n):
        u = up[h]
        assert uc[h] == (u if (u >= 0 and dn[u] == h) else -1)
        d = dn[h]
        assert dc[h] == (d if (d >= 0 and up[d] == h) else -1)
    m = uc >= 0
    assert np.all(dc[uc[m]] == np.nonzero(m)[0])
    # starts: chain heads with >= l_min_chain hits, ascending id
    starts = []
    for h in range(n):
        if dc[h] >= 0:
            continue
        ln, c = 1, h
        while uc[c] >= 0:
            c = uc[c]; ln += 1
        if ln >= P["l_min_chain"]:
            starts.append(h)
    assert np.array_equal(res["start_id"], np.array(starts, dtype=np.uint32))
    # selection
    T = len(starts)
    key = np.zeros(n, dtype=np.uint64)
    keys = []
    for t in range(T):
        k = (np.uint64(res["tl_nhits"][t]) << np.uint64(32)) | np.uint64(0xFFFFFFFF - int(res["start_id"][t]))
        keys.append(k)
        if res["tl_valid"][t]:
            hs = res["tl_hits"][t][res["tl_hits"][t] >= 0]
            key[hs] = np.maximum(key[hs], k)
    assert np.array_equal(key, res["hit_key"])
    owner = np.full(n, -1)
    for k in range(res["n_tracks"]):
        hs = res["trk_hits"][res["trk_off"][k]:res["trk_off"][k + 1]]
        t = res["trk_tl"][k]
        assert hs.size >= P["n_min_track"]
        assert np.all(owner[hs] == -1)
        owner[hs] = k
        assert np.all(key[hs] == keys[t])
        full = res["tl_hits"][t][res["tl_hits"][t] >= 0]
        assert np.array_equal(hs, full[key[full] == keys[t]])
        assert np.all(np.diff(ev.row[hs].astype(int)) > 0)
    assert np.all(np.diff(res["trk_tl"]) > 0)


def _truth_state(ev, i):
    ph, t, q = ev.exact["phi_loc"][i], ev.exact["dzds"][i], ev.exact["qpt"][i]
    s = math.sin(ph)
    if math.cos(ph) < 0:
        s, t, q = -s, -t, -q
    return np.array([ev.exact["y_true"][i], ev.exact["z_true"][i], s, t, q])


@pytest.mark.parametrize("seed", [7, 8, 9])
def test_noise_free_exact_recovery(seed):
    """sigma = 0 clusters (fit errors kept nominal), full efficiency, no noise, pT >= 0.5, phi0 at least
    3 degrees inside the sector: exactly one track per findable leg, its exact hit set, truth state."""
    w = dataclasses.replace(synth.sector_event(seed), pt_lo=0.5, sigma_y=0.0, sigma_z=0.0, eff=1.0, noise_frac=0.0,
                            phi_inset_deg=3.0)
    ev = synth.generate(w, want_exact=True)
    res = oracle.track(ev.y, ev.z, ev.row, ev.sector, synth.geometry(w), P, synth.BZ)
    legs, counts = np.unique(ev.leg, return_counts=True)
    findable = {int(l) for l, c in zip(legs, counts) if c >= P["n_min_track"]}
    got = {}
    for k in range(res["n_tracks"]):
        hs = res["trk_hits"][res["trk_off"][k]:res["trk_off"][k + 1]]
        lg = np.unique(ev.leg[hs])
        assert lg.size == 1, "impure track"
        lg = int(lg[0])
        assert lg not in got, "clone"
        got[lg] = k
        assert np.array_equal(np.sort(hs), np.sort(np.nonzero(ev.leg == lg)[0])), "hit set differs"
        t = res["trk_tl"][k]
        inner = res["tl_hits"][t][res["tl_row_ref"][t]]
        truth = _truth_state(ev, inner)
        # Clusters are stored in FP32 (rounding up to 7.6e-6 cm at z = 250) and the fit keeps its weak
        # prior on (s, t, q/pT), so the state is exact up to a tiny fraction of its own error.
        sig = np.sqrt(np.diag(oracle.sym15_to_full(res["tl_cov"][t])))
        err = np.abs(res["tl_state"][t] - truth)
        assert np.all(err <= 1e-3 * sig), (err / sig)
        if hs.size >= 100:
            assert err[0] < 1e-5 and err[1] < 1e-5 and err[2] < 1e-6 and err[3] < 1e-6, err
            assert err[4] < 1e-5 * max(1.0, abs(truth[4])), err
    assert set(got) == findable


@pytest.mark.parametrize("seed", [11, 12])
def test_noise_free_loopers_are_pure(seed):
    w = dataclasses.replace(synth.sector_event(seed), pt_lo=0.06, pt_hi=0.4, sigma_y=0.0, sigma_z=0.0, eff=1.0,
                            noise_frac=0.0)
    ev = synth.generate(w)
    res = oracle.track(ev.y, ev.z, ev.row, ev.sector, synth.geometry(w), P, synth.BZ)
    assert res["n_tracks"] > 10
    for k in range(res["n_tracks"]):
        hs = res["trk_hits"][res["trk_off"][k]:res["trk_off"][k + 1]]
        assert np.unique(ev.leg[hs]).size == 1


def test_invalid_rows_and_sectors_are_ignored():
    y = np.array([0.0, 0.1, 0.2], dtype=np.float32)
    z = np.array([10.0, 10.0, 10.0], dtype=np.float32)
    row = np.array([10, 200, 11], dtype=np.uint8)
    sector = np.array([0, 0, 5], dtype=np.uint8)
    res = oracle.track(y, z, row, sector, geom(n_sectors=2), P, synth.BZ)
    assert res["n_valid"] == 1 and res["n_tracks"] == 0


def test_oracle_thread_count_does_not_change_results(pbpb_small):
    w, ev = pbpb_small
    a = oracle.track(ev.y, ev.z, ev.row, ev.sector, synth.geometry(w), P, synth.BZ, n_threads=1)
    b = oracle.track(ev.y, ev.z, ev.row, ev.sector, synth.geometry(w), P, synth.BZ, n_threads=7)
    for k in ("up", "dn", "nb_flag", "start_id", "tl_hits", "tl_state", "tl_cov", "tl_flag", "hit_key", "trk_hits"):
        assert np.array_equal(a[k], b[k]), k


def test_input_order_only_relabels_ids():
    """A seeded permutation of the input changes cluster ids (and so id tie-breaks) but, away from
    flagged near-ties, not which clusters form a track."""
    w = synth.scaled(synth.PBPB_EVENT, 0.05)
    a_ev = synth.generate(w)
    b_ev = synth.generate(dataclasses.replace(w, order=1))
    geom = synth.geometry(w)
    a = oracle.track(a_ev.y, a_ev.z, a_ev.row, a_ev.sector, geom, P, synth.BZ, n_threads=4)
    b = oracle.track(b_ev.y, b_ev.z, b_ev.row, b_ev.sector, geom, P, synth.BZ, n_threads=4)

    def track_sets(ev, r):
        key = ev.particle.astype(np.int64) * 1000 + ev.crossing  # identity of a cluster across orders
        key[ev.particle < 0] = -1 - np.arange((ev.particle < 0).sum())
        return {tuple(sorted(key[r["trk_hits"][r["trk_off"][k]:r["trk_off"][k + 1]]].tolist()))
                for k in range(r["n_tracks"])}

    sa, sb = track_sets(a_ev, a), track_sets(b_ev, b)
    assert len(sa ^ sb) <= 0.01 * len(sa), len(sa ^ sb)
