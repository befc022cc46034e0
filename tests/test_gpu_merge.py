"""Track merging and the merged refit on the GPU (Sec. 4) against the oracle: every track's helix and
its covariance, the merge labels (identical), and each merged track's refit (parameters within the
fit's convergence tolerance, chi2, covariance, ndf), on looper events, a Pb-Pb event with the GPU's
own tracks (sampled), malformed and empty track sets."""
import dataclasses
import sys

import numpy as np
import pytest

import oracle
import synth
from oracle import merge as om
from tests.test_gpu_flags import tracks_to_device

pytestmark = pytest.mark.gpu
P = synth.TRACKER_PARAMS


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    import torch

    assert torch.cuda.is_available()
    from paper_1910_12214_amd import tpcca

    c = tpcca.Context(0)
    yield c
    c.close()


def dev(a):
    import torch

    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


def looper_event(seed, sigma=0.0, n=60):
    w = dataclasses.replace(synth.sector_event(seed), only_sector=-1, phi_mode=1, pt_lo=0.06, pt_hi=0.4,
                            sigma_y=sigma, sigma_z=sigma, eff=1.0, noise_frac=0.0, mult_fixed=n)
    return w, synth.generate(w)


def oracle_track_set(ev, geom):
    """The oracle's tracks with their covariances rounded to FP32 (as the tracker stores them)."""
    o = oracle.track(ev.y, ev.z, ev.row, ev.sector, geom, P, synth.BZ)
    t = oracle.tracks_for_flags(o, geom, ev.sector)
    nt = int(o["n_tracks"])
    t["cov"] = np.asarray(o["tl_cov"][o["trk_tl"][:nt]], dtype=np.float32).reshape(-1, 15)
    d = tracks_to_device(t)
    ct = max(1, nt)
    cov = np.zeros((ct, 15), np.float32)
    cov[:nt] = t["cov"]
    d["cov"] = dev(cov)
    return t, d


def host(out, nt):
    return {k: out[k][:nt].cpu().numpy() for k in ("label", "n_members", "helix", "helix_cov", "theta", "theta_cov",
                                                   "chi2", "ndf")}


def check_refit(g, ids, hh, X, Y, Z, H, m, sy, sz):
    """GPU refit of component g against the oracle's: within the convergence tolerance.

    Both fits stop when a step lowers chi2 by at most 1e-12 of it, so each lies within about
    sqrt(2e-12 chi2) standard deviations of the minimum; 1e-4 sigma covers both."""
    th, cov, chi2, ndf, _ = om.refit(X[ids], Y[ids], Z[ids], H[g], sy, sz, hh)
    sig = np.sqrt(np.abs(np.diag(cov)))
    d = np.abs(m["theta"][g] - th)
    assert np.all(d <= 1e-4 * sig + 1e-9 * np.abs(th) + 1e-12), (g, d / sig)
    assert m["chi2"][g] == pytest.approx(chi2, rel=1e-6, abs=1e-9)
    assert int(m["ndf"][g]) == ndf
    ii, jj = np.tril_indices(5)
    assert np.allclose(m["theta_cov"][g], cov[ii, jj], rtol=1e-5, atol=1e-12 * np.abs(cov).max())


def full_check(ctx, ev, geom, t, d, sy, sz, mparams=None):
    nt = len(t["nh"])
    ten = [dev(a) for a in (ev.y, ev.z, ev.row, ev.sector)]
    out = ctx.merge(*ten, geom, synth.BZ, d, params=P, mparams=mparams)
    m = host(out, nt)
    H, CH = om.helix_params(t["state"], t["x_ref"], t["sector"], t["cov"].astype(np.float64), synth.BZ)
    scale = np.abs(H).max(axis=0)
    assert np.allclose(m["helix"], H, rtol=1e-10, atol=1e-11 * scale), np.abs(m["helix"] - H).max(axis=0)
    ii = np.tril_indices(5)
    ch = CH[:, ii[0], ii[1]]
    assert np.allclose(m["helix_cov"], ch, rtol=1e-8, atol=1e-12 * np.abs(ch).max())
    lab = om.merge_labels(H, CH)
    assert np.array_equal(m["label"], lab)
    roots, cnt = np.unique(lab, return_counts=True)
    assert np.array_equal(m["n_members"][roots], cnt)
    assert np.all(m["n_members"][np.setdiff1d(np.arange(nt), roots)] == 0)
    X, Y, Z = om.hit_points(ev.y, ev.z, ev.row, ev.sector, geom["row_x"])
    for g, n_mem in zip(roots, cnt):
        if n_mem < 2:  # only merged tracks are refit
            assert np.isnan(m["theta"][g]).all() and np.isnan(m["chi2"][g]) and m["ndf"][g] == 0
            continue
        mem = np.nonzero(lab == g)[0]
        ids = np.concatenate([t["hits"][t["off"][k]:t["off"][k] + t["nh"][k]] for k in mem])
        hh = np.concatenate([np.repeat(H[k:k + 1], t["nh"][k], axis=0) for k in mem])
        check_refit(g, ids, hh, X, Y, Z, H, m, sy, sz)
    c = out["counts"].cpu().numpy()
    assert c[0] == len(roots) and c[1] == int((cnt >= 2).sum()) and c[6] == 0
    return m, lab, c


@pytest.mark.parametrize("seed", [11, 12])
def test_noise_free_loopers_equal_oracle(ctx, seed):
    w, ev = looper_event(seed)
    geom = synth.geometry(w)
    t, d = oracle_track_set(ev, geom)
    m, lab, c = full_check(ctx, ev, geom, t, d, P["sigma_y"], P["sigma_z"])
    say(f"[merge] loopers seed {seed}: {len(lab)} tracks -> {c[0]} merged tracks ({c[1]} of several pieces); "
        f"{c[2]} pairs tested, {c[3]} passed, largest cell {c[4]}")


def test_smeared_loopers_equal_oracle(ctx):
    w, _ = looper_event(14, sigma=0.06, n=40)
    w = dataclasses.replace(w, sigma_z=0.1)
    ev = synth.generate(w)
    geom = synth.geometry(w)
    t, d = oracle_track_set(ev, geom)
    m, lab, c = full_check(ctx, ev, geom, t, d, 0.06, 0.1)
    say(f"[merge] smeared loopers: {len(lab)} tracks -> {c[0]}; chi2/ndf "
        f"{np.nansum(m['chi2']) / m['ndf'][m['ndf'] > 0].sum():.3f}")


def test_pair_queue_overflow_gives_the_same_merge(ctx):
    """Candidate pairs that do not fit the pair queue go through the rescan path: with no queue at
    all a looper event still equals the oracle, and on the Pb-Pb event's GPU tracks a queue of zero
    or one pair per track slot gives labels, refits and the count of tested pairs identical to the
    default queue's."""
    w, ev = looper_event(11)
    geom = synth.geometry(w)
    t, d = oracle_track_set(ev, geom)
    full_check(ctx, ev, geom, t, d, P["sigma_y"], P["sigma_z"], mparams={"pair_queue": 0})
    w = synth.PBPB_EVENT
    ev = synth.generate(w)
    geom = synth.geometry(w)
    ten = [dev(a) for a in (ev.y, ev.z, ev.row, ev.sector)]
    trk = ctx.track(*ten, geom, synth.BZ, P)
    nt = int(trk["counts"][0].item())
    out = ctx.merge(*ten, geom, synth.BZ, trk, params=P)
    ref, ref_c = host(out, nt), out["counts"].cpu().numpy()
    for q in (0, 1):
        out = ctx.merge(*ten, geom, synth.BZ, trk, params=P, mparams={"pair_queue": q})
        m, c = host(out, nt), out["counts"].cpu().numpy()
        for k in ref:
            assert np.array_equal(m[k], ref[k], equal_nan=m[k].dtype.kind == "f"), (q, k)
        assert c[2] == ref_c[2] and c[0] == ref_c[0] and c[1] == ref_c[1], (q, c, ref_c)
    say(f"[merge] pair queue 0 and 1: Pb-Pb event merge identical ({ref_c[2]} pairs tested)")


def sampled_merge_check(ctx, ev, geom, trk, n_samples, n_components, seed):
    """Merge the GPU's own tracks; check every track's helix against the oracle's, that every oracle
    partner of sampled tracks (searched by brute force over the tracks in its centre window) carries
    its label, and that sampled merged tracks are connected by the oracle's relation, labelled by
    their lowest member and refit as the oracle refits them."""
    from paper_1910_12214_amd import tpcca

    ten = [dev(a) for a in (ev.y, ev.z, ev.row, ev.sector)]
    h = tpcca.tracks_to_host(trk)
    nt = len(h["n_hits"])
    out = ctx.merge(*ten, geom, synth.BZ, trk, params=P)
    m = host(out, nt)
    cov = trk["cov"][:nt].cpu().numpy().astype(np.float64)
    H, CH = om.helix_params(h["state"], h["x_ref"], h["sector"], cov, synth.BZ)
    scale = np.abs(H).max(axis=0)
    assert np.allclose(m["helix"], H, rtol=1e-10, atol=1e-11 * scale)
    rng = np.random.default_rng(seed)
    ok = np.all(np.isfinite(H), axis=1) & (1.0 / H[:, 2] <= om.RHO_MAX)
    lab = m["label"]
    order = np.argsort(H[:, 0])  # tracks by Xc, for the window search
    xs = H[order, 0]
    for i in rng.choice(nt, n_samples, replace=False):
        if not ok[i]:
            assert lab[i] == i
            continue
        lo, hi = np.searchsorted(xs, H[i, 0] - om.CENTRE_WINDOW, "left"), np.searchsorted(xs, H[i, 0] + om.CENTRE_WINDOW, "right")
        near = order[lo:hi]
        near = near[ok[near] & (np.abs(H[near, 1] - H[i, 1]) <= om.CENTRE_WINDOW)]
        for j in near:
            if j != i:
                a, b = min(i, j), max(i, j)
                if om.compatible(H[a], CH[a], H[b], CH[b]):
                    assert lab[j] == lab[i], (i, j)
    roots = np.unique(lab)
    multi = roots[m["n_members"][roots] >= 2]
    X, Y, Z = om.hit_points(ev.y, ev.z, ev.row, ev.sector, geom["row_x"])
    for g in rng.choice(multi, min(n_components, len(multi)), replace=False):
        mem = np.nonzero(lab == g)[0]
        assert mem.min() == g
        # connected through the oracle's relation
        seen, todo = {mem[0]}, [mem[0]]
        while todo:
            a = todo.pop()
            for b in mem:
                if b not in seen and om.compatible(H[min(a, b)], CH[min(a, b)], H[max(a, b)], CH[max(a, b)]):
                    seen.add(b)
                    todo.append(b)
        assert len(seen) == len(mem), g
        ids = np.concatenate([h["hit_ids"][h["hit_offset"][k]:h["hit_offset"][k] + h["n_hits"][k]] for k in mem])
        hh = np.concatenate([np.repeat(H[k:k + 1], h["n_hits"][k], axis=0) for k in mem])
        check_refit(g, ids, hh, X, Y, Z, H, m, P["sigma_y"], P["sigma_z"])
    return nt, out["counts"].cpu().numpy()


def test_pbpb_event_gpu_tracks_sampled(ctx):
    """The full Pb-Pb event with the GPU's own tracks (sampled checks, see sampled_merge_check)."""
    w = synth.PBPB_EVENT
    ev = synth.generate(w)
    geom = synth.geometry(w)
    trk = ctx.track(*[dev(a) for a in (ev.y, ev.z, ev.row, ev.sector)], geom, synth.BZ, P)
    nt, c = sampled_merge_check(ctx, ev, geom, trk, 200, 40, 5)
    say(f"[merge] Pb-Pb event: {nt} tracks -> {c[0]} ({c[1]} of several pieces), {c[2]} pairs tested, "
        f"{c[3]} passed, largest cell {c[4]}, refits failed {c[6]}")


def test_pbpb_timeframe_gpu_tracks_sampled(ctx):
    """The full 570-collision Pb-Pb frame (72.8M clusters) tracked in one launch, its 1.27M tracks
    merged: sampled checks against the oracle, including cells too long for LDS."""
    w = synth.PBPB_TIMEFRAME
    ev = synth.generate(w)
    geom = synth.geometry(w)
    ten = [dev(a) for a in (ev.y, ev.z, ev.row, ev.sector)]
    trk = ctx.alloc_tracks(ev.n // 8, ev.n)
    ctx.set_tuning(dict(bin_y=8.0, bin_z=8.0, tracklet_chunk=1, blocks_per_cu=6, waves_per_simd=3))
    ctx.track(*ten, geom, synth.BZ, P, out=trk, timeframe=True)
    ctx.set_tuning(None)
    nt, c = sampled_merge_check(ctx, ev, geom, trk, 100, 20, 7)
    assert c[5] >= 1  # some cells exceeded the LDS sort
    say(f"[merge] Pb-Pb frame: {nt} tracks -> {c[0]} ({c[1]} of several pieces), {c[2]} pairs tested, "
        f"{c[3]} passed, largest cell {c[4]} ({c[5]} cells sorted in global memory), refits failed {c[6]}")


def test_malformed_and_empty_track_sets(ctx):
    import torch

    from paper_1910_12214_amd import tpcca

    w, ev = looper_event(13)
    geom = synth.geometry(w)
    t, d = oracle_track_set(ev, geom)
    nt = len(t["nh"])
    ten = [dev(a) for a in (ev.y, ev.z, ev.row, ev.sector)]
    # a track with a cluster id out of range and one with a NaN state: singletons without a fit
    hits = t["hits"].copy()
    hits[t["off"][2] + 1] = ev.n + 7
    state = np.asarray(t["state"], np.float32).copy()
    state[5, 2] = np.nan
    t2 = dict(t, hits=hits, state=state)
    d2 = tracks_to_device(t2)
    d2["cov"] = d["cov"]
    m = host(ctx.merge(*ten, geom, synth.BZ, d2, params=P), nt)
    for k in (2, 5):
        assert m["label"][k] == k and m["n_members"][k] == 1 and np.isnan(m["theta"][k]).all() and m["ndf"][k] == 0
    # the others: the oracle's labels with tracks 2 and 5 left out
    H, CH = om.helix_params(t["state"], t["x_ref"], t["sector"], t["cov"].astype(np.float64), synth.BZ)
    H[[2, 5]] = np.nan
    assert np.array_equal(m["label"], om.merge_labels(H, CH))
    # no tracks
    trk = ctx.alloc_tracks(16, 16)
    out = ctx.merge(*ten, geom, synth.BZ, trk, params=P)
    assert out["counts"].cpu().numpy()[0] == 0
    # argument errors
    small = ctx.alloc_merged(8)
    with pytest.raises(tpcca.TpcError):
        ctx.merge(*ten, geom, synth.BZ, d, params=P, out=small)
    with pytest.raises(tpcca.TpcError):
        ctx.merge(*ten, geom, synth.BZ, d, params=P, mparams={"sectors_per_side": 9})
    torch.cuda.synchronize()


def test_cell_longer_than_the_lds_sort(ctx):
    """4500 tracks with one helix centre (one cell, sorted in global memory): pairs of identical
    tracks, the pairs 50 cm apart in z with zero pitch, so exactly the pairs merge."""
    import torch

    w = synth.SECTOR_EVENT
    ev = synth.generate(w)
    geom = dict(synth.geometry(w), z_max=120000.0)
    n2 = 2250
    nt = 2 * n2
    state = np.tile(np.array([0.0, 0.0, 0.2, 0.0, 2.0], np.float32), (nt, 1))
    state[:, 1] = np.repeat(50.0 * np.arange(n2, dtype=np.float32), 2)
    cov = np.zeros((nt, 15), np.float32)
    cov[:, [0, 2, 5, 9, 14]] = [0.01, 0.01, 1e-6, 1e-6, 1e-4]
    hits = np.tile(np.arange(10, dtype=np.int32), nt)
    t = {"off": (10 * np.arange(nt)).astype(np.int32), "nh": np.full(nt, 10, np.int32), "hits": hits,
         "sector": np.zeros(nt, np.int32), "x_ref": np.full(nt, 100.0, np.float32), "state": state}
    d = tracks_to_device(t)
    d["cov"] = dev(cov)
    ten = [dev(a) for a in (ev.y, ev.z, ev.row, ev.sector)]
    out = ctx.merge(*ten, geom, synth.BZ, d, params=P)
    lab = out["label"][:nt].cpu().numpy()
    c = out["counts"].cpu().numpy()
    assert c[4] == nt and c[5] == 1, c
    assert np.array_equal(lab, np.repeat(2 * np.arange(n2), 2))
    H, CH = om.helix_params(state, t["x_ref"], t["sector"], cov.astype(np.float64), synth.BZ)
    for i in (0, 1000, 4498):  # the oracle's relation on samples: a pair merges, neighbours do not
        assert om.compatible(H[i], CH[i], H[i + 1], CH[i + 1])
        if i + 2 < nt:
            assert not om.compatible(H[i], CH[i], H[i + 2], CH[i + 2])
    torch.cuda.synchronize()
    say(f"[merge] one cell of {nt} tracks: {c[0]} merged tracks")


def test_large_component_is_deterministic(ctx):
    """300 copies of one track form one merged track (its members sorted by the workgroup path for
    components beyond 64 members): labels, member count, and a refit bit-identical between runs."""
    import torch

    w = synth.SECTOR_EVENT
    ev = synth.generate(w)
    geom = synth.geometry(w)
    nt = 300
    state = np.tile(np.array([1.5, 40.0, 0.2, 0.3, 2.0], np.float32), (nt, 1))
    cov = np.zeros((nt, 15), np.float32)
    cov[:, [0, 2, 5, 9, 14]] = [0.01, 0.01, 1e-6, 1e-6, 1e-4]
    t = {"off": (10 * np.arange(nt)).astype(np.int32), "nh": np.full(nt, 10, np.int32),
         "hits": np.tile(np.arange(10, dtype=np.int32), nt), "sector": np.zeros(nt, np.int32),
         "x_ref": np.full(nt, 100.0, np.float32), "state": state}
    d = tracks_to_device(t)
    d["cov"] = dev(cov)
    ten = [dev(a) for a in (ev.y, ev.z, ev.row, ev.sector)]
    r1 = host(ctx.merge(*ten, geom, synth.BZ, d, params=P), nt)
    r2 = host(ctx.merge(*ten, geom, synth.BZ, d, params=P), nt)
    assert np.all(r1["label"] == 0) and r1["n_members"][0] == nt
    for k in ("theta", "theta_cov", "chi2"):
        assert np.array_equal(r1[k], r2[k], equal_nan=True), k
    assert r1["ndf"][0] == 2 * 10 * nt - 5
    torch.cuda.synchronize()


def test_overlapping_hit_lists_get_no_fit(ctx):
    """300 copies of one track that all point at the same ten hit entries (overlapping hit lists,
    which the tracker never writes): they merge into one track whose hits exceed the track set's hit
    capacity, so it gets no fit (NaN, ndf 0) and counts as a failed refit."""
    import torch

    w = synth.SECTOR_EVENT
    ev = synth.generate(w)
    geom = synth.geometry(w)
    nt = 300
    state = np.tile(np.array([1.5, 40.0, 0.2, 0.3, 2.0], np.float32), (nt, 1))
    cov = np.zeros((nt, 15), np.float32)
    cov[:, [0, 2, 5, 9, 14]] = [0.01, 0.01, 1e-6, 1e-6, 1e-4]
    t = {"off": np.zeros(nt, np.int32), "nh": np.full(nt, 10, np.int32), "hits": np.arange(10, dtype=np.int32),
         "sector": np.zeros(nt, np.int32), "x_ref": np.full(nt, 100.0, np.float32), "state": state}
    d = tracks_to_device(t)
    d["cov"] = dev(cov)
    ten = [dev(a) for a in (ev.y, ev.z, ev.row, ev.sector)]
    out = ctx.merge(*ten, geom, synth.BZ, d, params=P)
    r = host(out, nt)
    c = out["counts"].cpu().numpy()
    assert np.all(r["label"] == 0) and r["n_members"][0] == nt
    assert np.isnan(r["theta"][0]).all() and np.isnan(r["theta_cov"][0]).all() and np.isnan(r["chi2"][0])
    assert r["ndf"][0] == 0 and c[6] == 1, c
    torch.cuda.synchronize()
