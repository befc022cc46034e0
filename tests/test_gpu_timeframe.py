"""Continuous-readout time frames: graph-captured, autotuned path vs the per-sector path and the
oracle (needs an MI355X)."""
import dataclasses
import os
import sys

import numpy as np
import pytest

import oracle
import synth
from tests import parity

pytestmark = pytest.mark.gpu
THREADS = min(16, os.cpu_count() or 1)
KEYS = ("hit_offset", "n_hits", "hit_ids", "start_id", "sector", "row_ref", "x_ref", "state", "cov", "chi2", "ndf")


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


def same(a, b):
    for k in KEYS:
        assert np.array_equal(a[k], b[k]), k
    assert np.array_equal(a["counts"][:8], b["counts"][:8])


@pytest.fixture(scope="module")
def small_tf():
    w = synth.scaled(synth.PBPB_TIMEFRAME, 0.02)
    return w, synth.generate(w)


def test_timeframe_equals_sector_path(ctx, small_tf):
    from paper_1910_12214_amd import tpcca

    w, ev = small_tf
    geom = synth.geometry(w)
    ten = [dev(a) for a in (ev.y, ev.z, ev.row, ev.sector)]
    ctx.set_tuning(None)
    a = tpcca.tracks_to_host(ctx.track(*ten, geom, synth.BZ, synth.TRACKER_PARAMS, timeframe=True))
    tun = ctx.tuning()
    say(f"[tf] tuned: {tun}")
    assert tun["n_candidates"] >= 4
    b = tpcca.tracks_to_host(ctx.track(*ten, geom, synth.BZ, dict(synth.TRACKER_PARAMS, bin_y=3.0, bin_z=7.0)))
    same(a, b)
    c = tpcca.tracks_to_host(ctx.track(*ten, geom, synth.BZ, synth.TRACKER_PARAMS, timeframe=True))  # graph replay
    same(a, c)


@pytest.mark.parametrize("tiles", [dict(bin_y=8.0, bin_z=16.0, tracklet_chunk=1, blocks_per_cu=4),
                                   dict(bin_y=16.0, bin_z=32.0, tracklet_chunk=4, blocks_per_cu=8, waves_per_simd=2),
                                   dict(bin_y=5.0, bin_z=11.0, tracklet_chunk=2, blocks_per_cu=1, waves_per_simd=3)])
def test_every_tile_choice_gives_identical_tracks(ctx, small_tf, tiles):
    from paper_1910_12214_amd import tpcca

    w, ev = small_tf
    geom = synth.geometry(w)
    ten = [dev(a) for a in (ev.y, ev.z, ev.row, ev.sector)]
    ref = tpcca.tracks_to_host(ctx.track(*ten, geom, synth.BZ, synth.TRACKER_PARAMS))
    ctx.set_tuning(tiles)
    got = tpcca.tracks_to_host(ctx.track(*ten, geom, synth.BZ, synth.TRACKER_PARAMS, timeframe=True))
    ctx.set_tuning(None)
    same(ref, got)


def test_tile_cache_persists_across_contexts(small_tf, tmp_path):
    """A second context with the same cache file takes the first one's tiles without tuning, and
    tracks identically; a malformed line in the file is ignored."""
    import time

    from paper_1910_12214_amd import tpcca

    w, ev = small_tf
    geom = synth.geometry(w)
    ten = [dev(a) for a in (ev.y, ev.z, ev.row, ev.sector)]
    path = tmp_path / "tiles.txt"
    path.write_text("garbage line\n0123 1 2 3\n")
    a = tpcca.Context(0)
    a.set_tune_cache(str(path))
    ta = tpcca.tracks_to_host(a.track(*ten, geom, synth.BZ, synth.TRACKER_PARAMS, timeframe=True))
    tun_a = a.tuning()
    entries = [ln for ln in path.read_text().splitlines() if ln and not ln.startswith("#")]
    assert len(entries) == 3 and tun_a["n_candidates"] >= 4, entries
    a.close()
    b = tpcca.Context(0)
    b.set_tune_cache(str(path))
    t0 = time.perf_counter()
    tb = tpcca.tracks_to_host(b.track(*ten, geom, synth.BZ, synth.TRACKER_PARAMS, timeframe=True))
    dt = time.perf_counter() - t0
    tun_b = b.tuning()
    say(f"[tf] cached tiles {tun_b} in {dt * 1e3:.1f} ms (tuned {tun_a['best_ms']:.2f} ms per candidate run)")
    for k in ("bin_y", "bin_z", "tracklet_chunk", "blocks_per_cu", "waves_per_simd", "n_candidates"):
        assert tun_b[k] == pytest.approx(tun_a[k]), k
    assert [ln for ln in path.read_text().splitlines() if ln and not ln.startswith("#")] == entries
    same(ta, tb)
    b.close()


def test_graph_replay_sees_new_data_in_the_same_buffers(ctx):
    """The captured graph bakes pointers, not data: refill the same tensors with another frame."""
    import torch

    from paper_1910_12214_amd import tpcca

    w1 = synth.scaled(synth.PBPB_TIMEFRAME, 0.01)
    w2 = dataclasses.replace(w1, seed=w1.seed + 99)
    e1, e2 = synth.generate(w1), synth.generate(w2)
    n = min(e1.n, e2.n)
    geom = synth.geometry(w1)
    ten = [dev(a[:n]) for a in (e1.y, e1.z, e1.row, e1.sector)]
    out = ctx.alloc_tracks(n // 4, n)
    ctx.set_tuning(dict(bin_y=8.0, bin_z=16.0, tracklet_chunk=1, blocks_per_cu=8))
    ctx.track(*ten, geom, synth.BZ, synth.TRACKER_PARAMS, out=out, timeframe=True)
    r1 = tpcca.tracks_to_host(out)
    for t, a in zip(ten, (e2.y, e2.z, e2.row, e2.sector)):
        t.copy_(torch.from_numpy(np.ascontiguousarray(a[:n])))
    torch.cuda.synchronize()
    for rep in range(3):  # several replays, eager work in between
        _ = torch.ones(1000, device="cuda:0").sum().item()
        ctx.track(*ten, geom, synth.BZ, synth.TRACKER_PARAMS, out=out, timeframe=True)
        r2 = tpcca.tracks_to_host(out)
        ref = tpcca.tracks_to_host(ctx.track(*ten, geom, synth.BZ, dict(synth.TRACKER_PARAMS, bin_y=8.0, bin_z=16.0)))
        same(r2, ref)
    ctx.set_tuning(None)
    assert r1["counts"][0] != r2["counts"][0] or not np.array_equal(r1["hit_ids"], r2["hit_ids"])


def test_full_pbpb_timeframe_sampled_sectors(ctx):
    """The full 570-collision frame in one graph launch; the oracle checks two whole sectors."""
    from paper_1910_12214_amd import tpcca

    w = synth.PBPB_TIMEFRAME
    ev = synth.generate(w)
    geom = synth.geometry(w)
    say(f"[tf] full frame: {ev.n} clusters")
    ten = [dev(a) for a in (ev.y, ev.z, ev.row, ev.sector)]
    out = ctx.alloc_tracks(ev.n // 8, ev.n)
    ctx.set_tuning(dict(bin_y=8.0, bin_z=16.0, tracklet_chunk=1, blocks_per_cu=8))
    ctx.track(*ten, geom, synth.BZ, synth.TRACKER_PARAMS, out=out, timeframe=True)
    ctx.set_tuning(None)
    trk = tpcca.tracks_to_host(out)
    st = parity.gpu_stages(ctx, synth.N_ROWS)
    sectors = [3, 22]
    sel = np.isin(ev.sector, sectors)
    ids = np.nonzero(sel)[0]
    prm = dict(synth.TRACKER_PARAMS, bin_y=8.0, bin_z=16.0)
    # the oracle runs on the two sectors only (every step is per sector); map its ids back
    o = oracle.track(ev.y[sel], ev.z[sel], ev.row[sel], ev.sector[sel], geom, prm, synth.BZ, n_threads=THREADS)
    o_fma = oracle.track(ev.y[sel], ev.z[sel], ev.row[sel], ev.sector[sel], geom, prm, synth.BZ, n_threads=THREADS,
                         fma=True)
    o = lift(o, ids, ev.n)
    o_fma = lift(o_fma, ids, ev.n)
    rep = parity.compare(o, st, trk, ev.n, synth.N_ROWS, sectors=sectors, sector_of=ev.sector, o_fma=o_fma,
                         row_of=ev.row, row_x=synth.row_x(), bz=synth.BZ)
    say(f"[tf] full frame sectors {sectors}: {rep.line()}")
    assert rep["tracks_compared"] > 20000


def lift(o, ids, n):
    """Re-index an oracle result computed on a subset of clusters to the full cluster ids."""
    ids = ids.astype(np.int64)
    r = dict(o)
    for k in ("up", "dn", "up_c", "dn_c"):
        a = np.full(n, -1, dtype=np.int64)
        v = o[k].astype(np.int64)
        a[ids] = np.where(v >= 0, ids[np.maximum(v, 0)], -1)
        r[k] = a
    f = np.zeros(n, dtype=np.uint8)
    f[ids] = o["nb_flag"]
    r["nb_flag"] = f
    r["start_id"] = ids[o["start_id"].astype(np.int64)]
    th = o["tl_hits"].astype(np.int64)
    r["tl_hits"] = np.where(th >= 0, ids[np.maximum(th, 0)], -1)
    # hit keys carry the start id: rebuild them with the global ids (the id map is monotonic,
    # so which tracklet owns a hit does not change)
    key = np.zeros(n, dtype=np.uint64)
    for t in np.nonzero(o["tl_valid"])[0]:
        k = (np.uint64(o["tl_nhits"][t]) << np.uint64(32)) | np.uint64(0xFFFFFFFF - int(r["start_id"][t]))
        hs = r["tl_hits"][t][r["tl_hits"][t] >= 0]
        key[hs] = np.maximum(key[hs], k)
    r["hit_key"] = key
    r["trk_hits"] = ids[o["trk_hits"].astype(np.int64)]
    return r


def test_pp_timeframe_with_fused_scorer_equals_sector_path(ctx):
    """pp time frame (many tiny collisions, 10% noise) with the trained scorer fused into neighbour
    finding, through the graph path, equals the per-sector path with the same scorer."""
    from paper_1910_12214_amd import scorer as sc
    from paper_1910_12214_amd import tpcca

    w = synth.scaled(synth.PP_TIMEFRAME, 0.1)
    ev = synth.generate(w)
    geom = synth.geometry(w)
    ten = [dev(a) for a in (ev.y, ev.z, ev.row, ev.sector)]
    params, tau = sc.load()
    mlp = dev(params)
    ctx.set_tuning(dict(bin_y=8.0, bin_z=16.0, tracklet_chunk=2, blocks_per_cu=6, waves_per_simd=3))
    a = tpcca.tracks_to_host(ctx.track(*ten, geom, synth.BZ, synth.TRACKER_PARAMS, mlp=mlp, tau_logit=tau,
                                       timeframe=True))
    a2 = tpcca.tracks_to_host(ctx.track(*ten, geom, synth.BZ, synth.TRACKER_PARAMS, mlp=mlp, tau_logit=tau,
                                        timeframe=True))  # graph replay
    ctx.set_tuning(None)
    b = tpcca.tracks_to_host(ctx.track(*ten, geom, synth.BZ, dict(synth.TRACKER_PARAMS, bin_y=8.0, bin_z=16.0),
                                       mlp=mlp, tau_logit=tau))
    same(a, b)
    same(a2, b)
    c = a["counts"]
    say(f"[tf] pp frame {ev.n} clusters: pairs {c[tpcca.CNT_PAIRS]} kept {c[tpcca.CNT_PAIRS_KEPT]} tracks {c[0]}")
    assert c[tpcca.CNT_PAIRS_KEPT] < c[tpcca.CNT_PAIRS]


@pytest.mark.parametrize("pruned", [False, True])
def test_pp_timeframe_slice_equals_oracle(ctx, pruned):
    """A tenth of the pp time frame (1140 collisions over 1.14 ms, Poisson(12) each, 10% noise), in
    one graph launch of the time-frame entry point, plain and with the pp scorer fused into
    neighbour finding, equals the oracle stage by stage (with the same BF16 scorer in FP64)."""
    from oracle import mlp as omlp
    from paper_1910_12214_amd import scorer as sc
    from paper_1910_12214_amd import tpcca

    w = synth.scaled(synth.PP_TIMEFRAME, 0.1)
    ev = synth.generate(w)
    geom = synth.geometry(w)
    ten = [dev(a) for a in (ev.y, ev.z, ev.row, ev.sector)]
    prm = dict(synth.TRACKER_PARAMS, bin_y=8.0, bin_z=16.0)
    kw, q = {}, None
    if pruned:
        theta, tau = sc.load(sc.PP_CKPT)
        kw = dict(mlp=dev(theta), tau_logit=tau)
        q = omlp.quantize(theta.astype(np.float64))
        prm.update(mlp_tau_logit=tau, mlp_flag_abs=1e-4)
    say(f"[tf] pp slice {ev.n} clusters, pruned={pruned}")
    ctx.set_tuning(dict(bin_y=8.0, bin_z=16.0, tracklet_chunk=2, blocks_per_cu=6, waves_per_simd=3))
    out = ctx.alloc_tracks(ev.n // 8, ev.n)
    ctx.track(*ten, geom, synth.BZ, synth.TRACKER_PARAMS, out=out, timeframe=True, **kw)
    ctx.track(*ten, geom, synth.BZ, synth.TRACKER_PARAMS, out=out, timeframe=True, **kw)  # graph replay
    ctx.set_tuning(None)
    trk = tpcca.tracks_to_host(out)
    st = parity.gpu_stages(ctx, synth.N_ROWS)
    o = oracle.track(ev.y, ev.z, ev.row, ev.sector, geom, prm, synth.BZ, mlp=q, n_threads=THREADS)
    o_fma = oracle.track(ev.y, ev.z, ev.row, ev.sector, geom, prm, synth.BZ, mlp=q, n_threads=THREADS, fma=True)
    rep = parity.compare(o, st, trk, ev.n, synth.N_ROWS, leg=ev.leg, o_fma=o_fma,
                         row_of=ev.row, row_x=synth.row_x(), bz=synth.BZ)
    c = trk["counts"]
    say(f"[tf] pp slice parity (pruned={pruned}): {rep.line()} pairs={c[tpcca.CNT_PAIRS]} "
        f"kept={c[tpcca.CNT_PAIRS_KEPT]}")
    assert rep["tracks_compared"] > 5000


def test_graph_replay_with_shifted_z_window(ctx):
    """The same clusters shifted in z by D, tracked with the z window [z_min + D, z_max + D] of the
    same width: the grid has the same number of z bins and every buffer stays where it is, so only
    the z origin differs between the two calls.  The second call must not replay the first graph
    (whose kernels would place every cluster in the wrong bins): its tracks are the same as the
    unshifted ones, with z shifted, and equal the per-sector path's."""
    import torch

    from paper_1910_12214_amd import tpcca

    w = synth.scaled(synth.PBPB_TIMEFRAME, 0.01)
    ev = synth.generate(w)
    geom = synth.geometry(w)
    D = 400.0
    geom2 = dict(geom, z_min=geom["z_min"] + D, z_max=geom["z_max"] + D)
    # z on a 2^-13 cm lattice, so that z and z + D are both exact in FP32 (z + D < 2048)
    zq = (np.round(ev.z.astype(np.float64) * 8192.0) / 8192.0).astype(np.float32)
    assert np.array_equal((zq + np.float32(D)) - np.float32(D), zq)
    ten = [dev(a) for a in (ev.y, zq, ev.row, ev.sector)]
    out = ctx.alloc_tracks(ev.n // 4, ev.n)
    ctx.set_tuning(dict(bin_y=8.0, bin_z=16.0, tracklet_chunk=1, blocks_per_cu=8))
    ctx.track(*ten, geom, synth.BZ, synth.TRACKER_PARAMS, out=out, timeframe=True)
    a = tpcca.tracks_to_host(out)
    ten[1].copy_(torch.from_numpy(zq + np.float32(D)))
    ctx.track(*ten, geom2, synth.BZ, synth.TRACKER_PARAMS, out=out, timeframe=True)
    b = tpcca.tracks_to_host(out)
    ctx.set_tuning(None)
    ref = tpcca.tracks_to_host(ctx.track(*ten, geom2, synth.BZ, dict(synth.TRACKER_PARAMS, bin_y=8.0, bin_z=16.0)))
    same(b, ref)
    assert a["counts"][0] > 100
    assert np.array_equal(a["hit_ids"], b["hit_ids"]) and np.array_equal(a["n_hits"], b["n_hits"])
