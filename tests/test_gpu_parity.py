"""HIP path vs FP64 oracle, stage by stage, on seeded synthetic inputs (needs an MI355X)."""
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


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    import torch

    assert torch.cuda.is_available(), "no GPU visible"
    from paper_1910_12214_amd import tpcca

    c = tpcca.Context(0)
    yield c
    c.close()


def to_dev(ev):
    import torch

    d = torch.device("cuda", 0)
    return (torch.from_numpy(ev.y).to(d), torch.from_numpy(ev.z).to(d), torch.from_numpy(ev.row).to(d),
            torch.from_numpy(ev.sector).to(d))


def run_gpu(ctx, ev, geom, params, timeframe=False):
    from paper_1910_12214_amd import tpcca

    y, z, r, s = to_dev(ev)
    out = ctx.track(y, z, r, s, geom, synth.BZ, params, timeframe=timeframe)
    return tpcca.tracks_to_host(out)


def check(ctx, w, ev, params=None, label="", geom=None):
    params = dict(synth.TRACKER_PARAMS, **(params or {}))
    geom = synth.geometry(w) if geom is None else geom
    say(f"[parity] {label or w.name}: n={ev.n} bins=({params['bin_y']},{params['bin_z']})")
    trk = run_gpu(ctx, ev, geom, params)
    st = parity.gpu_stages(ctx, synth.N_ROWS)
    o = oracle.track(ev.y, ev.z, ev.row, ev.sector, geom, params, synth.BZ, n_threads=THREADS)
    o_fma = oracle.track(ev.y, ev.z, ev.row, ev.sector, geom, params, synth.BZ, n_threads=THREADS, fma=True)
    rep = parity.compare(o, st, trk, ev.n, synth.N_ROWS, leg=ev.leg, l_min=params["l_min_chain"], o_fma=o_fma,
                         row_of=ev.row, row_x=synth.row_x(), bz=synth.BZ)
    c = trk["counts"]
    assert c[0] == o["n_tracks"] or rep["track_near_ties"] > 0
    say(f"[parity] {label or w.name}: {rep.line()} gpu_tracks={c[0]} oracle_tracks={o['n_tracks']}")
    return rep, trk, o


def test_sector_event(ctx):
    ev = synth.generate(synth.SECTOR_EVENT)
    rep, _, _ = check(ctx, synth.SECTOR_EVENT, ev)
    assert rep["tracks_compared"] > 100


def test_pbpb_slice_shuffled_input(ctx):
    w = dataclasses.replace(synth.scaled(synth.PBPB_EVENT, 0.1), order=1)
    ev = synth.generate(w)
    rep, _, _ = check(ctx, w, ev)
    assert rep["tracks_compared"] > 1000


@pytest.mark.parametrize("bins", [(2.5, 3.0), (40.0, 120.0), (1.0, 1.0)])
def test_other_bin_sizes(ctx, bins):
    """Other bin sizes; at 1 x 1 cm every row-sector's grid is built in several runs of z-bins."""
    w = synth.scaled(synth.PBPB_EVENT, 0.05)
    ev = synth.generate(w)
    check(ctx, w, ev, dict(bin_y=bins[0], bin_z=bins[1]), label=f"bins{bins}")


def test_bin_counting_grid_path(ctx):
    """Bins so fine (0.1 x 0.2 cm, one sector) that a row-sector would need more runs of z-bins than
    the LDS-only grid path takes: the grid is built by counting clusters per bin in global memory,
    and every stage still equals the oracle."""
    w = synth.SECTOR_EVENT
    ev = synth.generate(w)
    assert (ev.sector == 0).all()
    geom = dict(synth.geometry(w), n_sectors=1)
    check(ctx, w, ev, dict(bin_y=0.1, bin_z=0.2), label="bin-counting grid path", geom=geom)


def test_pbpb_full_event(ctx):
    ev = synth.generate(synth.PBPB_EVENT)
    rep, _, _ = check(ctx, synth.PBPB_EVENT, ev)
    assert rep["tracks_compared"] > 10000


def test_deterministic_and_bin_invariant(ctx):
    w = synth.scaled(synth.PBPB_EVENT, 0.1)
    ev = synth.generate(w)
    geom = synth.geometry(w)
    a = run_gpu(ctx, ev, geom, synth.TRACKER_PARAMS)
    b = run_gpu(ctx, ev, geom, synth.TRACKER_PARAMS)
    c = run_gpu(ctx, ev, geom, dict(synth.TRACKER_PARAMS, bin_y=3.0, bin_z=20.0))
    for x in (b, c):
        for k in ("hit_offset", "n_hits", "hit_ids", "start_id", "state", "cov", "chi2", "ndf"):
            assert np.array_equal(a[k], x[k]), k


def test_noise_free_recovery_on_gpu(ctx):
    w = dataclasses.replace(synth.sector_event(7), pt_lo=0.5, sigma_y=0.0, sigma_z=0.0, eff=1.0, noise_frac=0.0,
                            phi_inset_deg=3.0)
    ev = synth.generate(w)
    trk = run_gpu(ctx, ev, synth.geometry(w), synth.TRACKER_PARAMS)
    legs, counts = np.unique(ev.leg, return_counts=True)
    findable = {int(l) for l, c in zip(legs, counts) if c >= 10}
    got = set()
    for k in range(len(trk["start_id"])):
        hs = trk["hit_ids"][trk["hit_offset"][k]:trk["hit_offset"][k] + trk["n_hits"][k]]
        lg = np.unique(ev.leg[hs])
        assert lg.size == 1
        assert np.array_equal(np.sort(hs), np.nonzero(ev.leg == lg[0])[0])
        got.add(int(lg[0]))
    assert got == findable


def test_time_frame_slice_z_extended(ctx):
    w = synth.scaled(synth.PBPB_TIMEFRAME, 0.02)
    ev = synth.generate(w)
    rep, _, _ = check(ctx, w, ev, dict(bin_y=8.0, bin_z=16.0))
    assert rep["tracks_compared"] > 1000


def test_time_frame_slice_row_sector_grid(ctx):
    """A slice of the Pb-Pb frame large enough (about 1000 clusters per row-sector) for the
    row-sector grid path, its row-sectors built in several runs of z-bins: every stage equals the
    oracle."""
    w = synth.scaled(synth.PBPB_TIMEFRAME, 0.08)
    ev = synth.generate(w)
    assert ev.n >= 1024 * synth.N_ROWS * 36
    rep, _, _ = check(ctx, w, ev, dict(bin_y=8.0, bin_z=16.0))
    assert rep["tracks_compared"] > 10000


def test_degenerate_inputs(ctx):
    from paper_1910_12214_amd import tpcca

    geom = synth.geometry(synth.SECTOR_EVENT)
    empty = synth.Event(synth.SECTOR_EVENT, *(np.zeros(0, dt) for dt in (np.float32, np.float32, np.uint8, np.uint8,
                                                                         np.int32, np.int32, np.int32, np.int32)),
                        0, 0, 0, 0)
    for ev, label in ((empty, "empty"),):
        trk = run_gpu(ctx, ev, geom, synth.TRACKER_PARAMS)
        assert trk["counts"][tpcca.CNT_TRACKS] == 0
        say(f"[degenerate] {label}: ok")
    # one cluster; clusters only in invalid rows/sectors; a single straight track in rows 0..2
    cases = {
        "one": (np.array([1.0], np.float32), np.array([5.0], np.float32), np.array([4], np.uint8), np.array([0], np.uint8)),
        "invalid": (np.array([1.0, 2.0], np.float32), np.array([5.0, 6.0], np.float32),
                    np.array([200, 3], np.uint8), np.array([0, 40], np.uint8)),
        "nan": (np.array([np.nan, 0.0, 0.0], np.float32), np.array([5.0, np.nan, 5.0], np.float32),
                np.array([3, 4, 5], np.uint8), np.array([0, 0, 0], np.uint8)),
    }
    for label, (y, z, r, s) in cases.items():
        ev = dataclasses.replace(empty, y=y, z=z, row=r, sector=s, leg=np.full(y.size, -1, np.int32))
        trk = run_gpu(ctx, ev, geom, synth.TRACKER_PARAMS)
        st = parity.gpu_stages(ctx, synth.N_ROWS)
        o = oracle.track(y, z, r, s, geom, synth.TRACKER_PARAMS, synth.BZ)
        parity.compare(o, st, trk, y.size, synth.N_ROWS, leg=None)
        say(f"[degenerate] {label}: ok, valid clusters {trk['counts'][tpcca.CNT_VALID_CLUSTERS]}")


def test_capacity_error_reports_sizes(ctx):
    from paper_1910_12214_amd import tpcca

    ev = synth.generate(synth.SECTOR_EVENT)
    y, z, r, s = to_dev(ev)
    out = ctx.alloc_tracks(3, 50)
    with pytest.raises(tpcca.TpcError) as e:
        ctx.track(y, z, r, s, synth.geometry(synth.SECTOR_EVENT), synth.BZ, synth.TRACKER_PARAMS, out=out)
    assert e.value.code == tpcca.TPC_ERR_CAPACITY
    counts = out["counts"].cpu().numpy()
    assert counts[tpcca.CNT_TRACKS] > 3
    # a track is written iff its index and its hits fit; those are the full output's first tracks
    full = run_gpu(ctx, ev, synth.geometry(synth.SECTOR_EVENT), synth.TRACKER_PARAMS)
    got = tpcca.tracks_to_host(out)
    for k in range(3):
        if full["hit_offset"][k] + full["n_hits"][k] <= 50:
            assert got["start_id"][k] == full["start_id"][k]
            o, n = full["hit_offset"][k], full["n_hits"][k]
            assert np.array_equal(out["hit_ids"][o:o + n].cpu().numpy(), full["hit_ids"][o:o + n])


def test_argument_errors(ctx):
    from paper_1910_12214_amd import tpcca

    ev = synth.generate(synth.SECTOR_EVENT)
    y, z, r, s = to_dev(ev)
    geom = synth.geometry(synth.SECTOR_EVENT)
    for bad in (dict(l_min_chain=1), dict(sigma_y=0.0), dict(s_max=1.5), dict(bin_y=0.0), dict(nb_chi2_max=-1.0)):
        with pytest.raises(tpcca.TpcError) as e:
            ctx.track(y, z, r, s, geom, synth.BZ, dict(synth.TRACKER_PARAMS, **bad))
        assert e.value.code == tpcca.TPC_ERR_ARG, bad
    g2 = dict(geom, row_x=geom["row_x"][::-1].copy())
    with pytest.raises(tpcca.TpcError):
        ctx.track(y, z, r, s, g2, synth.BZ, synth.TRACKER_PARAMS)


@pytest.mark.parametrize("bins", [(8.0, 8.0), (0.9, 1.7)])
def test_clusters_outside_the_grid_range(ctx, bins):
    """Clusters beyond the grid's y range (lines that leave the sector, clusters far past the edge)
    and outside its z range are stored in the edge bins; every step must still find them exactly as
    the oracle does, for any bin size (a query box beyond the grid visits the edge bins)."""
    rng = np.random.default_rng(77)
    ev = synth.generate(synth.SECTOR_EVENT)
    rx = synth.row_x().astype(np.float64)
    th = float(synth.tan_half())
    extra_y, extra_z, extra_r = [], [], []
    # two straight lines leaving the sector on either side, clusters on every row
    for y0, slope, z0, tz in ((-3.0, 0.35, 40.0, 0.2), (4.0, -0.42, 120.0, -0.1)):
        c = 1.0 / np.sqrt(1.0 + slope * slope)
        extra_y += list(y0 + slope * (rx - 85.0)); extra_z += list(z0 + tz * (rx - 85.0) / c)
        extra_r += list(range(synth.N_ROWS))
    # a line running below z_min and one above z_max
    for z0, tz in ((5.0, -0.3), (240.0, 0.35)):
        extra_y += list(0.02 * (rx - 85.0)); extra_z += list(z0 + tz * (rx - 85.0)); extra_r += list(range(synth.N_ROWS))
    # scattered clusters far beyond the edges, in y and in z
    k = 400
    rr = rng.integers(0, synth.N_ROWS, k)
    side = rng.choice([-1.0, 1.0], k)
    extra_y += list(side * (rx[rr] * th + rng.uniform(0.5, 60.0, k))); extra_z += list(rng.uniform(-30, 280, k))
    extra_r += list(rr)
    y = np.concatenate([ev.y, np.array(extra_y, np.float32)])
    z = np.concatenate([ev.z, np.array(extra_z, np.float32)])
    row = np.concatenate([ev.row, np.array(extra_r, np.uint8)])
    sec = np.zeros_like(row)
    leg = np.concatenate([ev.leg, np.full(len(extra_y), -1, np.int32)])
    evx = dataclasses.replace(ev, y=y, z=z, row=row, sector=sec, leg=leg)
    rep, trk, o = check(ctx, synth.SECTOR_EVENT, evx, dict(bin_y=bins[0], bin_z=bins[1]), label=f"outside{bins}")
    # the lines beyond the edge are tracked up to the edge stop, the z lines in full
    assert rep["tracks_compared"] > 100
    n_out = int(((np.abs(y) > synth.row_x()[row] * synth.tan_half()) | (z < 0) | (z > 250)).sum())
    on_tracks = np.isin(np.arange(ev.n, y.size), trk["hit_ids"]).sum()
    say(f"[parity] outside{bins}: {n_out} clusters outside the grid, {on_tracks} added clusters on tracks")
    assert on_tracks > 300
