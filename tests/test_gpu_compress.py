"""Cluster compression on the GPU (Sec. 4, steps 2-4) against the oracle: symbol streams, cluster
order, escapes, ANS frequency tables and coded bytes identical (residuals at oracle-flagged
rounding near-ties excluded and counted), and the GPU decoder returning every cluster."""
import sys

import numpy as np
import pytest

import oracle
import synth
from oracle import compress as oc
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


def oracle_track_set(ev, geom):
    o = oracle.track(ev.y, ev.z, ev.row, ev.sector, geom, P, synth.BZ)
    t = oracle.tracks_for_flags(o, geom, ev.sector)
    host = {"hit_offset": t["off"], "n_hits": t["nh"], "hit_ids": t["hits"], "sector": t["sector"],
            "row_ref": np.array([ev.row[t["hits"][a]] for a in t["off"]], dtype=np.int32), "x_ref": t["x_ref"],
            "state": t["state"]}
    d = tracks_to_device(t)
    d["row_ref"] = dev(np.concatenate([host["row_ref"], np.zeros(max(0, 1 - len(host["row_ref"])), np.int32)]))
    return host, d


def gpu_streams(c, comp):
    """Host copies of the GPU's streams: {name: (symbols, escapes)}, bytes per stream, blocks."""
    from paper_1910_12214_amd import tpcca as T

    cnt = comp["counts"].cpu().numpy()
    sym = comp["sym"].cpu().numpy().view(np.uint16).reshape(T.N_CSTREAMS, comp["cap_sym"])
    esc = comp["esc"].cpu().numpy().view(np.uint32).reshape(T.N_CSTREAMS, -1)
    freq = comp["freq"].cpu().numpy().view(np.uint32).reshape(T.N_CSTREAMS, T.CS_ALPHABET)
    bb = comp["block_bytes"].cpu().numpy().view(np.uint32).reshape(T.N_CSTREAMS, -1)
    data = comp["bytes"].cpu().numpy()
    out, pos = {}, 0
    for s, name in enumerate(T.CSTREAMS):
        ns, ne, nbytes, nblk = (int(v) for v in cnt[s * T.CSC_N:(s + 1) * T.CSC_N])
        out[name] = dict(sym=sym[s, :ns].copy(), esc=esc[s, :ne].copy(), freq=freq[s].copy(),
                         blocks=bb[s, :nblk].copy(), bytes=data[pos:pos + nbytes].copy())
        pos += nbytes
    tot = cnt[T.N_CSTREAMS * T.CSC_N:]
    return out, tot


def check_against_oracle(ctx, ev, geom, host_trk, dev_trk, props, cap_esc=None):
    from paper_1910_12214_amd import tpcca as T

    q, sy, sz = props
    ten = [dev(a) for a in (ev.y, ev.z, ev.row, ev.sector)]
    out = ctx.alloc_compressed(ev.n, geom["n_sectors"] * geom["n_rows"], int(dev_trk["cap_tracks"]), cap_esc=cap_esc)
    comp = ctx.compress(*ten, dev(q.view(np.int16)), dev(sy), dev(sz), geom, synth.BZ, dev_trk, P, out=out)
    g, tot = gpu_streams(ctx, comp)
    o = oc.compress(ev.y, ev.z, ev.row, ev.sector, q, sy, sz, geom, synth.BZ, host_trk)
    assert int(tot[T.CST_ATTACHED]) == o["n_attached"] and int(tot[T.CST_UNATTACHED]) == o["n_unattached"]
    assert int(tot[T.CST_SKIPPED]) == o["n_skipped"] and int(tot[T.CST_PRED_FAIL]) == o["pred_fail"]
    n_all = o["n_attached"] + o["n_unattached"]
    assert np.array_equal(comp["order"][:n_all].cpu().numpy(), o["order"])
    assert np.array_equal(comp["track_len"][:len(o["track_len"])].cpu().numpy(), o["track_len"])
    tie = np.zeros(o["n_attached"], dtype=bool)
    tie[o["tie"]] = True
    for name in T.CSTREAMS:
        a, b = g[name]["sym"], o["streams"][name]
        assert len(a) == len(b), name
        if name in ("a_ry", "a_rz"):
            assert np.array_equal(a[~tie], b[~tie]), name
        else:
            assert np.array_equal(a, b), name
        if not tie.any() or name not in ("a_ry", "a_rz"):
            assert np.array_equal(g[name]["esc"], o["escapes"][name]), name
        # ANS: frequencies of the GPU's own symbols, then the coded bytes, equal the oracle's coder
        f = oc.ans_freqs(np.bincount(a, minlength=T.CS_ALPHABET))
        assert np.array_equal(g[name]["freq"], f), name
        _, data, per = oc.ans_encode(a, f)
        assert np.array_equal(g[name]["blocks"], per), name
        assert np.array_equal(g[name]["bytes"], data), name
    # decoding: the symbols back, and every cluster's quantised position and properties
    d = ctx.decompress(comp, geom, synth.BZ, dev_trk, P)
    dsym = d["sym"].cpu().numpy().view(np.uint16).reshape(T.N_CSTREAMS, comp["cap_sym"])
    for s, name in enumerate(T.CSTREAMS):
        assert np.array_equal(dsym[s, :len(g[name]["sym"])], g[name]["sym"]), name
    order = o["order"]
    n = d["n"]
    assert n == n_all
    assert np.array_equal(d["sector"][:n].cpu().numpy(), ev.sector[order])
    assert np.array_equal(d["row"][:n].cpu().numpy(), ev.row[order])
    assert np.array_equal(d["yq"][:n].cpu().numpy(), o["yq"][order])
    assert np.array_equal(d["zq"][:n].cpu().numpy(), o["zq"][order])
    for k, v, nb in (("qtot", q, 4), ("sigma_y", sy, 3), ("sigma_z", sz, 3)):
        got = d[k][:n].cpu().numpy()
        got = got.view(np.uint16) if k == "qtot" else got
        want = np.array([oc.dynprec(int(x), nb) for x in v[order]])
        assert np.array_equal(got.astype(np.int64), want), k
    bits = ctx.compress_sizes(comp)
    for s, name in enumerate(T.CSTREAMS):
        cnt = np.bincount(g[name]["sym"], minlength=T.CS_ALPHABET)
        ent, huf, ans = bits[s]
        assert ent == pytest.approx(oc.entropy_bits(cnt), rel=1e-9, abs=1e-6)
        assert huf == oc.huffman_bits(cnt)[0]
        assert ans == 8 * len(g[name]["bytes"])
    return comp, o, bits, int(tie.sum())


def test_sector_event_streams_and_bytes_equal_oracle(ctx):
    w = synth.SECTOR_EVENT
    ev = synth.generate(w)
    geom = synth.geometry(w)
    host, d = oracle_track_set(ev, geom)
    _, o, bits, ties = check_against_oracle(ctx, ev, geom, host, d, synth.cluster_properties(ev))
    say(f"[cmp] sector event: {o['n_attached']} on tracks, {o['n_unattached']} others, {ties} near-ties; "
        f"entropy {bits[:, 0].sum() / 8:.0f} B, Huffman {bits[:, 1].sum() / 8:.0f} B, ANS {bits[:, 2].sum() / 8:.0f} B")


def test_pbpb_slice_with_malformed_tracks(ctx):
    """A tenth of a Pb-Pb event, shuffled clusters, plus tracks with an id out of range and an
    offset beyond the hit list: those tracks are left out and their clusters stored as others."""
    w = synth.scaled(synth.PBPB_EVENT, 0.1)
    ev = synth.generate(w)
    geom = synth.geometry(w)
    host, _ = oracle_track_set(ev, geom)
    nt = len(host["n_hits"])
    assert nt > 10
    host["hit_ids"] = host["hit_ids"].copy()
    host["hit_ids"][host["hit_offset"][3] + 1] = ev.n + 5  # id out of range
    host["hit_offset"] = host["hit_offset"].copy()
    host["hit_offset"][7] = len(host["hit_ids"]) - 2       # runs past the hit list
    t = {"off": host["hit_offset"], "nh": host["n_hits"], "hits": host["hit_ids"], "sector": host["sector"],
         "x_ref": host["x_ref"], "state": host["state"]}
    d = tracks_to_device(t)
    d["row_ref"] = dev(host["row_ref"])
    _, o, _, ties = check_against_oracle(ctx, ev, geom, host, d, synth.cluster_properties(ev))
    assert o["track_len"][3] == 0 and o["track_len"][7] == 0 and o["track_len"][4] > 0
    say(f"[cmp] Pb-Pb slice: {o['n_attached']} on tracks, {o['n_unattached']} others, {ties} near-ties")


def test_full_event_gpu_tracks(ctx):
    """The whole Pb-Pb event with the GPU's own tracks: streams equal to the oracle's on the same
    tracks, decoder exact."""
    from paper_1910_12214_amd import tpcca

    w = synth.PBPB_EVENT
    ev = synth.generate(w)
    geom = synth.geometry(w)
    ten = [dev(a) for a in (ev.y, ev.z, ev.row, ev.sector)]
    out = ctx.track(*ten, geom, synth.BZ, P)
    h = tpcca.tracks_to_host(out)
    host = {k: h[k] for k in ("hit_offset", "n_hits", "hit_ids", "sector", "row_ref", "x_ref", "state")}
    _, o, bits, ties = check_against_oracle(ctx, ev, geom, host, out, synth.cluster_properties(ev))
    raw = 14 * ev.n
    say(f"[cmp] Pb-Pb event: {ev.n} clusters, {o['n_attached']} on {len(h['n_hits'])} tracks, {ties} near-ties; "
        f"raw {raw} B -> ANS {bits[:, 2].sum() / 8:.0f} B (x{raw / (bits[:, 2].sum() / 8):.2f}), Huffman "
        f"{bits[:, 1].sum() / 8:.0f} B, entropy {bits[:, 0].sum() / 8:.0f} B")
    assert bits[:, 2].sum() < bits[:, 1].sum() + 64 * 9 * (ev.n // 4096 + 2)


def test_no_clusters(ctx):
    import torch

    from paper_1910_12214_amd import tpcca

    w = synth.SECTOR_EVENT
    geom = synth.geometry(w)
    e = torch.zeros(0, dtype=torch.float32, device="cuda")
    b = torch.zeros(0, dtype=torch.uint8, device="cuda")
    trk = ctx.alloc_tracks(16, 16)
    comp = ctx.compress(e, e, b, b, torch.zeros(0, dtype=torch.int16, device="cuda"), b, b, geom, synth.BZ, trk, P)
    cnt = comp["counts"].cpu().numpy()
    assert cnt[tpcca.N_CSTREAMS * tpcca.CSC_N + tpcca.CST_ATTACHED] == 0
    assert cnt[tpcca.N_CSTREAMS * tpcca.CSC_N + tpcca.CST_UNATTACHED] == 0
    # the per-row counts stream holds one zero per row
    assert cnt[tpcca.CSTREAMS.index("u_n") * tpcca.CSC_N] == geom["n_rows"] * geom["n_sectors"]
    d = ctx.decompress(comp, geom, synth.BZ, trk, P)
    assert d["n"] == 0


def test_row_longer_than_the_lds_sort(ctx):
    """Without tracks every cluster is stored as an other cluster; one row gets 6000 extra
    clusters, more than one workgroup sorts in LDS, so that row is ordered by the ranking
    fallback.  Streams and decoding equal the oracle's."""
    import dataclasses

    w = synth.SECTOR_EVENT
    ev = synth.generate(w)
    geom = synth.geometry(w)
    rng = np.random.default_rng(77)
    k = 6000
    r0 = 40
    half = float(geom["row_x"][r0]) * float(geom["tan_half"])
    ev = dataclasses.replace(
        ev,
        y=np.concatenate([ev.y, rng.uniform(-half, half, k).astype(np.float32)]),
        z=np.concatenate([ev.z, rng.uniform(0.0, float(geom["z_max"]), k).astype(np.float32)]),
        row=np.concatenate([ev.row, np.full(k, r0, ev.row.dtype)]),
        sector=np.concatenate([ev.sector, np.full(k, ev.sector[0], ev.sector.dtype)]),
        particle=np.concatenate([ev.particle, np.full(k, -1, ev.particle.dtype)]))
    host = {"hit_offset": np.zeros(0, np.int32), "n_hits": np.zeros(0, np.int32), "hit_ids": np.zeros(0, np.int32),
            "sector": np.zeros(0, np.int32), "row_ref": np.zeros(0, np.int32), "x_ref": np.zeros(0, np.float32),
            "state": np.zeros((0, 5), np.float32)}
    trk = ctx.alloc_tracks(16, 16)
    # random y along the long row: most of its y differences exceed the alphabet (escapes)
    _, o, _, _ = check_against_oracle(ctx, ev, geom, host, trk, synth.cluster_properties(ev), cap_esc=2 * ev.n)
    assert o["n_attached"] == 0 and o["n_unattached"] == ev.n
    say(f"[cmp] no tracks, one long row: {ev.n} clusters stored as others")
