"""Pins of the oracle's tracklet following rules (C19, C20 of the written reading).

* Row search: the hit of smallest chi2 = r^T S^-1 r (S = HCH^T + R) within the cut, ties to the
  smallest cluster id, must equal an exhaustive scan of every cluster of the row (no grid, no
  box).  The chi2 ellipse's bounding box the oracle uses is an exact pre-filter only if it is
  built from S (with R) and the ranking is by chi2, not by distance: random covariances with
  strong y-z correlation and C_yy far below or above sigma_y^2 separate those readings.
* Gap rule: a tracklet continues across up to N_miss consecutive rows without a hit and stops
  after N_miss + 1.  Noise-free tracks with hand-made gaps are recovered with their exact hit
  sets; the gap is placed where only pass A (near the outer end) or only pass B (near the inner
  end) can bridge it, so each pass's rule is pinned on its own.
* Sector-edge stop: a pass ends at the first row where the predicted |y| exceeds
  x tan(half angle) + edge margin.  A hand-built straight line and circle that leave the sector
  (clusters placed beyond the edge, which the grid accepts in its edge bins) must end exactly at
  that row, computed here from the closed-form curve.
"""
import dataclasses
import math

import numpy as np
import pytest

import oracle
import synth

P = synth.TRACKER_PARAMS
R_ROWS = synth.N_ROWS


def geom1(z_max=250.0):
    return dict(n_rows=R_ROWS, row_x=synth.row_x(), tan_half=synth.tan_half(), n_sectors=1, z_min=0.0, z_max=z_max)


# ------------------------------------------------------------------ row search vs exhaustive scan
def exhaustive_search(y, z, row, r, p, C, prm):
    """Every cluster of row r: chi2 with S = C_yz + diag(sigma^2); smallest within the cut, ties by id.
    Returns (id or -1, sorted chi2 values within the cut)."""
    S = np.array([[C[0, 0] + prm["sigma_y"] ** 2, C[0, 1]], [C[1, 0], C[1, 1] + prm["sigma_z"] ** 2]])
    Si = np.linalg.inv(S)
    best = None
    vals = []
    for i in range(len(y)):
        if row[i] != r:
            continue
        d = np.array([float(y[i]) - p[0], float(z[i]) - p[1]])
        c2 = float(d @ Si @ d)
        if c2 > prm["fol_chi2_max"]:
            continue
        vals.append(c2)
        if best is None or (c2, i) < best:
            best = (c2, i)
    return (-1 if best is None else best[1]), sorted(vals)


def random_cov(rng):
    """Random SPD 5x5 covariance: y/z block with correlation up to +-0.98 and variances from far
    below to far above the cluster errors; the other parameters correlated with y and z."""
    sy = 10 ** rng.uniform(-2.5, 0.0)
    sz = 10 ** rng.uniform(-2.5, 0.0)
    rho = rng.uniform(-0.98, 0.98)
    A = rng.normal(size=(5, 5)) * 0.1
    M = A @ A.T + np.diag([0, 0, 1e-3, 1e-3, 1e-2])
    M[0, 0], M[1, 1], M[0, 1] = sy * sy, sz * sz, rho * sy * sz
    M[1, 0] = M[0, 1]
    # keep the whole matrix positive definite
    w = np.linalg.eigvalsh(M)
    if w.min() <= 0:
        M += np.eye(5) * (1e-9 - w.min())
    return M


@pytest.mark.parametrize("seed", range(4))
def test_row_search_equals_exhaustive_chi2_scan(seed):
    rng = np.random.default_rng(500 + seed)
    r = 40
    n_cases = n_found = n_ties = 0
    for case in range(60):
        C = random_cov(rng)
        p = np.array([rng.uniform(-10, 10), rng.uniform(20, 200), 0.1, 0.2, 0.5])
        S = C[:2, :2] + np.diag([P["sigma_y"] ** 2, P["sigma_z"] ** 2])
        L = np.linalg.cholesky(S)
        k = int(rng.integers(1, 25))
        # candidates around the prediction, spread over the chi2 ellipse and somewhat beyond it
        pts = (L @ rng.normal(size=(2, k)) * rng.uniform(0.5, 4.0)).T + p[:2]
        y = list(pts[:, 0]); z = list(pts[:, 1]); row = [r] * k
        # exact ties: duplicated clusters (identical chi2, broken by id)
        for _ in range(int(rng.integers(0, 3))):
            i = int(rng.integers(0, k))
            y.append(y[i]); z.append(z[i]); row.append(r)
        # clusters of the neighbouring rows at the same place must be ignored
        for rr in (r - 1, r + 1):
            y.append(p[0]); z.append(p[1]); row.append(rr)
        perm = rng.permutation(len(y))
        y = np.array(y, dtype=np.float32)[perm]; z = np.array(z, dtype=np.float32)[perm]
        row = np.array(row, dtype=np.uint8)[perm]
        sec = np.zeros_like(row)
        want, vals = exhaustive_search(y, z, row, r, p, C, P)
        for by, bz in ((8.0, 8.0), (0.9, 1.3)):
            got, flag = oracle.follow_search(y, z, row, sec, geom1(), dict(P, bin_y=by, bin_z=bz), 0, r, p,
                                             oracle.full_to_sym15(C))
            if flag & (oracle.F_ARGMIN | oracle.F_CUT):
                # a decision within 1e-5 of another value or of the cut: the winner must be one of
                # the (near-)equal best values, or nothing if the best sits on the cut
                n_ties += 1
                if got >= 0:
                    assert want >= 0
                    d = np.array([float(y[got]) - p[0], float(z[got]) - p[1]])
                    c2 = float(d @ np.linalg.inv(S) @ d)
                    assert c2 <= vals[0] * (1 + 1e-5) + 1e-12
                else:
                    assert want < 0 or vals[0] >= P["fol_chi2_max"] * (1 - 1e-5)
                continue
            assert got == want, (case, by, got, want, vals[:3])
        n_cases += 1
        n_found += want >= 0
    assert n_found > 20 and n_cases > 40


@pytest.mark.parametrize("dy,dz", [(0.1, 0.0), (0.0, 0.2), (-0.15, -0.1)])
def test_row_search_box_includes_the_cluster_error(dy, dz):
    """A well-measured state (C far below the cluster errors): the only hit lies inside the chi2 cut
    but outside the box sqrt(cut C_ii) a box without the cluster errors would use."""
    r = 30
    C = np.diag([1e-5, 1e-5, 1e-3, 1e-3, 1e-2])
    p = np.array([1.0, 80.0, 0, 0, 0])
    y = np.array([p[0] + dy], dtype=np.float32)
    z = np.array([p[1] + dz], dtype=np.float32)
    assert abs(dy) > math.sqrt(P["fol_chi2_max"] * 1e-5) or abs(dz) > math.sqrt(P["fol_chi2_max"] * 1e-5)
    want, vals = exhaustive_search(y, z, np.array([r], np.uint8), r, p, C, P)
    assert want == 0 and vals[0] < P["fol_chi2_max"]
    got, _ = oracle.follow_search(y, z, np.array([r], np.uint8), np.zeros(1, np.uint8), geom1(), P, 0, r, p,
                                  oracle.full_to_sym15(C))
    assert got == 0


def test_row_search_exact_tie_takes_smallest_id_and_flags():
    r = 12
    y = np.array([0.30, 0.10, -0.10, 0.10, -0.10], dtype=np.float32)
    z = np.array([30.0, 30.0, 30.0, 30.0, 30.0], dtype=np.float32)
    row = np.full(5, r, dtype=np.uint8)
    C = np.diag([0.01, 0.01, 1, 1, 1])
    got, flag = oracle.follow_search(y, z, row, np.zeros(5, np.uint8), geom1(), P, 0, r, np.array([0, 30.0, 0, 0, 0]),
                                     oracle.full_to_sym15(C))
    assert got == 1 and flag & oracle.F_ARGMIN  # ids 1..4 all at chi2 = 0.01/(0.01+0.0036); smallest id wins


def test_row_search_prefers_chi2_over_distance():
    """Strong y-z correlation: the nearer hit in distance has the larger chi2."""
    r = 20
    C = np.diag([0.5, 0.5, 1, 1, 1]).astype(float)
    C[0, 1] = C[1, 0] = 0.49
    p = np.array([0.0, 100.0, 0, 0, 0])
    # along the correlation axis (far, small chi2) and across it (near, large chi2)
    y = np.array([0.8, 0.25], dtype=np.float32)
    z = np.array([100.8, 99.75], dtype=np.float32)
    row = np.full(2, r, dtype=np.uint8)
    got, _ = oracle.follow_search(y, z, row, np.zeros(2, np.uint8), geom1(), P, 0, r, p, oracle.full_to_sym15(C))
    want, _ = exhaustive_search(y, z, row, r, p, C, P)
    assert got == want == 0


# ------------------------------------------------------------------------------ N_miss gap rule
def one_clean_track(seed):
    """A single noise-free helix crossing every pad row of one sector exactly once."""
    w = dataclasses.replace(synth.sector_event(seed), mult_fixed=1, pt_lo=1.0, pt_hi=10.0, sigma_y=0.0, sigma_z=0.0,
                            eff=1.0, noise_frac=0.0, phi_inset_deg=3.0, eta_max=0.6)
    ev = synth.generate(w)
    ok = ev.n == R_ROWS and np.array_equal(np.sort(ev.row), np.arange(R_ROWS))
    return ev, w, ok


def clean_tracks(n_want=3):
    out = []
    seed = 300
    while len(out) < n_want:
        ev, w, ok = one_clean_track(seed)
        if ok:
            out.append((ev, w))
        seed += 1
    return out


@pytest.mark.parametrize("n_miss", [10, 4])
@pytest.mark.parametrize("where", ["outer", "inner"])
def test_gap_of_n_miss_rows_is_bridged_and_one_more_ends_the_tracklet(n_miss, where):
    """A gap of N_miss rows is bridged (one track, every remaining hit); N_miss + 1 rows end the pass.

    'outer': the gap leaves only three rows above it, too few for a chain of their own, so only pass A
    of the long chain below can cross it.  'inner': three rows below the gap, crossed only by pass B
    of the chain above."""
    prm = dict(P, n_miss_max=n_miss)
    for ev, w in clean_tracks():
        for gap in (n_miss, n_miss + 1):
            if where == "outer":
                lo = R_ROWS - 3 - gap
            else:
                lo = 3
            hi = lo + gap  # rows lo .. hi-1 removed
            keep = (ev.row < lo) | (ev.row >= hi)
            y, z, row, sec = ev.y[keep], ev.z[keep], ev.row[keep], ev.sector[keep]
            ids = np.nonzero(keep)[0]
            res = oracle.track(y, z, row, sec, synth.geometry(w), prm, synth.BZ)
            assert res["n_tracks"] == 1, (gap, res["n_tracks"])
            hs = np.sort(ids[res["trk_hits"]])
            assert not any(res["tl_flag"])
            if gap == n_miss:
                assert np.array_equal(hs, np.sort(ids)), (where, gap, hs.size, ids.size)
            else:
                side = ev.row[ids] < lo if where == "inner" else ev.row[ids] >= hi
                expect = np.sort(ids[~side])  # the long side only
                assert np.array_equal(hs, expect), (where, gap, hs.size, expect.size)


# ------------------------------------------------------------------------------ sector-edge stop
def edge_case_clusters(curve):
    """Clusters on every pad row along `curve(x) -> (y, z)`, placed even where the curve has left
    the sector (|y| > x tan(half angle))."""
    rx = synth.row_x().astype(np.float64)
    y = np.empty(R_ROWS); z = np.empty(R_ROWS)
    for r in range(R_ROWS):
        y[r], z[r] = curve(rx[r])
    return y.astype(np.float32), z.astype(np.float32), np.arange(R_ROWS, dtype=np.uint8), np.zeros(R_ROWS, np.uint8)


def line(y0, slope, z0, tz):
    """Straight line y = y0 + slope (x - 85), z linear in the path length (dz/ds = tz)."""
    c = 1.0 / math.sqrt(1.0 + slope * slope)
    return lambda x: (y0 + slope * (x - 85.0), z0 + tz * (x - 85.0) / c)


def circle(y0, slope0, radius, turn, z0, tz):
    """Circle through (85, y0) with slope slope0, bending towards +y (turn=+1) or -y (turn=-1);
    z linear in the arc length (dz/ds = tz).  Closed-form geometry of the curve, no propagation."""
    phi0 = math.atan(slope0)
    # centre on the inner side of the turn
    xc = 85.0 - turn * radius * math.sin(phi0)
    yc = y0 + turn * radius * math.cos(phi0)

    def f(x):
        u = (x - xc) / radius
        y = yc - turn * radius * math.sqrt(1.0 - u * u)
        ang = math.asin(u) - math.asin((85.0 - xc) / radius)
        return y, z0 + tz * radius * ang

    return f


@pytest.mark.parametrize("curve", [line(-3.0, 0.35, 40.0, 0.2), line(4.0, -0.42, 120.0, -0.1),
                                   circle(-2.0, 0.13, 500.0, +1, 60.0, 0.3),
                                   circle(1.0, -0.08, 300.0, -1, 180.0, 0.25)])
def test_pass_ends_at_first_row_beyond_edge_plus_margin(curve):
    y, z, row, sec = edge_case_clusters(curve)
    rx = synth.row_x().astype(np.float64)
    th = float(synth.tan_half())
    yy = np.array([curve(x)[0] for x in rx])
    lim = rx * th + P["edge_margin"]
    beyond = np.abs(yy) > lim
    assert beyond.any() and not beyond[:20].any()
    r_stop = int(np.argmax(beyond))
    # a clear crossing: no row within 0.02 cm of the limit, and the margin matters
    assert np.all(np.abs(np.abs(yy) - lim) > 0.02)
    assert int(np.argmax(np.abs(yy) > rx * th)) < r_stop - 3
    res = oracle.track(y, z, row, sec, geom1(), P, synth.BZ)
    assert res["n_tracks"] == 1
    assert not any(res["tl_flag"] & oracle.F_EDGE)
    hs = np.sort(res["trk_hits"])
    assert np.array_equal(hs, np.arange(r_stop)), (r_stop, hs.size)
    # without the edge stop the same clusters give the whole curve
    res2 = oracle.track(y, z, row, sec, geom1(), dict(P, edge_margin=500.0), synth.BZ)
    assert res2["n_tracks"] == 1 and np.array_equal(np.sort(res2["trk_hits"]), np.arange(R_ROWS))


def test_bin_size_invariance_with_clusters_outside_the_grid():
    """Clusters beyond the grid's y range and outside [z_min, z_max] live in the edge bins; a query
    box beyond the grid must still visit them, so no result depends on the bin size."""
    rng = np.random.default_rng(77)
    ev = synth.generate(synth.SECTOR_EVENT)
    rx = synth.row_x().astype(np.float64)
    th = float(synth.tan_half())
    ys, zs, rs = [ev.y], [ev.z], [ev.row]
    for curve in (line(-3.0, 0.35, 40.0, 0.2), line(4.0, -0.42, 120.0, -0.1), line(0.0, 0.02, 5.0, -0.3),
                  line(0.0, 0.02, 240.0, 0.35)):
        y, z, r, _ = edge_case_clusters(curve)
        ys.append(y); zs.append(z); rs.append(r)
    k = 400
    rr = rng.integers(0, R_ROWS, k)
    side = rng.choice([-1.0, 1.0], k)
    ys.append((side * (rx[rr] * th + rng.uniform(0.5, 60.0, k))).astype(np.float32))
    zs.append(rng.uniform(-30, 280, k).astype(np.float32))
    rs.append(rr.astype(np.uint8))
    y, z, row = np.concatenate(ys), np.concatenate(zs), np.concatenate(rs)
    sec = np.zeros_like(row)
    outs = [oracle.track(y, z, row, sec, geom1(), dict(P, bin_y=by, bin_z=bz), synth.BZ)
            for by, bz in ((8.0, 8.0), (0.9, 1.7), (30.0, 60.0))]
    added = np.isin(np.arange(ev.n, y.size), outs[0]["trk_hits"]).sum()
    assert added > 300  # the added lines are tracked (up to the edge stop for the two leaving the sector)
    for o in outs[1:]:
        for key in ("up", "dn", "up_c", "dn_c", "start_id", "tl_hits", "trk_off", "trk_hits", "hit_key"):
            assert np.array_equal(outs[0][key], o[key]), key
