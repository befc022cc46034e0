"""Pins of the oracle's cluster flags (Sec. 4, cluster removal) on hand-built geometries.

Every expected flag follows from closed forms: with Bz = 0 a track is a straight line
(y = y0 + tan(phi) dx, z = z0 + t dx / cos(phi)); with Bz != 0 and sin(phi0) = 0 it is the circle
y = y0 + (1 - sqrt(1 - (k dx)^2)) / k, k = -0.00299792458 Bz q/pT.
"""
import numpy as np
import pytest

import oracle

A, J, P, RA, RB = (oracle.FLAG_ATTACHED, oracle.FLAG_ADJACENT, oracle.FLAG_PROTECTED, oracle.FLAG_REMOVE_A,
                   oracle.FLAG_REMOVE_B)
ROWS = 16
GEOM = {"n_rows": ROWS, "row_x": (100.0 + np.arange(ROWS)).astype(np.float32), "n_sectors": 2}


class Event:
    def __init__(self):
        self.y, self.z, self.row, self.sector = [], [], [], []
        self.tracks = []  # (hit ids, sector, state)

    def cluster(self, y, z, r, s=0):
        self.y.append(y)
        self.z.append(z)
        self.row.append(r)
        self.sector.append(s)
        return len(self.y) - 1

    def track(self, pos, rows, state, s=0):
        """a track with one cluster per row at pos(r) and its state at the first row"""
        ids = [self.cluster(*pos(r), r, s) for r in rows]
        self.tracks.append((ids, s, rows[0], state))
        return ids

    def flags(self, bz=0.0):
        off, nh, hits, sec, xr, st = [], [], [], [], [], []
        for ids, s, r0, state in self.tracks:
            off.append(len(hits))
            nh.append(len(ids))
            hits += ids
            sec.append(s)
            xr.append(GEOM["row_x"][r0])
            st.append(state)
        t = {"off": np.array(off, np.int32), "nh": np.array(nh, np.int32), "hits": np.array(hits, np.int32),
             "sector": np.array(sec, np.int32), "x_ref": np.array(xr, np.float32),
             "state": np.array(st, np.float32).reshape(-1, 5)}
        f, tie = oracle.cluster_flags(np.array(self.y, np.float32), np.array(self.z, np.float32),
                                      np.array(self.row, np.uint8), np.array(self.sector, np.uint8), GEOM, bz, t)
        assert not tie.any()
        return f


def test_tube_radius_and_span():
    e = Event()
    hits = e.track(lambda r: (0.0, 0.0), list(range(2, 10)), [0, 0, 0, 0, 0.5])
    near = e.cluster(1.4, 0.0, 5)            # 1.4 cm: adjacent
    far = e.cluster(1.6, 0.0, 5)             # 1.6 cm: not
    diag_in = e.cluster(1.0, 1.0, 6)         # sqrt(2) = 1.414: adjacent
    diag_out = e.cluster(1.1, 1.1, 6)        # 1.556: not
    other_sector = e.cluster(0.0, 0.0, 5, 1)
    past_span = e.cluster(0.0, 0.0, 12)      # the track spans rows 2..9 only
    f = e.flags()
    assert np.all(f[hits] == A | J | P)
    assert f[near] == J | P and f[diag_in] == J | P
    for c in (far, diag_out, other_sector, past_span):
        assert f[c] == RB


def test_sloped_line_in_z():
    # t = dz/ds = 0.5 and phi = 0: z = 0.5 dx on the row plane
    e = Event()
    e.track(lambda r: (0.0, 0.5 * (r - 2)), list(range(2, 10)), [0, 0, 0, 0.5, 0.5])
    on = e.cluster(0.0, 0.5 * 6 + 1.4, 8)
    off = e.cluster(0.0, 0.5 * 6 - 1.6, 8)
    f = e.flags()
    assert f[on] == J | P and f[off] == RB


def test_low_momentum_circle_is_removable_by_strategy_a():
    bz, qpt = 0.5, 25.0                      # pT = 40 MeV/c <= 50: not protected
    k = -0.00299792458 * bz * qpt
    x0 = float(GEOM["row_x"][2])

    def yc(r):
        dx = float(GEOM["row_x"][r]) - x0
        return (1.0 - np.sqrt(1.0 - (k * dx) ** 2)) / k

    e = Event()
    hits = e.track(lambda r: (yc(r), 0.0), list(range(2, 12)), [0, 0, 0, 0, qpt])
    inside = e.cluster(yc(9) + 1.4, 0.0, 9)
    outside = e.cluster(yc(9) - 1.6, 0.0, 9)
    f = e.flags(bz)
    assert np.all(f[hits] == A | J | RA | RB)
    assert f[inside] == J | RA | RB and f[outside] == RB
    # the same circle at 60 MeV/c is protected
    e2 = Event()
    k2 = -0.00299792458 * bz * (1 / 0.06)
    h2 = e2.track(lambda r: ((1.0 - np.sqrt(1.0 - (k2 * (float(GEOM["row_x"][r]) - x0)) ** 2)) / k2, 0.0),
                  list(range(2, 12)), [0, 0, 0, 0, 1 / 0.06])
    assert np.all(e2.flags(bz)[h2] == A | J | P)


@pytest.mark.parametrize("sphi, protected", [(0.90, True), (0.95, False)])
def test_local_inclination_limit(sphi, protected):
    tphi = sphi / np.sqrt(1 - sphi * sphi)   # |phi| = 64.2 or 71.8 degrees
    e = Event()
    hits = e.track(lambda r: (tphi * (r - 2), 0.0), list(range(2, 8)), [0, 0, sphi, 0, 0.5])
    f = e.flags()
    assert np.all(f[hits] == (A | J | P if protected else A | J | RA | RB))


def test_ambiguity_goes_to_the_higher_momentum_track():
    e = Event()
    e.track(lambda r: (0.0, 0.0), list(range(2, 10)), [0, 0, 0, 0, 0.5])     # pT 2 GeV/c
    e.track(lambda r: (1.0, 0.0), list(range(2, 10)), [1.0, 0, 0, 0, 25.0])  # pT 40 MeV/c
    both = e.cluster(0.5, 0.0, 5)
    low_only = e.cluster(2.0, 0.0, 5)
    high_only = e.cluster(-1.0, 0.0, 5)
    f = e.flags()
    assert f[both] == J | P and f[high_only] == J | P
    assert f[low_only] == J | RA | RB


@pytest.mark.parametrize("flat_first", [True, False])
def test_equal_momentum_goes_to_the_smaller_index(flat_first):
    # same |q/pT|; one flat track and one at 71.8 degrees crossing it at row 5
    sphi = 0.95
    tphi = sphi / np.sqrt(1 - sphi * sphi)
    e = Event()
    flat = lambda: e.track(lambda r: (0.0, 0.0), list(range(2, 10)), [0, 0, 0, 0, 0.5])
    steep = lambda: e.track(lambda r: (tphi * (r - 5), 0.0), list(range(3, 8)), [-2 * tphi, 0, sphi, 0, -0.5])
    if flat_first:
        flat(); steep()
    else:
        steep(); flat()
    shared = e.cluster(0.3, 0.0, 5)          # inside both tubes
    f = e.flags()
    assert f[shared] == (J | P if flat_first else J | RA | RB)


def test_no_tracks_everything_is_removable_by_b_only():
    e = Event()
    c = [e.cluster(float(i), 0.0, i % ROWS) for i in range(5)]
    assert np.all(e.flags()[c] == RB)
