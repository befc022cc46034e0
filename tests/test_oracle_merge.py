"""Pins of the merging oracle (looper legs and sector segments of one helix, then one refit):
the helix of a track equals the circle through three of its exact crossings, noise-free loopers
merge into exactly one track per particle, the refit of noise-free hits passes through every
exact crossing, and on smeared hits the refit is the weighted least-squares minimum."""
import dataclasses
import math

import numpy as np
import pytest

import oracle
import synth
from oracle import merge as om

P = synth.TRACKER_PARAMS


def looper_event(seed, sigma=0.0, n=60):
    w = dataclasses.replace(synth.sector_event(seed), only_sector=-1, phi_mode=1, pt_lo=0.06, pt_hi=0.4,
                            sigma_y=sigma, sigma_z=sigma, eff=1.0, noise_frac=0.0, mult_fixed=n)
    return w, synth.generate(w, want_exact=True)


def tracked(ev, geom):
    o = oracle.track(ev.y, ev.z, ev.row, ev.sector, geom, P, synth.BZ)
    t = oracle.tracks_for_flags(o, geom, ev.sector)
    nt = int(o["n_tracks"])
    H, CH = om.helix_params(t["state"], t["x_ref"], t["sector"], o["tl_cov"][o["trk_tl"][:nt]], synth.BZ)
    part = np.array([np.bincount(np.maximum(ev.particle[t["hits"][t["off"][k]:t["off"][k] + t["nh"][k]]], 0)).argmax()
                     for k in range(nt)])
    return o, t, H, CH, part


def circumcentre(p1, p2, p3):
    (ax, ay), (bx, by), (cx, cy) = p1, p2, p3
    d = 2 * (ax * (by - cy) + bx * (cy - ay) + cx * (ay - by))
    ux = ((ax * ax + ay * ay) * (by - cy) + (bx * bx + by * by) * (cy - ay) + (cx * cx + cy * cy) * (ay - by)) / d
    uy = ((ax * ax + ay * ay) * (cx - bx) + (bx * bx + by * by) * (ax - cx) + (cx * cx + cy * cy) * (bx - ax)) / d
    return ux, uy


@pytest.mark.parametrize("seed", [31, 32])
def test_helix_of_a_track_is_the_circle_through_its_exact_crossings(seed):
    """Each leg's exact state at its innermost crossing (FP32, as the tracker stores states): its
    centre and radius equal those of the circle through three of the leg's exact crossings, and its
    pitch and phase reproduce the exact z of every crossing."""
    w, ev = looper_event(seed)
    geom = synth.geometry(w)
    X, Y, Zt = om.hit_points(ev.exact["y_true"], ev.exact["z_true"], ev.row, ev.sector, geom["row_x"])
    legs = [l for l in np.unique(ev.leg[ev.leg >= 0]) if (ev.leg == l).sum() >= 10]
    st, xr, sec, hits = [], [], [], []
    for lg in legs:
        h = np.nonzero(ev.leg == lg)[0]
        h = h[np.argsort(ev.row[h])]
        i = h[0]
        ph, tt, q = ev.exact["phi_loc"][i], ev.exact["dzds"][i], ev.exact["qpt"][i]
        s = math.sin(ph)
        if math.cos(ph) < 0:
            s, tt, q = -s, -tt, -q
        st.append([ev.exact["y_true"][i], ev.exact["z_true"][i], s, tt, q])
        xr.append(geom["row_x"][ev.row[i]])
        sec.append(ev.sector[i])
        hits.append(h)
    H, _ = om.helix_params(np.array(st, dtype=np.float32), np.array(xr, dtype=np.float32), np.array(sec),
                           np.zeros((len(st), 15)), synth.BZ)
    assert len(legs) > 100
    for k, h in enumerate(hits):
        i = h[[0, len(h) // 2, -1]]
        xc, yc = circumcentre(*zip(X[i], Y[i]))
        rho = math.hypot(X[i[0]] - xc, Y[i[0]] - yc)
        assert abs(H[k, 0] - xc) < 2e-3 * max(1.0, rho / 50) and abs(H[k, 1] - yc) < 2e-3 * max(1.0, rho / 50), k
        assert abs(1.0 / H[k, 2] - rho) < 1e-4 * rho, k
        psi = np.arctan2(Y[h] - H[k, 1], X[h] - H[k, 0])
        dz = Zt[h] - H[k, 4] - H[k, 3] * psi  # multiples of one turn 2 pi w
        turns = dz / (2 * math.pi * H[k, 3])
        assert np.abs(turns - np.round(turns)).max() * abs(2 * math.pi * H[k, 3]) < 1e-2, k


@pytest.mark.parametrize("seed", [11, 12, 13])
def test_noise_free_loopers_merge_into_one_track_per_particle(seed):
    w, ev = looper_event(seed)
    o, t, H, CH, part = tracked(ev, synth.geometry(w))
    lab = om.merge_labels(H, CH)
    assert len(part) > 2 * len(np.unique(part))  # several legs per particle before merging
    for g in np.unique(lab):
        assert len(np.unique(part[lab == g])) == 1, "a merged track mixes particles"
        assert g == np.nonzero(lab == g)[0].min()  # labelled by the lowest member
    for p in np.unique(part):
        assert len(np.unique(lab[part == p])) == 1, f"particle {p} split"


def test_noise_free_refit_passes_through_every_exact_crossing():
    w, ev = looper_event(11)
    geom = synth.geometry(w)
    o, t, H, CH, part = tracked(ev, geom)
    lab = om.merge_labels(H, CH)
    X, Y, Z = om.hit_points(ev.y, ev.z, ev.row, ev.sector, geom["row_x"])
    Xt, Yt, Zt = om.hit_points(ev.exact["y_true"], ev.exact["z_true"], ev.row, ev.sector, geom["row_x"])
    n_checked = 0
    for g in np.unique(lab):
        ids = np.concatenate([t["hits"][t["off"][k]:t["off"][k] + t["nh"][k]] for k in np.nonzero(lab == g)[0]])
        hh = np.concatenate([np.repeat(H[k:k + 1], t["nh"][k], axis=0) for k in np.nonzero(lab == g)[0]])
        th, cov, chi2, ndf, ps = om.refit(X[ids], Y[ids], Z[ids], H[g], P["sigma_y"], P["sigma_z"], hh)
        rt = np.hypot(Xt[ids] - th[0], Yt[ids] - th[1]) - th[2]
        rz = Zt[ids] - th[3] - th[4] * ps
        assert np.abs(rt).max() < 1e-4 and np.abs(rz).max() < 1e-4, (g, np.abs(rt).max(), np.abs(rz).max())
        n_checked += len(ids)
    assert n_checked > 5000


def test_refit_is_the_weighted_least_squares_minimum():
    """Smeared loopers: at the refit the gradient of chi2 vanishes, every small step raises chi2, and
    chi2/ndf is of order one (the model is the generator's)."""
    w, ev = looper_event(14, sigma=0.06, n=40)
    w = dataclasses.replace(w, sigma_z=0.1)
    ev = synth.generate(w, want_exact=True)
    geom = synth.geometry(w)
    o, t, H, CH, part = tracked(ev, geom)
    lab = om.merge_labels(H, CH)
    X, Y, Z = om.hit_points(ev.y, ev.z, ev.row, ev.sector, geom["row_x"])
    rng = np.random.default_rng(3)
    tot_chi2 = tot_ndf = 0
    for g in np.unique(lab):
        ids = np.concatenate([t["hits"][t["off"][k]:t["off"][k] + t["nh"][k]] for k in np.nonzero(lab == g)[0]])
        if len(np.unique(part[lab == g])) != 1:
            continue
        hh = np.concatenate([np.repeat(H[k:k + 1], t["nh"][k], axis=0) for k in np.nonzero(lab == g)[0]])
        th, cov, chi2, ndf, ps = om.refit(X[ids], Y[ids], Z[ids], H[g], 0.06, 0.1, hh)
        def chi2_at(v):
            dx, dy = X[ids] - v[0], Y[ids] - v[1]
            d = np.arctan2(dy, dx) - ps
            pp = ps + d - 2 * math.pi * np.round(d / (2 * math.pi))
            return float(np.sum(((np.hypot(dx, dy) - v[2]) / 0.06) ** 2 + ((Z[ids] - v[3] - v[4] * pp) / 0.1) ** 2))

        assert chi2_at(th) == pytest.approx(chi2, rel=1e-10)
        sig = np.sqrt(np.diag(cov))
        for _ in range(20):  # along the fit's own error ellipse a 0.1-sigma step raises chi2 by ~0.01
            d = rng.normal(size=5) * sig * 0.1
            assert chi2_at(th + d) > chi2 - 1e-9 * chi2
        num = np.array([(chi2_at(th + e * s * 1e-5) - chi2_at(th - e * s * 1e-5)) / (2e-5 * s)
                        for e, s in zip(np.eye(5), sig)])
        assert np.all(np.abs(num * sig) < 1e-3), num * sig  # gradient in units of one sigma: ~0
        tot_chi2 += chi2
        tot_ndf += ndf
    # the transverse residual is the distance from the circle, the pad-row error projected on the
    # circle's normal, so it is weighted with an upper bound of its error: chi2/ndf a bit below one
    assert 0.6 < tot_chi2 / tot_ndf < 1.1, tot_chi2 / tot_ndf
