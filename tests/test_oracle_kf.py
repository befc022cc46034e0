"""Pins of the oracle's Kalman filter.

* On a linear(ised) model with no process noise, a Kalman filter is exactly the weighted
  least-squares estimate; the oracle's update and covariance transport must reproduce the
  closed form (normal equations) to rounding.
* On smeared tracks from the generator (whose model the fit matches), pulls of the fitted
  parameters are standard normal and chi2/ndf is about 1.
* Every output covariance is symmetric positive definite.
"""
import dataclasses
import math

import numpy as np
import pytest

import oracle
import synth

SY, SZ = 0.06, 0.1


@pytest.mark.parametrize("seed", range(8))
def test_kf_equals_closed_form_wls(seed):
    rng = np.random.default_rng(100 + seed)
    bz = synth.BZ
    n_pts = rng.integers(5, 40)
    xs = 85.0 + np.sort(rng.choice(152, size=n_pts, replace=False)) * 162.0 / 151.0
    # reference trajectory and its linearisation, step by step
    p_ref = [np.array([rng.uniform(-10, 10), rng.uniform(10, 200), rng.uniform(-0.3, 0.3), rng.uniform(-0.9, 0.9),
                       rng.choice([-1, 1]) * rng.uniform(0.1, 1.5)])]
    Fs, As = [], []
    for i in range(n_pts - 1):
        p1, F, failed = oracle.propagate(p_ref[-1], xs[i], xs[i + 1], bz)
        assert not failed
        Fs.append(F)
        As.append(p1 - F @ p_ref[-1])
        p_ref.append(p1)
    # measurements scattered around the reference
    m = np.array([[p[0] + rng.normal(0, SY), p[1] + rng.normal(0, SZ)] for p in p_ref])
    c0 = np.array([SY * SY, SZ * SZ, 1.0, 1.0, 100.0])
    p_pr = p_ref[0] + np.array([0, 0, rng.normal(0, 0.2), rng.normal(0, 0.2), rng.normal(0, 3)])
    # Kalman filter: first point through the prior (y, z = first measurement), then updates
    p = np.array([m[0, 0], m[0, 1], p_pr[2], p_pr[3], p_pr[4]])
    C = oracle.full_to_sym15(np.diag(c0))
    for i in range(n_pts - 1):
        p = Fs[i] @ p + As[i]
        C = oracle.cov_propagate(C, Fs[i])
        p, C, _, bad = oracle.kf_update(p, C, m[i + 1, 0], m[i + 1, 1], SY * SY, SZ * SZ)
        assert not bad
    # closed form: unknown p0 at the first point; prior information on (s, t, q) only
    Phi = [np.eye(5)]
    phi = [np.zeros(5)]
    for i in range(n_pts - 1):
        Phi.append(Fs[i] @ Phi[-1])
        phi.append(Fs[i] @ phi[-1] + As[i])
    H = np.zeros((2, 5)); H[0, 0] = H[1, 1] = 1
    Vi = np.diag([1 / SY ** 2, 1 / SZ ** 2])
    Pi = np.diag([0, 0, 1 / c0[2], 1 / c0[3], 1 / c0[4]])
    A = Pi.copy()
    b = Pi @ p_pr
    for i in range(n_pts):
        J = H @ Phi[i]
        A += J.T @ Vi @ J
        b += J.T @ Vi @ (m[i] - H @ phi[i])
    cov0 = np.linalg.inv(A)
    pN = Phi[-1] @ (cov0 @ b) + phi[-1]
    covN = Phi[-1] @ cov0 @ Phi[-1].T
    Cf = oracle.sym15_to_full(C)
    assert np.allclose(p, pN, rtol=1e-9, atol=1e-9 * np.abs(pN).max())
    assert np.allclose(Cf, covN, rtol=1e-7, atol=1e-9 * np.abs(covN).max())


def test_update_chi2_is_residual_form():
    C = oracle.full_to_sym15(np.diag([0.01, 0.02, 0.1, 0.1, 1.0]))
    p = np.array([1.0, 2.0, 0.1, 0.2, 0.5])
    _, _, chi2, bad = oracle.kf_update(p, C, 1.3, 1.6, SY * SY, SZ * SZ)
    assert not bad
    assert chi2 == pytest.approx(0.3 ** 2 / (0.01 + SY * SY) + 0.4 ** 2 / (0.02 + SZ * SZ), rel=1e-13)


@pytest.fixture(scope="module")
def fitted_sector_events():
    """Smeared single-sector events (no noise, full efficiency, pT >= 0.3) and their oracle fits."""
    out = []
    for seed in range(40, 52):
        w = dataclasses.replace(synth.sector_event(seed), pt_lo=0.3, eff=1.0, noise_frac=0.0, phi_inset_deg=3.0)
        ev = synth.generate(w, want_exact=True)
        res = oracle.track(ev.y, ev.z, ev.row, ev.sector, synth.geometry(w), synth.TRACKER_PARAMS, synth.BZ)
        out.append((ev, res))
    return out


def _truth_state(ev, i):
    ph, t, q = ev.exact["phi_loc"][i], ev.exact["dzds"][i], ev.exact["qpt"][i]
    s = math.sin(ph)
    if math.cos(ph) < 0:
        s, t, q = -s, -t, -q
    return np.array([ev.exact["y_true"][i], ev.exact["z_true"][i], s, t, q])


def test_pulls_and_chi2(fitted_sector_events):
    pulls = []
    chi2ndf = []
    for ev, res in fitted_sector_events:
        for k in range(res["n_tracks"]):
            t = res["trk_tl"][k]
            hits = res["trk_hits"][res["trk_off"][k]:res["trk_off"][k + 1]]
            if np.unique(ev.leg[hits]).size != 1 or res["tl_nhits"][t] != hits.size or hits.size < 40:
                continue
            inner = res["tl_hits"][t][res["tl_row_ref"][t]]
            truth = _truth_state(ev, inner)
            C = oracle.sym15_to_full(res["tl_cov"][t])
            pulls.append((res["tl_state"][t] - truth) / np.sqrt(np.diag(C)))
            # the outermost hit enters through the prior, so 2 n_hits - 5 = ndf - 3 degrees of freedom
            chi2ndf.append(res["tl_chi2"][t] / max(1, res["tl_ndf"][t] - 3))
    pulls = np.array(pulls)
    assert pulls.shape[0] > 800
    mean, rms = pulls.mean(0), pulls.std(0)
    print("pull mean", mean, "rms", rms, "chi2/ndf", np.mean(chi2ndf))
    assert np.all(np.abs(mean) < 0.1), mean
    assert np.all(np.abs(rms - 1) < 0.1), rms
    assert abs(np.mean(chi2ndf) - 1.0) < 0.05


def test_covariances_are_spd(fitted_sector_events):
    n = 0
    for _, res in fitted_sector_events:
        for t in np.nonzero(res["tl_valid"])[0]:
            C = oracle.sym15_to_full(res["tl_cov"][t])
            np.linalg.cholesky(C)
            n += 1
    assert n > 1000
