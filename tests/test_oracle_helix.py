"""Pins of the oracle's sector-local helix model (propagation and its Jacobian).

* Exact geometry: propagating the generator's exact state between consecutive plane crossings
  of one leg lands on the next crossing (the generator finds crossings by circle/plane
  intersection in the global frame, a different formulation).
* Physics: the closed form agrees with an RK4 integration of the Lorentz force in 3-D.
* The zero-curvature limit is a straight line.
* The analytic Jacobian agrees with central differences.
"""
import dataclasses
import math

import numpy as np
import pytest

import oracle
import synth

KC = 0.00299792458


def tracker_state(ev, i):
    """Exact state of cluster i in the increasing-x convention (y, z, sin phi, dz/ds, q/pT)."""
    ph, t, q = ev.exact["phi_loc"][i], ev.exact["dzds"][i], ev.exact["qpt"][i]
    s = math.sin(ph)
    if math.cos(ph) < 0:  # the leg runs towards smaller x: describe it reversed
        s, t, q = -s, -t, -q
    return np.array([ev.exact["y_true"][i], ev.exact["z_true"][i], s, t, q])


@pytest.fixture(scope="module")
def exact_event():
    w = dataclasses.replace(synth.scaled(synth.PBPB_EVENT, 0.04), sigma_y=0.0, sigma_z=0.0, eff=1.0,
                            noise_frac=0.0)
    return synth.generate(w, want_exact=True)


def test_propagation_hits_next_crossing(exact_event):
    ev = exact_event
    rx = synth.row_x().astype(np.float64)
    order = np.lexsort((ev.crossing, ev.particle))
    worst = 0.0
    n = 0
    for a, b in zip(order[:-1], order[1:]):
        if ev.leg[a] != ev.leg[b] or ev.crossing[b] != ev.crossing[a] + 1:
            continue
        p0 = tracker_state(ev, a)
        p1, _, failed = oracle.propagate(p0, rx[ev.row[a]], rx[ev.row[b]], synth.BZ)
        e = tracker_state(ev, b)
        if failed:  # only allowed where the true |sin phi| reaches the propagation limit
            assert max(abs(p0[2]), abs(e[2])) >= 0.999
            continue
        worst = max(worst, abs(p1[0] - e[0]), abs(p1[1] - e[1]), abs(p1[2] - e[2]))
        n += 1
    assert n > 5000
    assert worst < 1e-9, worst


def test_propagation_long_steps_both_directions(exact_event):
    """Steps over many rows (up to 40) forwards and backwards, low pT included."""
    ev = exact_event
    rx = synth.row_x().astype(np.float64)
    order = np.lexsort((ev.crossing, ev.particle))
    leg = ev.leg[order]
    worst = 0.0
    for lg in np.unique(leg)[:300]:
        idx = order[leg == lg]
        if idx.size < 20:
            continue
        for a, b in ((idx[0], idx[-1]), (idx[-1], idx[0]), (idx[3], idx[min(idx.size - 1, 43)])):
            p1, _, failed = oracle.propagate(tracker_state(ev, a), rx[ev.row[a]], rx[ev.row[b]], synth.BZ)
            if failed:
                continue
            e = tracker_state(ev, b)
            worst = max(worst, abs(p1[0] - e[0]), abs(p1[1] - e[1]), abs(p1[2] - e[2]))
    assert worst < 1e-8, worst


def rk4_lorentz(p, x0, x1, bz, h=0.02):
    """3-D RK4 of dr/dl = u, du/dl = (c q Bz / |p|) u x z_hat, stopped on the plane x = x1."""
    y, z, s, t, q = p
    c = math.sqrt(1 - s * s)
    pt = 1.0 / abs(q)
    charge = math.copysign(1.0, q)
    pmag = pt * math.sqrt(1 + t * t)
    kappa = KC * charge * bz / pmag

    def f(st):
        r, u = st[:3], st[3:]
        du = kappa * np.array([u[1], -u[0], 0.0])  # u x z_hat = (u_y, -u_x, 0)
        return np.concatenate([u, du])

    st = np.array([x0, y, z, c, s, t]) / np.array([1, 1, 1, math.sqrt(1 + t * t), math.sqrt(1 + t * t), math.sqrt(1 + t * t)])
    st[:3] = [x0, y, z]
    sgn = 1.0 if x1 > x0 else -1.0
    hh = sgn * h

    def step(st, hh):
        k1 = f(st); k2 = f(st + 0.5 * hh * k1); k3 = f(st + 0.5 * hh * k2); k4 = f(st + hh * k3)
        return st + hh / 6.0 * (k1 + 2 * k2 + 2 * k3 + k4)

    while True:
        nxt = step(st, hh)
        if (nxt[0] - x1) * sgn >= 0:
            break
        st = nxt
    # Newton on the step length to land on x = x1
    a = 0.0
    for _ in range(30):
        cur = step(st, a)
        g = cur[0] - x1
        a -= g / cur[3]
        if abs(g) < 1e-14:
            break
    end = step(st, a)
    return end[1], end[2]


@pytest.mark.parametrize("pt,charge,s0,t0", [(0.08, 1, 0.3, 0.5), (0.15, -1, -0.6, -0.2), (1.0, 1, 0.0, 0.9),
                                             (5.0, -1, 0.2, 0.0), (0.3, -1, 0.7, 1.2)])
def test_closed_form_matches_rk4_lorentz(pt, charge, s0, t0):
    p = np.array([1.5, 40.0, s0, t0, charge / pt])
    for dx in (1.07, 5.0, -3.2, 12.0):
        p1, _, failed = oracle.propagate(p, 100.0, 100.0 + dx, synth.BZ)
        if failed:
            continue
        ry, rz = rk4_lorentz(p, 100.0, 100.0 + dx, synth.BZ, h=0.005)
        assert abs(p1[0] - ry) < 1e-8 and abs(p1[1] - rz) < 1e-8, (dx, p1[:2], ry, rz)


def test_positive_charge_bends_to_negative_y():
    p1, _, _ = oracle.propagate(np.array([0.0, 0.0, 0.0, 0.0, 1.0 / 0.5]), 100.0, 120.0, synth.BZ)
    assert p1[0] < 0 and p1[2] < 0


def test_zero_curvature_is_a_straight_line():
    for s, t in ((0.3, 0.7), (-0.8, -0.1), (0.0, 2.0)):
        p = np.array([3.0, 20.0, s, t, 0.0])
        p1, _, _ = oracle.propagate(p, 90.0, 131.0, synth.BZ)
        c = math.sqrt(1 - s * s)
        assert p1[0] == pytest.approx(3.0 + 41.0 * s / c, abs=1e-12)
        assert p1[1] == pytest.approx(20.0 + t * 41.0 / c, abs=1e-12)
        assert p1[2] == s


def test_propagation_failure_at_s_max():
    p = np.array([0.0, 0.0, 0.95, 0.0, -20.0])  # turns fast towards |sin phi| = 1
    _, _, failed = oracle.propagate(p, 100.0, 110.0, synth.BZ)
    assert failed


@pytest.mark.parametrize("seed", range(12))
def test_jacobian_matches_central_differences(seed):
    rng = np.random.default_rng(seed)
    p = np.array([rng.uniform(-20, 20), rng.uniform(0, 250), rng.uniform(-0.7, 0.7), rng.uniform(-1, 1),
                  rng.choice([-1, 1]) * 10 ** rng.uniform(-1, 1.2)])
    x0 = rng.uniform(85, 240)
    dx = rng.choice([-1, 1]) * rng.uniform(0.5, 15)
    _, F, failed = oracle.propagate(p, x0, x0 + dx, synth.BZ)
    if failed:
        pytest.skip("step leaves |sin phi| < s_max")
    num = np.zeros((5, 5))
    for j in range(5):
        h = 1e-6 * max(1.0, abs(p[j]))
        pp, pm = p.copy(), p.copy()
        pp[j] += h
        pm[j] -= h
        fp, _, f1 = oracle.propagate(pp, x0, x0 + dx, synth.BZ)
        fm, _, f2 = oracle.propagate(pm, x0, x0 + dx, synth.BZ)
        assert not (f1 or f2)
        num[:, j] = (fp - fm) / (2 * h)
    err = np.abs(num - F) / np.maximum(1.0, np.abs(F))
    assert err.max() < 1e-6, (err.max(), F, num)
