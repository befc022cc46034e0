"""CPU oracle of track merging and the merged refit (TEST INFRASTRUCTURE ONLY).

Sec. 4 of arXiv:1910.12214: the tracker finds the legs of looping tracks (and the segments of a
track in neighbouring sectors) one by one, and they are then merged into one track; about three
instances of each low-pT looper are found without merging.  Only ``tests/`` may use it.  FP64,
numpy, plain loops.

Readings (the paper names the step, not its method):
* Every track is a piece of one helix.  Its global circle (centre Xc, Yc; curvature k > 0 in the
  counter-clockwise orientation), its pitch w = dz/dpsi (z advance per radian around the centre;
  the same whichever way a leg was fitted) and its phase z0 = z - w psi at its reference point
  (psi = the angle of the point around the centre) describe that helix.  From the sector-local
  state (y, z, sin phi, dz/ds, q/pT) at x_ref in sector s (centre angle 20 deg (s mod 18) + 10 deg,
  z mirrored for s >= 18): phi_g = asin(sin phi) + alpha, kappa = -c Bz q/pT, centre = point +
  (-sin phi_g, cos phi_g) / kappa, k = |kappa|, w = t_g / kappa (t_g the global dz/ds).
* Two tracks are pieces of the same helix when both radii are at most RHO_MAX, their centres lie
  within CENTRE_WINDOW in X and in Y, chi2 of (Xc, Yc, k, w) with the sum of both propagated
  covariances is at most CHI2_HELIX, and their phases agree modulo one turn 2 pi w (at most
  MAX_TURNS turns apart) within PHASE_SIGMAS standard deviations.  Merged tracks are the
  connected components of that relation (union of all such pairs); a component is labelled by
  its lowest track index.
* The refit of a merged track fits one helix (Xc, Yc, rho, z0, w) to all its hits by weighted
  least squares: transverse residual = distance of the hit from the circle (sigma_y), longitudinal
  residual = z - z0 - w psi (sigma_z), each hit's psi unwrapped to the turn that its own track's
  helix predicts, shifted by the whole turns between its track's phase and the first member's, and
  kept continuous from there while the centre moves; Gauss-Newton, each step halved until chi2 does
  not grow, to convergence.
"""
from __future__ import annotations

import math

import numpy as np

RHO_MAX = 600.0          # cm: only helices this tight are merged (their centres are well measured)
CENTRE_WINDOW = 16.0     # cm: |dXc|, |dYc| at most this
CHI2_HELIX = 60.0        # chi2 (4 dof) of (Xc, Yc, k, w)
PHASE_SIGMAS = 5.0       # phase agreement in standard deviations of z0
PHASE_FLOOR = 0.1        # cm added in quadrature to the phase error (FP32 states)
MAX_TURNS = 5            # phases at most this many turns apart
C_LIGHT = 2.99792458e-3  # cm^-1 T^-1 (GeV/c)


def sector_alpha(sector):
    return np.deg2rad(20.0 * (np.asarray(sector) % 18) + 10.0)


def helix_params(state, x_ref, sector, cov15, bz: float, n_sectors_side: int = 18):
    """Per track: h = (Xc, Yc, k, w, z0) and the 5x5 covariance of h, from the FP32 states."""
    st = np.asarray(state, dtype=np.float64).reshape(-1, 5)
    n = len(st)
    x = np.asarray(x_ref, dtype=np.float64)
    sec = np.asarray(sector, dtype=np.int64)
    side = np.where(sec >= n_sectors_side, -1.0, 1.0)
    a = sector_alpha(sec)
    y, z, s, t, q = st.T
    kq = -C_LIGHT * bz
    kap = kq * q
    c = np.sqrt(np.maximum(1.0 - s * s, 0.0))
    phi = np.arcsin(s) + a
    X = x * np.cos(a) - y * np.sin(a)
    Y = x * np.sin(a) + y * np.cos(a)
    with np.errstate(divide="ignore", invalid="ignore"):
        Xc = X - np.sin(phi) / kap
        Yc = Y + np.cos(phi) / kap
        tg = side * t
        w = tg / kap
        psi = np.arctan2(Y - Yc, X - Xc)
        z0 = side * z - w * psi
        k = np.abs(kap)
        # Jacobian d(Xc, Yc, k, w, z0) / d(y, z, s, t, q)
        J = np.zeros((n, 5, 5))
        J[:, 0, 0] = -np.sin(a)
        J[:, 0, 2] = -np.cos(phi) / (kap * c)
        J[:, 0, 4] = np.sin(phi) * kq / kap ** 2
        J[:, 1, 0] = np.cos(a)
        J[:, 1, 2] = -np.sin(phi) / (kap * c)
        J[:, 1, 4] = -np.cos(phi) * kq / kap ** 2
        J[:, 2, 4] = np.sign(kap) * kq
        J[:, 3, 3] = side / kap
        J[:, 3, 4] = -tg * kq / kap ** 2
        # psi = phi - sign(kappa) pi/2 (mod 2 pi): d psi / ds = 1 / c
        J[:, 4, 1] = side
        J[:, 4, 2] = -w / c
        J[:, 4, 3] = -psi * J[:, 3, 3]
        J[:, 4, 4] = -psi * J[:, 3, 4]
    C = np.zeros((n, 5, 5))
    ii, jj = np.tril_indices(5)
    cv = np.asarray(cov15, dtype=np.float64).reshape(-1, 15)
    C[:, ii, jj] = cv
    C[:, jj, ii] = cv
    H = np.stack([Xc, Yc, k, w, z0], axis=1)
    CH = np.einsum("nij,njk,nlk->nil", J, C, J)
    return H, CH


def compatible(hA, CA, hB, CB) -> bool:
    """Same helix test (the reading in the module docstring)."""
    if not (np.all(np.isfinite(hA)) and np.all(np.isfinite(hB))):
        return False
    if not (1.0 / hA[2] <= RHO_MAX and 1.0 / hB[2] <= RHO_MAX):
        return False
    if abs(hA[0] - hB[0]) > CENTRE_WINDOW or abs(hA[1] - hB[1]) > CENTRE_WINDOW:
        return False
    d = hA[:4] - hB[:4]
    S = CA[:4, :4] + CB[:4, :4]
    try:
        chi2 = float(d @ np.linalg.solve(S, d))
    except np.linalg.LinAlgError:
        return False
    if not (chi2 <= CHI2_HELIX):
        return False
    pitch = 2.0 * math.pi * 0.5 * (hA[3] + hB[3])
    if not (abs(pitch) > 0.0):
        return abs(hA[4] - hB[4]) <= PHASE_SIGMAS * math.sqrt(CA[4, 4] + CB[4, 4] + PHASE_FLOOR ** 2)
    m = round((hA[4] - hB[4]) / pitch)
    if abs(m) > MAX_TURNS:
        return False
    dz = hA[4] - hB[4] - m * pitch
    # the m turns between the phases carry the pitch's error too
    var = CA[4, 4] + CB[4, 4] + (math.pi * m) ** 2 * (CA[3, 3] + CB[3, 3]) + PHASE_FLOOR ** 2
    return dz * dz <= PHASE_SIGMAS ** 2 * var


def merge_labels(H, CH) -> np.ndarray:
    """Component label (lowest member index) of every track: brute force over all pairs."""
    n = len(H)
    parent = np.arange(n)

    def find(i):
        while parent[i] != i:
            parent[i] = parent[parent[i]]
            i = parent[i]
        return i

    for a in range(n):
        for b in range(a + 1, n):
            if compatible(H[a], CH[a], H[b], CH[b]):
                ra, rb = find(a), find(b)
                if ra != rb:
                    parent[max(ra, rb)] = min(ra, rb)
    return np.array([find(i) for i in range(n)])


def hit_points(y, z, row, sector, row_x, n_sectors_side: int = 18):
    """Global (X, Y, Z) of clusters."""
    a = sector_alpha(sector)
    x = np.asarray(row_x, dtype=np.float32)[np.asarray(row)].astype(np.float64)
    yy = np.asarray(y, dtype=np.float32).astype(np.float64)
    side = np.where(np.asarray(sector) >= n_sectors_side, -1.0, 1.0)
    return (x * np.cos(a) - yy * np.sin(a), x * np.sin(a) + yy * np.cos(a),
            side * np.asarray(z, dtype=np.float32).astype(np.float64))


def refit(X, Y, Z, h0, sigma_y: float, sigma_z: float, h_hit=None, n_iter: int = 50):
    """Gauss-Newton helix fit of one merged track.  h0 = starting (Xc, Yc, k, w, z0) (the first
    member's helix); h_hit[i] = the helix of the track hit i comes from (default h0).  Each hit's
    turn is that of its own track's helix at the hit, shifted by the whole turns between its track's
    phase and the first member's.  Returns theta = (Xc, Yc, rho, z0, w), its covariance, chi2, ndf
    and the unwrapped psi of every hit."""
    Xc, Yc, rho, w, z0 = h0[0], h0[1], 1.0 / h0[2], h0[3], h0[4]
    hh = np.broadcast_to(np.asarray(h0, dtype=np.float64), (len(X), 5)) if h_hit is None else np.asarray(h_hit)
    psi = np.arctan2(Y - Yc, X - Xc)
    if w == 0:
        turns = np.zeros(len(X))
    else:
        own = np.round((Z - hh[:, 4] - hh[:, 3] * np.arctan2(Y - hh[:, 1], X - hh[:, 0])) / (2 * math.pi * hh[:, 3]))
        shift = np.round((hh[:, 4] - z0) / (2 * math.pi * w))
        # the same point's psi around the first member's centre may differ by one turn from the
        # angle around its own track's centre: take the turn that brings z closest
        base = own + shift
        z_of = z0 + w * (psi + 2 * math.pi * base)
        turns = base + np.round((Z - z_of) / (2 * math.pi * w))
    th = np.array([Xc, Yc, rho, z0, w])
    W = np.concatenate([np.full(len(X), 1.0 / sigma_y ** 2), np.full(len(X), 1.0 / sigma_z ** 2)])

    # each hit's unwrapped angle at the start; later angles move continuously from it (a centre
    # step never makes a hit jump a turn across the branch of atan2)
    psi_start = psi + 2 * math.pi * turns

    def model(v):
        dx, dy = X - v[0], Y - v[1]
        r = np.hypot(dx, dy)
        d = np.arctan2(dy, dx) - psi_start
        ps = psi_start + (d - 2 * math.pi * np.round(d / (2 * math.pi)))
        return dx, dy, r, ps, np.concatenate([r - v[2], Z - v[3] - v[4] * ps])

    dx, dy, r, ps, res = model(th)
    chi2 = float(np.sum(W * res * res))
    for _ in range(n_iter):
        Jt = np.zeros((len(X), 5))
        Jt[:, 0] = -dx / r
        Jt[:, 1] = -dy / r
        Jt[:, 2] = -1.0
        Jz = np.zeros((len(X), 5))
        # d psi / dXc = dy / r^2, d psi / dYc = -dx / r^2
        Jz[:, 0] = -th[4] * dy / r ** 2
        Jz[:, 1] = th[4] * dx / r ** 2
        Jz[:, 3] = -1.0
        Jz[:, 4] = -ps
        J = np.concatenate([Jt, Jz])  # d residual / d theta
        N = J.T @ (W[:, None] * J)
        g = J.T @ (W * res)
        step = np.linalg.solve(N, -g)
        # Gauss-Newton step, halved until chi2 does not grow (at most 30 times)
        for _ in range(30):
            cand = th + step
            c = model(cand)
            c2 = float(np.sum(W * c[4] * c[4]))
            if c2 <= chi2:
                break
            step = 0.5 * step
        else:
            break
        th, (dx, dy, r, ps, res), done = cand, c, chi2 - c2 <= 1e-12 * chi2
        chi2 = c2
        if done:
            break
    N = np.concatenate([np.stack([-dx / r, -dy / r, -np.ones(len(X)), np.zeros(len(X)), np.zeros(len(X))], 1),
                        np.stack([-th[4] * dy / r ** 2, th[4] * dx / r ** 2, np.zeros(len(X)), -np.ones(len(X)), -ps],
                                 1)])
    N = N.T @ (W[:, None] * N)
    return th, np.linalg.inv(N), chi2, 2 * len(X) - 5, ps
