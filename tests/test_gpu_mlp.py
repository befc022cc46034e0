"""Learned triplet scorer on the GPU vs the FP64 reference (needs an MI355X)."""
import os
import sys

import numpy as np
import pytest

import oracle
import synth
from oracle import mlp as omlp
from tests import parity

pytestmark = pytest.mark.gpu
THREADS = min(16, os.cpu_count() or 1)


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


def theta_random(seed, scale=1.0):
    rng = np.random.default_rng(seed)
    return omlp.pack(dict(W1=rng.normal(0, 0.6 * scale, (12, 64)), b1=rng.normal(0, 0.2, 64),
                          W2=rng.normal(0, 0.25 * scale, (64, 64)), b2=rng.normal(0, 0.2, 64),
                          w3=rng.normal(0, 0.3 * scale, 64), b3=rng.normal(0, 0.1, 1))).astype(np.float32)


def dev(a):
    import torch

    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


@pytest.mark.parametrize("n", [1, 15, 16, 17, 1000, 70001])
def test_inference_matches_fp64(ctx, n):
    theta = theta_random(n)
    X = np.random.default_rng(n + 1).normal(0, 1.5, (n, 12)).astype(np.float32)
    got = ctx.mlp_infer(dev(X), dev(theta)).cpu().numpy()
    ref, _ = omlp.forward(omlp.quantize(theta), X.astype(np.float64))
    err = np.abs(got - ref) / np.maximum(1.0, np.abs(ref))
    say(f"[mlp] n={n} max rel err {err.max():.2e}")
    # activations carried as three BF16 terms: FP32-faithful logits
    assert err.max() < 2e-5


def test_gradient_matches_fp64_at_bf16_tolerance(ctx):
    import torch

    theta = theta_random(7)
    rng = np.random.default_rng(8)
    N = 5000
    X = rng.normal(0, 1.2, (N, 12)).astype(np.float32)
    y = (rng.uniform(size=N) < 0.4).astype(np.uint8)
    idx = rng.choice(N, size=4096, replace=False).astype(np.int32)
    grad, loss = ctx.mlp_grad(dev(X), dev(y), dev(idx), dev(theta))
    grad = grad.cpu().numpy()
    loss = float(loss.cpu().numpy()[0])
    ref_loss, ref = omlp.backward(omlp.quantize(theta), X[idx].astype(np.float64), y[idx])
    assert abs(loss - ref_loss) <= 1e-3 * abs(ref_loss)
    scale = np.abs(ref).max()
    err = np.abs(grad - ref) / (np.abs(ref) + 1e-2 * scale)
    say(f"[mlp] grad max err {err.max():.2e} (loss {loss:.6f} vs {ref_loss:.6f})")
    assert err.max() < 2e-2
    cos = float(grad @ ref / np.linalg.norm(grad) / np.linalg.norm(ref))
    assert cos > 0.9999


def test_adam_training_follows_fp64(ctx):
    import torch

    rng = np.random.default_rng(11)
    N = 20000
    X = rng.normal(0, 1.0, (N, 12)).astype(np.float32)
    w_true = rng.normal(0, 1, 12)
    y = ((X @ w_true + 0.3 * rng.normal(size=N)) > 0).astype(np.uint8)
    theta = theta_random(12, 0.5)
    batch, steps = 1024, 30
    order = np.concatenate([rng.permutation(N)[:batch] for _ in range(steps)]).astype(np.int32)
    t_gpu = dev(theta.copy())
    m = torch.zeros(5057, device="cuda:0")
    v = torch.zeros(5057, device="cuda:0")
    losses = ctx.mlp_train(dev(X), dev(y), dev(order), t_gpu, m, v, batch=batch, n_steps=steps, lr=3e-3).cpu().numpy()
    th = theta.astype(np.float64)
    mm = np.zeros_like(th)
    vv = np.zeros_like(th)
    ref_losses = []
    for k in range(steps):
        ids = order[k * batch:(k + 1) * batch]
        lo, g = omlp.backward(omlp.quantize(th), X[ids].astype(np.float64), y[ids])
        ref_losses.append(lo)
        th, mm, vv = omlp.adam_step(th, mm, vv, g, k + 1, lr=3e-3)
    ref_losses = np.array(ref_losses)
    say(f"[mlp] loss {losses[0]:.4f} -> {losses[-1]:.4f}; fp64 {ref_losses[0]:.4f} -> {ref_losses[-1]:.4f}")
    assert losses[-1] < 0.8 * losses[0]
    assert np.all(np.abs(losses - ref_losses) < 2e-2 * np.abs(ref_losses) + 2e-3)
    # Adam moves every parameter by about lr per step whatever the gradient's size, so parameters
    # with near-zero gradients may drift apart; the bulk follows the FP64 trajectory
    final = t_gpu.cpu().numpy()
    assert np.median(np.abs(final - th)) < 5e-4


def test_triplets_match_oracle_windows(ctx):
    w = synth.SECTOR_EVENT
    ev = synth.generate(w)
    geom = synth.geometry(w)
    trip, feats = ctx.triplets(dev(ev.y), dev(ev.z), dev(ev.row), dev(ev.sector), geom, synth.TRACKER_PARAMS)
    trip = trip.cpu().numpy()
    feats = feats.cpu().numpy()
    o = oracle.track(ev.y, ev.z, ev.row, ev.sector, geom, synth.TRACKER_PARAMS, synth.BZ,
                     stages=oracle.STAGE_GRID | oracle.STAGE_NEIGHBOURS)
    # same number of window pairs per middle hit
    cnt = np.bincount(trip[:, 1], minlength=ev.n)
    assert np.array_equal(cnt, o["n_pairs"]), "pair counts differ"
    assert len(np.unique(trip[:, 0].astype(np.int64) * 2 ** 40 + trip[:, 1].astype(np.int64) * 2 ** 20 + trip[:, 2])) == len(trip)
    # features against the FP64 definition
    rx = synth.row_x().astype(np.float64)
    rng = np.random.default_rng(3)
    for k in rng.choice(len(trip), size=min(3000, len(trip)), replace=False):
        d, m, u = trip[k]
        nu = int(np.sum((ev.row == ev.row[m] + 1) & (ev.sector == ev.sector[m])
                        & (np.abs(ev.y.astype(np.float64) - ev.y[m]) <= 2.0 * (rx[ev.row[m] + 1] - rx[ev.row[m]]))
                        & (np.abs(ev.z.astype(np.float64) - ev.z[m]) <= 2.0 * (rx[ev.row[m] + 1] - rx[ev.row[m]]))))
        nd = int(o["n_pairs"][m] // max(1, nu))
        f = oracle.features(rx[ev.row[d]], ev.y[d], ev.z[d], rx[ev.row[m]], ev.y[m], ev.z[m], rx[ev.row[u]], ev.y[u],
                            ev.z[u], 2.0, 2.0, nu, nd)
        assert np.allclose(feats[k], f, rtol=2e-5, atol=2e-5), (k, feats[k], f)
    say(f"[mlp] triplets {len(trip)} on {ev.n} clusters")


@pytest.mark.parametrize("frac", [0.5])
def test_pruned_tracking_parity(ctx, frac):
    """Random scorer, tau at the median logit: about half of the pairs are pruned."""
    from paper_1910_12214_amd import tpcca

    w = synth.scaled(synth.PBPB_EVENT, 0.1)
    ev = synth.generate(w)
    geom = synth.geometry(w)
    theta = theta_random(21)
    trip, feats = ctx.triplets(dev(ev.y), dev(ev.z), dev(ev.row), dev(ev.sector), geom, synth.TRACKER_PARAMS)
    lg = ctx.mlp_infer(feats, dev(theta)).cpu().numpy()
    tau = float(np.quantile(lg, frac))
    out = ctx.track(dev(ev.y), dev(ev.z), dev(ev.row), dev(ev.sector), geom, synth.BZ, synth.TRACKER_PARAMS,
                    mlp=dev(theta), tau_logit=tau)
    trk = tpcca.tracks_to_host(out)
    st = parity.gpu_stages(ctx, synth.N_ROWS)
    prm = dict(synth.TRACKER_PARAMS, mlp_tau_logit=tau, mlp_flag_abs=1e-4)
    qtheta = omlp.quantize(theta)
    o = oracle.track(ev.y, ev.z, ev.row, ev.sector, geom, prm, synth.BZ, mlp=qtheta, n_threads=THREADS)
    o_fma = oracle.track(ev.y, ev.z, ev.row, ev.sector, geom, prm, synth.BZ, mlp=qtheta, n_threads=THREADS, fma=True)
    rep = parity.compare(o, st, trk, ev.n, synth.N_ROWS, leg=ev.leg, o_fma=o_fma,
                         row_of=ev.row, row_x=synth.row_x(), bz=synth.BZ)
    c = trk["counts"]
    say(f"[mlp] pruned parity: {rep.line()} pairs={c[tpcca.CNT_PAIRS]} kept={c[tpcca.CNT_PAIRS_KEPT]}")
    # kept = pairs within the plain criterion's cut whose logit reaches tau: below the
    # half that tau alone keeps, and at least one per linked hit
    assert c[tpcca.CNT_LINKS_RAW] <= c[tpcca.CNT_PAIRS_KEPT] < 0.7 * c[tpcca.CNT_PAIRS]
    assert rep["tracks_compared"] > 500


def test_pruned_parity_when_candidate_lists_overflow(ctx):
    """The one-sector event with windows three times as wide: some 64-hit groups have more window
    candidates than the scoring kernel's LDS list holds (or than their list segment has room
    for); the per-lane kernel scores those groups, and every stage still matches the oracle."""
    from paper_1910_12214_amd import tpcca

    w = synth.SECTOR_EVENT
    ev = synth.generate(w)
    geom = synth.geometry(w)
    prm0 = dict(synth.TRACKER_PARAMS, win_y=6.0, win_z=6.0)
    theta = theta_random(23)
    trip, feats = ctx.triplets(dev(ev.y), dev(ev.z), dev(ev.row), dev(ev.sector), geom, prm0)
    lg = ctx.mlp_infer(feats, dev(theta)).cpu().numpy()
    tau = float(np.quantile(lg, 0.5))
    out = ctx.track(dev(ev.y), dev(ev.z), dev(ev.row), dev(ev.sector), geom, synth.BZ, prm0, mlp=dev(theta),
                    tau_logit=tau)
    trk = tpcca.tracks_to_host(out)
    st = parity.gpu_stages(ctx, synth.N_ROWS)
    prm = dict(prm0, mlp_tau_logit=tau, mlp_flag_abs=1e-4)
    qtheta = omlp.quantize(theta)
    o = oracle.track(ev.y, ev.z, ev.row, ev.sector, geom, prm, synth.BZ, mlp=qtheta, n_threads=THREADS)
    o_fma = oracle.track(ev.y, ev.z, ev.row, ev.sector, geom, prm, synth.BZ, mlp=qtheta, n_threads=THREADS, fma=True)
    c = trk["counts"]
    groups = (ev.n + 63) // 64
    say(f"[mlp] wide windows: {len(trip)} pairs, {c[tpcca.CNT_NB_OVERFLOW]} of {groups} groups overflowed")
    assert 0 < c[tpcca.CNT_NB_OVERFLOW] <= groups
    assert c[tpcca.CNT_PAIRS] == len(trip)
    rep = parity.compare(o, st, trk, ev.n, synth.N_ROWS, leg=ev.leg, o_fma=o_fma,
                         row_of=ev.row, row_x=synth.row_x(), bz=synth.BZ)
    say(f"[mlp] wide windows parity: {rep.line()}")
    assert rep["tracks_compared"] > 50


def test_trained_scorer_gain_over_untrained(ctx):
    """What the trained network gains over the method without it.  On held-out one-sector events it
    removes about half of the candidate pairs before the automaton, keeps nearly every true triplet
    and tracks within 0.5% of the plain finder's efficiency; an untrained network of the same shape,
    with its threshold set to remove the same share of pairs, keeps far fewer true triplets."""
    import torch

    from paper_1910_12214_amd import scorer as sc
    from synth import metrics

    params, tau = sc.load()
    seeds = list(sc.TEST_SEEDS)[:6]
    theta_r = theta_random(21)
    logits_t, logits_r, labels = [], [], []
    for sd in seeds:
        w = synth.sector_event(sd)
        ev = synth.generate(w)
        trip, feats = ctx.triplets(dev(ev.y), dev(ev.z), dev(ev.row), dev(ev.sector), synth.geometry(w),
                                   synth.TRACKER_PARAMS)
        t = trip.cpu().numpy().astype(np.int64)
        labels.append(metrics.triplet_labels(ev.leg, ev.crossing, t[:, 0], t[:, 1], t[:, 2]))
        logits_t.append(ctx.mlp_infer(feats, dev(params)).cpu().numpy())
        logits_r.append(ctx.mlp_infer(feats, dev(theta_r)).cpu().numpy())
    torch.cuda.synchronize()
    lab = np.concatenate(labels).astype(bool)
    lt, lr = np.concatenate(logits_t), np.concatenate(logits_r)
    keep_t = lt >= tau
    share = keep_t.mean()
    tau_r = float(np.quantile(lr, 1.0 - share))
    keep_r = lr >= tau_r
    true_t, true_r = keep_t[lab].mean(), keep_r[lab].mean()
    plain = sc.evaluate(ctx, seeds, repeat=1)
    pruned = sc.evaluate(ctx, seeds, params, tau, repeat=1)
    untrained = sc.evaluate(ctx, seeds, theta_r, tau_r, repeat=1)
    say(f"[mlp] gain: triplets {lab.size} true {lab.mean():.3f}; trained keeps {share:.3f} of pairs and "
        f"{true_t:.4f} of true triplets, untrained (same share) {keep_r.mean():.3f} / {true_r:.4f}")
    say(f"[mlp] efficiency plain {plain['efficiency']:.4f} trained {pruned['efficiency']:.4f} "
        f"untrained {untrained['efficiency']:.4f}; fake {plain['fake_rate']:.4f} / {pruned['fake_rate']:.4f} / "
        f"{untrained['fake_rate']:.4f}; clusters/s plain {plain['clusters_per_s']:.3e} "
        f"trained {pruned['clusters_per_s']:.3e}")
    assert share < 0.6, "the trained scorer should remove at least 40% of the candidate pairs"
    # measured on these seeds: 0.980 of true triplets kept by the trained net, 0.389 by the untrained
    assert true_t > 0.95 and true_r < 0.6
    assert plain["efficiency"] - pruned["efficiency"] <= 0.005
    assert pruned["efficiency"] > untrained["efficiency"]


def test_full_event_pruned_sampled_sectors(ctx):
    """The full Pb-Pb event with the Pb-Pb scorer at its validated threshold, in the launch the
    benchmark times (candidate + scoring kernels, all 36 sectors); the oracle, with the same
    BF16 scorer in FP64, checks two whole sectors stage by stage."""
    from paper_1910_12214_amd import scorer as sc
    from paper_1910_12214_amd import tpcca
    from tests.test_gpu_timeframe import lift

    w = synth.PBPB_EVENT
    ev = synth.generate(w)
    geom = synth.geometry(w)
    theta, tau = sc.load(sc.PBPB_CKPT)
    out = ctx.track(dev(ev.y), dev(ev.z), dev(ev.row), dev(ev.sector), geom, synth.BZ, synth.TRACKER_PARAMS,
                    mlp=dev(theta), tau_logit=tau)
    trk = tpcca.tracks_to_host(out)
    st = parity.gpu_stages(ctx, synth.N_ROWS)
    sectors = [7, 25]
    sel = np.isin(ev.sector, sectors)
    ids = np.nonzero(sel)[0]
    prm = dict(synth.TRACKER_PARAMS, mlp_tau_logit=tau, mlp_flag_abs=1e-4)
    q = omlp.quantize(theta.astype(np.float64))
    args = (ev.y[sel], ev.z[sel], ev.row[sel], ev.sector[sel], geom, prm, synth.BZ)
    o = lift(oracle.track(*args, mlp=q, n_threads=THREADS), ids, ev.n)
    o_fma = lift(oracle.track(*args, mlp=q, n_threads=THREADS, fma=True), ids, ev.n)
    rep = parity.compare(o, st, trk, ev.n, synth.N_ROWS, sectors=sectors, sector_of=ev.sector, o_fma=o_fma,
                         row_of=ev.row, row_x=synth.row_x(), bz=synth.BZ)
    c = trk["counts"]
    say(f"[mlp] full event, tau {tau}, sectors {sectors}: {rep.line()} pairs={c[tpcca.CNT_PAIRS]} "
        f"kept={c[tpcca.CNT_PAIRS_KEPT]} overflow groups={c[tpcca.CNT_NB_OVERFLOW]}")
    assert rep["tracks_compared"] > 500


def test_interrupted_training_resumes_to_the_same_parameters(ctx, tmp_path):
    """Two epochs in one run, and one epoch, a saved state, then a second run that resumes it for the
    second epoch: identical parameters and losses (deterministic kernels, same batch order)."""
    from paper_1910_12214_amd import scorer

    rng = np.random.default_rng(17)
    N = 24576
    X = rng.normal(0, 1.0, (N, 12)).astype(np.float32)
    y = ((X @ rng.normal(0, 1, 12) + 0.3 * rng.normal(size=N)) > 0).astype(np.uint8)
    F, Y = dev(X), dev(y)
    p_full, h_full = scorer.train(ctx, F, Y, epochs=2, batch=2048, lr=2e-3, seed=9)
    state = str(tmp_path / "state.npz")
    p_one, h_one = scorer.train(ctx, F, Y, epochs=1, batch=2048, lr=2e-3, seed=9, state_path=state)
    assert scorer.load_state(state)["epoch"] == 1 and not np.array_equal(p_one, p_full)
    p_res, h_res = scorer.train(ctx, F, Y, epochs=2, batch=2048, lr=2e-3, seed=9, state_path=state)
    assert np.array_equal(p_res, p_full) and h_res == h_full
    assert scorer.load_state(state)["epoch"] == 2
    with pytest.raises(ValueError):  # a state saved for other settings is refused
        scorer.train(ctx, F, Y, epochs=3, batch=1024, lr=2e-3, seed=9, state_path=state)
