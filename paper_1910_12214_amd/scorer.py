"""Training, threshold choice and evaluation of the learned triplet scorer.

The scorer (MLP 12-64-64-1, BF16 weights, FP32 accumulation) prunes candidate neighbour pairs
before the cellular automaton chooses links.  It is trained on the GPU by the library's own
forward/backward kernels (``tpc_mlp_train``) on truth-labelled window triplets of synthetic
events; the plain finder is both the fallback and the judge of the efficiency the pruning costs.

    python -m paper_1910_12214_amd.scorer train --set sector     # -> scorer_sector200.npz
    python -m paper_1910_12214_amd.scorer train --set pbpb       # -> scorer_pbpb.npz
    python -m paper_1910_12214_amd.scorer train --set pp         # -> scorer_pp.npz

Training sets (every window candidate triplet of the events, label 1 iff the three clusters are
consecutive crossings of one leg, uniformly subsampled to 10^7 if there are more):
  sector: one-sector 200-helix events, training seeds 1..200, threshold seeds 201..210, held-out
          test seeds 1001..1020;
  pbpb:   central Pb-Pb-like full-TPC events (the benchmark event's generator), training seeds
          0x10001..0x10008, threshold seeds 0x20001..0x20002, test seeds 0x30001..0x30002 — all
          disjoint from the benchmark event's seed and its validation seed;
  pp:     pp-like time frames of 570 collisions at 1 MHz (a twentieth of the benchmark frame, same
          rate, multiplicity and noise), training seeds 0x40001..0x40008, threshold seeds
          0x50001..0x50002, test seeds 0x60001..0x60002.
He-uniform initialisation from a seeded generator, Adam (lr 1e-3, betas 0.9/0.999) for 5 epochs
of batch 4096; the threshold tau (on the logit) is the largest candidate whose efficiency on the
threshold seeds is within 0.5% of the plain finder's.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(_HERE)
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

DEFAULT_CKPT = os.path.join(_HERE, "scorer_sector200.npz")
PBPB_CKPT = os.path.join(_HERE, "scorer_pbpb.npz")
TRAIN_SEEDS = range(1, 201)
VAL_SEEDS = range(201, 211)
TEST_SEEDS = range(1001, 1021)


def _sector_events(seeds):
    import synth

    return [synth.sector_event(s) for s in seeds]


def _pbpb_events(seeds):
    import dataclasses

    import synth

    return [dataclasses.replace(synth.PBPB_EVENT, name=f"pbpb_event_5000_s{s:#x}", seed=s) for s in seeds]


PP_CKPT = os.path.join(_HERE, "scorer_pp.npz")


def _pp_events(seeds):
    import dataclasses

    import synth

    base = synth.scaled(synth.PP_TIMEFRAME, 0.05)  # 570 pp collisions over 0.57 ms
    return [dataclasses.replace(base, name=f"pp_timeframe_570_s{s:#x}", seed=s) for s in seeds]


# name -> (training, threshold, test workloads, checkpoint, description)
SETS = {
    "sector": (lambda: _sector_events(TRAIN_SEEDS), lambda: _sector_events(VAL_SEEDS),
               lambda: _sector_events(TEST_SEEDS), DEFAULT_CKPT, "one-sector 200-helix events, seeds 1-200"),
    "pbpb": (lambda: _pbpb_events(range(0x10001, 0x10009)), lambda: _pbpb_events(range(0x20001, 0x20003)),
             lambda: _pbpb_events(range(0x30001, 0x30003)), PBPB_CKPT,
             "central Pb-Pb-like full-TPC events, seeds 0x10001-0x10008"),
    "pp": (lambda: _pp_events(range(0x40001, 0x40009)), lambda: _pp_events(range(0x50001, 0x50003)),
           lambda: _pp_events(range(0x60001, 0x60003)), PP_CKPT,
           "pp-like time frames of 570 collisions at 1 MHz, seeds 0x40001-0x40008"),
}
MAX_TRIPLETS = 10_000_000
N_PARAMS = 5057


def _dev(a):
    import torch

    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


def init_params(seed: int) -> np.ndarray:
    """He-uniform weights (bounds sqrt(6 / fan_in)), zero biases; layout W1, b1, W2, b2, w3, b3."""
    import synth

    u = synth.uniform01(seed, 768 + 4096 + 64)
    p = np.zeros(N_PARAMS, dtype=np.float32)
    p[0:768] = (2 * u[:768] - 1) * math.sqrt(6 / 12)
    p[832:4928] = (2 * u[768:4864] - 1) * math.sqrt(6 / 64)
    p[4992:5056] = (2 * u[4864:] - 1) * math.sqrt(6 / 64)
    return p


def event_tensors(ev):
    return _dev(ev.y), _dev(ev.z), _dev(ev.row), _dev(ev.sector)


def training_set(ctx, workloads=None, max_triplets=MAX_TRIPLETS, subsample_seed=77):
    """Features and labels of every window triplet of the given events (GPU tensors)."""
    import torch

    import synth
    from synth import metrics

    feats, labels = [], []
    for w in workloads if workloads is not None else _sector_events(TRAIN_SEEDS):
        ev = synth.generate(w)
        trip, f = ctx.triplets(*event_tensors(ev), synth.geometry(w), synth.TRACKER_PARAMS)
        t = trip.cpu().numpy().astype(np.int64)
        lab = metrics.triplet_labels(ev.leg, ev.crossing, t[:, 0], t[:, 1], t[:, 2])
        feats.append(f)
        labels.append(_dev(lab))
    F = torch.cat(feats)
    Y = torch.cat(labels)
    n = F.shape[0]
    if n > max_triplets:
        keep = np.sort(synth.permutation(subsample_seed, n)[:max_triplets])
        kt = _dev(keep.astype(np.int64))
        F, Y = F[kt].contiguous(), Y[kt].contiguous()
    return F, Y


STATE_KEYS = ("params", "m", "v", "step", "epoch", "loss_per_epoch", "seed", "batch", "lr", "n_rows")


def save_state(path: str, **st) -> None:
    """Write a training state (master parameters, Adam moments, step and epoch counters, the
    settings that fix the batch order) atomically: a crash leaves the previous state intact."""
    tmp = path + ".tmp"
    with open(tmp, "wb") as f:
        np.savez(f, **{k: np.asarray(st[k]) for k in STATE_KEYS})
    os.replace(tmp, path)


def load_state(path: str) -> dict:
    ck = np.load(path)  # plain arrays only (no pickled objects)
    st = {k: ck[k] for k in STATE_KEYS}
    for k in ("step", "epoch", "seed", "batch", "n_rows"):
        st[k] = int(st[k])
    st["lr"] = float(st["lr"])
    st["loss_per_epoch"] = [float(x) for x in np.atleast_1d(st["loss_per_epoch"])]
    return st


def train(ctx, F, Y, epochs=5, batch=4096, lr=1e-3, seed=5, log=None, state_path=None):
    """Adam training on the GPU; returns (params as numpy float32, per-epoch mean loss).

    With ``state_path`` the state is saved after every epoch, and a state already there is resumed
    (same rows, batch, learning rate and seed required): the epochs it holds are skipped and the
    run continues with identical batches, so an interrupted run ends with the same parameters as
    an uninterrupted one."""
    import torch

    import synth

    n = int(F.shape[0])
    params = _dev(init_params(seed))
    m = torch.zeros(N_PARAMS, device="cuda:0")
    v = torch.zeros(N_PARAMS, device="cuda:0")
    steps = n // batch
    hist = []
    step0 = 0
    ep0 = 0
    if state_path and os.path.exists(state_path):
        st = load_state(state_path)
        if (st["n_rows"], st["batch"], st["seed"]) != (n, batch, seed) or st["lr"] != float(lr):
            raise ValueError(f"{state_path}: saved for rows/batch/seed/lr {st['n_rows']}/{st['batch']}/"
                             f"{st['seed']}/{st['lr']}, not {n}/{batch}/{seed}/{lr}")
        params = _dev(st["params"].astype(np.float32))
        m = _dev(st["m"].astype(np.float32))
        v = _dev(st["v"].astype(np.float32))
        step0, ep0, hist = st["step"], st["epoch"], list(st["loss_per_epoch"])
        if log:
            log(f"resumed {state_path} after epoch {ep0} (Adam step {step0})")
    for ep in range(ep0, epochs):
        order = synth.permutation(seed * 1000 + ep, n)[: steps * batch].astype(np.int32)
        loss = ctx.mlp_train(F, Y, _dev(order), params, m, v, batch=batch, n_steps=steps, step0=step0, lr=lr)
        step0 += steps
        hist.append(float(loss.mean().item()))
        if log:
            log(f"epoch {ep}: mean loss {hist[-1]:.5f} ({steps} steps)")
        if state_path:
            save_state(state_path, params=params.cpu().numpy(), m=m.cpu().numpy(), v=v.cpu().numpy(),
                       step=step0, epoch=ep + 1, loss_per_epoch=np.array(hist), seed=seed, batch=batch, lr=lr,
                       n_rows=n)
    return params.cpu().numpy(), hist


def evaluate(ctx, workloads, params=None, tau=0.0, repeat=3):
    """Aggregate efficiency / fake / clone rates and tracking time over events (workloads, or
    one-sector event seeds)."""
    import torch

    import synth
    from paper_1910_12214_amd import tpcca
    from synth import metrics

    tot = dict(n_findable=0, n_matched_findable=0, n_tracks=0, n_good=0, clones=0, clusters=0, ms=0.0,
               tracklets=0, pairs=0, kept=0, links=0)
    mlp = _dev(params) if params is not None else None
    for w in workloads:
        if isinstance(w, int):
            w = synth.sector_event(w)
        ev = synth.generate(w)
        ten = event_tensors(ev)
        geom = synth.geometry(w)
        out = ctx.track(*ten, geom, synth.BZ, synth.TRACKER_PARAMS, mlp=mlp, tau_logit=tau)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(repeat):
            ctx.track(*ten, geom, synth.BZ, synth.TRACKER_PARAMS, mlp=mlp, tau_logit=tau, out=out, sync_check=False)
        torch.cuda.synchronize()
        tot["ms"] += (time.perf_counter() - t0) * 1e3 / repeat
        h = tpcca.tracks_to_host(out)
        off = np.concatenate([[0], np.cumsum(h["n_hits"])])
        r = metrics.match(ev.leg, off, h["hit_ids"])
        for k in ("n_findable", "n_matched_findable", "n_tracks", "n_good"):
            tot[k] += r[k]
        tot["clones"] += int(round(r["clone_rate"] * r["n_good"]))
        tot["clusters"] += ev.n
        c = h["counts"]
        tot["tracklets"] += int(c[tpcca.CNT_TRACKLETS])
        tot["pairs"] += int(c[tpcca.CNT_PAIRS])
        tot["kept"] += int(c[tpcca.CNT_PAIRS_KEPT]) if mlp is not None else int(c[tpcca.CNT_PAIRS])
        tot["links"] += int(c[tpcca.CNT_LINKS_RAW])
    tot["efficiency"] = tot["n_matched_findable"] / max(1, tot["n_findable"])
    tot["fake_rate"] = (tot["n_tracks"] - tot["n_good"]) / max(1, tot["n_tracks"])
    tot["clone_rate"] = tot["clones"] / max(1, tot["n_good"])
    tot["clusters_per_s"] = tot["clusters"] / (tot["ms"] * 1e-3)
    return tot


def choose_tau(ctx, params, workloads=None, max_loss=0.005, log=None):
    """Largest logit threshold whose validation efficiency is within max_loss of the plain finder's."""
    workloads = workloads if workloads is not None else _sector_events(VAL_SEEDS)
    plain = evaluate(ctx, workloads, repeat=1)
    best = None
    for tau in np.arange(-8.0, 4.01, 0.5):
        r = evaluate(ctx, workloads, params, float(tau), repeat=1)
        ok = plain["efficiency"] - r["efficiency"] <= max_loss
        if log:
            log(f"tau {tau:+.1f}: eff {r['efficiency']:.4f} (plain {plain['efficiency']:.4f}) "
                f"kept {r['kept'] / max(1, r['pairs']):.3f} tracklets {r['tracklets']} ({plain['tracklets']}) {'ok' if ok else ''}")
        if ok:
            best = float(tau)
    return best if best is not None else -1e30, plain


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    t = sub.add_parser("train")
    t.add_argument("--set", choices=sorted(SETS), default="sector", help="training/threshold/test events")
    t.add_argument("--out", default=None, help="checkpoint (default: the set's file in the package)")
    t.add_argument("--epochs", type=int, default=5)
    t.add_argument("--report", default=None, help="write the training/validation/test summary as JSON")
    t.add_argument("--state", default=None,
                   help="training state file: saved after every epoch, resumed if present")
    e = sub.add_parser("eval")
    e.add_argument("--ckpt", default=DEFAULT_CKPT)
    args = ap.parse_args(argv)

    from paper_1910_12214_amd import tpcca

    def log(*a):
        print("[scorer]", *a, flush=True)

    ctx = tpcca.Context(0)
    if args.cmd == "train":
        tr, va, te, ckpt, desc = SETS[args.set]
        out_path = args.out or ckpt
        t0 = time.perf_counter()
        train_w = tr()
        F, Y = training_set(ctx, train_w)
        log(f"training set: {F.shape[0]} triplets from {len(train_w)} events, positives "
            f"{float(Y.float().mean()):.3f} ({time.perf_counter() - t0:.1f} s)")
        t0 = time.perf_counter()
        params, hist = train(ctx, F, Y, epochs=args.epochs, log=log, state_path=args.state)
        log(f"trained in {time.perf_counter() - t0:.2f} s")
        tau, plain_val = choose_tau(ctx, params, va(), log=log)
        log(f"tau = {tau}")
        test_plain = evaluate(ctx, te())
        test_mlp = evaluate(ctx, te(), params, tau)
        rep = {"set": args.set, "trained_on": desc, "n_train_triplets": int(F.shape[0]), "loss_per_epoch": hist,
               "tau_logit": tau,
               "val_plain_efficiency": plain_val["efficiency"],
               "test_plain": {k: v for k, v in test_plain.items()}, "test_pruned": {k: v for k, v in test_mlp.items()}}
        log("test plain ", json.dumps({k: round(v, 5) if isinstance(v, float) else v for k, v in test_plain.items()}))
        log("test pruned", json.dumps({k: round(v, 5) if isinstance(v, float) else v for k, v in test_mlp.items()}))
        np.savez(out_path, params=params, tau_logit=np.float64(tau), loss_per_epoch=np.array(hist),
                 n_train_triplets=np.int64(F.shape[0]), trained_on=np.array(desc))
        if args.report:
            json.dump(rep, open(args.report, "w"), indent=1)
        log("wrote", out_path)
    else:
        ck = np.load(args.ckpt)
        test_plain = evaluate(ctx, TEST_SEEDS)
        test_mlp = evaluate(ctx, TEST_SEEDS, ck["params"], float(ck["tau_logit"]))
        log("plain ", test_plain)
        log("pruned", test_mlp)
    ctx.close()


def load(path: str = DEFAULT_CKPT):
    """(params float32[5057], tau_logit) of a saved scorer."""
    ck = np.load(path)
    return ck["params"].astype(np.float32), float(ck["tau_logit"])


def trained_on(path: str = DEFAULT_CKPT) -> str:
    """Description of the events a saved scorer was trained on."""
    ck = np.load(path)
    return str(ck["trained_on"]) if "trained_on" in ck.files else SETS["sector"][4]


if __name__ == "__main__":
    main()
