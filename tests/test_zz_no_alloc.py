"""The allocation-free training entry point equals the allocating one.

tpc_mlp_train_noalloc runs the kernels of tpc_mlp_train on the library's fixed per-device
scratch.  Two calls in a row (the second with a smaller, ragged batch and fewer rows) must give
bit-identical parameters, Adam moments and losses to tpc_mlp_train on the same inputs: the same
kernels in the same order, with deterministic reductions.  Batches above the fixed scratch's
maximum are rejected before anything is enqueued.
"""
import numpy as np
import pytest

from paper_1910_12214_amd import scorer, tpcca

pytestmark = pytest.mark.gpu


def _inputs(n, seed):
    import torch

    rng = np.random.default_rng(seed)
    X = rng.normal(0.0, 1.0, (n, 12)).astype(np.float32)
    w = rng.normal(0.0, 1.0, 12)
    y = ((X @ w + 0.3 * rng.normal(size=n)) > 0).astype(np.uint8)
    d = torch.device("cuda", 0)
    return torch.from_numpy(X).to(d), torch.from_numpy(y).to(d), rng


def _run(ctx, feats, labels, order, theta0, batch, steps, noalloc):
    import torch

    mlp = theta0.clone()
    m = torch.zeros_like(theta0)
    v = torch.zeros_like(theta0)
    loss = ctx.mlp_train(feats, labels, order, mlp, m, v, batch=batch, n_steps=steps, lr=3e-3, noalloc=noalloc)
    torch.cuda.synchronize()
    return mlp.cpu(), m.cpu(), v.cpu(), loss[:steps].cpu()


def test_noalloc_training_equals_allocating_entry_point():
    import torch

    ctx = tpcca.Context(0)
    theta0 = torch.from_numpy(scorer.init_params(3).astype(np.float32)).to("cuda:0")
    # call 1: 60 000 rows, batch 16 384 (64 blocks), 3 steps; call 2: 9 000 rows, batch 1 000 (ragged), 2 steps
    cases = []
    for n, batch, steps, seed in ((60000, 16384, 3, 21), (9000, 1000, 2, 22)):
        feats, labels, rng = _inputs(n, seed)
        order = torch.from_numpy(
            np.concatenate([rng.permutation(n)[:batch] for _ in range(steps)]).astype(np.int32)).to("cuda:0")
        cases.append((feats, labels, order, batch, steps))
    print(f"[noalloc] cases {[(int(c[0].shape[0]), c[3], c[4]) for c in cases]}", flush=True)
    ref = [_run(ctx, f, lab, o, theta0, b, s, noalloc=False) for f, lab, o, b, s in cases]
    got = [_run(ctx, f, lab, o, theta0, b, s, noalloc=True) for f, lab, o, b, s in cases]  # two calls in a row
    for (f, _, _, b, s), r, g in zip(cases, ref, got):
        for name, a, e in zip(("params", "m", "v", "loss"), g, r):
            assert torch.equal(a, e), f"{name} differs (batch {b}, {s} steps)"
        assert bool(torch.isfinite(g[3]).all()) and not torch.equal(g[0], theta0.cpu())
    ctx.close()


def test_noalloc_rejects_batches_above_its_maximum():
    import torch

    ctx = tpcca.Context(0)
    n = tpcca.MLP_NOALLOC_MAX_BATCH + 1
    feats = torch.zeros((n, 12), dtype=torch.float32, device="cuda:0")
    labels = torch.zeros(n, dtype=torch.uint8, device="cuda:0")
    order = torch.arange(n, dtype=torch.int32, device="cuda:0")
    theta = torch.zeros(tpcca.MLP_N_PARAMS, dtype=torch.float32, device="cuda:0")
    with pytest.raises(tpcca.TpcError) as e:
        ctx.mlp_train(feats, labels, order, theta, theta.clone(), theta.clone(), batch=n, n_steps=1, noalloc=True)
    assert e.value.code == tpcca.TPC_ERR_ARG and "maximum" in str(e.value)
    ctx.close()
