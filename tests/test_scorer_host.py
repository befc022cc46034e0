"""Host-side parts of the learned scorer driver (no GPU)."""
import math
import os

import numpy as np

from paper_1910_12214_amd import scorer
from synth import metrics


def test_init_is_seeded_he_uniform():
    from paper_1910_12214_amd import scorer

    a, b = scorer.init_params(5), scorer.init_params(5)
    assert np.array_equal(a, b) and not np.array_equal(a, scorer.init_params(6))
    assert np.abs(a[:768]).max() <= math.sqrt(6 / 12) and np.abs(a[832:4928]).max() <= math.sqrt(6 / 64)
    assert np.all(a[768:832] == 0) and np.all(a[4928:4992] == 0) and a[5056] == 0


def test_triplet_labels_need_consecutive_crossings_of_one_leg():
    leg = np.array([3, 3, 3, 3, 4, -1])
    crossing = np.array([0, 1, 2, 4, 3, -1])
    d, m, u = np.array([0, 2, 0, 0, 5]), np.array([1, 1, 1, 2, 1]), np.array([2, 0, 3, 4, 2])
    assert metrics.triplet_labels(leg, crossing, d, m, u).tolist() == [1, 1, 0, 0, 0]


def test_checkpoint_is_present_and_well_formed():
    from paper_1910_12214_amd import scorer

    p, tau = scorer.load()
    assert p.shape == (5057,) and p.dtype == np.float32 and np.isfinite(p).all() and np.isfinite(tau)


def test_pbpb_checkpoint_is_present_and_well_formed():
    from paper_1910_12214_amd import scorer

    p, tau = scorer.load(scorer.PBPB_CKPT)
    assert p.shape == (5057,) and p.dtype == np.float32 and np.isfinite(p).all() and np.isfinite(tau)
    assert "Pb-Pb" in scorer.trained_on(scorer.PBPB_CKPT)


def test_pp_checkpoint_is_present_and_well_formed():
    from paper_1910_12214_amd import scorer

    p, tau = scorer.load(scorer.PP_CKPT)
    assert p.shape == (5057,) and p.dtype == np.float32 and np.isfinite(p).all() and np.isfinite(tau)
    assert "pp-like" in scorer.trained_on(scorer.PP_CKPT)


def test_training_state_round_trip(tmp_path):
    """A saved training state reads back exactly, holds plain arrays only, and is replaced
    atomically (no temporary file left behind)."""
    rng = np.random.default_rng(3)
    st = dict(params=rng.normal(size=5057).astype(np.float32), m=rng.normal(size=5057).astype(np.float32),
              v=rng.random(5057).astype(np.float32), step=1234, epoch=3, loss_per_epoch=np.array([0.5, 0.4, 0.3]),
              seed=5, batch=4096, lr=1e-3, n_rows=5 * 10 ** 6)
    path = str(tmp_path / "state.npz")
    scorer.save_state(path, **st)
    scorer.save_state(path, **dict(st, epoch=4))
    assert not os.path.exists(path + ".tmp")
    got = scorer.load_state(path)
    for k in ("params", "m", "v"):
        assert np.array_equal(got[k], st[k]) and got[k].dtype == np.float32
    assert (got["step"], got["epoch"], got["seed"], got["batch"], got["n_rows"]) == (1234, 4, 5, 4096, 5 * 10 ** 6)
    assert got["lr"] == 1e-3 and got["loss_per_epoch"] == [0.5, 0.4, 0.3]
    with np.load(path) as z:  # readable without pickle
        assert set(z.files) == set(scorer.STATE_KEYS)
