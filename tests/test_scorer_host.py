"""Host-side parts of the learned scorer driver (no GPU)."""
import math

import numpy as np

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
