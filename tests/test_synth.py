"""Input generator: determinism and the structure the workloads are meant to have."""
import dataclasses

import numpy as np

import synth


def test_thread_count_independent_and_seeded():
    w = synth.scaled(synth.PBPB_EVENT, 0.05)
    a = synth.generate(w, n_threads=1)
    b = synth.generate(w, n_threads=5)
    assert a.sha256() == b.sha256()
    c = synth.generate(dataclasses.replace(w, seed=w.seed + 1))
    assert c.sha256() != a.sha256()


def test_sector_event_shape():
    ev = synth.generate(synth.SECTOR_EVENT)
    assert set(np.unique(ev.sector)) == {0}
    rx = synth.row_x()
    assert ev.row.max() < synth.N_ROWS
    # noise is 5% of the signal (rounded)
    assert ev.n_noise == int(np.floor(0.05 * ev.n_signal + 0.5))
    sig = ev.particle >= 0
    # signal clusters lie inside the sector acceptance up to the smearing
    lim = rx[ev.row[sig]].astype(np.float64) * float(synth.tan_half())
    assert np.all(np.abs(ev.y[sig]) <= lim + 6 * 0.06)
    assert np.all((ev.z[sig] > -1.0) & (ev.z[sig] < 251.0))


def test_legs_are_row_monotonic_runs():
    w = dataclasses.replace(synth.scaled(synth.PBPB_EVENT, 0.02), sigma_y=0.0, sigma_z=0.0, eff=1.0, noise_frac=0.0)
    ev = synth.generate(w, want_exact=True)
    order = np.lexsort((ev.crossing, ev.particle))
    leg, row, sec, part = ev.leg[order], ev.row[order].astype(int), ev.sector[order], ev.particle[order]
    for lg in np.unique(leg)[:400]:
        sel = leg == lg
        assert np.unique(part[sel]).size == 1 and np.unique(sec[sel]).size == 1
        d = np.diff(row[sel])
        assert np.all(d > 0) or np.all(d < 0)


def test_time_frame_z_shift():
    w = synth.scaled(synth.PBPB_TIMEFRAME, 0.01)
    ev = synth.generate(w)
    assert ev.z.max() > 260.0  # collisions after t0 > 4 us are shifted beyond one drift length
    assert ev.z.max() <= w.z_max + 1.0
