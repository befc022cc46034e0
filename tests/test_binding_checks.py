"""The Python binding rejects arguments the C ABI cannot read safely, before any pointer reaches
the library: wrong dtype, non-contiguous views, unequal lengths, a short scorer vector, host
tensors, undersized outputs and out-of-range row indices.  Runs on the CPU (the checks come first)."""
import pytest
import torch

from paper_1910_12214_amd import tpcca


def clusters(n=10, **over):
    c = dict(y=torch.zeros(n), z=torch.zeros(n), row=torch.zeros(n, dtype=torch.uint8),
             sector=torch.zeros(n, dtype=torch.uint8))
    c.update(over)
    return c


def rejects(fn, *a, match=None, **kw):
    with pytest.raises(tpcca.TpcError, match=match) as e:
        fn(*a, **kw)
    assert e.value.code == tpcca.TPC_ERR_ARG


@pytest.mark.parametrize("over,match", [
    (dict(y=torch.zeros(10, dtype=torch.float64)), "y: dtype"),
    (dict(z=torch.zeros(10, dtype=torch.float16)), "z: dtype"),
    (dict(row=torch.zeros(10, dtype=torch.int64)), "row: dtype"),
    (dict(sector=torch.zeros(10, dtype=torch.int32)), "sector: dtype"),
    (dict(z=torch.zeros(9)), "z: 9 elements"),
    (dict(row=torch.zeros(20, dtype=torch.uint8)[::2]), "row: must be contiguous"),
    (dict(y=torch.zeros(20)[::2]), "y: must be contiguous"),
    ({}, "must be on a GPU"),  # every check passes but the tensors are host memory
])
def test_cluster_arrays_are_checked(over, match):
    c = clusters(**over)
    rejects(tpcca.check_clusters, c["y"], c["z"], c["row"], c["sector"], match=match)


def test_two_dimensional_clusters_are_rejected():
    rejects(tpcca.check_clusters, torch.zeros(2, 5), torch.zeros(2, 5), torch.zeros(2, 5, dtype=torch.uint8),
            torch.zeros(2, 5, dtype=torch.uint8), match="1-D")


@pytest.mark.parametrize("mlp,match", [(torch.zeros(5056), "5056 elements"), (torch.zeros(5057, dtype=torch.float64),
                                                                               "dtype"),
                                       (torch.zeros(5057), "must be on a GPU")])
def test_scorer_vector_is_checked(mlp, match):
    rejects(tpcca.check_mlp, mlp, match=match)


def test_track_outputs_are_checked():
    ct, ch = 8, 100
    i32, f32 = dict(dtype=torch.int32), dict(dtype=torch.float32)
    good = dict(counts=torch.zeros(16, **i32), hit_offset=torch.zeros(ct, **i32), n_hits=torch.zeros(ct, **i32),
                hit_ids=torch.zeros(ch, **i32), start_id=torch.zeros(ct, **i32), sector=torch.zeros(ct, **i32),
                row_ref=torch.zeros(ct, **i32), x_ref=torch.zeros(ct, **f32), state=torch.zeros(ct, 5, **f32),
                cov=torch.zeros(ct, 15, **f32), chi2=torch.zeros(ct, **f32), ndf=torch.zeros(ct, **i32),
                cap_tracks=ct, cap_hits=ch)
    rejects(tpcca.check_tracks, good, match="must be on a GPU")  # complete, but host memory
    for k, bad, match in (("cov", torch.zeros(ct, 14, **f32), "cov: 112 elements"),
                          ("hit_ids", torch.zeros(ch - 1, **i32), "hit_ids: 99"),
                          ("state", torch.zeros(ct, 5, dtype=torch.float64), "state: dtype"),
                          ("counts", torch.zeros(8, **i32), "counts: 8"),
                          ("n_hits", torch.zeros(2 * ct, **i32)[::2], "contiguous")):
        rejects(tpcca.check_tracks, dict(good, **{k: bad}), match=match)
    rejects(tpcca.check_tracks, dict(good, cap_tracks=-1), match="capacities")


def test_row_indices_are_checked():
    rejects(tpcca.check_rows, torch.tensor([0, 5, 10], dtype=torch.int32), 10, "idx", match=r"\[0, 10\)")
    rejects(tpcca.check_rows, torch.tensor([-1], dtype=torch.int32), 10, "idx")
    tpcca.check_rows(torch.tensor([0, 9], dtype=torch.int32), 10, "idx")


def test_merge_outputs_are_checked():
    ct = 8
    f64, i32 = dict(dtype=torch.float64), dict(dtype=torch.int32)
    good = dict(cap_tracks=ct, label=torch.zeros(ct, **i32), n_members=torch.zeros(ct, **i32),
                helix=torch.zeros(ct, 5, **f64), helix_cov=torch.zeros(ct, 15, **f64),
                theta=torch.zeros(ct, 5, **f64), theta_cov=torch.zeros(ct, 15, **f64), chi2=torch.zeros(ct, **f64),
                ndf=torch.zeros(ct, **i32), counts=torch.zeros(len(tpcca.MG_COUNTS), dtype=torch.int64))
    rejects(tpcca.check_merged, good, ct, match="must be on a GPU")  # complete, but host memory
    rejects(tpcca.check_merged, good, ct + 1, match="below the track set's")
    for k, bad, match in (("helix", torch.zeros(ct, 4, **f64), "helix: 32 elements"),
                          ("theta_cov", torch.zeros(ct, 15, dtype=torch.float32), "theta_cov: dtype"),
                          ("label", torch.zeros(ct, dtype=torch.int64), "label: dtype"),
                          ("counts", torch.zeros(3, dtype=torch.int64), "counts: 3 elements"),
                          ("chi2", torch.zeros(2 * ct, **f64)[::2], "chi2: must be contiguous")):
        rejects(tpcca.check_merged, dict(good, **{k: bad}), ct, match=match)
