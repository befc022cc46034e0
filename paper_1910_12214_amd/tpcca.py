"""Python binding of ``libtpcca.so`` (argument marshalling only).

PyTorch provides device memory and the HIP stream; every step of the track finding runs in
the library's HIP kernels.  Importing this module on a machine without the built library
raises: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libtpcca.so")

TPC_OK, TPC_ERR_ARG, TPC_ERR_CAPACITY, TPC_ERR_HIP, TPC_ERR_STATE = 0, -1, -2, -3, -4
(CNT_TRACKS, CNT_TRACK_HITS, CNT_TRACKLETS, CNT_VALID_TRACKLETS, CNT_FIT_FAILURES, CNT_LINKS_RAW,
 CNT_LINKS_CLEAN, CNT_VALID_CLUSTERS, CNT_PAIRS, CNT_PAIRS_KEPT, CNT_NB_OVERFLOW) = range(11)
N_COUNTS = 16
(STAGE_HITS, STAGE_ROW_OFF, STAGE_BIN_BASE, STAGE_BIN_OFF, STAGE_UP, STAGE_DN, STAGE_UP_CLEAN, STAGE_DN_CLEAN,
 STAGE_STARTS, STAGE_TL_NHITS, STAGE_TL_HITS, STAGE_TL_STATE, STAGE_TL_COV, STAGE_TL_FLAGS, STAGE_HIT_KEY,
 STAGE_PAIR_LOGIT) = range(16)
MLP_N_PARAMS = 5057

_vp = ctypes.c_void_p


class Clusters(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("y", _vp), ("z", _vp), ("row", _vp), ("sector", _vp)]


class Geometry(ctypes.Structure):
    _fields_ = [("n_rows", ctypes.c_int32), ("row_x", ctypes.POINTER(ctypes.c_float)), ("tan_half", ctypes.c_float),
                ("n_sectors", ctypes.c_int32), ("z_min", ctypes.c_float), ("z_max", ctypes.c_float)]


class Params(ctypes.Structure):
    _fields_ = [("win_y", ctypes.c_double), ("win_z", ctypes.c_double), ("nb_chi2_max", ctypes.c_double),
                ("fol_chi2_max", ctypes.c_double), ("sigma_y", ctypes.c_double), ("sigma_z", ctypes.c_double),
                ("s_max", ctypes.c_double), ("edge_margin", ctypes.c_double), ("l_min_chain", ctypes.c_int32),
                ("n_miss_max", ctypes.c_int32), ("n_min_tracklet", ctypes.c_int32), ("n_min_track", ctypes.c_int32),
                ("c0_sinphi", ctypes.c_double), ("c0_dzds", ctypes.c_double), ("c0_qpt", ctypes.c_double),
                ("bin_y", ctypes.c_float), ("bin_z", ctypes.c_float), ("mlp", _vp), ("mlp_tau_logit", ctypes.c_double)]


class Tracks(ctypes.Structure):
    _fields_ = [("cap_tracks", ctypes.c_int32), ("cap_hits", ctypes.c_int32), ("counts", _vp), ("hit_offset", _vp),
                ("n_hits", _vp), ("hit_ids", _vp), ("start_id", _vp), ("sector", _vp), ("row_ref", _vp),
                ("x_ref", _vp), ("state", _vp), ("cov", _vp), ("chi2", _vp), ("ndf", _vp)]


class FlagParams(ctypes.Structure):
    _fields_ = [("tube_cm", ctypes.c_double), ("pt_min", ctypes.c_double), ("phi_max_deg", ctypes.c_double)]


FLAG_ATTACHED, FLAG_ADJACENT, FLAG_PROTECTED, FLAG_REMOVE_A, FLAG_REMOVE_B = 1, 2, 4, 8, 16

# cluster compression (include/tpc_ca.h)
CSTREAMS = ("a_drow", "a_ry", "a_rz", "u_n", "u_dz", "u_dy", "q", "sy", "sz")
N_CSTREAMS, CS_ALPHABET, CS_BLOCK, CS_PROB_BITS = 9, 4096, 4096, 14
CSC_N, CST_N = 4, 4  # per-stream counts (symbols, escapes, bytes, blocks); totals
CST_ATTACHED, CST_UNATTACHED, CST_SKIPPED, CST_PRED_FAIL = 0, 1, 2, 3


class CompressParams(ctypes.Structure):
    _fields_ = [("q_y", ctypes.c_double), ("q_z", ctypes.c_double), ("n_charge", ctypes.c_int32),
                ("n_width", ctypes.c_int32)]


class ClusterProps(ctypes.Structure):
    _fields_ = [("qtot", _vp), ("sigma_y", _vp), ("sigma_z", _vp)]


class Compressed(ctypes.Structure):
    _fields_ = [("cap_sym", ctypes.c_int64), ("cap_esc", ctypes.c_int64), ("cap_bytes", ctypes.c_int64),
                ("counts", _vp), ("sym", _vp), ("esc", _vp), ("freq", _vp), ("block_bytes", _vp), ("bytes", _vp),
                ("order", _vp), ("track_len", _vp)]


class MergeParams(ctypes.Structure):
    _fields_ = [("rho_max", ctypes.c_double), ("centre_window", ctypes.c_double), ("chi2_max", ctypes.c_double),
                ("phase_sigmas", ctypes.c_double), ("phase_floor", ctypes.c_double), ("max_turns", ctypes.c_int32),
                ("sectors_per_side", ctypes.c_int32), ("max_iter", ctypes.c_int32), ("pair_queue", ctypes.c_int32)]


class Merged(ctypes.Structure):
    _fields_ = [("cap_tracks", ctypes.c_int32), ("label", _vp), ("n_members", _vp), ("helix", _vp),
                ("helix_cov", _vp), ("theta", _vp), ("theta_cov", _vp), ("chi2", _vp), ("ndf", _vp),
                ("counts", _vp)]


MG_COUNTS = ("components", "merged", "pairs_tested", "pairs_passed", "max_cell", "big_cells", "refit_failed")


class Tuning(ctypes.Structure):
    _fields_ = [("bin_y", ctypes.c_float), ("bin_z", ctypes.c_float), ("tracklet_chunk", ctypes.c_int32),
                ("blocks_per_cu", ctypes.c_int32), ("waves_per_simd", ctypes.c_int32), ("best_ms", ctypes.c_float),
                ("n_candidates", ctypes.c_int32)]


class TrainCfg(ctypes.Structure):
    _fields_ = [("batch", ctypes.c_int32), ("n_steps", ctypes.c_int32), ("step0", ctypes.c_int32),
                ("lr", ctypes.c_float), ("beta1", ctypes.c_float), ("beta2", ctypes.c_float), ("eps", ctypes.c_float)]


EXPORTS = ("tpc_ctx_create", "tpc_ctx_destroy", "tpc_last_error", "tpc_params_default", "tpc_track_sectors",
           "tpc_track_timeframe", "tpc_timeframe_tuning", "tpc_timeframe_set_tuning", "tpc_stage_size",
           "tpc_stage_copy", "tpc_mlp_infer", "tpc_triplets", "tpc_mlp_grad", "tpc_mlp_train",
           "tpc_profile_enable", "tpc_profile_read", "tpc_cluster_flags", "tpc_flag_params_default",
           "tpc_mlp_train_noalloc", "tpc_timeframe_tune_cache", "tpc_compress", "tpc_decompress",
           "tpc_compress_params_default", "tpc_compress_sizes", "tpc_merge", "tpc_merge_params_default")
MLP_NOALLOC_MAX_BATCH = 65536
N_PROF = 5
PROF_STAGES = ("grid", "neighbours", "clean_starts", "tracklets", "selection")

_lib = None


def load():
    """Load the HIP library (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_1910_12214_amd/build.py "
                           "(the track finder has no CPU fallback)")
    # Import torch first.  torch bundles its own HIP runtime with the same soname
    # (libamdhip64.so.7) as the system one this library links; whichever loads first serves
    # the whole process.  Loading torch's first gives one runtime, so torch's allocations
    # and streams are native to the library's calls.
    import torch  # noqa: F401

    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.POINTER
    lib.tpc_ctx_create.argtypes = [P(_vp), ctypes.c_int]
    lib.tpc_ctx_create.restype = ctypes.c_int
    lib.tpc_ctx_destroy.argtypes = [_vp]
    lib.tpc_ctx_destroy.restype = None
    lib.tpc_last_error.argtypes = [_vp]
    lib.tpc_last_error.restype = ctypes.c_char_p
    lib.tpc_params_default.argtypes = [P(Params)]
    lib.tpc_params_default.restype = None
    for f in ("tpc_track_sectors", "tpc_track_timeframe"):
        getattr(lib, f).argtypes = [_vp, P(Clusters), P(Geometry), ctypes.c_double, P(Params), P(Tracks), _vp,
                                    ctypes.c_int]
        getattr(lib, f).restype = ctypes.c_int
    lib.tpc_cluster_flags.argtypes = [_vp, P(Clusters), P(Geometry), ctypes.c_double, P(Params), P(FlagParams),
                                      P(Tracks), _vp, _vp]
    lib.tpc_cluster_flags.restype = ctypes.c_int
    lib.tpc_flag_params_default.argtypes = [P(FlagParams)]
    lib.tpc_flag_params_default.restype = None
    lib.tpc_timeframe_tuning.argtypes = [_vp, P(Tuning)]
    lib.tpc_timeframe_tuning.restype = ctypes.c_int
    lib.tpc_timeframe_set_tuning.argtypes = [_vp, P(Tuning)]
    lib.tpc_timeframe_set_tuning.restype = ctypes.c_int
    lib.tpc_timeframe_tune_cache.argtypes = [_vp, ctypes.c_char_p]
    lib.tpc_timeframe_tune_cache.restype = ctypes.c_int
    lib.tpc_stage_size.argtypes = [_vp, ctypes.c_int, P(ctypes.c_size_t)]
    lib.tpc_stage_size.restype = ctypes.c_int
    lib.tpc_stage_copy.argtypes = [_vp, ctypes.c_int, _vp, ctypes.c_size_t]
    lib.tpc_stage_copy.restype = ctypes.c_int
    lib.tpc_mlp_infer.argtypes = [_vp, _vp, ctypes.c_int64, _vp, _vp, _vp]
    lib.tpc_mlp_infer.restype = ctypes.c_int
    lib.tpc_triplets.argtypes = [_vp, P(Clusters), P(Geometry), P(Params), _vp, _vp, ctypes.c_int64,
                                 P(ctypes.c_int64), _vp]
    lib.tpc_triplets.restype = ctypes.c_int
    lib.tpc_mlp_grad.argtypes = [_vp, _vp, _vp, _vp, ctypes.c_int32, _vp, _vp, _vp, _vp]
    lib.tpc_mlp_grad.restype = ctypes.c_int
    lib.tpc_mlp_train.argtypes = [_vp, _vp, _vp, _vp, P(TrainCfg), _vp, _vp, _vp, _vp, _vp]
    lib.tpc_mlp_train.restype = ctypes.c_int
    lib.tpc_mlp_train_noalloc.argtypes = [_vp, _vp, _vp, _vp, P(TrainCfg), _vp, _vp, _vp, _vp, _vp]
    lib.tpc_mlp_train_noalloc.restype = ctypes.c_int
    lib.tpc_compress_params_default.argtypes = [P(CompressParams)]
    lib.tpc_compress_params_default.restype = None
    lib.tpc_compress.argtypes = [_vp, P(Clusters), P(ClusterProps), P(Geometry), ctypes.c_double, P(Params),
                                 P(CompressParams), P(Tracks), P(Compressed), _vp, ctypes.c_int]
    lib.tpc_compress.restype = ctypes.c_int
    lib.tpc_decompress.argtypes = [_vp, P(Compressed), P(Geometry), ctypes.c_double, P(Params), P(CompressParams),
                                   P(Tracks), _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp]
    lib.tpc_decompress.restype = ctypes.c_int
    lib.tpc_compress_sizes.argtypes = [_vp, P(Compressed), ctypes.POINTER(ctypes.c_double)]
    lib.tpc_compress_sizes.restype = ctypes.c_int
    lib.tpc_merge_params_default.argtypes = [P(MergeParams)]
    lib.tpc_merge_params_default.restype = None
    lib.tpc_merge.argtypes = [_vp, P(Clusters), P(Geometry), ctypes.c_double, P(Params), P(MergeParams), P(Tracks),
                              P(Merged), _vp]
    lib.tpc_merge.restype = ctypes.c_int
    lib.tpc_profile_enable.argtypes = [_vp, ctypes.c_int]
    lib.tpc_profile_enable.restype = ctypes.c_int
    lib.tpc_profile_read.argtypes = [_vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int)]
    lib.tpc_profile_read.restype = ctypes.c_int
    _lib = lib
    return lib


class TpcError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"tpc error {code}: {msg}")
        self.code = code


def default_params() -> dict:
    p = Params()
    load().tpc_params_default(ctypes.byref(p))
    return {f: getattr(p, f) for f, _ in Params._fields_ if f not in ("mlp",)}


def _ptr(t) -> int:
    return 0 if t is None else int(t.data_ptr())


def need(t, name: str, dtype, numel: int | None = None, min_numel: int | None = None, cols: int | None = None,
         on_gpu: bool = True):
    """Reject a tensor the library cannot read as a plain device array of this type and size:
    dtype, contiguity, size (exact, minimum, or rows of `cols` values), then that it lives on a GPU.
    Raised before any pointer reaches the C ABI, so a wrong argument never becomes a bad access."""
    import torch

    if not isinstance(t, torch.Tensor):
        raise TpcError(TPC_ERR_ARG, f"{name}: expected a torch tensor, got {type(t).__name__}")
    if t.dtype != dtype:
        raise TpcError(TPC_ERR_ARG, f"{name}: dtype {t.dtype}, expected {dtype}")
    if not t.is_contiguous():
        raise TpcError(TPC_ERR_ARG, f"{name}: must be contiguous")
    if cols is not None and (t.dim() != 2 or t.shape[1] != cols):
        raise TpcError(TPC_ERR_ARG, f"{name}: shape {tuple(t.shape)}, expected (n, {cols})")
    if numel is not None and t.numel() != numel:
        raise TpcError(TPC_ERR_ARG, f"{name}: {t.numel()} elements, expected {numel}")
    if min_numel is not None and t.numel() < min_numel:
        raise TpcError(TPC_ERR_ARG, f"{name}: {t.numel()} elements, need at least {min_numel}")
    if on_gpu:
        need_gpu(t, name)
    return t


def need_gpu(t, name: str):
    if not t.is_cuda:
        raise TpcError(TPC_ERR_ARG, f"{name}: must be on a GPU (device memory), got {t.device}")


def check_clusters(y, z, row, sector) -> int:
    """Cluster arrays: float32 y, z and uint8 row, sector, 1-D, contiguous, equal lengths, on one GPU."""
    import torch

    n = int(y.shape[0]) if hasattr(y, "shape") and len(y.shape) == 1 else -1
    if n < 0:
        raise TpcError(TPC_ERR_ARG, "y: expected a 1-D tensor")
    arrays = ((y, "y", torch.float32), (z, "z", torch.float32), (row, "row", torch.uint8),
              (sector, "sector", torch.uint8))
    for t, nm, dt in arrays:
        need(t, nm, dt, numel=n, on_gpu=False)
        if t.dim() != 1:
            raise TpcError(TPC_ERR_ARG, f"{nm}: expected a 1-D tensor")
    for t, nm, _ in arrays:
        need_gpu(t, nm)
    if len({t.device for t in (y, z, row, sector)}) != 1:
        raise TpcError(TPC_ERR_ARG, "cluster arrays must be on the same device")
    return n


def check_mlp(mlp):
    """Scorer parameters: 5057 float32 values on the GPU."""
    import torch

    if mlp is not None:
        need(mlp, "mlp", torch.float32, numel=MLP_N_PARAMS)


def check_rows(idx, n_rows: int, name: str):
    """Row indices must address rows of the feature array (checked on the device, one sync)."""
    if idx.numel() and (int(idx.min()) < 0 or int(idx.max()) >= n_rows):
        raise TpcError(TPC_ERR_ARG, f"{name}: row indices must lie in [0, {n_rows})")


def check_tracks(o: dict):
    """A track output (as ``Context.alloc_tracks`` returns): every array large enough for its capacity."""
    import torch

    ct, ch = int(o["cap_tracks"]), int(o["cap_hits"])
    if ct < 0 or ch < 0 or ct >= 2 ** 31 or ch >= 2 ** 31:
        raise TpcError(TPC_ERR_ARG, "capacities must be in [0, 2^31)")
    arrays = (("counts", torch.int32, N_COUNTS, 0), ("hit_offset", torch.int32, 0, 1), ("n_hits", torch.int32, 0, 1),
              ("start_id", torch.int32, 0, 1), ("sector", torch.int32, 0, 1), ("row_ref", torch.int32, 0, 1),
              ("x_ref", torch.float32, 0, 1), ("state", torch.float32, 0, 5), ("cov", torch.float32, 0, 15),
              ("chi2", torch.float32, 0, 1), ("ndf", torch.int32, 0, 1))
    for k, dt, fixed, per in arrays:
        need(o[k], k, dt, min_numel=fixed + per * ct, on_gpu=False)
    need(o["hit_ids"], "hit_ids", torch.int32, min_numel=ch, on_gpu=False)
    for k, *_ in arrays:
        need_gpu(o[k], k)
    need_gpu(o["hit_ids"], "hit_ids")


def check_merged(out: dict, cap_tracks: int):
    """A merge output (as ``Context.alloc_merged`` returns) large enough for cap_tracks tracks."""
    import torch

    if int(out["cap_tracks"]) < cap_tracks:
        raise TpcError(TPC_ERR_ARG, f"merge output: cap_tracks {int(out['cap_tracks'])} below the track set's "
                                    f"{cap_tracks}")
    c = max(1, cap_tracks)
    arrays = (("label", torch.int32, 1), ("n_members", torch.int32, 1), ("helix", torch.float64, 5),
              ("helix_cov", torch.float64, 15), ("theta", torch.float64, 5), ("theta_cov", torch.float64, 15),
              ("chi2", torch.float64, 1), ("ndf", torch.int32, 1))
    for k, dt, per in arrays:
        need(out[k], k, dt, min_numel=per * c, on_gpu=False)
    need(out["counts"], "counts", torch.int64, min_numel=len(MG_COUNTS), on_gpu=False)
    for k, *_ in arrays:
        need_gpu(out[k], k)
    need_gpu(out["counts"], "counts")


def _stream(stream) -> int:
    import torch

    s = stream if stream is not None else torch.cuda.current_stream()
    return int(s.cuda_stream)


def make_params(params: dict | None = None, mlp=None, tau_logit: float = 0.0) -> Params:
    p = Params()
    load().tpc_params_default(ctypes.byref(p))
    for k, v in (params or {}).items():
        if k in ("mlp", "tie_rel", "mlp_flag_abs"):
            continue
        if any(k == f for f, _ in Params._fields_):
            setattr(p, k, v)
    p.mlp = _ptr(mlp) if mlp is not None else None
    p.mlp_tau_logit = float(tau_logit) if mlp is not None else float((params or {}).get("mlp_tau_logit", 0.0))
    return p


def make_geometry(geom: dict):
    rx = np.ascontiguousarray(geom["row_x"], dtype=np.float32)
    g = Geometry()
    g.n_rows = int(geom["n_rows"])
    g.row_x = rx.ctypes.data_as(ctypes.POINTER(ctypes.c_float))
    g.tan_half = float(geom["tan_half"])
    g.n_sectors = int(geom["n_sectors"])
    g.z_min = float(geom["z_min"])
    g.z_max = float(geom["z_max"])
    return g, rx  # keep rx alive


class Context:
    """A library context on one HIP device; owns the scratch memory."""

    def __init__(self, device: int = 0):
        self.lib = load()
        h = _vp()
        rc = self.lib.tpc_ctx_create(ctypes.byref(h), device)
        if rc != TPC_OK:
            raise TpcError(rc, f"tpc_ctx_create(device={device}) failed")
        self.h = h
        self.device = device

    def close(self):
        if getattr(self, "h", None):
            self.lib.tpc_ctx_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc: int):
        if rc != TPC_OK:
            raise TpcError(rc, self.lib.tpc_last_error(self.h).decode())

    # ------------------------------------------------------------------ tracking
    def alloc_tracks(self, cap_tracks: int, cap_hits: int):
        import torch

        dev = torch.device("cuda", self.device)
        i32 = dict(dtype=torch.int32, device=dev)
        f32 = dict(dtype=torch.float32, device=dev)
        ct = max(1, cap_tracks)
        return dict(counts=torch.zeros(N_COUNTS, **i32), hit_offset=torch.empty(ct, **i32),
                    n_hits=torch.empty(ct, **i32), hit_ids=torch.empty(max(1, cap_hits), **i32),
                    start_id=torch.empty(ct, **i32), sector=torch.empty(ct, **i32), row_ref=torch.empty(ct, **i32),
                    x_ref=torch.empty(ct, **f32), state=torch.empty(ct, 5, **f32), cov=torch.empty(ct, 15, **f32),
                    chi2=torch.empty(ct, **f32), ndf=torch.empty(ct, **i32), cap_tracks=cap_tracks, cap_hits=cap_hits)

    @staticmethod
    def _tracks_struct(o: dict) -> Tracks:
        check_tracks(o)
        t = Tracks()
        t.cap_tracks = o["cap_tracks"]
        t.cap_hits = o["cap_hits"]
        for k in ("counts", "hit_offset", "n_hits", "hit_ids", "start_id", "sector", "row_ref", "x_ref", "state",
                  "cov", "chi2", "ndf"):
            setattr(t, k, _ptr(o[k]))
        return t

    @staticmethod
    def _clusters(y, z, row, sector) -> Clusters:
        c = Clusters()
        c.n = check_clusters(y, z, row, sector)
        c.y, c.z, c.row, c.sector = _ptr(y), _ptr(z), _ptr(row), _ptr(sector)
        return c

    def track(self, y, z, row, sector, geom: dict, bz: float, params: dict | None = None, mlp=None,
              tau_logit: float = 0.0, out: dict | None = None, stream=None, sync_check: bool = True,
              timeframe: bool = False) -> dict:
        """Track clusters given as CUDA tensors (float32 y, z; uint8 row, sector)."""
        cl = self._clusters(y, z, row, sector)
        check_mlp(mlp)
        n = int(cl.n)
        if out is None:
            out = self.alloc_tracks(max(16, n // 8), max(16, n))
        g, _keep = make_geometry(geom)
        p = make_params(params, mlp, tau_logit)
        t = self._tracks_struct(out)
        fn = self.lib.tpc_track_timeframe if timeframe else self.lib.tpc_track_sectors
        rc = fn(self.h, ctypes.byref(cl), ctypes.byref(g), float(bz), ctypes.byref(p), ctypes.byref(t),
                _stream(stream), 1 if sync_check else 0)
        self._check(rc)
        return out

    def cluster_flags(self, y, z, row, sector, geom: dict, bz: float, tracks: dict, params: dict | None = None,
                      tube_cm: float = 1.5, pt_min: float = 0.05, phi_max_deg: float = 70.0, flags=None,
                      stream=None):
        """Attachment / adjacency / protection / removal flags (uint8 per cluster, CUDA tensor) for a
        track set in the form ``alloc_tracks`` returns (counts, hit_offset, n_hits, hit_ids, sector,
        x_ref, state are read)."""
        import torch

        cl = self._clusters(y, z, row, sector)
        n = int(cl.n)
        if flags is None:
            flags = torch.empty(max(1, n), dtype=torch.uint8, device=y.device)
        need(flags, "flags", torch.uint8, min_numel=n)
        g, _keep = make_geometry(geom)
        p = make_params(params)
        fp = FlagParams(tube_cm, pt_min, phi_max_deg)
        t = self._tracks_struct(tracks)
        self._check(self.lib.tpc_cluster_flags(self.h, ctypes.byref(cl), ctypes.byref(g), float(bz), ctypes.byref(p),
                                               ctypes.byref(fp), ctypes.byref(t), _ptr(flags), _stream(stream)))
        return flags[:n]

    # ------------------------------------------------------------- compression
    def alloc_compressed(self, n: int, n_rows_total: int, cap_tracks: int, cap_esc: int | None = None,
                         cap_bytes: int | None = None) -> dict:
        """Output buffers of ``compress`` for n clusters, n_sectors * n_rows rows and cap_tracks tracks."""
        import torch

        d = torch.device("cuda", self.device)
        cap_sym = n + n_rows_total
        nb = cap_sym // CS_BLOCK + 1
        cap_esc = cap_esc if cap_esc is not None else max(16, cap_sym // 4)
        cap_bytes = cap_bytes if cap_bytes is not None else 2 * N_CSTREAMS * cap_sym + 4 * N_CSTREAMS * nb
        return dict(cap_sym=cap_sym, cap_esc=cap_esc, cap_bytes=cap_bytes,
                    counts=torch.zeros(N_CSTREAMS * CSC_N + CST_N, dtype=torch.int64, device=d),
                    sym=torch.zeros(N_CSTREAMS * cap_sym, dtype=torch.int16, device=d),
                    esc=torch.zeros(N_CSTREAMS * max(1, cap_esc), dtype=torch.int32, device=d),
                    freq=torch.zeros(N_CSTREAMS * CS_ALPHABET, dtype=torch.int32, device=d),
                    block_bytes=torch.zeros(N_CSTREAMS * nb, dtype=torch.int32, device=d),
                    bytes=torch.zeros(max(1, cap_bytes), dtype=torch.uint8, device=d),
                    order=torch.zeros(max(1, n), dtype=torch.int32, device=d),
                    track_len=torch.zeros(max(1, cap_tracks), dtype=torch.int32, device=d))

    @staticmethod
    def _compressed_struct(c: dict) -> Compressed:
        return Compressed(c["cap_sym"], c["cap_esc"], c["cap_bytes"], _ptr(c["counts"]), _ptr(c["sym"]),
                          _ptr(c["esc"]), _ptr(c["freq"]), _ptr(c["block_bytes"]), _ptr(c["bytes"]), _ptr(c["order"]),
                          _ptr(c["track_len"]))

    @staticmethod
    def _cparams(cparams: dict | None) -> CompressParams:
        cp = CompressParams()
        load().tpc_compress_params_default(ctypes.byref(cp))
        for k, v in (cparams or {}).items():
            setattr(cp, k, v)
        return cp

    def compress(self, y, z, row, sector, qtot, sigma_y, sigma_z, geom: dict, bz: float, tracks: dict,
                 params: dict | None = None, cparams: dict | None = None, out: dict | None = None, stream=None,
                 sync_check: bool = True) -> dict:
        """Compress clusters given as CUDA tensors (positions as for ``track``; uint16 charge, uint8
        widths) with their tracks (the layout ``alloc_tracks`` returns)."""
        import torch

        cl = self._clusters(y, z, row, sector)
        n = int(cl.n)
        need(qtot, "qtot", torch.int16 if qtot.dtype == torch.int16 else torch.uint16, numel=n)
        need(sigma_y, "sigma_y", torch.uint8, numel=n)
        need(sigma_z, "sigma_z", torch.uint8, numel=n)
        check_tracks(tracks)
        g, _keep = make_geometry(geom)
        if out is None:
            out = self.alloc_compressed(n, int(geom["n_sectors"]) * int(geom["n_rows"]), int(tracks["cap_tracks"]))
        p = make_params(params)
        cp = self._cparams(cparams)
        pr = ClusterProps(_ptr(qtot), _ptr(sigma_y), _ptr(sigma_z))
        t = self._tracks_struct(tracks)
        o = self._compressed_struct(out)
        self._check(self.lib.tpc_compress(self.h, ctypes.byref(cl), ctypes.byref(pr), ctypes.byref(g), float(bz),
                                          ctypes.byref(p), ctypes.byref(cp), ctypes.byref(t), ctypes.byref(o),
                                          _stream(stream), 1 if sync_check else 0))
        return out

    def decompress(self, comp: dict, geom: dict, bz: float, tracks: dict, params: dict | None = None,
                   cparams: dict | None = None, stream=None) -> dict:
        """Decode ``compress`` output: symbols and the clusters in stream order (device tensors)."""
        import torch

        check_tracks(tracks)
        counts = comp["counts"].cpu().numpy()
        n = int(counts[N_CSTREAMS * CSC_N + CST_ATTACHED] + counts[N_CSTREAMS * CSC_N + CST_UNATTACHED])
        d = torch.device("cuda", self.device)
        m = max(1, n)
        res = dict(sym=torch.zeros(N_CSTREAMS * comp["cap_sym"], dtype=torch.int16, device=d),
                   sector=torch.zeros(m, dtype=torch.uint8, device=d), row=torch.zeros(m, dtype=torch.uint8, device=d),
                   yq=torch.zeros(m, dtype=torch.int32, device=d), zq=torch.zeros(m, dtype=torch.int32, device=d),
                   qtot=torch.zeros(m, dtype=torch.int16, device=d),
                   sigma_y=torch.zeros(m, dtype=torch.uint8, device=d),
                   sigma_z=torch.zeros(m, dtype=torch.uint8, device=d))
        g, _keep = make_geometry(geom)
        p = make_params(params)
        cp = self._cparams(cparams)
        t = self._tracks_struct(tracks)
        o = self._compressed_struct(comp)
        self._check(self.lib.tpc_decompress(self.h, ctypes.byref(o), ctypes.byref(g), float(bz), ctypes.byref(p),
                                            ctypes.byref(cp), ctypes.byref(t), *(_ptr(res[k]) for k in (
                                                "sym", "sector", "row", "yq", "zq", "qtot", "sigma_y", "sigma_z")),
                                            _stream(stream)))
        res["n"] = n
        return res

    def compress_sizes(self, comp: dict) -> np.ndarray:
        """[stream][entropy bits, Huffman bits, range-ANS bits] of the last ``compress`` call."""
        b = (ctypes.c_double * (3 * N_CSTREAMS))()
        self._check(self.lib.tpc_compress_sizes(self.h, ctypes.byref(self._compressed_struct(comp)), b))
        return np.array(b[:], dtype=np.float64).reshape(N_CSTREAMS, 3)

    # ------------------------------------------------------------------ merging
    def alloc_merged(self, cap_tracks: int) -> dict:
        """Output buffers of ``merge`` for a track set of capacity cap_tracks."""
        import torch

        d = torch.device("cuda", self.device)
        c = max(1, cap_tracks)
        f64 = dict(dtype=torch.float64, device=d)
        return dict(cap_tracks=cap_tracks, label=torch.empty(c, dtype=torch.int32, device=d),
                    n_members=torch.empty(c, dtype=torch.int32, device=d), helix=torch.empty(c, 5, **f64),
                    helix_cov=torch.empty(c, 15, **f64), theta=torch.empty(c, 5, **f64),
                    theta_cov=torch.empty(c, 15, **f64), chi2=torch.empty(c, **f64),
                    ndf=torch.empty(c, dtype=torch.int32, device=d),
                    counts=torch.zeros(len(MG_COUNTS), dtype=torch.int64, device=d))

    @staticmethod
    def merge_params(mparams: dict | None = None) -> MergeParams:
        mp = MergeParams()
        load().tpc_merge_params_default(ctypes.byref(mp))
        for k, v in (mparams or {}).items():
            setattr(mp, k, v)
        return mp

    def merge(self, y, z, row, sector, geom: dict, bz: float, tracks: dict, params: dict | None = None,
              mparams: dict | None = None, out: dict | None = None, stream=None) -> dict:
        """Merge the pieces of one helix among ``tracks`` (the layout ``alloc_tracks`` returns) and
        refit every merged track over its hits (clusters as CUDA tensors, as for ``track``)."""
        cl = self._clusters(y, z, row, sector)
        check_tracks(tracks)
        if out is None:
            out = self.alloc_merged(int(tracks["cap_tracks"]))
        check_merged(out, int(tracks["cap_tracks"]))
        g, _keep = make_geometry(geom)
        p = make_params(params)
        mp = self.merge_params(mparams)
        t = self._tracks_struct(tracks)
        o = Merged(int(out["cap_tracks"]), *(_ptr(out[k]) for k in ("label", "n_members", "helix", "helix_cov",
                                                                     "theta", "theta_cov", "chi2", "ndf",
                                                                     "counts")))
        self._check(self.lib.tpc_merge(self.h, ctypes.byref(cl), ctypes.byref(g), float(bz), ctypes.byref(p),
                                       ctypes.byref(mp), ctypes.byref(t), ctypes.byref(o), _stream(stream)))
        return out

    def stage(self, stage: int, dtype) -> np.ndarray:
        nb = ctypes.c_size_t(0)
        self._check(self.lib.tpc_stage_size(self.h, stage, ctypes.byref(nb)))
        a = np.empty(nb.value // np.dtype(dtype).itemsize, dtype=dtype)
        self._check(self.lib.tpc_stage_copy(self.h, stage, a.ctypes.data, nb.value))
        return a

    def profile(self, on: bool):
        self._check(self.lib.tpc_profile_enable(self.h, 1 if on else 0))

    def profile_read(self) -> tuple[dict, int]:
        ms = (ctypes.c_double * N_PROF)()
        n = ctypes.c_int(0)
        self._check(self.lib.tpc_profile_read(self.h, ms, ctypes.byref(n)))
        return {k: ms[i] for i, k in enumerate(PROF_STAGES)}, n.value

    # --------------------------------------------------------------- time frames
    def tuning(self) -> dict:
        t = Tuning()
        self._check(self.lib.tpc_timeframe_tuning(self.h, ctypes.byref(t)))
        return {f: getattr(t, f) for f, _ in Tuning._fields_}

    def set_tune_cache(self, path: str | None):
        """Persist time-frame tiles in a text file (None: no cache); see tpc_timeframe_tune_cache."""
        self._check(self.lib.tpc_timeframe_tune_cache(self.h, os.fsencode(path) if path else None))

    def set_tuning(self, tiles: dict | None):
        if tiles is None:
            self._check(self.lib.tpc_timeframe_set_tuning(self.h, None))
            return
        t = Tuning()
        t.waves_per_simd = 2
        for k, v in tiles.items():
            setattr(t, k, v)
        self._check(self.lib.tpc_timeframe_set_tuning(self.h, ctypes.byref(t)))

    # ------------------------------------------------------------- learned scorer
    def mlp_infer(self, feats, mlp, logits=None, stream=None):
        import torch

        need(feats, "feats", torch.float32, cols=12)
        check_mlp(mlp)
        if mlp is None:
            raise TpcError(TPC_ERR_ARG, "mlp is required")
        n = int(feats.shape[0])
        if logits is None:
            logits = torch.empty(max(1, n), dtype=torch.float32, device=feats.device)
        need(logits, "logits", torch.float32, min_numel=n)
        self._check(self.lib.tpc_mlp_infer(self.h, _ptr(feats), n, _ptr(mlp), _ptr(logits), _stream(stream)))
        return logits[:n]

    def triplets(self, y, z, row, sector, geom: dict, params: dict | None = None, cap: int | None = None,
                 stream=None):
        import torch

        cl = self._clusters(y, z, row, sector)
        n = int(cl.n)
        cap = cap or max(64, 4 * n)
        dev = y.device
        trip = torch.empty(cap, 3, dtype=torch.int32, device=dev)
        feats = torch.empty(cap, 12, dtype=torch.float32, device=dev)
        g, _keep = make_geometry(geom)
        p = make_params(params)
        nout = ctypes.c_int64(0)
        self._check(self.lib.tpc_triplets(self.h, ctypes.byref(cl), ctypes.byref(g), ctypes.byref(p), _ptr(trip),
                                          _ptr(feats), cap, ctypes.byref(nout), _stream(stream)))
        if nout.value > cap:
            return self.triplets(y, z, row, sector, geom, params, cap=int(nout.value), stream=stream)
        return trip[:nout.value], feats[:nout.value]

    def mlp_grad(self, feats, labels, idx, mlp, stream=None):
        import torch

        need(feats, "feats", torch.float32, cols=12)
        need(labels, "labels", torch.uint8, numel=int(feats.shape[0]))
        need(idx, "idx", torch.int32)
        if idx.dim() != 1:
            raise TpcError(TPC_ERR_ARG, "idx: expected a 1-D tensor")
        check_mlp(mlp)
        check_rows(idx, int(feats.shape[0]), "idx")
        grad = torch.empty(MLP_N_PARAMS, dtype=torch.float32, device=feats.device)
        loss = torch.empty(1, dtype=torch.float32, device=feats.device)
        self._check(self.lib.tpc_mlp_grad(self.h, _ptr(feats), _ptr(labels), _ptr(idx), int(idx.shape[0]), _ptr(mlp),
                                          _ptr(grad), _ptr(loss), _stream(stream)))
        return grad, loss

    def mlp_train(self, feats, labels, order, mlp, m, v, batch: int, n_steps: int, step0: int = 0,
                  lr: float = 1e-3, beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8, stream=None,
                  loss=None, noalloc: bool = False):
        """Adam steps on the scorer (tpc_mlp_train; tpc_mlp_train_noalloc with ``noalloc``, which uses the
        library's fixed per-device scratch and allocates nothing).  ``loss`` (device, >= n_steps floats)
        receives each step's loss; if None a tensor is allocated here."""
        import torch

        need(feats, "feats", torch.float32, cols=12)
        need(labels, "labels", torch.uint8, numel=int(feats.shape[0]))
        need(order, "order", torch.int32, min_numel=int(batch) * int(n_steps))
        for t, nm in ((mlp, "mlp"), (m, "m"), (v, "v")):
            need(t, nm, torch.float32, numel=MLP_N_PARAMS)
        check_rows(order[:int(batch) * int(n_steps)], int(feats.shape[0]), "order")
        if loss is None:
            loss = torch.empty(max(1, n_steps), dtype=torch.float32, device=feats.device)
        else:
            need(loss, "loss", torch.float32, min_numel=max(1, int(n_steps)))
        cfg = TrainCfg(batch=batch, n_steps=n_steps, step0=step0, lr=lr, beta1=beta1, beta2=beta2, eps=eps)
        fn = self.lib.tpc_mlp_train_noalloc if noalloc else self.lib.tpc_mlp_train
        self._check(fn(self.h, _ptr(feats), _ptr(labels), _ptr(order), ctypes.byref(cfg), _ptr(mlp), _ptr(m), _ptr(v),
                       _ptr(loss), _stream(stream)))
        return loss


def tracks_to_host(out: dict) -> dict:
    """Counts and the filled part of a track output, as numpy arrays (synchronises)."""
    counts = out["counts"].cpu().numpy()
    nt = min(int(counts[CNT_TRACKS]), out["cap_tracks"])
    nh = min(int(counts[CNT_TRACK_HITS]), out["cap_hits"])
    res = {"counts": counts}
    for k in ("hit_offset", "n_hits", "start_id", "sector", "row_ref", "x_ref", "state", "cov", "chi2", "ndf"):
        res[k] = out[k][:nt].cpu().numpy()
    res["hit_ids"] = out["hit_ids"][:nh].cpu().numpy()
    return res
