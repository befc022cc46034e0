"""FP64 CPU oracle (TEST INFRASTRUCTURE ONLY).

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py`` may
import this package.  It shares no code with the HIP library ``paper_1910_12214_amd``:
the tracker is plain C in ``tpc_oracle.c`` (built with gcc, ``-ffp-contract=off``), the
learned-scorer reference is plain numpy in ``mlp.py``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libtpcoracle.so")
# The same source compiled with FMA contraction: only the rounding differs.  Parity checks use
# the difference between the two builds as the oracle's own sensitivity to rounding.
_LIB_FMA_PATH = os.path.join(_HERE, "libtpcoracle_fma.so")

F_ARGMIN, F_CUT, F_WINDOW, F_SMAX, F_EDGE, F_MLP = 1, 2, 4, 8, 16, 32
N_MLP_PARAMS = 5057


def build() -> None:
    """Compile the oracle with gcc (no fast-math, no FMA contraction), and its FMA-contracted twin."""
    srcs = [os.path.join(_HERE, "tpc_oracle.c"), os.path.join(_HERE, "tpc_codec.c")]
    for path, fl in ((_LIB_PATH, ["-ffp-contract=off"]), (_LIB_FMA_PATH, ["-ffp-contract=fast", "-mfma"])):
        tmp = path + ".tmp"
        subprocess.check_call(["gcc", "-O2", *fl, "-fno-fast-math", "-fPIC", "-shared", "-o", tmp, *srcs, "-lm",
                               "-lpthread"])
        os.replace(tmp, path)


class _Params(ctypes.Structure):
    _fields_ = [
        ("win_y", ctypes.c_double), ("win_z", ctypes.c_double),
        ("nb_chi2_max", ctypes.c_double), ("fol_chi2_max", ctypes.c_double),
        ("sigma_y", ctypes.c_double), ("sigma_z", ctypes.c_double),
        ("s_max", ctypes.c_double), ("edge_margin", ctypes.c_double),
        ("l_min_chain", ctypes.c_int32), ("n_miss_max", ctypes.c_int32),
        ("n_min_tracklet", ctypes.c_int32), ("n_min_track", ctypes.c_int32),
        ("c0_sinphi", ctypes.c_double), ("c0_dzds", ctypes.c_double), ("c0_qpt", ctypes.c_double),
        ("bin_y", ctypes.c_float), ("bin_z", ctypes.c_float),
        ("tie_rel", ctypes.c_double),
        ("mlp", ctypes.POINTER(ctypes.c_double)),
        ("mlp_tau_logit", ctypes.c_double), ("mlp_flag_abs", ctypes.c_double),
    ]


class _Input(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int64),
        ("y", ctypes.POINTER(ctypes.c_float)), ("z", ctypes.POINTER(ctypes.c_float)),
        ("row", ctypes.POINTER(ctypes.c_uint8)), ("sector", ctypes.POINTER(ctypes.c_uint8)),
        ("n_rows", ctypes.c_int32), ("row_x", ctypes.POINTER(ctypes.c_float)),
        ("tan_half", ctypes.c_float), ("n_sectors", ctypes.c_int32),
        ("z_min", ctypes.c_float), ("z_max", ctypes.c_float),
        ("bz", ctypes.c_double), ("n_threads", ctypes.c_int32),
    ]


_P = ctypes.POINTER


class _Output(ctypes.Structure):
    _fields_ = [
        ("n_valid", ctypes.c_int64), ("n_bins", ctypes.c_int64),
        ("sorted_id", _P(ctypes.c_uint32)), ("row_off", _P(ctypes.c_uint32)),
        ("bin_base", _P(ctypes.c_uint32)), ("bin_off", _P(ctypes.c_uint32)),
        ("up", _P(ctypes.c_int32)), ("dn", _P(ctypes.c_int32)),
        ("up_c", _P(ctypes.c_int32)), ("dn_c", _P(ctypes.c_int32)),
        ("nb_flag", _P(ctypes.c_uint8)), ("n_pairs", _P(ctypes.c_int32)),
        ("n_starts", ctypes.c_int64), ("start_id", _P(ctypes.c_uint32)),
        ("tl_nhits", _P(ctypes.c_int32)), ("tl_hits", _P(ctypes.c_int32)),
        ("tl_state", _P(ctypes.c_double)), ("tl_cov", _P(ctypes.c_double)),
        ("tl_chi2", _P(ctypes.c_double)), ("tl_ndf", _P(ctypes.c_int32)),
        ("tl_row_ref", _P(ctypes.c_int32)), ("tl_valid", _P(ctypes.c_uint8)),
        ("tl_fail", _P(ctypes.c_uint8)), ("tl_flag", _P(ctypes.c_uint8)),
        ("hit_key", _P(ctypes.c_uint64)),
        ("n_tracks", ctypes.c_int64), ("n_track_hits", ctypes.c_int64),
        ("trk_tl", _P(ctypes.c_int32)), ("trk_off", _P(ctypes.c_int32)), ("trk_hits", _P(ctypes.c_int32)),
        ("n_fit_fail", ctypes.c_int64), ("n_links_raw", ctypes.c_int64), ("n_links_clean", ctypes.c_int64),
    ]


_libs: dict = {}


def _load(path: str = _LIB_PATH):
    lib = _libs.get(path)
    if lib is None:
        if not os.path.exists(path):
            build()
        lib = ctypes.CDLL(path)
        d = ctypes.POINTER(ctypes.c_double)
        lib.or_track.argtypes = [ctypes.POINTER(_Input), ctypes.POINTER(_Params), ctypes.c_int, ctypes.POINTER(_Output)]
        lib.or_track.restype = ctypes.c_int
        lib.or_free.argtypes = [ctypes.POINTER(_Output)]
        lib.or_free.restype = None
        lib.or_propagate.argtypes = [d, ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                     ctypes.c_double, d, d, ctypes.POINTER(ctypes.c_int)]
        lib.or_propagate.restype = ctypes.c_int
        lib.or_cov_propagate.argtypes = [d, d]
        lib.or_cov_propagate.restype = None
        lib.or_kf_update.argtypes = [d, d, ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_double, d]
        lib.or_kf_update.restype = ctypes.c_int
        lib.or_mlp_logit.argtypes = [d, d]
        lib.or_mlp_logit.restype = ctypes.c_double
        lib.or_features.argtypes = [ctypes.c_double] * 11 + [ctypes.c_int, ctypes.c_int, d]
        lib.or_features.restype = None
        lib.or_follow_search.argtypes = [ctypes.POINTER(_Input), ctypes.POINTER(_Params), ctypes.c_int, ctypes.c_int,
                                         d, d, ctypes.POINTER(ctypes.c_int)]
        lib.or_follow_search.restype = ctypes.c_int64
        lib.or_cluster_flags.argtypes = [ctypes.POINTER(_FlagsIn), ctypes.POINTER(ctypes.c_uint8),
                                         ctypes.POINTER(ctypes.c_uint8)]
        lib.or_cluster_flags.restype = ctypes.c_int
        _libs[path] = lib
    return lib


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


KQ_PER_TESLA = -0.00299792458  # curvature per (q/pT) per Tesla, cm^-1 (GeV/c)^-1 T^-1


def propagate(p, x0: float, x1: float, bz: float, s_max: float = 0.999):
    """Sector-local helix step.  Returns (p1, F, failed)."""
    lib = _load()
    p0 = np.ascontiguousarray(p, dtype=np.float64)
    p1 = np.zeros(5)
    F = np.zeros(25)
    fl = ctypes.c_int(0)
    rc = lib.or_propagate(_dptr(p0), x0, x1, KQ_PER_TESLA * bz, s_max, 1e-5, _dptr(p1), _dptr(F), ctypes.byref(fl))
    return p1, F.reshape(5, 5), bool(rc)


def cov_propagate(c15, F):
    lib = _load()
    c = np.ascontiguousarray(c15, dtype=np.float64).copy()
    Fm = np.ascontiguousarray(F, dtype=np.float64).reshape(25)
    lib.or_cov_propagate(_dptr(c), _dptr(Fm))
    return c


def kf_update(p, c15, my, mz, vy, vz):
    lib = _load()
    pp = np.ascontiguousarray(p, dtype=np.float64).copy()
    cc = np.ascontiguousarray(c15, dtype=np.float64).copy()
    chi2 = np.zeros(1)
    bad = lib.or_kf_update(_dptr(pp), _dptr(cc), my, mz, vy, vz, _dptr(chi2))
    return pp, cc, float(chi2[0]), bool(bad)


def mlp_logit(params: np.ndarray, f: np.ndarray) -> float:
    lib = _load()
    w = np.ascontiguousarray(params, dtype=np.float64)
    ff = np.ascontiguousarray(f, dtype=np.float64)
    return float(lib.or_mlp_logit(_dptr(w), _dptr(ff)))


def features(xd, yd, zd, xm, ym, zm, xu, yu, zu, win_y, win_z, n_up, n_dn) -> np.ndarray:
    lib = _load()
    f = np.zeros(12)
    lib.or_features(xd, yd, zd, xm, ym, zm, xu, yu, zu, win_y, win_z, n_up, n_dn, _dptr(f))
    return f


def sym15_to_full(c15) -> np.ndarray:
    M = np.zeros((5, 5))
    k = 0
    for i in range(5):
        for j in range(i + 1):
            M[i, j] = M[j, i] = c15[k]
            k += 1
    return M


def full_to_sym15(M) -> np.ndarray:
    return np.array([M[i, j] for i in range(5) for j in range(i + 1)])


def _make_input(y, z, row, sector, geometry: dict, bz: float, n_threads: int, keep: list) -> "_Input":
    y = np.ascontiguousarray(y, dtype=np.float32)
    z = np.ascontiguousarray(z, dtype=np.float32)
    row = np.ascontiguousarray(row, dtype=np.uint8)
    sector = np.ascontiguousarray(sector, dtype=np.uint8)
    rx = np.ascontiguousarray(geometry["row_x"], dtype=np.float32)
    keep += [y, z, row, sector, rx]
    inp = _Input()
    inp.n = y.shape[0]
    inp.y = y.ctypes.data_as(_P(ctypes.c_float)); inp.z = z.ctypes.data_as(_P(ctypes.c_float))
    inp.row = row.ctypes.data_as(_P(ctypes.c_uint8)); inp.sector = sector.ctypes.data_as(_P(ctypes.c_uint8))
    inp.n_rows = int(geometry["n_rows"]); inp.row_x = rx.ctypes.data_as(_P(ctypes.c_float))
    inp.tan_half = float(geometry["tan_half"]); inp.n_sectors = int(geometry["n_sectors"])
    inp.z_min = float(geometry["z_min"]); inp.z_max = float(geometry["z_max"])
    inp.bz = float(bz); inp.n_threads = int(n_threads)
    return inp


def _make_params(params: dict) -> "_Params":
    prm = _Params()
    for f, _ in _Params._fields_:
        if f in params and f != "mlp":
            setattr(prm, f, params[f])
    prm.tie_rel = params.get("tie_rel", 1e-5)
    return prm


def follow_search(y, z, row, sector, geometry: dict, params: dict, s: int, r: int, p, c15):
    """The oracle's following search of row-sector (s, r) on its own: the cluster id of the
    smallest chi2 inside the cut (ties: smallest id), or -1, and the near-tie flag bits."""
    lib = _load(_LIB_PATH)
    keep: list = []
    inp = _make_input(y, z, row, sector, geometry, 0.0, 1, keep)
    prm = _make_params(params)
    pp = np.ascontiguousarray(p, dtype=np.float64)
    cc = np.ascontiguousarray(c15, dtype=np.float64)
    fl = ctypes.c_int(0)
    rc = lib.or_follow_search(ctypes.byref(inp), ctypes.byref(prm), int(s), int(r), _dptr(pp), _dptr(cc),
                              ctypes.byref(fl))
    if rc < -1:
        raise ValueError("oracle rejected its input")
    return int(rc), int(fl.value)


STAGE_GRID, STAGE_NEIGHBOURS, STAGE_CLEAN, STAGE_TRACKLETS, STAGE_SELECT = 1, 2, 4, 8, 16
ALL_STAGES = 31


def track(y, z, row, sector, geometry: dict, params: dict, bz: float, mlp: np.ndarray | None = None,
          stages: int = ALL_STAGES, n_threads: int = 1, fma: bool = False) -> dict:
    """Run the oracle on host arrays.  Returns a dict of numpy arrays (copies).

    geometry: n_rows, row_x (float32 array), tan_half, n_sectors, z_min, z_max.
    params: the tracker settings (see ``_Params``); tie_rel defaults to 1e-5.
    mlp: 5057 BF16-valued parameters (float64 array) or None for the plain finder.
    fma: run the FMA-contracted build (same arithmetic, different rounding).
    """
    lib = _load(_LIB_FMA_PATH if fma else _LIB_PATH)
    keep: list = []
    inp = _make_input(y, z, row, sector, geometry, bz, n_threads, keep)
    prm = _make_params(params)
    mlp_arr = None
    if mlp is not None:
        mlp_arr = np.ascontiguousarray(mlp, dtype=np.float64)
        assert mlp_arr.shape == (N_MLP_PARAMS,)
        prm.mlp = _dptr(mlp_arr)
        prm.mlp_tau_logit = float(params.get("mlp_tau_logit", 0.0))
        prm.mlp_flag_abs = float(params.get("mlp_flag_abs", 1e-4))
    out = _Output()
    rc = lib.or_track(ctypes.byref(inp), ctypes.byref(prm), stages, ctypes.byref(out))
    if rc != 0:
        lib.or_free(ctypes.byref(out))
        raise ValueError(f"oracle rejected its input ({rc})")
    n = inp.n
    R = inp.n_rows
    S = inp.n_sectors

    def cp(ptr, count, dt):
        if not ptr or count == 0:
            return np.zeros(count, dtype=dt)
        return np.ctypeslib.as_array(ptr, shape=(count,)).astype(dt, copy=True)

    res = {"n_valid": out.n_valid, "n_bins": out.n_bins,
           "sorted_id": cp(out.sorted_id, out.n_valid, np.uint32),
           "row_off": cp(out.row_off, S * R + 1, np.uint32),
           "bin_base": cp(out.bin_base, S * R + 1, np.uint32),
           "bin_off": cp(out.bin_off, out.n_bins + 1, np.uint32)}
    if stages & STAGE_NEIGHBOURS:
        for k in ("up", "dn", "up_c", "dn_c", "n_pairs"):
            res[k] = cp(getattr(out, k), n, np.int32)
        res["nb_flag"] = cp(out.nb_flag, n, np.uint8)
        res["n_links_raw"] = out.n_links_raw
    if stages & STAGE_CLEAN:
        res["start_id"] = cp(out.start_id, out.n_starts, np.uint32)
        res["n_links_clean"] = out.n_links_clean
    if stages & STAGE_TRACKLETS:
        T = out.n_starts
        res["tl_nhits"] = cp(out.tl_nhits, T, np.int32)
        res["tl_hits"] = cp(out.tl_hits, T * R, np.int32).reshape(T, R)
        res["tl_state"] = cp(out.tl_state, T * 5, np.float64).reshape(T, 5)
        res["tl_cov"] = cp(out.tl_cov, T * 15, np.float64).reshape(T, 15)
        res["tl_chi2"] = cp(out.tl_chi2, T, np.float64)
        res["tl_ndf"] = cp(out.tl_ndf, T, np.int32)
        res["tl_row_ref"] = cp(out.tl_row_ref, T, np.int32)
        res["tl_valid"] = cp(out.tl_valid, T, np.uint8)
        res["tl_fail"] = cp(out.tl_fail, T, np.uint8)
        res["tl_flag"] = cp(out.tl_flag, T, np.uint8)
        res["n_fit_fail"] = out.n_fit_fail
    if stages & STAGE_SELECT:
        res["hit_key"] = cp(out.hit_key, n, np.uint64)
        nt = out.n_tracks
        res["trk_tl"] = cp(out.trk_tl, nt, np.int32)
        res["trk_off"] = cp(out.trk_off, nt + 1, np.int32)
        res["trk_hits"] = cp(out.trk_hits, out.n_track_hits, np.int32)
        res["n_tracks"] = nt
    lib.or_free(ctypes.byref(out))
    return res


# ---------------------------------------------------------------- cluster flags (Sec. 4)
FLAG_ATTACHED, FLAG_ADJACENT, FLAG_PROTECTED, FLAG_REMOVE_A, FLAG_REMOVE_B = 1, 2, 4, 8, 16


class _FlagsIn(ctypes.Structure):
    _P = ctypes.POINTER
    _fields_ = [("n", ctypes.c_int64), ("y", _P(ctypes.c_float)), ("z", _P(ctypes.c_float)),
                ("row", _P(ctypes.c_uint8)), ("sector", _P(ctypes.c_uint8)),
                ("n_rows", ctypes.c_int), ("n_sectors", ctypes.c_int), ("row_x", _P(ctypes.c_float)),
                ("kq", ctypes.c_double), ("s_max", ctypes.c_double), ("n_tracks", ctypes.c_int32),
                ("off", _P(ctypes.c_int32)), ("nh", _P(ctypes.c_int32)), ("hits", _P(ctypes.c_int32)),
                ("trk_sector", _P(ctypes.c_int32)), ("x_ref", _P(ctypes.c_float)), ("state", _P(ctypes.c_float)),
                ("tube", ctypes.c_double), ("pt_min", ctypes.c_double), ("sin_phi_max", ctypes.c_double)]


def tracks_for_flags(o: dict, geometry: dict, sector) -> dict:
    """The oracle's tracks (from ``track``) in the form ``cluster_flags`` takes: CSR hits,
    sector of the start hit, x of the reference row and the FP32-rounded state there."""
    nt = int(o["n_tracks"])
    off = o["trk_off"][:nt].astype(np.int32)
    nh = np.diff(o["trk_off"][:nt + 1]).astype(np.int32)
    hits = o["trk_hits"].astype(np.int32)
    tl = o["trk_tl"][:nt]
    rx = np.asarray(geometry["row_x"], dtype=np.float32)
    sec = np.asarray(sector)[hits[off]] if nt else np.zeros(0, np.int32)
    return {"off": off, "nh": nh, "hits": hits, "sector": sec.astype(np.int32),
            "x_ref": rx[o["tl_row_ref"][tl]].astype(np.float32),
            "state": o["tl_state"][tl].astype(np.float32)}


def cluster_flags(y, z, row, sector, geometry: dict, bz: float, tracks: dict, tube: float = 1.5,
                  pt_min: float = 0.05, phi_max_deg: float = 70.0, s_max: float = 0.999, fma: bool = False):
    """Attachment / adjacency / protection / removal flags per cluster (Sec. 4).

    tracks: off, nh, hits (CSR of cluster ids, ascending row), sector, x_ref (float32) and
    state (float32 [n, 5]).  Returns (flags uint8[n], tie uint8[n]); tie marks clusters whose
    decision lies within 1e-9 (relative) of a cut.
    """
    lib = _load(_LIB_FMA_PATH if fma else _LIB_PATH)
    keep = []

    def arr(a, dt):
        a = np.ascontiguousarray(a, dtype=dt)
        keep.append(a)
        return a.ctypes.data_as(ctypes.POINTER(np.ctypeslib.as_ctypes_type(dt)))

    inp = _FlagsIn()
    n = int(np.asarray(y).shape[0])
    inp.n = n
    inp.y, inp.z = arr(y, np.float32), arr(z, np.float32)
    inp.row, inp.sector = arr(row, np.uint8), arr(sector, np.uint8)
    inp.n_rows, inp.n_sectors = int(geometry["n_rows"]), int(geometry["n_sectors"])
    inp.row_x = arr(geometry["row_x"], np.float32)
    inp.kq, inp.s_max = KQ_PER_TESLA * float(bz), float(s_max)
    inp.n_tracks = int(len(tracks["off"]))
    inp.off, inp.nh, inp.hits = arr(tracks["off"], np.int32), arr(tracks["nh"], np.int32), arr(
        tracks["hits"] if len(tracks["hits"]) else np.zeros(1), np.int32)
    inp.trk_sector = arr(tracks["sector"], np.int32)
    inp.x_ref = arr(tracks["x_ref"], np.float32)
    inp.state = arr(np.asarray(tracks["state"]).reshape(-1), np.float32)
    inp.tube, inp.pt_min = float(tube), float(pt_min)
    inp.sin_phi_max = float(np.sin(np.deg2rad(phi_max_deg)))
    flags = np.zeros(max(n, 1), dtype=np.uint8)
    tie = np.zeros(max(n, 1), dtype=np.uint8)
    u8 = ctypes.POINTER(ctypes.c_uint8)
    rc = lib.or_cluster_flags(ctypes.byref(inp), flags.ctypes.data_as(u8), tie.ctypes.data_as(u8))
    if rc != 0:
        raise MemoryError("oracle cluster flags: allocation failed")
    return flags[:n], tie[:n]
