"""Seeded synthetic TPC workloads (input generator shared by the oracle and the HIP path).

The paper's TPC studies run on ALICE simulated Pb-Pb and pp collisions (Sec. 4, Figs. 4-7);
that simulation is not available, so these generators stand in for it.  Geometry and
rates follow the workloads the tracker is measured on:

* 36 sectors (18 per z side, 20 degrees each), 152 pad rows at 85-247 cm, z in [0, 250] cm
  per side, Bz = 0.5 T;
* clusters (row, y, z) in FP32 in each sector's local frame (the reconstruction works on
  single-precision clusters, Sec. 4 step 2);
* continuous-readout time frames at 50 kHz Pb-Pb and 1 MHz pp (Sec. 1) shift every
  collision's clusters in z by v_drift * t0 with v_drift = 2.58 cm/us.

Nothing here implements the tracking method: crossings are computed analytically in the
global frame by ``tpcsynth.c``.  The module only draws inputs and truth.
"""
from __future__ import annotations

import ctypes
import hashlib
import math
import os
from dataclasses import dataclass, field, replace

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libtpcsynth.so")

N_ROWS = 152
N_SECTORS = 36
BZ = 0.5
V_DRIFT = 2.58  # cm / us
Z_LEN = 250.0


def row_x() -> np.ndarray:
    """Pad-row radii: 152 rows uniformly spaced at 85..247 cm (endpoints inclusive), as FP32."""
    return np.array([85.0 + i * 162.0 / 151.0 for i in range(N_ROWS)], dtype=np.float32)


def tan_half() -> np.float32:
    """tan of the 10 degree sector half-angle, as FP32."""
    return np.float32(math.tan(math.radians(10.0)))


class _Cfg(ctypes.Structure):
    _fields_ = [
        ("seed", ctypes.c_uint64),
        ("n_collisions", ctypes.c_int32),
        ("mult_mode", ctypes.c_int32),
        ("mult_fixed", ctypes.c_int32),
        ("mult_cap", ctypes.c_int32),
        ("mult_mean", ctypes.c_double),
        ("pt_mode", ctypes.c_int32),
        ("pt_lo", ctypes.c_double),
        ("pt_hi", ctypes.c_double),
        ("pt_mean", ctypes.c_double),
        ("pt_floor", ctypes.c_double),
        ("eta_max", ctypes.c_double),
        ("eta_one_side", ctypes.c_int32),
        ("phi_mode", ctypes.c_int32),
        ("phi_inset_deg", ctypes.c_double),
        ("sec_frac", ctypes.c_double),
        ("sec_rmax", ctypes.c_double),
        ("only_sector", ctypes.c_int32),
        ("sigma_y", ctypes.c_double),
        ("sigma_z", ctypes.c_double),
        ("eff", ctypes.c_double),
        ("noise_frac", ctypes.c_double),
        ("bz", ctypes.c_double),
        ("max_turns", ctypes.c_double),
        ("z_len", ctypes.c_double),
        ("t_frame_us", ctypes.c_double),
        ("v_drift", ctypes.c_double),
        ("order", ctypes.c_int32),
        ("want_exact", ctypes.c_int32),
        ("n_threads", ctypes.c_int32),
        ("n_rows", ctypes.c_int32),
        ("row_x", ctypes.POINTER(ctypes.c_float)),
        ("tan_half", ctypes.c_float),
    ]


class _Out(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int64),
        ("y", ctypes.POINTER(ctypes.c_float)),
        ("z", ctypes.POINTER(ctypes.c_float)),
        ("row", ctypes.POINTER(ctypes.c_uint8)),
        ("sector", ctypes.POINTER(ctypes.c_uint8)),
        ("particle", ctypes.POINTER(ctypes.c_int32)),
        ("leg", ctypes.POINTER(ctypes.c_int32)),
        ("crossing", ctypes.POINTER(ctypes.c_int32)),
        ("collision", ctypes.POINTER(ctypes.c_int32)),
        ("y_true", ctypes.POINTER(ctypes.c_double)),
        ("z_true", ctypes.POINTER(ctypes.c_double)),
        ("phi_loc", ctypes.POINTER(ctypes.c_double)),
        ("dzds", ctypes.POINTER(ctypes.c_double)),
        ("qpt", ctypes.POINTER(ctypes.c_double)),
        ("n_signal", ctypes.c_int64),
        ("n_noise", ctypes.c_int64),
        ("n_particles", ctypes.c_int64),
        ("n_legs", ctypes.c_int64),
    ]


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        lib = ctypes.CDLL(_LIB_PATH)
        lib.synth_generate.argtypes = [ctypes.POINTER(_Cfg), ctypes.POINTER(_Out)]
        lib.synth_generate.restype = ctypes.c_int
        lib.synth_free.argtypes = [ctypes.POINTER(_Out)]
        lib.synth_free.restype = None
        _lib = lib
    return _lib


def build() -> None:
    """Compile the generator (plain C, gcc)."""
    import subprocess

    src = os.path.join(_HERE, "tpcsynth.c")
    tmp = _LIB_PATH + ".tmp"
    subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", "-o", tmp, src, "-lm", "-lpthread"])
    os.replace(tmp, _LIB_PATH)


@dataclass(frozen=True)
class Workload:
    """One synthetic workload.  Field meanings follow ``synth_cfg_t`` in tpcsynth.c."""

    name: str
    seed: int
    n_collisions: int = 1
    mult_mode: int = 0
    mult_fixed: int = 200
    mult_cap: int = 0
    mult_mean: float = 0.0
    pt_mode: int = 0
    pt_lo: float = 0.1
    pt_hi: float = 10.0
    pt_mean: float = 0.5
    pt_floor: float = 0.05
    eta_max: float = 0.9
    eta_one_side: int = 0
    phi_mode: int = 1
    phi_inset_deg: float = 0.0
    sec_frac: float = 0.0
    sec_rmax: float = 50.0
    only_sector: int = -1
    sigma_y: float = 0.06
    sigma_z: float = 0.1
    eff: float = 0.9
    noise_frac: float = 0.05
    bz: float = BZ
    max_turns: float = 5.0
    z_len: float = Z_LEN
    t_frame_us: float = 0.0
    v_drift: float = V_DRIFT
    order: int = 0

    @property
    def z_max(self) -> float:
        """Upper end of the z range the tracker must cover (time frames extend it)."""
        return self.z_len + (self.v_drift * self.t_frame_us if self.t_frame_us > 0 else 0.0)


# The five workloads.  Seeds are fixed; events of the learned-scorer study use seeds
# 1..200 (training), 201..210 (threshold choice) and 1001..1020 (held-out test).
SECTOR_EVENT = Workload(  # one sector, 200 helices from the origin, log-uniform pT
    name="sector_event_200", seed=0xC0F1, mult_fixed=200, pt_mode=0, phi_mode=0, eta_one_side=1,
    only_sector=0, noise_frac=0.05)
PBPB_EVENT = Workload(  # full TPC, central Pb-Pb-like: 5000 primaries + 10% displaced secondaries
    name="pbpb_event_5000", seed=0xC0F2, mult_fixed=5000, pt_mode=1, pt_mean=0.5, pt_floor=0.05,
    phi_mode=1, sec_frac=0.1, noise_frac=0.05)
PBPB_TIMEFRAME = Workload(  # 570 collisions over 11.4 ms (50 kHz), multiplicity Exp(700) capped at 5000
    name="pbpb_timeframe_570", seed=0xC0F3, n_collisions=570, mult_mode=1, mult_mean=700.0,
    mult_cap=5000, pt_mode=1, phi_mode=1, sec_frac=0.1, noise_frac=0.05, t_frame_us=11400.0)
PP_TIMEFRAME = Workload(  # 11400 pp collisions at 1 MHz, multiplicity Poisson(12), 10% noise
    name="pp_timeframe_11400", seed=0xC0F5, n_collisions=11400, mult_mode=2, mult_mean=12.0,
    pt_mode=1, phi_mode=1, sec_frac=0.0, noise_frac=0.10, t_frame_us=11400.0)

WORKLOADS = {w.name: w for w in (SECTOR_EVENT, PBPB_EVENT, PBPB_TIMEFRAME, PP_TIMEFRAME)}


def sector_event(seed: int) -> Workload:
    """A one-sector, 200-helix event with the given seed (learned-scorer training/validation/test)."""
    return replace(SECTOR_EVENT, name=f"sector_event_200_s{seed}", seed=seed)


def scaled(w: Workload, frac: float, name: str | None = None) -> Workload:
    """The same workload with fewer collisions (time frames) or particles (events)."""
    if w.n_collisions > 1:
        return replace(w, name=name or f"{w.name}_x{frac:g}", n_collisions=max(1, int(round(w.n_collisions * frac))),
                       t_frame_us=w.t_frame_us * frac)
    return replace(w, name=name or f"{w.name}_x{frac:g}", mult_fixed=max(1, int(round(w.mult_fixed * frac))))


@dataclass
class Event:
    workload: Workload
    y: np.ndarray
    z: np.ndarray
    row: np.ndarray
    sector: np.ndarray
    particle: np.ndarray
    leg: np.ndarray
    crossing: np.ndarray
    collision: np.ndarray
    n_signal: int
    n_noise: int
    n_particles: int
    n_legs: int
    exact: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.y.shape[0])

    def sha256(self) -> str:
        h = hashlib.sha256()
        for a in (self.y, self.z, self.row, self.sector):
            h.update(np.ascontiguousarray(a).tobytes())
        return h.hexdigest()


def generate(w: Workload, want_exact: bool = False, n_threads: int | None = None) -> Event:
    """Generate one workload.  Output is independent of ``n_threads``."""
    lib = _load()
    rx = row_x()
    cfg = _Cfg()
    for f, _ in _Cfg._fields_:
        if hasattr(w, f):
            setattr(cfg, f, getattr(w, f))
    cfg.seed = w.seed
    cfg.want_exact = 1 if want_exact else 0
    cfg.n_threads = n_threads or min(16, os.cpu_count() or 1)
    cfg.n_rows = N_ROWS
    cfg.row_x = rx.ctypes.data_as(ctypes.POINTER(ctypes.c_float))
    cfg.tan_half = float(tan_half())
    out = _Out()
    rc = lib.synth_generate(ctypes.byref(cfg), ctypes.byref(out))
    if rc != 0:
        raise RuntimeError(f"synth_generate failed ({rc})")
    n = out.n

    def arr(p, dt):
        if n == 0 or not p:
            return np.zeros(0, dtype=dt)
        return np.ctypeslib.as_array(p, shape=(n,)).astype(dt, copy=True)

    ev = Event(
        workload=w,
        y=arr(out.y, np.float32), z=arr(out.z, np.float32),
        row=arr(out.row, np.uint8), sector=arr(out.sector, np.uint8),
        particle=arr(out.particle, np.int32), leg=arr(out.leg, np.int32),
        crossing=arr(out.crossing, np.int32), collision=arr(out.collision, np.int32),
        n_signal=int(out.n_signal), n_noise=int(out.n_noise),
        n_particles=int(out.n_particles), n_legs=int(out.n_legs),
    )
    if want_exact:
        ev.exact = {k: arr(getattr(out, k), np.float64) for k in ("y_true", "z_true", "phi_loc", "dzds", "qpt")}
    lib.synth_free(ctypes.byref(out))
    return ev


def cluster_properties(ev: Event, seed: int = 0x51CE) -> tuple[np.ndarray, np.ndarray, np.ndarray]:
    """Seeded synthetic charge and widths of every cluster (the generator's clusters carry only
    positions): total charge in ADC counts (uint16), log-normal around 120 for track clusters and
    40 for noise, and the widths along y and z in units of 1/64 cm (uint8), around 0.20 cm and
    0.30 cm, the z width growing with the drift distance 250 - (z mod 250) as diffusion does.
    Independent of the positions' random stream."""
    rng = np.random.Generator(np.random.PCG64([seed, ev.workload.seed, ev.n]))
    n = ev.n
    noise = ev.particle < 0
    mu = np.where(noise, np.log(40.0), np.log(120.0))
    q = np.exp(mu + 0.4 * rng.standard_normal(n))
    qtot = np.clip(np.rint(q), 1, 65535).astype(np.uint16)
    drift = 250.0 - np.mod(ev.z.astype(np.float64), 250.0)
    sy = 0.20 * np.exp(0.15 * rng.standard_normal(n))
    sz = np.sqrt(0.25 ** 2 + (0.0012 * drift)) * np.exp(0.15 * rng.standard_normal(n))
    sig_y = np.clip(np.rint(sy * 64.0), 1, 255).astype(np.uint8)
    sig_z = np.clip(np.rint(sz * 64.0), 1, 255).astype(np.uint8)
    return qtot, sig_y, sig_z


def uniform01(seed: int, n: int) -> np.ndarray:
    """Seeded uniform draws in [0, 1) for host-side sampling decisions (subsampling, batch order,
    initial weights).  numpy's PCG64 is used: these draws never reach a kernel except as inputs."""
    return np.random.Generator(np.random.PCG64(seed)).random(n)


def permutation(seed: int, n: int) -> np.ndarray:
    return np.random.Generator(np.random.PCG64(seed)).permutation(n)


# Tracker settings the workloads are run with (cuts, errors, initial covariance, grid bins).
# They are configuration handed to both the oracle and the HIP library, not arithmetic.
TRACKER_PARAMS = dict(
    win_y=2.0, win_z=2.0,          # neighbour window: |dy|, |dz| <= 2.0 * row pitch
    nb_chi2_max=13.8,              # straight-line triplet criterion cut (2 dof, p ~ 1e-3)
    fol_chi2_max=13.8,             # following / link acceptance chi2 cut (2 dof)
    sigma_y=0.06, sigma_z=0.1,     # cluster errors, cm
    s_max=0.999,                   # |sin phi| limit of the propagation
    edge_margin=2.0,               # stop when |y| > x tan(10 deg) + 2 cm
    l_min_chain=3, n_miss_max=10, n_min_tracklet=10, n_min_track=10,
    c0_sinphi=1.0, c0_dzds=1.0, c0_qpt=100.0,
    bin_y=8.0, bin_z=8.0,          # grid bins (cm); results do not depend on them
)


def geometry(w: Workload) -> dict:
    return dict(n_rows=N_ROWS, row_x=row_x(), tan_half=tan_half(), n_sectors=N_SECTORS,
                z_min=0.0, z_max=w.z_max)
