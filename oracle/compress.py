"""CPU oracle of the TPC cluster compression (TEST INFRASTRUCTURE ONLY).

Sec. 4 of arXiv:1910.12214 (TPC data reduction), steps 2-4, written from the readings below;
the integer and codec parts are in ``tpc_codec.c`` (plain C), the rest is numpy.  Only
``tests/`` may use it.

Readings (the paper gives the steps, not their constants):
* Step 2.  Positions become integers in quanta of sigma/8 of the cluster resolution
  (Q_Y = 0.0075 cm, Q_Z = 0.0125 cm): yq = rint(y * (1 / Q_Y)) in FP64 from the FP32 coordinate,
  ties to even, the same for z.  Clusters with row or sector out of range, or |yq| or |zq| >= 2^29
  (differences must fit 31 bits), are skipped and counted.  Charge and the two widths keep the leading one and the n bits
  after it, rounded (n = 4 for the charge, 3 for the widths); stored as (e << (n+1)) | (v >> e).
* Step 3.  A track's clusters (the tracker's hit lists, ascending rows) are stored as the row
  step from the previous hit (from the track's reference row for the first) and the residuals of
  the quantised position to the quantised prediction, the track's reference state carried along
  the helix to the hit's row in one closed-form step (FP64 from the FP32 state); where that step
  fails the previous hit's position is the prediction.  Every other cluster is stored per
  (sector, row), in ascending (zq, yq, cluster id), as the number of such clusters of the row and,
  per cluster, the differences of zq (>= 0) and yq to the previous one (to 0 for the first).
  Charges and widths follow the cluster order of the streams (track clusters first).
* Step 4.  Each stream is a sequence of symbols < 4096 (signed values zigzag-mapped; values >=
  4095 become the escape symbol 4095 with the value kept raw) coded by range ANS (31-bit state,
  byte output, 14-bit probabilities) in blocks of 4096 symbols; Huffman coding of the same
  symbols is the comparison.
"""
from __future__ import annotations

import ctypes
import math

import numpy as np

Q_Y, Q_Z = 0.0075, 0.0125
INV_QY, INV_QZ = 1.0 / Q_Y, 1.0 / Q_Z
N_CHARGE, N_WIDTH = 4, 3
ALPHABET, ESC = 4096, 4095
PROB_BITS, BLOCK = 14, 4096
STREAMS = ("a_drow", "a_ry", "a_rz", "u_n", "u_dz", "u_dy", "q", "sy", "sz")
TIE_ABS = 1e-6  # a prediction within this many quanta of a rounding boundary is flagged
Q_LIMIT = 2.0 ** 29  # clusters (and predictions) at |yq| or |zq| >= 2^29 are not representable

_lib = None


def _codec():
    global _lib
    if _lib is None:
        from oracle import _LIB_PATH, _load

        lib = _load(_LIB_PATH)
        u32p, u16p, dp = (ctypes.POINTER(ctypes.c_uint32), ctypes.POINTER(ctypes.c_uint16),
                          ctypes.POINTER(ctypes.c_double))
        lib.or_dynprec.argtypes = [ctypes.c_uint32, ctypes.c_int]
        lib.or_dynprec.restype = ctypes.c_uint32
        lib.or_dynprec_code.argtypes = [ctypes.c_uint32, ctypes.c_int]
        lib.or_dynprec_code.restype = ctypes.c_uint32
        lib.or_dynprec_decode.argtypes = [ctypes.c_uint32, ctypes.c_int]
        lib.or_dynprec_decode.restype = ctypes.c_uint32
        lib.or_predict.argtypes = [ctypes.c_int64, dp, dp, dp, ctypes.c_double, ctypes.c_double, dp, dp,
                                   ctypes.POINTER(ctypes.c_int32)]
        lib.or_predict.restype = None
        lib.or_ans_freqs.argtypes = [u32p, ctypes.c_int, ctypes.c_int, u32p]
        lib.or_ans_freqs.restype = ctypes.c_int
        u8p = ctypes.POINTER(ctypes.c_uint8)
        lib.or_ans_encode_block.argtypes = [u16p, ctypes.c_int64, u32p, u32p, ctypes.c_int, u8p]
        lib.or_ans_encode_block.restype = ctypes.c_int64
        lib.or_ans_decode_block.argtypes = [u8p, ctypes.c_int64, ctypes.c_int64, u32p, u32p, u16p, ctypes.c_int,
                                            u16p]
        lib.or_ans_decode_block.restype = ctypes.c_int64
        lib.or_huffman_lengths.argtypes = [u32p, ctypes.c_int, ctypes.POINTER(ctypes.c_uint8)]
        lib.or_huffman_lengths.restype = ctypes.c_uint64
        _lib = lib
    return _lib


def _p(a, t):
    return a.ctypes.data_as(ctypes.POINTER(t))


# ---------------------------------------------------------------- step 2
def dynprec(v: int, n: int) -> int:
    return int(_codec().or_dynprec(int(v), n))


def dynprec_code(v: int, n: int) -> int:
    return int(_codec().or_dynprec_code(int(v), n))


def dynprec_decode(code: int, n: int) -> int:
    return int(_codec().or_dynprec_decode(int(code), n))


def dynprec_codes(values, n: int) -> np.ndarray:
    lib = _codec()
    return np.array([lib.or_dynprec_code(lib.or_dynprec(int(v), n), n) for v in np.asarray(values)], dtype=np.int64)


def quantise(v, inv_q: float) -> np.ndarray:
    return np.rint(np.asarray(v, dtype=np.float32).astype(np.float64) * inv_q).astype(np.int64)


def zigzag(v) -> np.ndarray:
    v = np.asarray(v, dtype=np.int64)
    return np.where(v >= 0, 2 * v, -2 * v - 1)


def unzigzag(u) -> np.ndarray:
    u = np.asarray(u, dtype=np.int64)
    return np.where(u % 2 == 0, u // 2, -(u + 1) // 2)


# ---------------------------------------------------------------- step 3
def predict(states, x_ref, x_row, bz: float, s_max: float = 0.999):
    """Closed-form helix prediction (y, z, failed) for each (state, x_ref, x_row)."""
    from oracle import KQ_PER_TESLA

    n = len(x_row)
    st = np.ascontiguousarray(states, dtype=np.float64).reshape(n, 5)
    xr = np.ascontiguousarray(x_ref, dtype=np.float64)
    xw = np.ascontiguousarray(x_row, dtype=np.float64)
    yo, zo, fl = np.zeros(n), np.zeros(n), np.zeros(n, dtype=np.int32)
    if n:
        _codec().or_predict(n, _p(st, ctypes.c_double), _p(xr, ctypes.c_double), _p(xw, ctypes.c_double),
                            KQ_PER_TESLA * bz, s_max, _p(yo, ctypes.c_double), _p(zo, ctypes.c_double),
                            _p(fl, ctypes.c_int32))
    return yo, zo, fl.astype(bool)


def _to_symbols(values):
    """Symbols < 4096 of non-negative values, escapes for the rest."""
    v = np.asarray(values, dtype=np.int64)
    sym = np.where(v >= ESC, ESC, v).astype(np.uint16)
    return sym, v[v >= ESC].astype(np.uint32)


def compress(y, z, row, sector, qtot, sig_y, sig_z, geometry: dict, bz: float, tracks: dict,
             s_max: float = 0.999) -> dict:
    """Symbol streams of the clusters.  ``tracks``: hit_offset, n_hits, hit_ids (ascending rows),
    sector, row_ref, x_ref, state (the tracker's output).  Returns streams (uint16 symbols),
    escapes, the cluster order, the flagged (near-tie) positions of the track streams, counts."""
    R, S = int(geometry["n_rows"]), int(geometry["n_sectors"])
    row_x = np.asarray(geometry["row_x"], dtype=np.float32)
    row = np.asarray(row, dtype=np.int64)
    sector = np.asarray(sector, dtype=np.int64)
    n = len(row)
    with np.errstate(invalid="ignore"):
        fy = np.rint(np.asarray(y, dtype=np.float32).astype(np.float64) * INV_QY)
        fz = np.rint(np.asarray(z, dtype=np.float32).astype(np.float64) * INV_QZ)
        valid = (row < R) & (sector < S) & (np.abs(fy) < Q_LIMIT) & (np.abs(fz) < Q_LIMIT)
    yq = np.where(valid, fy, 0).astype(np.int64)
    zq = np.where(valid, fz, 0).astype(np.int64)
    # clusters on tracks, in track order; a track with an unusable entry (offset beyond the hit
    # list, id out of range or of a skipped cluster, sector or reference row out of range) is
    # left out and its clusters count as others
    off = np.asarray(tracks["hit_offset"], dtype=np.int64)
    nh = np.asarray(tracks["n_hits"], dtype=np.int64).copy()
    hid = np.asarray(tracks["hit_ids"], dtype=np.int64)
    for k in range(len(nh)):
        ok = off[k] >= 0 and nh[k] >= 0 and off[k] + nh[k] <= len(hid) and 0 <= tracks["sector"][k] < S and \
            0 <= tracks["row_ref"][k] < R
        if ok:
            ids = hid[off[k]:off[k] + nh[k]]
            ok = bool(np.all((ids >= 0) & (ids < n))) and bool(np.all(valid[np.clip(ids, 0, max(n - 1, 0))]))
        if not ok:
            nh[k] = 0
    n_trk = len(nh)
    t_of = np.repeat(np.arange(n_trk), nh)
    a_ids = np.concatenate([hid[off[k]:off[k] + nh[k]] for k in range(n_trk)]) if n_trk else np.zeros(0, np.int64)
    first = np.zeros(len(a_ids), dtype=bool)
    if n_trk:
        first[np.concatenate([[0], np.cumsum(nh)[:-1]])[nh > 0]] = True
    st = np.asarray(tracks["state"], dtype=np.float32).reshape(-1, 5)[t_of].astype(np.float64)
    xref = np.asarray(tracks["x_ref"], dtype=np.float32)[t_of].astype(np.float64)
    rref = np.asarray(tracks["row_ref"], dtype=np.int64)[t_of]
    a_row = row[a_ids]
    yp, zp, fail = predict(st, xref, row_x[a_row].astype(np.float64), bz, s_max)
    with np.errstate(invalid="ignore"):
        fail |= ~(np.abs(np.rint(yp * INV_QY)) < Q_LIMIT) | ~(np.abs(np.rint(zp * INV_QZ)) < Q_LIMIT)
    yp, zp = np.where(fail, 0.0, yp), np.where(fail, 0.0, zp)
    py, pz = np.rint(yp * INV_QY).astype(np.int64), np.rint(zp * INV_QZ).astype(np.int64)
    tie = (np.abs(np.abs(yp * INV_QY - np.floor(yp * INV_QY)) - 0.5) < TIE_ABS) | \
          (np.abs(np.abs(zp * INV_QZ - np.floor(zp * INV_QZ)) - 0.5) < TIE_ABS)
    prev_row = np.where(first, rref, np.concatenate([[0], a_row[:-1]]))
    prev_yq = np.where(first, 0, np.concatenate([[0], yq[a_ids][:-1]]))
    prev_zq = np.where(first, 0, np.concatenate([[0], zq[a_ids][:-1]]))
    py = np.where(fail, prev_yq, py)
    pz = np.where(fail, prev_zq, pz)
    tie &= ~fail
    a_drow = zigzag(a_row - prev_row)
    a_ry, a_rz = zigzag(yq[a_ids] - py), zigzag(zq[a_ids] - pz)
    # the other clusters, per (sector, row) in ascending (zq, yq, id)
    on_track = np.zeros(n, dtype=bool)
    on_track[a_ids] = True
    u_ids = np.nonzero(valid & ~on_track)[0]
    rs = sector[u_ids] * R + row[u_ids]
    u_ids = u_ids[np.lexsort((u_ids, yq[u_ids], zq[u_ids], rs))]
    rs = sector[u_ids] * R + row[u_ids]
    u_n = np.bincount(rs, minlength=S * R)
    newrow = np.ones(len(u_ids), dtype=bool)
    newrow[1:] = rs[1:] != rs[:-1]
    uz, uy = zq[u_ids], yq[u_ids]
    u_dz = uz - np.where(newrow, 0, np.concatenate([[0], uz[:-1]]))
    u_dy = zigzag(uy - np.where(newrow, 0, np.concatenate([[0], uy[:-1]])))
    u_dz = np.where(newrow, zigzag(uz), u_dz)  # the first of a row may lie below zero
    order = np.concatenate([a_ids, u_ids])
    vals = {"a_drow": a_drow, "a_ry": a_ry, "a_rz": a_rz, "u_n": u_n, "u_dz": u_dz, "u_dy": u_dy,
            "q": dynprec_codes(np.asarray(qtot)[order], N_CHARGE),
            "sy": dynprec_codes(np.asarray(sig_y)[order], N_WIDTH),
            "sz": dynprec_codes(np.asarray(sig_z)[order], N_WIDTH)}
    streams, escapes = {}, {}
    for k in STREAMS:
        streams[k], escapes[k] = _to_symbols(vals[k])
    return {"streams": streams, "escapes": escapes, "order": order, "n_attached": len(a_ids), "track_len": nh,
            "n_unattached": len(u_ids), "n_skipped": int((~valid).sum()), "tie": np.nonzero(tie)[0],
            "pred_fail": int(fail.sum()), "yq": yq, "zq": zq}


def decompress(streams: dict, escapes: dict, tracks: dict, geometry: dict, bz: float, s_max: float = 0.999):
    """Quantised clusters (sector, row, yq, zq, charge, width_y, width_z) in stream order."""
    R, S = int(geometry["n_rows"]), int(geometry["n_sectors"])
    row_x = np.asarray(geometry["row_x"], dtype=np.float32)

    def values(k):
        s = np.asarray(streams[k], dtype=np.int64).copy()
        s[s == ESC] = np.asarray(escapes[k], dtype=np.int64)
        return s

    nh = np.asarray(tracks.get("track_len", tracks["n_hits"]), dtype=np.int64)
    drow, ry, rz = unzigzag(values("a_drow")), unzigzag(values("a_ry")), unzigzag(values("a_rz"))
    st = np.asarray(tracks["state"], dtype=np.float32).reshape(-1, 5)
    out_s, out_r, out_y, out_z = [], [], [], []
    i = 0
    for k in range(len(nh)):
        r = int(tracks["row_ref"][k])
        py = pz = 0
        for j in range(int(nh[k])):
            r = r + int(drow[i])
            yp, zp, fl = predict(st[k:k + 1].astype(np.float64), [float(np.float32(tracks["x_ref"][k]))],
                                 [float(row_x[min(max(r, 0), R - 1)])], bz, s_max)
            with np.errstate(invalid="ignore"):
                fl = fl | ~(np.abs(np.rint(yp * INV_QY)) < Q_LIMIT) | ~(np.abs(np.rint(zp * INV_QZ)) < Q_LIMIT)
            if not fl[0]:
                py, pz = int(np.rint(yp[0] * INV_QY)), int(np.rint(zp[0] * INV_QZ))
            yq, zq = py + int(ry[i]), pz + int(rz[i])
            out_s.append(int(tracks["sector"][k]))
            out_r.append(r)
            out_y.append(yq)
            out_z.append(zq)
            py, pz = yq, zq
            i += 1
    u_n, u_dz, u_dy = values("u_n"), values("u_dz"), unzigzag(values("u_dy"))
    i = 0
    for rs in range(S * R):
        zq = yq = 0
        for j in range(int(u_n[rs])):
            zq = int(unzigzag(u_dz[i])) if j == 0 else zq + int(u_dz[i])
            yq = yq + int(u_dy[i])
            out_s.append(rs // R)
            out_r.append(rs % R)
            out_y.append(yq)
            out_z.append(zq)
            i += 1
    q = [dynprec_decode(c, N_CHARGE) for c in values("q")]
    sy = [dynprec_decode(c, N_WIDTH) for c in values("sy")]
    sz = [dynprec_decode(c, N_WIDTH) for c in values("sz")]
    return {"sector": np.array(out_s), "row": np.array(out_r), "yq": np.array(out_y), "zq": np.array(out_z),
            "q": np.array(q), "sy": np.array(sy), "sz": np.array(sz)}


# ---------------------------------------------------------------- step 4
def ans_freqs(count) -> np.ndarray:
    c = np.ascontiguousarray(count, dtype=np.uint32)
    f = np.zeros(len(c), dtype=np.uint32)
    rc = _codec().or_ans_freqs(_p(c, ctypes.c_uint32), len(c), PROB_BITS, _p(f, ctypes.c_uint32))
    assert rc >= 0
    return f


def ans_encode(syms, freq=None):
    """Range-ANS blocks of one stream: (freq, bytes uint8, bytes per block)."""
    syms = np.ascontiguousarray(syms, dtype=np.uint16)
    if freq is None:
        freq = ans_freqs(np.bincount(syms, minlength=ALPHABET))
    freq = np.ascontiguousarray(freq, dtype=np.uint32)
    cum = np.ascontiguousarray(np.concatenate([[0], np.cumsum(freq)[:-1]]).astype(np.uint32))
    lib = _codec()
    out, per = [], []
    buf = np.zeros(2 * BLOCK + 4, dtype=np.uint8)
    for b0 in range(0, len(syms), BLOCK):
        blk = np.ascontiguousarray(syms[b0:b0 + BLOCK])
        w = lib.or_ans_encode_block(_p(blk, ctypes.c_uint16), len(blk), _p(freq, ctypes.c_uint32),
                                    _p(cum, ctypes.c_uint32), PROB_BITS, _p(buf, ctypes.c_uint8))
        out.append(buf[:w].copy())
        per.append(w)
    return freq, (np.concatenate(out) if out else np.zeros(0, np.uint8)), np.array(per, dtype=np.int64)


def ans_decode(data, per_block, n: int, freq) -> np.ndarray:
    freq = np.ascontiguousarray(freq, dtype=np.uint32)
    cum = np.ascontiguousarray(np.concatenate([[0], np.cumsum(freq)[:-1]]).astype(np.uint32))
    slot = np.ascontiguousarray(np.repeat(np.arange(len(freq)), freq).astype(np.uint16))
    lib = _codec()
    out = np.zeros(n, dtype=np.uint16)
    pos = 0
    for b, w in enumerate(per_block):
        m = min(BLOCK, n - b * BLOCK)
        blk = np.ascontiguousarray(data[pos:pos + w])
        o = np.zeros(m, dtype=np.uint16)
        r = lib.or_ans_decode_block(_p(blk, ctypes.c_uint8), int(w), m, _p(freq, ctypes.c_uint32),
                                    _p(cum, ctypes.c_uint32), _p(slot, ctypes.c_uint16), PROB_BITS,
                                    _p(o, ctypes.c_uint16))
        assert r == w, (r, w)
        out[b * BLOCK:b * BLOCK + m] = o
        pos += w
    return out


def huffman_bits(count) -> tuple[int, np.ndarray]:
    c = np.ascontiguousarray(count, dtype=np.uint32)
    ln = np.zeros(len(c), dtype=np.uint8)
    bits = _codec().or_huffman_lengths(_p(c, ctypes.c_uint32), len(c), _p(ln, ctypes.c_uint8))
    return int(bits), ln


def entropy_bits(count) -> float:
    c = np.asarray(count, dtype=np.float64)
    t = c.sum()
    c = c[c > 0]
    return float(-(c * np.log2(c / t)).sum()) if t else 0.0


def ideal_ans_bits(syms, freq) -> float:
    """Sum over the symbols of log2(2^P / f): the length range ANS reaches up to its flush."""
    f = np.asarray(freq, dtype=np.float64)[np.asarray(syms, dtype=np.int64)]
    return float(np.sum(PROB_BITS - np.log2(f)))


def code_lengths_are_prefix_free(ln) -> bool:
    ln = np.asarray(ln, dtype=np.int64)
    ln = ln[ln > 0]
    return len(ln) == 1 or math.isclose(float(np.sum(2.0 ** -ln)), 1.0)
