"""The plain-C host code (the FP64 oracle and the input generator) under AddressSanitizer and
UndefinedBehaviorSanitizer.

Both libraries are rebuilt with ``-fsanitize=address,undefined`` into a temporary folder and
driven from a child Python process that preloads the ASan runtime: a one-sector event and a slice
of a Pb-Pb event are generated and tracked (neighbours, tracklets, selection, cluster flags, the
scorer logit), and the outputs must equal those of the regular builds.  Any sanitizer report
aborts the child (``halt_on_error``), which fails the test.  CPU only.
"""
import json
import os
import shutil
import subprocess
import sys
import tempfile

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

CHILD = r'''
import json, sys
import numpy as np
sys.path.insert(0, sys.argv[1])
import synth, oracle
synth._LIB_PATH = sys.argv[2]
oracle._libs[oracle._LIB_PATH] = oracle._load(sys.argv[3])
oracle._libs[oracle._LIB_FMA_PATH] = oracle._load(sys.argv[4])
from tests.test_sanitizers import workload_digest
print("DIGEST " + json.dumps(workload_digest()), flush=True)
'''


def workload_digest() -> dict:
    """Generate two small workloads and run the oracle's steps on them; return checksums."""
    import oracle
    import synth

    out = {}
    for w in (synth.SECTOR_EVENT, synth.scaled(synth.PBPB_EVENT, 0.02)):
        ev = synth.generate(w, want_exact=True)
        geom = synth.geometry(w)
        o = oracle.track(ev.y, ev.z, ev.row, ev.sector, geom, synth.TRACKER_PARAMS, synth.BZ, n_threads=2)
        trk = oracle.tracks_for_flags(o, geom, ev.sector)
        fl, tie = oracle.cluster_flags(ev.y, ev.z, ev.row, ev.sector, geom, synth.BZ, trk)
        d = {"n": int(ev.n), "y": float(np.sum(ev.y, dtype=np.float64)), "leg": int(ev.leg.astype(np.int64).sum()),
             "qpt": float(np.nansum(ev.exact["qpt"]))}
        for k in ("up", "dn", "start_id", "trk_hits", "hit_key"):
            d[k] = int(np.asarray(o[k]).astype(np.int64).sum())
        d["tl_state"] = float(np.nansum(np.asarray(o["tl_state"], dtype=np.float64)))
        d["flags"] = int(fl.astype(np.int64).sum())
        d["tie"] = int(np.asarray(tie).astype(np.int64).sum())
        out[w.name] = d
    rng = np.random.default_rng(5)
    theta = rng.normal(0, 0.3, oracle.N_MLP_PARAMS)
    x = rng.normal(0, 1, 12)
    out["logit"] = float(oracle.mlp_logit(theta, x))
    return out


def _asan_runtime():
    try:
        p = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True).stdout.strip()
    except OSError:
        return None
    return p if p and os.path.isabs(p) and os.path.exists(p) else None


@pytest.mark.skipif(shutil.which("gcc") is None or _asan_runtime() is None, reason="gcc with ASan runtime needed")
def test_oracle_and_generator_are_clean_under_asan_and_ubsan():
    import oracle
    import synth

    tmp = tempfile.mkdtemp(prefix="tpc_san_")
    try:
        san = ["gcc", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
               "-fno-omit-frame-pointer", "-fno-fast-math", "-fPIC", "-shared"]
        libs = {}
        osrc = [os.path.join(ROOT, "oracle", "tpc_oracle.c"), os.path.join(ROOT, "oracle", "tpc_codec.c")]
        for name, src, extra in (("synth", [os.path.join(ROOT, "synth", "tpcsynth.c")], []),
                                 ("oracle", osrc, ["-ffp-contract=off"]),
                                 ("oracle_fma", osrc, ["-ffp-contract=fast", "-mfma"])):
            libs[name] = os.path.join(tmp, f"lib{name}_san.so")
            subprocess.check_call(san + extra + ["-o", libs[name], *src, "-lm", "-lpthread"])
        env = dict(os.environ)
        env["LD_PRELOAD"] = _asan_runtime()
        env["ASAN_OPTIONS"] = "detect_leaks=0:halt_on_error=1:abort_on_error=1"
        env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1"
        env["PYTHONPATH"] = ROOT
        r = subprocess.run([sys.executable, "-c", CHILD, ROOT, libs["synth"], libs["oracle"], libs["oracle_fma"]],
                           capture_output=True, text=True, env=env, timeout=600)
        assert r.returncode == 0, f"sanitized run failed ({r.returncode}):\n{r.stdout[-3000:]}\n{r.stderr[-6000:]}"
        assert "ERROR: AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr, r.stderr[-4000:]
        line = [ln for ln in r.stdout.splitlines() if ln.startswith("DIGEST ")]
        assert line, r.stdout[-2000:]
        got = json.loads(line[-1][len("DIGEST "):])
        want = json.loads(json.dumps(workload_digest()))
        assert got == want
    finally:
        shutil.rmtree(tmp, ignore_errors=True)
    del oracle, synth
