"""The oracle under AddressSanitizer and UndefinedBehaviorSanitizer.

oracle/asan_check.c drives every oracle entry point on one small seeded
problem; here it is compiled with the oracle's sources by gcc with
-fsanitize=address,undefined (host code only: the oracle has no GPU code)
and run.  Any out-of-bounds access, use after free, leak or undefined
operation aborts it with a report."""
import os
import shutil
import subprocess

import numpy as np
import pytest

import synth

ORACLE = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "oracle")
SOURCES = ["bsr.c", "decouple.c", "amg.c", "cpr.c", "ras.c", "thermal.c", "asan_check.c"]


def _write_problem(p, d):
    np.asarray([p.nx, p.ny, p.nz, p.well_cell.shape[0]], np.int32).tofile(os.path.join(d, "dims.i32"))
    np.ascontiguousarray(p.logk, np.float64).tofile(os.path.join(d, "logk.f64"))
    np.asarray([p.kvkh, p.tscale, p.dt], np.float64).tofile(os.path.join(d, "par.f64"))
    np.ascontiguousarray(p.Mf, np.float64).tofile(os.path.join(d, "mf.f64"))
    np.ascontiguousarray(p.Mb, np.float64).tofile(os.path.join(d, "mb.f64"))
    np.ascontiguousarray(p.B, np.float64).tofile(os.path.join(d, "b.f64"))
    np.ascontiguousarray(p.well_cell, np.int32).tofile(os.path.join(d, "wcell.i32"))
    np.ascontiguousarray(p.well_u, np.float64).tofile(os.path.join(d, "wu.f64"))
    np.ascontiguousarray(p.b, np.float64).tofile(os.path.join(d, "rhs.f64"))


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
@pytest.mark.parametrize("dims", [(7, 5, 4), (1, 1, 3), (12, 3, 2)])
def test_oracle_asan(tmp_path, dims):
    exe = str(tmp_path / "asan_check")
    cmd = ["gcc", "-O1", "-g", "-std=c11", "-ffp-contract=off", "-fno-omit-frame-pointer",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
           "-o", exe] + [os.path.join(ORACLE, s) for s in SOURCES] + ["-lm"]
    subprocess.run(cmd, check=True)
    p = synth.small(*dims, seed=41)
    _write_problem(p, str(tmp_path))
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:exitcode=23:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe, str(tmp_path)], capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0 and "asan_check ok" in r.stdout, (r.returncode, r.stdout, r.stderr[-4000:])
