"""The oracle's C code under AddressSanitizer and UndefinedBehaviorSanitizer.

The oracle library is rebuilt with gcc -fsanitize=address,undefined (host
code only: the oracle has no device code) and driven, in a child process
that preloads the ASan runtime, through every entry point of oracle.py on
small problems: sampling, the trajectory run with states, contributions and
amplitudes, the single-trajectory stepper, the determinants, the
double-time form and the monitor probe.  Any sanitizer report, or a
non-zero exit, fails the test.
"""
import os
import subprocess
import sys

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
ORACLE = os.path.join(ROOT, "oracle")
SRCS = [os.path.join(ORACLE, f) for f in ("scivr_oracle.c", "precision_probe.c", "ta_full.c")]

DRIVER = r"""
import numpy as np
from paper_1312_4698_amd import inputs
from oracle import oracle as O
for F, n, ns, K in ((1, 5, 40, 16), (3, 6, 40, 24), (9, 4, 24, 16), (17, 2, 8, 8)):
    prob = inputs.morse_quartic(F, F, n_steps=ns, n_energies=K, e_max=0.1)
    p0, q0, lr = O.sample_husimi(prob, 11, n)
    res = O.run(prob, p0, q0, lr, want_amps=True)
    assert np.all(np.isfinite(res.spectrum)), F
    tr = O.Trajectory(prob, p0[:, 0], q0[:, 0])
    tr.advance(ns // 2)
    assert np.isfinite(tr.state.phi)
    rng = np.random.default_rng(F)
    a = rng.standard_normal((2 * F, 2 * F))
    assert np.isfinite(O.det_real(a))
    c = rng.standard_normal((F, F)) + 1j * rng.standard_normal((F, F))
    assert np.isfinite(O.det_complex(c))
    if F <= 9:
        full = O.run_full(prob, p0, q0, lr, want_lags=True)
        assert np.all(np.isfinite(full.spectrum)), F
    mp = O.monitor_probe(prob, p0[:, 0], q0[:, 0], ns, 4)
    assert np.all(np.isfinite(mp["normM"])), F
print("sanitized oracle driver done")
"""


def _runtime(name):
    p = subprocess.run(["gcc", f"-print-file-name={name}"], capture_output=True, text=True).stdout.strip()
    return p if os.path.isabs(p) and os.path.exists(p) else None


@pytest.mark.skipif(_runtime("libasan.so") is None, reason="no ASan runtime for gcc here")
def test_oracle_under_address_and_undefined_sanitizers(tmp_path):
    lib = str(tmp_path / "libscivr_oracle_san.so")
    cmd = ["gcc", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=undefined", "-fno-fast-math", "-ffp-contract=off", "-fopenmp",
           "-shared", "-fPIC", "-std=gnu11", "-Wall", "-o", lib, *SRCS, "-lquadmath", "-lm"]
    subprocess.run(cmd, check=True, capture_output=True)
    env = dict(os.environ)
    env.update(SCIVR_ORACLE_SO=lib, LD_PRELOAD=_runtime("libasan.so"), OMP_NUM_THREADS="2",
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=0:halt_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1",
               PYTHONPATH=ROOT + os.pathsep + env.get("PYTHONPATH", ""))
    r = subprocess.run([sys.executable, "-c", DRIVER], env=env, capture_output=True, text=True, cwd=ROOT,
                       timeout=600)
    report = r.stdout[-2000:] + r.stderr[-4000:]
    assert r.returncode == 0, report
    assert "AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr, report
    assert "sanitized oracle driver done" in r.stdout, report
