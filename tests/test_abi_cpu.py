"""Host-side checks of the C ABI: the library loads, exports every symbol the
header declares, and rejects invalid problems before touching a device."""
import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

from paper_1312_4698_amd import inputs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _lib():
    from paper_1312_4698_amd import scivr as S
    return S, S.load()


def test_header_declarations_are_all_exported():
    S, _ = _lib()
    hdr = open(os.path.join(ROOT, "include", "scivr.h")).read()
    declared = set(re.findall(r"\b(scivr_[a-z_]+)\s*\(", hdr))
    out = subprocess.run(["nm", "-D", "--defined-only", S.LIB_PATH], capture_output=True, text=True,
                         check=True).stdout
    exported = {ln.split()[-1] for ln in out.splitlines() if ln.strip()}
    assert declared, "no declarations parsed"
    assert declared <= exported, declared - exported
    assert declared == set(S.EXPORTED)
    assert S.abi_version() == 2


def _create(S, lib, prob, max_traj=16):
    s = S._Problem()
    keep = [np.ascontiguousarray(np.asarray(getattr(prob, nm), dtype=np.float64))
            for nm in ("k_harm", "morse_D", "morse_a", "lam", "gamma", "p_eq", "q_eq")]
    (s.k_harm, s.morse_D, s.morse_a, s.lam, s.gamma, s.p_eq, s.q_eq) = [a.ctypes.data for a in keep]
    s.F = prob.F
    s.dt = prob.dt
    s.n_steps = prob.n_steps
    s.e_min = prob.e_min
    s.e_max = prob.e_max
    s.n_energies = prob.n_energies
    s.det_tol = prob.det_tol
    s.check_every = prob.check_every
    s.precision = prob.precision
    s.max_traj = max_traj
    h = ctypes.c_void_p(12345)
    st = lib.scivr_create(ctypes.byref(s), 0, ctypes.byref(h))
    return st, h, s, keep


@pytest.mark.parametrize("field,value", [
    ("F", 0), ("F", 33), ("n_steps", 0), ("n_energies", 1), ("e_max", -1.0), ("dt", 0.0), ("dt", float("nan")),
    ("check_every", 0), ("det_tol", -1.0), ("precision", 7),
])
def test_create_rejects_invalid_problems(field, value):
    S, lib = _lib()
    prob = inputs.morse_quartic(3, 3)
    prob = prob.replace(**{field: value}) if field != "F" else prob
    if field == "F":
        st, h, s, keep = _create(S, lib, prob)
        s.F = value
        st = lib.scivr_create(ctypes.byref(s), 0, ctypes.byref(h))
    else:
        st, h, _, _ = _create(S, lib, prob)
    assert st == S.EINVAL
    assert h.value is None


def test_create_rejects_nonpositive_width_and_nonfinite_input():
    S, lib = _lib()
    prob = inputs.morse_quartic(3, 3)
    g = prob.gamma.copy()
    g[1] = 0.0
    st, h, _, _ = _create(S, lib, prob.replace(gamma=g))
    assert st == S.EINVAL and h.value is None
    lam = prob.lam.copy()
    lam[0, 2] = np.inf
    st, h, _, _ = _create(S, lib, prob.replace(lam=lam))
    assert st == S.EINVAL and h.value is None
    st, h, _, _ = _create(S, lib, prob, max_traj=0)
    assert st == S.EINVAL


def test_null_arguments_are_rejected():
    S, lib = _lib()
    assert lib.scivr_create(None, 0, ctypes.byref(ctypes.c_void_p())) == S.EINVAL
    assert lib.scivr_propagate(None, 0, 1, None) == S.EINVAL
    assert lib.scivr_accumulate_spectrum(None, None) == S.EINVAL
    assert lib.scivr_accumulate_spectrum_fft(None, None) == S.EINVAL
    assert lib.scivr_accumulate_spectrum_fft_noalloc(None, None) == S.EINVAL
    assert lib.scivr_read_spectrum(None, None, None, None) == S.EINVAL
    lib.scivr_destroy(None)
    assert lib.scivr_last_error(None) == b"null context"


def test_flow_entry_points_reject_null_without_a_device():
    S, lib = _lib()
    h = ctypes.c_void_p(12345)
    assert lib.scivr_flow_create(None, 4, 128, 0, ctypes.byref(h)) == S.EINVAL
    assert lib.scivr_flow_param_count(None) == -1
    lib.scivr_flow_destroy(None)
    d = ctypes.c_double()
    assert lib.scivr_flow_train(None, 1, None, None, None, 0, 1, 1, 1e-3, None, ctypes.byref(d)) == S.EINVAL
    assert lib.scivr_flow_train_on_batch(None, 1, 1, 1e-3, None, None) == S.EINVAL
    assert lib.scivr_flow_loss_grad(None, 1, None, None, None, 0, None, None) == S.EINVAL
    assert lib.scivr_flow_log_density(None, 1, None, None, 0, 0, None, None) == S.EINVAL
    assert lib.scivr_flow_set_params(None, None, 0, 0, None) == S.EINVAL
    assert lib.scivr_flow_get_params(None, None, 0) == S.EINVAL
    assert lib.scivr_flow_sample(None, 0, 0, 1, 0.1, 0.1, None, None, None) == S.EINVAL
