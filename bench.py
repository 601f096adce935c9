"""Benchmark of the TA-SC-IVR power-spectrum hot path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload F9_fp64]

One step is one pass of the whole hot path over one batch of synthetic input:
Husimi sampling of the batch on the GPU, propagation of every trajectory over
all time steps (symplectic step with Hessian, monodromy, action, prefactor
phase, stability monitor, amplitudes) and the Fourier GEMM with its weighted
|A|^2 reduction into the spectrum.  Inputs (the problem constants) are
resident in HBM before the timed region.  The metric is trajectory-steps/s:
n_traj * n_steps per step / seconds per step.

The JSON line also carries the roofline of the dominant kernel (the
trajectory kernel, bound by FP64 vector ALU), its per-launch duration from HIP
events recorded by the library around each launch on its stream, the HBM
traffic measured with rocprofv3 counters when a matching summary is present
under profiles/, and the oracle timed on a bounded sample on the host cores.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FP64_VALU_PEAK_TFLOPS = 78.6   # MI355X FP64 vector: 256 CU x 2.4 GHz x 128 flop/clk
FP64_MFMA_PEAK_TFLOPS = 78.6   # MI355X FP64 matrix (dense)
F16_MFMA_PEAK_TFLOPS = 2500.0  # MI355X FP16 matrix (dense)
HBM_PEAK_GBS = 8000.0


def traj_flops_per_step(F: int) -> float:
    """Algorithmic FP64 flops of one trajectory-step (FMA = 2), transcendentals excluded.

    drifts 4 x (2F^2 FMA on the tangent q-rows + 5F + 2), kicks 3 x (H M_q: 2F^3 FMA,
    potential/gradient/Hessian 2F^2 + 12F, momentum and action 2F + 2), det(M) by LU
    (2/3)(2F)^3, prefactor matrix 8F^2, complex LU of A (8/3)F^3, amplitude and
    phase 12F + 10.
    """
    drift = 4 * (4 * F * F + 5 * F + 2)
    kick = 3 * (4 * F ** 3 + 2 * F * F + 14 * F + 2)
    detm = (2.0 / 3.0) * (2 * F) ** 3
    pref = 8 * F * F
    deta = (8.0 / 3.0) * F ** 3
    amp = 12 * F + 10
    return float(drift + kick + detm + pref + deta + amp)


def full_flops_per_segment_step(F: int) -> float:
    """Algorithmic FP64 flops of one segment step of the double-time form of
    Eq. (9): the trajectory step without the monitor's real elimination
    (segments are not monitored), plus the product with conj(<chi|z(c1)>)."""
    return traj_flops_per_step(F) - (2.0 / 3.0) * (2 * F) ** 3 + 6.0


def fourier_flops(n_traj: int, n_times: int, K: int) -> float:
    """8 flops per complex multiply-add of amp[j][c] exp(i E_k c dt)."""
    return 8.0 * n_traj * n_times * K


def _source_hash(*names):
    h = hashlib.sha256()
    for nm in names:
        with open(os.path.join(ROOT, "paper_1312_4698_amd", "csrc", nm), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def _profile_traffic(kernel_prefix: str, src_hash: str, n_launch: int):
    """HBM bytes per launch from a committed rocprofv3 counter summary, if it
    was taken on the current kernel source with as many trajectories per
    launch; else None."""
    path = os.path.join(ROOT, "profiles", f"traj_{kernel_prefix}_counters.txt")
    if not os.path.exists(path):
        return None
    txt = open(path).read()
    m = re.search(r"source_hash:\s*(\w+)", txt)
    b = re.search(r"hbm_bytes_per_launch:\s*([0-9.eE+]+)", txt)
    t = re.search(r"trajectories_per_launch:\s*(\d+)", txt)
    if not m or not b or m.group(1) != src_hash or (t and int(t.group(1)) != n_launch):
        return None
    return float(b.group(1))


def _cpu_model() -> str:
    try:
        for ln in open("/proc/cpuinfo"):
            if ln.startswith("model name"):
                return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(prob, n_sample: int, seed: int, n_single: int = 0):
    """The oracle as it stands, on all host cores, over a bounded sample; and,
    if n_single > 0, on one thread over the first n_single of those points (the
    paper times its CPU code on a single thread)."""
    from oracle import oracle as O
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    p0, q0, lr = O.sample_husimi(prob, seed, n_sample)
    t0 = time.perf_counter()
    O.run(prob, p0, q0, lr, want_state=False, want_contrib=False, n_threads=threads)
    dt = time.perf_counter() - t0
    out = {"value": n_sample * prob.n_steps / dt, "unit": "trajectory-steps/s", "cores": threads,
           "kind": "oracle", "cpu_model": _cpu_model(),
           "sample": f"{n_sample} trajectories of the same workload (all {prob.n_steps} steps, "
                     f"{prob.n_energies} energies), {dt:.1f} s wall"}
    if n_single > 0:
        t0 = time.perf_counter()
        O.run(prob, p0[:, :n_single], q0[:, :n_single], lr[:n_single], want_state=False, want_contrib=False,
              n_threads=1)
        d1 = time.perf_counter() - t0
        out["single_thread"] = {"value": n_single * prob.n_steps / d1, "unit": "trajectory-steps/s", "cores": 1,
                                "sample": f"the first {n_single} of those trajectories, {d1:.1f} s wall"}
    return out


def oracle_full(name: str, chunk: int = 2048):
    """The oracle over a whole workload on all host cores, in chunks of
    trajectories with a progress line each; its rate and the host."""
    from oracle import oracle as O
    from paper_1312_4698_amd import inputs
    prob, n = inputs.workload(name)
    prob = prob.replace(precision=inputs.PRECISION_FP64)
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    total = 0.0
    for j0 in range(0, n, chunk):
        m = min(chunk, n - j0)
        p0, q0, lr = O.sample_husimi(prob, 77, m, first_index=j0)
        t0 = time.perf_counter()
        O.run(prob, p0, q0, lr, want_state=False, want_contrib=False, n_threads=threads)
        total += time.perf_counter() - t0
        print(f"[oracle] {name}: {j0 + m} of {n} trajectories, {total:.1f} s", file=sys.stderr, flush=True)
    return {"workload": name, "n_traj": n, "n_steps": prob.n_steps, "n_energies": prob.n_energies, "seconds": total,
            "trajectory_steps_per_s": n * prob.n_steps / total, "cores": threads, "cpu_model": _cpu_model()}


def x1_sweep(scivr, torch, inputs, name: str, log2_sizes, reps: int = 3):
    """Throughput of one form against the trajectory count (one batch of N
    trajectories per step, sample + propagate + accumulate), median of `reps`
    timed steps after one warm-up step per size; one JSON line per size on
    stdout and the knee (the smallest N within 10 % of the largest rate)."""
    prob, _ = inputs.workload(name)
    stream = torch.cuda.current_stream()
    rows = []
    for lg in log2_sizes:
        n = 1 << lg
        ctx = scivr.Context(prob, max_traj=n)
        times = []
        for i in range(reps + 1):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            ctx.sample_husimi(seed=500 + i, n_traj=n, stream=stream)
            ctx.propagate(0, prob.n_steps, stream=stream)
            ctx.accumulate(stream=stream)
            torch.cuda.synchronize()
            if i > 0:
                times.append(time.perf_counter() - t0)
        ctx.close()
        t = float(np.median(times))
        row = {"sweep": name, "n_traj": n, "s_per_step": t, "trajectory_steps_per_s": n * prob.n_steps / t}
        rows.append(row)
        print(json.dumps(row), flush=True)
    best = max(r["trajectory_steps_per_s"] for r in rows)
    knee = next(r["n_traj"] for r in rows if r["trajectory_steps_per_s"] >= 0.9 * best)
    return {"workload": name, "rows": rows, "knee_n_traj": knee, "best_trajectory_steps_per_s": best}


def _energy_reader():
    """A function returning the GPU's accumulated energy in joules (amdsmi), or None."""
    try:
        import amdsmi
        amdsmi.amdsmi_init()
        handle = amdsmi.amdsmi_get_processor_handles()[0]

        def read():
            e = amdsmi.amdsmi_get_energy_count(handle)
            return e["energy_accumulator"] * e["counter_resolution"] * 1e-6
        read()
        return read
    except Exception as exc:  # no SMI access on this machine
        print(f"[bench] energy counter unavailable: {exc}", file=sys.stderr, flush=True)
        return None


def run_form(scivr, torch, prob, n, steps, warmup, seed0=1000, chunk=0, energy=None, stop_flagged=False):
    """Time `steps` whole passes (sample + propagate + accumulate) of one form."""
    stream = torch.cuda.current_stream()
    ctx = scivr.Context(prob, max_traj=n)
    ctx.set_stop_flagged(stop_flagged)

    def one_step(i):
        ctx.sample_husimi(seed=seed0 + i, n_traj=n, stream=stream)
        if chunk and chunk < prob.n_steps:
            for b in range(0, prob.n_steps, chunk):
                ctx.propagate(b, min(prob.n_steps, b + chunk), stream=stream)
                torch.cuda.synchronize()
                print(f"[bench] {prob.name} step {i}: {min(prob.n_steps, b + chunk)} of {prob.n_steps} time steps",
                      file=sys.stderr, flush=True)
        else:
            ctx.propagate(0, prob.n_steps, stream=stream)
        ctx.accumulate(stream=stream)

    for i in range(warmup):
        one_step(i)
        print(f"[bench] {prob.name} warmup {i} done", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    ctx.reset_spectrum(stream=stream)
    ctx.timing(True)
    torch.cuda.synchronize()
    e0 = energy() if energy else None
    t0 = time.perf_counter()
    for i in range(steps):
        one_step(warmup + i)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    e1 = energy() if energy else None
    kt = ctx.kernel_times()
    I, n_good, n_total = ctx.read_spectrum()
    ctx.close()
    print(f"[bench] {prob.name}: {steps} steps in {wall:.3f} s; kernels {kt}", file=sys.stderr, flush=True)
    joules = (e1 - e0) if (e0 is not None and e1 is not None) else None
    return {"wall": wall, "kt": kt, "I": I, "n_good": n_good, "n_total": n_total, "joules": joules}


def fft_form(scivr, torch, prob, n, seed=4321):
    """The Fourier step of one batch by the GEMM and by the exact FFT
    autocorrelation form, on identical trajectories: launch times and the
    spectra's largest relative difference."""
    stream = torch.cuda.current_stream()
    ctx = scivr.Context(prob, max_traj=n)
    res = {}
    for form in ("gemm", "fft"):
        ctx.reset_spectrum(stream=stream)
        ctx.sample_husimi(seed=seed, n_traj=n, stream=stream)
        ctx.propagate(0, prob.n_steps, stream=stream)
        ctx.timing(True)
        if form == "fft":
            ctx.accumulate_fft(stream=stream)
        else:
            ctx.accumulate(stream=stream)
        kt = ctx.kernel_times()
        I, _, _ = ctx.read_spectrum()
        res[form] = (kt["fourier"][1], I)
        print(f"[bench] {prob.name} Fourier step by {form}: {kt['fourier'][1]:.1f} ms", file=sys.stderr, flush=True)
    ctx.close()
    (g_ms, Ig), (f_ms, If) = res["gemm"], res["fft"]
    return {"gemm_ms": g_ms, "fft_ms": f_ms, "speedup": g_ms / f_ms,
            "max_rel_diff": float(np.max(np.abs(If - Ig)) / np.max(np.abs(Ig)))}


def refs_form(scivr, torch, inputs, n=65536, n_refs=8, reps=2, cpu_sample=64, seed=777):
    """Several reference states on one batch (scivr_set_references), F = 9
    FP64, 4096 steps, 2048 energies: whole passes with all n_refs states
    against passes with chi alone, the multi-reference trajectory kernel's
    rate against the FP64 vector peak, the Fourier GEMM (one right-hand side
    per state) against the FP64 matrix peak, and the oracle (one run per
    state, as it stands) on a bounded sample on the host cores."""
    from oracle import oracle as O
    prob, _ = inputs.workload("F9_fp64")
    rng = np.random.default_rng(seed)
    sg = np.sqrt(prob.gamma)
    pe = rng.uniform(-0.8, 0.8, (n_refs - 1, prob.F)) * sg
    qe = rng.uniform(-0.8, 0.8, (n_refs - 1, prob.F)) / sg
    stream = torch.cuda.current_stream()
    res = {}
    for key, k, fft in (("chi_only", 1, False), ("all_states", n_refs, False), ("all_states_fft", n_refs, True)):
        ctx = scivr.Context(prob, max_traj=n)
        if k > 1:
            ctx.set_references(pe, qe)

        def one(i):
            ctx.sample_husimi(seed=seed + i, n_traj=n, stream=stream)
            ctx.propagate(0, prob.n_steps, stream=stream)
            if fft:
                ctx.accumulate_fft(stream=stream)
            else:
                ctx.accumulate(stream=stream)

        one(0)
        torch.cuda.synchronize()
        ctx.reset_spectrum(stream=stream)
        ctx.timing(True)
        t0 = time.perf_counter()
        for i in range(reps):
            one(1 + i)
        torch.cuda.synchronize()
        wall = (time.perf_counter() - t0) / reps
        kt = ctx.kernel_times()
        ctx.close()
        res[key] = {"wall_s": wall, "traj_ms": kt["trajectory"][1] / max(kt["trajectory"][0], 1),
                    "fourier_ms": kt["fourier"][1] / max(kt["fourier"][0], 1)}
        print(f"[bench] several reference states: {k} state(s){' (FFT form)' if fft else ''}, {wall:.3f} s per pass",
              file=sys.stderr, flush=True)
    a = res["all_states"]
    steps = n * prob.n_steps
    fl_traj = steps * (traj_flops_per_step(prob.F) + (n_refs - 1) * (12 * prob.F + 10))
    fl_four = n_refs * fourier_flops(n, prob.n_steps + 1, prob.n_energies)
    achieved = fl_traj / (a["traj_ms"] / 1e3) / 1e12
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    p0, q0, lr = O.sample_husimi(prob, seed, cpu_sample)
    t0 = time.perf_counter()
    for m in range(n_refs):
        pm = prob if m == 0 else prob.replace(p_eq=pe[m - 1], q_eq=qe[m - 1])
        O.run(pm, p0, q0, lr, want_state=False, want_contrib=False, n_threads=threads)
    cpu = time.perf_counter() - t0
    return {
        "workload": f"F9_fp64 with {n_refs} reference states (chi and {n_refs - 1} displaced), {n} Husimi "
                    f"trajectories, {prob.n_steps} steps, {prob.n_energies} energies",
        "value": steps / a["wall_s"], "unit": "trajectory-steps/s (every state's spectrum)",
        "chi_only_value": steps / res["chi_only"]["wall_s"],
        "value_with_fft": steps / res["all_states_fft"]["wall_s"],
        "passes": res,
        "roofline": {"kernel": "traj_kernel (multi-reference variant)", "bound": "alu", "achieved": achieved,
                     "peak": FP64_VALU_PEAK_TFLOPS, "unit": "TFLOP/s", "frac": achieved / FP64_VALU_PEAK_TFLOPS,
                     "flops_per_launch": fl_traj},
        "fourier": {"kernel": "fourier_fp64_kernel", "bound": "mfma",
                    "achieved_TFLOPs": fl_four / (a["fourier_ms"] / 1e3) / 1e12,
                    "peak_TFLOPs": FP64_MFMA_PEAK_TFLOPS},
        "cpu_baseline": {"value": cpu_sample * prob.n_steps / cpu, "unit": "trajectory-steps/s (every state)",
                         "cores": threads, "kind": "oracle",
                         "sample": f"{cpu_sample} trajectories, one oracle run per state ({n_refs}), {cpu:.1f} s wall"},
    }


def full_form_study(scivr, torch, inputs, n=4096, n_steps=512, reps=2, cpu_sample=32, seed=888):
    """The double-time form of Eq. (9) (scivr_accumulate_spectrum_full), F = 9
    FP64, n_steps steps: segment-steps/s of the double-time kernel against the
    FP64 vector peak, whole passes (sample + propagate + double-time
    accumulation), and the oracle's double-time form on a bounded sample."""
    from oracle import oracle as O
    prob = inputs.workload("F9_fp64")[0].replace(n_steps=n_steps)
    stream = torch.cuda.current_stream()
    ctx = scivr.Context(prob, max_traj=n)

    def one(i):
        ctx.sample_husimi(seed=seed + i, n_traj=n, stream=stream)
        ctx.propagate(0, prob.n_steps, stream=stream)
        ctx.accumulate_full(stream=stream)

    one(0)
    torch.cuda.synchronize()
    ctx.reset_spectrum(stream=stream)
    ctx.timing(True)
    t0 = time.perf_counter()
    for i in range(reps):
        one(1 + i)
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) / reps
    kt = ctx.kernel_times()
    ctx.close()
    full_ms = kt["fourier"][1] / max(kt["fourier"][0], 1)
    seg = n * n_steps * (n_steps + 1) / 2  # segment steps: sum over c1 of (n_steps - c1)
    fl = seg * full_flops_per_segment_step(prob.F)
    achieved = fl / (full_ms / 1e3) / 1e12
    print(f"[bench] double-time form: {wall:.3f} s per pass, {full_ms:.1f} ms in the double-time kernels",
          file=sys.stderr, flush=True)
    p0, q0, lr = O.sample_husimi(prob, seed, cpu_sample)
    t0 = time.perf_counter()
    O.run_full(prob, p0, q0, lr)
    cpu = time.perf_counter() - t0
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {
        "workload": f"F9_fp64 at {n_steps} steps, double-time form of Eq. (9): {n} Husimi trajectories, "
                    f"{prob.n_energies} energies",
        "value": seg / (full_ms / 1e3), "unit": "segment-steps/s",
        "pass_s": wall, "double_time_ms": full_ms, "segment_steps_per_pass": seg,
        "roofline": {"kernel": "ta_full_kernel (with the lag sums and the spectrum)", "bound": "alu",
                     "achieved": achieved, "peak": FP64_VALU_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / FP64_VALU_PEAK_TFLOPS, "flops_per_launch": fl},
        "cpu_baseline": {"value": cpu_sample * n_steps * (n_steps + 1) / 2 / cpu, "unit": "segment-steps/s",
                         "cores": threads, "kind": "oracle",
                         "sample": f"{cpu_sample} trajectories of the same problem, {cpu:.1f} s wall"},
    }


def _peak_error_cm(peaks, inputs, E, T, ref_peaks, I):
    """Largest peak shift (cm^-1) of I against the reference peaks; inf if a peak is missing."""
    pt = peaks.find_peaks(E, I, T)
    worst, missing = peaks.peak_errors(ref_peaks, pt, tol=20.0 / inputs.CM1_PER_HARTREE)
    return float("inf") if missing else worst * inputs.CM1_PER_HARTREE


def _half_max_centre(E, I, e0, tol):
    """Midpoint of the half-maximum crossings of the peak nearest e0 (linear
    interpolation between grid points): a position that stays defined on a
    broad, flat-topped peak."""
    k0 = int(np.argmin(np.abs(E - e0)))
    lo, hi = max(k0 - int(tol / (E[1] - E[0])), 1), min(k0 + int(tol / (E[1] - E[0])), E.size - 2)
    k = lo + int(np.argmax(I[lo:hi + 1]))
    half = 0.5 * I[k]
    a = k
    while a > 0 and I[a] > half:
        a -= 1
    b = k
    while b < E.size - 1 and I[b] > half:
        b += 1
    if I[a] > half or I[b] > half:
        return None
    ea = E[a] + (half - I[a]) / (I[a + 1] - I[a]) * (E[1] - E[0])
    eb = E[b - 1] + (I[b - 1] - half) / (I[b - 1] - I[b]) * (E[1] - E[0])
    return 0.5 * (ea + eb)


def learned_study(scivr, inputs, peaks, prob, ref_I, sizes, seeds, n_train, layers, width, epochs, batch, lr,
                  alpha, judge_batches=4, window=0.01, n_fine=2048, n_boot=2000):
    """The learned proposal against plain Husimi sampling, in the form of `prob`.

    The comparison runs on a fine energy grid (n_fine points over +-window
    hartree around the main peak of the timed run's spectrum `ref_I`), where
    a plain FP64 judge of judge_batches x max(sizes) Husimi trajectories gives
    the reference spectrum and peak.  For each of the seeds and each N in
    `sizes`, an independent batch of N trajectories (Philox indices disjoint
    from the judge's) gives a spectrum, its peak position error (R13 vertex,
    and the half-maximum midpoint), and its relative RMS error.  Reported:
      * the variance ratio plain / learned at equal N (median over N of the
        squared RMS ratio), the robust figure;
      * per N, the median peak error over the seeds with a bootstrap 16-84 %
        interval (resampling seeds);
      * N_to_1cm: the smallest N from which on the median stays <= 1 cm^-1,
        and N_to_1cm_fit: where a * N^-1/2, fitted to the medians, crosses 1.
    The flow is trained once on the contributions of a Husimi batch of n_train
    trajectories on the fine grid."""
    CM = inputs.CM1_PER_HARTREE
    E0, T = prob.energies(), prob.total_time
    e_peak = peaks.find_peaks(E0, ref_I, T)
    e_main = max(e_peak, key=lambda p: p[1])[0]
    fine = prob.replace(e_min=e_main - window, e_max=e_main + window, n_energies=n_fine)
    E = fine.energies()
    tol = 20.0 / CM
    cap = max(max(sizes), n_train)
    # the judge: plain FP64 on the fine grid
    jprob = fine.replace(precision=inputs.PRECISION_FP64)
    jctx = scivr.Context(jprob, max_traj=max(sizes))
    for b in range(judge_batches):
        jctx.run(seed=9001, n_traj=max(sizes), first_index=b * max(sizes))
    judge, _, _ = jctx.read_spectrum()
    jctx.close()
    jp = [p for p in peaks.find_peaks(E, judge, T) if abs(p[0] - e_main) < tol]
    e_ref = jp[0][0] if jp else e_main
    h_ref = _half_max_centre(E, judge, e_ref, tol)
    ctx = scivr.Context(fine, max_traj=cap)
    base = 1 << 40  # Philox indices far from the judge's

    def sweep(draw):
        vert = np.full((len(seeds), len(sizes)), np.inf)
        half = np.full_like(vert, np.inf)
        rms = np.zeros_like(vert)
        for a, sd in enumerate(seeds):
            for b, N in enumerate(sizes):
                ctx.reset_spectrum()
                draw(sd, N)
                ctx.propagate()
                ctx.accumulate()
                I, _, _ = ctx.read_spectrum()
                pk = [p for p in peaks.find_peaks(E, I, T) if abs(p[0] - e_ref) < tol]
                if pk:
                    vert[a, b] = abs(min(pk, key=lambda p: abs(p[0] - e_ref))[0] - e_ref) * CM
                hc = _half_max_centre(E, I, e_ref, tol)
                if hc is not None and h_ref is not None:
                    half[a, b] = abs(hc - h_ref) * CM
                rms[a, b] = float(np.sqrt(np.mean((I - judge) ** 2)) / judge.max())
        rng = np.random.default_rng(12345)
        boots = np.array([np.median(vert[rng.integers(0, len(seeds), len(seeds))], axis=0) for _ in range(n_boot)])
        med = np.median(vert, axis=0)
        n1 = None
        for b in range(len(sizes) - 1, -1, -1):
            if med[b] <= 1.0:
                n1 = sizes[b]
            else:
                break
        fin = np.isfinite(med) & (med > 0)
        a_fit = float(np.exp(np.mean(np.log(med[fin] * np.sqrt(np.array(sizes)[fin]))))) if fin.any() else None
        return {"N_to_1cm": n1, "N_to_1cm_fit": None if a_fit is None else a_fit ** 2,
                "median_peak_error_cm1": med.tolist(),
                "peak_error_cm1_16_84": [np.percentile(boots, 16, axis=0).tolist(),
                                         np.percentile(boots, 84, axis=0).tolist()],
                "median_half_max_error_cm1": np.median(half, axis=0).tolist(),
                "median_rel_rms": np.median(rms, axis=0).tolist()}

    t0 = time.perf_counter()
    plain = sweep(lambda sd, N: ctx.sample_husimi(seed=sd, n_traj=N, first_index=base))
    t_plain = time.perf_counter() - t0
    print("[bench] learned-proposal study: plain sweep done", file=sys.stderr, flush=True)
    flow = scivr.Flow(ctx, layers, width, seed=5)
    ctx.reset_spectrum()
    ctx.run(seed=4242, n_traj=n_train, first_index=2 * base)
    ctx.read_totals()  # waits for the training batch: its time is counted apart, at the measured throughput
    t0 = time.perf_counter()
    loss = flow.train_on_batch(epochs=epochs, batch=batch, lr=lr)
    t_train = time.perf_counter() - t0
    info = {}

    def draw_flow(sd, N):
        t = time.perf_counter()
        ess, used = flow.sample(seed=sd, n_traj=N, first_index=base, alpha=alpha)  # returns after the draw
        info.setdefault("sample_s_per_point", []).append((time.perf_counter() - t) / N)
        info.setdefault("ess", []).append(ess)
        info.setdefault("used", []).append(used)

    t0 = time.perf_counter()
    learned = sweep(draw_flow)
    t_learned = time.perf_counter() - t0
    flow.close()
    ctx.close()
    ratio = np.array(plain["median_rel_rms"]) / np.array(learned["median_rel_rms"])
    return {
        "variance_ratio_plain_over_learned": float(np.median(ratio ** 2)),
        "variance_ratio_per_N": (ratio ** 2).tolist(),
        "N_ratio_fit_plain_over_learned": (None if not (plain["N_to_1cm_fit"] and learned["N_to_1cm_fit"]) else
                                           plain["N_to_1cm_fit"] / learned["N_to_1cm_fit"]),
        "sizes": list(sizes), "seeds": len(seeds), "fine_grid": {"e_min": fine.e_min, "e_max": fine.e_max,
                                                                 "n_energies": n_fine,
                                                                 "spacing_cm1": (E[1] - E[0]) * CM},
        "judge": {"trajectories": judge_batches * max(sizes), "peak_cm1": e_ref * CM,
                  "half_max_centre_cm1": None if h_ref is None else h_ref * CM},
        "plain": plain, "learned": learned,
        "flow": {"layers": layers, "width": width, "params": int(FLOW_PARAMS(prob.F, width, layers)),
                 "n_train": n_train, "epochs": epochs, "batch": batch, "lr": lr, "alpha": alpha,
                 "final_loss": loss, "train_s": t_train, "ess_min": float(min(info["ess"])),
                 "ess_median": float(np.median(info["ess"])), "fallbacks": int(sum(1 for u in info["used"] if not u)),
                 # drawing from the mixture, at the sweep's largest N
                 "sample_s_per_point": float(np.median(info["sample_s_per_point"][len(sizes) - 1::len(sizes)]))},
        "sweep_s": {"plain": t_plain, "learned": t_learned},
    }


def _jackknife_peaks(peaks, E, T, tots, Gs, scale, ref, tol):
    """Peaks of the pooled spectrum sum(tots) / sum(Gs) matched to the reference
    peaks `ref`, each with its jackknife standard error over the batches
    (leave-one-batch-out spectra); unmatched peaks give None."""
    tots, Gs = np.asarray(tots), np.asarray(Gs)
    B = len(Gs)

    def match(I):
        pk = peaks.find_peaks(E, I, T)
        out = []
        for e, _ in ref:
            d = [abs(e - t) for t, _ in pk]
            out.append(None if not d or min(d) > tol else pk[int(np.argmin(d))][0])
        return out

    full = match(scale * tots.sum(axis=0) / Gs.sum())
    loo = [match(scale * (tots.sum(axis=0) - tots[b]) / (Gs.sum() - Gs[b])) for b in range(B)]
    res = []
    for i, e in enumerate(full):
        xs = [l[i] for l in loo if l[i] is not None]
        if e is None or len(xs) < B:
            res.append((e, None))
            continue
        xs = np.array(xs)
        res.append((e, float(np.sqrt((B - 1) / B * np.sum((xs - xs.mean()) ** 2)))))
    return res


def c5_study(scivr, torch, inputs, peaks, n, B=8, seed=303, n_train=32768, layers=4, width=256, epochs=10,
             batch=4096, lr=1e-3, chunk=2048, frac=0.2, min_ess=0.05, variants=((1.0, 0.1), (0.0, 0.1)), stop_flagged=True):
    """The F=30 configuration: mixed form + learned proposal against the plain
    FP64 GPU judge, with Monte Carlo error bars.

    * Judge: the FP64 form on n Husimi points in B batches.
    * Precision alone: the mixed form on the same points; then both forms
      again on the points that are good in both (identical good subsets), so
      their peak difference holds no sampling or flagging difference.
    * Mixed + learned: a flow trained on the mixed form's contributions of a
      separate Husimi batch, sampled (defensive mixture) for n points in B
      batches, importance-weighted.
    Peaks are those of the judge with I >= frac * max (and >= 5 % for the
    full list), matched within 20 cm^-1; each carries the jackknife standard
    error over the B batches."""
    def _ctx(prob, max_traj):
        # flagged trajectories stop at their flag: the estimates are bit-identical
        c = scivr.Context(prob, max_traj=max_traj)
        c.set_stop_flagged(stop_flagged)
        return c

    CM = inputs.CM1_PER_HARTREE
    pf, _ = inputs.workload("F30_fp64")
    pm, _ = inputs.workload("F30_mixed")
    E, T = pf.energies(), pf.total_time
    scale = pf.dt ** 2 / (2 * np.pi * T)
    nb = n // B
    tol = 20.0 / CM

    def propagate(ctx, prob, label):
        for b0 in range(0, prob.n_steps, chunk):
            ctx.propagate(b0, min(prob.n_steps, b0 + chunk))
            torch.cuda.synchronize()
        print(f"[c5] {label} done", file=sys.stderr, flush=True)

    def batched(prob, fill, label):
        ctx = _ctx(prob, max_traj=nb)
        tots, Gs, goods, pts = [], [], [], []
        for b in range(B):
            ctx.reset_spectrum()
            fill(ctx, b)
            propagate(ctx, prob, f"{label} batch {b}")
            ctx.accumulate()
            tot, G, ng, _ = ctx.read_totals()
            tots.append(tot)
            Gs.append(G)
            goods.append(ctx.read_state(want_M=False)["good"].astype(bool))
            pts.append(ctx.read_initial())
        ctx.close()
        return tots, Gs, goods, pts

    t0 = time.perf_counter()
    husimi = lambda ctx, b: ctx.sample_husimi(seed=seed, n_traj=nb, first_index=b * nb)
    jt, jG, jgood, jpts = batched(pf, husimi, "fp64 judge")
    t_judge = time.perf_counter() - t0
    t0 = time.perf_counter()
    mt, mG, mgood, _ = batched(pm, husimi, "mixed")
    t_mixed = time.perf_counter() - t0
    I_judge = scale * np.sum(jt, axis=0) / np.sum(jG)
    ref_all = peaks.find_peaks(E, I_judge, T)
    ref = [p for p in ref_all if p[1] >= frac * I_judge.max()]

    # identical good subsets: the points good in both forms, both forms again
    both = [jg & mg for jg, mg in zip(jgood, mgood)]
    sub = {}
    for form, prob in (("fp64", pf), ("mixed", pm)):
        ctx = _ctx(prob, max_traj=max(1, max(int(x.sum()) for x in both)))
        tots, Gs = [], []
        for b in range(B):
            keep = np.flatnonzero(both[b])
            if keep.size == 0:
                tots.append(np.zeros(pf.n_energies))
                Gs.append(0.0)
                continue
            p0, q0, logrho = jpts[b]
            ctx.reset_spectrum()
            ctx.set_initial(p0[:, keep], q0[:, keep], logrho[keep])
            propagate(ctx, prob, f"identical subset {form} batch {b}")
            ctx.accumulate()
            tot, G, ng, _ = ctx.read_totals()
            tots.append(tot)
            Gs.append(G)
        ctx.close()
        sub[form] = (tots, Gs)
    Isub = {f: scale * np.sum(sub[f][0], axis=0) / np.sum(sub[f][1]) for f in sub}
    ref_sub = [p for p in peaks.find_peaks(E, Isub["fp64"], T) if p[1] >= frac * Isub["fp64"].max()]
    pk_sub = _jackknife_peaks(peaks, E, T, *sub["mixed"], scale, ref_sub, tol)
    pk_sub_j = _jackknife_peaks(peaks, E, T, *sub["fp64"], scale, ref_sub, tol)

    # learned proposals, trained on a separate Husimi batch of the mixed form.
    # The proposal's target is a design choice that leaves the estimator
    # unbiased (the weights use the proposal's own density): the trajectories'
    # contributions c_j (temper 1), or c_j^temper, down to the good-trajectory
    # indicator (temper 0), which asks for the region where trajectories stay
    # good with equal weight.
    t0 = time.perf_counter()
    ctx = _ctx(pm, max_traj=max(nb, n_train))
    ctx.sample_husimi(seed=seed + 1, n_traj=n_train, first_index=1 << 40)
    propagate(ctx, pm, "training batch")
    ctx.accumulate()
    tp0, tq0, _ = ctx.read_initial()
    tc = ctx.read_contributions()
    t_batch = time.perf_counter() - t0
    runs = {}
    for temper, alpha in variants:
        c = (tc > 0).astype(np.float64) if temper == 0 else np.where(tc > 0, tc, 0.0) ** temper
        t0 = time.perf_counter()
        flow = scivr.Flow(ctx, layers, width, seed=9)
        loss = flow.train(tp0, tq0, c / c.mean(), epochs=epochs, batch=batch, lr=lr)
        t_train = time.perf_counter() - t0
        lt, lG, lgood, ess = [], [], [], []
        t0 = time.perf_counter()
        for b in range(B):
            ctx.reset_spectrum()
            e_, used = flow.sample(seed=seed + 2, n_traj=nb, first_index=b * nb, alpha=alpha, min_ess_frac=min_ess)
            ess.append((e_, used))
            propagate(ctx, pm, f"learned (temper {temper}, alpha {alpha}) batch {b}")
            ctx.accumulate()
            tot, G, ng, _ = ctx.read_totals()
            lt.append(tot)
            lG.append(G)
            lgood.append(ng / nb)
        flow.close()
        runs[(temper, alpha)] = {"lt": lt, "lG": lG, "lgood": lgood, "ess": ess, "loss": loss, "train_s": t_train,
                                 "wall_s": time.perf_counter() - t0}
    ctx.close()

    def compare(pk_test, pk_ref):
        rows = []
        for (e_r, s_r), (e_t, s_t) in zip(pk_ref, pk_test):
            if e_r is None or e_t is None:
                rows.append({"judge_cm1": None if e_r is None else e_r * CM, "missing": True})
                continue
            sig = None if (s_r is None or s_t is None) else float(np.hypot(s_r, s_t)) * CM
            rows.append({"judge_cm1": e_r * CM, "test_cm1": e_t * CM, "delta_cm1": (e_t - e_r) * CM,
                         "sigma_cm1": sig})
        return rows

    # statistics a broad band of close levels keeps stable against Monte Carlo
    # ripples: the main peak of the spectrum smoothed at twice the time
    # window's resolution, and the first moment over the judge's band (I >= 5 %
    # of max), each with the jackknife error over the batches
    sig = 2.0 * 2.0 * np.pi / T / 2.355
    band = E[I_judge >= 0.05 * I_judge.max()]
    lo, hi = float(band.min()), float(band.max())

    def jack(stat, tots, Gs):
        tots, Gs = np.asarray(tots), np.asarray(Gs)
        full = stat(scale * tots.sum(axis=0) / Gs.sum())
        loo = np.array([stat(scale * (tots.sum(axis=0) - tots[b]) / (Gs.sum() - Gs[b])) for b in range(B)])
        return full, float(np.sqrt((B - 1) / B * np.sum((loo - loo.mean()) ** 2)))

    def main_peak(I):
        Is = peaks.smooth(E, I, sig)
        k = int(np.argmax(Is))
        k = min(max(k, 1), E.size - 2)
        y0, y1, y2 = Is[k - 1], Is[k], Is[k + 1]
        return E[k] + 0.5 * (y0 - y2) / (y0 - 2 * y1 + y2) * (E[1] - E[0])

    def cen(I):
        return peaks.centroid(E, I, lo, hi)

    def stable(tots_t, Gs_t, tots_r, Gs_r):
        out = {}
        for name, st in (("smoothed_main_peak", main_peak), ("band_centroid", cen)):
            (vt, st_t), (vr, st_r) = jack(st, tots_t, Gs_t), jack(st, tots_r, Gs_r)
            out[name] = {"judge_cm1": vr * CM, "test_cm1": vt * CM, "delta_cm1": (vt - vr) * CM,
                         "sigma_cm1": float(np.hypot(st_t, st_r)) * CM, "sigma_judge_cm1": st_r * CM,
                         "sigma_test_cm1": st_t * CM}
        return out

    # per-energy jackknife variance over the judge's band: judge vs learned at equal N
    def jvar(tots, Gs):
        tots, Gs = np.asarray(tots), np.asarray(Gs)
        loo = np.array([scale * (tots.sum(axis=0) - tots[b]) / (Gs.sum() - Gs[b]) for b in range(B)])
        return (B - 1) / B * np.sum((loo - loo.mean(axis=0)) ** 2, axis=0)

    inband = I_judge >= 0.05 * I_judge.max()
    pk_judge = _jackknife_peaks(peaks, E, T, jt, jG, scale, ref, tol)
    pk_mixed = _jackknife_peaks(peaks, E, T, mt, mG, scale, ref, tol)
    worst = lambda rows: max([abs(r["delta_cm1"]) for r in rows if not r.get("missing")] or [float("nan")])
    learned = {}
    for (temper, alpha), v in runs.items():
        I_learn = scale * np.sum(v["lt"], axis=0) / np.sum(v["lG"])
        rows = compare(_jackknife_peaks(peaks, E, T, v["lt"], v["lG"], scale, ref, tol), pk_judge)
        learned[f"temper_{temper}_alpha_{alpha}"] = {
            "good_fraction": float(np.mean(v["lgood"])),
            "variance_ratio_judge_over_learned": float(np.median(jvar(jt, jG)[inband] / jvar(v["lt"], v["lG"])[inband])),
            "stable_vs_judge": stable(v["lt"], v["lG"], jt, jG),
            "peaks_vs_judge": {"peaks": rows, "worst_abs_delta_cm1": worst(rows),
                               "missing": int(sum(1 for r in rows if r.get("missing")))},
            "rel_rms_vs_judge": float(np.sqrt(np.mean((I_learn - I_judge) ** 2)) / I_judge.max()),
            "ess": [float(e) for e, _ in v["ess"]], "fallbacks": int(sum(1 for _, u in v["ess"] if not u)),
            "final_loss": v["loss"], "train_s": v["train_s"], "wall_s": v["wall_s"],
        }
    out = {
        "n_traj": n, "batches": B, "peak_threshold_frac": frac,
        "judge_peaks_cm1": [e * CM for e, _ in ref], "judge_peaks_5pct": len(ref_all),
        "good_fraction": {"fp64": float(np.mean(np.concatenate(jgood))), "mixed": float(np.mean(np.concatenate(mgood))),
                          "both": float(np.mean(np.concatenate(both)))},
        "smoothing_fwhm_cm1": sig * 2.355 * CM, "band_cm1": [lo * CM, hi * CM],
        "precision_identical_subset": {"n_traj": int(sum(int(x.sum()) for x in both)),
                                       "peaks": compare(pk_sub, pk_sub_j), "worst_abs_delta_cm1": None},
        "stable_precision_identical_subset": stable(*sub["mixed"], *sub["fp64"]),
        "mixed_vs_judge": {"peaks": compare(pk_mixed, pk_judge)},
        "stable_mixed_vs_judge": stable(mt, mG, jt, jG),
        "learned": learned,
        "flow": {"width": width, "layers": layers, "n_train": n_train, "epochs": epochs,
                 "min_ess_frac": min_ess, "training_batch_s": t_batch},
        "wall_s": {"judge": t_judge, "mixed": t_mixed}, "stop_flagged": stop_flagged,
    }
    for key in ("precision_identical_subset", "mixed_vs_judge"):
        out[key]["worst_abs_delta_cm1"] = worst(out[key]["peaks"])
        out[key]["missing"] = int(sum(1 for r in out[key]["peaks"] if r.get("missing")))
    return out


def _energy_summary(run, steps):
    """GPU energy of one step (one batch) from the SMI accumulator, or None."""
    if run.get("joules") is None:
        return None
    j = run["joules"] / steps
    return {"J_per_step": j, "kWh_per_step": j / 3.6e6, "avg_W": run["joules"] / run["wall"],
            "source": "amdsmi energy accumulator around the timed steps"}


def FLOW_PARAMS(F, H, L):
    return L * (H * F + H + H * H + H + 2 * F * H + 2 * F)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="F9_mixed")
    ap.add_argument("--plain", default="F9_fp64", help="plain FP64 form timed alongside ('' to skip)")
    ap.add_argument("--n-traj", type=int, default=0, help="override the trajectory count")
    ap.add_argument("--cpu-sample", type=int, default=512, help="oracle trajectories for the CPU baseline (0: skip)")
    ap.add_argument("--learned", type=int, default=1, help="run the learned-proposal study (1) or not (0)")
    ap.add_argument("--fft", type=int, default=1,
                    help="also time the exact FFT-autocorrelation Fourier step against the GEMM (1) or not (0)")
    ap.add_argument("--stop-flagged", type=int, default=0,
                    help="stop trajectories at the step the stability monitor flags them (F > 16 kernel); "
                         "the value then still counts every trajectory-step of the batch")
    ap.add_argument("--chunk", type=int, default=0,
                    help="propagate in calls of this many time steps, printing progress (0: one call)")
    ap.add_argument("--cpu-single", type=int, default=64,
                    help="oracle trajectories for the single-thread CPU rate (0: skip)")
    ap.add_argument("--c5", type=int, default=0,
                    help="only run the F=30 mixed + learned vs FP64 judge study on this many trajectories and exit")
    ap.add_argument("--c5-variants", default="1:0.1,0:0.1",
                    help="learned-proposal variants of the F=30 study, temper:alpha pairs (temper 0: good indicator)")
    ap.add_argument("--c5-train", type=int, default=32768, help="training batch of the F=30 study's flows")
    ap.add_argument("--c5-stop-flagged", type=int, default=1,
                    help="stop flagged trajectories in the F=30 study (bit-identical estimates, shorter runs)")
    ap.add_argument("--oracle-full", default="",
                    help="only time the oracle over this whole workload on the host cores and exit")
    ap.add_argument("--sweep", default="",
                    help="only run the throughput sweep of this workload over N = 2^7 .. 2^18 and exit")
    ap.add_argument("--next-rows", type=int, default=1,
                    help="also measure several reference states on one batch and the double-time form (1) or not (0)")
    ap.add_argument("--next-rows-only", type=int, default=0,
                    help="only measure several reference states and the double-time form, and exit")
    ap.add_argument("--copy-calibration", type=int, default=0,
                    help="only copy this many bytes device-to-device (counter calibration) and exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "only one GPU is supported: the path shards by trajectory index (first_index "
                                   "ranges) with one all-reduce of the K-vector, but no multi-GPU run is provided",
                          "n_gpus": args.gpus}))
        sys.exit(2)

    if args.oracle_full:  # host cores only
        print(json.dumps({"oracle_full": oracle_full(args.oracle_full)}))
        return
    import torch
    from paper_1312_4698_amd import inputs, peaks, scivr

    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU visible"}))
        sys.exit(1)
    if args.copy_calibration:
        a = torch.ones(args.copy_calibration // 8, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copied_bytes": a.numel() * 8}))
        return
    if args.c5:
        vs = tuple(tuple(float(x) for x in v.split(":")) for v in args.c5_variants.split(","))
        res = c5_study(scivr, torch, inputs, peaks, args.c5, n_train=args.c5_train, variants=vs,
                       stop_flagged=bool(args.c5_stop_flagged))
        print(json.dumps({"c5_study": res}))
        return
    if args.sweep:
        res = x1_sweep(scivr, torch, inputs, args.sweep, range(7, 19))
        print(json.dumps({"sweep_summary": res}))
        return
    if args.next_rows_only:
        print(json.dumps({"several_references": refs_form(scivr, torch, inputs),
                          "double_time_form": full_form_study(scivr, torch, inputs)}))
        return
    prob, n = inputs.workload(args.workload)
    if args.n_traj:
        n = args.n_traj
    print(f"[bench] {args.workload}: F={prob.F} n={n} steps={prob.n_steps} K={prob.n_energies}", file=sys.stderr,
          flush=True)
    energy = _energy_reader()
    main_run = run_form(scivr, torch, prob, n, args.steps, args.warmup, chunk=args.chunk, energy=energy,
                        stop_flagged=bool(args.stop_flagged))
    plain = None
    if args.plain:
        pprob, _ = inputs.workload(args.plain)
        plain = run_form(scivr, torch, pprob, n, args.steps, args.warmup, chunk=args.chunk, energy=energy,
                         stop_flagged=bool(args.stop_flagged))

    wall = main_run["wall"]
    kt = main_run["kt"]
    ms_step = wall / args.steps * 1e3
    traj_steps = n * prob.n_steps
    value = traj_steps / (wall / args.steps)
    n_tr, ms_tr = kt["trajectory"]
    n_fo, ms_fo = kt["fourier"]
    # one pass may be several trajectory launches (chunked propagation): the
    # rate is the pass's algorithmic flops over the summed launch durations
    t_launch = ms_tr / max(n_tr, 1) / 1e3
    launches_per_pass = max(n_tr, 1) / args.steps
    fl_launch = traj_flops_per_step(prob.F) * traj_steps / launches_per_pass
    achieved = fl_launch / t_launch / 1e12
    big = prob.F > 16
    src_hash = _source_hash(*(("traj_big.hip", "traj_common.h") if big else ("traj.hip", "traj_common.h", "group_lu.h")))
    traffic = _profile_traffic(prob.name, src_hash, n)
    fo_launch = ms_fo / max(n_fo, 1) / 1e3
    fo_fl = fourier_flops(n, prob.n_steps + 1, prob.n_energies)
    mixed = prob.precision == inputs.PRECISION_MIXED

    out = {
        "metric": f"trajectory-steps/s at F={prob.F}",
        "value": value,
        "unit": "trajectory-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64 trajectory, f16x2 MFMA Fourier" if mixed else "f64",
        "data": "synthetic",
        "config": {
            "workload": f"{args.workload}: Morse + quartic coupling, F={prob.F}, {n} Husimi trajectories, "
                        f"{prob.n_steps} steps of dt={prob.dt} au, {prob.n_energies} energies on "
                        f"[{prob.e_min}, {prob.e_max}] hartree",
            "F": prob.F, "n_traj": n, "n_steps": prob.n_steps, "n_energies": prob.n_energies,
            "precision": "mixed" if mixed else "fp64", "parallelism": "single GPU",
        },
        "roofline": {
            "kernel": "traj_big_kernel" if big else "traj_kernel",
            "bound": "alu",
            "achieved": achieved,
            "peak": FP64_VALU_PEAK_TFLOPS,
            "unit": "TFLOP/s",
            "frac": achieved / FP64_VALU_PEAK_TFLOPS,
            "traffic": traffic,
            "launch_ms": t_launch * 1e3,
            "flops_per_launch": fl_launch,
            "source_hash": src_hash,
        },
        "fourier": {
            "kernel": "fourier_f16_kernel" if mixed else "fourier_fp64_kernel",
            "bound": "mfma",
            "achieved_useful_TFLOPs": fo_fl / fo_launch / 1e12,
            "peak_TFLOPs": F16_MFMA_PEAK_TFLOPS / 3.0 if mixed else FP64_MFMA_PEAK_TFLOPS,
            "launch_ms": fo_launch * 1e3,
        },
        "composite_roofline": {
            # sum over the step's parts of (algorithmic flops / that part's peak), over the measured step time
            "frac": (traj_flops_per_step(prob.F) * traj_steps / (FP64_VALU_PEAK_TFLOPS * 1e12)
                     + fo_fl * n_fo / args.steps / ((F16_MFMA_PEAK_TFLOPS / 3.0 if mixed else FP64_MFMA_PEAK_TFLOPS) * 1e12))
                    / (ms_step / 1e3),
            "parts": "trajectory kernel on the FP64 vector peak; Fourier step on "
                     + ("the dense FP16 MFMA peak / 3" if mixed else "the FP64 MFMA peak"),
        },
        "n_good_fraction": main_run["n_good"] / max(main_run["n_total"], 1),
        "stop_flagged": bool(args.stop_flagged) and {
            "note": "flagged trajectories stopped at their flag (F > 16 kernel): value and the roofline count every "
                    "trajectory-step of the batch, so they are the time-to-spectrum rate, not the kernel's"},
        "energy": _energy_summary(main_run, args.steps),
        "cpu_baseline": None,
    }
    if mixed:
        out["fourier"]["note"] = ("three FP16 products per real product (hi*hi + hi*lo + lo*hi): the useful "
                                  "peak is the dense FP16 MFMA peak / 3")
    if plain is not None:
        pv = traj_steps / (plain["wall"] / args.steps)
        E = prob.energies()
        T = prob.total_time
        pr = peaks.find_peaks(E, plain["I"], T)
        pt = peaks.find_peaks(E, main_run["I"], T)
        worst, missing = peaks.peak_errors(pr, pt, tol=20.0 / inputs.CM1_PER_HARTREE)
        out["plain_fp64"] = {
            "value": pv, "ms_per_step": plain["wall"] / args.steps * 1e3,
            "trajectory_ms": plain["kt"]["trajectory"][1] / max(plain["kt"]["trajectory"][0], 1),
            "fourier_ms": plain["kt"]["fourier"][1] / max(plain["kt"]["fourier"][0], 1),
            "speedup_of_value": value / pv,
            "n_good_fraction": plain["n_good"] / max(plain["n_total"], 1),
            "energy": _energy_summary(plain, args.steps),
            "peak_error_cm1": worst * inputs.CM1_PER_HARTREE, "peaks_compared": len(pr), "peaks_missing": missing,
            "same_samples": True,
        }
    if args.learned and plain is not None:
        print("[bench] learned-proposal study", file=sys.stderr, flush=True)
        sizes = [1 << k for k in range(10, 19)]
        out["learned_proposal"] = learned_study(scivr, inputs, peaks, prob, plain["I"], sizes,
                                                seeds=tuple(range(11, 31)),
                                                n_train=65536, layers=4, width=128, epochs=20, batch=4096, lr=1e-3,
                                                alpha=0.1)
        lp = out["learned_proposal"]
        vp, vm = out["plain_fp64"]["value"], value
        n_plain, n_learn = lp["plain"]["N_to_1cm"], lp["learned"]["N_to_1cm"]
        train_s = lp["flow"]["train_s"] + lp["flow"]["n_train"] * prob.n_steps / vm
        draw_s = lp["flow"]["sample_s_per_point"]
        both = n_plain is not None and n_learn is not None
        out["time_to_1cm"] = {
            "equal_variance_speedup": lp["variance_ratio_plain_over_learned"] * vm / vp,
            "equal_variance_energy_ratio": (
                None if not (out["energy"] and out["plain_fp64"]["energy"]) else
                lp["variance_ratio_plain_over_learned"] * out["plain_fp64"]["energy"]["J_per_step"]
                / out["energy"]["J_per_step"]),
            # only when both sides reach 1 cm^-1 within the sweep
            "plain_fp64_s": n_plain * prob.n_steps / vp if both else None,
            "mixed_learned_s": n_learn * (prob.n_steps / vm + draw_s) + train_s if both else None,
            "fit_plain_fp64_s": (None if lp["plain"]["N_to_1cm_fit"] is None else
                                 lp["plain"]["N_to_1cm_fit"] * prob.n_steps / vp),
            "fit_mixed_learned_s": (None if lp["learned"]["N_to_1cm_fit"] is None else
                                    lp["learned"]["N_to_1cm_fit"] * (prob.n_steps / vm + draw_s) + train_s),
            "mixed_learned_training_s": train_s,
            "note": ("plain: FP64 path with Husimi sampling; mixed_learned: mixed path with the learned proposal, "
                     "including its training batch, training time and the draws from the mixture; equal_variance_speedup = (plain/learned "
                     "spectrum variance at equal N) x (mixed/plain throughput); fit_*: from the N^-1/2 fit of the "
                     "median peak error"),
        }
    if args.fft:
        # a separate wall-time line: the Fourier step of one batch of each form
        # by the FFT autocorrelation against the GEMM (not part of `value`)
        forms = [(prob, "main")] + ([(inputs.workload(args.plain)[0], "plain_fp64")] if args.plain else [])
        out["fft_fourier"] = {}
        for fp, key in forms:
            if fp.n_steps > 4096:
                out["fft_fourier"][key] = {"skipped": "the FFT form holds at most 4096 steps"}
                continue
            r = fft_form(scivr, torch, fp, n)
            tr_ms = (kt if key == "main" else plain["kt"])["trajectory"][1] / args.steps  # per pass
            r["value_with_fft"] = traj_steps / ((tr_ms + r["fft_ms"]) / 1e3)
            out["fft_fourier"][key] = r
        out["fft_fourier"]["note"] = ("exact FFT autocorrelation form of the Fourier step (scivr_accumulate_spectrum_fft) "
                                      "on one batch of identical trajectories; value_with_fft = trajectory-steps/s "
                                      "with the measured trajectory kernel time and the FFT form in place of the GEMM")
    if args.next_rows and prob.F <= 16:
        # separate lines for the rows beyond the single-state, separable path
        for key, fn in (("several_references", refs_form), ("double_time_form", full_form_study)):
            try:
                out[key] = fn(scivr, torch, inputs)
            except Exception as e:  # reported in the line instead of losing the headline
                out[key] = {"error": f"{type(e).__name__}: {e}"}
    if args.cpu_sample > 0:
        print(f"[bench] cpu baseline: oracle on {args.cpu_sample} trajectories", file=sys.stderr, flush=True)
        pprob = prob.replace(precision=inputs.PRECISION_FP64)
        out["cpu_baseline"] = cpu_baseline(pprob, args.cpu_sample, seed=77, n_single=args.cpu_single)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
