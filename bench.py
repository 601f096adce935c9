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


def fourier_flops(n_traj: int, n_times: int, K: int) -> float:
    """8 flops per complex multiply-add of amp[j][c] exp(i E_k c dt)."""
    return 8.0 * n_traj * n_times * K


def _source_hash(*names):
    h = hashlib.sha256()
    for nm in names:
        with open(os.path.join(ROOT, "paper_1312_4698_amd", "csrc", nm), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def _profile_traffic(kernel_prefix: str, src_hash: str):
    """HBM bytes per launch from a committed rocprofv3 counter summary, if it
    was taken on the current kernel source; else None."""
    path = os.path.join(ROOT, "profiles", f"traj_{kernel_prefix}_counters.txt")
    if not os.path.exists(path):
        return None
    txt = open(path).read()
    m = re.search(r"source_hash:\s*(\w+)", txt)
    b = re.search(r"hbm_bytes_per_launch:\s*([0-9.eE+]+)", txt)
    if not m or not b or m.group(1) != src_hash:
        return None
    return float(b.group(1))


def cpu_baseline(prob, n_sample: int, seed: int):
    """The oracle as it stands, on all host cores, over a bounded sample."""
    from oracle import oracle as O
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    p0, q0, lr = O.sample_husimi(prob, seed, n_sample)
    t0 = time.perf_counter()
    O.run(prob, p0, q0, lr, want_state=False, want_contrib=False, n_threads=threads)
    dt = time.perf_counter() - t0
    return {"value": n_sample * prob.n_steps / dt, "unit": "trajectory-steps/s", "cores": threads,
            "kind": "oracle",
            "sample": f"{n_sample} trajectories of the same workload (all {prob.n_steps} steps, "
                      f"{prob.n_energies} energies), {dt:.1f} s wall"}


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


def run_form(scivr, torch, prob, n, steps, warmup, seed0=1000, chunk=0, energy=None):
    """Time `steps` whole passes (sample + propagate + accumulate) of one form."""
    stream = torch.cuda.current_stream()
    ctx = scivr.Context(prob, max_traj=n)

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


def _peak_error_cm(peaks, inputs, E, T, ref_peaks, I):
    """Largest peak shift (cm^-1) of I against the reference peaks; inf if a peak is missing."""
    pt = peaks.find_peaks(E, I, T)
    worst, missing = peaks.peak_errors(ref_peaks, pt, tol=20.0 / inputs.CM1_PER_HARTREE)
    return float("inf") if missing else worst * inputs.CM1_PER_HARTREE


def learned_study(scivr, inputs, peaks, prob, ref_I, sizes, seeds, n_train, layers, width, epochs, batch, lr,
                  alpha):
    """Trajectories needed for a 1 cm^-1 peak error against the reference spectrum,
    plain Husimi sampling vs the learned proposal, in the given form of `prob`.

    For each seed and each N in `sizes` an independent batch of N trajectories
    (Philox indices disjoint from the reference run's) gives a spectrum; its largest
    peak shift against the reference is recorded; N_to_1cm is the smallest N whose
    median shift over the seeds is <= 1 cm^-1.  The flow is trained once on the
    contributions of a Husimi batch of n_train trajectories.
    """
    E, T = prob.energies(), prob.total_time
    jp = peaks.find_peaks(E, ref_I, T)
    cap = max(max(sizes), n_train)
    ctx = scivr.Context(prob, max_traj=cap)
    base = 1 << 40  # Philox indices far from the reference run's

    def sweep(draw):
        errs = np.zeros((len(seeds), len(sizes)))
        rms = np.zeros_like(errs)
        for a, sd in enumerate(seeds):
            for b, N in enumerate(sizes):
                ctx.reset_spectrum()
                draw(sd, N)
                ctx.propagate()
                ctx.accumulate()
                I, _, _ = ctx.read_spectrum()
                errs[a, b] = _peak_error_cm(peaks, inputs, E, T, jp, I)
                rms[a, b] = float(np.sqrt(np.mean((I - ref_I) ** 2)) / ref_I.max())
        med = np.median(errs, axis=0)
        # smallest N from which on every larger N of the sweep also meets 1 cm^-1
        n1 = None
        for b in range(len(sizes) - 1, -1, -1):
            if med[b] <= 1.0:
                n1 = sizes[b]
            else:
                break
        return {"N_to_1cm": n1, "median_peak_error_cm1": med.tolist(),
                "median_rel_rms": np.median(rms, axis=0).tolist()}

    t0 = time.perf_counter()
    plain = sweep(lambda sd, N: ctx.sample_husimi(seed=sd, n_traj=N, first_index=base))
    t_plain = time.perf_counter() - t0
    flow = scivr.Flow(ctx, layers, width, seed=5)
    ctx.reset_spectrum()
    ctx.run(seed=4242, n_traj=n_train, first_index=2 * base)
    t0 = time.perf_counter()
    loss = flow.train_on_batch(epochs=epochs, batch=batch, lr=lr)
    t_train = time.perf_counter() - t0
    info = {}

    def draw_flow(sd, N):
        ess, used = flow.sample(seed=sd, n_traj=N, first_index=base, alpha=alpha)
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
        "sizes": list(sizes), "seeds": list(seeds), "ref_peaks_cm1": [e * inputs.CM1_PER_HARTREE for e, _ in jp],
        "plain": plain, "learned": learned,
        "flow": {"layers": layers, "width": width, "params": int(FLOW_PARAMS(prob.F, width, layers)),
                 "n_train": n_train, "epochs": epochs, "batch": batch, "lr": lr, "alpha": alpha,
                 "final_loss": loss, "train_s": t_train, "ess_min": float(min(info["ess"])),
                 "ess_median": float(np.median(info["ess"])), "fallbacks": int(sum(1 for u in info["used"] if not u))},
        "sweep_s": {"plain": t_plain, "learned": t_learned},
    }


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
    ap.add_argument("--chunk", type=int, default=0,
                    help="propagate in calls of this many time steps, printing progress (0: one call)")
    ap.add_argument("--copy-calibration", type=int, default=0,
                    help="only copy this many bytes device-to-device (counter calibration) and exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "only one GPU is supported: the path shards by trajectory index (first_index "
                                   "ranges) with one all-reduce of the K-vector, but no multi-GPU run is provided",
                          "n_gpus": args.gpus}))
        sys.exit(2)

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
    prob, n = inputs.workload(args.workload)
    if args.n_traj:
        n = args.n_traj
    print(f"[bench] {args.workload}: F={prob.F} n={n} steps={prob.n_steps} K={prob.n_energies}", file=sys.stderr,
          flush=True)
    energy = _energy_reader()
    main_run = run_form(scivr, torch, prob, n, args.steps, args.warmup, chunk=args.chunk, energy=energy)
    plain = None
    if args.plain:
        pprob, _ = inputs.workload(args.plain)
        plain = run_form(scivr, torch, pprob, n, args.steps, args.warmup, chunk=args.chunk, energy=energy)

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
    src_hash = _source_hash("traj_big.hip" if big else "traj.hip", "traj_common.h")
    traffic = _profile_traffic(prob.name, src_hash)
    fo_launch = ms_fo / max(n_fo, 1) / 1e3
    fo_fl = fourier_flops(n, prob.n_steps + 1, prob.n_energies)
    mixed = prob.precision == inputs.PRECISION_MIXED

    out = {
        "metric": "trajectory-steps/s at F=9",
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
        "n_good_fraction": main_run["n_good"] / max(main_run["n_total"], 1),
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
                                                seeds=(11, 12, 13, 14, 15),
                                                n_train=65536, layers=4, width=128, epochs=20, batch=4096, lr=1e-3,
                                                alpha=0.1)
        out["learned_proposal"]["reference"] = (f"plain FP64 spectrum of the timed run: {args.steps} batches of {n} "
                                            f"Husimi trajectories")
        lp = out["learned_proposal"]
        vp, vm = out["plain_fp64"]["value"], value
        n_plain, n_learn = lp["plain"]["N_to_1cm"], lp["learned"]["N_to_1cm"]
        train_s = lp["flow"]["train_s"] + lp["flow"]["n_train"] * prob.n_steps / vm
        out["time_to_1cm"] = {
            "plain_fp64_s": None if n_plain is None else n_plain * prob.n_steps / vp,
            "plain_fp64_lower_bound_s": sizes[-1] * prob.n_steps / vp if n_plain is None else None,
            "mixed_learned_s": None if n_learn is None else n_learn * prob.n_steps / vm + train_s,
            "mixed_learned_training_s": train_s,
            "equal_variance_speedup": lp["variance_ratio_plain_over_learned"] * vm / vp,
            "equal_variance_energy_ratio": (
                None if not (out["energy"] and out["plain_fp64"]["energy"]) else
                lp["variance_ratio_plain_over_learned"] * out["plain_fp64"]["energy"]["J_per_step"]
                / out["energy"]["J_per_step"]),
            "note": ("plain: FP64 path with Husimi sampling; mixed_learned: mixed path with the learned proposal, "
                     "including its training batch and training time; equal_variance_speedup = (plain/learned "
                     "spectrum variance at equal N) x (mixed/plain throughput)"),
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
    if args.cpu_sample > 0:
        print(f"[bench] cpu baseline: oracle on {args.cpu_sample} trajectories", file=sys.stderr, flush=True)
        pprob = prob.replace(precision=inputs.PRECISION_FP64)
        out["cpu_baseline"] = cpu_baseline(pprob, args.cpu_sample, seed=77)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
