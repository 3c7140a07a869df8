"""Benchmark of the FW-H far-field hot path on one MI355X.

Workload: convected dipole, 32768-panel sphere (128 x 256), 2048 source samples,
360 observers every 1 deg at radius 100, M0 0.5, AoA 10 deg (FP64 surface data,
analytic, seeded).  One step = setup (pair delays, observer windows, pair
tables) + forward (source terms, derivatives, spline coefficients, gather-sum
over panels) + adjoint (transposed gather, source-stage transpose, chain rule)
of J = sum p'^2, i.e. every stage of the path, on inputs already resident in
HBM.  value = U / step time with U = P * sum_o N_t(o) panel-observer-samples.

Also reported: the plain FP64 GPU form on the same step, BF16 coefficient
storage, per-stage HIP-event timings, the roofline of the dominant kernel and
the FP64 CPU oracle timed on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK = 8.0e12                 # B/s, MI355X HBM3E
FP32_VALU_PEAK = 256 * 4 * 16 * 2 * 2.4e9   # 78.6 TFLOP/s: non-packed FP32 FMA (packed FP32 is not used)
FP32_PACKED_PEAK = 157.3e12       # published FP32 vector peak (needs packed FP32 FMA)
FLOP_PER_UNIT = 24                # 8 FMA channel combine + 4 FMA taps per (panel, observer, sample)


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def rel_l2(a, b, mask):
    a = np.asarray(a, dtype=np.float64) * mask
    b = np.asarray(b, dtype=np.float64) * mask
    return float(np.sqrt(np.sum((a - b) ** 2) / np.sum(b * b)))


def run_steps(plan, d, steps, sync):
    """`steps` full steps (setup + forward + adjoint of J = sum p'^2)."""
    for _ in range(steps):
        plan.setup()
        p = plan.forward(*d)
        plan.adjoint(*d, 2.0 * p)
    sync()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--plain-steps", type=int, default=2)
    ap.add_argument("--cpu-seconds", type=float, default=15.0, help="target CPU time of the oracle sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--profile-run", action="store_true",
                    help="short run for rocprofv3: 1 warmup + `--steps` FP32 steps, then a 1 GiB device copy "
                         "(the reference kernel for HBM byte counters); prints no JSON")
    ap.add_argument("--mode", default="f32", choices=["f32", "bf16"], help="mode of the profile run")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}, WORLD_SIZE {world}); this build has no "
              "multi-GPU path.", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2312_16263_amd as fwh
    from workloads import configs

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    c = configs.dipole_sphere()
    log(f"[bench] {fwh.version()}; workload {c.name}: P={c.n_panels} O={c.n_obs} N={c.n_tau}")
    t0 = time.time()
    rho, u, pp = c.data()
    d = [torch.from_numpy(a).to(dev) for a in (rho, u, pp)]
    torch.cuda.synchronize()
    log(f"[bench] inputs generated and resident in HBM ({time.time() - t0:.1f} s)")

    sync = torch.cuda.synchronize
    if args.profile_run:
        plan = fwh.Plan(c.surface.y, c.surface.normal, c.surface.dS, c.x_obs, c.mach, c.aoa_deg, c.dtau, c.tau0,
                        c.n_tau, mode=args.mode)
        run_steps(plan, d, 1 + args.steps, sync)
        src = torch.empty(1 << 28, dtype=torch.float32, device=dev).fill_(1.0)
        dst = torch.empty_like(src)
        dst.copy_(src)
        sync()
        log(f"[bench] profile run done: {1 + args.steps} steps ({args.mode}), then a 1 GiB copy")
        return
    plan = fwh.Plan(c.surface.y, c.surface.normal, c.surface.dS, c.x_obs, c.mach, c.aoa_deg, c.dtau, c.tau0,
                    c.n_tau, mode="f32")
    nt = plan.window.n_t
    U = int(c.n_panels * int(nt.sum()))
    run_steps(plan, d, args.warmup, sync)
    plan.profile_read()
    plan.profile(True)
    sync()
    t0 = time.perf_counter()
    run_steps(plan, d, args.steps, sync)
    t1 = time.perf_counter()
    plan.profile(False)
    stages = plan.profile_read()
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    value = U / (ms_per_step * 1e-3)
    log(f"[bench] f32: {ms_per_step:.3f} ms/step, {value:.3e} units/s")
    avg = {k: (v[0] / v[1] if v[1] else 0.0) for k, v in stages.items()}
    per_launch = {k: (v[0] / v[1] if v[1] else None) for k, v in stages.items()}

    # accuracy of this launch configuration against the FP64 oracle on sampled observers
    import oracle
    sample_obs = np.array([0, 90, 180, 270])
    p32 = plan.forward(*d).double().cpu().numpy()
    t_o = time.perf_counter()
    p_ref, _, nt_ref = oracle.forward(c.surface, c.x_obs, c.mach, c.aoa_deg, c.dtau, c.tau0, rho, u, pp,
                                      obs_idx=sample_obs)
    t_o = time.perf_counter() - t_o
    mask = (np.arange(p_ref.shape[1])[None, :] < nt_ref[sample_obs][:, None]).astype(float)
    err32 = rel_l2(p32[sample_obs], p_ref, mask)
    log(f"[bench] f32 rel L2 vs FP64 oracle on observers {sample_obs.tolist()}: {err32:.3e}")

    # BF16 coefficient storage
    plan_b = fwh.Plan(c.surface.y, c.surface.normal, c.surface.dS, c.x_obs, c.mach, c.aoa_deg, c.dtau, c.tau0,
                      c.n_tau, mode="bf16")
    run_steps(plan_b, d, 2, sync)
    tb = time.perf_counter()
    run_steps(plan_b, d, max(2, args.steps // 2), sync)
    ms_b = (time.perf_counter() - tb) * 1e3 / max(2, args.steps // 2)
    errb = rel_l2(plan_b.forward(*d).double().cpu().numpy()[sample_obs], p_ref, mask)
    del plan_b
    log(f"[bench] bf16: {ms_b:.3f} ms/step, err {errb:.3e}")

    plain = None
    if not args.no_plain:
        plan64 = fwh.Plan(c.surface.y, c.surface.normal, c.surface.dS, c.x_obs, c.mach, c.aoa_deg, c.dtau, c.tau0,
                          c.n_tau, mode="f64")
        run_steps(plan64, d, 1, sync)
        plan64.profile(True)
        tp = time.perf_counter()
        run_steps(plan64, d, args.plain_steps, sync)
        ms64 = (time.perf_counter() - tp) * 1e3 / args.plain_steps
        st64 = plan64.profile_read()
        err64 = rel_l2(plan64.forward(*d).cpu().numpy()[sample_obs], p_ref, mask)
        del plan64
        plain = {"value": U / (ms64 * 1e-3), "ms_per_step": ms64, "err_vs_oracle": err64,
                 "stage_ms": {k: (v[0] / v[1] if v[1] else None) for k, v in st64.items()}}
        log(f"[bench] plain f64: {ms64:.3f} ms/step, err {err64:.3e}")

    # roofline of the dominant kernel (the larger of the two gathers), FP32 VALU bound
    dom = "gather" if avg["gather"] >= avg["adj_gather"] else "adj_gather"
    t_dom = avg[dom] * 1e-3
    achieved = FLOP_PER_UNIT * U / t_dom / 1e12
    roofline = {"bound": "alu", "kernel": "gather_tuned_kernel<float>" if dom == "gather" else
                "adj_gather_tuned_kernel", "achieved": achieved, "peak": FP32_VALU_PEAK / 1e12, "unit": "TFLOP/s",
                "frac": achieved * 1e12 / FP32_VALU_PEAK, "traffic": None,
                "frac_of_packed_fp32_peak": achieved * 1e12 / FP32_PACKED_PEAK,
                "flop_per_unit": FLOP_PER_UNIT, "units_per_launch": U, "avg_launch_ms": avg[dom]}
    # source stage: HBM-bound streaming (inputs read once, coefficients written once)
    NS = ((c.n_tau + 12 + 63) // 64) * 64
    src_bytes = 5 * 8 * c.n_panels * c.n_tau + 8 * 4 * c.n_panels * NS
    src = {"bound": "hbm", "kernel": "source_fwd_kernel", "achieved": src_bytes / (avg["source"] * 1e-3) / 1e9,
           "peak": HBM_PEAK / 1e9, "unit": "GB/s", "algorithmic_bytes": src_bytes, "avg_launch_ms": avg["source"]}
    src["frac"] = src["achieved"] * 1e9 / HBM_PEAK

    cpu = None
    if not args.no_cpu_baseline:
        # oracle forward + adjoint (the same step) on a bounded observer sample
        def oracle_step(idx):
            xs = c.x_obs[idx]
            t = time.perf_counter()
            pr, _, ntr = oracle.forward(c.surface, xs, c.mach, c.aoa_deg, c.dtau, c.tau0, rho, u, pp)
            oracle.adjoint(c.surface, xs, c.mach, c.aoa_deg, c.dtau, c.tau0, rho, u, pp, 2.0 * pr)
            return time.perf_counter() - t, int(c.n_panels * int(ntr.sum()))
        t1o, _ = oracle_step(np.array([0]))
        n_s = int(min(c.n_obs, max(1, round(args.cpu_seconds / max(t1o, 1e-3)))))
        idx = np.unique(np.linspace(0, c.n_obs - 1, n_s).round().astype(int))
        t_cpu, u_cpu = oracle_step(idx)
        cpu = {"value": u_cpu / t_cpu, "unit": "panel-obs-samples/s", "cores": oracle.num_threads(), "kind": "oracle",
               "sample": f"forward + adjoint of the FP64 oracle on {len(idx)} of {c.n_obs} observers (all "
                         f"{c.n_panels} panels, {c.n_tau} samples): {u_cpu:.3e} units in {t_cpu:.1f} s; "
                         f"excludes input generation", "seconds": t_cpu}
        log(f"[bench] cpu oracle: {cpu['value']:.3e} units/s on {cpu['cores']} threads")

    out = {
        "metric": "FW-H panel-obs-samples/s (fwd, adjoint) vs FP64 plain at stated err; % HBM peak",
        "value": value, "unit": "panel-obs-samples/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms_per_step, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": "convected dipole (axis x2), sphere r=1 128x256=32768 panels, N=2048 at dtau=1/256, "
                              "360 observers every 1 deg at r=100, M0=0.5, AoA=10 deg; FP64 analytic surface data; "
                              "step = setup + forward + adjoint",
                   "panels": c.n_panels, "samples": c.n_tau, "observers": c.n_obs, "units_per_step": U},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "err_vs_oracle": err32,
        "stage_ms_per_launch": per_launch,
        "fwd_units_per_s": U / ((avg["source"] + avg["gather"] + avg["reduce"]) * 1e-3),
        "adj_units_per_s": U / ((avg["adj_gather"] + avg["source_adj"]) * 1e-3),
        "source_roofline": src,
        "bf16_storage": {"value": U / (ms_b * 1e-3), "ms_per_step": ms_b, "err_vs_oracle": errb},
        "plain_f64": plain,
        "speedup_vs_plain_f64": (value / plain["value"]) if plain else None,
        "oracle_sampled_forward_s": t_o,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
