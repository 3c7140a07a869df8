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
FP32_PEAK = 157.3e12              # published FP32 vector peak of MI355X (reached only with packed FP32 FMA)
FP32_NONPACKED_PEAK = 256 * 4 * 16 * 2 * 2.4e9   # 78.6 TFLOP/s: FP32 FMA without packing (packed FP32 is not used)
FLOP_PER_UNIT = 24                # 8 FMA channel combine + 4 FMA taps per (panel, observer, sample)
TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "hbm_traffic_dipole32768_f32.md")
GM_TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "hbm_traffic_general_motion_orbit8192_f64.md")
LOWO_TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "hbm_traffic_dipole32768_obs8.md")


def measured_traffic(kernel, path=TRAFFIC_PROFILE):
    """HBM bytes per launch of `kernel` (read + written, copy-calibrated) from the
    committed rocprofv3 FETCH_SIZE / WRITE_SIZE summary, or None.  A name `k<T>` also
    takes the rows `k<T, s>` of its wave shapes s (one launch each per gather), summed."""
    total, found = 0.0, False
    shaped = kernel[:-1] + ", " if kernel.endswith(">") else None
    try:
        with open(path) as f:
            for line in f:
                cells = [c.strip() for c in line.strip().strip("|").split("|")]
                if len(cells) != 5:
                    continue
                name = cells[0].strip("`")
                if name == kernel or (shaped and name.startswith(shaped)):
                    total += (float(cells[3]) + float(cells[4])) * 1e9
                    found = True
    except (OSError, ValueError):
        return None
    return total if found else None


GATHER_KERNELS = {"lds": "gather_lds_kernel", "stream": "gather_stream_kernel", "mfma": "gather_mfma_kernel",
                  "direct": "gather_tuned_kernel"}


def gather_kernel(plan, mode):
    """Name of the forward gather kernel the plan runs, as the traffic summaries list it."""
    kind = plan.info()[0]
    name = GATHER_KERNELS.get(kind, "gather_f64_kernel")
    if kind in ("lds", "stream", "mfma"):
        name += "<float>" if mode == "f32" else "<unsigned short>"
    return name


def gm_traffic():
    """HBM bytes of one general-motion gather launch (gather + panel-range sum), or None."""
    g = measured_traffic("gm_gather_kernel", GM_TRAFFIC_PROFILE)
    r = measured_traffic("gm_reduce_kernel", GM_TRAFFIC_PROFILE)
    return None if g is None or r is None else g + r


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def rel_l2(a, b, mask):
    a = np.asarray(a, dtype=np.float64) * mask
    b = np.asarray(b, dtype=np.float64) * mask
    return float(np.sqrt(np.sum((a - b) ** 2) / np.sum(b * b)))


def bench_low_obs(c_full, d, steps, sync, n_obs=8):
    """The dipole sphere's surface and data with 8 observers (every 45 deg at r =
    100): 8 coefficient channels of 4 (FP32) or 2 (BF16) bytes per sample serve
    only 8 observers, so the forward gather reads about 4 (2) bytes per unit
    against 24 flop and is bound by HBM.  Reports the gather's algorithmic bytes
    (coefficients read once, 52 B of pair table per pair, the output) over its
    HIP-event time against the 8 TB/s peak."""
    import torch

    import paper_2312_16263_amd as fwh
    from workloads import configs
    c = configs.dipole_sphere(n_obs=n_obs)
    out = {"workload": f"dipole sphere (32768 panels, N=2048, M0=0.5, AoA 10 deg) with {n_obs} observers every "
                       f"{360 // n_obs} deg at r=100; forward only"}
    for mode, esz in (("f32", 4), ("bf16", 2)):
        plan = fwh.Plan(c.surface.y, c.surface.normal, c.surface.dS, c.x_obs, c.mach, c.aoa_deg, c.dtau, c.tau0,
                        c.n_tau, mode=mode)
        U = int(c.n_panels * int(plan.window.n_t.sum()))
        p = plan.forward(*d)
        sync()
        plan.profile(True)
        for _ in range(steps):
            plan.forward(*d, out=p)
        sync()
        st = plan.profile_read()
        g_ms = st["gather"][0] / st["gather"][1]
        r_ms = st["reduce"][0] / st["reduce"][1]
        s_ms = st["source"][0] / st["source"][1]
        alg = 8 * esz * (c.n_tau + 3) * c.n_panels + 52 * n_obs * c.n_panels + 4 * int(plan.window.n_t.sum())
        gbs = alg / (g_ms * 1e-3)
        kern = gather_kernel(plan, mode)
        out[mode] = {"units": U, "gather_ms": g_ms, "reduce_ms": r_ms, "source_ms": s_ms,
                     "gather_units_per_s": U / (g_ms * 1e-3),
                     "roofline": {"bound": "hbm", "kernel": kern, "achieved": gbs / 1e9, "peak": HBM_PEAK / 1e9,
                                  "unit": "GB/s", "frac": gbs / HBM_PEAK, "algorithmic_bytes": alg,
                                  "traffic": measured_traffic(kern, LOWO_TRAFFIC_PROFILE)},
                     "gather": plan.info()}
        log(f"[bench] {n_obs} observers {mode}: gather {g_ms:.3f} ms ({gbs / 1e9:.0f} GB/s algorithmic, "
            f"{gbs / HBM_PEAK:.2f} of HBM peak), reduce {r_ms:.3f} ms, source {s_ms:.3f} ms, {plan.info()}")
        del plan, p
        torch.cuda.empty_cache()
    return out


def run_steps(plan, d, steps, sync):
    """`steps` full steps (setup + forward + adjoint of J = sum p'^2)."""
    for _ in range(steps):
        plan.setup()
        p = plan.forward(*d)
        plan.adjoint(*d, 2.0 * p)
    sync()


def bench_airfoil(steps, sync):
    """Airfoil-like extruded Joukowski surface with broadband data (240000
    panels, 4096 samples, 72 observers), FP32 and BF16 coefficient storage:
    step time and error against the FP64 oracle on two sampled observers."""
    import torch

    import oracle
    import paper_2312_16263_amd as fwh
    from workloads import configs
    c = configs.airfoil_broadband()
    log(f"[bench] airfoil: P={c.n_panels} O={c.n_obs} N={c.n_tau}")
    d = c.data_device("cuda")
    sync()
    host = [t.cpu().numpy() for t in d]
    sample = np.array([0, 36])
    p_ref, _, nt_ref = oracle.forward(c.surface, c.x_obs, c.mach, c.aoa_deg, c.dtau, c.tau0, *host, obs_idx=sample)
    del host
    out = {"workload": "Joukowski contour (1200 points, chord 1) x 200 stations = 240000 panels, N=4096, 72 "
                       "observers at R=10, M0=0.17, AoA=5.5 deg; seeded broadband FP32 data (k^-5/3, RMS 1%)"}
    for mode in ("f32", "bf16"):
        plan = fwh.Plan(c.surface.y, c.surface.normal, c.surface.dS, c.x_obs, c.mach, c.aoa_deg, c.dtau, c.tau0,
                        c.n_tau, mode=mode)
        U = int(c.n_panels * int(plan.window.n_t.sum()))
        run_steps(plan, d, 1, sync)
        plan.profile(True)
        t0 = time.perf_counter()
        run_steps(plan, d, steps, sync)
        ms = (time.perf_counter() - t0) * 1e3 / steps
        st = plan.profile_read()
        p = plan.forward(*d).double().cpu().numpy()[sample]
        m = (np.arange(p_ref.shape[1])[None, :] < nt_ref[sample][:, None]).astype(float)
        err = rel_l2(p, p_ref, m)
        out[mode] = {"value": U / (ms * 1e-3), "ms_per_step": ms, "err_vs_oracle": err,
                     "stage_ms": {k: (v[0] / v[1] if v[1] else None) for k, v in st.items()}}
        log(f"[bench] airfoil {mode}: {ms:.2f} ms/step, {U / (ms * 1e-3):.3e} units/s, err {err:.3e}")
        if mode == "f32":
            # post-processing of Sec. IV C on the device: RMS and Welch PSD (1024-sample Hann segments, 50 %
            # overlap, spanwise correction 650 / 50.8) of all observers, against the oracle on the sample
            from oracle import post
            pt = plan.forward(*d)
            seg, span = 1024, 650.0 / 50.8
            plan.post(pt, seg, span)
            sync()
            t0 = time.perf_counter()
            for _ in range(5):
                psd, rms = plan.post(pt, seg, span)
            sync()
            ms_post = (time.perf_counter() - t0) * 1e3 / 5
            pn = pt.double().cpu().numpy()[sample]
            nts = plan.window.n_t[sample]
            e_psd = rel_l2(psd.double().cpu().numpy()[sample], post.welch_all(pn, nts, c.dtau, seg, span),
                           np.ones((len(sample), seg // 2 + 1)))
            e_rms = rel_l2(rms.double().cpu().numpy()[sample][:, None], post.rms(pn, nts)[:, None],
                           np.ones((len(sample), 1)))
            out["post"] = {"seg_len": seg, "span_ratio": span, "ms": ms_post, "psd_err_vs_oracle": e_psd,
                           "rms_err_vs_oracle": e_rms}
            log(f"[bench] airfoil post (RMS + Welch PSD, L={seg}): {ms_post:.3f} ms, errs {e_psd:.2e} {e_rms:.2e}")
        out["units_per_step"] = U
        del plan
        torch.cuda.empty_cache()
    del d
    torch.cuda.empty_cache()
    return out


GM_FLOP_PER_UNIT = 402  # final evaluation 222 (19 channels x 4 taps, weights, integrand) + 2 Newton steps x 90


def bench_general_motion(steps, sync, profile_only=False):
    """General-motion form (Sec. II B): a 64 x 128 sphere (8192 panels) spinning
    about an axis off its centre around a still-air monopole, 1024 frames, 72
    observers at rest; FP64.  Forward time (channels + spline coefficients,
    retarded-time gather), throughput, roofline of the gather (FP64 VALU),
    error against the oracle on sampled outputs and against the closed form."""
    import torch

    import oracle
    import paper_2312_16263_amd as fwh
    from workloads import motion
    c = motion.orbiting_sphere_case()
    dv = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()
    plan = fwh.GMPlan(dv(c.ms.y), dv(c.ms.normal), dv(c.ms.vel), dv(c.ms.dS), dv(c.x_obs), c.mach, c.dtau, c.tau0)
    data = [dv(c.rho), dv(c.u), dv(c.pp)]
    P, O, N = plan.P, plan.O, plan.N
    U = int(P * int(plan.window.n_t.sum()))
    log(f"[bench] general motion: P={P} O={O} N={N}, {U:.3e} units per forward")
    p = plan.forward(*data)
    sync()
    if profile_only:
        for _ in range(steps):
            plan.forward(*data, out=p)
        sync()
        return None
    plan.profile(True)
    t0 = time.perf_counter()
    for _ in range(steps):
        plan.forward(*data, out=p)
    sync()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    st = plan.profile_read()
    src_ms = st["source"][0] / max(st["source"][1], 1)
    gat_ms = st["gather"][0] / max(st["gather"][1], 1)
    ph = p.cpu().numpy()
    rng = np.random.default_rng(11)
    so = rng.integers(0, O, 24)
    sk = np.array([rng.integers(0, plan.window.n_t[o]) for o in so])
    ref = oracle.gm_forward_samples(c.ms, c.x_obs, c.mach, c.dtau, c.tau0, c.rho, c.u, c.pp, so, sk)
    err = float(np.abs(ph[so, sk] - ref).max() / np.abs(ref).max())
    t = plan.window.t_start[:, None] + c.dtau * np.arange(ph.shape[1])[None, :]
    ex = c.exact(t)
    m = (np.arange(ph.shape[1])[None, :] < plan.window.n_t[:, None]).astype(float)
    err_exact = rel_l2(ph, ex, m)
    achieved = GM_FLOP_PER_UNIT * U / (gat_ms * 1e-3) / 1e12
    out = {"workload": "sphere r=1.2 (64x128 = 8192 panels) centred at (0.3,0,0) spinning at 0.5 about the z axis "
                       "around a still-air monopole (w = 2 pi), N=1024 at dtau=1/128, 72 observers at r=20, z=3, "
                       "M0=0.3; FP64; forward = channels + spline coefficients + retarded-time gather",
           "units_per_forward": U, "ms_per_forward": ms, "value": U / (ms * 1e-3), "unit": "panel-obs-samples/s",
           "stage_ms": {"source": src_ms, "gather": gat_ms},
           "err_vs_oracle_sampled": err, "err_vs_closed_form": err_exact,
           "roofline": {"bound": "alu", "kernel": "gm_gather_kernel + gm_reduce_kernel", "achieved": achieved,
                        "peak": 78.6432, "unit": "TFLOP/s", "frac": achieved / 78.6432,
                        "flop_per_unit": GM_FLOP_PER_UNIT, "units_per_launch": U, "avg_launch_ms": gat_ms,
                        "traffic": gm_traffic(),
                        "traffic_unit": "bytes per launch (HBM, rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)"}}
    log(f"[bench] general motion: {ms:.2f} ms/forward (source {src_ms:.2f}, gather {gat_ms:.2f}), "
        f"{U / (ms * 1e-3):.3e} units/s, err vs oracle {err:.2e}, vs closed form {err_exact:.2e}")
    del plan, data, p
    torch.cuda.empty_cache()
    return out


def bench_batch(replays, sync):
    """64 seeded uneven cases (spheres with analytic sources, extruded contours
    with broadband data; P 2048-65536, N 512-4096, O 8-360, M0 0.1-0.5, AoA
    0-10 deg), BF16 storage, FP32 inputs: one step (forward, dJ/dp', adjoint)
    of all cases as one HIP-graph replay, tiles tuned per class of case sizes,
    against 64 separate plain FP64 steps."""
    import torch

    import paper_2312_16263_amd as fwh
    from workloads import configs
    cases = configs.batched_cases()
    t0 = time.time()
    inputs = [c.data_device("cuda") for c in cases]
    sync()
    log(f"[bench] batch: {len(cases)} cases generated on the device ({time.time() - t0:.1f} s), "
        f"{torch.cuda.memory_allocated() / 1e9:.1f} GB")
    plans = [fwh.Plan(c.surface.y, c.surface.normal, c.surface.dS, c.x_obs, c.mach, c.aoa_deg, c.dtau, c.tau0,
                      c.n_tau, mode="bf16") for c in cases]
    batch = fwh.Batch(plans, inputs)
    log(f"[bench] batch: plans and batch bound, {torch.cuda.memory_allocated() / 1e9:.1f} GB; gather {batch.gather}")
    t0 = time.time()
    tune = fwh.autotune(batch, reps=1)
    log(f"[bench] batch: autotune {time.time() - t0:.1f} s: " +
        "; ".join(f"{k} ({v['cases']}) -> rows {v['choice'][0]}, {v['choice'][1]:.0e}" for k, v in tune["classes"].items())
        + f"; {tune['blocks_per_cu']} blocks/CU")
    info = batch.info()
    graph = batch.capture()
    graph.replay()
    sync()
    t0 = time.perf_counter()
    for _ in range(replays):
        graph.replay()
    sync()
    ms = (time.perf_counter() - t0) * 1e3 / replays
    # forward and adjoint apart (eager, HIP events around each)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    ev[0].record()
    batch.forward()
    ev[1].record()
    batch.adjoint()
    ev[2].record()
    sync()
    fwd_ms, adj_ms = ev[0].elapsed_time(ev[1]), ev[1].elapsed_time(ev[2])
    # the same adjoint as 64 single-case launches: HIP events around all of them back to back, and the
    # sum of their transposed-gather and source-adjoint stage times (kernel time without launch gaps)
    # (into the batch's own gradient buffers: the device has no room for a second set)
    for pl, d, gp, g in zip(plans, inputs, batch.grad_p, batch.grads):
        pl.adjoint(*d, gp, out=g)
    for pl in plans:
        pl.profile(True)
    ev[0].record()
    for pl, d, gp, g in zip(plans, inputs, batch.grad_p, batch.grads):
        pl.adjoint(*d, gp, out=g)
    ev[1].record()
    sync()
    adj_single_ms = ev[0].elapsed_time(ev[1])
    adj_single_stage_ms = 0.0
    for pl in plans:
        st = pl.profile_read()
        adj_single_stage_ms += st["adj_gather"][0] + st["source_adj"][0]
        pl.profile(False)
    p_b = [t.double().cpu().numpy() for t in batch.p_out]
    del graph, batch
    del plans
    torch.cuda.empty_cache()
    # 64 separate plain FP64 steps (setup + forward + adjoint per case)
    t_plain = 0.0
    errs = []
    for c, d, pb in zip(cases, inputs, p_b):
        plan = fwh.Plan(c.surface.y, c.surface.normal, c.surface.dS, c.x_obs, c.mach, c.aoa_deg, c.dtau, c.tau0,
                        c.n_tau, mode="f64")
        sync()
        t1 = time.perf_counter()
        run_steps(plan, d, 1, sync)
        t_plain += time.perf_counter() - t1
        p64 = plan.forward(*d).cpu().numpy()
        m = (np.arange(p64.shape[1])[None, :] < plan.window.n_t[:, None]).astype(float)
        errs.append(rel_l2(pb, p64, m))
        del plan
        torch.cuda.empty_cache()
    U = info["units"]
    out = {"workload": "64 seeded uneven cases (sphere monopole/dipole and extruded-contour broadband; P 2048-65536, "
                       "N 512-4096, O 8-360, M0 0.1-0.5, AoA 0-10 deg), BF16 storage, FP32 inputs",
           "panels": [c.n_panels for c in cases], "samples": [c.n_tau for c in cases],
           "observers": [c.n_obs for c in cases],
           "units_per_step": U, "ms_per_step": ms, "value": U / (ms * 1e-3),
           "forward_ms": fwd_ms, "adjoint_ms": adj_ms,
           "adjoint_64_single_launches_ms": adj_single_ms, "adjoint_64_single_stage_sum_ms": adj_single_stage_ms,
           "plain_f64_64_launches": {"ms_per_step": t_plain * 1e3, "value": U / t_plain},
           "speedup_vs_plain_f64": t_plain * 1e3 / ms, "max_rel_l2_vs_plain_f64": max(errs),
           "work_items": info["items"], "grid": info["grid"], "autotune": tune}
    log(f"[bench] batch: {ms:.2f} ms/step ({U / (ms * 1e-3):.3e} units/s; forward {fwd_ms:.1f} ms, adjoint "
        f"{adj_ms:.1f} ms; 64 single-case adjoints {adj_single_ms:.1f} ms, their kernels {adj_single_stage_ms:.1f} ms) "
        f"vs 64 plain FP64 steps {t_plain * 1e3:.1f} ms; max rel L2 vs FP64 {max(errs):.3e}")
    del inputs
    torch.cuda.empty_cache()
    return out


def bench_ingest(sync, n_frames=256, n_ascii=8, threads=16):
    """Ingestion of OpenCFD-FWH dataset files (Appendix A layouts) for the
    dipole workload's 32768 panels: n_frames binary frames (40 B per panel)
    written to a temporary directory, read by the library's threaded reader into
    page-locked FP64 host tensors, then copied to the device; a few ASCII
    frames for comparison.  The files were just written, so reads come from the
    page cache: this is parse + scatter speed, not disk speed."""
    import tempfile

    import torch

    from paper_2312_16263_amd import fileio
    from workloads import configs
    c = configs.dipole_sphere(n_tau=n_frames)
    rho, u, pp = c.data()
    dims = np.array([[128, 256, 1]], dtype=np.int64)
    P = c.n_panels
    out = {"workload": f"dipole sphere, {P} panels, one Face; {n_frames} binary frames, {n_ascii} ASCII frames; "
                       f"{threads} reader threads; warm page cache", "panels": P}
    with tempfile.TemporaryDirectory(prefix="fwh_ingest_") as d:
        for fmt, nf, key in ((fileio.BINARY, n_frames, "binary"), (fileio.ASCII, n_ascii, "ascii")):
            for k in range(nf):
                fileio.write_frame(fileio.frame_path(d, k), fmt, dims, rho[k], u[:, k], pp[k])
            nbytes = sum(os.path.getsize(fileio.frame_path(d, k)) for k in range(nf))
            host = (torch.empty((nf, P), dtype=torch.float64, pin_memory=True),
                    torch.empty((3, nf, P), dtype=torch.float64, pin_memory=True),
                    torch.empty((nf, P), dtype=torch.float64, pin_memory=True))
            fileio.read_frames(d, 0, 1, nf, fmt, dims, out=host, threads=threads)  # warm
            t0 = time.perf_counter()
            fileio.read_frames(d, 0, 1, nf, fmt, dims, out=host, threads=threads)
            t_read = time.perf_counter() - t0
            assert np.array_equal(host[1].numpy(), u[:, :nf])
            dev = [torch.empty_like(h, device="cuda") for h in host]
            for dv, h in zip(dev, host):  # first copy maps the pages; the timed one is the second
                dv.copy_(h, non_blocking=True)
            sync()
            t0 = time.perf_counter()
            for dv, h in zip(dev, host):
                dv.copy_(h, non_blocking=True)
            sync()
            t_h2d = time.perf_counter() - t0
            arr = 5 * nf * P * 8
            out[key] = {"frames": nf, "file_bytes": nbytes, "read_s": t_read, "file_GB_per_s": nbytes / t_read / 1e9,
                        "frames_per_s": nf / t_read, "h2d_s": t_h2d, "h2d_GB_per_s": arr / t_h2d / 1e9,
                        "read_plus_h2d_panel_frames_per_s": nf * P / (t_read + t_h2d)}
            log(f"[bench] ingest {key}: {nf} frames, {nbytes / 1e6:.1f} MB read in {t_read * 1e3:.1f} ms "
                f"({nbytes / t_read / 1e9:.2f} GB/s), H2D {arr / t_h2d / 1e9:.1f} GB/s")
            if fmt == fileio.BINARY:
                # files -> device in blocks of 128 frames, parsing overlapped with the copies
                fileio.read_frames_to_device(d, 0, 1, nf, fmt, dims, dtype="f64", block=128, threads=threads)
                sync()
                t0 = time.perf_counter()
                dv = fileio.read_frames_to_device(d, 0, 1, nf, fmt, dims, dtype="f64", block=128, threads=threads)
                sync()
                t_st = time.perf_counter() - t0
                assert torch.equal(dv[0].cpu(), host[0])
                out[key]["streamed_to_device_s"] = t_st
                out[key]["streamed_panel_frames_per_s"] = nf * P / t_st
                out[key]["streamed_file_GB_per_s"] = nbytes / t_st / 1e9
                log(f"[bench] ingest {key} streamed to HBM (blocks of 128 frames): {t_st * 1e3:.1f} ms "
                    f"({nbytes / t_st / 1e9:.2f} GB/s of file)")
                del dv
            for k in range(nf):
                os.remove(fileio.frame_path(d, k))
            del dev, host
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--plain-steps", type=int, default=2)
    ap.add_argument("--cpu-seconds", type=float, default=20.0, help="target CPU time of the oracle sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-extra", action="store_true", help="skip the airfoil and batched workloads")
    ap.add_argument("--profile-run", action="store_true",
                    help="short run for rocprofv3: 1 warmup + `--steps` FP32 steps, then a 1 GiB device copy "
                         "(the reference kernel for HBM byte counters); prints no JSON")
    ap.add_argument("--mode", default="f32", choices=["f32", "bf16"], help="mode of the profile run")
    ap.add_argument("--ingest-only", action="store_true", help="only the file-ingestion measurement (JSON line)")
    ap.add_argument("--workload", default="dipole_sphere",
                    choices=["dipole_sphere", "dipole_sphere_obs8", "airfoil_broadband", "general_motion"],
                    help="workload of the profile run")
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
    sync = torch.cuda.synchronize
    if args.ingest_only:
        print(json.dumps({"ingest": bench_ingest(sync)}), flush=True)
        return
    if args.profile_run and args.workload == "general_motion":
        bench_general_motion(args.steps, sync, profile_only=True)
        src = torch.empty(1 << 28, dtype=torch.float32, device=dev).fill_(1.0)
        dst = torch.empty_like(src)
        dst.copy_(src)
        sync()
        log(f"[bench] profile run done: 1 + {args.steps} general-motion forwards, then a 1 GiB copy")
        return
    if args.profile_run:
        c = configs.by_name(args.workload)
        log(f"[bench] profile run: workload {c.name}: P={c.n_panels} O={c.n_obs} N={c.n_tau}")
        d = list(c.data_device(dev))
        plan = fwh.Plan(c.surface.y, c.surface.normal, c.surface.dS, c.x_obs, c.mach, c.aoa_deg, c.dtau, c.tau0,
                        c.n_tau, mode=args.mode)
        run_steps(plan, d, 1 + args.steps, sync)
        src = torch.empty(1 << 28, dtype=torch.float32, device=dev).fill_(1.0)
        dst = torch.empty_like(src)
        dst.copy_(src)
        sync()
        log(f"[bench] profile run done: {1 + args.steps} steps ({args.mode}), then a 1 GiB copy")
        return
    c = configs.dipole_sphere()
    log(f"[bench] {fwh.version()}; workload {c.name}: P={c.n_panels} O={c.n_obs} N={c.n_tau}")
    t0 = time.time()
    rho, u, pp = c.data()
    d = [torch.from_numpy(a).to(dev) for a in (rho, u, pp)]
    torch.cuda.synchronize()
    log(f"[bench] inputs generated and resident in HBM ({time.time() - t0:.1f} s)")

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
    plan_info = plan.info()
    log(f"[bench] f32: {ms_per_step:.3f} ms/step, {value:.3e} units/s; forward gather {plan_info}")
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
    # and against the closed-form convected dipole (Sec. IV B) on all observers
    t_obs = plan.window.t_start[:, None] + c.dtau * np.arange(p32.shape[1])[None, :]
    err32_exact = rel_l2(p32, c.exact(t_obs), (np.arange(p32.shape[1])[None, :] < nt[:, None]).astype(float))
    log(f"[bench] f32 rel L2 vs the closed-form dipole, all observers: {err32_exact:.3e}")

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
    low_obs = bench_low_obs(c, d, max(5, args.steps // 2), sync)

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
    fwd_kernel = gather_kernel(plan, "f32")
    adj_kernel = "adj_gather_mfma_kernel"
    dom_kernel = fwd_kernel if dom == "gather" else adj_kernel
    # algorithmic bytes per launch: coefficients (8 channels FP32 over NS) + pair records + output/input signal
    NSd = ((c.n_tau + 12 + 63) // 64) * 64
    alg_bytes = 8 * 4 * c.n_panels * NSd + 64 * c.n_obs * c.n_panels + 4 * c.n_obs * int(nt.max())
    # the forward gather is VALU work, the transposed gather runs its channel sums on the matrix cores
    # (FP32 MFMA, the same 157.3 TFLOP/s peak)
    roofline = {"bound": "alu" if dom == "gather" else "mfma", "kernel": dom_kernel, "achieved": achieved, "peak": FP32_PEAK / 1e12,
                "unit": "TFLOP/s", "frac": achieved * 1e12 / FP32_PEAK, "traffic": measured_traffic(dom_kernel),
                "traffic_unit": "bytes per launch (HBM, rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
                "algorithmic_bytes": alg_bytes,
                "frac_of_nonpacked_fp32_peak": achieved * 1e12 / FP32_NONPACKED_PEAK,
                "flop_per_unit": FLOP_PER_UNIT, "units_per_launch": U, "avg_launch_ms": avg[dom],
                "other_gather": {"kernel": adj_kernel if dom == "gather" else fwd_kernel,
                                 "avg_launch_ms": avg["adj_gather" if dom == "gather" else "gather"],
                                 "frac": FLOP_PER_UNIT * U / (avg["adj_gather" if dom == "gather" else "gather"]
                                                              * 1e-3) / FP32_PEAK}}
    # source stage: HBM-bound streaming (inputs read once, coefficients written once)
    NS = ((c.n_tau + 12 + 63) // 64) * 64
    src_bytes = 5 * 8 * c.n_panels * c.n_tau + 8 * 4 * c.n_panels * NS
    src = {"bound": "hbm", "kernel": "src_interior_kernel + src_general_kernel", "achieved": src_bytes / (avg["source"] * 1e-3) / 1e9,
           "peak": HBM_PEAK / 1e9, "unit": "GB/s", "algorithmic_bytes": src_bytes, "avg_launch_ms": avg["source"]}
    src["frac"] = src["achieved"] * 1e9 / HBM_PEAK

    cpu = None
    if not args.no_cpu_baseline:
        # oracle forward + adjoint (the same step) on a bounded observer sample, built for this host
        flags = oracle.use_native()
        n_threads = oracle.num_threads()

        def oracle_step(idx):
            xs = c.x_obs[idx]
            t = time.perf_counter()
            pr, _, ntr = oracle.forward(c.surface, xs, c.mach, c.aoa_deg, c.dtau, c.tau0, rho, u, pp)
            oracle.adjoint(c.surface, xs, c.mach, c.aoa_deg, c.dtau, c.tau0, rho, u, pp, 2.0 * pr)
            return time.perf_counter() - t, int(c.n_panels * int(ntr.sum()))
        # two probes separate the fixed cost (layout transposes, window) from the per-observer cost;
        # a first call warms the thread pool and the allocations so that it does not inflate them
        oracle_step(np.array([0]))
        t1o, _ = oracle_step(np.array([0]))
        t9o, _ = oracle_step(np.linspace(0, c.n_obs - 1, 9).round().astype(int))
        per_obs = max((t9o - t1o) / 8.0, 1e-3)
        fixed = max(t1o - per_obs, 0.0)
        n_s = int(min(c.n_obs, max(1, round((args.cpu_seconds - fixed) / per_obs))))
        idx = np.unique(np.linspace(0, c.n_obs - 1, n_s).round().astype(int))
        t_cpu, u_cpu = oracle_step(idx)
        # the same on one thread: one and two observers, whose difference is the per-observer cost
        # without the fixed per-panel work (layout transposes, source terms)
        oracle.set_num_threads(1)
        t_1, u_1 = oracle_step(np.array([c.n_obs // 2]))
        t_2, u_2 = oracle_step(np.array([c.n_obs // 2, c.n_obs // 2 + 1]))
        oracle.set_num_threads(n_threads)
        cpu = {"value": u_cpu / t_cpu, "unit": "panel-obs-samples/s", "cores": n_threads, "kind": "oracle",
               "sample": f"forward + adjoint of the FP64 oracle on {len(idx)} of {c.n_obs} observers (all "
                         f"{c.n_panels} panels, {c.n_tau} samples): {u_cpu:.3e} units in {t_cpu:.1f} s; "
                         f"excludes input generation", "seconds": t_cpu,
               "cpu_model": cpu_model(), "nproc": os.cpu_count(), "affinity_cpus": len(os.sched_getaffinity(0)),
               "compile_flags": flags,
               "value_1thread": u_1 / t_1, "sample_1thread": f"one observer, {u_1:.3e} units in {t_1:.1f} s",
               "value_1thread_per_observer": (u_2 - u_1) / max(t_2 - t_1, 1e-6),
               "sample_1thread_per_observer": f"two observers minus one: {u_2 - u_1:.3e} units in "
                                              f"{t_2 - t_1:.1f} s"}
        log(f"[bench] cpu oracle: {cpu['value']:.3e} units/s on {cpu['cores']} threads, {u_1 / t_1:.3e} on one "
            f"(one observer; {cpu['value_1thread_per_observer']:.3e} per added observer) "
            f"({cpu['cpu_model']}, nproc {cpu['nproc']})")

    extra = {}
    if not args.no_extra:
        del plan
        torch.cuda.empty_cache()
        extra["airfoil_broadband"] = bench_airfoil(3, sync)
        extra["batched"] = bench_batch(5, sync)
        extra["general_motion"] = bench_general_motion(5, sync)
        extra["ingest"] = bench_ingest(sync)

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
        "err_vs_closed_form": err32_exact,
        "stage_ms_per_launch": per_launch,
        "fwd_units_per_s": U / ((avg["source"] + avg["gather"] + avg["reduce"]) * 1e-3),
        "adj_units_per_s": U / ((avg["adj_gather"] + avg["source_adj"]) * 1e-3),
        "source_roofline": src,
        "bf16_storage": {"value": U / (ms_b * 1e-3), "ms_per_step": ms_b, "err_vs_oracle": errb},
        "hbm_bound_8_observers": low_obs,
        "gather": plan_info,
        "plain_f64": plain,
        "speedup_vs_plain_f64": (value / plain["value"]) if plain else None,
        "oracle_sampled_forward_s": t_o,
    }
    out.update(extra)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
