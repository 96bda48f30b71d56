#!/usr/bin/env python3
"""Benchmark: Gcell-steps/s of the FP32 pseudo-spectral elastic solver on one GPU.

Workload (default): the 384 x 384 x 256 layered marine model (water over 6
sediment layers with a seeded +-5 % correlated perturbation), dx = 10 m,
dt = 0.8 ms, 20-cell PML, one double-couple source with a 25 Hz Ricker
wavelet, 128 x 128 four-component seabed receivers, a shot of 4000 leapfrog
steps.  One bench step is a chunk of 200 leapfrog steps of that shot through
the HIP kernels (spectral derivatives, split-PML updates, source injection,
receiver gathers); the shot is reset when its 4000 steps are done, so the
default 20 timed steps are one whole shot.  The model tables and the trace
buffer are resident in HBM when the timed region starts.

Prints one JSON line with the throughput, the roofline position of the
dominant kernel (HIP-event timing), the whole step against the algorithmic
bytes, the parity of the same launch configuration against the stored FP64
oracle state, and the FP64 CPU oracle timed on a bounded sample of the same
shot.

    python bench.py [--steps K] [--warmup W] [--gpus 1] [--workload ...]
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "Gcell-steps/s FP32 PSTD elastic @1e-4 L2; surrogate vs solver seismograms/s"
KERNEL_SOURCES = ["paper_1705_04874_amd/csrc/pstd_kernels.hpp", "paper_1705_04874_amd/csrc/fft_lds.hpp",
                  "paper_1705_04874_amd/csrc/pstd3d.hip"]

# HBM bytes per launch measured with rocprofv3 (FETCH_SIZE x 2.0 + WRITE_SIZE x 1.0, the
# factors a 1 GiB device copy gives) on kernel sources whose digest is recorded here; the
# summaries are in profiles/.  Reported only while the sources are unchanged.
MEASURED_TRAFFIC = {
    "source_digest": "93651babde9ca969",
    "layered384": {"y_fwd_stress": 1821.6e6, "z_op_V": 2429.5e6, "y_inv_V": 2732.3e6, "vel_update": 3888.4e6,
                   "y_fwd_vel": 910.9e6, "z_op_S": 1822.4e6, "y_inv_S": 2732.3e6, "stress_update": 5882.8e6},
    "layered128": {"y_fwd_stress": 102.4e6, "z_op_V": 136.5e6, "y_inv_V": 153.6e6, "vel_update": 254.1e6,
                   "y_fwd_vel": 51.2e6, "z_op_S": 102.4e6, "y_inv_S": 153.6e6, "stress_update": 377.1e6},
}

# the same for seis_combine's kernel (its own source file): bytes per launch on the
# bench's combine workload
COMBINE_SOURCES = ["paper_1705_04874_amd/csrc/combine.hip"]
COMBINE_TRAFFIC = {"source_digest": "d1bab7cd28ce269e", "bytes": 9482.8e6}


def kernel_source_digest(files=KERNEL_SOURCES):
    import hashlib
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def kernel_bytes_per_cell(nx, nxh, fu=0.0):
    """Algorithmic HBM bytes per cell and launch for each kernel kind (one shot):
    every input read once and every output written once; half spectra count
    nxh/nx complex values per cell (8 bytes each), real fields 4 bytes.  A
    fraction fu of the cells is undamped by the absorbing layer: there the
    update kernels read and write one split part per field (3 velocity, 6
    stress) instead of all (9, 15)."""
    S = 8.0 * nxh / nx
    R = 4.0
    K = 4.0 * nxh / nx  # kappa table (the stress phase's z operator evaluates kappa instead)
    pv = 9.0 * (1.0 - fu) + 3.0 * fu
    ps = 15.0 * (1.0 - fu) + 6.0 * fu
    return {
        "y_fwd_stress": 6 * 2 * S,
        "z_op_V": 6 * S + 9 * S + K,
        "y_inv_V": 9 * 2 * S,
        "vel_update": 9 * S + 2 * pv * R + 3 * R + 3 * S,
        "y_fwd_vel": 3 * 2 * S,
        "z_op_S": 3 * S + 9 * S,
        "y_inv_S": 9 * 2 * S,
        "stress_update": 9 * S + 2 * ps * R + 5 * R + 6 * S,
    }


def undamped_fraction(s):
    """Fraction of the solver's cells that the absorbing layer leaves undamped."""
    lo, hi = s.undamped_range()
    f = 1.0
    for d, n in enumerate(s.shape[::-1]):
        f *= max(0, hi[d] - lo[d] + 1) / n
    return f


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


GOLDEN = {"layered128": "layered128_oracle_traces.npz", "layered384": "layered384_oracle_planes.npz"}


def parity_check(args, w, s, binding, torch, np, chunk_traces):
    """rel-L2 of this launch configuration against the stored FP64 oracle results:
    traces of a whole 128^3 shot, or the nine fields (and their 24 split parts,
    on the field's scale) of the 384 x 384 x 256 shot on three planes through the
    source after the golden's step count."""
    gold = os.path.join(ROOT, "tests", "golden", GOLDEN.get(args.workload, ""))
    if args.workload not in GOLDEN or not os.path.exists(gold):
        return None
    g = np.load(gold, allow_pickle=False)
    nt = int(g["nt"])
    from tests.golden.make_layered128_golden import model_digest
    wg = {"layered128": inputs_mod().layered128_workload,
          "layered384": inputs_mod().layered384_workload}[args.workload](nt=nt)
    if str(g["digest"]) != model_digest(wg):
        return {"error": "workload generator changed since the golden was written"}
    s.reset()
    if args.workload == "layered128":
        tr = s.run(nt).cpu().numpy()[0][:, g["receivers"]].astype(np.float64)
        ref = g["traces"]
        return {c: float(np.linalg.norm(tr[i] - ref[i]) / np.linalg.norm(ref[i]))
                for i, c in enumerate(["p", "vx", "vy", "vz"])}
    s.run(nt)
    st = s.get_state()
    from tests.golden.make_layered384_golden import planes
    from tests.physics import collapse_undamped, undamped_mask
    # the nine fields are sums of their split parts (state order: vx, vy, vz
    # in 3 parts each, sxx, syy, szz in 3, sxy, sxz, syz in 2); a part's error
    # is measured on the scale of its field.  The solver keeps each field in
    # its first part in the cells the absorbing layer leaves undamped, so the
    # oracle's parts are summed the same way there.
    parts = [[0, 1, 2], [3, 4, 5], [6, 7, 8], [9, 10, 11], [12, 13, 14], [15, 16, 17], [18, 19], [20, 21], [22, 23]]
    mask3 = undamped_mask(w.model.shape, *s.undamped_range())
    field_err, part_err = [], []
    for name, zs, ys, xs in planes(w):
        got = st[:, zs, ys, xs].astype(np.float64)
        ref = collapse_undamped(g[name].astype(np.float64), mask3[zs, ys, xs])
        for pp in parts:
            nf = np.linalg.norm(ref[pp].sum(axis=0))
            if nf > 0:
                field_err.append(float(np.linalg.norm(got[pp].sum(axis=0) - ref[pp].sum(axis=0)) / nf))
                part_err += [float(np.linalg.norm(got[f] - ref[f]) / nf) for f in pp]
    del st
    return {"state_after_steps": nt, "planes": 3, "fields": 9, "split_parts": 24,
            "max_rel_l2": max(field_err), "median_rel_l2": float(np.median(field_err)),
            "max_split_part_err_on_field_scale": max(part_err)}


def inputs_mod():
    from paper_1705_04874_amd import inputs
    return inputs


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20, help="timed bench steps (chunks of --chunk leapfrog steps)")
    ap.add_argument("--warmup", type=int, default=5, help="untimed bench steps")
    ap.add_argument("--nt", type=int, default=None, help="leapfrog steps per shot (default: the workload's)")
    ap.add_argument("--chunk", type=int, default=200, help="leapfrog steps per bench step")
    ap.add_argument("--workload", default="layered384",
                    choices=["layered384", "layered128", "paper125x75x300", "batched", "combine", "surrogate"],
                    help="batched: 64 shots on the 128^3 model plus 24 uneven models advanced together in one "
                         "graph per step pair, then seis_combine of 300 events; combine: seis_combine alone "
                         "on the batched configuration's record size; surrogate: training steps and inference "
                         "of the spectral operator surrogate at its full shape")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-parity", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0, help="target oracle sample time")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run 1 GiB device copies first (reference kernels for HBM counters)")
    ap.add_argument("--no-profile", action="store_true", help="skip the per-kernel event pass")
    ap.add_argument("--profile-steps", type=int, default=1, help="bench steps in the per-kernel event pass")
    ap.add_argument("--tuning", default="",
                    help="pin the launch shapes instead of autotuning: y_tile,z_tile,vel_threads,str_threads,"
                         "z_threads,z_fields (e.g. 16,16,256,256,256,6; 0 leaves a knob to the autotuner)")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus > 1 or world > 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(shots would shard across GPUs with no exchange); run with --gpus 1", file=sys.stderr)
        return 2

    import numpy as np
    import torch

    from paper_1705_04874_amd import binding, inputs

    torch.cuda.set_device(0)
    if args.workload == "batched":
        return bench_batched(args, binding, inputs, torch)
    if args.workload == "combine":
        return bench_combine(args, binding, inputs, torch)
    if args.workload == "surrogate":
        return bench_surrogate(args, binding, inputs, torch)
    dev = torch.device("cuda:0")
    make = {"layered128": inputs.layered128_workload, "layered384": inputs.layered384_workload,
            "paper125x75x300": inputs.paper_shaped_workload}[args.workload]
    w = make() if args.nt is None else make(nt=args.nt)
    nt = w.nt
    chunk = min(args.chunk, nt)
    nz, ny, nx = w.model.shape
    cells = nx * ny * nz
    s = binding.Solver.from_workload(w)
    if args.tuning:
        s.set_tuning(*[int(v) for v in args.tuning.split(",")])
    s.set_workload_sources(w)
    traces = torch.empty((s.n_shots, 4, s.n_rec, chunk), dtype=torch.float32, device=dev)
    print(f"workload {w.name}: {nx}x{ny}x{nz}, shot of {nt} steps, bench step = {chunk} steps",
          file=sys.stderr, flush=True)

    if args.copy_calibration:
        a = torch.empty(1 << 28, dtype=torch.float32, device=dev)   # 1 GiB
        b = torch.empty_like(a)
        a.fill_(1.0)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        torch.mul(a, 1.0, out=b)          # plain elementwise copy kernel: 1 GiB read, 1 GiB written
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes_read": a.numel() * 4,
                          "copy_calibration_bytes_written": b.numel() * 4}), file=sys.stderr, flush=True)
        del a, b

    def bench_step():
        # the shot restarts when its nt steps are done (the reset is part of the work)
        if s.step + chunk > nt:
            s.reset()
        s.run(chunk, out=traces)

    s.reset()
    for i in range(args.warmup):
        bench_step()
        print(f"warmup step {i + 1}/{args.warmup} done", file=sys.stderr, flush=True)
    s.reset()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        bench_step()
        print(f"timed step {i + 1}/{args.steps} done", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0

    # per-kernel durations: HIP events recorded by the library on its stream
    # around every launch, over bench steps run again eagerly (the timed region
    # above replays graphs of step pairs)
    prof = {}
    prof_wall = None
    if not args.no_profile:
        s.reset()
        s.profile(True)
        torch.cuda.synchronize()
        tp = time.perf_counter()
        for i in range(args.profile_steps):
            bench_step()
        torch.cuda.synchronize()
        prof_wall = (time.perf_counter() - tp) / (args.profile_steps * chunk)
        prof = s.profile_read()
        s.profile(False)
        print("profiled pass done", file=sys.stderr, flush=True)

    cell_steps = float(cells) * chunk * args.steps * s.n_shots
    value = cell_steps / elapsed / 1e9
    ms_per_step = elapsed / args.steps * 1e3

    parity = None
    if not args.no_parity:
        parity = parity_check(args, w, s, binding, torch, np, traces)
        print("parity check done", file=sys.stderr, flush=True)

    roofline = None
    kernels = None
    if prof:
        bpc = kernel_bytes_per_cell(nx, nx // 2 + 1, undamped_fraction(s))
        kernels = {}
        for k, (ms, n) in prof.items():
            if n:
                avg_us = ms / n * 1e3
                alg = bpc[k] * cells * s.n_shots
                kernels[k] = {"launches": n, "avg_us": round(avg_us, 2),
                              "alg_bytes": int(alg), "alg_GBs": round(alg / (avg_us * 1e-6) / 1e9, 1)}
        dom = max(kernels, key=lambda k: kernels[k]["avg_us"] * kernels[k]["launches"])
        ach = kernels[dom]["alg_GBs"]
        traffic = None
        meas = MEASURED_TRAFFIC.get(args.workload)
        if meas and MEASURED_TRAFFIC["source_digest"] == kernel_source_digest() and s.n_shots == 1:
            traffic = meas.get(dom)
        roofline = {"bound": "hbm", "kernel": dom, "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": traffic,
                    "traffic_unit": "bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
                    "alg_bytes_per_launch": kernels[dom]["alg_bytes"]}
        tot_bytes = sum(bpc.values()) * cells * s.n_shots
        step_us = sum(v["avg_us"] for v in kernels.values())
        # the whole step: this design's algorithmic bytes (one HBM pass per
        # kernel) and the one-pass bound of 548 B per cell-step, both at the
        # throughput of the timed region
        roofline["step_alg_bytes_per_cell"] = round(sum(bpc.values()), 1)
        roofline["step_alg_GBs"] = round(tot_bytes / (step_us * 1e-6) / 1e9, 1)
        roofline["step_frac"] = round(sum(bpc.values()) * value / HBM_PEAK_GBS, 4)
        roofline["step_frac_548"] = round(548.0 * value / HBM_PEAK_GBS, 4)
        roofline["timing"] = "HIP events around each launch on the solver's stream, separate eager pass"
        roofline["profiled_ms_per_leapfrog_step"] = round(prof_wall * 1e3, 3)

    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        so = oracle.Solver.from_workload(w)
        so.set_sources(w.src_ijk, w.src_m, w.wavelet)
        so.run(1)
        t = time.perf_counter()
        n_cpu = 0
        while time.perf_counter() - t < args.cpu_seconds and n_cpu < nt:
            so.run(1)
            n_cpu += 1
        dt_cpu = time.perf_counter() - t
        so.close()
        cpu = {"value": round(cells * n_cpu / dt_cpu / 1e9, 6), "unit": "Gcell-steps/s", "cores": oracle.threads(),
               "kind": "oracle", "cpu_model": cpu_model(),
               "sample": f"{n_cpu} FP64 oracle steps (after 1 untimed) of the same {nx}x{ny}x{nz} shot, "
                         f"{dt_cpu:.1f} s; the rate of a whole {nt}-step shot is extrapolated from them"}
        print("cpu baseline done", file=sys.stderr, flush=True)

    out = {
        "metric": METRIC,
        "value": round(value, 4),
        "unit": "Gcell-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": w.name, "grid": [nx, ny, nz], "nt_per_shot": nt, "leapfrog_steps_per_step": chunk,
                   "shots_per_step": s.n_shots, "receivers": s.n_rec, "pml": w.pml, "dx_m": w.d[0], "dt_s": w.dt,
                   "step": f"{chunk} leapfrog steps of the shot (reset after {nt})"},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "parity_rel_l2": parity,
        "kernels": kernels,
        "device_bytes": s.device_bytes,
        "tuning": s.tuning(),
    }
    print(json.dumps(out), flush=True)
    s.close()
    return 0


def bench_combine(args, binding, inputs, torch):
    """seis_combine alone on the batched configuration's record: 64 sources x 4
    components x 4096 receivers x 2000 samples at 0.8 ms (seeded random traces),
    300 events (amplitudes LogNormal(0, 1), origins U[0, 10 s)) into a 12 s record
    at 1 ms.  One bench step is one call; the kernel time comes from HIP events
    on the stream the call runs on."""
    import numpy as np
    n_src, n_rec, nt_in, dt_in, nt_out = 64, 4096, 2000, 0.8e-3, 12000
    g = torch.Generator(device="cuda").manual_seed(5)
    tr = torch.randn((n_src, 4, n_rec, nt_in), device="cuda", generator=g)
    ev = inputs.event_catalogue(300, n_src, 10.0, 1.0, seed=2)
    t0 = [dt_in, 0.5 * dt_in, 0.5 * dt_in, 0.5 * dt_in]
    rec = torch.empty((4, n_rec, nt_out), dtype=torch.float32, device="cuda")

    def call():
        binding.seis_combine(tr, t0, ev.src_idx, ev.amp, ev.t_origin, nt_out, dt_in, 1e-3, out=rec)

    for _ in range(max(1, args.warmup)):
        call()
    torch.cuda.synchronize()
    evs = []
    t_start = time.perf_counter()
    for _ in range(args.steps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        call()
        e1.record()
        evs.append((e0, e1))
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t_start) / args.steps
    ms = float(np.mean([a.elapsed_time(b) for a, b in evs]))
    used = sorted(set(int(v) for v in ev.src_idx))
    alg = len(used) * 4 * n_rec * nt_in * 4 + 4 * n_rec * nt_out * 4
    # event-samples: output samples m of each (event, component) whose input
    # position lies inside the trace, over every receiver; a lane spends 9
    # vector instructions on each (position add, clamp, address, fraction
    # convert and scale, difference, lerp, conversion to double, double fma:
    # the kernel's inner loop), and a CU issues one wave64 instruction (64
    # lanes) per cycle: 256 CUs at 2.4 GHz bound the kernel's arithmetic
    dt_out = 1e-3
    m = np.arange(nt_out)
    ev_samples = 0
    for to in ev.t_origin:
        for c in range(4):
            u = m * (dt_out / dt_in) - (to + t0[c]) / dt_in
            ev_samples += int(np.count_nonzero((u > -1.0) & (u < nt_in)))
    ev_samples *= n_rec
    alu_ms = ev_samples * 9 / (256 * 64 * 2.4e9) * 1e3
    traffic = COMBINE_TRAFFIC["bytes"] if COMBINE_TRAFFIC["source_digest"] == kernel_source_digest(COMBINE_SOURCES) else None
    out = {
        "metric": "seis_combine GB/s (algorithmic bytes)", "value": round(alg / (ms * 1e-3) / 1e9, 1),
        "unit": "GB/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(wall * 1e3, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "seis_combine_300_events_64x4x4096x2000_to_12s", "n_src": n_src, "n_rec": n_rec,
                   "nt_in": nt_in, "nt_out": nt_out, "events": 300},
        "roofline": {"bound": "hbm", "kernel": "k_combine", "achieved": round(alg / (ms * 1e-3) / 1e9, 1),
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(alg / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                     "traffic": traffic, "alg_bytes_per_launch": alg,
                     "traffic_unit": "bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
                     "timing": "HIP events on the call's stream (includes the event-list upload)"},
        "kernel_ms": round(ms, 3), "call_wall_ms": round(wall * 1e3, 3),
        "sources_used": len(used),
        "alu_issue": {"event_samples": ev_samples, "instructions_per_event_sample": 9,
                      "bound_ms": round(alu_ms, 3), "frac": round(alu_ms / ms, 3),
                      "basis": "9 vector instructions per event-sample and lane, one wave64 instruction per cycle per CU, 256 CUs at 2.4 GHz"},
    }
    print(json.dumps(out), flush=True)
    return 0


def sno_gemm_flops(C, K, L, H, T, n_lift, fo):
    """Multiply-add FLOPs of one sample's forward pass through the surrogate's
    GEMMs: lift, per layer the truncated DFT, the mode mixing (four real
    products per mode), the pointwise weight and the inverse DFT, then the
    hidden projection and the moment-weighted output projection."""
    k2 = 2 * K
    layer = 2 * C * k2 * T + 4 * K * 2 * C * C + 2 * C * C * T + 2 * C * T * k2
    return 2 * C * T * n_lift + L * layer + 2 * H * T * C + 2 * fo * T * H


def bench_surrogate(args, binding, inputs, torch):
    """The surrogate at its full shape: 4 layers of width 64, 16 retained modes,
    1024 hidden outputs, travel-time aligned P and S frames, 4 components x 64
    receivers x 1024 samples.  Synthetic data: 512 seeded sources in the 500 m
    cube of the 128^3 layered model (0.8 double couple + 0.2 isotropic moment
    tensors) with seeded random target traces (the rates do not depend on the
    values).  Timed: --steps epochs of training (batch 16: forward, backward,
    Adam) and --steps inference passes over the 512 sources."""
    import numpy as np
    n, batch, T, C, K, L, H = 512, 16, 1024, 64, 16, 4, 1024
    model = inputs.layered128_model(0)
    rec = inputs.receiver_line_x(32, 96, 64, 20)
    n_rec = rec.shape[0]
    rng = np.random.default_rng(7)
    ctr = np.array([64.0, 64.0, 70.0])
    pos = np.floor(inputs.latin_hypercube(n, ctr - 25, ctr + 25, rng)).astype(np.int32)
    mts = np.stack([inputs.dc_plus_iso(rng, inputs.DV_UNIT_MOMENT) for _ in range(n)])
    X = torch.tensor(np.concatenate([pos, mts], axis=1), dtype=torch.float32, device="cuda")
    g = torch.Generator(device="cuda").manual_seed(3)
    Y = torch.randn((n, 4, n_rec, T), device="cuda", generator=g)
    four = inputs.sno_fourier_cycles(32, 4.0, 128.0)
    n_lift = 4 + 2 * len(four) + 6 * len(four)
    frames = 2
    fo = frames * 4 * n_rec
    theta0 = inputs.sno_init_params(C, K, L, H, fo, n_lift, 3)
    slow_p, slow_s = inputs.depth_slowness(model)
    t_ref = inputs.straight_ray_reference_times(slow_p, slow_s, ctr.astype(int), rec[n_rec // 2], (10.0,) * 3)
    fr = dict(rec_ijk=rec, slow_p=slow_p, slow_s=slow_s, h=(10.0,) * 3, dt=1.6e-3, t_ref=t_ref)
    sur = binding.Surrogate(n_rec, T, C, K, L, H, [64.0, 64.0, 70.0] + [0.0] * 6,
                            [25.0] * 3 + [inputs.DV_UNIT_MOMENT] * 6, theta0, four_cycles=four, pos_mod=True,
                            frames=fr)
    sur.train(X, Y, max(1, args.warmup), batch, 1e-4, seed=1, n_calib=0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sur.train(X, Y, args.steps, batch, 1e-4, seed=2, n_calib=0)
    torch.cuda.synchronize()
    t_train = (time.perf_counter() - t0) / args.steps
    sur.predict(X)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        sur.predict(X)
    torch.cuda.synchronize()
    t_inf = (time.perf_counter() - t0) / args.steps
    sur.close()
    f_fwd = sno_gemm_flops(C, K, L, H, T, n_lift, fo)
    inf_rate = n / t_inf
    tf_inf = f_fwd * n / t_inf / 1e12
    tf_train = 3 * f_fwd * n / t_train / 1e12
    out = {
        "metric": "surrogate seismograms/s (inference)", "value": round(inf_rate, 1), "unit": "seismograms/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(t_inf * 1e3, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "bf16", "data": "synthetic",
        "config": {"workload": "sno_4x64_16modes_H1024_aligned_4x64x1024", "sources": n, "batch": batch,
                   "layers": L, "width": C, "modes": K, "hidden": H, "frames": frames, "receivers": n_rec,
                   "samples": T, "step": "one inference pass over the sources"},
        "roofline": {"bound": "mfma", "achieved": round(tf_inf, 2), "peak": 2500.0, "unit": "TFLOP/s",
                     "frac": round(tf_inf / 2500.0, 5), "traffic": None,
                     "flops_per_sample": f_fwd,
                     "timing": "GEMM FLOPs over the wall time of whole inference passes (all kernels)"},
        "training_seismograms_per_s": round(n / t_train, 1), "training_TFLOPs": round(tf_train, 2),
        "training_epoch_ms": round(t_train * 1e3, 2),
    }
    print(json.dumps(out), flush=True)
    return 0


def bench_batched(args, binding, inputs, torch):
    """The batched configuration: 64 single-source shots on the 128^3 layered model
    (one context) and 24 uneven models (one context each), advanced together by
    pstd3d_run_many (one graph per step pair, a stream branch per context); one
    bench step is a reset of every context plus nt steps of all of them.  Then
    seis_combine sums 300 events of the 64 shots' traces into 12 s records at
    1 ms, timed on its own."""
    nt = args.nt or 2000
    w64 = inputs.layered128_shots(64, nt=nt)
    ws = [w64] + inputs.ragged_models(24, nt=nt)
    ss = []
    for w in ws:
        s = binding.Solver.from_workload(w)
        if args.tuning:
            s.set_tuning(*[int(v) for v in args.tuning.split(",")])
        s.set_workload_sources(w)
        ss.append(s)
    outs = [torch.empty((s.n_shots, 4, s.n_rec, nt), dtype=torch.float32, device="cuda") for s in ss]
    cells = sum(w.cells * w.n_shots for w in ws)
    shots = sum(w.n_shots for w in ws)

    def one_step():
        for s in ss:
            s.reset()
        binding.run_many(ss, nt, outs=outs)

    for i in range(args.warmup):
        one_step()
        print(f"warmup step {i + 1}/{args.warmup} done", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        one_step()
        print(f"timed step {i + 1}/{args.steps} done", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    value = cells * nt * args.steps / elapsed / 1e9

    # seis_combine of 300 events over the 64 shots' traces
    ev = inputs.event_catalogue(300, 64, 10.0, 1.0, seed=2)
    t0s = [w64.dt, 0.5 * w64.dt, 0.5 * w64.dt, 0.5 * w64.dt]
    rec = torch.empty((4, ss[0].n_rec, 12000), dtype=torch.float32, device="cuda")
    binding.seis_combine(outs[0], t0s, ev.src_idx, ev.amp, ev.t_origin, 12000, w64.dt, 1e-3, out=rec)
    torch.cuda.synchronize()
    tc = time.perf_counter()
    reps = 5
    for _ in range(reps):
        binding.seis_combine(outs[0], t0s, ev.src_idx, ev.amp, ev.t_origin, 12000, w64.dt, 1e-3, out=rec)
    torch.cuda.synchronize()
    combine_ms = (time.perf_counter() - tc) / reps * 1e3
    finite = bool(torch.isfinite(rec).all().item()) and all(bool(torch.isfinite(o).all().item()) for o in outs)

    # per-kernel HIP-event pass over the 64-shot context alone (a few steps)
    s = ss[0]
    nxyz = w64.model.shape[::-1]
    bpc = kernel_bytes_per_cell(nxyz[0], nxyz[0] // 2 + 1, undamped_fraction(s))
    s.profile(True)
    s.reset()
    s.run(min(nt, 40))
    torch.cuda.synchronize()
    prof = s.profile_read()
    s.profile(False)
    kernels = {}
    c64 = w64.cells * w64.n_shots
    for k, (ms, n) in prof.items():
        if n:
            avg_us = ms / n * 1e3
            kernels[k] = {"launches": n, "avg_us": round(avg_us, 2), "alg_bytes": int(bpc[k] * c64),
                          "alg_GBs": round(bpc[k] * c64 / (avg_us * 1e-6) / 1e9, 1)}
    dom = max(kernels, key=lambda k: kernels[k]["avg_us"] * kernels[k]["launches"])
    ach = kernels[dom]["alg_GBs"]
    out = {
        "metric": METRIC,
        "value": round(value, 4),
        "unit": "Gcell-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(elapsed / args.steps * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "batched_64shots_128cubed_plus_24_ragged_models", "contexts": len(ss),
                   "shots": shots, "cells_per_step": cells, "nt_per_shot": nt,
                   "step": "reset of every context + nt leapfrog steps of all of them (pstd3d_run_many)"},
        "seismograms_per_s": round(shots * args.steps / elapsed, 3),
        "seis_combine_ms": round(combine_ms, 3),
        "seis_combine": "300 events of the 64 shots' traces (4 x 4096 receivers x nt) into [4][4096][12000] at 1 ms",
        "roofline": {"bound": "hbm", "kernel": dom + " (64-shot context)", "achieved": ach, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": None,
                     "alg_bytes_per_launch": kernels[dom]["alg_bytes"]},
        "cpu_baseline": None,
        "outputs_finite": finite,
        "kernels_64shot_context": kernels,
    }
    print(json.dumps(out), flush=True)
    for s in ss:
        s.close()
    return 0


if __name__ == "__main__":
    sys.exit(main())
