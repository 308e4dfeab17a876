"""Benchmark of the pole-shifted TEM hot path on one MI355X.

One step = one pass of the whole hot path over the 64^3 precision workload
(762,048 unknowns, 16 poles, 8 loop sources, 60 times, 16 receivers):
assemble M(sigma) on the device, factor all 16 shifted matrices, solve all
poles x sources with FP64 refinement to 1e-10, assemble the data at all
times, then one J v and one J^T w through the cached factors.

Reported metric "all-pole factor+solve s & J^T v/s at 64^3, FP32+IR vs FP64,
same GPU": value = factor+solve seconds of the FP32+IR path
(median over the timed steps); J^T v per second and the FP64 figures are in
``phases``.  The roofline object covers the dominant kernel (the MFMA front
update, FP32) from HIP events inside the library; the CPU baseline is the
FP64 oracle on a bounded sample.

Before the timed steps of each precision the update kernels are autotuned
per tree level (tem_autotune; untimed set-up, like assembly and analysis).

Usage: python bench.py [--gpus 1] [--steps 1] [--warmup 1] [--no-cpu-baseline]
                       [--no-autotune] [--no-ragged] [--fp32-only]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "all-pole factor+solve s & Jᵀv/s at 64³ edge mesh, FP32+IR vs FP64, same GPU"
PEAK_FP32 = 157.3e12      # dense FP32 MFMA, MI355X
PEAK_FP64 = 78.6e12
PEAK_HBM = 8.0e12
TRAFFIC_RECORD = os.path.join(ROOT, "profiles", "front_update_hex64_fp32_traffic.json")
UPDATE_SOURCE = os.path.join(ROOT, "paper_2605_19951_amd", "csrc", "k_factor.hip")


def source_hash(path):
    import hashlib
    with open(path, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def recorded_traffic():
    """HBM bytes per launch of the FP32 front update from the committed
    rocprofv3 FETCH_SIZE / WRITE_SIZE record, if it was taken on the current
    kernel source (else None)."""
    if not os.path.exists(TRAFFIC_RECORD):
        return None
    with open(TRAFFIC_RECORD) as f:
        rec = json.load(f)
    if rec.get("source_sha256_16") != source_hash(UPDATE_SOURCE):
        return None
    return rec.get("hbm_bytes_per_launch")


def copy_probe(torch, dev, n_bytes=1 << 30, reps=5):
    """A plain device copy of n_bytes, reps times: the calibration run for the
    FETCH_SIZE / WRITE_SIZE counters (read n_bytes, write n_bytes each)."""
    a = torch.ones(n_bytes // 4, dtype=torch.float32, device=dev)
    b = torch.empty_like(a)
    for _ in range(reps):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps(dict(copy_probe_bytes=n_bytes, reps=reps)), flush=True)


def run_precision(t, wl, prec, steps, warmup, torch, dev, F, v, w, autotune=False):
    import numpy as np
    K, R = len(wl.poles.t), wl.rx.n
    tuned = None
    if autotune:   # untimed set-up: per-level choice of the update kernel variant
        ta = time.perf_counter()
        tuned = t.autotune(wl.poles.xi, prec)
        tuned["seconds"] = time.perf_counter() - ta
        print("# prec=%d autotune: candidates %s ms, tuned %.1f ms" % (
            prec, ["%.1f" % x for x in tuned["candidate_ms"]], tuned["tuned_ms"]),
            file=sys.stderr, flush=True)
    d = torch.zeros((wl.S, K, R), dtype=torch.float64, device=dev)
    jv = torch.zeros_like(d)
    jtw = torch.zeros(len(wl.params), dtype=torch.float64, device=dev)
    sigma = torch.tensor(wl.sigma, device=dev)
    me = wl.mesh
    rec = []
    for it in range(warmup + steps):
        timed = it >= warmup
        t.set_profiling(timed)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        t.assemble(me.nx, me.ny, me.nz, me.h, 4e-7 * math.pi, sigma, wl.params)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        t.factor_poles(wl.poles.xi, prec)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        ir = t.forward(F, wl.rx.ptr, wl.rx.col, wl.rx.val, wl.poles.alpha, d)
        torch.cuda.synchronize()
        t3 = time.perf_counter()
        t.jvp(v, jv)
        torch.cuda.synchronize()
        t4 = time.perf_counter()
        t.vjp(w, jtw)
        torch.cuda.synchronize()
        t5 = time.perf_counter()
        st = t.stats()
        if timed:
            rec.append(dict(assemble=t1 - t0, factor=t2 - t1, forward=t3 - t2, jvp=t4 - t3,
                            vjp=t5 - t4, step=t5 - t0, solves=int(ir["iters"].max()), stats=st))
        print("# prec=%d step %d: assemble %.3f factor %.3f forward %.3f jvp %.3f vjp %.3f s"
              % (prec, it, t1 - t0, t2 - t1, t3 - t2, t4 - t3, t5 - t4), file=sys.stderr, flush=True)
    med = lambda k: sorted(r[k] for r in rec)[len(rec) // 2]  # noqa: E731
    out = dict(assemble_s=med("assemble"), factor_s=med("factor"), forward_s=med("forward"),
               jvp_s=med("jvp"), vjp_s=med("vjp"), step_s=med("step"),
               factor_solve_s=med("factor") + med("forward"), jtv_per_s=1.0 / med("vjp"),
               ir_solves=rec[-1]["solves"], groups=rec[-1]["stats"]["n_groups"],
               group_size=rec[-1]["stats"]["group_size"],
               factor_gb=rec[-1]["stats"]["factor_bytes"] / 1e9)
    st = rec[-1]["stats"]
    out["update_ms"] = st["update_ms"]
    out["update_flops"] = st["update_flops"]
    out["update_launches"] = st["update_launches"]
    out["sweep_ms"] = st["sweep_ms"]
    out["sweep_bytes"] = st["sweep_bytes"]
    out["sweeps"] = st["sweeps"]
    if tuned is not None:
        out["autotune"] = tuned
    return out, d.cpu().numpy(), jtw.cpu().numpy()


def ragged_phase(torch, dev, prec, reps=2):
    """Twelve meshes (16^3 .. 40^3, 8-16 poles, 1-4 sources, 40 times):
    factor + forward of the whole batch through the batch entry points
    against the same meshes one at a time through the single-mesh path.
    Assemble and analyse are outside the timed region in both cases."""
    import numpy as np
    import tem_inputs as ti
    from paper_2605_19951_amd import Tem
    wls = ti.ragged_batch()
    K = len(wls[0].poles.t)
    # one mesh at a time
    singles = []
    for wl in wls:
        me = wl.mesh
        t = Tem(0)
        t.assemble(me.nx, me.ny, me.nz, me.h, 4e-7 * math.pi, torch.tensor(wl.sigma, device=dev),
                   wl.params)
        t.analyse()
        F = torch.tensor(wl.F.T.copy(), device=dev)
        d = torch.zeros((wl.S, K, wl.rx.n), dtype=torch.float64, device=dev)
        singles.append((t, F, d))
    one = []
    for it in range(reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for (t, F, d), wl in zip(singles, wls):
            t.factor_poles(wl.poles.xi, prec)
            t.forward(F, wl.rx.ptr, wl.rx.col, wl.rx.val, wl.poles.alpha, d)
        torch.cuda.synchronize()
        one.append(time.perf_counter() - t0)
    d_one = np.concatenate([d.cpu().numpy().reshape(-1) for _, _, d in singles])
    for t, _, _ in singles:
        t.close()
    del singles
    # the batch
    t = Tem(0)
    t.assemble_batch([(w.mesh.nx, w.mesh.ny, w.mesh.nz, w.mesh.h) for w in wls], 4e-7 * math.pi,
                     torch.tensor(np.concatenate([w.sigma for w in wls]), device=dev))
    info = t.analyse()
    F = torch.tensor(np.concatenate([w.F.T.reshape(-1) for w in wls]), device=dev)
    d = torch.zeros(sum(w.S * K * w.rx.n for w in wls), dtype=torch.float64, device=dev)
    bat = []
    for it in range(reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        t.factor_poles_batch([w.poles.xi for w in wls], prec)
        ir = t.forward_batch(F, [w.S for w in wls], [(w.rx.ptr, w.rx.col, w.rx.val) for w in wls],
                             [w.poles.alpha for w in wls], d)
        torch.cuda.synchronize()
        bat.append(time.perf_counter() - t0)
    d_bat = d.cpu().numpy()
    t.close()
    systems = sum(len(w.poles.xi) * w.S for w in wls)
    tb, to = min(bat), min(one)
    return dict(meshes=[w.mesh.nx for w in wls], poles=[len(w.poles.xi) for w in wls],
                sources=[w.S for w in wls], n_unknowns_total=info["n_unknowns"],
                flops_total=float(sum(len(w.poles.xi) * info_w for w, info_w in
                                      zip(wls, _flops_per_mesh(wls)))),
                batch_s=tb, one_at_a_time_s=to, speedup=to / tb,
                systems_per_s_batch=systems / tb, systems_per_s_one_at_a_time=systems / to,
                ir_solves=int(ir["iters"].max()),
                rel_diff_batch_vs_single=float(np.linalg.norm(d_bat - d_one) / np.linalg.norm(d_one)))


def _flops_per_mesh(wls):
    from paper_2605_19951_amd import symbolic_host
    return [symbolic_host(w.mesh.nx, w.mesh.ny, w.mesh.nz)["flops_per_pole"] for w in wls]


def cpu_baseline(flops64):
    """The FP64 oracle on the host: factor + solve of one pole of the same
    generator on a 32^3 mesh (8 sources), scaled to all 16 poles at 64^3 by
    the ratio of multifrontal factor flops.  The oracle runs as it stands:
    its sparse LU calls the host BLAS, which may use several threads, so
    `cores` is the process CPU time of the timed solve over its wall time."""
    import numpy as np
    import tem_inputs as ti
    from oracle.ordering import analyse, factor_flops
    from oracle.tem import OracleTEM
    wl = ti.smooth_workload(32, 4, S=8, m=16, K=60, g=4, seed=3, name="hex32_sample")
    me = wl.mesh
    o = OracleTEM(me.nx, me.ny, me.nz, me.h, wl.sigma, wl.F, wl.rx.ptr, wl.rx.col, wl.rx.val,
                  wl.poles.xi, wl.poles.alpha, wl.params)
    o.ordering()
    c0 = time.process_time()
    t0 = time.perf_counter()
    o.solve(0, o.F)
    dt = time.perf_counter() - t0
    cpu = time.process_time() - c0
    nodes, _, _ = analyse(o.mesh)
    f32 = factor_flops(nodes)
    scale = 16.0 * flops64 / f32
    return dict(value=dt * scale, unit="s", cores=max(1, int(round(cpu / dt))), kind="oracle",
                sample="factor+solve of 1 pole x 8 sources on a 32^3 mesh of the same generator "
                       "(%.1f s wall, %.1f s CPU over its threads), scaled x%.0f (16 poles x "
                       "factor-flop ratio 64^3/32^3)" % (dt, cpu, scale))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--fp32-only", action="store_true")
    ap.add_argument("--no-ragged", action="store_true")
    ap.add_argument("--no-autotune", action="store_true",
                    help="skip the (untimed) per-level autotuning of the update kernels")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only run the counter-calibration copy (1 GiB, 5 times)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the pole-sharded multi-GPU path is not part of this "
              "build (run with --gpus 1)", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch
    import tem_inputs as ti
    from paper_2605_19951_amd import FP32_IR, FP64, Tem
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    dev = torch.device("cuda:0")
    if args.copy_probe:
        copy_probe(torch, dev)
        return
    wl = ti.workload(2)
    me = wl.mesh
    t = Tem(0)
    t.assemble(me.nx, me.ny, me.nz, me.h, 4e-7 * math.pi, torch.tensor(wl.sigma, device=dev),
               wl.params)
    ta = time.perf_counter()
    info = t.analyse()
    analyse_s = time.perf_counter() - ta
    F = torch.tensor(wl.F.T.copy(), device=dev)
    rng = np.random.default_rng(7)
    v = torch.tensor(rng.standard_normal(len(wl.params)), device=dev)
    w = torch.tensor(rng.standard_normal((wl.S, len(wl.poles.t), wl.rx.n)), device=dev)
    phases = {}
    res32, d32, g32 = run_precision(t, wl, FP32_IR, args.steps, args.warmup, torch, dev, F, v, w,
                                    not args.no_autotune)
    phases["fp32_ir"] = res32
    acc = None
    if not args.fp32_only:
        res64, d64, g64 = run_precision(t, wl, FP64, args.steps, args.warmup, torch, dev, F, v, w,
                                        not args.no_autotune)
        phases["fp64"] = res64
        acc = dict(data_rel_fp32_vs_fp64=float(np.linalg.norm(d32 - d64) / np.linalg.norm(d64)),
                   jtw_rel_fp32_vs_fp64=float(np.linalg.norm(g32 - g64) / np.linalg.norm(g64)))
    t.close()
    del t
    if not args.no_ragged:
        phases["ragged_batch_fp32_ir"] = ragged_phase(torch, dev, FP32_IR)
    ach = res32["update_flops"] / (res32["update_ms"] * 1e-3) if res32["update_ms"] > 0 else 0.0
    roof = dict(bound="mfma", kernel="k_front_update<float>", achieved=ach / 1e12,
                peak=PEAK_FP32 / 1e12, unit="TFLOP/s", frac=ach / PEAK_FP32,
                traffic=recorded_traffic(), launches=res32["update_launches"],
                flops_per_launch=res32["update_flops"] / max(res32["update_launches"], 1),
                ms_per_launch=res32["update_ms"] / max(res32["update_launches"], 1))
    sweep_bw = res32["sweep_bytes"] / (res32["sweep_ms"] * 1e-3) if res32["sweep_ms"] > 0 else 0.0
    line = dict(metric=METRIC, value=res32["factor_solve_s"], unit="s", n_gpus=1,
                steps=args.steps, warmup=args.warmup, ms_per_step=res32["step_s"] * 1e3,
                higher_is_better=False, scaling="weak", vs_baseline=None,
                dtype="c64 factors + f64 refinement", data="synthetic",
                config=dict(workload=wl.name, mesh="64x64x64", h_m=25.0, n_unknowns=info["n_unknowns"],
                            poles=len(wl.poles.xi), sources=wl.S, times=len(wl.poles.t),
                            receivers=wl.rx.n, params=len(wl.params), ir_rtol=1e-10,
                            flops_per_pole=info["flops_per_pole"], analyse_s=analyse_s),
                phases=phases, accuracy=acc, roofline=roof,
                sweep=dict(bound="hbm", achieved=sweep_bw / 1e9, peak=PEAK_HBM / 1e9, unit="GB/s",
                           frac=sweep_bw / PEAK_HBM))
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(info["flops_per_pole"])
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
