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

The default run also times one step of each precision on a jittered
48^3-cube tetrahedral mesh (``phases.tet``; ``--no-tet`` skips it).
``--tet`` runs only that workload (both
precisions, autotuned the same way) and prints that workload's own line.

Usage: python bench.py [--gpus 1] [--steps 1] [--warmup 1] [--no-cpu-baseline]
                       [--no-autotune] [--no-ragged] [--no-tet] [--fp32-only]
                       [--tet [--tet-cubes 48]]
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
TET_TRAFFIC_RECORD = os.path.join(ROOT, "profiles", "front_update_tet48_fp32_traffic.json")
UPDATE_SOURCE = os.path.join(ROOT, "paper_2605_19951_amd", "csrc", "k_factor.hip")


def source_hash(path):
    import hashlib
    with open(path, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def recorded_traffic(record=TRAFFIC_RECORD):
    """HBM bytes per launch of the FP32 front update from a committed
    rocprofv3 FETCH_SIZE / WRITE_SIZE record, if it was taken on the current
    kernel source (else None)."""
    if not os.path.exists(record):
        return None
    with open(record) as f:
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


def inversion_phase(torch, dev, prec, max_gn=25, lsqr_iters=20, lambda0=10.0,
                    runtime_counts=(1, 5, 10, 20, 35)):
    """The paper's inversion experiment on a uniform-hex analogue of its
    four-block model (tem_inputs.four_block_workload: 32^3 cells of 5 m, a
    40 m loop, 7 x 7 dB_z/dt receivers, 31 times in [1e-6, 1e-3] s, 21 RKFIT
    pole pairs, 24,576 parameters): observed data = the forward response of
    the true model plus 3 % Gaussian noise (+1e-9 absolute); Gauss-Newton
    from the 0.1 S/m half-space with line search and lambda cooling
    (tem_invert).  Then one Gauss-Newton iteration from the same start per
    LSQR count in runtime_counts, and a least-squares fit of the paper's
    linear runtime model t = a + b n_LSQR to them."""
    import numpy as np
    import tem_inputs as ti
    from paper_2605_19951_amd import Tem, rkfit
    times = ti.log_times(1e-6, 1e-3, 31)
    tab = rkfit.rkfit_exp(times, 21)
    wl = ti.four_block_workload(poles=ti.PoleTable(t=tab.t, xi=tab.xi, alpha=tab.alpha,
                                                   err=tab.err))
    me = wl.mesh
    K, R, P = len(times), wl.rx.n, len(wl.params)
    t = Tem(0)
    t.assemble(me.nx, me.ny, me.nz, me.h, 4e-7 * math.pi, torch.tensor(wl.sigma, device=dev),
               wl.params)
    t.analyse()
    t.factor_poles(wl.poles.xi, prec)
    F = torch.tensor(wl.F.T.copy(), device=dev)
    d = torch.zeros((wl.S, K, R), dtype=torch.float64, device=dev)
    t.forward(F, wl.rx.ptr, wl.rx.col, wl.rx.val, wl.poles.alpha, d)
    d_true = d.cpu().numpy()
    sd = 0.03 * np.abs(d_true) + 1e-9
    d_obs = torch.tensor(d_true + sd * wl.extra["rng_noise"].standard_normal(d_true.shape),
                         device=dev)
    wd = torch.tensor(1.0 / sd, device=dev)
    m0 = torch.full((P,), math.log(0.1), dtype=torch.float64, device=dev)

    def restart():
        m = m0.clone()
        t.set_model(m)
        t.factor_poles(wl.poles.xi, prec)
        t.forward(F, wl.rx.ptr, wl.rx.col, wl.rx.val, wl.poles.alpha, d)
        return m

    m = restart()
    t0 = time.perf_counter()
    log = t.invert(d_obs, wd, m, m0, lambda0, max_gn, lsqr_iters)
    total = time.perf_counter() - t0
    # recovered conductivity of the four blocks (mean log10 over each block)
    mf = m.cpu().numpy() / math.log(10.0)
    c, k = me.nx // 2, me.k_if - 3
    blocks = []
    for (i0, j0), val in (((c - 7, c - 7), 1.0), ((c + 2, c + 2), 1.0),
                          ((c + 2, c - 7), 0.01), ((c - 7, c + 2), 0.01)):
        ids = [i + me.nx * (j + me.ny * k) for j in range(j0, j0 + 5) for i in range(i0, i0 + 5)]
        blocks.append(dict(true_log10=math.log10(val), recovered_log10=float(mf[ids].mean())))
    # runtime model: one iteration per LSQR count from the same start
    pts = []
    for n in runtime_counts:
        m = restart()
        r = t.invert(d_obs, wd, m, m0, lambda0, 1, n)[0]
        pts.append(dict(lsqr=n, seconds=r["seconds"], factor_seconds=r["factor_seconds"],
                        trials=r["trials"]))
    A = np.array([[1.0, p_["lsqr"]] for p_ in pts])
    y = np.array([p_["seconds"] for p_ in pts])
    (a, b), *_ = np.linalg.lstsq(A, y, rcond=None)
    t.close()
    return dict(workload=wl.name, mesh="%dx%dx%d" % (me.nx, me.ny, me.nz), h_m=me.h,
                n_unknowns=3 * me.nx * (me.nx - 1) ** 2, poles=len(wl.poles.xi),
                rkfit_max_err=float(tab.err.max()), receivers=R, times=K, params=P,
                precision="fp32_ir" if prec == 1 else "fp64", lambda0=lambda0,
                lsqr_iters=lsqr_iters, seconds=total, iterations=log, blocks=blocks,
                runtime_points=pts, runtime_model=dict(fixed_s=float(a), per_lsqr_s=float(b)))


ORACLE_RECORD = os.path.join(ROOT, "profiles", "oracle_hex64_pole_cpu.json")


def tet_phase(torch, dev, steps, warmup, n=48, autotune=True):
    """The same step on a jittered tetrahedral mesh (n^3 cubes, six
    tetrahedra each; 8 loops, 16 poles, 60 times, 4 x 4 receivers) in both
    precisions: M(sigma) re-assembled on the device, all poles factored,
    forward, J v, J^T w.  Returns that workload's JSON line (value: the
    FP32+IR factor+solve seconds, as for the hexahedral line)."""
    import numpy as np
    from paper_2605_19951_amd import FP32_IR, FP64, Tem
    from tem_inputs.tet import tet_workload
    wl = tet_workload(n, n // 8, h=25.0, S=8, m=16, K=60, g=4, seed=51, name="tet%d" % n)
    me = wl.mesh
    t = Tem(0)
    sigma = torch.tensor(wl.sigma, device=dev)
    t.assemble_tet(me.xyz, me.tets, wl.mu, sigma, wl.params)
    ta = time.perf_counter()
    info = t.analyse()
    analyse_s = time.perf_counter() - ta
    F = torch.tensor(wl.F.T.copy(), device=dev)
    rng = np.random.default_rng(7)
    v = torch.tensor(rng.standard_normal(len(wl.params)), device=dev)
    w = torch.tensor(rng.standard_normal((wl.S, len(wl.poles.t), wl.rx.n)), device=dev)
    d = torch.zeros((wl.S, len(wl.poles.t), wl.rx.n), dtype=torch.float64, device=dev)
    jv = torch.zeros_like(d)
    jtw = torch.zeros(len(wl.params), dtype=torch.float64, device=dev)
    m = torch.log(sigma[torch.tensor(wl.params, device=dev, dtype=torch.long)])
    phases, outs = {}, {}
    for name, prec in (("fp32_ir", FP32_IR), ("fp64", FP64)):
        tuned = None
        if autotune:   # untimed set-up, as for the hexahedral workload
            ta = time.perf_counter()
            tuned = t.autotune(wl.poles.xi, prec)
            tuned["seconds"] = time.perf_counter() - ta
            print("# tet %s autotune: candidates %s ms, tuned %.1f ms" % (
                name, ["%.1f" % x for x in tuned["candidate_ms"]], tuned["tuned_ms"]),
                file=sys.stderr, flush=True)
        rec = []
        for it in range(warmup + steps):
            timed = it >= warmup
            t.set_profiling(timed)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            t.set_model(m)            # M(sigma) re-assembled on the device
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
                                vjp=t5 - t4, solves=int(ir["iters"].max()), stats=st))
            print("# tet %s step %d: assemble %.3f factor %.3f forward %.3f jvp %.3f vjp %.3f s"
                  % (name, it, t1 - t0, t2 - t1, t3 - t2, t4 - t3, t5 - t4), file=sys.stderr,
                  flush=True)
        med = lambda k: sorted(r[k] for r in rec)[len(rec) // 2]  # noqa: E731
        st = rec[-1]["stats"]
        phases[name] = dict(
            assemble_s=med("assemble"), factor_s=med("factor"), forward_s=med("forward"),
            jvp_s=med("jvp"), vjp_s=med("vjp"), factor_solve_s=med("factor") + med("forward"),
            jtv_per_s=1.0 / med("vjp"), ir_solves=rec[-1]["solves"],
            factor_gb=st["factor_bytes"] / 1e9, update_ms=st["update_ms"],
            update_flops=st["update_flops"], update_launches=st["update_launches"],
            sweep_ms=st["sweep_ms"], sweep_bytes=st["sweep_bytes"])
        if tuned is not None:
            phases[name]["autotune"] = tuned
        outs[name] = (d.cpu().numpy(), jtw.cpu().numpy())
    t.close()
    acc = dict(data_rel_fp32_vs_fp64=float(np.linalg.norm(outs["fp32_ir"][0] - outs["fp64"][0])
                                           / np.linalg.norm(outs["fp64"][0])),
               jtw_rel_fp32_vs_fp64=float(np.linalg.norm(outs["fp32_ir"][1] - outs["fp64"][1])
                                          / np.linalg.norm(outs["fp64"][1])))
    r32 = phases["fp32_ir"]
    ach = r32["update_flops"] / (r32["update_ms"] * 1e-3) if r32["update_ms"] > 0 else 0.0
    bw = r32["sweep_bytes"] / (r32["sweep_ms"] * 1e-3) if r32["sweep_ms"] > 0 else 0.0
    return dict(
        metric="all-pole factor+solve s & J\u1d40v/s on a tetrahedral edge mesh, FP32+IR vs FP64",
        value=r32["factor_solve_s"], unit="s", n_gpus=1, steps=steps, warmup=warmup,
        ms_per_step=1e3 * sum(r32[k] for k in ("assemble_s", "factor_s", "forward_s", "jvp_s",
                                                 "vjp_s")),
        higher_is_better=False, scaling="weak", vs_baseline=None,
        dtype="c64 factors + f64 refinement", data="synthetic",
        config=dict(workload=wl.name, cubes="%dx%dx%d" % (n, n, n), tets=me.n_tets,
                    n_unknowns=info["n_unknowns"], poles=len(wl.poles.xi), sources=wl.S,
                    times=len(wl.poles.t), receivers=wl.rx.n, params=len(wl.params),
                    flops_per_pole=info["flops_per_pole"], max_front=info["max_front"],
                    analyse_s=analyse_s),
        phases=phases, accuracy=acc,
        roofline=dict(bound="mfma", kernel="k_front_update<float>", achieved=ach / 1e12,
                      peak=PEAK_FP32 / 1e12, unit="TFLOP/s", frac=ach / PEAK_FP32,
                      traffic=recorded_traffic(TET_TRAFFIC_RECORD) if n == 48 else None),
        sweep=dict(bound="hbm", achieved=bw / 1e9, peak=PEAK_HBM / 1e9, unit="GB/s",
                   frac=bw / PEAK_HBM))


def cpu_baseline():
    """The FP64 oracle on the host, as it stands: factor + solve of pole 0 x
    8 sources on the 32^3 sample mesh of the same generator, timed here
    (about 10-20 s), scaled to all 16 poles at 64^3 by the ratio of the
    oracle's 64^3 pole to the same 32^3 sample, both measured on one host
    (profiles/oracle_hex64_pole_cpu.json, written by
    tests/golden/make_hex64_pole.py).  The oracle's sparse LU calls the host
    BLAS, which may use several threads, so `cores` is the process CPU time
    of the timed solve over its wall time."""
    import tem_inputs as ti
    from oracle.tem import OracleTEM
    with open(ORACLE_RECORD) as f:
        rec = json.load(f)
    wl = ti.smooth_workload(32, 4, S=8, m=16, K=60, g=4, seed=3, name="hex32_sample")
    me = wl.mesh
    o = OracleTEM(me.nx, me.ny, me.nz, me.h, wl.sigma, wl.F, wl.rx.ptr, wl.rx.col, wl.rx.val,
                  wl.poles.xi[:1], wl.poles.alpha[:, :1], wl.params)
    o.ordering()
    c0 = time.process_time()
    t0 = time.perf_counter()
    o.solve(0, o.F)
    dt = time.perf_counter() - t0
    cpu = time.process_time() - c0
    ratio = rec["ratio_hex64_over_hex32"]
    pole64 = rec["factor_s"] + rec["solve_s"]
    host = rec["host"]
    return dict(value=16.0 * ratio * dt, unit="s", cores=max(1, int(round(cpu / dt))),
                kind="oracle",
                sample="factor+solve of 1 pole x 8 sources on the 32^3 sample mesh of the same "
                       "generator, timed here (%.1f s wall, %.1f s CPU over its threads), x16 "
                       "poles x %.1f, the measured ratio of the oracle's 64^3 pole (%.0f s "
                       "factor+solve, peak %.0f GB) to the same 32^3 sample on one host (%s, "
                       "%s CPUs)" % (dt, cpu, ratio, pole64, rec["peak_rss_gb"],
                                     host.get("Model name", "?"), host.get("CPU(s)", "?")),
                oracle_hex64_pole_s=pole64,
                oracle_hex64_vjp_per_pole_s=rec["vjp_s"])


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
    ap.add_argument("--inversion", action="store_true",
                    help="only run the four-block Gauss-Newton inversion and the runtime-model "
                         "fit (prints its own JSON line)")
    ap.add_argument("--inversion-precision", type=int, default=1)
    ap.add_argument("--tet", action="store_true",
                    help="only run the tetrahedral-mesh workload (prints its own JSON line)")
    ap.add_argument("--tet-cubes", type=int, default=48)
    ap.add_argument("--no-tet", action="store_true",
                    help="skip the tetrahedral-mesh phase of the default run")
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
    if args.inversion:
        print(json.dumps(inversion_phase(torch, dev, args.inversion_precision)), flush=True)
        return
    if args.tet:
        print(json.dumps(tet_phase(torch, dev, args.steps, args.warmup, args.tet_cubes,
                                   not args.no_autotune)), flush=True)
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
    if not args.no_tet:
        # the paper's discretisation: the same step on a 48^3-cube tetrahedral mesh
        tl = tet_phase(torch, dev, 1, 1, args.tet_cubes, not args.no_autotune)
        phases["tet"] = dict(config=tl["config"], phases=tl["phases"], accuracy=tl["accuracy"],
                             roofline=tl["roofline"], sweep=tl["sweep"])
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
        line["cpu_baseline"] = cpu_baseline()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
