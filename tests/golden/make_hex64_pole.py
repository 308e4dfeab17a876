"""Write the FP64 oracle's values for one pole of the 64^3 precision workload.

Calls only ``oracle/`` and the seeded input generators of ``tem_inputs``;
nothing here comes from the GPU library.  The workload is the 64^3 mesh
(h = 25 m, 8 air layers, smoothed random earth with a 1 S/m block, 8 loop
sources, 4 x 4 dB_z/dt receivers, 60 times, 16 contour poles).  For pole
``--pole`` (default 0, the pole of smallest modulus and the one nearest the
negative real axis) the script keeps

* ``qg``   (R, S) complex: Q g_s with g_s = (K - xi M)^{-1} f_s
  (Algorithm 1, one pole);
* ``d``    (S, K, R): that pole's term 2 Re alpha_j (Q g_s)_r of the data,
  and ``cond`` its summation condition 2 |alpha_j| |(Q g_s)_r|;
* ``jv``   (S, K, R): that pole's term of J v for the seeded v of the
  benchmark (section "Jacobian computation");
* that pole's term of J^T w for the seeded w of the benchmark, as its
  2-norm, its inner products with two seeded unit-normal vectors and its
  values at 4096 seeded parameter cells (the whole vector is 229,376
  doubles).

v and w are drawn as the benchmark draws them: default_rng(7), v first
(P normal values), then w (S x K x R normal values).

The oracle's phase times and the host (lscpu model, CPUs, peak memory) are
written to ``profiles/oracle_hex64_pole_cpu.json``; the script also times
the same factor + solve on the 32^3 mesh the benchmark's CPU leg samples,
so that the two sizes are measured on one host.

Usage: python tests/golden/make_hex64_pole.py [--pole 0]   (about 20-30 min
and up to ~40 GB of host memory on 8 cores)
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import resource
import subprocess
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import tem_inputs as ti  # noqa: E402
from oracle.tem import OracleTEM  # noqa: E402

N_SAMPLE = 4096


def _lscpu():
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True).stdout
    except OSError:
        return {}
    keep = ("Model name", "CPU(s)", "Thread(s) per core", "Core(s) per socket", "Socket(s)")
    rec = {}
    for line in out.splitlines():
        k, _, v = line.partition(":")
        if k.strip() in keep:
            rec[k.strip()] = v.strip()
    return rec


def _timed(fn):
    c0, t0 = time.process_time(), time.perf_counter()
    out = fn()
    return out, time.perf_counter() - t0, time.process_time() - c0


def one_pole(wl, pole):
    me = wl.mesh
    return OracleTEM(me.nx, me.ny, me.nz, me.h, wl.sigma, wl.F, wl.rx.ptr, wl.rx.col, wl.rx.val,
                     wl.poles.xi[pole:pole + 1], wl.poles.alpha[:, pole:pole + 1], wl.params)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--pole", type=int, default=0)
    ap.add_argument("--out", default=os.path.join(HERE, "hex64_pole.npz"))
    ap.add_argument("--record", default=os.path.join(ROOT, "profiles", "oracle_hex64_pole_cpu.json"))
    args = ap.parse_args()
    wl = ti.workload(2)
    P = len(wl.params)
    K, R = len(wl.poles.t), wl.rx.n
    rng = np.random.default_rng(7)
    v = rng.standard_normal(P)
    w = rng.standard_normal((wl.S, K, R))
    o = one_pole(wl, args.pole)
    times = {}
    _, times["ordering_s"], _ = _timed(o.ordering)
    _, times["factor_s"], times["factor_cpu_s"] = _timed(lambda: o.lu(0))
    print("factor %.1f s" % times["factor_s"], flush=True)
    G, times["solve_s"], times["solve_cpu_s"] = _timed(o.solve_poles)
    qg = o.observe(G)[0]                                   # (R, S)
    d = o.data()
    cond = o.data_condition()
    jv, times["jvp_s"], _ = _timed(lambda: o.jvp(v))
    jtw, times["vjp_s"], _ = _timed(lambda: o.vjp(w))
    print("solve %.1f s, jvp %.1f s, vjp %.1f s" % (times["solve_s"], times["jvp_s"],
                                                    times["vjp_s"]), flush=True)
    srng = np.random.default_rng(11)
    idx = np.sort(srng.choice(P, N_SAMPLE, replace=False))
    proj = srng.standard_normal((2, P))
    peak_gb = resource.getrusage(resource.RUSAGE_SELF).ru_maxrss / 1e6
    np.savez_compressed(args.out, pole=args.pole, xi=wl.poles.xi[args.pole],
                        alpha=wl.poles.alpha[:, args.pole], qg=qg, d=d, cond=cond, jv=jv,
                        jtw_norm=np.linalg.norm(jtw), jtw_proj=proj @ jtw, jtw_idx=idx,
                        jtw_sample=jtw[idx])
    del o, G
    # the 32^3 sample of the benchmark's CPU leg, timed on the same host
    ws = ti.smooth_workload(32, 4, S=8, m=16, K=60, g=4, seed=3, name="hex32_sample")
    o32 = one_pole(ws, 0)
    o32.ordering()
    _, t32, c32 = _timed(lambda: o32.solve(0, o32.F))
    rec = dict(workload="hex64_precision, pole %d of 16, 8 sources" % args.pole,
               host=_lscpu(),
               python=platform.python_version(), numpy=np.__version__,
               threads_env={k: os.environ.get(k) for k in ("OMP_NUM_THREADS",
                                                            "OPENBLAS_NUM_THREADS")},
               peak_rss_gb=peak_gb, **times,
               hex32_sample_factor_solve_s=t32, hex32_sample_factor_solve_cpu_s=c32,
               ratio_hex64_over_hex32=(times["factor_s"] + times["solve_s"]) / t32,
               threads_used_factor=times["factor_cpu_s"] / times["factor_s"],
               command="python tests/golden/make_hex64_pole.py --pole %d" % args.pole)
    with open(args.record, "w") as f:
        json.dump(rec, f, indent=1)
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
