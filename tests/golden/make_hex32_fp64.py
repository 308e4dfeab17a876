"""Write the FP64 oracle's outputs for the whole 32^3 workload.

Calls only ``oracle/`` and the seeded input generators of ``tem_inputs``;
nothing here comes from the GPU library.  The workload is the 32^3 mesh
(h = 25 m, 4 air layers, smoothed random earth with a 1 S/m block, 4 loop
sources, 4 x 4 dB_z/dt receivers, 40 times, 12 contour poles).  Kept in
``hex32_fp64.npz``:

* ``qg``    (m, R, S) complex: Q g_is for every pole and source
  (Algorithm 1);
* ``d``     (S, K, R): the data 2 Re sum_i alpha_ij (Q g_is)_r at every time,
  and ``cond`` the summation condition sum_i 2 |alpha_ij| |(Q g_is)_r|;
* ``jv``    (S, K, R): J v for v = default_rng(21) normal values (P);
* ``jtw``   (P,): J^T w for w = default_rng(22) normal values (S, K, R)
  (section "Jacobian computation").

Usage: python tests/golden/make_hex32_fp64.py   (a few minutes on 8 cores,
about 20 GB of host memory: the oracle keeps the 12 sparse LU factors)
"""
from __future__ import annotations

import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import tem_inputs as ti  # noqa: E402
from oracle.tem import OracleTEM  # noqa: E402


def seeded_vectors(P, shape):
    """v and w of the 32^3 golden: v ~ N(0, 1)^P, w ~ N(0, 1)^shape."""
    return (np.random.default_rng(21).standard_normal(P),
            np.random.default_rng(22).standard_normal(shape))


def main(out=os.path.join(HERE, "hex32_fp64.npz")):
    t0 = time.perf_counter()
    wl = ti.workload(1)
    me = wl.mesh
    o = OracleTEM(me.nx, me.ny, me.nz, me.h, wl.sigma, wl.F, wl.rx.ptr, wl.rx.col, wl.rx.val,
                  wl.poles.xi, wl.poles.alpha, wl.params)
    G = o.solve_poles()
    qg = o.observe(G)
    d = o.data()
    cond = o.data_condition()
    v, w = seeded_vectors(len(wl.params), d.shape)
    jv = o.jvp(v)
    jtw = o.vjp(w)
    np.savez_compressed(out, qg=qg, d=d, cond=cond, jv=jv, jtw=jtw)
    print("wrote %s in %.1f s" % (out, time.perf_counter() - t0), flush=True)


if __name__ == "__main__":
    main()
