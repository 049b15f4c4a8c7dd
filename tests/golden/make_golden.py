"""Write the stored oracle values used by the GPU parity tests.

Calls only the CPU oracle and the seeded input generators.  Each file records the
workload recipe next to the values:

    python tests/golden/make_golden.py small     # Gamma-only and 3x3x1 systems, all points
    python tests/golden/make_golden.py sampled   # sampled points of the two large systems
    python tests/golden/make_golden.py dual      # the 3x3x1 slab on dual k/q grids, all points
    python tests/golden/make_golden.py sampledao # sampled points of the atomic-orbital slab
    python tests/golden/make_golden.py sampled2400  # the 3x3x1 N_aux 2400 slab (adds missing points)
"""
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import rpa_oracle as orc          # noqa: E402
from paper_2505_06021_amd import inputs        # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))


def write(name, payload):
    with open(os.path.join(HERE, name + ".json"), "w") as f:
        json.dump(payload, f, indent=1)


def recipe(s):
    return dict(name=s.name, grid=list(s.grid), nocc=s.nocc, nvirt=s.nvirt, naux=s.naux,
                nw=s.nw, seed=s.seed, sigma=s.sigma, is_complex=s.is_complex)


def full(make):
    s = make()
    t = time.time()
    E, g = orc.energy(s)
    return dict(recipe=recipe(s), E=E, eps=g.tolist(), oracle_seconds=time.time() - t)


def sampled(make, pts, keep=None):
    """Oracle values of the listed (q, j) points.  keep: a file this script wrote before
    for the same recipe; its points are reused and only the missing ones are computed."""
    s = make()
    old = {}
    if keep and os.path.exists(os.path.join(HERE, keep + ".json")):
        prev = json.load(open(os.path.join(HERE, keep + ".json")))
        if prev["recipe"] == recipe(s):
            old = {(p["iq"], p["j"]): p for p in prev["points"]}
    out = []
    t = time.time()
    for iq, j in pts:
        if (iq, j) in old:
            out.append(old[(iq, j)])
            continue
        out.append(dict(iq=iq, j=j, omega=float(s.omega[j]), eps=orc.point(s, iq, j, row_block=4)))
        print(f"  point q={iq} j={j}: {out[-1]['eps']!r}  ({time.time() - t:.0f} s)", flush=True)
    return dict(recipe=recipe(s), points=out, oracle_seconds=time.time() - t)


if __name__ == "__main__":
    what = sys.argv[1] if len(sys.argv) > 1 else "small"
    if what == "small":
        write("gamma_real_naux128", full(inputs.gamma_real_128))
        write("slab3x3_naux384", full(inputs.slab_3x3_384))
    elif what == "dual":
        g = full(inputs.slab_3x3_dual_384)
        g["recipe"]["dual_grid_frac"] = 0.1
        write("slab3x3_dual_naux384", g)
    elif what == "sampledao":
        g = sampled(inputs.slab_3x3_ao_384, [(0, 0), (4, 7)])
        g["recipe"].update(nbas=144, n_lowdep=4, eps_d=1e-4)
        write("slab3x3_ao_naux384_sampled", g)
    elif what == "sampled6x6":
        write("slab6x6_naux1200_sampled", sampled(inputs.slab_6x6_1200, [(0, 0), (0, 7), (17, 0), (17, 7)]))
    elif what == "sampled2400":
        # two pairs of points on one q each, so that the paired (two frequencies per
        # workgroup) contraction runs on an oracle-checked pair at this size
        name = "slab3x3_naux2400_sampled"
        write(name, sampled(inputs.slab_3x3_2400, [(0, 0), (0, 15), (4, 7), (4, 8)], keep=name))
