"""Write tests/golden/oracle_records.json: the oracle's full state (as
digests, see tests/parity_util.py) after runs at the workloads' real shapes
that take the oracle minutes, for the GPU parity tests to compare with.

TEST INFRASTRUCTURE: runs only the oracle (oracle/) on inputs described by
qsg_workloads; nothing here touches the HIP library.

    python tests/golden/make_oracle_records.py [--threads N] [--only NAME]

Cases:
  production_g0: the production shape (L=24, L_tau=2048, beta=128, 48 Gammas
      geometric in [2.8, 3.6], 64 samples one per lane: J seeds 1..64, group
      0 of 2), 10 sweeps and the PT step after sweep 10 (every slot, the
      exchange tables of every pair);
  uneven_17, uneven_82, uneven_16: samples 17 (L=20, L_tau=256, 39 Gammas),
      82 (L=24, L_tau=256, 42 Gammas) and 16 (L=20, L_tau=64, 40 Gammas) of
      the 256-sample uneven ensemble, 20 sweeps with PT every 10;
  ladder_eval_learned_0, ladder_eval_learned_3: samples 0 and 3 of the
      learned-ladder evaluation set (L_tau=256, beta=16),
      each on a 32-point ladder decoded from the oracle MLP with fixed
      parameters (init_params(7) scaled by 0.5) and the sample's features
      (samples 0 and 3 have L = 20 and L = 24),
      20 sweeps with PT every 10.  The ladders are stored as exact doubles.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import qsg_workloads as W  # noqa: E402
from oracle import chain, mlp  # noqa: E402
from tests.parity_util import oracle_record  # noqa: E402

OUT = os.path.join(HERE, "oracle_records.json")
LEARNED_EVAL_SAMPLES = (0, 3)
MLP_SEED, MLP_SCALE = 7, 0.5


def frustrated_fraction(Jx, Jy, L, lane=0):
    """Fraction of plaquettes (x,y)-(x+1,y)-(x+1,y+1)-(x,y+1) whose four
    couplings multiply to -1 (bit 1 <=> J = -1)."""
    bit = lambda w: (int(w) >> lane) & 1
    odd = 0
    for y in range(L):
        for x in range(L):
            s = (bit(Jx[x + L * y]) + bit(Jy[(x + 1) % L + L * y]) +
                 bit(Jx[x + L * ((y + 1) % L)]) + bit(Jy[x + L * y]))
            odd += s & 1
    return odd / (L * L)


def learned_ladder(g):
    """32-point ladder of the oracle MLP for group g's features."""
    Jx, Jy = chain.couplings(g.L, g.j_seeds)
    ff = frustrated_fraction(Jx, Jy, g.L)
    gmin, gmax = float(g.gammas[0]), float(g.gammas[-1])
    x = np.array([[g.L / 16.0, math.log2(g.L_tau) / 8.0, math.log(g.beta) / 4.0,
                   (ff - 0.5) * 4.0, math.log(gmin), math.log(gmax)]])
    z = mlp.forward(mlp.init_params(MLP_SEED) * MLP_SCALE, x)["out"]
    return mlp.decode(z, [gmin], [gmax])[0]


def cases():
    out = {}
    prod = W.production()
    out["production_g0"] = dict(group=prod.groups[0], sweeps=10, pt_every=10, index=0,
                                workload="production")
    un = W.uneven_ensemble()
    for i in (17, 82, 16):
        out[f"uneven_{i}"] = dict(group=un.groups[i], sweeps=20, pt_every=10, index=i,
                                  workload="uneven")
    ev = W.ladder_eval()
    for i in LEARNED_EVAL_SAMPLES:
        g = ev.groups[i]
        lad = learned_ladder(g)
        from dataclasses import replace
        out[f"ladder_eval_learned_{i}"] = dict(group=replace(g, gammas=lad), sweeps=20,
                                               pt_every=10, index=i, workload="ladder-eval",
                                               ladder_hex=[float(v).hex() for v in lad])
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--threads", type=int, default=len(os.sched_getaffinity(0)))
    ap.add_argument("--only", default=None)
    a = ap.parse_args()
    data = json.load(open(OUT)) if os.path.exists(OUT) else {}
    for name, c in cases().items():
        if a.only and name != a.only:
            continue
        g = c["group"]
        t0 = time.time()
        og = chain.OracleGroup.from_workload_group(g, log_cap=16)
        og.run(c["sweeps"], c["pt_every"], threads=a.threads)
        rec = oracle_record(og)
        rec.update(workload=c["workload"], index=c["index"], sweeps=c["sweeps"],
                   pt_every=c["pt_every"], L=g.L, L_tau=g.L_tau, n_gamma=g.n_gamma)
        if "ladder_hex" in c:
            rec["ladder_hex"] = c["ladder_hex"]
        data[name] = rec
        print(f"{name}: L={g.L} L_tau={g.L_tau} N={g.n_gamma}, {c['sweeps']} sweeps, "
              f"{time.time() - t0:.1f} s", flush=True)
        with open(OUT, "w") as f:
            json.dump(data, f, indent=1, sort_keys=True)


if __name__ == "__main__":
    main()
