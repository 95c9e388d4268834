"""Write the stored expected values under tests/golden/ from the oracle alone.

  python tests/golden/make_golden.py [--c3-gens N] [--batched]

Outputs
  graphs_manifest.json   SHA-256 of every synthetic graph the tests and the
                         benchmark use (pins the seeded generators).
  trajectories.json      per-generation hash of (population, fitness) of the
                         oracle GA for the named workloads.
Everything here calls only the seeded input generators and ``oracle/``.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import cnd_oracle as O  # noqa: E402
from paper_2412_20980_amd import inputs  # noqa: E402


def state_hash(pop, F) -> str:
    h = hashlib.sha256()
    h.update(pop.astype("<i4").tobytes())
    h.update(F.astype("<i8").tobytes())
    return h.hexdigest()[:32]


def trajectory(w: inputs.Workload, gens: int) -> dict:
    t = time.time()
    ga = O.OracleGA(w.graph, w.k, w.pop, w.seed, w.pc, w.pm, w.tournament, w.offspring)
    hashes = [state_hash(ga.pop, ga.F)]
    best = [int(ga.F[0])]
    for _ in range(gens):
        ga.step()
        hashes.append(state_hash(ga.pop, ga.F))
        best.append(int(ga.F[0]))
    print(f"{w.name}: {gens} generations in {time.time() - t:.1f}s, best {best[0]} -> {best[-1]}", flush=True)
    return {"graph_sha256": w.graph.sha256(), "k": w.k, "pop": w.pop, "seed": w.seed, "pc": w.pc, "pm": w.pm,
            "tournament": w.tournament, "generations": gens, "hash": hashes, "best": best}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--c3-gens", type=int, default=3)
    ap.add_argument("--batched", action="store_true", help="also record the 64-instance batched workload")
    args = ap.parse_args()

    manifest = {}
    for name, fn in (("ba200", inputs.ba200), ("ba10k", inputs.ba10k), ("chung_lu_200k", inputs.chung_lu_200k)):
        g = fn()
        manifest[name] = {"n": g.n, "m": g.m, "sha256": g.sha256()}
    inst = inputs.batched_instances()
    manifest["batched_sizes"] = [w.graph.n for w in inst]
    manifest["batched"] = [{"n": w.graph.n, "m": w.graph.m, "sha256": w.graph.sha256()} for w in inst]
    with open(os.path.join(HERE, "graphs_manifest.json"), "w") as f:
        json.dump(manifest, f, indent=1)

    traj = {}
    path = os.path.join(HERE, "trajectories.json")
    if os.path.exists(path):
        with open(path) as f:
            traj = json.load(f)
    w1 = inputs.workload("ba200_k10_p32")
    traj[w1.name] = trajectory(w1, w1.generations)
    w2 = inputs.workload("ba10k_k100_p256")
    traj[w2.name] = trajectory(w2, w2.generations)
    w3 = inputs.workload("cl200k_k2000_p1024")
    traj[w3.name] = trajectory(w3, args.c3_gens)
    if args.batched:
        traj["batched"] = [trajectory(w, w.generations) for w in inst]
    with open(path, "w") as f:
        json.dump(traj, f, indent=1)


if __name__ == "__main__":
    main()
