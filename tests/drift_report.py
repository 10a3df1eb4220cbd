"""Drift of the GPU forms against the FP64 oracle over many steps (a report, not a test).

Both GPU forms and the oracle step the same scene from the same state with their own
adaptive time steps; every `--every` steps the script prints the largest position
error in units of dx, the velocity error relative to the oracle's largest speed, the
density error relative to rho0, and the relative difference of the simulated times.
The trajectories of a chaotic flow separate, so no bound is asserted.

    python tests/drift_report.py --scene drop3d --steps 1000 --every 100

runs the 3D drop (335,728 particles); the oracle uses every host thread.
"""
import argparse
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--scene", default="drop3d")
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--every", type=int, default=100)
    args = ap.parse_args()
    import oracle
    from paper_1702_07760_amd import binding, inputs
    s = getattr(inputs, args.scene)()
    dx, rho0 = s.dx[0], max(p[0] for p in s.phases[0])
    print(f"drift {args.scene}: n={s.n}, oracle threads {oracle.get_threads()}", flush=True)
    o = oracle.Oracle(s)
    o.set_neighbor_method(2)
    sims = {"fp64": binding.Sim(s, precision=binding.FP64),
            "fp32": binding.Sim(s, precision=binding.FP32_CELLREL)}
    t0 = time.time()
    done = 0
    while done < args.steps:
        k = min(args.every, args.steps - done)
        o.step(k)
        done += k
        xo, uo, ro = o.get(oracle.X), o.get(oracle.U), o.get(oracle.RHO)
        ur = max(np.abs(uo).max(), 1e-30)
        row = [f"step {done:5d} t={o.t:.5f}"]
        for name, sim in sims.items():
            sim.step(k)
            sim.sync()
            ex = np.abs(sim.get_field(binding.F_X) - xo).max() / dx
            eu = np.abs(sim.get_field(binding.F_U) - uo).max() / ur
            er = np.abs(sim.get_field(binding.F_RHO) - ro).max() / rho0
            et = abs(sim.stats()["t"] - o.t) / o.t
            row.append(f"{name}: x/dx {ex:.2e} u {eu:.2e} rho {er:.2e} t {et:.1e}")
        print("  ".join(row) + f"  ({time.time() - t0:.0f} s)", flush=True)


if __name__ == "__main__":
    main()
