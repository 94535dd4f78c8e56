"""Preconditioner study on the GPU path: Jacobi (Eq 2.8), ASSOR I (Eq 3.2) and ASSOR II
(Eq 3.3-3.6) with the relaxation factor swept over omega = 0.1 + 0.18 i, i = 0..10 (the grid
of the paper's omega study), on one assembled joint system.  Every solve runs on the HIP
kernels through the C ABI; the study only chooses options and reads the clock.

    python3 -m paper_2511_06824_amd.study [--workload joint_smooth_512x256] [--seed 0]
"""

import argparse
import json
import os
import sys
import time

PRECONDS = {"jacobi": 0, "assor1": 1, "assor2": 2}
OMEGAS = [round(0.1 + 0.18 * i, 2) for i in range(11)]


def precond_study(solver, eps=1e-10, omegas=OMEGAS, preconds=("jacobi", "assor1", "assor2"), repeats=1):
    """Solve the assembled system of `solver` (a JointGapSolver) for every preconditioner and
    omega; returns rows of {precond, omega, iterations, ms_per_solve, us_per_iteration}.
    Jacobi does not depend on omega and is run once."""
    import torch
    rows = []
    for name in preconds:
        for omega in ([1.0] if name == "jacobi" else omegas):
            opts = solver.options(omega=omega, eps=eps, precond=PRECONDS[name])
            _, info = solver.solve(opts)                       # warm-up (kernels, graphs, diagonals)
            best = None
            for _ in range(repeats):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                _, info = solver.solve(opts)
                torch.cuda.synchronize()
                dt = time.perf_counter() - t0
                best = dt if best is None else min(best, dt)
            rows.append({"precond": name, "omega": None if name == "jacobi" else omega,
                         "iterations": info.iterations, "ms_per_solve": round(1e3 * best, 3),
                         "us_per_iteration": round(1e6 * best / max(info.iterations, 1), 2)})
    return rows


def summarize(rows):
    """Best omega per preconditioner and the iteration ratio of the best ASSOR II to Jacobi."""
    out = {}
    for name in PRECONDS:
        rs = [r for r in rows if r["precond"] == name]
        if rs:
            b = min(rs, key=lambda r: (r["iterations"], r["ms_per_solve"]))
            out[name] = {"omega": b["omega"], "iterations": b["iterations"], "ms_per_solve": b["ms_per_solve"]}
    if "jacobi" in out and "assor2" in out:
        out["assor2_over_jacobi_iterations"] = round(out["assor2"]["iterations"] / out["jacobi"]["iterations"], 3)
        out["assor2_over_jacobi_time"] = round(out["assor2"]["ms_per_solve"] / out["jacobi"]["ms_per_solve"], 3)
    return out


def main():
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", default="joint_smooth_512x256")
    ap.add_argument("--seed", type=int, default=0)
    args = ap.parse_args()
    import synth
    from paper_2511_06824_amd.solver import JointGapSolver
    case = synth.make_case(args.workload, args.seed)
    s = JointGapSolver.from_case(case, max_cond=9)
    s.assemble(case.e, case.edot, case.delta, 9)
    s.tune(iterations=20, omega=case.omega)
    rows = precond_study(s, eps=case.eps)
    for r in rows:
        print(json.dumps(r), flush=True)
    print(json.dumps({"workload": args.workload, "summary": summarize(rows)}), flush=True)
    s.close()


if __name__ == "__main__":
    main()
