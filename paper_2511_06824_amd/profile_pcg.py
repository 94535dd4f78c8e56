"""Profiling driver: short joint solves on the 2048 x 1024 textured workload, with the
two-launch iteration (Table 1 as printed: k_pcg_a, k_pcg_b) and the one-launch iteration
(k_pcg_f), plus a plain device copy of known size, for hardware-counter runs (rocprofv3
--pmc / --kernel-trace).

    python3 paper_2511_06824_amd/profile_pcg.py [--iterations N] [--copy-mib M] [--no-tune]
                                                [--iteration one|two|both]

The copy (torch's elementwise copy kernel, M MiB read and M MiB written) calibrates what
the FETCH_SIZE / WRITE_SIZE counters read per byte actually moved.
"""

import argparse
import os
import sys

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--iterations", type=int, default=20)
    ap.add_argument("--copy-mib", type=int, default=1024)
    ap.add_argument("--workload", default="joint_textured_2048x1024")
    ap.add_argument("--no-tune", action="store_true")
    ap.add_argument("--iteration", choices=["one", "two", "both"], default="both")
    args = ap.parse_args()

    import torch
    import synth
    from paper_2511_06824_amd import gapsolve as G
    from paper_2511_06824_amd.solver import JointGapSolver

    dev = torch.device("cuda:0")
    n = args.copy_mib * (1 << 20) // 8
    src = torch.ones(n, dtype=torch.float64, device=dev)
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(f"profile: copy of {args.copy_mib} MiB done 3 times", flush=True)

    case = synth.make_case(args.workload, 0)
    s = JointGapSolver.from_case(case, max_cond=9, device=dev)
    s.assemble(case.e, case.edot, case.delta, 9)
    kinds = {"two": [G.GAP_ITERATION_TWO_LAUNCH], "one": [G.GAP_ITERATION_ONE_LAUNCH],
             "both": [G.GAP_ITERATION_TWO_LAUNCH, G.GAP_ITERATION_ONE_LAUNCH]}[args.iteration]
    for it in kinds:
        if not args.no_tune:
            cfg, _ = s.tune(iterations=20, omega=case.omega, iteration=it)   # the configuration the benchmark times
            print(f"profile: iteration kind {it}, PCG kernel configuration {cfg}", flush=True)
        _, info = s.solve(omega=case.omega, eps=1e-30, max_iter=args.iterations, check_every=args.iterations,
                          raise_on_error=False, iteration=it)
        s.integrate()
        torch.cuda.synchronize()
        print(f"profile: {case.label}, iteration kind {it}, {info.iterations} PCG iterations", flush=True)
    s.close()


if __name__ == "__main__":
    main()
