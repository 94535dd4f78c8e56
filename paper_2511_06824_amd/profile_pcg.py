"""Profiling driver: short joint solves on the 2048 x 1024 textured workload, with the
two-launch iteration (Table 1 as printed: k_pcg_a, k_pcg_b), the whole-ring one-launch
iteration (k_pcg_f) and the strip iteration (k_pcg_w), plus a plain device copy of known
size, for hardware-counter runs (rocprofv3 --pmc / --kernel-trace).

    python3 paper_2511_06824_amd/profile_pcg.py [--iterations N] [--copy-mib M] [--no-tune]
                                                [--iteration strips|one|two|all]
    python3 paper_2511_06824_amd/profile_pcg.py --summarize FETCH_CSV WRITE_CSV

The copy (a device-to-device copy, M MiB read and M MiB written) calibrates what the
FETCH_SIZE / WRITE_SIZE counters read per byte actually moved.  --summarize reads the two
counter-collection CSVs of such runs (no GPU needed) and prints the calibrated bytes per
launch of each iteration kernel in the steady state: a solve's first launch (j = 0, no
u_prev yet) and its closing launch (which only reads the partials and stops) are left out,
and the one-launch kernels are averaged over odd and even iterations separately, since p
moves on odd iterations only.
"""

import argparse
import csv
import os
import sys

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))


def _dispatches(path, counter):
    """{kernel name: [counter value in KiB by dispatch order]} from a rocprofv3 counter CSV."""
    out = {}
    with open(path) as f:
        for row in csv.DictReader(f):
            if row.get("Counter_Name") != counter:
                continue
            out.setdefault(row["Kernel_Name"], []).append((int(row["Dispatch_Id"]), float(row["Counter_Value"])))
    return {k: [v for _, v in sorted(x)] for k, x in out.items()}


def _is_initial_residual(name):
    """Whether a PCG kernel name is an initial-residual instantiation: the INIT template
    argument is the fourth of k_pcg_w<Q, PK, M, INIT, SYNC> and the last of k_pcg_b / k_pcg_f
    <NT, Q, INIT>."""
    args = [x.strip() for x in name[name.index("<") + 1:name.index(">")].split(",")]
    if name.startswith("void k_pcg_w"):
        return args[3] == "true"
    return len(args) == 3 and args[2] == "true"


def summarize(fetch_csv, write_csv, copy_mib=1024):
    fetch, write = _dispatches(fetch_csv, "FETCH_SIZE"), _dispatches(write_csv, "WRITE_SIZE")
    copy_kib = copy_mib * 1024.0
    cf = [v for v in fetch.get("__amd_rocclr_copyBuffer", []) if v > copy_kib / 4]
    cw = [v for v in write.get("__amd_rocclr_copyBuffer", []) if v > copy_kib / 4]
    if not cf or not cw:
        raise SystemExit("no calibration copy found in the counter files")
    sf = copy_kib / (sum(cf) / len(cf))
    sw = copy_kib / (sum(cw) / len(cw))
    print(f"calibration: FETCH_SIZE {sum(cf) / len(cf):.1f} KiB per copy of {copy_kib:.0f} KiB -> scale {sf:.3f}; "
          f"WRITE_SIZE {sum(cw) / len(cw):.1f} KiB -> scale {sw:.3f}")
    print("| kernel | launches used | FETCH_SIZE KiB | WRITE_SIZE KiB | HBM bytes (scaled) |")
    print("|---|---|---|---|---|")
    mean = lambda x: sum(x) / len(x)
    for name in sorted(fetch):
        if not name.startswith("void k_pcg_") or _is_initial_residual(name):
            continue
        f, w = fetch[name][1:-1], write.get(name, [])[1:-1]
        if not f or len(f) != len(w):
            continue
        short = name.split("(")[0].replace("void ", "").replace(" ", "")
        if short.startswith("k_pcg_f") or short.startswith("k_pcg_w"):
            groups = [("odd j", f[0::2], w[0::2]), ("even j", f[1::2], w[1::2])]
            tot = []
            for label, ff, ww in groups:
                b = mean(ff) * 1024 * sf + mean(ww) * 1024 * sw
                tot.append(b)
                print(f"| {short}, {label} | {len(ff)} | {mean(ff):.1f} | {mean(ww):.1f} | {b:.0f} |")
            print(f"| {short}, average | {len(f)} | | | {mean(tot):.0f} |")
        else:
            b = mean(f) * 1024 * sf + mean(w) * 1024 * sw
            print(f"| {short} | {len(f)} | {mean(f):.1f} | {mean(w):.1f} | {b:.0f} |")


def main():
    if len(sys.argv) >= 2 and sys.argv[1] == "--summarize":
        if len(sys.argv) != 4:
            raise SystemExit("usage: profile_pcg.py --summarize FETCH_CSV WRITE_CSV")
        summarize(sys.argv[2], sys.argv[3])
        return
    ap = argparse.ArgumentParser()
    ap.add_argument("--iterations", type=int, default=20)
    ap.add_argument("--copy-mib", type=int, default=1024)
    ap.add_argument("--workload", default="joint_textured_2048x1024")
    ap.add_argument("--no-tune", action="store_true")
    ap.add_argument("--iteration", choices=["strips", "one", "two", "all"], default="all")
    ap.add_argument("--strip-config", default=None,
                    help="Q,W: the strip kernel's columns per lane and workgroups per CU (instead of tuning it)")
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
             "strips": [G.GAP_ITERATION_STRIPS],
             "all": [G.GAP_ITERATION_TWO_LAUNCH, G.GAP_ITERATION_ONE_LAUNCH,
                     G.GAP_ITERATION_STRIPS]}[args.iteration]
    if args.strip_config:
        q, w = (int(x) for x in args.strip_config.split(","))
        print(f"profile: strip configuration {s.set_strip_config(q, w)}", flush=True)
    for it in kinds:
        if it == G.GAP_ITERATION_STRIPS and args.strip_config:
            pass
        elif not args.no_tune:
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
