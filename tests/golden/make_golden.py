"""Writes the stored oracle values of the large workloads, from ``oracle/`` alone.

The oracle's exact solves at these sizes take minutes and tens of GB of memory, too much
for a test run, so their results are stored here and the GPU tests read them.  Nothing
below touches the GPU library: inputs come from ``synth``, every number from ``oracle``.

    python tests/golden/make_golden.py joint_textured_2048x1024   # ~34 GB, ~10 min
    python tests/golden/make_golden.py adjoint_textured_1024x512  # ~5 GB, ~10 min

joint_textured_2048x1024 (seed 0): the exact discrete pressure p* = A^-1 S of conditions
0, 1 and 5 of Eq 2.17-2.19 by banded Cholesky (natural order, bandwidth n_theta); conditions
0 and 5 share A_0, so two factorizations.  Stored per condition: the forces of p*
(Fx, Fy, Mx, My), ||p*||_2, the true residual of p*, a strided sample of p* and four
random projections w_m . p* with the seeded weights of ``synth.projection_weights``.

adjoint_textured_1024x512 (seed 0): the 4 x 8 Jacobian d(Fx, Fy, Mx, My)/d(e1..e4,
edot1..edot4) three ways: the complex-step derivative (exact for this analytic map), central
differences with banded-Cholesky solves at the step of Eq 2.17-2.19, and the forward
differences of Eq 2.13-2.14 over the 9 conditions; plus the base forces.
"""

import json
import os
import platform
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import synth  # noqa: E402


def gap_and_texture(case):
    gap = oracle.Gap(R=case.R, c=case.c, L=case.L, mu=case.mu, U=case.U, V=case.V, p_in=case.p_in,
                     p_out=case.p_out, n_theta=case.n_theta, n_axial=case.n_axial)
    if case.n_dimples == 0:
        return gap, oracle.no_texture
    return gap, oracle.dimple_texture(case.R, case.dimple_theta, case.dimple_z, case.dimple_radius,
                                      case.dimple_depth)


def log(msg):
    print(f"[{time.strftime('%H:%M:%S')}] {msg}", flush=True)


def provenance(name, extra):
    d = {"generator": f"python tests/golden/make_golden.py {name}",
         "written": time.strftime("%Y-%m-%d"), "numpy": np.__version__, "python": platform.python_version()}
    d.update(extra)
    return d


def joint_textured_2048x1024():
    name = "joint_textured_2048x1024"
    case = synth.make_case(name, 0)
    gap, tex = gap_and_texture(case)
    nt, nz = case.n_theta, case.n_axial
    conds = oracle.conditions(case.e, case.edot, case.delta)
    rows, cols = synth.golden_sample_index(nt, nz)
    W = synth.projection_weights(nt * nz)
    out = {}
    for group in ((0, 5), (1,)):
        A, S0 = oracle.assemble(gap, *conds[group[0]], tex)
        rhs = [S0]
        for k in group[1:]:
            Ak, Sk = oracle.assemble(gap, *conds[k], tex)
            if (Ak != A).nnz != 0:
                raise RuntimeError(f"condition {k} does not share the operator of condition {group[0]}")
            del Ak
            rhs.append(Sk)
        log(f"factor the operator of conditions {group} (n {A.shape[0]}, bandwidth {nt})")
        t = time.time()
        cb = oracle.band_factor(A, nt)
        log(f"  factorized in {time.time() - t:.0f} s")
        P = oracle.band_solve(cb, np.stack(rhs, axis=1))
        del cb
        for col, k in enumerate(group):
            p, S = P[:, col], rhs[col]
            F = oracle.forces_for_condition(gap, conds[k][0], p, tex)
            res = float(np.linalg.norm(S - A @ p) / np.linalg.norm(S))
            out[str(k)] = {
                "e": list(map(float, conds[k][0])), "edot": list(map(float, conds[k][1])),
                "forces": [float(x) for x in F],
                "norm": float(np.linalg.norm(p)),
                "true_rel_residual": res,
                "projections": [float(x) for x in W @ p],
                "sample": p.reshape(nz, nt)[np.ix_(rows, cols)].tolist(),
            }
            log(f"  condition {k}: F {F}, ||p*|| {np.linalg.norm(p):.6e}, residual {res:.2e}")
        del A, P
    doc = provenance(name, {
        "about": "Exact discrete pressure p* = A^-1 S (banded Cholesky, oracle.band_factor / band_solve) of "
                 "conditions 0, 1, 5 of the joint textured 2048 x 1024 workload, seed 0, and the forces "
                 "oracle.forces_for_condition gives for it (cavitation none).",
        "workload": name, "seed": 0, "n_theta": nt, "n_axial": nz,
        "sample_rows": rows.tolist(), "sample_cols": cols.tolist(),
        "projection": "synth.projection_weights(n_theta * n_axial) (4 x n, seeds 7000..7003) @ p*",
        "conditions": out})
    return name, doc


def adjoint_textured_1024x512():
    name = "adjoint_textured_1024x512"
    case = synth.make_case(name, 0)
    gap, tex = gap_and_texture(case)
    log("complex-step Jacobian")
    J_cs = oracle.jacobian_complex_step(gap, case.e, case.edot, tex)
    log("central differences, banded Cholesky")
    J_c = oracle.jacobian_central(gap, case.e, case.edot, case.delta, tex)
    log("forward differences over the 9 conditions, banded Cholesky")
    F9 = np.stack([oracle.condition_forces(gap, ek, edk, tex)[0]
                   for ek, edk in oracle.conditions(case.e, case.edot, case.delta)])
    J_f = oracle.jacobian_fd(F9, case.delta)
    doc = provenance(name, {
        "about": "Jacobian d(Fx, Fy, Mx, My)/d(e1..e4, edot1..edot4) of the textured 1024 x 512 workload, "
                 "seed 0, cavitation none: oracle.jacobian_complex_step (exact derivative), "
                 "oracle.jacobian_central and oracle.jacobian_fd (Eq 2.13-2.14) with banded-Cholesky solves "
                 "at the steps delta of Eq 2.17-2.19; rows Fx, Fy, Mx, My.",
        "workload": name, "seed": 0, "n_theta": case.n_theta, "n_axial": case.n_axial,
        "delta": case.delta.tolist(),
        "forces_9": F9.tolist(),
        "jacobian_complex_step": J_cs.tolist(),
        "jacobian_central": J_c.tolist(),
        "jacobian_forward": J_f.tolist()})
    return name, doc


TARGETS = {"joint_textured_2048x1024": joint_textured_2048x1024,
           "adjoint_textured_1024x512": adjoint_textured_1024x512}


def main(argv):
    for target in argv or list(TARGETS):
        name, doc = TARGETS[target]()
        path = os.path.join(HERE, f"{name}_seed0.json")
        with open(path, "w") as f:
            json.dump(doc, f, indent=1)
            f.write("\n")
        log(f"wrote {path}")


if __name__ == "__main__":
    main(sys.argv[1:])
