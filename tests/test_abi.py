"""C-ABI contract on the CPU: the library loads, exports every declared entry point, and
rejects invalid arguments before touching a device."""

import ctypes
import os
import re

import pytest

from paper_2511_06824_amd import gapsolve as G

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = []
    for fn in sorted(os.listdir(os.path.join(ROOT, "include"))):
        if not fn.endswith(".h"):
            continue
        text = open(os.path.join(ROOT, "include", fn)).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        names += re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\*?\s*([a-z_][a-z0-9_]*)\s*\(", text, flags=re.M)
    return names


@pytest.fixture(scope="module")
def lib():
    return G.load()


def test_every_declared_symbol_is_exported(lib):
    names = declared_functions()
    assert {"create_gap_grid", "destroy_gap_grid", "assemble_joint_system", "solve_joint_pcg",
            "integrate_force_moment", "jacobian_fd", "jacobian_adjoint", "solve_with_adjoint",
            "general_iteration_step", "set_operating_point", "gap_tune_pcg", "gap_get_pcg_config",
            "gap_set_pcg_config", "gap_batch_create", "gap_batch_add", "gap_batch_step", "gap_batch_hold",
            "gap_batch_poll", "gap_batch_remove", "gap_last_error"} <= set(names)
    for name in names:
        assert hasattr(lib, name), name


def test_binding_names_match_abi():
    for name in declared_functions():
        assert hasattr(G, name), name


def good_geom(**over):
    d = dict(R=0.01, clearance=2e-5, length=0.04, mu=0.04, U=2.0, V=0.0, p_in=1e7, p_out=1e5,
             n_theta=64, n_axial=32)
    d.update(over)
    return G.make_geom(**d)


@pytest.mark.parametrize("over,msg", [
    (dict(n_theta=2), "n_theta"), (dict(n_theta=16385), "n_theta"), (dict(n_axial=1), "n_axial"),
    (dict(R=-1.0), "R"), (dict(clearance=0.0), "clearance"), (dict(mu=float("nan")), "mu"),
    (dict(length=float("inf")), "length"), (dict(p_in=float("nan")), "finite")])
def test_create_rejects_bad_geometry(over, msg):
    with pytest.raises(G.GapError) as ei:
        G.create_gap_grid(good_geom(**over), None, 9)
    assert ei.value.status == G.GAP_EINVAL and msg in str(ei.value)


def test_create_rejects_bad_dimples_and_max_cond():
    with pytest.raises(G.GapError) as ei:
        G.create_gap_grid(good_geom(), G.make_dimples([0.1], [0.02], [5e-4], [6e-4]), 9)
    assert ei.value.status == G.GAP_EINVAL and "dimple 0" in str(ei.value)
    with pytest.raises(G.GapError) as ei:
        G.create_gap_grid(good_geom(), None, 4)
    assert ei.value.status == G.GAP_EINVAL
    lib = G.load()
    assert lib.create_gap_grid(ctypes.byref(good_geom()), None, 9, None) == G.GAP_EINVAL


def test_null_handle_rejected_everywhere():
    lib = G.load()
    o = G.gap_default_opts()
    d4 = (ctypes.c_double * 4)()
    d8 = (ctypes.c_double * 8)(*([1e-9] * 8))
    assert lib.assemble_joint_system(None, d4, d4, d8, 9, None) == G.GAP_EINVAL
    assert lib.solve_joint_pcg(None, ctypes.byref(o), None, None, None) == G.GAP_EINVAL
    assert lib.integrate_force_moment(None, None, 0, 0.0, None, None) == G.GAP_EINVAL
    assert lib.jacobian_fd(None, None, None, None) == G.GAP_EINVAL
    assert lib.gap_read_system(None, 0, None, None, None, None) == G.GAP_EINVAL
    assert "NULL" in G.gap_last_error()
    assert lib.destroy_gap_grid(None) == G.GAP_OK
    assert lib.gap_default_opts(None) == G.GAP_EINVAL


def test_default_opts():
    o = G.gap_default_opts()
    assert (o.omega, o.eps, o.max_iter, o.precond, o.neumann, o.scalars, o.warm_start, o.check_every, o.graph,
            o.strategy) == (1.6, 1e-10, 100000, G.GAP_PRECOND_ASSOR2, 1, G.GAP_SCALARS_GLOBAL, 0, 32, 1,
                            G.GAP_STRATEGY_SYNC)


def test_create_rejects_out_of_range_dimples():
    for th, z, a in [(1e9, 0.02, 5e-4), (0.1, 1.0, 5e-4), (0.1, 0.02, 0.05)]:
        with pytest.raises(G.GapError) as ei:
            G.create_gap_grid(good_geom(), G.make_dimples([th], [z], [a], [1e-5]), 9)
        assert ei.value.status == G.GAP_EINVAL


def test_new_entry_points_reject_null_handles(lib):
    """Argument checks that run before any device call."""
    P = ctypes.c_void_p
    assert lib.set_operating_point(None, 1.0, 0.0, 1e6, 1e5) == G.GAP_EINVAL
    assert lib.gap_batch_hold(None, 1, 1) == G.GAP_EINVAL
    assert lib.gap_get_pcg_config(None, None) == G.GAP_EINVAL
    assert lib.gap_set_pcg_config(None, None) == G.GAP_EINVAL
    assert lib.gap_pcg_history(None, 16) == G.GAP_EINVAL
    a = (ctypes.c_double * 4)()
    n = ctypes.c_int32(0)
    assert lib.gap_get_pcg_history(None, a, a, 4, ctypes.byref(n), None) == G.GAP_EINVAL
    opts = G.gap_default_opts()
    J = (ctypes.c_double * 32)()
    assert lib.solve_with_adjoint(None, ctypes.byref(opts), P(8), None, J, None, None) == G.GAP_EINVAL
    assert lib.gap_tune_pcg(None, ctypes.byref(opts), P(8), 20, None, None, None) == G.GAP_EINVAL
    prm = G.gap_step_params()
    e = (ctypes.c_double * 4)()
    F = (ctypes.c_double * 4)()
    assert lib.general_iteration_step(None, ctypes.byref(opts), ctypes.byref(prm), None, P(8), e, e, F, None, None,
                                      None) == G.GAP_EINVAL
    assert "non-NULL" in G.gap_last_error() or "NULL" in G.gap_last_error()


def test_struct_layouts_match_the_header(tmp_path):
    """The binding's ctypes structs have the header's size and field offsets (a C program built
    with gcc against include/gapsolve.h prints them)."""
    import shutil
    import subprocess
    if shutil.which("gcc") is None:
        pytest.skip("no gcc")
    structs = [G.gap_geom, G.gap_dimples, G.gap_solver_opts, G.gap_solve_info, G.gap_pcg_config, G.gap_step_params]
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "gapsolve.h"', "int main(void) {"]
    for st in structs:
        lines.append(f'printf("{st.__name__} size %zu\\n", sizeof({st.__name__}));')
        for name, _ in st._fields_:
            lines.append(f'printf("{st.__name__} {name} %zu\\n", offsetof({st.__name__}, {name}));')
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = dict(line.rsplit(" ", 1) for line in subprocess.run([str(exe)], check=True, capture_output=True,
                                                                text=True).stdout.splitlines())
    for st in structs:
        assert int(got[f"{st.__name__} size"]) == ctypes.sizeof(st), st.__name__
        for name, _ in st._fields_:
            assert int(got[f"{st.__name__} {name}"]) == getattr(st, name).offset, (st.__name__, name)
