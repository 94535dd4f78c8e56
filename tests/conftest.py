import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: CPU test that takes more than a few seconds")


def gap_of(case, **over):
    """oracle.Gap from a synth.GapCase (field-by-field, optional overrides)."""
    import oracle
    d = dict(R=case.R, c=case.c, L=case.L, mu=case.mu, U=case.U, V=case.V, p_in=case.p_in,
             p_out=case.p_out, n_theta=case.n_theta, n_axial=case.n_axial)
    d.update(over)
    return oracle.Gap(**d)


def texture_of(case):
    import oracle
    if case.n_dimples == 0:
        return oracle.no_texture
    return oracle.dimple_texture(case.R, case.dimple_theta, case.dimple_z, case.dimple_radius,
                                 case.dimple_depth)
