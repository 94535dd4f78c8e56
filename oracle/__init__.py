"""Plain FP64 CPU oracle for the piston-gap joint Reynolds solve.

TEST INFRASTRUCTURE ONLY.  This package is the slow, obviously-correct
reference that the GPU path is checked against.  Only ``tests/``,
``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py`` may
import, call or link anything in it; the product library under
``paper_2511_06824_amd/`` never does, and the two share no code.

What it computes (paper: arXiv 2511.06824):

* ``film``      film thickness h(e) of Eq 2.3 (stable algebraic form), its time
                derivative through the eccentricity rates, spherical-cap dimples.
* ``fvm``       the 5-point finite-volume system A p = S of Eq 2.1/2.4 with
                Dirichlet ends and a periodic circumferential axis (Sec 2.1),
                the 9 working conditions of Eq 2.17-2.19 and the block-diagonal
                joint system of Eq 3.7.
* ``direct``    the exact discrete solution by banded Cholesky elimination,
                a dense solve for tiny grids and an SOR/Gauss-Seidel iteration
                (plain C) as an independent check.
* ``pcg``       the adjusted PCG of Table 1 with the Jacobi (Eq 2.8), ASSOR I
                (Eq 3.2) and ASSOR II (Eq 3.3-3.6) preconditioners, on one system
                or on the joint system with the synchronized test of Eq 3.9.
* ``forces``    pressure + viscous-shear force and moment integrals (Sec 2.4-III).
* ``jacobian``  forward differences of Eq 2.13-2.14, central differences, and
                an exact complex-step derivative.
* ``dynamics``  one general-iteration step of the equilibrium F_E + F_I + F_O = 0
                (Eq 2.10, 2.12; the conventional scheme of Eq 2.20-2.22).

The paper does not state the Reynolds equation, the shear formula, the force
definitions or a cavitation rule; the readings taken here are listed in each
module's docstring.  Every function is pinned by a ``-m "not gpu"`` test
against a closed form, an invariant, a brute-force solve or a textbook limit.
"""

from .film import Gap, cell_centers, film, film_naive, film_rate, dimple_texture, no_texture
from .fvm import face_conductances, source, cell_values, stencil_matrix, assemble, conditions, assemble_joint
from .direct import solve_band, band_factor, band_solve, solve_dense, sor_solve
from .pcg import pcg, pcg_blocks, jacobi_precond, assor1_precond, assor2_precond, assor2_explicit
from .forces import (effective_pressure, force_moment, forces_for_condition, force_moment_split,
                     forces_split_for_condition, rebuild_field)
from .jacobian import (solve_condition, condition_forces, jacobian_fd, jacobian_central,
                       jacobian_complex_step)
from . import dynamics

__all__ = [
    "Gap", "cell_centers", "film", "film_naive", "film_rate", "dimple_texture", "no_texture",
    "face_conductances", "source", "cell_values", "stencil_matrix", "assemble", "conditions", "assemble_joint",
    "solve_band", "band_factor", "band_solve", "solve_dense", "sor_solve",
    "pcg", "pcg_blocks", "jacobi_precond", "assor1_precond", "assor2_precond", "assor2_explicit",
    "effective_pressure", "force_moment", "forces_for_condition", "force_moment_split",
    "forces_split_for_condition", "rebuild_field",
    "solve_condition", "condition_forces", "jacobian_fd", "jacobian_central",
    "jacobian_complex_step", "dynamics",
]
