"""FP64 CPU oracle for the nodal finite-difference micromagnetic hot path.

TEST INFRASTRUCTURE, NOT PRODUCT CODE.  Only the test suite, the smoke check
and the CPU-baseline leg of the benchmark may import this package.  It shares
no code, tables or constants with the HIP library: every function here is a
plain numpy (float64) transcription of the paper's definitions, written for
readability, not speed.

Sections of the paper followed (Abert et al., "NeuralMag: an open-source nodal
finite-difference code for inverse micromagnetics"):
  * Sec. 2, Eq. (llg), Eq. (heff), Eq. (exchange_energy) -- the model;
  * Sec. 3.1, Eqs. (nodal_basis), (ms_discrete), (cell_basis),
    (weak_form_discrete), (weak_form_impl_f), (weak_form_impl),
    (mass_lumping) -- the nodal discretisation of the local terms;
  * Sec. 3.2 -- the demagnetisation field by FFT convolution of cuboid cells
    with nodal<->cell averaging;
  * Sec. 5.3 -- RK4 and Dormand-Prince time integration.

Array conventions (shared with the HIP library only by specification):
  nodal vector field   shape (3, N3+1, N2+1, N1+1)  [component, z, y, x]
  cell scalar field    shape (N3, N2, N1)
  cell vector field    shape (3, N3, N2, N1)
so that flattening in C order gives the structure-of-arrays, x-fastest layout.
"""
from .mesh import Mesh, Material, MU0
from .newell import newell_octant, newell_offset, dipole_tensor
from .field import (heff, gradient, energies, lumped_mass, cell_average,
                    demag_cell_field, demag_cell_field_direct, nodal_alpha,
                    external_cell_field)
from .llg import (llg_rhs, rk4_step, rk4_solve, DP45, dp45_attempt,
                  dp45_solve, dp45_replay, error_norm)

__all__ = [
    "Mesh", "Material", "MU0", "newell_octant", "newell_offset", "dipole_tensor",
    "heff", "gradient", "energies", "lumped_mass", "cell_average",
    "demag_cell_field", "demag_cell_field_direct", "nodal_alpha",
    "external_cell_field", "llg_rhs", "rk4_step", "rk4_solve", "DP45",
    "dp45_attempt", "dp45_solve", "dp45_replay", "error_norm",
]
