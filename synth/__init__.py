"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the benchmark.

This package builds atomic configurations (FCC copper-like lattices, vacancies, voids,
surfaces, thermal displacements, Maxwell velocities) and draws the random parameters
of the synthetic potentials.  It contains none of the method's arithmetic: no
neighbour search, no centro-symmetry, no switching function, no energies or forces.
Everything here is plain geometry and random-number draws from
``numpy.random.default_rng(seed)`` in a fixed draw order, so that the CPU oracle and
the HIP library receive bit-identical inputs.
"""

from .systems import (  # noqa: F401
    A_CU,
    MASS_CU,
    KB_EV,
    EV_PER_AMU_A2_PS2,
    System,
    fcc_positions,
    fcc111_positions,
    remove_random_sites,
    remove_sphere,
    gaussian_displace,
    maxwell_velocities,
    wrap_positions,
    thermal_sigma,
)
from .params import (  # noqa: F401
    EamParams,
    Eam2Params,
    AceParams,
    PrecisionParams,
    eam_cu_like,
    eam2_original,
    eam2_fit300k,
    eam_anchor,
    eam_label_anchor,
    ace_random,
    ace_label_model,
    precision_cfg0,
    precision_hyb1,
    precision_hyb2,
    precision_static,
)
from . import configs  # noqa: F401
