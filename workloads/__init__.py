"""Seeded synthetic workloads for the made-to-measure (chi^2 M2M) step.

This package draws inputs only: initial particle models, realizations of the
target distribution functions, observation noise and the parameter sets of the
five benchmark workloads. It holds none of the arithmetic of the M2M step
itself (force-of-change, leapfrog push, observable deposit, chi^2, priors);
both the FP64 CPU oracle and the HIP library consume what it produces, and
neither of them is imported here.

Random numbers come from numpy's Philox counter-based generator, keyed by an
explicit integer seed, so every draw is reproducible on any host.
"""

from .dynamics import (  # noqa: F401
    Potential,
    HernquistTracer,
    PlummerTracer,
    EddingtonDF,
    hernquist_isotropic_df,
    sample_positions,
    sample_om_velocities,
    sample_gaussian_jeans_velocities,
    sample_hernquist_isotropic,
    sample_om_model,
    sample_plummer_jeans,
    hernquist_projected_mass,
)
from .configs import (  # noqa: F401
    WORKLOADS,
    Workload,
    workload,
    make_layout,
    make_params,
    make_potential,
    J_of,
    rng,
    with_alm,
    with_scf,
)
from .targets import (  # noqa: F401
    add_noise, density_length, fit_gauss_hermite_centres, floor_model_noise, make_targets)
