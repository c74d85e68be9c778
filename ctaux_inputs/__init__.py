"""Seeded synthetic inputs for the CT-AUX submatrix-update path.

This package builds the *inputs* of a CT-AUX run: bare Green's function
tables G0(tau) on a uniform imaginary-time grid, cluster geometries and the
site-pair -> table map, and the model parameters of the workloads used by the
tests and the benchmark.  It holds none of the Monte Carlo method's arithmetic
(no N matrix, no determinant ratio, no update); both the CPU oracle and the
GPU path consume what it produces.

Convention (the bare propagator enters the determinant representation of the
paper, Sec. II A, Eq. (Nmatrix)): tables hold the "plus" propagator
G0_xy(tau) = <T c_x(tau) c_y^dagger(0)>_0 for 0 < tau < beta, sampled at
tau_m = m * beta / (n_tau - 1); entry 0 holds the tau -> 0+ limit and the last
entry the tau -> beta- limit.
"""

from .g0 import (  # noqa: F401
    tau_grid,
    fermi_weight,
    semicircle_g0,
    finite_system_g0,
    Cluster,
    make_cluster,
    dca_cluster_g0,
    cluster_density,
    solve_mu_for_density,
)
from .workloads import (  # noqa: F401
    Workload,
    anderson_semicircle,
    hubbard_atom,
    hubbard_dimer,
    hubbard_plaquette,
    anderson_bath,
    dca_square,
    dca_cubic,
    batched_mix,
    named_workload,
)
