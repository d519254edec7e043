"""FP64 CPU oracle of the fine-box lattice-Boltzmann step (test infrastructure).

Only the tests, the smoke check and the benchmark's CPU-baseline leg may
import this package.  It shares no code with the GPU library: its C source
(``lb_oracle.c``) is compiled with gcc by :func:`build` and bound here with
ctypes.
"""
from .oracle import (OracleBox, build, threads, lattice, mrt_basis, equilibrium, collide,  # noqa: F401
                     chain_md, chain_md_noise, collide_noise, philox, unit_uniform, BGK, MRT, BC_AFFINE, BC_SAMPLED, OK, ERR_ARG, ERR_FENE,
                     ERR_BEAD_OUT, ERR_UNSTABLE, ERR_STATE)
