"""Seeded synthetic inputs for two-site DMRG problems.

This package defines *problems*, not the method that solves them: lattices and
their couplings, matrix product operators (MPOs) built as finite-state machines,
bond-dimension sector models taken from the block-size model of the paper's
complexity table (Table 2, b_l = floor((m/q) r^l)), and seeded random block
values.  It holds none of the method's arithmetic (no contraction, eigensolver,
SVD or environment update), so both the CPU oracle and the GPU path can take
their inputs from here without sharing any code of the method itself.

Every random value is a pure function of (seed, tag, block key): the order in
which a consumer enumerates blocks never changes what it receives.
"""

from .lattice import chain_bonds, cylinder_j1_bonds, cylinder_j2_bonds, merge_bonds
from .mpo import (MPO, SPIN_PHYS, HUB_PHYS, heisenberg_mpo, hubbard_mpo,
                  synthetic_heisenberg_bond, synthetic_hubbard_bond, heisenberg_j2_derivative)
from .sectors import spin_bond_leg, electron_bond_leg, mps_bond_legs
from .blocks import gaussian_block, env_block, BondSpec, c2_bond, c3_batch, c4_bond

__all__ = [
    "chain_bonds", "cylinder_j1_bonds", "cylinder_j2_bonds", "merge_bonds",
    "MPO", "SPIN_PHYS", "HUB_PHYS", "heisenberg_mpo", "hubbard_mpo",
    "synthetic_heisenberg_bond", "synthetic_hubbard_bond", "heisenberg_j2_derivative",
    "spin_bond_leg", "electron_bond_leg", "mps_bond_legs",
    "gaussian_block", "env_block", "BondSpec", "c2_bond", "c3_batch", "c4_bond",
]
