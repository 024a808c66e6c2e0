"""Seeded synthetic workloads for the one-site TDVP sweep of a tree tensor network.

This package only *describes* problems: tree shape, requested bond dimensions,
sum-of-product (SOP) operator terms and the initial product state.  It holds
none of the propagation arithmetic, so the CPU oracle and the HIP library can
both consume the very same inputs without sharing any of the method's code.
"""
from .problem import Problem, TreeBuilder
from .models import (sbm_problem, vibronic_problem, exciton_problem,
                     heom_sbm_problem, pseudomode_sbm_problem, batch_sbm_problems, random_isometric_state,
                     chain_transform, ipchain_sbm_problem, ipchain_coefficients, multiset_vibronic_problem,
                     CONFIGS, config_problem)

__all__ = ["Problem", "TreeBuilder", "sbm_problem", "vibronic_problem",
           "exciton_problem", "heom_sbm_problem", "pseudomode_sbm_problem", "batch_sbm_problems",
           "random_isometric_state", "chain_transform", "ipchain_sbm_problem", "ipchain_coefficients",
           "multiset_vibronic_problem", "CONFIGS", "config_problem"]
