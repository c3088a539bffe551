"""Seeded synthetic inputs shared by the oracle and the GPU path.

This package holds no arithmetic of the assembly method itself: it only
produces the problem data the method is applied to (triangular meshes of
Omega plus the interaction layer, quadrature-rule tables, source and
volume-constraint data, and counter-based random numbers).
"""
from .mesh import Mesh, structured_mesh, splitmix64_uniform
from .rules import Rule, get_rule, RULE_NAMES
from .problems import (Problem, constant_kernel_c, fractional_kernel_c,
                       CONFIGS, make_config, manufactured, batch_instances, paper_workload)

__all__ = ["Mesh", "structured_mesh", "splitmix64_uniform", "Rule", "get_rule",
           "RULE_NAMES", "Problem", "constant_kernel_c", "fractional_kernel_c",
           "CONFIGS", "make_config", "manufactured", "batch_instances", "paper_workload"]
