"""Helpers shared by the GPU parity tests: run the library and the oracle on
the same seeded inputs and compare them element by element."""
import numpy as np
import torch

import oracle
from paper_2005_10775_amd import Plan
from workloads import manufactured


def gpu_assemble(mesh, prob, man="quadratic", with_load=True):
    u, f = manufactured(man)
    plan = Plan(mesh, prob)
    if with_load:
        xq = plan.outer_points()
        fo = f(xq[..., 0], xq[..., 1]).contiguous()
        g = torch.tensor(u(mesh.xy[:, 0], mesh.xy[:, 1]), dtype=torch.float64, device="cuda")
        plan.assemble(fo, g)
    else:
        plan.assemble()
    torch.cuda.synchronize()
    return plan


def host(t):
    return t.detach().cpu().numpy()


def row_scaled_error(rowptr, val, ref_val):
    """max_ij |a_ij - r_ij| / max_j |r_ij| over every row."""
    J = len(rowptr) - 1
    rows = np.repeat(np.arange(J), np.diff(rowptr))
    nz = np.diff(rowptr) > 0
    scale = np.zeros(J)
    scale[nz] = np.maximum.reduceat(np.abs(ref_val), rowptr[:-1][nz])
    return float(np.max(np.abs(val - ref_val) / scale[rows])) if len(val) else 0.0


def oracle_full(mesh, prob, man="quadratic"):
    return oracle.solve_problem(mesh, prob, man)
