"""The allocation-free CG (nla_cg_noalloc) against nla_cg through the C ABI:
two calls in a row on different plans, the second with fewer free nodes than
the first, each bitwise equal to nla_cg's solution on the same plan (same
kernels and summation order; the shared scratch keeps the last call's
contents, which the next call must not read)."""
import sys

import numpy as np
import pytest
import torch

from gpu_util import gpu_assemble, host
from workloads import Problem, constant_kernel_c, make_config, structured_mesh

pytestmark = pytest.mark.gpu


def _plans():
    d = 0.1
    big = structured_mesh(d, d / 4, jitter=0.1, seed=41)
    pb = Problem(delta=d, kernel_c=constant_kernel_c(d), ball="retri", cap_edges=8)
    small, ps, _ = make_config("c1")
    return [(big, pb), (small, ps)]


def test_cg_noalloc_matches_cg_twice():
    sizes = []
    for mesh, prob in _plans():
        print("case noalloc CG K", mesh.n_triangles, flush=True)
        sys.stdout.flush()
        plan = gpu_assemble(mesh, prob)
        b = plan.load()
        u0, it0, rel0 = plan.cg(b, rtol=1e-12)
        u1, it1, rel1 = plan.cg(b, rtol=1e-12, noalloc=True)
        torch.cuda.synchronize()
        n = plan.info()["n_free"]
        sizes.append(n)
        print("n_free", n, "iterations", it0, it1, "relres", rel0, rel1, flush=True)
        assert it1 == it0 and rel1 == rel0
        assert np.array_equal(host(u1), host(u0))
        # a start vector other than zero takes the same path
        x0 = torch.full((n,), 0.5, dtype=torch.float64, device="cuda")
        v0, j0, _ = plan.cg(b, u0=x0, rtol=1e-10)
        v1, j1, _ = plan.cg(b, u0=x0, rtol=1e-10, noalloc=True)
        torch.cuda.synchronize()
        assert j0 == j1 and np.array_equal(host(v1), host(v0))
    assert sizes[1] < sizes[0]
