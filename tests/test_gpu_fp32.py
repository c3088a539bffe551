"""GPU parity of the FP32 path (compensated sums, FP64 geometry) and of the
singular-kernel near-diagonal blocks, against the FP64 oracle.

Bars: pair list and pattern bitwise; near-diagonal blocks (computed in FP64,
stored in FP32) within 2e-7 of the oracle's, relative to the block (storage
rounding alone is up to 2^-24 ~ 6e-8); matrix entries row-scaled within
1e-6.  Every sum longer than one item's dozen subtriangle terms is
compensated, so an entry carries the rounding of its stored FP32 value
(2^-24) plus the FP32 errors of the individual terms: the kernel evaluation
2^(e log2 r^2) with the hardware log2/exp2 (about |e log2 r^2| * 2^-24
relative per point, averaging out over the points of a term) and the plain
FP32 sums of one item (a few 2^-24).  Measured: at most 1.5e-7 over every
FP32 case of the suite (constant and fractional kernels, delta/h = 2..8, the
whole c3 matrix 1.1e-7); the bar leaves a factor of about 7.
"""
import sys

import numpy as np
import pytest
import torch

import oracle
from gpu_util import gpu_assemble, host, row_scaled_error
from workloads import Problem, constant_kernel_c, fractional_kernel_c, structured_mesh

pytestmark = pytest.mark.gpu
TOL32 = 1e-6


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def _setup():
    oracle.build(force=False)
    assert torch.cuda.is_available()


def _check(mesh, prob, name):
    _say("case", name, "K", mesh.n_triangles, prob)
    plan = gpu_assemble(mesh, prob)
    ref = oracle.solve_problem(mesh, prob, "quadratic", nthreads=0)
    rr = ref["res"]
    ptr, kp = (host(t) for t in plan.pairs())
    assert np.array_equal(ptr, rr["pair_ptr"]) and np.array_equal(kp, rr["pair_kp"])
    rowptr, col, val = (host(t) for t in plan.csr(0))
    assert val.dtype == np.float32
    assert np.array_equal(rowptr, rr["rowptr"]) and np.array_equal(col, rr["col"])
    err = row_scaled_error(rowptr, val.astype(np.float64), rr["val"])
    D = rr["D"].copy()
    D.data = val.astype(np.float64)
    assert (D != D.T).nnz == 0
    _say("row-scaled entry error %.3e" % err)
    assert err < TOL32
    return plan, ref, err


def test_fp32_constant_kernel_retri():
    d = 0.1
    mesh = structured_mesh(d, 0.025, jitter=0.1, seed=12)
    prob = Problem(delta=d, kernel_c=constant_kernel_c(d), ball="retri", cap_edges=8, precision="fp32")
    _check(mesh, prob, "fp32 const retri")


@pytest.mark.parametrize("ball,seed", [("retri", 21), ("barycenter", 22)])
def test_fp32_constant_kernel_deep_pairs_jittered(ball, seed):
    """FP32 constant kernel on a strongly jittered mesh at h = delta/6, where
    most pairs are deep (blocks summed from element areas, their Myy per
    element)."""
    d = 0.1
    mesh = structured_mesh(d, d / 6, jitter=0.25, seed=seed)
    prob = Problem(delta=d, kernel_c=constant_kernel_c(d), ball=ball, cap_edges=8 if ball == "retri" else 0,
                   precision="fp32")
    _check(mesh, prob, "fp32 const %s h=delta/6" % ball)


def test_fp32_constant_kernel_many_deep_pairs():
    """FP32 constant kernel at delta/h = 10: 320 to about 500 deep pairs per
    interior element, so that the FP32 deep row-block walk takes both its
    paths, the areas kept in LDS (up to 320) and read from memory beyond."""
    h = 1.0 / 30
    d = 10 * h
    mesh = structured_mesh(d, h, jitter=0.1, seed=32)
    prob = Problem(delta=d, kernel_c=constant_kernel_c(d), ball="retri", cap_edges=8, precision="fp32")
    _check(mesh, prob, "fp32 const retri delta/h=10")


@pytest.mark.parametrize("h", [0.05, 0.1])
def test_fp32_fractional_retri_with_near_pairs(h):
    """delta/h = 4, and delta/h = 2, where the ball cuts vertex-sharing pairs
    and the singular rule stops its radial integrals at delta."""
    d, s = 0.2, 0.4
    mesh = structured_mesh(d, h, jitter=0.1, seed=13)
    prob = Problem(delta=d, kernel="fractional", kernel_c=fractional_kernel_c(d, s), kernel_s=s, ball="retri",
                   cap_edges=8, precision="fp32", duffy_order=12)
    plan, ref, err = _check(mesh, prob, "fp32 fractional retri delta/h=%g" % (d / h))
    near_p, blocks = (host(t) for t in plan.near())
    ptr = ref["res"]["pair_ptr"]
    kp = ref["res"]["pair_kp"]
    ks = np.repeat(np.arange(mesh.n_triangles), np.diff(ptr))
    shares = np.array([len(set(mesh.tri[a]) & set(mesh.tri[b])) > 0 for a, b in zip(ks, kp)])
    assert np.array_equal(near_p, np.nonzero(shares)[0])
    op = ref["op"]
    iu = np.triu_indices(6)
    rng = np.random.default_rng(0)
    worst = 0.0
    for i in rng.choice(len(near_p), min(40, len(near_p)), replace=False):
        p = near_p[i]
        blk = oracle.pair_block(op, ks[p], kp[p])["blk"]
        got = blocks[i].astype(np.float64)
        e = np.max(np.abs(got - blk[iu])) / np.max(np.abs(blk))
        worst = max(worst, e)
        assert e <= 2e-7
    _say("near blocks: worst relative error %.3e" % worst)


def test_fp32_barycenter_fractional():
    d, s = 0.2, 0.4
    mesh = structured_mesh(d, 0.05)
    prob = Problem(delta=d, kernel="fractional", kernel_c=fractional_kernel_c(d, s), kernel_s=s, ball="barycenter",
                   outer="dunavant7", inner="dunavant7", precision="fp32", duffy_order=12)
    _check(mesh, prob, "fp32 fractional barycenter")


def test_fp32_deterministic():
    d, s = 0.2, 0.4
    mesh = structured_mesh(d, 0.05, jitter=0.1, seed=14)
    prob = Problem(delta=d, kernel="fractional", kernel_c=fractional_kernel_c(d, s), kernel_s=s, ball="retri",
                   cap_edges=8, precision="fp32", duffy_order=8)
    plan = gpu_assemble(mesh, prob)
    v1 = host(plan.csr(0)[2]).copy()
    plan.assemble()
    torch.cuda.synchronize()
    assert np.array_equal(v1.view(np.uint32), host(plan.csr(0)[2]).view(np.uint32))
