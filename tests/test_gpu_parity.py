"""GPU parity: libnlasm (through its C ABI) against the FP64 oracle.

Bar: pair list and CSR pattern bitwise; FP64 entries within 1e-12 of the
oracle, row-scaled (|a_ij - r_ij| <= 1e-12 max_j |r_ij|); D bitwise symmetric;
repeated assemblies bitwise identical.
"""
import sys

import numpy as np
import pytest
import torch

import oracle
from gpu_util import gpu_assemble, host, row_scaled_error
from workloads import Problem, constant_kernel_c, make_config, structured_mesh, manufactured

pytestmark = pytest.mark.gpu

TOL = 1e-12


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def _setup():
    oracle.build(force=False)
    assert torch.cuda.is_available()


def _problem(d, ball, caps=0, outer="dunavant7", inner="dunavant16", **kw):
    return Problem(delta=d, kernel_c=constant_kernel_c(d), ball=ball, cap_edges=caps, outer=outer, inner=inner, **kw)


def _full_parity(mesh, prob, man="quadratic", name=""):
    _say("case", name, "K", mesh.n_triangles, prob)
    plan = gpu_assemble(mesh, prob, man)
    ref = oracle.solve_problem(mesh, prob, man)
    rr = ref["res"]
    ptr, kp = (host(t) for t in plan.pairs())
    assert np.array_equal(ptr, rr["pair_ptr"]), "pair counts differ"
    assert np.array_equal(kp, rr["pair_kp"]), "pair list differs"
    rowptr, col, val = (host(t) for t in plan.csr(0))
    assert np.array_equal(rowptr, rr["rowptr"]) and np.array_equal(col, rr["col"]), "pattern differs"
    err = row_scaled_error(rowptr, val, rr["val"])
    assert err < TOL, "row-scaled entry error %g" % err
    # bitwise symmetry
    D = ref["res"]["D"].copy()
    D.data = val.copy()
    assert (D != D.T).nnz == 0
    # A and b
    arp, acol, aval = (host(t) for t in plan.csr(1))
    A = ref["A"]
    assert np.array_equal(arp, A.indptr) and np.array_equal(acol, A.indices)
    assert np.max(np.abs(aval - A.data)) <= TOL * np.max(np.abs(A.data))
    b = host(plan.load())
    assert np.max(np.abs(b - ref["b"])) <= 1e-11 * np.max(np.abs(ref["b"]))
    info = plan.info()
    assert info["n_pairs"] == len(rr["pair_kp"])
    return plan, ref, err


def test_c1_barycenter():
    """The small barycenter workload: delta=0.1, h=0.05, 7x7 points."""
    mesh, prob, man = make_config("c1")
    plan, ref, err = _full_parity(mesh, prob, man, "c1")
    # CG solution against the oracle's dense solve
    u, f = manufactured(man)
    U, its, rel = plan.cg(plan.load(), rtol=1e-13)
    fn = host(plan.free_nodes())
    Uo = ref["U"][fn]
    assert np.max(np.abs(host(U) - Uo)) < 1e-9 * np.max(np.abs(Uo))
    _say("c1 ok: err %.2e, cg %d its, relres %.1e" % (err, its, rel))


def test_many_deep_pairs_per_element():
    """delta/h = 13: up to about 900 deep pairs per outer element, so that the
    pair kernel's deep row-block walk takes both its paths, the deep pairs'
    areas kept in LDS (up to 768 of them) and read from memory beyond that."""
    h = 1.0 / 25
    d = 13 * h
    mesh = structured_mesh(d, h, jitter=0.1, seed=31)
    _full_parity(mesh, _problem(d, "retri", caps=8), name="retri-8 delta/h=13")


@pytest.mark.parametrize("caps", [0, 2, 8, 64])
def test_retri_small(caps):
    """Retriangulated ball, jittered mesh, every cap count (0 = inscribed polygon)."""
    mesh = structured_mesh(0.1, 0.05, jitter=0.1, seed=20050)
    _full_parity(mesh, _problem(0.1, "retri", caps), name="retri h=0.05 caps=%d" % caps)


def test_retri_several_tiles():
    """h = delta/4 with 8-arc caps: several wavefront chunks per element, ragged tails."""
    mesh = structured_mesh(0.1, 0.025, jitter=0.1, seed=11)
    _full_parity(mesh, _problem(0.1, "retri", 8), name="retri h=0.025")


@pytest.mark.parametrize("ball,seed", [("retri", 3), ("retri", 4), ("overlap", 5), ("barycenter", 6)])
def test_deep_band_split_jittered(ball, seed):
    """Strongly jittered meshes (jitter 0.25) at h = delta/4: the plan's split
    of each element's pairs into band and deep ones (every item whole; their
    blocks summed from element areas) must give the oracle's matrix, whatever
    the element shapes."""
    mesh = structured_mesh(0.1, 0.025, jitter=0.25, seed=seed)
    caps = 8 if ball == "retri" else 0
    _full_parity(mesh, _problem(0.1, ball, caps), name="%s jitter 0.25 seed %d" % (ball, seed))


def test_deep_pairs_dominant():
    """h = delta/6: most pairs are deep, so most of the row block comes from the
    deep-pair sums and the element blocks from the per-element deep factor."""
    mesh = structured_mesh(0.1, 0.1 / 6, jitter=0.1, seed=12)
    _full_parity(mesh, _problem(0.1, "retri", 8), name="retri h=delta/6")


def test_lattice_ties_barycenter_vertex_rule():
    """Outer points on vertices and mid-sides of an unjittered lattice hit
    |x - b_k'| = delta exactly; the pair list must still be bitwise equal."""
    mesh = structured_mesh(0.1, 0.025)
    _full_parity(mesh, _problem(0.1, "barycenter", outer="vertex7", inner="gauss3"), name="ties")


def test_tiny_meshes():
    """Degenerate small cases: a 4x4-cell mesh with delta = h, both balls."""
    mesh = structured_mesh(0.5, 0.5)
    _full_parity(mesh, _problem(0.5, "barycenter", inner="dunavant7"), name="tiny bary")
    mesh = structured_mesh(0.25, 0.125, jitter=0.1, seed=3)
    _full_parity(mesh, _problem(0.25, "retri", 8), name="tiny retri")


def test_determinism_and_symmetry():
    """Two assemblies of the same plan are bitwise identical; D == D^T bitwise."""
    mesh = structured_mesh(0.1, 0.025, jitter=0.1, seed=5)
    prob = _problem(0.1, "retri", 8)
    plan = gpu_assemble(mesh, prob)
    v1 = host(plan.csr(0)[2]).copy()
    plan.assemble()
    torch.cuda.synchronize()
    v2 = host(plan.csr(0)[2])
    assert np.array_equal(v1.view(np.uint64), v2.view(np.uint64))
    plan2 = gpu_assemble(mesh, prob)
    v3 = host(plan2.csr(0)[2])
    assert np.array_equal(v1.view(np.uint64), v3.view(np.uint64))


def test_skip_ixi_keeps_system():
    """Dropping Omega_I x Omega_I pairs changes neither A nor b."""
    mesh = structured_mesh(0.1, 0.05, jitter=0.1, seed=8)
    p0 = _problem(0.1, "retri", 8)
    p1 = _problem(0.1, "retri", 8, skip_ixi=True)
    a = gpu_assemble(mesh, p0)
    b = gpu_assemble(mesh, p1)
    assert b.info()["n_pairs"] < a.info()["n_pairs"]
    A0, A1 = host(a.csr(1)[2]), host(b.csr(1)[2])
    assert np.max(np.abs(A0 - A1)) <= 1e-13 * np.max(np.abs(A0))
    assert np.max(np.abs(host(a.load()) - host(b.load()))) <= 1e-12 * np.max(np.abs(host(a.load())))
