"""Pins of the oracle's rule for vertex-sharing pairs under the singular
kernel (oracle/nlo_duffy.c), against facts that do not come from it:

* psi constant (s = -1) with a horizon covering both elements: the integrand
  (phi(x) - phi(y)) (phi'(x) - phi'(y)) is a polynomial of degree 2 in (x, y),
  so the joint integral is given exactly by a tensor of two degree-8 triangle
  rules; the node-level matrix of the merged block must match it;
* the merged differences of all distinct nodes sum to zero pointwise, so each
  row of the block sums to zero to rounding (a dropped or wrong-signed term
  breaks it), and the block is symmetric;
* for s = 0.4 the blocks converge as the rule order grows.
"""
import numpy as np
import pytest

import oracle
import oracle.binding as ob
from workloads import Problem, get_rule, structured_mesh


@pytest.fixture(scope="module", autouse=True)
def _built():
    oracle.build(force=False)


def _mesh():
    return structured_mesh(0.5, 0.25, jitter=0.1, seed=4)


def _pairs_sharing(mesh, k):
    tri = mesh.tri
    out = []
    for kp in range(mesh.n_triangles):
        n = len(set(tri[k]) & set(tri[kp]))
        if n:
            out.append((kp, n))
    return out


def _node_matrix(mesh, k, kp, blk):
    nodes = list(mesh.tri[k]) + list(mesh.tri[kp])
    ids = sorted(set(nodes))
    M = np.zeros((len(ids), len(ids)))
    for i in range(6):
        for j in range(6):
            M[ids.index(nodes[i]), ids.index(nodes[j])] += blk[i, j]
    return ids, M


def _exact_joint(mesh, k, kp, kc):
    """int_Ek int_Ek' (phi_j(x) - phi_j(y)) (phi_j'(x) - phi_j'(y)) kc, by a tensor of
    degree-8 rules (exact: the integrand is quadratic in (x, y))."""
    r = get_rule("dunavant16")
    V = mesh.xy[mesh.tri[k]]
    W = mesh.xy[mesh.tri[kp]]
    ids = sorted(set(mesh.tri[k]) | set(mesh.tri[kp]))
    ak = abs((V[1, 0] - V[0, 0]) * (V[2, 1] - V[0, 1]) - (V[1, 1] - V[0, 1]) * (V[2, 0] - V[0, 0]))
    aw = abs((W[1, 0] - W[0, 0]) * (W[2, 1] - W[0, 1]) - (W[1, 1] - W[0, 1]) * (W[2, 0] - W[0, 0]))

    def phi(node, tri, lam):
        t = list(mesh.tri[tri])
        return lam[t.index(node)] if node in t else 0.0
    M = np.zeros((len(ids), len(ids)))
    for qx in range(r.n):
        for qy in range(r.n):
            w = r.w[qx] * ak * r.w[qy] * aw * kc
            d = np.array([phi(j, k, r.lam[qx]) - phi(j, kp, r.lam[qy]) for j in ids])
            M += w * np.outer(d, d)
    return ids, M


def _problem(s, n, delta):
    return Problem(delta=delta, kernel="fractional", kernel_c=1.0, kernel_s=s, ball="retri", cap_edges=8,
                   outer="dunavant7", inner="dunavant16", precision="fp32", duffy_order=n)


def test_duffy_nonsingular_limit_is_exact():
    """The merged block converges to the exact joint integral (measured: 3.5e-4,
    4.9e-6, 8.0e-7, 1.3e-7 at orders 8, 16, 24, 32: algebraic, the angular
    integrand has kinks at the vertex directions); a wrong term would stall."""
    mesh = _mesh()
    k = 37
    errs = []
    for n_order in (8, 16, 32):
        op = ob.OracleProblem(mesh, _problem(-1.0, n_order, 3.0))
        worst = 0.0
        for kp, ns in _pairs_sharing(mesh, k):
            blk = ob.pair_block(op, k, kp)["blk"]
            ids, M = _node_matrix(mesh, k, kp, blk)
            ids2, E = _exact_joint(mesh, k, kp, 1.0)
            assert ids == ids2
            worst = max(worst, np.abs(M - E).max() / np.abs(E).max())
        errs.append(worst)
    assert errs[0] > 20 * errs[1] > 20 * 20 * errs[2] and errs[2] < 3e-7, errs


def test_duffy_rows_sum_to_zero_and_symmetric():
    mesh = _mesh()
    op = ob.OracleProblem(mesh, _problem(0.4, 8, 0.5))
    for k in (5, 37, 60):
        for kp, ns in _pairs_sharing(mesh, k):
            blk = ob.pair_block(op, k, kp)["blk"]
            scale = np.abs(blk).max()
            assert scale > 0
            assert np.abs(blk - blk.T).max() <= 1e-13 * scale
            assert np.abs(blk.sum(1)).max() <= 1e-12 * scale
            # positive semidefinite (a sum of rank-one terms with positive weights)
            assert np.linalg.eigvalsh(0.5 * (blk + blk.T)).min() >= -1e-12 * scale


def test_duffy_singular_converges_with_order():
    mesh = _mesh()
    k = 37
    ref = {}
    op = ob.OracleProblem(mesh, _problem(0.4, 32, 0.5))
    for kp, ns in _pairs_sharing(mesh, k):
        ref[kp] = ob.pair_block(op, k, kp)["blk"]
    errs = []
    for n in (6, 10, 16):
        op = ob.OracleProblem(mesh, _problem(0.4, n, 0.5))
        e = max(np.abs(ob.pair_block(op, k, kp)["blk"] - ref[kp]).max() / np.abs(ref[kp]).max() for kp in ref)
        errs.append(e)
    # measured 4.1e-3, 5.2e-4, 7.0e-5 against order 32
    assert errs[0] > 4 * errs[1] > 16 * errs[2] and errs[2] < 1.5e-4, errs
