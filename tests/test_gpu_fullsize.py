"""Parity at the full sizes the benchmark times, in the launch configuration it
times (one plan, nla_assemble with f at the outer points and g at the nodes):

  * the headline workload (delta = 0.1, h = delta/8 jittered, K = 18,432,
    8-arc caps, 7 x 16 rules, FP64);
  * the fractional workload (delta = 0.05, h = delta/4, s = 0.4, FP32 with the
    vertex-sharing pairs in FP64);
  * the paper's finest grid (Sec. 8, h = 0.00625, K = 73,728, approxcaps, the
    switched outer rule, 124M pairs);
  * the learned-cap workload on the headline mesh (FP32, a seeded network: the
    path, not the training, is under test).

The headline and fractional workloads are also compared whole: one oracle
assembly of each (about 10 s on 16 host threads) against the GPU's pair list
and CSR pattern (bitwise) and every entry of D and b (FP64 1e-12, FP32 bar
row-scaled).  For the paper's finest grid and the learned workload the oracle
cannot assemble the matrix whole in seconds, so it builds sampled rows of D one at
a time (nodes in the interior, next to the boundary of Omega, at a corner and
in Omega_I): columns bitwise, values within the path's bar row-scaled (FP64
1e-12, FP32 and learned 1e-6); the pair lists of sampled outer elements
bitwise; the load vector b = G - D[free, Dirichlet] g at the sampled free
nodes."""
import sys

import numpy as np
import pytest
import torch

import oracle
import oracle.binding as ob
from gpu_util import gpu_assemble, host, row_scaled_error
from paper_2005_10775_amd import Mlp, Plan
from workloads import make_config, manufactured, paper_workload
from workloads.learned import mlp_init

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def _setup():
    oracle.build(force=False)
    assert torch.cuda.is_available()


def _sample_nodes(mesh, rng, n_free=8, n_dir=2):
    free = np.nonzero(mesh.node_free)[0]
    dirichlet = np.nonzero(mesh.node_free == 0)[0]
    xy = mesh.xy
    pick = set(rng.choice(free, n_free, replace=False).tolist())
    pick |= set(rng.choice(dirichlet, n_dir, replace=False).tolist())
    # the free node nearest to Omega's corner, one next to its lower boundary, one in the middle
    for target in ((0.0, 0.0), (0.5, 0.0), (0.5, 0.5)):
        d = np.hypot(xy[free, 0] - target[0], xy[free, 1] - target[1])
        pick.add(int(free[np.argmin(d)]))
    return sorted(pick)


def _check_full(mesh, prob, man, tol, seed, mlp=None, mlp_w=None, mlp_scale=1.0):
    u, f = manufactured(man)
    _say("full size: K", mesh.n_triangles, "J", mesh.n_vertices)
    if mlp is None:
        plan = gpu_assemble(mesh, prob, man)
    else:
        plan = Plan(mesh, prob, mlp=mlp)
        xq = plan.outer_points()
        plan.assemble(f(xq[..., 0], xq[..., 1]).contiguous(),
                      torch.tensor(u(mesh.xy[:, 0], mesh.xy[:, 1]), dtype=torch.float64, device="cuda"))
        torch.cuda.synchronize()
        _say("learned items", plan.info()["items"]["learned"])
        assert plan.info()["items"]["learned"] > 0
    rowptr, col, val = (host(t) for t in plan.csr(0))
    val = val.astype(np.float64)
    op = oracle.OracleProblem(mesh, prob, mlp_w=mlp_w, mlp_scale=mlp_scale)
    rng = np.random.default_rng(seed)
    worst = 0.0
    for j in _sample_nodes(mesh, rng):
        c_ref, v_ref = oracle.row(op, j)
        c, v = col[rowptr[j]:rowptr[j + 1]], val[rowptr[j]:rowptr[j + 1]]
        assert np.array_equal(c, c_ref), ("row pattern", j)
        err = float(np.max(np.abs(v - v_ref)) / np.max(np.abs(v_ref)))
        worst = max(worst, err)
        assert err < tol, ("row", j, err)
    _say("sampled rows: worst row-scaled error %.3e" % worst)
    # pair lists of sampled outer elements
    ptr, kp = (host(t) for t in plan.pairs())
    for k in rng.choice(mesh.n_triangles, 6, replace=False):
        assert np.array_equal(kp[ptr[k]:ptr[k + 1]], oracle.pairs_of(op, int(k))), ("pairs", k)
    # load vector at sampled free nodes: b_i = G_i - sum over Dirichlet j of D_ij g_j
    xq = oracle.outer_points(op)
    G = oracle.load_vector(op, f(xq[..., 0], xq[..., 1]))
    g = u(mesh.xy[:, 0], mesh.xy[:, 1])
    free_nodes = host(plan.free_nodes())
    b = host(plan.load())
    pos = {int(n): i for i, n in enumerate(free_nodes)}
    for j in _sample_nodes(mesh, rng, n_free=6, n_dir=0):
        c_ref, v_ref = oracle.row(op, j)
        dirichlet = mesh.node_free[c_ref] == 0
        b_ref = G[j] - np.sum(v_ref[dirichlet] * g[c_ref[dirichlet]])
        scale = max(abs(G[j]), float(np.sum(np.abs(v_ref[dirichlet] * g[c_ref[dirichlet]]))), 1e-300)
        assert abs(b[pos[j]] - b_ref) <= tol * scale, ("load", j, b[pos[j]], b_ref)
    return plan


def test_headline_fp64_full_size():
    mesh, prob, man = make_config("c2")
    _check_full(mesh, prob, man, 1e-12, seed=1)


def test_fractional_fp32_full_size():
    mesh, prob, man = make_config("c3")
    _check_full(mesh, prob, man, 1e-6, seed=2)


def test_paper_finest_grid_full_size():
    mesh, prob, man = paper_workload(0.00625, "approxcaps")
    _check_full(mesh, prob, man, 1e-12, seed=3)


def test_learned_full_size():
    mesh, prob, man = make_config("c5")
    scale = 1e-5
    w = mlp_init(12, bias_scale=0.3)
    m = Mlp()
    m.set_weights(w, scale)
    _check_full(mesh, prob, man, 1e-6, seed=4, mlp=m, mlp_w=ob.effective_weights(w), mlp_scale=scale)


def _check_whole(mesh, prob, man, tol):
    """Every pair, every pattern entry (bitwise), every entry of D and b
    (row-scaled within tol) against one oracle assembly of the whole mesh."""
    _say("whole: K", mesh.n_triangles, "oracle assembly")
    plan = gpu_assemble(mesh, prob, man)
    ref = oracle.solve_problem(mesh, prob, man, nthreads=0)
    rr = ref["res"]
    ptr, kp = (host(t) for t in plan.pairs())
    _say("pairs", len(kp), "oracle", len(rr["pair_kp"]))
    assert np.array_equal(ptr, rr["pair_ptr"]) and np.array_equal(kp, rr["pair_kp"])
    rowptr, col, val = (host(t) for t in plan.csr(0))
    assert np.array_equal(rowptr, rr["rowptr"]) and np.array_equal(col, rr["col"])
    err = row_scaled_error(rowptr, val.astype(np.float64), rr["val"])
    _say("every entry: row-scaled error %.3e (bar %.0e)" % (err, tol))
    assert err < tol
    # b_i = G_i - sum over Dirichlet j of D_ij g_j, on the scale of its terms
    u, _ = manufactured(man)
    free = mesh.node_free.astype(bool)
    fi, di = np.nonzero(free)[0], np.nonzero(~free)[0]
    g = np.abs(u(mesh.xy[:, 0], mesh.xy[:, 1]))
    scale = np.abs(ref["G"][fi]) + abs(rr["D"].tocsr()[fi][:, di]) @ g[di]
    b = host(plan.load())
    berr = float(np.max(np.abs(b - ref["b"]) / scale))
    _say("load vector: scaled error %.3e" % berr)
    assert berr < tol
    return plan, ref


def test_headline_fp64_whole_matrix():
    mesh, prob, man = make_config("c2")
    _check_whole(mesh, prob, man, 1e-12)


def test_fractional_fp32_whole_matrix():
    mesh, prob, man = make_config("c3")
    plan, ref = _check_whole(mesh, prob, man, 1e-6)
    # the vertex-sharing pairs' blocks (FP64 rule, stored in FP32), sampled
    near_p, blocks = (host(t) for t in plan.near())
    rr = ref["res"]
    ks = np.repeat(np.arange(mesh.n_triangles), np.diff(rr["pair_ptr"]))
    iu = np.triu_indices(6)
    rng = np.random.default_rng(7)
    worst = 0.0
    for i in rng.choice(len(near_p), 60, replace=False):
        p = near_p[i]
        blk = oracle.pair_block(ref["op"], ks[p], rr["pair_kp"][p])["blk"]
        e = np.max(np.abs(blocks[i].astype(np.float64) - blk[iu])) / np.max(np.abs(blk))
        worst = max(worst, e)
    _say("near blocks: worst relative error %.3e" % worst)
    assert worst <= 2e-7
