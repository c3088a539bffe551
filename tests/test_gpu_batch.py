"""Batched assembly: one persistent launch over uneven instances, captured in
a hipGraph, gives bitwise the values of assembling each instance alone; so
does every (chunk, grid) the autotuner may pick, and so does the graph of
every instance's own launches (chunk 0).  Every instance of the test batch,
and the fractional delta/h = 2 instances of the 64-instance workload (where
the ball cuts vertex-sharing pairs, so the singular rule truncates its radial
integrals at delta), is compared with the FP64 oracle: pair list and pattern
bitwise, entries within the FP32 bar (row-scaled)."""
import sys

import numpy as np
import pytest
import torch

import oracle
from gpu_util import host, row_scaled_error
from paper_2005_10775_amd import Batch, Plan
from workloads import (Problem, batch_instances, constant_kernel_c, fractional_kernel_c, manufactured,
                       structured_mesh)

TOL32 = 1e-6     # the FP32 path's bar (tests/test_gpu_fp32.py)

pytestmark = pytest.mark.gpu


def _instances():
    out = []
    specs = [(0.2, 4, "constant", "barycenter"), (0.15, 3, "fractional", "barycenter"),
             (0.1, 2, "constant", "retri"), (0.2, 5, "fractional", "retri"), (0.25, 2, "constant", "retri"),
             (0.125, 4, "fractional", "retri"), (0.2, 2, "fractional", "retri")]
    for d, k, kern, ball in specs:
        h = d / k
        mesh = structured_mesh(d, h, jitter=0.1 if ball == "retri" else 0.0, seed=k)
        kw = dict(kernel="constant", kernel_c=constant_kernel_c(d)) if kern == "constant" else \
            dict(kernel="fractional", kernel_c=fractional_kernel_c(d, 0.4), kernel_s=0.4, duffy_order=6)
        bw = dict(ball="barycenter", outer="dunavant7", inner="dunavant7") if ball == "barycenter" else \
            dict(ball="retri", cap_edges=8, outer="dunavant7", inner="dunavant16")
        out.append((mesh, Problem(delta=d, precision="fp32", **kw, **bw)))
    return out


def _inputs(b):
    u, f = manufactured("quadratic")
    fs, gs = [], []
    for (mesh, prob), plan in zip(b.instances, b.plans):
        xq = plan.outer_points()
        fs.append(f(xq[..., 0], xq[..., 1]).contiguous())
        gs.append(torch.tensor(u(mesh.xy[:, 0], mesh.xy[:, 1]), dtype=torch.float64, device="cuda"))
    return fs, gs


def _values(b):
    return [(host(p.csr(0)[2]).copy(), host(p.load()).copy()) for p in b.plans]


def test_batch_bitwise_equals_sequential(tmp_path):
    print("batch of", len(_instances()), flush=True)
    b = Batch(_instances())
    fs, gs = _inputs(b)
    b.assemble(mode=0, f_outer=fs, g_node=gs)
    torch.cuda.synchronize()
    seq = _values(b)
    for rep in range(3):       # several graph replays, eager work in between
        b.assemble(mode=1, f_outer=fs, g_node=gs)
        torch.cuda.synchronize()
        bat = _values(b)
        for (v0, b0), (v1, b1) in zip(seq, bat):
            assert np.array_equal(v0.view(np.uint32), v1.view(np.uint32))
            assert np.array_equal(b0, b1)
        _ = torch.ones(10, device="cuda").sum().item()
    info = b.autotune(str(tmp_path / "tune.txt"))
    assert info["chunk"] in (0, 1, 2, 4, 8) and info["grid"] > 0
    b.assemble(mode=1, f_outer=fs, g_node=gs)
    torch.cuda.synchronize()
    for (v0, _), (v1, _) in zip(seq, _values(b)):
        assert np.array_equal(v0.view(np.uint32), v1.view(np.uint32))
    # a single plan of the same instance gives the same bits as well
    mesh, prob = b.instances[3]
    p = Plan(mesh, prob)
    p.assemble(fs[3], gs[3])
    torch.cuda.synchronize()
    assert np.array_equal(host(p.csr(0)[2]).view(np.uint32), seq[3][0].view(np.uint32))


def test_batch_graph_of_instance_launches(tmp_path):
    """chunk 0 (forced through the autotuner's cache file): the graph of each
    instance's own launches, replayed several times with eager work between
    the replays, gives the sequential values bitwise."""
    b = Batch(_instances())
    fs, gs = _inputs(b)
    b.assemble(mode=0, f_outer=fs, g_node=gs)
    torch.cuda.synchronize()
    seq = _values(b)
    i = b.info()
    cu = torch.cuda.get_device_properties(0).multi_processor_count
    key = "n%d_pairs%d_K%d_near%d_cu%d" % (i["n"], i["total_pairs"], i["total_elements"], i["total_near"], cu)
    path = tmp_path / "tune.txt"
    path.write_text("%s 0 1\n" % key)
    assert b.autotune(str(path))["chunk"] == 0
    for rep in range(3):
        b.assemble(mode=1, f_outer=fs, g_node=gs)
        torch.cuda.synchronize()
        for (v0, b0), (v1, b1) in zip(seq, _values(b)):
            assert np.array_equal(v0.view(np.uint32), v1.view(np.uint32))
            assert np.array_equal(b0, b1)
        _ = torch.ones(10, device="cuda").sum().item()


def _against_oracle(b, label):
    worst = 0.0
    for i, ((mesh, prob), plan) in enumerate(zip(b.instances, b.plans)):
        rr = oracle.assemble(oracle.OracleProblem(mesh, prob))
        ptr, kp = (host(t) for t in plan.pairs())
        assert np.array_equal(ptr, rr["pair_ptr"]) and np.array_equal(kp, rr["pair_kp"]), (label, i)
        rowptr, col, val = (host(t) for t in plan.csr(0))
        assert np.array_equal(rowptr, rr["rowptr"]) and np.array_equal(col, rr["col"]), (label, i)
        err = row_scaled_error(rowptr, val.astype(np.float64), rr["val"])
        print("%s instance %d: K %d delta/h %.0f %s %s, row-scaled error %.3e" % (
            label, i, mesh.n_triangles, prob.delta / mesh.h, prob.kernel, prob.ball, err), flush=True)
        worst = max(worst, err)
        assert err < TOL32, (label, i, err)
    return worst


def test_batch_instances_match_oracle():
    """Each instance of the test batch (constant and fractional kernels,
    barycenter and 8-arc balls, delta/h from 2 to 5), assembled by the
    persistent graph-replayed launch, against the oracle."""
    b = Batch(_instances())
    fs, gs = _inputs(b)
    b.assemble(mode=1, f_outer=fs, g_node=gs)
    torch.cuda.synchronize()
    _against_oracle(b, "test batch")


def test_workload_delta_h_2_fractional_instances_match_oracle():
    """The 64-instance workload's fractional instances with delta/h = 2 (there
    the singular rule's radial integrals stop at the ball), batched by
    themselves, against the oracle."""
    inst = batch_instances()
    pick = [i for i, (m, p) in enumerate(inst) if p.kernel == "fractional" and round(p.delta / m.h) == 2]
    print("workload instances", pick, flush=True)
    assert len(pick) >= 2
    b = Batch([inst[i] for i in pick])
    fs, gs = _inputs(b)
    b.assemble(mode=1, f_outer=fs, g_node=gs)
    torch.cuda.synchronize()
    _against_oracle(b, "workload")
