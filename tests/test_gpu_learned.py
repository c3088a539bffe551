"""GPU tests of the learned cap corrector against the FP64 oracle.

Bars (derivations): the GPU network rounds its hidden activations and W2, W3
to bfloat16 (relative spacing 2^-8, rounding error <= 2^-9 ~ 2e-3) and
accumulates in FP32; the oracle runs the same weights (W2, W3 rounded the
same way) in FP64 with unrounded activations.  Each output is a 128-term
sum of such products, so its error is a few 1e-3 of the output scale:
forward within 2e-2 of the largest output, gradients within 3e-2 (relative
2-norm per weight group, one more rounded layer).  Assembly with learned
caps: the FP32 path's 1e-6 row-scaled bar (tests/test_gpu_fp32.py); the
network's own error (a few 1e-3 of its outputs) falls on the cap moments,
about 1e-3 of an item's mass, times a small output scale (1e-5 here):
below 1e-7 of an entry.  Measured 1.4e-7 (h = delta/4), 7.1e-8 (the
headline mesh, sampled rows).  Sample
generation is FP64 on both sides: labels within 1e-6 relative (float
output), features within 1 float ulp.
"""
import sys

import numpy as np
import pytest
import torch

import oracle
import oracle.binding as ob
from gpu_util import gpu_assemble, host, row_scaled_error
from paper_2005_10775_amd import Mlp, Plan
from workloads import Problem, constant_kernel_c, manufactured, structured_mesh
from workloads.learned import OFFSETS, cap_uniforms, mlp_init

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def _setup():
    oracle.build(force=False)
    assert torch.cuda.is_available()


def test_samples_match_oracle():
    _say("case samples 3000 candidates")
    feat, lab = Mlp.samples(3000, 20052, first=17)
    U = cap_uniforms(20052, 17, 3000)
    valid, f_ref, l_ref, _ = ob.cap_candidates(U, 0.125, 0.1, 0.02)
    f, l = host(feat), host(lab)
    _say("kept", f.shape[0], "oracle", int(valid.sum()))
    assert f.shape[0] == int(valid.sum())
    assert np.max(np.abs(f - f_ref[valid])) <= 2e-6
    assert np.max(np.abs(l - l_ref[valid])) <= 1e-6 * np.abs(l_ref[valid]).max()


def _seeded_mlp(seed=9, bias=0.2, scale=1.0):
    w = mlp_init(seed, bias_scale=bias)
    m = Mlp()
    m.set_weights(w, scale)
    return m, w


def test_forward_matches_oracle():
    _say("case forward")
    m, w = _seeded_mlp()
    U = cap_uniforms(20052, 0, 4000)
    valid, f_ref, _, _ = ob.cap_candidates(U, 0.125, 0.1, 0.02)
    f32 = f_ref[valid][:517].astype(np.float32)        # a ragged tile count
    y = host(m.forward(torch.from_numpy(f32).cuda()))
    ref = ob.mlp_forward(ob.effective_weights(w), f32.astype(np.float64))
    err = np.max(np.abs(y - ref)) / np.abs(ref).max()
    _say("forward max error / max output %.3e" % err)
    assert err < 2e-2
    assert np.sqrt(np.mean((y - ref) ** 2)) < 5e-3 * np.sqrt(np.mean(ref ** 2))
    # bfloat16 weights round-trip
    w_back, sc = m.get_weights()
    assert np.array_equal(w_back, w) and sc == 1.0


def test_backward_matches_oracle():
    _say("case backward")
    m, w = _seeded_mlp(seed=10)
    rng = np.random.default_rng(1)
    f32 = rng.uniform(-1.2, 1.2, (100, 6)).astype(np.float32)
    dout = rng.normal(size=(100, 3)).astype(np.float32)
    dw = host(m.backward(torch.from_numpy(f32).cuda(), torch.from_numpy(dout).cuda()))
    ref = ob.mlp_backward(ob.effective_weights(w), f32.astype(np.float64), dout.astype(np.float64))
    for name, (off, shape) in OFFSETS.items():
        n = int(np.prod(shape))
        a, r = dw[off:off + n], ref[off:off + n]
        rel = np.linalg.norm(a - r) / np.linalg.norm(r)
        _say("grad %s relative error %.3e" % (name, rel))
        assert rel < 3e-2, name


def test_training_reduces_loss_and_predicts_labels():
    _say("case training")
    feat, lab = Mlp.samples(300_000, 20052)
    n = feat.shape[0]
    m = Mlp(seed=3)
    log = m.train(feat, lab, epochs=12, batch=1024, lr=2e-3, seed=7)
    _say("samples", n, "loss", ["%.4f" % v for v in log])
    assert log[-1] < 0.25 * log[0]
    assert all(np.isfinite(log))
    # held-out candidates
    fh, lh = Mlp.samples(50_000, 20052, first=10_000_000)
    w, sc = m.get_weights()
    pred = host(m.forward(fh)) * sc
    lab_h = host(lh)
    rel = np.sqrt(np.mean((pred - lab_h) ** 2)) / np.sqrt(np.mean(lab_h ** 2))
    _say("held-out relative rms error %.3f" % rel)
    assert rel < 0.3          # measured 0.225 with this short recipe (300k samples, 12 epochs)
    # checkpoint round trip
    import tempfile, os
    with tempfile.TemporaryDirectory() as d:
        path = os.path.join(d, "net.bin")
        m.save(path)
        m2 = Mlp.load(path)
        assert np.array_equal(m2.get_weights()[0], w)
        assert torch.equal(m2.forward(fh[:64]), m.forward(fh[:64]))
        assert np.array_equal(m2.get_domain(), m.get_domain())


def _learned_problem(d, band=0.02):
    return Problem(delta=d, kernel_c=constant_kernel_c(d), ball="retri", cap_edges=8, outer="dunavant7",
                   inner="dunavant16", precision="learned", fallback_band=band)


def _narrow_domain():
    """The training domain of 400 oracle candidates of the h = delta/4 family
    with its edge-length range narrowed by a tenth of its width at each end:
    about a quarter of a jittered delta/4 mesh's far-from-tangency items fall
    outside it."""
    U = cap_uniforms(20053, 0, 2500)
    valid, feat, _, _ = ob.cap_candidates(U, 0.25, 0.1, 0.02)
    dom = ob.feature_domain(feat[valid][:400])
    w = dom[3] - dom[2]
    dom[2] += 0.1 * w
    dom[3] -= 0.1 * w
    return dom


@pytest.mark.parametrize("domain", ["unbounded", "narrow"])
def test_learned_assembly_matches_oracle(domain):
    d = 0.1
    mesh = structured_mesh(d, d / 4, jitter=0.1, seed=31)
    scale = 1e-5
    m, w = _seeded_mlp(seed=12, bias=0.3, scale=scale)
    dom = None
    if domain == "narrow":
        dom = _narrow_domain()
        m.set_domain(dom)
        assert np.array_equal(m.get_domain(), dom)
    prob = _learned_problem(d)
    _say("case learned assembly K", mesh.n_triangles, "domain", domain)
    u, f = manufactured("quadratic")
    plan = Plan(mesh, prob, mlp=m)
    xq = plan.outer_points()
    plan.assemble(f(xq[..., 0], xq[..., 1]).contiguous(),
                  torch.tensor(u(mesh.xy[:, 0], mesh.xy[:, 1]), dtype=torch.float64, device="cuda"))
    torch.cuda.synchronize()
    info = plan.info()
    _say("items", info["items"])
    assert info["items"]["learned"] > 0
    if dom is not None:
        # the domain sends part of the far-from-tangency items back to the exact caps
        m0, _ = _seeded_mlp(seed=12, bias=0.3, scale=scale)
        full = Plan(mesh, prob, mlp=m0)
        full.assemble()
        torch.cuda.synchronize()
        _say("routed without the domain", full.info()["items"]["learned"])
        assert 0 < info["items"]["learned"] < 0.9 * full.info()["items"]["learned"]
    ref = oracle.solve_problem(mesh, prob, "quadratic", mlp_w=ob.effective_weights(w), mlp_scale=scale,
                               mlp_domain=dom)
    rr = ref["res"]
    rowptr, col, val = (host(t) for t in plan.csr(0))
    assert np.array_equal(rowptr, rr["rowptr"]) and np.array_equal(col, rr["col"])
    err = row_scaled_error(rowptr, val.astype(np.float64), rr["val"])
    _say("learned row-scaled entry error %.3e" % err)
    assert err < 1e-6
    # the network's share is visible: the plain FP32 exact-cap matrix differs by more
    plain = gpu_assemble(mesh, Problem(delta=d, kernel_c=constant_kernel_c(d), ball="retri", cap_edges=8,
                                       outer="dunavant7", inner="dunavant16", precision="fp32"))
    pv = host(plain.csr(0)[2]).astype(np.float64)
    assert row_scaled_error(rowptr, pv, rr["val"]) > 4 * err


def test_band_infinite_is_the_fp32_exact_path():
    d = 0.1
    mesh = structured_mesh(d, d / 4, jitter=0.1, seed=32)
    m, _ = _seeded_mlp(seed=13, scale=1e-5)
    _say("case band=inf")
    p_learn = Plan(mesh, _learned_problem(d, band=1e9), mlp=m)
    p_learn.assemble()
    p32 = Plan(mesh, Problem(delta=d, kernel_c=constant_kernel_c(d), ball="retri", cap_edges=8, outer="dunavant7",
                             inner="dunavant16", precision="fp32"))
    p32.assemble()
    torch.cuda.synchronize()
    assert p_learn.info()["items"]["learned"] == 0
    assert torch.equal(p_learn.csr(0)[2], p32.csr(0)[2])


def _solve(plan, mesh, u):
    U, its, rel = plan.cg(plan.load(), rtol=1e-12)
    full = u(mesh.xy[:, 0], mesh.xy[:, 1]).copy()
    full[host(plan.free_nodes())] = host(U)
    return full


def _assembled(mesh, prob, man, mlp=None):
    u, f = manufactured(man)
    plan = Plan(mesh, prob, mlp=mlp)
    xq = plan.outer_points()
    plan.assemble(f(xq[..., 0], xq[..., 1]).contiguous(),
                  torch.tensor(u(mesh.xy[:, 0], mesh.xy[:, 1]), dtype=torch.float64, device="cuda"))
    torch.cuda.synchronize()
    return plan, _solve(plan, mesh, u)


def test_trained_network_gains_over_no_caps():
    """What the trained network gains: train on the GPU with the workload's
    recipe (4M samples of the h = delta/8 family labelled by the FP64 8-arc
    caps, 20 epochs), then on the headline mesh (delta = 0.1, h = delta/8
    jittered) solve with the FP64 exact (8-arc) caps, with no caps (the
    inscribed polygon, FP32) and with the learned caps (FP32).  The learned
    solution must lie within 1e-4 of the exact-cap solution in L2(Omega) and
    at least ten times closer to it than the no-cap solution.  The network
    records its training domain; a h = delta/4 mesh, outside it, routes no
    item to the network."""
    from dataclasses import replace
    from workloads import make_config
    from workloads.learned import TRAIN
    feat, lab = Mlp.samples(int(TRAIN["samples"] / 0.17), TRAIN["seed"], L=TRAIN["L"], jitter=TRAIN["jitter"],
                            band=TRAIN["band"], cap_edges=TRAIN["cap_edges"])
    feat, lab = feat[:TRAIN["samples"]].contiguous(), lab[:TRAIN["samples"]].contiguous()
    _say("case gain: training on", feat.shape[0], "samples")
    net = Mlp(seed=TRAIN["seed"])
    log = net.train(feat, lab, epochs=TRAIN["epochs"], batch=TRAIN["batch"], lr=TRAIN["lr"], seed=TRAIN["seed"])
    _say("loss", ["%.4f" % v for v in log])
    dom = net.get_domain()
    _say("training domain", np.round(dom, 4).tolist())
    assert np.all(np.isfinite(dom))
    assert np.array_equal(dom, ob.feature_domain(host(feat)))
    fh, lh = Mlp.samples(400_000, TRAIN["seed"], first=10 ** 9)
    w, sc = net.get_weights()
    pred = host(net.forward(fh)) * sc
    held = float(np.sqrt(np.mean((pred - host(lh)) ** 2)) / np.sqrt(np.mean(host(lh) ** 2)))
    _say("held-out relative rms error %.4f" % held)
    assert held < 0.06

    mesh, p64, man = make_config("c2")
    _, U_exact = _assembled(mesh, p64, man)
    _, U_nocap = _assembled(mesh, replace(p64, precision="fp32", cap_edges=0), man)
    plan, U_learn = _assembled(mesh, replace(p64, precision="learned"), man, mlp=net)
    n_learn = plan.info()["items"]["learned"]
    zero = lambda x, y: 0.0 * x
    d_learn = oracle.l2_error(mesh, U_learn - U_exact, zero)
    d_nocap = oracle.l2_error(mesh, U_nocap - U_exact, zero)
    _say("routed %d items; ||u_learned - u_exact|| = %.3e, ||u_nocaps - u_exact|| = %.3e (ratio %.1f)" % (
        n_learn, d_learn, d_nocap, d_nocap / d_learn))
    assert n_learn > 0.3 * plan.info()["items"]["partial"]
    assert d_learn <= 1e-4
    assert d_learn <= 0.1 * d_nocap

    # out of distribution: elements twice the training size route nothing
    m4 = structured_mesh(0.1, 0.025, jitter=0.1, seed=5)
    p4 = Plan(m4, replace(p64, precision="learned"), mlp=net)
    p4.assemble()
    torch.cuda.synchronize()
    _say("h = delta/4 mesh: items", p4.info()["items"])
    assert p4.info()["items"]["partial"] > 0 and p4.info()["items"]["learned"] == 0
