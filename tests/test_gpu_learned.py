"""GPU tests of the learned cap corrector against the FP64 oracle.

Bars (derivations): the GPU network rounds its hidden activations and W2, W3
to bfloat16 (relative spacing 2^-8, rounding error <= 2^-9 ~ 2e-3) and
accumulates in FP32; the oracle runs the same weights (W2, W3 rounded the
same way) in FP64 with unrounded activations.  Each output is a 128-term
sum of such products, so its error is a few 1e-3 of the output scale:
forward within 2e-2 of the largest output, gradients within 3e-2 (relative
2-norm per weight group, one more rounded layer).  Assembly with learned
caps: the FP32 path's 2e-5 row-scaled bar plus the network error on the cap
share of an entry (caps are ~1e-3 of an item's mass) -> 5e-5.  Sample
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
    assert rel < 0.35
    # checkpoint round trip
    import tempfile, os
    with tempfile.TemporaryDirectory() as d:
        path = os.path.join(d, "net.bin")
        m.save(path)
        m2 = Mlp.load(path)
        assert np.array_equal(m2.get_weights()[0], w)
        assert torch.equal(m2.forward(fh[:64]), m.forward(fh[:64]))


def _learned_problem(d, band=0.02):
    return Problem(delta=d, kernel_c=constant_kernel_c(d), ball="retri", cap_edges=8, outer="dunavant7",
                   inner="dunavant16", precision="learned", fallback_band=band)


def test_learned_assembly_matches_oracle():
    d = 0.1
    mesh = structured_mesh(d, d / 4, jitter=0.1, seed=31)
    scale = 1e-5
    m, w = _seeded_mlp(seed=12, bias=0.3, scale=scale)
    prob = _learned_problem(d)
    _say("case learned assembly K", mesh.n_triangles)
    u, f = manufactured("quadratic")
    plan = Plan(mesh, prob, mlp=m)
    xq = plan.outer_points()
    plan.assemble(f(xq[..., 0], xq[..., 1]).contiguous(),
                  torch.tensor(u(mesh.xy[:, 0], mesh.xy[:, 1]), dtype=torch.float64, device="cuda"))
    torch.cuda.synchronize()
    info = plan.info()
    _say("items", info["items"])
    assert info["items"]["learned"] > 0
    ref = oracle.solve_problem(mesh, prob, "quadratic", mlp_w=ob.effective_weights(w), mlp_scale=scale)
    rr = ref["res"]
    rowptr, col, val = (host(t) for t in plan.csr(0))
    assert np.array_equal(rowptr, rr["rowptr"]) and np.array_equal(col, rr["col"])
    err = row_scaled_error(rowptr, val.astype(np.float64), rr["val"])
    _say("learned row-scaled entry error %.3e" % err)
    assert err < 5e-5
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
