"""The C ABI without a GPU: the library loads, exports every function
declared in include/nlasm.h, and rejects invalid input on the host with the
documented status codes (no device call is made before validation)."""
import ctypes as C
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "nlasm.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(nla_[a-z_0-9]+)\s*\(", src)))


@pytest.fixture(scope="module")
def L():
    path = os.path.join(ROOT, "paper_2005_10775_amd", "libnlasm.so")
    if not os.path.exists(path):
        from paper_2005_10775_amd import build
        build.build()
    return C.CDLL(path)


def test_exports_every_declared_symbol(L):
    names = _declared()
    assert len(names) >= 14
    for n in names:
        assert hasattr(L, n), n


from paper_2005_10775_amd import binding as B  # noqa: E402  (ctypes structs only)
from workloads import Problem, constant_kernel_c, get_rule, structured_mesh  # noqa: E402


def _create(L, mesh, prob, mutate_mesh=None):
    keep = []
    xy = np.ascontiguousarray(mesh.xy)
    tri = np.ascontiguousarray(mesh.tri)
    tin = np.ascontiguousarray(mesh.tri_in_omega)
    nfr = np.ascontiguousarray(mesh.node_free)
    if mutate_mesh:
        xy, tri, tin, nfr = mutate_mesh(xy.copy(), tri.copy(), tin.copy(), nfr.copy())
    keep += [xy, tri, tin, nfr]
    m = B.nla_mesh(xy.shape[0], tri.shape[0], xy.ctypes.data, tri.ctypes.data, tin.ctypes.data, nfr.ctypes.data)
    p = B.nla_problem()
    p.delta, p.kernel, p.kernel_c, p.kernel_s = prob.delta, B.KERNELS[prob.kernel], prob.kernel_c, prob.kernel_s
    p.outer = B._rule(get_rule(prob.outer), keep)
    p.inner = B._rule(get_rule(prob.inner), keep)
    p.ball, p.cap_edges, p.precision = B.BALLS[prob.ball], prob.cap_edges, B.PRECISIONS[prob.precision]
    h = C.c_void_p()
    L.nla_last_error.restype = C.c_char_p
    code = L.nla_plan_create(C.byref(m), C.byref(p), None, C.byref(h))
    return code, L.nla_last_error().decode()


@pytest.fixture
def small():
    d = 0.1
    return structured_mesh(d, 0.05), Problem(delta=d, kernel_c=constant_kernel_c(d), ball="retri", cap_edges=8)


def test_clockwise_triangle_rejected(L, small):
    def flip(xy, tri, tin, nfr):
        tri[3] = tri[3][[0, 2, 1]]
        return xy, tri, tin, nfr
    code, msg = _create(L, *small, mutate_mesh=flip)
    assert code == -2 and "counter-clockwise" in msg


def test_index_out_of_range_rejected(L, small):
    def bad(xy, tri, tin, nfr):
        tri[0, 1] = xy.shape[0] + 5
        return xy, tri, tin, nfr
    assert _create(L, *small, mutate_mesh=bad)[0] == -2


def test_free_node_on_layer_rejected(L, small):
    def bad(xy, tri, tin, nfr):
        nfr[tri[np.nonzero(tin == 0)[0][0], 0]] = 1
        return xy, tri, tin, nfr
    code, msg = _create(L, *small, mutate_mesh=bad)
    assert code == -2 and "free node" in msg


def test_invalid_problem_fields(L, small):
    mesh, prob = small
    from dataclasses import replace
    assert _create(L, mesh, replace(prob, delta=-1.0))[0] == -1
    assert _create(L, mesh, replace(prob, cap_edges=1))[0] == -1
    assert _create(L, mesh, replace(prob, cap_edges=65))[0] == -1
    assert _create(L, mesh, replace(prob, kernel_c=0.0))[0] == -1


def test_ball_inside_triangle_unsupported(L):
    """The balls that cut elements need every element's inradius < delta/2 (no
    ball inside an element, every cap less than a half circle): a mesh scaled
    by 4 has inradius 0.29 * 2 > 0.25 and is refused before any device work;
    the unscaled one (inradius 0.15) passes validation."""
    mesh = structured_mesh(0.5, 0.5)
    prob = Problem(delta=0.5, kernel_c=1.0, ball="retri", cap_edges=8)
    for ball in ("retri", "shifted", "barysupport"):
        from dataclasses import replace
        pb = replace(prob, ball=ball, outer="strang4", inner="gauss3")
        code, msg = _create(L, mesh, pb, mutate_mesh=lambda xy, tri, tin, nfr: (xy * 4.0, tri, tin, nfr))
        assert code == -5 and "inradius" in msg, (ball, code, msg)
        code, msg = _create(L, mesh, pb)
        assert code != -5, (ball, msg)


def _create_prob(L, mesh, prob):
    """nla_plan_create through the binding's marshalling (every problem field)."""
    keep = []
    m, p = B.marshal(mesh, prob, keep)
    h = C.c_void_p()
    L.nla_last_error.restype = C.c_char_p
    code = L.nla_plan_create(C.byref(m), C.byref(p), None, C.byref(h))
    msg = L.nla_last_error().decode()
    if code == 0:
        L.nla_plan_destroy(h)
    return code, msg


def test_paper_workloads_pass_validation(L):
    """Every workload of Sec. 8 is accepted: on a host without a GPU the first
    device call then fails (NLA_E_DEVICE), after validation; with one, the
    plan is made."""
    from workloads import paper_workload
    for ball in ("exactcaps", "approxcaps", "nocaps", "barycenter", "overlap", "shifted", "barynocaps",
                 "baryapproxcaps", "analyticcaps"):
        for h, grid in ((0.1, "a"), (0.05, "b")):
            mesh, prob, _ = paper_workload(h, ball, grid=grid)
            code, msg = _create_prob(L, mesh, prob)
            assert code in (0, -4), (ball, h, grid, code, msg)


def test_ball_and_cap_rules_unsupported(L):
    """The balls and cap modes that need the constant kernel, FP64, one outer
    rule, arc caps or rules exact for quadratics are refused with
    NLA_E_UNSUPPORTED and a message naming the requirement."""
    from dataclasses import replace
    from workloads import paper_workload
    mesh = structured_mesh(0.1, 0.05)
    shifted = paper_workload(0.05, "shifted")[1]
    bary = paper_workload(0.05, "barynocaps")[1]
    overlap = paper_workload(0.05, "overlap")[1]
    analytic = paper_workload(0.05, "analyticcaps")[1]
    cases = [
        (replace(shifted, kernel="fractional", kernel_s=0.4, duffy_order=8), "constant kernel"),
        (replace(overlap, precision="fp32", outer2="", switch_dist=0.0), "NLA_FP64"),
        (replace(shifted, outer2="vertex7", switch_dist=0.01), "one outer rule"),
        (replace(bary, cap_mode="centroid"), "arc caps"),
        (replace(shifted, inner="centroid1"), "inner rule exact for quadratics"),
        (replace(bary, outer="centroid1"), "outer rule exact for quadratics"),
        (replace(analytic, precision="fp32", outer2="", switch_dist=0.0), "exact caps"),
        (replace(analytic, inner="centroid1"), "exact caps"),
        (replace(analytic, ball="barycenter"), "exact caps"),
    ]
    for prob, need in cases:
        code, msg = _create_prob(L, mesh, prob)
        assert code == -5 and need in msg, (prob, code, msg)


def test_invalid_ball_fields(L):
    from dataclasses import replace
    from workloads import paper_workload
    mesh = structured_mesh(0.1, 0.05)
    prob = paper_workload(0.05, "approxcaps")[1]
    code, msg = _create_prob(L, mesh, replace(prob, switch_dist=-1.0))
    assert code == -1 and "switch_dist" in msg
    keep = []
    m, p = B.marshal(mesh, prob, keep)
    h = C.c_void_p()
    for field, bad in (("ball", 5), ("cap_mode", 3)):
        saved = getattr(p, field)
        setattr(p, field, bad)
        assert L.nla_plan_create(C.byref(m), C.byref(p), None, C.byref(h)) == -1, field
        assert field.split("_")[-1] in L.nla_last_error().decode()
        setattr(p, field, saved)
