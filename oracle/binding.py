"""ctypes marshalling for liboracle.so plus plain numpy solves.

Test infrastructure only (see the package docstring).
"""
import ctypes as C
import os
import subprocess
import numpy as np
import scipy.sparse as sp

from workloads.rules import get_rule, gauss_legendre01

_DIR = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_DIR, "liboracle.so")
_LIB = None


def build(force=True):
    """Compile liboracle.so (gcc, FP64, no contraction, OpenMP for timing only)."""
    srcs = [os.path.join(_DIR, f) for f in ("nlo.c", "nlo_duffy.c", "nlo_mlp.c")]
    if not force and os.path.exists(_SO) and all(os.path.getmtime(_SO) >= os.path.getmtime(s) for s in srcs):
        return _SO
    cmd = ["gcc", "-O2", "-std=c99", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
           "-fopenmp", "-o", _SO] + srcs + ["-lm"]
    subprocess.check_call(cmd)
    return _SO


class _Mesh(C.Structure):
    _fields_ = [("nv", C.c_int32), ("nt", C.c_int32), ("xy", C.c_void_p), ("tri", C.c_void_p),
                ("tri_in_omega", C.c_void_p), ("node_free", C.c_void_p)]


class _Problem(C.Structure):
    _fields_ = [("delta", C.c_double), ("kernel", C.c_int32), ("kc", C.c_double), ("ks", C.c_double),
                ("ball", C.c_int32), ("cap_mode", C.c_int32), ("cap_edges", C.c_int32),
                ("n_out", C.c_int32), ("out_lam", C.c_void_p), ("out_w", C.c_void_p),
                ("n_in", C.c_int32), ("in_lam", C.c_void_p), ("in_w", C.c_void_p),
                ("n_out2", C.c_int32), ("out2_lam", C.c_void_p), ("out2_w", C.c_void_p),
                ("switch_dist", C.c_double),
                ("duffy_n", C.c_int32), ("gl_x", C.c_void_p), ("gl_w", C.c_void_p),
                ("skip_ixi", C.c_int32),
                ("learned", C.c_int32), ("band", C.c_double), ("mlp_w", C.c_void_p), ("mlp_scale", C.c_double),
                ("mlp_domain", C.c_void_p)]


def _lib():
    global _LIB
    if _LIB is None:
        if not os.path.exists(_SO):
            build()
        L = C.CDLL(_SO)
        P, I32, I64, D = C.c_void_p, C.c_int32, C.c_int64, C.c_double
        L.nlo_pairs_of.argtypes = [P, P, I32, P, I32]
        L.nlo_pairs_of.restype = C.c_int
        L.nlo_pair_block.argtypes = [P, P, I32, I32, P, P, P, P]
        L.nlo_pair_block.restype = C.c_int
        L.nlo_region.argtypes = [P, P, P, P, I32, P, P, P]
        L.nlo_region.restype = C.c_int
        L.nlo_inner_sums.argtypes = [P, P, P, P, P, P]
        L.nlo_inner_sums.restype = C.c_int
        L.nlo_assemble.argtypes = [P, P, I32]
        L.nlo_assemble.restype = P
        L.nlo_result_sizes.argtypes = [P, P, P, P]
        L.nlo_result_copy.argtypes = [P, P, P, P, P, P]
        L.nlo_result_free.argtypes = [P]
        L.nlo_row.argtypes = [P, P, I32, P, P, I32]
        L.nlo_row.restype = C.c_int
        L.nlo_load.argtypes = [P, P, P, P]
        L.nlo_outer_points.argtypes = [P, P, P]
        L.nlo_blocks_range.argtypes = [P, P, I32, I32, I32, P]
        L.nlo_blocks_range.restype = I64
        L.nlo_flops_census.argtypes = [P, P, I32, I32, P]
        L.nlo_flops_census.restype = I64
        L.nlo_gelu.argtypes = [D]
        L.nlo_gelu.restype = D
        L.nlo_mlp_forward.argtypes = [P, P, I64, P]
        L.nlo_mlp_backward.argtypes = [P, P, P, I64, P]
        L.nlo_cap_moments.argtypes = [P, P, P, P]
        L.nlo_cap_moments.restype = C.c_int
        L.nlo_routed.argtypes = [D, D, P, P]
        L.nlo_routed.restype = C.c_int
        L.nlo_in_domain.argtypes = [P, P, P, D]
        L.nlo_in_domain.restype = C.c_int
        L.nlo_cap_candidate.argtypes = [P, D, D, D, I32, P, P, P]
        L.nlo_mlp_features.argtypes = [P, P, D, P]
        L.nlo_mlp_features.restype = None
        L.nlo_cap_candidate.restype = C.c_int
        _LIB = L
    return _LIB


def _ptr(a):
    return a.ctypes.data_as(C.c_void_p)


class OracleProblem:
    """Marshals a workloads.Problem (and a mesh) into the C structs; keeps the
    numpy buffers alive for the lifetime of this object."""

    def __init__(self, mesh, prob, mlp_w=None, mlp_scale=1.0, mlp_domain=None):
        self.mesh = mesh
        self.prob = prob
        self._keep = []
        m = _Mesh()
        xy = np.ascontiguousarray(mesh.xy, dtype=np.float64)
        tri = np.ascontiguousarray(mesh.tri, dtype=np.int32)
        tin = np.ascontiguousarray(mesh.tri_in_omega, dtype=np.uint8)
        nfr = np.ascontiguousarray(mesh.node_free, dtype=np.uint8)
        self._keep += [xy, tri, tin, nfr]
        m.nv, m.nt = xy.shape[0], tri.shape[0]
        m.xy, m.tri, m.tri_in_omega, m.node_free = _ptr(xy), _ptr(tri), _ptr(tin), _ptr(nfr)
        self.cmesh = m
        p = _Problem()
        p.delta = prob.delta
        p.kernel = {"constant": 0, "fractional": 1}[prob.kernel]
        p.kc = prob.kernel_c
        p.ks = prob.kernel_s
        p.ball = {"barycenter": 0, "retri": 1, "overlap": 2, "shifted": 3, "barysupport": 4}[prob.ball]
        if p.ball >= 2 and p.kernel != 0:
            raise ValueError("the overlap, shifted and barysupport balls take the constant kernel")
        p.cap_mode = {"poly": 0, "centroid": 1, "analytic": 2}[prob.cap_mode]
        if p.cap_mode == 2 and (p.kernel != 0 or p.ball not in (1, 3)):
            raise ValueError("analytic caps integrate the constant kernel over the intersection or shifted ball")
        p.cap_edges = prob.cap_edges
        ro = get_rule(prob.outer)
        ri = get_rule(prob.inner)
        self.outer = ro
        self.inner = ri
        for r, pre in ((ro, "out"), (ri, "in")):
            lam = np.ascontiguousarray(r.lam)
            w = np.ascontiguousarray(r.w)
            self._keep += [lam, w]
            setattr(p, "n_" + pre, r.n)
            setattr(p, pre + "_lam", _ptr(lam))
            setattr(p, pre + "_w", _ptr(w))
        if prob.outer2:
            r2 = get_rule(prob.outer2)
            lam = np.ascontiguousarray(r2.lam)
            w = np.ascontiguousarray(r2.w)
            self._keep += [lam, w]
            p.n_out2, p.out2_lam, p.out2_w = r2.n, _ptr(lam), _ptr(w)
            p.switch_dist = prob.switch_dist
        else:
            p.n_out2 = 0
        if prob.duffy_order > 0:
            gx, gw = gauss_legendre01(prob.duffy_order)
            self._keep += [gx, gw]
            p.duffy_n, p.gl_x, p.gl_w = prob.duffy_order, _ptr(gx), _ptr(gw)
        else:
            p.duffy_n = 0
        p.skip_ixi = int(prob.skip_ixi)
        if prob.precision == "learned":
            if mlp_w is None:
                raise ValueError("learned caps need the network weights (effective_weights(...))")
            w = np.ascontiguousarray(mlp_w, dtype=np.float64)
            self._keep.append(w)
            p.learned, p.band, p.mlp_w, p.mlp_scale = 1, prob.fallback_band, _ptr(w), mlp_scale
            if mlp_domain is not None:
                dom = np.ascontiguousarray(mlp_domain, dtype=np.float64)
                if dom.shape != (4,):
                    raise ValueError("the training domain has 4 limits")
                self._keep.append(dom)
                p.mlp_domain = _ptr(dom)
        self.cprob = p

    @property
    def args(self):
        return C.byref(self.cmesh), C.byref(self.cprob)


def assemble(op, nthreads=0):
    """Full matrix D (CSR, J x J) and the canonical pair list."""
    L = _lib()
    h = L.nlo_assemble(*op.args, nthreads)
    npairs, nnz, st = C.c_int64(), C.c_int64(), C.c_int32()
    L.nlo_result_sizes(h, C.byref(npairs), C.byref(nnz), C.byref(st))
    K, J = op.mesh.n_triangles, op.mesh.n_vertices
    out = dict(pair_ptr=np.empty(K + 1, np.int64), pair_kp=np.empty(max(1, npairs.value), np.int32),
               rowptr=np.empty(J + 1, np.int64), col=np.empty(max(1, nnz.value), np.int32),
               val=np.empty(max(1, nnz.value), np.float64))
    L.nlo_result_copy(h, *[_ptr(out[k]) for k in ("pair_ptr", "pair_kp", "rowptr", "col", "val")])
    L.nlo_result_free(h)
    out["pair_kp"] = out["pair_kp"][:npairs.value]
    out["col"] = out["col"][:nnz.value]
    out["val"] = out["val"][:nnz.value]
    out["status"] = st.value
    if st.value != 0:
        raise RuntimeError("oracle assembly failed with status %d" % st.value)
    out["D"] = sp.csr_matrix((out["val"], out["col"], out["rowptr"]), shape=(J, J))
    return out


def pairs_of(op, k):
    L = _lib()
    buf = np.empty(op.mesh.n_triangles, np.int32)
    n = L.nlo_pairs_of(*op.args, int(k), _ptr(buf), buf.shape[0])
    return buf[:n].copy()


def pair_block(op, k, kp):
    L = _lib()
    mxy, myy, s0q, blk = np.zeros(9), np.zeros(9), np.zeros(64), np.zeros(36)
    st = L.nlo_pair_block(*op.args, int(k), int(kp), _ptr(mxy), _ptr(myy), _ptr(s0q), _ptr(blk))
    if st < 0:
        raise RuntimeError("pair block status %d" % st)
    return dict(mxy=mxy.reshape(3, 3), myy=myy.reshape(3, 3), s0q=s0q[:op.outer.n],
                blk=blk.reshape(6, 6))


def row(op, j):
    L = _lib()
    J = op.mesh.n_vertices
    cols, vals = np.empty(J, np.int32), np.empty(J)
    n = L.nlo_row(*op.args, int(j), _ptr(cols), _ptr(vals), J)
    if n < 0:
        raise RuntimeError("row status %d" % n)
    return cols[:n].copy(), vals[:n].copy()


def outer_points(op):
    L = _lib()
    xq = np.empty((op.mesh.n_triangles, op.outer.n, 2))
    L.nlo_outer_points(*op.args, _ptr(xq))
    return xq


def load_vector(op, f_outer):
    L = _lib()
    f = np.ascontiguousarray(f_outer, dtype=np.float64)
    G = np.empty(op.mesh.n_vertices)
    L.nlo_load(*op.args, _ptr(f), _ptr(G))
    return G


def inner_sums(op, x, tri_xy):
    L = _lib()
    x = np.ascontiguousarray(x, dtype=np.float64)
    V = np.ascontiguousarray(np.asarray(tri_xy, dtype=np.float64).reshape(6))
    s0, s1, s2 = np.zeros(1), np.zeros(3), np.zeros(9)
    st = L.nlo_inner_sums(C.byref(op.cprob), _ptr(x), _ptr(V), _ptr(s0), _ptr(s1), _ptr(s2))
    if st < 0:
        raise RuntimeError("inner sums status %d" % st)
    return s0[0], s1, s2.reshape(3, 3)


def region(op, x, tri_xy, cap=2048):
    L = _lib()
    x = np.ascontiguousarray(x, dtype=np.float64)
    V = np.ascontiguousarray(np.asarray(tri_xy, dtype=np.float64).reshape(6))
    sub = np.empty(6 * cap)
    cp, cw, nc = np.empty(32), np.empty(8), C.c_int32()
    n = L.nlo_region(C.byref(op.cprob), _ptr(x), _ptr(V), _ptr(sub), cap, _ptr(cp), _ptr(cw), C.byref(nc))
    if n < 0:
        raise RuntimeError("region status %d" % n)
    per = 4 if op.prob.cap_mode == "analytic" else 2   # chord ends, or centroid points
    return sub[:6 * n].reshape(n, 3, 2).copy(), cp[:per * nc.value].reshape(-1, 2).copy(), cw[:nc.value].copy()


def blocks_range(op, k0, k1, nthreads=0):
    """Pair lists + local blocks of outer elements [k0, k1); returns (pairs, checksum)."""
    L = _lib()
    cs = C.c_double()
    n = L.nlo_blocks_range(*op.args, int(k0), int(k1), int(nthreads), C.byref(cs))
    return n, cs.value


def census(op, k0=0, k1=None):
    L = _lib()
    k1 = op.mesh.n_triangles if k1 is None else k1
    out = np.zeros(8, np.int64)
    L.nlo_flops_census(*op.args, int(k0), int(k1), _ptr(out))
    keys = ("pairs", "whole", "partial", "empty", "poly_tris", "caps", "cap_tris", "inner_pts")
    return dict(zip(keys, out.tolist()))


def system_from_full(mesh, D, G, g_node):
    """A = D[free, free], b = G[free] - D[free, dirichlet] g (Eqs. (appr), (intcon))."""
    free = mesh.node_free.astype(bool)
    fi = np.nonzero(free)[0]
    di = np.nonzero(~free)[0]
    Dc = D.tocsr()
    A = Dc[fi][:, fi]
    b = G[fi] - Dc[fi][:, di] @ g_node[di]
    return A.tocsr(), b, fi, di


def cg(A, b, rtol=1e-14, maxit=20000):
    """Plain conjugate gradients (Hestenes-Stiefel) on the SPD matrix A."""
    x = np.zeros_like(b)
    r = b - A @ x
    pvec = r.copy()
    rr = r @ r
    nb = np.linalg.norm(b)
    it = 0
    while np.sqrt(rr) > rtol * nb and it < maxit:
        Ap = A @ pvec
        a = rr / (pvec @ Ap)
        x += a * pvec
        r -= a * Ap
        rr_new = r @ r
        pvec = r + (rr_new / rr) * pvec
        rr = rr_new
        it += 1
    return x, it, np.sqrt(rr) / nb


def l2_error(mesh, U, u_exact, rule_name="dunavant7"):
    """||u - u_h||_{L2(Omega)} with a degree-5 rule on every element of Omega."""
    r = get_rule(rule_name)
    err = 0.0
    for k in np.nonzero(mesh.tri_in_omega)[0]:
        V = mesh.xy[mesh.tri[k]]
        a2 = abs((V[1, 0] - V[0, 0]) * (V[2, 1] - V[0, 1]) - (V[1, 1] - V[0, 1]) * (V[2, 0] - V[0, 0]))
        X = r.lam @ V
        uh = r.lam @ U[mesh.tri[k]]
        err += np.sum(r.w * a2 * (u_exact(X[:, 0], X[:, 1]) - uh) ** 2)
    return float(np.sqrt(err))


def solve_problem(mesh, prob, man, nthreads=0, dense=None, mlp_w=None, mlp_scale=1.0, mlp_domain=None):
    """Assemble, build A and b, solve, and return the L2 error against u."""
    from workloads.problems import manufactured
    u, f = manufactured(man)
    op = OracleProblem(mesh, prob, mlp_w=mlp_w, mlp_scale=mlp_scale, mlp_domain=mlp_domain)
    res = assemble(op, nthreads)
    xq = outer_points(op)
    G = load_vector(op, f(xq[..., 0], xq[..., 1]))
    g = u(mesh.xy[:, 0], mesh.xy[:, 1])
    A, b, fi, di = system_from_full(mesh, res["D"], G, g)
    if dense is None:
        dense = A.shape[0] <= 3000
    if dense:
        Uf = np.linalg.solve(A.toarray(), b)
        its = 0
    else:
        Uf, its, _ = cg(A, b)
    U = g.copy()
    U[fi] = Uf
    return dict(U=U, l2=l2_error(mesh, U, u), res=res, A=A, b=b, G=G, iters=its, op=op)


# ------------------------------------------------------------ learned caps

def bf16_round(a):
    """float32 -> nearest bfloat16 (ties to even), returned as float64."""
    u = np.ascontiguousarray(a, dtype=np.float32).view(np.uint32).astype(np.uint64)
    lsb = (u >> np.uint64(16)) & np.uint64(1)
    r = ((u + np.uint64(0x7FFF) + lsb) >> np.uint64(16)) << np.uint64(16)
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def effective_weights(w32):
    """The weights the network computes with: W2 and W3 rounded to bfloat16,
    W1 and the biases in float32 (flat layout of workloads.learned)."""
    from workloads.learned import OFFSETS
    w = np.asarray(w32, dtype=np.float32).astype(np.float64)
    for name in ("W2", "W3"):
        off, shape = OFFSETS[name]
        n = int(np.prod(shape))
        w[off:off + n] = bf16_round(np.asarray(w32, dtype=np.float32)[off:off + n])
    return w


def gelu(z):
    return _lib().nlo_gelu(float(z))


def mlp_forward(w, feat):
    w = np.ascontiguousarray(w, dtype=np.float64)
    f = np.ascontiguousarray(feat, dtype=np.float64).reshape(-1, 6)
    out = np.zeros((f.shape[0], 3))
    _lib().nlo_mlp_forward(_ptr(w), _ptr(f), f.shape[0], _ptr(out))
    return out


def mlp_backward(w, feat, dout):
    w = np.ascontiguousarray(w, dtype=np.float64)
    f = np.ascontiguousarray(feat, dtype=np.float64).reshape(-1, 6)
    d = np.ascontiguousarray(dout, dtype=np.float64).reshape(-1, 3)
    dw = np.zeros(w.shape[0])
    _lib().nlo_mlp_backward(_ptr(w), _ptr(f), _ptr(d), f.shape[0], _ptr(dw))
    return dw


def cap_moments(delta, x, tri_xy, cap_edges=8):
    """(number of cap triangles, int over the caps of the three basis functions)."""
    p = _Problem()
    p.delta, p.kc, p.ball, p.cap_edges = delta, 1.0, 1, cap_edges
    xx = np.ascontiguousarray(x, dtype=np.float64)
    V = np.ascontiguousarray(tri_xy, dtype=np.float64).reshape(6)
    m = np.zeros(3)
    n = _lib().nlo_cap_moments(C.byref(p), _ptr(xx), _ptr(V), _ptr(m))
    return n, m


def in_domain(dom, x, tri_xy, delta):
    """The item (x, E') inside the training domain dom[4] (None: unbounded)."""
    xx = np.ascontiguousarray(x, dtype=np.float64)
    V = np.ascontiguousarray(tri_xy, dtype=np.float64).reshape(6)
    d = None if dom is None else np.ascontiguousarray(dom, dtype=np.float64)
    return bool(_lib().nlo_in_domain(None if d is None else _ptr(d), _ptr(xx), _ptr(V), delta))


def feature_domain(feat):
    """The training domain {rlo, rhi, elo, ehi} of samples given by their float
    network inputs feat[n][6] (delta = 1, x = 0): the range of the squared
    vertex distances |v_a|^2 = (f_a0/8 + 1)^2 + (f_a1/8)^2 and of the squared
    edge lengths |f_b - f_a|^2 / 64."""
    g = np.asarray(feat, dtype=np.float32).astype(np.float64).reshape(-1, 6)
    r, e = [], []
    for a in range(3):
        b = (a + 1) % 3
        px, py = g[:, 2 * a] * 0.125 + 1.0, g[:, 2 * a + 1] * 0.125
        r.append(px * px + py * py)
        dx, dy = g[:, 2 * b] - g[:, 2 * a], g[:, 2 * b + 1] - g[:, 2 * a + 1]
        e.append((dx * dx + dy * dy) * (1.0 / 64.0))
    r, e = np.concatenate(r), np.concatenate(e)
    return np.array([r.min(), r.max(), e.min(), e.max()])


def routed(delta, band, x, tri_xy):
    xx = np.ascontiguousarray(x, dtype=np.float64)
    V = np.ascontiguousarray(tri_xy, dtype=np.float64).reshape(6)
    return bool(_lib().nlo_routed(delta, band, _ptr(xx), _ptr(V)))


def mlp_features(x, tri_xy, delta):
    xx = np.ascontiguousarray(x, dtype=np.float64)
    V = np.ascontiguousarray(tri_xy, dtype=np.float64).reshape(6)
    f = np.zeros(6)
    _lib().nlo_mlp_features(_ptr(xx), _ptr(V), delta, _ptr(f))
    return f


def cap_candidates(U, L, jitter, band, cap_edges=8):
    """Training candidates from uniforms U[n][10]:
    (valid[n], feat[n][6] network inputs, label[n][3], verts[n][6])."""
    U = np.ascontiguousarray(U, dtype=np.float64).reshape(-1, 10)
    n = U.shape[0]
    valid = np.zeros(n, dtype=bool)
    feat = np.zeros((n, 6))
    lab = np.zeros((n, 3))
    verts = np.zeros((n, 6))
    v6 = np.zeros(6)
    f6 = np.zeros(6)
    l3 = np.zeros(3)
    lib = _lib()
    for i in range(n):
        u = np.ascontiguousarray(U[i])
        valid[i] = lib.nlo_cap_candidate(_ptr(u), L, jitter, band, cap_edges, _ptr(v6), _ptr(f6), _ptr(l3)) == 1
        feat[i] = f6
        lab[i] = l3
        verts[i] = v6
    return valid, feat, lab, verts
