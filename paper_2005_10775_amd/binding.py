"""ctypes binding of libnlasm.so (argument marshalling only).

Every step of the assembly runs in the library's HIP kernels; PyTorch only
provides device memory and the current HIP stream.  Importing this module
raises if the built library is missing: there is no fallback path.
"""
import ctypes as C
import os

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libnlasm.so")

NLA_OK = 0
ERRORS = {-1: "NLA_E_INVALID", -2: "NLA_E_MESH", -3: "NLA_E_NOMEM", -4: "NLA_E_DEVICE",
          -5: "NLA_E_UNSUPPORTED", -6: "NLA_E_NOT_CONVERGED", -7: "NLA_E_STATE"}
KERNELS = {"constant": 0, "fractional": 1}
BALLS = {"barycenter": 0, "retri": 1, "overlap": 2, "shifted": 3, "barysupport": 4}
PRECISIONS = {"fp64": 0, "fp32": 1, "learned": 2}
NLA_SKIP_IXI = 1


class NlaError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("%s (%d): %s" % (ERRORS.get(code, "?"), code, msg))
        self.code = code


class nla_mesh(C.Structure):
    _fields_ = [("n_vertices", C.c_int32), ("n_triangles", C.c_int32), ("xy", C.c_void_p),
                ("tri", C.c_void_p), ("tri_in_omega", C.c_void_p), ("node_free", C.c_void_p)]


class nla_rule(C.Structure):
    _fields_ = [("n", C.c_int32), ("lam", C.c_void_p), ("w", C.c_void_p)]


class nla_problem(C.Structure):
    _fields_ = [("delta", C.c_double), ("kernel", C.c_int32), ("kernel_c", C.c_double),
                ("kernel_s", C.c_double), ("outer", nla_rule), ("inner", nla_rule),
                ("duffy_n", C.c_int32), ("duffy_x", C.c_void_p), ("duffy_w", C.c_void_p),
                ("ball", C.c_int32), ("cap_edges", C.c_int32), ("precision", C.c_int32),
                ("mlp", C.c_void_p), ("fallback_band", C.c_double), ("flags", C.c_uint32),
                ("outer2", nla_rule), ("switch_dist", C.c_double), ("cap_mode", C.c_int32)]


class nla_info(C.Structure):
    _fields_ = [("n_pairs", C.c_int64), ("nnz_full", C.c_int64), ("nnz_free", C.c_int64),
                ("n_free", C.c_int32), ("n_outer", C.c_int32), ("n_codes", C.c_int64),
                ("n_near", C.c_int64), ("items", C.c_int64 * 4), ("subtriangles", C.c_int64),
                ("caps", C.c_int64), ("n_deep", C.c_int64)]


PHASES = ("mlp", "pairs", "near", "segsum", "extract", "load")
MLP_WEIGHTS = 17795


_LIB = None
_HIP = None


def lib():
    """The loaded libnlasm.so; raises if it has not been built."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libnlasm.so is not built (run __graft_entry__.build()); no fallback exists")
        L = C.CDLL(LIB_PATH)
        P, I32, I64, D = C.c_void_p, C.c_int32, C.c_int64, C.c_double
        L.nla_last_error.restype = C.c_char_p
        L.nla_plan_create.argtypes = [P, P, P, C.POINTER(P)]
        L.nla_plan_info.argtypes = [P, P]
        L.nla_pairs_view.argtypes = [P, C.POINTER(P), C.POINTER(P)]
        L.nla_outer_points.argtypes = [P, P, P]
        L.nla_assemble.argtypes = [P, P, P, P]
        L.nla_csr_view.argtypes = [P, I32, C.POINTER(P), C.POINTER(P), C.POINTER(P), C.POINTER(I32)]
        L.nla_load_view.argtypes = [P, C.POINTER(P)]
        L.nla_free_nodes_view.argtypes = [P, C.POINTER(P)]
        L.nla_blocks_view.argtypes = [P, C.POINTER(P), C.POINTER(P), C.POINTER(P), C.POINTER(P),
                                      C.POINTER(P), C.POINTER(P), C.POINTER(I32)]
        L.nla_cg.argtypes = [P, P, P, D, I32, C.POINTER(I32), C.POINTER(D), P]
        L.nla_cg_noalloc.argtypes = [P, P, P, D, I32, C.POINTER(I32), C.POINTER(D), P]
        L.nla_near_view.argtypes = [P, C.POINTER(I64), C.POINTER(P), C.POINTER(P), C.POINTER(I32)]
        L.nla_batch_create.argtypes = [I32, P, P, P, C.POINTER(P)]
        L.nla_batch_assemble.argtypes = [P, I32, P, P, P]
        L.nla_batch_plan.argtypes = [P, I32, C.POINTER(P)]
        L.nla_batch_info.argtypes = [P, P]
        L.nla_batch_autotune.argtypes = [P, C.c_char_p, P]
        L.nla_batch_destroy.argtypes = [P]
        L.nla_batch_destroy.restype = None
        L.nla_set_timing.argtypes = [P, I32]
        L.nla_timings.argtypes = [P, P, C.POINTER(I32)]
        L.nla_plan_destroy.argtypes = [P]
        L.nla_plan_destroy.restype = None
        L.nla_mlp_create.argtypes = [C.c_uint64, C.POINTER(P)]
        L.nla_mlp_set_weights.argtypes = [P, P, C.c_float]
        L.nla_mlp_get_weights.argtypes = [P, P, C.POINTER(C.c_float)]
        L.nla_mlp_set_domain.argtypes = [P, P]
        L.nla_mlp_get_domain.argtypes = [P, P]
        L.nla_mlp_samples.argtypes = [I64, C.c_uint64, I64, D, D, D, I32, P, P, C.POINTER(I64), P]
        L.nla_mlp_train.argtypes = [P, P, P, I64, I32, I32, C.c_float, C.c_uint64, P, P]
        L.nla_mlp_forward.argtypes = [P, P, I64, P, P]
        L.nla_mlp_backward.argtypes = [P, P, P, I64, P, P]
        L.nla_mlp_save.argtypes = [P, C.c_char_p]
        L.nla_mlp_load.argtypes = [C.c_char_p, C.POINTER(P)]
        L.nla_mlp_destroy.argtypes = [P]
        L.nla_mlp_destroy.restype = None
        for name in ("nla_plan_create", "nla_plan_info", "nla_pairs_view", "nla_outer_points", "nla_assemble",
                     "nla_csr_view", "nla_load_view", "nla_free_nodes_view", "nla_blocks_view", "nla_cg", "nla_cg_noalloc",
                     "nla_set_timing", "nla_timings", "nla_near_view", "nla_batch_create",
                     "nla_batch_assemble", "nla_batch_plan", "nla_batch_info", "nla_batch_autotune",
                     "nla_mlp_create", "nla_mlp_set_weights", "nla_mlp_get_weights", "nla_mlp_samples",
                     "nla_mlp_train", "nla_mlp_forward", "nla_mlp_backward", "nla_mlp_save", "nla_mlp_load",
                     "nla_mlp_set_domain", "nla_mlp_get_domain"):
            getattr(L, name).restype = C.c_int
        _LIB = L
    return _LIB


def _hip():
    global _HIP
    if _HIP is None:
        _HIP = C.CDLL("libamdhip64.so.7")  # the runtime already loaded (by torch), matched by soname
        _HIP.hipMemcpyAsync.argtypes = [C.c_void_p, C.c_void_p, C.c_size_t, C.c_int, C.c_void_p]
        _HIP.hipMemcpyAsync.restype = C.c_int
    return _HIP


def _check(code):
    if code != NLA_OK:
        raise NlaError(code, lib().nla_last_error().decode())


def _stream(stream=None):
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


def _copy_from_device(ptr, count, dtype, stream=None):
    """A torch tensor holding a copy of `count` elements at device address ptr."""
    out = torch.empty(count, dtype=dtype, device="cuda")
    if count:
        st = _hip().hipMemcpyAsync(C.c_void_p(out.data_ptr()), C.c_void_p(ptr),
                                   count * out.element_size(), 3, _stream(stream))
        if st != 0:
            raise RuntimeError("hipMemcpyAsync failed (%d)" % st)
    return out


def _rule(r, keep):
    lam = np.ascontiguousarray(r.lam, dtype=np.float64)
    w = np.ascontiguousarray(r.w, dtype=np.float64)
    keep += [lam, w]
    return nla_rule(r.n, lam.ctypes.data, w.ctypes.data)


def marshal(mesh, prob, keep, mlp=None):
    """(nla_mesh, nla_problem) structs for a workloads mesh and problem; the
    numpy buffers they point to are appended to `keep` (and the network of a
    learned-caps problem, which must outlive the plan)."""
    from workloads.rules import get_rule, gauss_legendre01
    xy = np.ascontiguousarray(mesh.xy, dtype=np.float64)
    tri = np.ascontiguousarray(mesh.tri, dtype=np.int32)
    tin = np.ascontiguousarray(mesh.tri_in_omega, dtype=np.uint8)
    nfr = np.ascontiguousarray(mesh.node_free, dtype=np.uint8)
    keep += [xy, tri, tin, nfr]
    m = nla_mesh(xy.shape[0], tri.shape[0], xy.ctypes.data, tri.ctypes.data, tin.ctypes.data, nfr.ctypes.data)
    p = nla_problem()
    p.delta = prob.delta
    p.kernel = KERNELS[prob.kernel]
    p.kernel_c = prob.kernel_c
    p.kernel_s = prob.kernel_s
    p.outer = _rule(get_rule(prob.outer), keep)
    p.inner = _rule(get_rule(prob.inner), keep)
    if prob.duffy_order > 0:
        gx, gw = gauss_legendre01(prob.duffy_order)
        keep += [gx, gw]
        p.duffy_n, p.duffy_x, p.duffy_w = prob.duffy_order, gx.ctypes.data, gw.ctypes.data
    p.ball = BALLS[prob.ball]
    p.cap_mode = {"poly": 0, "centroid": 1, "analytic": 2}[prob.cap_mode]
    p.cap_edges = prob.cap_edges
    if prob.outer2:
        p.outer2 = _rule(get_rule(prob.outer2), keep)
        p.switch_dist = prob.switch_dist
    p.precision = PRECISIONS[prob.precision]
    p.fallback_band = prob.fallback_band
    p.flags = NLA_SKIP_IXI if prob.skip_ixi else 0
    if prob.precision == "learned":
        if mlp is None:
            raise ValueError("a learned-caps problem needs a network (mlp=Mlp(...))")
        p.mlp = mlp._h
        keep.append(mlp)
    return m, p


class nla_batch_summary(C.Structure):
    _fields_ = [("n", C.c_int32), ("total_pairs", C.c_int64), ("total_elements", C.c_int64),
                ("total_near", C.c_int64), ("chunk", C.c_int32), ("grid", C.c_int32)]


class Plan:
    """A plan for one mesh and problem (nla_plan_create ... nla_plan_destroy)."""

    def __init__(self, mesh, prob, stream=None, handle=None, mlp=None):
        self.mesh = mesh
        self.problem = prob
        self.K = mesh.n_triangles
        self.J = mesh.n_vertices
        from workloads.rules import get_rule
        self.outer_rule = get_rule(prob.outer)
        self._owned = handle is None
        if handle is not None:
            self._h = handle
            return
        keep = []
        m, p = marshal(mesh, prob, keep, mlp)
        self.mlp = mlp
        h = C.c_void_p()
        _check(lib().nla_plan_create(C.byref(m), C.byref(p), _stream(stream), C.byref(h)))
        self._h = h

    def close(self):
        if getattr(self, "_h", None) and getattr(self, "_owned", False):
            lib().nla_plan_destroy(self._h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def info(self):
        i = nla_info()
        _check(lib().nla_plan_info(self._h, C.byref(i)))
        return dict(n_pairs=i.n_pairs, nnz_full=i.nnz_full, nnz_free=i.nnz_free, n_free=i.n_free,
                    n_outer=i.n_outer, n_codes=i.n_codes, n_near=i.n_near,
                    items=dict(whole=i.items[0], partial=i.items[1], empty=i.items[2], learned=i.items[3]),
                    subtriangles=i.subtriangles, caps=i.caps, n_deep=i.n_deep)

    def set_timing(self, n):
        """Time the next n assemblies per phase (HIP events on their stream); 0 = off."""
        _check(lib().nla_set_timing(self._h, int(n)))

    def timings(self):
        """(mean milliseconds per phase, number of timed assemblies)."""
        ms = (C.c_double * len(PHASES))()
        n = C.c_int32()
        _check(lib().nla_timings(self._h, ms, C.byref(n)))
        return dict(zip(PHASES, list(ms))), n.value

    def pairs(self, stream=None):
        """(pair_ptr [K+1] int64, pair_kp [n_pairs] int32) as device tensors (copies)."""
        a, b = C.c_void_p(), C.c_void_p()
        _check(lib().nla_pairs_view(self._h, C.byref(a), C.byref(b)))
        n = self.info()["n_pairs"]
        return (_copy_from_device(a.value, self.K + 1, torch.int64, stream),
                _copy_from_device(b.value, n, torch.int32, stream))

    def outer_points(self, stream=None):
        xq = torch.empty((self.K, self.outer_rule.n, 2), dtype=torch.float64, device="cuda")
        _check(lib().nla_outer_points(self._h, C.c_void_p(xq.data_ptr()), _stream(stream)))
        return xq

    def assemble(self, f_outer=None, g_node=None, stream=None):
        fp = C.c_void_p(f_outer.data_ptr()) if f_outer is not None else None
        gp = C.c_void_p(g_node.data_ptr()) if g_node is not None else None
        if f_outer is not None:
            assert f_outer.dtype == torch.float64 and f_outer.is_cuda and f_outer.is_contiguous()
            assert f_outer.numel() == self.K * self.outer_rule.n
        if g_node is not None:
            assert g_node.dtype == torch.float64 and g_node.is_cuda and g_node.numel() == self.J
        _check(lib().nla_assemble(self._h, fp, gp, _stream(stream)))

    def csr(self, which=0, stream=None):
        """(rowptr, col, val) of D (which=0) or A (which=1) as device tensor copies."""
        rp, ci, v, dt = C.c_void_p(), C.c_void_p(), C.c_void_p(), C.c_int32()
        _check(lib().nla_csr_view(self._h, which, C.byref(rp), C.byref(ci), C.byref(v), C.byref(dt)))
        info = self.info()
        n = self.J if which == 0 else info["n_free"]
        nnz = info["nnz_full"] if which == 0 else info["nnz_free"]
        rowptr = _copy_from_device(rp.value, n + 1, torch.int64, stream)
        col = _copy_from_device(ci.value, nnz, torch.int32, stream)
        val = _copy_from_device(v.value, nnz, torch.float64 if dt.value == 0 else torch.float32, stream)
        return rowptr, col, val

    def load(self, stream=None):
        b = C.c_void_p()
        _check(lib().nla_load_view(self._h, C.byref(b)))
        return _copy_from_device(b.value, self.info()["n_free"], torch.float64, stream)

    def free_nodes(self, stream=None):
        f = C.c_void_p()
        _check(lib().nla_free_nodes_view(self._h, C.byref(f)))
        return _copy_from_device(f.value, self.info()["n_free"], torch.int32, stream)

    def blocks(self, stream=None):
        """Intermediate blocks (copies): Myy [P,6], Mxx [K,6], element blocks [K,6],
        row blocks R (flat), col_off [K+1], colset."""
        a, b, c, d, e, f, dt = (C.c_void_p(), C.c_void_p(), C.c_void_p(), C.c_void_p(), C.c_void_p(),
                                C.c_void_p(), C.c_int32())
        _check(lib().nla_blocks_view(self._h, C.byref(a), C.byref(b), C.byref(c), C.byref(d), C.byref(e),
                                     C.byref(f), C.byref(dt)))
        n = self.info()["n_pairs"]
        t = torch.float64 if dt.value == 0 else torch.float32
        col_off = _copy_from_device(e.value, self.K + 1, torch.int64, stream)
        ncols = int(col_off[-1].item())
        return dict(myy=_copy_from_device(a.value, 6 * n, t, stream).view(n, 6),
                    mxx=_copy_from_device(b.value, 6 * self.K, t, stream).view(self.K, 6),
                    elem=_copy_from_device(c.value, 6 * self.K, t, stream).view(self.K, 6),
                    rows=_copy_from_device(d.value, 3 * ncols, t, stream),
                    col_off=col_off, colset=_copy_from_device(f.value, ncols, torch.int32, stream))

    def near(self, stream=None):
        """(near pair indices [n], merged blocks [n, 21]) of the singular-kernel pairs (copies)."""
        n, a, b, dt = C.c_int64(), C.c_void_p(), C.c_void_p(), C.c_int32()
        _check(lib().nla_near_view(self._h, C.byref(n), C.byref(a), C.byref(b), C.byref(dt)))
        t = torch.float64 if dt.value == 0 else torch.float32
        return (_copy_from_device(a.value, n.value, torch.int64, stream),
                _copy_from_device(b.value, 21 * n.value, t, stream).view(-1, 21))

    def cg(self, b, u0=None, rtol=1e-12, maxit=10000, stream=None, noalloc=False):
        """noalloc: nla_cg_noalloc (scratch in the library's device array)."""
        n = self.info()["n_free"]
        u = torch.zeros(n, dtype=torch.float64, device="cuda") if u0 is None else u0.clone()
        it, rr = C.c_int32(), C.c_double()
        fn = lib().nla_cg_noalloc if noalloc else lib().nla_cg
        code = fn(self._h, C.c_void_p(b.data_ptr()), C.c_void_p(u.data_ptr()), rtol, maxit,
                  C.byref(it), C.byref(rr), _stream(stream))
        _check(code)
        return u, it.value, rr.value


class Batch:
    """Many instances assembled together (nla_batch_*)."""

    def __init__(self, instances, stream=None):
        keep = []
        ms = (nla_mesh * len(instances))()
        ps = (nla_problem * len(instances))()
        for i, (mesh, prob) in enumerate(instances):
            ms[i], ps[i] = marshal(mesh, prob, keep)
        h = C.c_void_p()
        _check(lib().nla_batch_create(len(instances), ms, ps, _stream(stream), C.byref(h)))
        self._h = h
        self.instances = instances
        self.plans = []
        for i, (mesh, prob) in enumerate(instances):
            ph = C.c_void_p()
            _check(lib().nla_batch_plan(self._h, i, C.byref(ph)))
            self.plans.append(Plan(mesh, prob, handle=ph))

    def assemble(self, mode=1, f_outer=None, g_node=None, stream=None):
        n = len(self.instances)
        if f_outer is not None:
            fa = (C.c_void_p * n)(*[t.data_ptr() for t in f_outer])
            ga = (C.c_void_p * n)(*[t.data_ptr() for t in g_node])
        else:
            fa = ga = None
        _check(lib().nla_batch_assemble(self._h, mode, fa, ga, _stream(stream)))

    def info(self):
        i = nla_batch_summary()
        _check(lib().nla_batch_info(self._h, C.byref(i)))
        return dict(n=i.n, total_pairs=i.total_pairs, total_elements=i.total_elements, total_near=i.total_near,
                    chunk=i.chunk, grid=i.grid)

    def autotune(self, cache_path=None, stream=None):
        _check(lib().nla_batch_autotune(self._h, cache_path.encode() if cache_path else None, _stream(stream)))
        return self.info()

    def close(self):
        for p in self.plans:
            p._h = None
        if getattr(self, "_h", None):
            lib().nla_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Mlp:
    """The learned cap corrector's network (nla_mlp_*): weights on the GPU,
    training and inference in the library's kernels."""

    def __init__(self, seed=0, handle=None):
        if handle is None:
            h = C.c_void_p()
            _check(lib().nla_mlp_create(C.c_uint64(seed), C.byref(h)))
            handle = h
        self._h = handle

    @classmethod
    def load(cls, path):
        h = C.c_void_p()
        _check(lib().nla_mlp_load(path.encode(), C.byref(h)))
        return cls(handle=h)

    def save(self, path):
        _check(lib().nla_mlp_save(self._h, path.encode()))

    def close(self):
        if getattr(self, "_h", None):
            lib().nla_mlp_destroy(self._h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_weights(self, w, scale):
        w = np.ascontiguousarray(w, dtype=np.float32)
        assert w.shape == (MLP_WEIGHTS,)
        _check(lib().nla_mlp_set_weights(self._h, w.ctypes.data, C.c_float(scale)))

    def get_weights(self):
        w = np.empty(MLP_WEIGHTS, dtype=np.float32)
        sc = C.c_float()
        _check(lib().nla_mlp_get_weights(self._h, w.ctypes.data, C.byref(sc)))
        return w, sc.value

    def set_domain(self, dom):
        """The training domain {rlo, rhi, elo, ehi} (None: unbounded)."""
        if dom is None:
            _check(lib().nla_mlp_set_domain(self._h, None))
            return
        d = np.ascontiguousarray(dom, dtype=np.float64)
        assert d.shape == (4,)
        _check(lib().nla_mlp_set_domain(self._h, d.ctypes.data))

    def get_domain(self):
        d = np.empty(4, dtype=np.float64)
        _check(lib().nla_mlp_get_domain(self._h, d.ctypes.data))
        return d

    @staticmethod
    def samples(n_cand, seed, first=0, L=0.125, jitter=0.1, band=0.02, cap_edges=8, stream=None):
        """Kept training samples (feat [n][6], label [n][3] float32 device tensors)."""
        feat = torch.empty((max(n_cand, 1), 6), dtype=torch.float32, device="cuda")
        lab = torch.empty((max(n_cand, 1), 3), dtype=torch.float32, device="cuda")
        nv = C.c_int64()
        _check(lib().nla_mlp_samples(n_cand, C.c_uint64(seed), first, L, jitter, band, cap_edges,
                                     C.c_void_p(feat.data_ptr()), C.c_void_p(lab.data_ptr()), C.byref(nv),
                                     _stream(stream)))
        return feat[:nv.value], lab[:nv.value]

    def train(self, feat, label, epochs, batch=4096, lr=1e-3, seed=0, stream=None):
        """Mean loss per epoch (list)."""
        assert feat.is_contiguous() and label.is_contiguous() and feat.dtype == torch.float32
        log = (C.c_float * epochs)()
        _check(lib().nla_mlp_train(self._h, C.c_void_p(feat.data_ptr()), C.c_void_p(label.data_ptr()),
                                   feat.shape[0], epochs, batch, C.c_float(lr), C.c_uint64(seed), log,
                                   _stream(stream)))
        return list(log)

    def forward(self, feat, stream=None):
        feat = feat.contiguous()
        out = torch.empty((feat.shape[0], 3), dtype=torch.float32, device="cuda")
        _check(lib().nla_mlp_forward(self._h, C.c_void_p(feat.data_ptr()), feat.shape[0],
                                     C.c_void_p(out.data_ptr()), _stream(stream)))
        return out

    def backward(self, feat, dout, stream=None):
        feat, dout = feat.contiguous(), dout.contiguous()
        dw = torch.empty(MLP_WEIGHTS, dtype=torch.float32, device="cuda")
        _check(lib().nla_mlp_backward(self._h, C.c_void_p(feat.data_ptr()), C.c_void_p(dout.data_ptr()),
                                      feat.shape[0], C.c_void_p(dw.data_ptr()), _stream(stream)))
        return dw
