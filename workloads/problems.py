"""Problem descriptions and the synthetic workloads the method is run on.

Kernel functions (Sec. 2.1, Eq. (inter)): gamma(x,y) = psi(x,y) * chi_{B_delta(x)}(y).
* constant: psi = 4/(pi delta^4) (Sec. 8), which makes the operator of
  Eq. (oper) reproduce the Laplacian on cubic polynomials;
* fractional (truncated): psi = c_s |x-y|^-(2+2s), with
  c_s = 2(1-s)/(pi delta^(2-2s)) chosen so that -L u = -4 for u = |x|^2 under
  the 2*int (u(x)-u(y)) gamma convention; c_s reduces to 4/(pi delta^4) at s=-1.
"""
from dataclasses import dataclass, replace, asdict
import math
import numpy as np
from .mesh import structured_mesh, splitmix64_uniform


def constant_kernel_c(delta):
    return 4.0 / (math.pi * delta ** 4)


def fractional_kernel_c(delta, s):
    return 2.0 * (1.0 - s) / (math.pi * delta ** (2.0 - 2.0 * s))


@dataclass
class Problem:
    delta: float
    kernel: str = "constant"          # "constant" | "fractional"
    kernel_c: float = 0.0
    kernel_s: float = 0.0
    ball: str = "barycenter"          # "barycenter" | "retri" | "overlap" | "shifted" | "barysupport"
    cap_mode: str = "poly"            # "poly": caps by cap_edges equal arcs ; "centroid": exact caps, 1-pt rule ;
                                      # "analytic": exact caps in closed form (constant kernel)
    cap_edges: int = 0                # 0 = the paper's nocaps polygon
    outer: str = "dunavant7"
    inner: str = "dunavant16"
    outer2: str = ""                  # optional second outer rule ...
    switch_dist: float = 0.0          # ... used for pairs with |b_k - b_k'| < switch_dist
    precision: str = "fp64"           # "fp64" | "fp32" | "learned"
    duffy_order: int = 0              # Gauss-Legendre order per axis for vertex-sharing pairs (fractional kernel)
    skip_ixi: bool = False            # drop Omega_I x Omega_I pairs (changes neither A nor b)
    fallback_band: float = 0.02       # learned caps: exact-cap fallback band, units of delta

    def as_dict(self):
        return asdict(self)


def manufactured(name):
    """(u, f) pairs: 'quadratic' u = x1^2 + x2^2, f = -4 ; 'paper' u = x1^2 x2 + x2^2,
    f = -2(x2+1) (Sec. 8)."""
    if name == "quadratic":
        return (lambda x, y: x * x + y * y), (lambda x, y: -4.0 + 0.0 * x)
    if name == "paper":
        return (lambda x, y: x * x * y + y * y), (lambda x, y: -2.0 * (y + 1.0))
    raise KeyError(name)


def paper_workload(h, ball, delta=0.1, grid="a"):
    """The workloads of Sec. 8 on grid (a) (or grid (b), the interior vertices
    mapped by (x1, x2) -> (x1, x2^2)) with spacing h, delta = 0.1, the constant
    kernel, u = x1^2 x2 + x2^2 with f = -2(x2 + 1), and the 3-point inner rule.
    Experiments (1)-(5) use the 7-point vertex/mid-side/centroid outer rule,
    switched to the 4-point rule for pairs with |b_k - b_k'| < delta - h_max
    (h_max = sqrt(2) h, the element diameter; no pair when h_max >= delta),
    with the balls "exactcaps"
    (one-point centroid rule on the true caps), "approxcaps" (one triangle per
    cap: two arcs fanned from the chord midpoint), "nocaps", "barycenter" and
    "overlap"; and "analyticcaps", the exact ball (caps integrated in closed
    form), which the paper recommends but does not run.  Experiments (6)-(10) use the 4-point outer rule throughout:
    "shifted" (the nocaps ball about b_k) and "barynocaps" / "baryapproxcaps"
    (barycenter ball with the outer integral over E_k n B_delta(b_k'),
    approximated by nocaps / approxcaps)."""
    first = {"approxcaps": dict(ball="retri", cap_edges=2), "nocaps": dict(ball="retri", cap_edges=0),
             "exactcaps": dict(ball="retri", cap_mode="centroid"), "barycenter": dict(ball="barycenter"),
             "analyticcaps": dict(ball="retri", cap_mode="analytic"),
             "overlap": dict(ball="overlap")}
    second = {"shifted": dict(ball="shifted", cap_edges=0), "barynocaps": dict(ball="barysupport", cap_edges=0),
              "baryapproxcaps": dict(ball="barysupport", cap_edges=2)}
    if ball in first:
        p = Problem(delta=delta, kernel_c=constant_kernel_c(delta), outer="vertex7", inner="gauss3",
                    outer2="strang4", switch_dist=max(0.0, delta - math.sqrt(2) * h), **first[ball])
    else:
        p = Problem(delta=delta, kernel_c=constant_kernel_c(delta), outer="strang4", inner="gauss3",
                    **second[ball])
    return structured_mesh(delta, h, grid=grid), p, "paper"


def _c1():
    d = 0.1
    p = Problem(delta=d, kernel="constant", kernel_c=constant_kernel_c(d), ball="barycenter",
                outer="dunavant7", inner="dunavant7")
    return structured_mesh(d, 0.05), p, "quadratic"


def _c2():
    d = 0.1
    p = Problem(delta=d, kernel="constant", kernel_c=constant_kernel_c(d), ball="retri",
                cap_edges=8, outer="dunavant7", inner="dunavant16")
    return structured_mesh(d, d / 8, jitter=0.1, seed=20050), p, "quadratic"


def _c3():
    d, s = 0.05, 0.4
    p = Problem(delta=d, kernel="fractional", kernel_c=fractional_kernel_c(d, s), kernel_s=s,
                ball="retri", cap_edges=8, outer="dunavant7", inner="dunavant16",
                precision="fp32", duffy_order=8)
    return structured_mesh(d, d / 4), p, "quadratic"


def _c5():
    m, p, u = _c2()
    return m, replace(p, precision="learned"), u


CONFIGS = {"c1": _c1, "c2": _c2, "c3": _c3, "c5": _c5}


def make_config(name):
    """(mesh, problem, manufactured-solution name) of a named workload."""
    return CONFIGS[name]()


def batch_instances(n=64, seed=20051):
    """The uneven batch: delta ~ U[0.05, 0.2], k ~ U{2..8}, snapped to
    n_omega = round(k/delta), h = 1/n_omega, delta := k h so that the layer is
    meshed exactly.  Even instances use the constant kernel, odd ones the
    fractional s = 0.4 kernel; i mod 4 in {0,1} barycenter 7x7, {2,3} retri with
    8-arc caps 7x16; all FP32 with compensated accumulation."""
    u = splitmix64_uniform(seed, 2 * n)
    out = []
    for i in range(n):
        d0 = 0.05 + 0.15 * u[2 * i]
        k = 2 + min(6, int(u[2 * i + 1] * 7))
        n_om = int(round(k / d0))
        h = 1.0 / n_om
        d = k * h
        if i % 2 == 0:
            kern = dict(kernel="constant", kernel_c=constant_kernel_c(d))
        else:
            kern = dict(kernel="fractional", kernel_c=fractional_kernel_c(d, 0.4), kernel_s=0.4,
                        duffy_order=8)
        if i % 4 in (0, 1):
            ball = dict(ball="barycenter", outer="dunavant7", inner="dunavant7")
        else:
            ball = dict(ball="retri", cap_edges=8, outer="dunavant7", inner="dunavant16")
        p = Problem(delta=d, precision="fp32", **kern, **ball)
        out.append((structured_mesh(d, h), p))
    return out
