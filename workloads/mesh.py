"""Structured triangulations of Omega=(0,1)^2 plus its interaction layer.

The mesh follows the paper's grid rules (Sec. 3.1): Omega and the layer
Omega_I = (-delta, 1+delta)^2 minus Omega are triangulated separately with
matching vertices on the boundary of Omega and a vertex at every corner, the
layer's rounded corners squared off.  Cells of side h are split along the
"/" diagonal into (SW, SE, NE) and (SW, NE, NW), both counter-clockwise
(the uniform grid of type (a) in Sec. 8).  Nodes on the boundary of Omega
belong to Omega_I (Sec. 3.1), so only nodes strictly inside Omega are free.
"""
from dataclasses import dataclass, field
import numpy as np

_MASK = (1 << 64) - 1


def splitmix64_uniform(seed, n):
    """n doubles in [0,1) from SplitMix64 (Steele, Lea, Flood 2014), taking the
    top 53 bits of each output: u = (z >> 11) * 2^-53."""
    out = np.empty(n, dtype=np.float64)
    s = seed & _MASK
    for i in range(n):
        s = (s + 0x9E3779B97F4A7C15) & _MASK
        z = s
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _MASK
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _MASK
        z = z ^ (z >> 31)
        out[i] = (z >> 11) * (1.0 / 9007199254740992.0)
    return out


@dataclass
class Mesh:
    xy: np.ndarray            # [J,2] float64
    tri: np.ndarray           # [K,3] int32, counter-clockwise
    tri_in_omega: np.ndarray  # [K] uint8 (1 = element of Omega)
    node_free: np.ndarray     # [J] uint8 (1 = node in the open Omega)
    delta: float
    h: float
    n_layer: int
    n_omega: int
    meta: dict = field(default_factory=dict)

    @property
    def n_vertices(self):
        return self.xy.shape[0]

    @property
    def n_triangles(self):
        return self.tri.shape[0]

    @property
    def n_free(self):
        return int(self.node_free.sum())


def structured_mesh(delta, h, jitter=0.0, seed=20050, grid="a", diagonal="/"):
    """Uniform mesh with cells of side h = 1/n_omega and a layer of
    n_layer = delta/h cells.  Vertex (i, j) sits at ((i-n_layer)/n_omega,
    (j-n_layer)/n_omega), so the boundary of Omega lies exactly on 0 and 1.

    jitter > 0 moves every vertex strictly inside Omega by independent
    uniform offsets in (-jitter*h, jitter*h) per coordinate (SplitMix64 from
    ``seed``, x then y per vertex in index order); boundary and layer
    vertices stay fixed, which keeps the interface and the corners.
    grid="b" is the non-uniform Cartesian grid (b) of Sec. 8.2: every grid
    line x2 = c with 0 < c < 1 moves to x2 = c^2, across the whole width, so
    that the grid stays a tensor product (mapping only the vertices inside
    Omega would kink each line at x1 = 0 and 1 and leave elements there of
    diameter near 1/4, against the printed h_max).
    diagonal: "/" splits each cell along sw-ne, "\\" along se-nw.
    """
    n_omega = int(round(1.0 / h))
    n_layer = int(round(delta / h))
    if abs(n_omega * h - 1.0) > 1e-9 or abs(n_layer * h - delta) > 1e-9 * max(1.0, delta):
        raise ValueError("h must divide 1 and delta")
    n = n_omega + 2 * n_layer
    ii, jj = np.meshgrid(np.arange(n + 1), np.arange(n + 1), indexing="xy")
    ii = ii.ravel()
    jj = jj.ravel()
    x = (ii - n_layer).astype(np.float64) / float(n_omega)
    y = (jj - n_layer).astype(np.float64) / float(n_omega)
    free = ((ii > n_layer) & (ii < n_layer + n_omega) &
            (jj > n_layer) & (jj < n_layer + n_omega))
    if grid == "b":
        y = np.where((y > 0.0) & (y < 1.0), y * y, y)
    elif grid != "a":
        raise ValueError("grid must be 'a' or 'b'")
    if jitter > 0.0:
        idx = np.nonzero(free)[0]
        u = splitmix64_uniform(seed, 2 * len(idx))
        x[idx] += (2.0 * u[0::2] - 1.0) * (jitter * h)
        y[idx] += (2.0 * u[1::2] - 1.0) * (jitter * h)
    xy = np.stack([x, y], axis=1)

    def vid(i, j):
        return j * (n + 1) + i

    ci, cj = np.meshgrid(np.arange(n), np.arange(n), indexing="xy")
    ci = ci.ravel()
    cj = cj.ravel()
    sw, se, ne, nw = vid(ci, cj), vid(ci + 1, cj), vid(ci + 1, cj + 1), vid(ci, cj + 1)
    if diagonal == "/":
        t1 = np.stack([sw, se, ne], axis=1)
        t2 = np.stack([sw, ne, nw], axis=1)
    elif diagonal == "\\":
        t1 = np.stack([sw, se, nw], axis=1)
        t2 = np.stack([se, ne, nw], axis=1)
    else:
        raise ValueError("diagonal must be '/' or '\\\\'")
    tri = np.empty((2 * n * n, 3), dtype=np.int32)
    tri[0::2] = t1
    tri[1::2] = t2
    cin = ((ci >= n_layer) & (ci < n_layer + n_omega) &
           (cj >= n_layer) & (cj < n_layer + n_omega))
    tin = np.repeat(cin, 2).astype(np.uint8)
    return Mesh(xy=np.ascontiguousarray(xy), tri=tri, tri_in_omega=tin,
                node_free=free.astype(np.uint8), delta=float(n_layer) / n_omega,
                h=1.0 / n_omega, n_layer=n_layer, n_omega=n_omega,
                meta={"jitter": jitter, "seed": seed, "grid": grid, "diagonal": diagonal})
