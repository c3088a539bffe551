"""Loader for the committed quadrature tables (see make_rules.py)."""
from dataclasses import dataclass
import json, os
import numpy as np

_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "rules.json")
_CACHE = {}


@dataclass
class Rule:
    name: str
    degree: int
    lam: np.ndarray   # [n,3] barycentric coordinates
    w: np.ndarray     # [n] weights, sum 1/2

    @property
    def n(self):
        return self.w.shape[0]


def _load():
    if not _CACHE:
        with open(_PATH) as f:
            _CACHE.update(json.load(f))
    return _CACHE


def get_rule(name):
    t = _load()["triangle"][name]
    lam = np.array([[float.fromhex(v) for v in row] for row in t["lam"]], dtype=np.float64)
    w = np.array([float.fromhex(v) for v in t["w"]], dtype=np.float64)
    return Rule(name=name, degree=int(t["degree"]), lam=np.ascontiguousarray(lam), w=w)


def gauss_legendre01(n):
    t = _load()["gauss_legendre_01"][str(n)]
    return (np.array([float.fromhex(v) for v in t["x"]]),
            np.array([float.fromhex(v) for v in t["w"]]))


RULE_NAMES = ("dunavant7", "dunavant16", "vertex7", "gauss3", "strang4", "centroid1")
