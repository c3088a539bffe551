"""Writes rules.json: triangle quadrature tables as hex floats.

Run once (``python -m workloads.make_rules``); both the oracle and the GPU
path read the committed table so their points agree bit for bit.

Every rule is given in barycentric form (lambda0, lambda1, lambda2) on the
reference triangle (0,0),(1,0),(0,1); weights sum to 1/2 (its area).

* dunavant7  - 7-point degree-5 rule (Radon's rule as tabulated by Dunavant).
* dunavant16 - 16-point degree-8 rule; orbit structure 1 + 3 x S21 + 1 x S111.
  Published 15-digit values seed a Newton solve of the degree <= 8 moment
  equations in extended precision, so the stored doubles are the correctly
  rounded solution rather than a 15-digit transcription.
* vertex7    - 7-point degree-3 rule on centroid, vertices and mid-sides with
  weights 27/60, 3/60, 8/60 (x 1/2); the paper's outer rule of choice in its
  final word on the outer integral (Sec. 6).
* gauss3     - 3-point degree-2 interior rule (2/3,1/6,1/6); the paper's inner
  rule (Sec. 5.3.1).
* strang4    - 4-point degree-3 rule with negative centroid weight; the
  paper's Case-1 outer rule (Sec. 6.1).
* centroid1  - 1-point degree-1 rule.
The 1D Gauss-Legendre tables on [0,1] (orders 1..40) serve the singular
near-diagonal (Duffy) quadrature.
"""
import itertools, json, math, os
import numpy as np

LD = np.longdouble


def _orbit_points(spec):
    pts, ws = [], []
    for kind, args, w in spec:
        if kind == "S3":
            cand = [(LD(1) / 3, LD(1) / 3, LD(1) / 3)]
        elif kind == "S21":
            a = args[0]
            cand = [(a, a, 1 - 2 * a), (a, 1 - 2 * a, a), (1 - 2 * a, a, a)]
        else:
            b, c = args
            d = 1 - b - c
            cand = list(dict.fromkeys(itertools.permutations((b, c, d))))
        for p in cand:
            pts.append(p)
            ws.append(w)
    return pts, ws


def _exact(a, b):
    return LD(math.factorial(a) * math.factorial(b)) / LD(math.factorial(a + b + 2))


def _newton16():
    # parameters: w0, (a1,w1), (a2,w2), (a3,w3), (b,c,w4); weights on area-1/2 triangle
    p = np.array([0.144315607677787 / 2, 0.459292588292723, 0.095091634267285 / 2,
                  0.170569307751760, 0.103217370534718 / 2, 0.050547228317031,
                  0.032458497623198 / 2, 0.008394777409958, 0.263112829634638,
                  0.027230314174435 / 2], dtype=LD)
    mons = [(a, d - a) for d in range(9) for a in range(d + 1)]

    def spec(p):
        return [("S3", (), p[0]), ("S21", (p[1],), p[2]), ("S21", (p[3],), p[4]),
                ("S21", (p[5],), p[6]), ("S111", (p[7], p[8]), p[9])]

    def res(p):
        pts, ws = _orbit_points(spec(p))
        out = []
        for a, b in mons:
            s = sum(w * q[1] ** a * q[2] ** b for q, w in zip(pts, ws))
            out.append((s - _exact(a, b)) / _exact(a, b))
        return np.array(out, dtype=LD)

    for _ in range(12):
        r = res(p)
        J = np.zeros((len(r), len(p)), dtype=LD)
        for i in range(len(p)):
            e = np.zeros(len(p), dtype=LD)
            e[i] = LD(1e-9)
            J[:, i] = (res(p + e) - res(p - e)) / LD(2e-9)
        dp = np.linalg.lstsq(J.astype(np.float64), -r.astype(np.float64), rcond=None)[0]
        p = p + dp.astype(LD)
    return spec(p)


def _as_table(spec, degree, name, note):
    pts, ws = _orbit_points(spec)
    lam = []
    for q in pts:
        l1, l2 = float(q[1]), float(q[2])
        l0 = float(LD(1) - LD(l1) - LD(l2))
        lam.append([l0.hex(), l1.hex(), l2.hex()])
    return {"name": name, "degree": degree, "note": note,
            "lam": lam, "w": [float(w).hex() for w in ws]}


def build():
    r15 = LD(15).__pow__(LD(0.5))
    third = LD(1) / 3
    half = LD(1) / 2
    rules = {}
    rules["dunavant7"] = _as_table(
        [("S3", (), LD(9) / 40 / 2),
         ("S21", ((6 - r15) / 21,), (155 - r15) / 1200 / 2),
         ("S21", ((6 + r15) / 21,), (155 + r15) / 1200 / 2)], 5, "dunavant7",
        "7-point degree-5 interior rule")
    rules["dunavant16"] = _as_table(_newton16(), 8, "dunavant16",
                                    "16-point degree-8 interior rule")
    v7 = [("S3", (), LD(27) / 60 / 2)]
    pts = [((LD(1), LD(0), LD(0)), LD(3) / 60 / 2), ((LD(0), LD(1), LD(0)), LD(3) / 60 / 2),
           ((LD(0), LD(0), LD(1)), LD(3) / 60 / 2), ((half, half, LD(0)), LD(8) / 60 / 2),
           ((LD(0), half, half), LD(8) / 60 / 2), ((half, LD(0), half), LD(8) / 60 / 2)]
    t = _as_table(v7, 3, "vertex7", "7-point degree-3 rule: centroid, vertices, mid-sides")
    for q, w in pts:
        t["lam"].append([float(q[0]).hex(), float(q[1]).hex(), float(q[2]).hex()])
        t["w"].append(float(w).hex())
    rules["vertex7"] = t
    rules["gauss3"] = _as_table([("S21", (LD(1) / 6,), LD(1) / 6)], 2, "gauss3",
                                "3-point degree-2 interior rule")
    rules["strang4"] = _as_table([("S3", (), LD(-27) / 48 / 2), ("S21", (LD(1) / 5,), LD(25) / 48 / 2)],
                                 3, "strang4", "4-point degree-3 rule, negative centroid weight")
    rules["centroid1"] = _as_table([("S3", (), half)], 1, "centroid1", "1-point centroid rule")
    gl = {}
    for n in range(1, 41):
        x, w = np.polynomial.legendre.leggauss(n)
        gl[str(n)] = {"x": [float((xi + 1) / 2).hex() for xi in x],
                      "w": [float(wi / 2).hex() for wi in w]}
    return {"triangle": rules, "gauss_legendre_01": gl}


if __name__ == "__main__":
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "rules.json")
    with open(out, "w") as f:
        json.dump(build(), f, indent=1)
    print("wrote", out)
