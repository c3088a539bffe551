// Device helpers shared by the numeric kernels: inner-rule moments, the P1
// basis of the inner element, subtriangle quadrature and the retriangulation
// of E' n B_delta(x).
#pragma once
#include "nla_internal.hpp"

// inner-rule moments as the kernels use them; sym = the rule is invariant
// under permutations of the barycentric coordinates, so sum_q w mu_i = m1c and
// sum_q w mu_i mu_j = o + dm [i == j]
struct RuleMom {
    double wsum, m1[3], m2[3][3];
    double m1c, o, dm;
};

__device__ __forceinline__ RuleMom load_moments(const RuleSet *__restrict__ R)
{
    RuleMom M;
    M.wsum = R->in_wsum;
#pragma unroll
    for (int i = 0; i < 3; i++) {
        M.m1[i] = R->in_m1[i];
#pragma unroll
        for (int j = 0; j < 3; j++) M.m2[i][j] = R->in_m2[i][j];
    }
    M.m1c = R->in_m1[0];
    M.o = R->in_m2[0][1];
    M.dm = R->in_m2[0][0] - R->in_m2[0][1];
    return M;
}

// geometric inner sums of one (x, E') item with psi = 1 (psi is constant and
// applied per pair): a2 = sum of twice-areas, s1_b ~ int beta_b (times m1c
// in the symmetric case), s2 = int beta_b beta_b' (upper triangle 00,01,02,11,12,22)
struct Acc {
    double a2;
    double s1[3];
    double s2[6];
};

// P1 basis of E' in coordinates relative to the outer point: beta1, beta2 from
// the offset to vertex 0 and the inverse of the edge matrix, beta0 = 1 - beta1 - beta2.
struct Basis {
    double x0, y0, i11, i12, i21, i22;
};

__device__ __forceinline__ void basis_at(const Basis &B, double px, double py, double &b0, double &b1, double &b2)
{
    double dx = px - B.x0, dy = py - B.y0;
    b1 = dx * B.i11 + dy * B.i12;
    b2 = dx * B.i21 + dy * B.i22;
    b0 = 1.0 - b1 - b2;
}

// the inner rule on the subtriangle with vertices t[i] = (x, y, beta0, beta1, beta2),
// evaluated from the basis values at its vertices: sum_q w_q beta(y_q) =
// sum_i m1_i beta(t_i) and sum_q w_q beta beta^T = B^T M2 B (B = vertex values);
// for a symmetric rule B^T M2 B = o cs cs^T + dm B^T B, cs = column sums of B
template <bool SYM>
__device__ __forceinline__ void tri_accum(const double (&t)[3][5], const RuleMom &M, Acc &A)
{
    const double a2 = fabs((t[1][0] - t[0][0]) * (t[2][1] - t[0][1]) - (t[1][1] - t[0][1]) * (t[2][0] - t[0][0]));
    A.a2 += a2;
    const int jj[6] = {0, 0, 0, 1, 1, 2}, ll[6] = {0, 1, 2, 1, 2, 2};
    if (SYM) {
        double cs[3];
#pragma unroll
        for (int l = 0; l < 3; l++) {
            cs[l] = t[0][2 + l] + t[1][2 + l] + t[2][2 + l];
            A.s1[l] += a2 * cs[l];
        }
        const double w = a2 * M.o, v = a2 * M.dm;
#pragma unroll
        for (int e = 0; e < 6; e++) {
            const int j = jj[e], l = ll[e];
            double q = t[0][2 + j] * t[0][2 + l] + t[1][2 + j] * t[1][2 + l] + t[2][2 + j] * t[2][2 + l];
            A.s2[e] += w * (cs[j] * cs[l]) + v * q;
        }
    } else {
        double U[3][3];
#pragma unroll
        for (int l = 0; l < 3; l++) {
            A.s1[l] += a2 * (M.m1[0] * t[0][2 + l] + M.m1[1] * t[1][2 + l] + M.m1[2] * t[2][2 + l]);
#pragma unroll
            for (int i = 0; i < 3; i++)
                U[i][l] = M.m2[i][0] * t[0][2 + l] + M.m2[i][1] * t[1][2 + l] + M.m2[i][2] * t[2][2 + l];
        }
#pragma unroll
        for (int e = 0; e < 6; e++) {
            const int j = jj[e], l = ll[e];
            A.s2[e] += a2 * (t[0][2 + j] * U[0][l] + t[1][2 + j] * U[1][l] + t[2][2 + j] * U[2][l]);
        }
    }
}

__device__ __forceinline__ void set5(double (&d)[5], double x, double y, double b0, double b1, double b2)
{
    d[0] = x; d[1] = y; d[2] = b0; d[3] = b1; d[4] = b2;
}

// Edge a->b of E' relative to the outer point (start p, direction e): whether
// p lies in the closed ball |z| <= delta, and the roots lambda in (0,1) of
// |p + lambda e|^2 = delta^2 (entry el1 < exit el2; 2 when absent).  Every
// product and sum is rounded on its own, so that vertices exactly on the circle
// (uniform grids put many there) are decided as the pair predicate and the
// oracle decide them.  iLp: 1 / |e|^2 when the caller has it (else <= 0).
__device__ __forceinline__ bool edge_roots(double epx, double epy, double eex, double eey, double dd, double &el1,
                                           double &el2, double iLp = 0.0)
{
#pragma clang fp contract(off)
    const double r2 = epx * epx + epy * epy;
    const double L = eex * eex + eey * eey;
    const double Bq = eex * epx + eey * epy;
    const double disc = Bq * Bq - L * (r2 - dd);
    el1 = 2.0;
    el2 = 2.0;
    if (disc > 0.0) {
        // the roots n / L; whether the rounded quotient lies in (0, 1) is decided
        // without dividing: fl(n/L) > 0 iff n > 0, and fl(n/L) < 1 iff
        // n/L < 1 - 2^-54 (the midpoint rounds to 1) iff n - L < -L 2^-54, where
        // n - L is exact whenever n is within a factor two of L (Sterbenz) and
        // its sign settles the test otherwise.  The root's value decides nothing.
        const double sq = sqrt(disc);
        const double n1 = -Bq - sq, n2 = -Bq + sq, tiny = L * 0x1p-54;
        const bool in1 = n1 > 0.0 && n1 - L < -tiny, in2 = n2 > 0.0 && n2 - L < -tiny;
        if (in1 || in2) {
            const double iL = iLp > 0.0 ? iLp : 1.0 / L;
            if (in1) el1 = n1 * iL;
            if (in2) el2 = n2 * iL;
        }
    }
    return r2 <= dd;
}

// E' n B_delta(x) retriangulated (Sec. 4.2.1-4.2.2 and Sec. 7.1 tasks 3-6) in
// two loops, each with one inlined copy of the subtriangle quadrature tri(t):
//  1. the edges are walked v0->v1->v2: vertices inside the closed ball and the
//     roots lambda in (0,1) of |v_a + lambda e - x|^2 = delta^2 (smaller root
//     entry, larger exit) arrive in order; every new point closes the fan
//     triangle (first, previous, new); every exit followed by an entry
//     (cyclically) is a cap, recorded in cb (at most three: one per exit);
//  2. each cap, the arc from exit X counter-clockwise to entry N, is split into
//     ncap equal arcs fanned from the chord midpoint.
// Separating the loops keeps a wavefront's lanes on the same code path (walk or
// fan) instead of paying both per step.  A cap span not in (0, pi] only arises
// from rounding when X and N coincide and is dropped (cross product <= 0).
// POW2: ncap is a power of two and the rotation comes from half-angle steps
// instead of atan2/sincos.  Vl: E' in absolute coordinates (6 values); all
// coordinates below are relative to the outer point.  cb: 12 doubles of
// scratch per call (cap endpoints).  nsub counts triangles, plus 2^16 per cap.
template <bool POW2, class TriF>
__device__ void partial_item(double xx, double xy, const double *Vl, double dd, int ncap, TriF &tri, int &nsub,
                             double *cb)
{
    Basis B;
    {
        const double e1x = Vl[2] - Vl[0], e1y = Vl[3] - Vl[1], e2x = Vl[4] - Vl[0], e2y = Vl[5] - Vl[1];
        const double id = 1.0 / (e1x * e2y - e1y * e2x);
        B.x0 = Vl[0] - xx;
        B.y0 = Vl[1] - xy;
        B.i11 = e2y * id;
        B.i12 = -e2x * id;
        B.i21 = -e1y * id;
        B.i22 = e1x * id;
    }
    int ev = 0, cnt = 0, ft = 0, pt = 0, ea = 0, eb = 0, ncp = 0;
    double f[5] = {0, 0, 0, 0, 0}, q[5] = {0, 0, 0, 0, 0};
    double epx = 0, epy = 0, eex = 0, eey = 0, el1 = 2.0, el2 = 2.0;
    auto record_cap = [&](double x0, double y0, double x1, double y1) {
        // span in (0, pi): counter-clockwise from X to N
        if (ncap < 2 || !(x0 * y1 - y0 * x1 > 0.0)) return;
        cb[4 * ncp] = x0;
        cb[4 * ncp + 1] = y0;
        cb[4 * ncp + 2] = x1;
        cb[4 * ncp + 3] = y1;
        ncp++;
    };
    while (true) {
        bool got = false;
        double n[5];
        int nt = 0;
        while (ev < 9 && !got) {
            const int a = ev / 3, kind = ev - 3 * (ev / 3);
            ev++;
            if (kind == 0) {
                const int b = a == 2 ? 0 : a + 1;
                // vertices picked by value (constant indices), so that Vl may point at registers
                const double ax = a == 0 ? Vl[0] : (a == 1 ? Vl[2] : Vl[4]);
                const double ay = a == 0 ? Vl[1] : (a == 1 ? Vl[3] : Vl[5]);
                const double bx = b == 0 ? Vl[0] : (b == 1 ? Vl[2] : Vl[4]);
                const double by = b == 0 ? Vl[1] : (b == 1 ? Vl[3] : Vl[5]);
                epx = ax - xx;
                epy = ay - xy;
                eex = bx - ax;
                eey = by - ay;
                ea = a;
                eb = b;
                if (edge_roots(epx, epy, eex, eey, dd, el1, el2)) {
                    set5(n, epx, epy, a == 0 ? 1.0 : 0.0, a == 1 ? 1.0 : 0.0, a == 2 ? 1.0 : 0.0);
                    nt = 0;
                    got = true;
                }
            } else {
                const double l = kind == 1 ? el1 : el2;
                if (l < 1.5) {
                    const double w1 = 1.0 - l;
                    set5(n, epx + l * eex, epy + l * eey, ea == 0 ? w1 : (eb == 0 ? l : 0.0),
                         ea == 1 ? w1 : (eb == 1 ? l : 0.0), ea == 2 ? w1 : (eb == 2 ? l : 0.0));
                    nt = kind;
                    got = true;
                }
            }
        }
        if (!got) {
            // the cap from the last exit back to the first entry
            if (cnt >= 2 && pt == 2 && ft == 1) record_cap(q[0], q[1], f[0], f[1]);
            break;
        }
        if (cnt >= 1 && pt == 2 && nt == 1) record_cap(q[0], q[1], n[0], n[1]);
        if (cnt >= 2) {
            double t[3][5];
#pragma unroll
            for (int i = 0; i < 5; i++) {
                t[0][i] = f[i];
                t[1][i] = q[i];
                t[2][i] = n[i];
            }
            tri(t);
            nsub++;
        }
        if (cnt == 0) {
#pragma unroll
            for (int i = 0; i < 5; i++) f[i] = n[i];
            ft = nt;
        }
#pragma unroll
        for (int i = 0; i < 5; i++) q[i] = n[i];
        pt = nt;
        cnt++;
    }
    for (int c = 0; c < ncp; c++) {
        double X[5], N[5], Mc[5], u[5];
        X[0] = cb[4 * c];
        X[1] = cb[4 * c + 1];
        N[0] = cb[4 * c + 2];
        N[1] = cb[4 * c + 3];
        basis_at(B, X[0], X[1], X[2], X[3], X[4]);
        basis_at(B, N[0], N[1], N[2], N[3], N[4]);
        const double cr = X[0] * N[1] - X[1] * N[0], dt = X[0] * N[0] + X[1] * N[1];
        double cc, ss;
        if (POW2) {
            // rotation by D/ncap from cos D, sin D by repeated half angles:
            // cos(t/2) = sqrt((1 + cos t)/2), sin(t/2) = sin t / (2 cos(t/2))
            const double r = 1.0 / sqrt((X[0] * X[0] + X[1] * X[1]) * (N[0] * N[0] + N[1] * N[1]));
            cc = dt * r;
            ss = cr * r;
            for (int m = ncap; m > 1; m >>= 1) {
                const double ch = sqrt(0.5 * (1.0 + cc));
                ss = ss / (2.0 * ch);
                cc = ch;
            }
        } else {
            const double D = atan2(cr, dt);
            sincos(D / (double)ncap, &ss, &cc);
        }
#pragma unroll
        for (int i = 0; i < 5; i++) {
            Mc[i] = 0.5 * (X[i] + N[i]);
            u[i] = X[i];
        }
        nsub += 1 << 16;
        for (int j = 1; j <= ncap; j++) {
            double v[5];
            if (j == ncap) {
#pragma unroll
                for (int i = 0; i < 5; i++) v[i] = N[i];
            } else {
                v[0] = cc * u[0] - ss * u[1];
                v[1] = ss * u[0] + cc * u[1];
                basis_at(B, v[0], v[1], v[2], v[3], v[4]);
            }
            double t[3][5];
#pragma unroll
            for (int i = 0; i < 5; i++) {
                t[0][i] = Mc[i];
                t[1][i] = u[i];
                t[2][i] = v[i];
                u[i] = v[i];
            }
            tri(t);
            nsub++;
        }
    }
}

// Barycenter ball: b_k' in the closed ball around x, rounded as the pair predicate.
__device__ __forceinline__ bool bary_in(double xx, double xy, double bx, double by, double dd)
{
#pragma clang fp contract(off)
    const double dx = xx - bx, dy = xy - by;
    return dx * dx + dy * dy <= dd;
}

// Item class of (x, E_k') under the intersection ball: 1 whole (every vertex
// in the closed ball), 2 partial (the ball meets the triangle otherwise), 0
// empty.  Every product and sum is rounded on its own, so the routing pass of
// the learned caps, the pair kernels and the oracle take identical decisions.
__device__ __forceinline__ int item_class(double xx, double xy, const double (&V)[6], double dd)
{
#pragma clang fp contract(off)
    int nin = 0;
#pragma unroll
    for (int a = 0; a < 3; a++) {
        const double dx = V[2 * a] - xx, dy = V[2 * a + 1] - xy;
        nin += dx * dx + dy * dy <= dd;
    }
    if (nin == 3) return 1;
    if (nin > 0) return 2;
    bool inside = true;
#pragma unroll
    for (int a = 0; a < 3; a++) {
        const int b = (a + 1) % 3;
        const double ex = V[2 * b] - V[2 * a], ey = V[2 * b + 1] - V[2 * a + 1];
        const double px = xx - V[2 * a], py = xy - V[2 * a + 1];
        if (ex * py - ey * px < 0.0) inside = false;
    }
    if (inside) return 2;
#pragma unroll
    for (int a = 0; a < 3; a++) {
        const int b = (a + 1) % 3;
        const double ex = V[2 * b] - V[2 * a], ey = V[2 * b + 1] - V[2 * a + 1];
        const double px = xx - V[2 * a], py = xy - V[2 * a + 1];
        const double t = ex * px + ey * py, L = ex * ex + ey * ey;
        if (t > 0.0 && t < L) {
            const double c = ex * py - ey * px;
            if (c * c <= dd * L) return 2;
        }
    }
    return 0;
}

// learned caps: a partial item far from tangency, | |v_a - x| - delta | >= band delta
// for every vertex, tested as |v_a - x|^2 >= (delta (1 + band))^2 or
// |v_a - x|^2 <= (delta (1 - band))^2
__device__ __forceinline__ bool item_routed(double xx, double xy, const double (&V)[6], double delta, double band)
{
#pragma clang fp contract(off)
    const double hi = delta * (1.0 + band), lo = band < 1.0 ? delta * (1.0 - band) : 0.0;
    const double hi2 = hi * hi, lo2 = lo * lo;
    bool ok = true;
#pragma unroll
    for (int a = 0; a < 3; a++) {
        const double dx = V[2 * a] - xx, dy = V[2 * a + 1] - xy;
        const double d2 = dx * dx + dy * dy;
        ok = ok && (d2 >= hi2 || d2 <= lo2);
    }
    return ok;
}


// Input of the learned cap network for (x, E_k'): the vertices in a frame
// centred at x, rotated so that the triangle's centroid lies on the positive
// first axis, shifted by the horizon and magnified by 8 (the element size of
// the h = delta/8 family): f_a = 8 (R(-phi)(v_a - x)/delta - (1, 0)).
__device__ __forceinline__ void mlp_features(double xx, double xy, const double (&V)[6], double delta, float (&f)[6])
{
#pragma clang fp contract(off)
    const double cx = ((V[0] + V[2]) + V[4]) / 3.0 - xx, cy = ((V[1] + V[3]) + V[5]) / 3.0 - xy;
    const double r = sqrt(cx * cx + cy * cy);
    const double c = r > 0.0 ? cx / r : 1.0, s = r > 0.0 ? cy / r : 0.0;
#pragma unroll
    for (int a = 0; a < 3; a++) {
        const double dx = (V[2 * a] - xx) / delta, dy = (V[2 * a + 1] - xy) / delta;
        f[2 * a] = (float)(8.0 * ((dx * c + dy * s) - 1.0));
        f[2 * a + 1] = (float)(8.0 * (dy * c - dx * s));
    }
}

// the item (x, E') inside the network's training domain (MlpDomain)
__device__ __forceinline__ bool in_domain(double xx, double xy, const double (&V)[6], double dd, const MlpDomain &D)
{
#pragma clang fp contract(off)
    const double rlo = D.rlo * dd, rhi = D.rhi * dd, elo = D.elo * dd, ehi = D.ehi * dd;
    bool ok = true;
#pragma unroll
    for (int a = 0; a < 3; a++) {
        const int b = (a + 1) % 3;
        const double dx = V[2 * a] - xx, dy = V[2 * a + 1] - xy;
        const double d2 = dx * dx + dy * dy;
        const double ex = V[2 * b] - V[2 * a], ey = V[2 * b + 1] - V[2 * a + 1];
        const double e2 = ex * ex + ey * ey;
        ok = ok && d2 >= rlo && d2 <= rhi && e2 >= elo && e2 <= ehi;
    }
    return ok;
}

// Boundary sums of a polygon's area and first and second moments (Green's
// theorem, counter-clockwise boundary, coordinates z about a local origin):
//   c = sum cr, mx = sum cr (ax + bx), my = sum cr (ay + by),
//   qxx = sum cr (ax^2 + ax bx + bx^2), qyy = likewise, qxy = sum cr (2 ax ay + ax by + bx ay + 2 bx by),
// cr = ax by - ay bx, so that A = c/2, int z = m/6, int zx^2 = qxx/12, int zx zy = qxy/24.
struct RegionMom {
    double c, mx, my, qxx, qxy, qyy;
};

__device__ __forceinline__ void edge_mom(RegionMom &R, double ax, double ay, double bx, double by)
{
    const double cr = ax * by - ay * bx;
    R.c += cr;
    R.mx += cr * (ax + bx);
    R.my += cr * (ay + by);
    R.qxx += cr * (ax * ax + ax * bx + bx * bx);
    R.qyy += cr * (ay * ay + ay * by + by * by);
    R.qxy += cr * (ax * (2.0 * ay + by) + bx * (ay + 2.0 * by));
}

// The same region E' n B_delta,h(x) as partial_item (inscribed polygon of
// Sec. 4.2.1 plus ncap equal-arc caps of Sec. 4.2.2), integrated through its
// boundary: walking the edges v0->v1->v2 gives the polygon's points in order
// (vertices in the closed ball, entry and exit roots); consecutive points are
// joined along an edge of E' except from an exit to the next entry, where the
// cap's arc chords X = P_0, P_1, ..., P_ncap = N replace the chord X N.  With
// psi constant and an inner rule exact for quadratics, the composite rule over
// the fan of the region gives exactly these moments.  Coordinates about
// vertex 0 of E'.  nseg counts boundary segments, plus 2^16 per cap.  cb: 12
// doubles of scratch per call.  iLv: the reciprocal squared lengths of the
// edges v0->v1, v1->v2, v2->v0 when the caller has them.
// 1/x to about an ulp: the hardware estimate and two Newton steps
__device__ __forceinline__ double rcp_nr(double x)
{
    double y = __builtin_amdgcn_rcp(x);
    double e = fma(-x, y, 1.0);
    y = fma(y, e, y);
    e = fma(-x, y, 1.0);
    return fma(y, e, y);
}

// 1/sqrt(v) to about an ulp: the hardware estimate and two Newton steps (for
// values that decide nothing: the exact decisions use the rounded sqrt)
__device__ __forceinline__ double rsqrt_nr(double v)
{
    double y = __builtin_amdgcn_rsq(v);
    y = y * (1.5 - 0.5 * v * y * y);
    y = y * (1.5 - 0.5 * v * y * y);
    return y;
}

// t - sin t, by its series where the difference cancels
__device__ __forceinline__ double t_sin_diff(double t)
{
    if (t < 0.1) {
        const double t2 = t * t;
        return t * t2 / 6.0 * (1.0 - t2 / 20.0 * (1.0 - t2 / 42.0 * (1.0 - t2 / 72.0 * (1.0 - t2 / 110.0))));
    }
    return t - sin(t);
}

// t/8 - sin(t)/6 + sin(2t)/48 = t^5/240 + O(t^7): for t < 1/2 by its series
// sum_{k>=2} (-1)^k t^(2k+1) (2^(2k+1) - 8) / (48 (2k+1)!)
__device__ __forceinline__ double segment_v2(double t)
{
    if (t < 0.5) {
        const double t2 = t * t;
        double pw = t * t2 * t2, fact = 120.0, two = 32.0, sum = 0.0;
        for (int k = 2; k <= 13; k++) {
            sum += ((k & 1) ? -1.0 : 1.0) * pw / fact * (two - 8.0) * (1.0 / 48.0);
            pw *= t2;
            fact *= (2.0 * k + 2.0) * (2.0 * k + 3.0);
            two *= 4.0;
        }
        return sum;
    }
    return t * (1.0 / 8.0) - sin(t) * (1.0 / 6.0) + sin(2.0 * t) * (1.0 / 48.0);
}

// The boundary-sum increments (RegionMom convention) of an exact cap in closed
// form: the circular segment from X = (ax, ay) counter-clockwise to N (cr, dt:
// cross and dot products of X and N, all relative to the centre) has, in the
// frame of the span's bisector (u along it, v across, t = the span),
// A = delta^2 (t - sin t)/2, int u = 2/3 delta^3 sin^3(t/2), int v = int uv = 0,
// int u^2 = delta^4 (2t - sin 2t)/16, int v^2 = delta^4 (t/8 - sin t/6 + sin 2t/48);
// rotated, and moved to the local origin o: int z = M1 - A o,
// int z z^T = M2 - M1 o^T - o M1^T + A o o^T.  Kept out of line: a rare path in
// kernels whose registers are spoken for.
__device__ __attribute__((noinline)) RegionMom analytic_cap(double ax, double ay, double cr, double dt, double ox,
                                                             double oy, double dd, double delta)
{
    RegionMom m = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    const double t = atan2(cr, dt);
    const double A = 0.5 * dd * t_sin_diff(t);
    if (!(A > 0.0)) return m;
    const double sh = sin(0.5 * t);
    const double iu = (2.0 / 3.0) * delta * dd * sh * sh * sh;
    const double iuu = dd * dd * t_sin_diff(2.0 * t) * (1.0 / 16.0), ivv = dd * dd * segment_v2(t);
    double sa, ca;
    sincos(atan2(ay, ax) + 0.5 * t, &sa, &ca);
    const double m1x = iu * ca, m1y = iu * sa;
    const double m2xx = iuu * ca * ca + ivv * sa * sa, m2yy = iuu * sa * sa + ivv * ca * ca;
    const double m2xy = (iuu - ivv) * ca * sa;
    m.c = 2.0 * A;
    m.mx = 6.0 * (m1x - A * ox);
    m.my = 6.0 * (m1y - A * oy);
    m.qxx = 12.0 * (m2xx - 2.0 * m1x * ox + A * ox * ox);
    m.qyy = 12.0 * (m2yy - 2.0 * m1y * oy + A * oy * oy);
    m.qxy = 24.0 * (m2xy - m1x * oy - m1y * ox + A * ox * oy);
    return m;
}

template <bool POW2, bool CEN = false>
__device__ void partial_boundary(double xx, double xy, const double *Vl, double dd, int ncap, RegionMom &R, int &nseg,
                                 double *cb, int centroid_rt = 0, double delta = 0.0, const double *iLv = nullptr)
{
    // CEN: the instantiation that can take exact caps (centroid_rt selects them at run
    // time: 1 the one-point centroid rule, 2 closed-form segment moments)
    const bool centroid = CEN && centroid_rt != 0;
    const double ox = Vl[0] - xx, oy = Vl[1] - xy;      // local origin (vertex 0) relative to x
    int cnt = 0, ft = 0, pt = 0, ncp = 0;
    double fx = 0.0, fy = 0.0, qx = 0.0, qy = 0.0;
    // caps found on the walk (at most three, one per exit) are kept in cb (12
    // doubles) and integrated after it, so that the lanes of a wavefront fan
    // their caps together
    // (the counters move by arithmetic, not in the branches: an increment in
    // both arms is merged through a selected address, which puts them in memory)
    auto connect = [&](double ax, double ay, int at, double bx, double by, int bt) __attribute__((always_inline)) {
        const bool cap = at == 2 && bt == 1 && (ncap >= 2 || centroid) && ax * by - ay * bx > 0.0;
        if (cap) {
            cb[4 * ncp] = ax;
            cb[4 * ncp + 1] = ay;
            cb[4 * ncp + 2] = bx;
            cb[4 * ncp + 3] = by;
        }
        if (!cap || centroid) edge_mom(R, ax - ox, ay - oy, bx - ox, by - oy);   // exact caps keep the chord
        ncp += cap ? 1 : 0;
        nseg += cap ? 0 : 1;
    };
    auto emit = [&](double nx, double ny, int nt) __attribute__((always_inline)) {
        if (cnt == 0) {
            fx = nx;
            fy = ny;
            ft = nt;
        } else {
            connect(qx, qy, pt, nx, ny, nt);
        }
        qx = nx;
        qy = ny;
        pt = nt;
        cnt++;
    };
#pragma unroll
    for (int a = 0; a < 3; a++) {
        const int b = a == 2 ? 0 : a + 1;
        const double epx = Vl[2 * a] - xx, epy = Vl[2 * a + 1] - xy;
        const double eex = Vl[2 * b] - Vl[2 * a], eey = Vl[2 * b + 1] - Vl[2 * a + 1];
        double el1, el2;
        if (edge_roots(epx, epy, eex, eey, dd, el1, el2, iLv ? iLv[a] : 0.0)) emit(epx, epy, 0);
        if (el1 < 1.5) emit(epx + el1 * eex, epy + el1 * eey, 1);
        if (el2 < 1.5) emit(epx + el2 * eex, epy + el2 * eey, 2);
    }
    if (cnt >= 2) connect(qx, qy, pt, fx, fy, ft);
    // each cap: the arc from X counter-clockwise to N in ncap equal pieces
    for (int ci = 0; ci < ncp; ci++) {
        const double ax = cb[4 * ci], ay = cb[4 * ci + 1], bx = cb[4 * ci + 2], by = cb[4 * ci + 3];
        const double cr = ax * by - ay * bx, dt = ax * bx + ay * by;
        if (centroid && centroid_rt == 2) {
            const RegionMom m = analytic_cap(ax, ay, cr, dt, ox, oy, dd, delta);
            R.c += m.c;
            R.mx += m.mx;
            R.my += m.my;
            R.qxx += m.qxx;
            R.qyy += m.qyy;
            R.qxy += m.qxy;
            nseg += 1 << 16;
            continue;
        }
        if (centroid) {
            // exact cap by the one-point rule of Sec. 5.2: weight = cap area
            // (delta^2/2)(2t - sin 2t), point on the bisector at 4 delta sin^3 t / (3 (2t - sin 2t)),
            // t = half the span; a point mass adds (w, w z, w z z^T) to the moments
            const double th = 0.5 * atan2(cr, dt);
            double seg = 2.0 * th - sin(2.0 * th);
            if (th < 1e-2) {                        // series of 2t - sin 2t, free of cancellation
                const double u = 2.0 * th, u2 = u * u;
                seg = u * u2 / 6.0 * (1.0 - u2 / 20.0 * (1.0 - u2 / 42.0 * (1.0 - u2 / 72.0)));
            }
            if (!(seg > 0.0)) continue;
            const double s3 = sin(th);
            const double dist = 4.0 * delta * s3 * s3 * s3 / (3.0 * seg);
            const double ang = atan2(ay, ax) + th;
            const double w = 0.5 * dd * seg;
            const double zx = dist * cos(ang) - ox, zy = dist * sin(ang) - oy;
            R.c += 2.0 * w;
            R.mx += 6.0 * w * zx;
            R.my += 6.0 * w * zy;
            R.qxx += 12.0 * w * zx * zx;
            R.qyy += 12.0 * w * zy * zy;
            R.qxy += 24.0 * w * zx * zy;
            nseg += 1 << 16;
            continue;
        }
        if (POW2) {
            // The inscribed arc X = P_0, ..., P_ncap = N in closed form: the chord
            // X N joins the region's polygon, and the closed polygon P_0 ... P_ncap
            // (the fan of triangles (x, P_j, P_j+1) less the triangle (x, X, N))
            // adds its area and moments.  In the frame of the span's bisector (u
            // along it, v across; the v and uv moments vanish by symmetry), with
            // t the span, phi = t / ncap, alpha_j = -t/2 + j phi and sums over
            // j = 0..ncap:
            //   A    = delta^2 (ncap sin phi - sin t) / 2
            //   I_u  = delta^3 (sin phi (S - cos(t/2)) - sin t cos(t/2)) / 3,
            //          S = sum cos alpha_j = sin((ncap+1) phi/2) / sin(phi/2)
            //   I_uu = delta^4 (sin phi (2 C - 2 cos^2(t/2) + ncap cos(phi)/2) + sin t/2 - 3 sin t cos^2(t/2)) / 12
            //   I_vv = delta^4 (sin phi (2 C' - 2 sin^2(t/2) + ncap cos(phi)/2) - sin t/2 - sin t sin^2(t/2)) / 12
            //   C, C' = sum cos^2, sin^2 alpha_j = (ncap+1)/2 +- sin((ncap+1) phi) / (2 sin phi)
            // (fan triangles (0, a, b): area a x b / 2, first moment area (a + b)/3,
            // second area (a a^T + b b^T + (a b^T + b a^T)/2)/6).  The half span
            // comes from the chord lengths, |X + N| = 2 delta cos(t/2) and
            // |X - N| = 2 delta sin(t/2) (accurate at either end of (0, pi)),
            // the smaller angles by halving: cos(s/2) = sqrt((1 + cos s)/2),
            // sin(s/2) = sin s / (2 cos(s/2)), both from one reciprocal square
            // root.  The bisector is X + N, or X - N turned by a right angle
            // when the span is past a right angle.
            edge_mom(R, ax - ox, ay - oy, bx - ox, by - oy);
            const double sx = ax + bx, sy = ay + by, qx = ax - bx, qy = ay - by;
            const double P = sx * sx + sy * sy, Q = qx * qx + qy * qy;
            const double rho = rsqrt_nr(P + Q), rP = rsqrt_nr(P), rQ = rsqrt_nr(Q);   // rho = 1 / (2 delta)
            const double ch = P * rP * rho, sh = Q * rQ * rho;                       // t/2
            const double st = 2.0 * sh * ch, ct = (ch - sh) * (ch + sh);
            double cc = ch, ss = sh, cp = ch, sp = sh;
            for (int lvl = 2; lvl < 2 * ncap; lvl <<= 1) {
                const double h = 0.5 * (1.0 + cc);
                const double rh = rsqrt_nr(h);
                ss = 0.5 * ss * rh;
                cc = h * rh;
                if (2 * lvl == ncap) {
                    cp = cc;                                                        // phi
                    sp = ss;
                }
            }
            const double n = (double)ncap;
            const double S = (sh * cc + ch * ss) * rcp_nr(ss);                      // (cc, ss): phi/2
            const double Sc = (st * cp + ct * sp) * rcp_nr(sp);
            const double C = 0.5 * (n + 1.0) + 0.5 * Sc, Cs = 0.5 * (n + 1.0) - 0.5 * Sc;
            const double nc = 0.5 * n * cp, ch2 = ch * ch, sh2 = sh * sh;
            const double A = 0.5 * dd * (n * sp - st);
            const double iu = dd * (1.0 / 3.0) * (sp * (S - ch) - st * ch);          // I_u / delta
            const double d4 = dd * dd * (1.0 / 12.0);
            const double iuu = d4 * (sp * (2.0 * C - 2.0 * ch2 + nc) + 0.5 * st - 3.0 * st * ch2);
            const double ivv = d4 * (sp * (2.0 * Cs - 2.0 * sh2 + nc) - 0.5 * st - st * sh2);
            const bool wide = Q > P;
            const double ux = wide ? -qy * rQ : sx * rP, uy = wide ? qx * rQ : sy * rP;
            const double dl = 2.0 * rho * dd;                                        // delta
            const double m1x = iu * ux * dl, m1y = iu * uy * dl;
            const double m2xx = iuu * ux * ux + ivv * uy * uy, m2yy = iuu * uy * uy + ivv * ux * ux;
            const double m2xy = (iuu - ivv) * ux * uy;
            R.c += 2.0 * A;
            R.mx += 6.0 * (m1x - A * ox);
            R.my += 6.0 * (m1y - A * oy);
            R.qxx += 12.0 * (m2xx - 2.0 * m1x * ox + A * ox * ox);
            R.qyy += 12.0 * (m2yy - 2.0 * m1y * oy + A * oy * oy);
            R.qxy += 24.0 * (m2xy - m1x * oy - m1y * ox + A * ox * oy);
            nseg += (1 << 16) + ncap;
            continue;
        }
        // rotation by phi = span / ncap
        double cc, ss;
        {
            const double D = atan2(cr, dt);
            sincos(D / (double)ncap, &ss, &cc);
        }
        double ux = ax, uy = ay;
        for (int j = 1; j <= ncap; j++) {
            double vx, vy;
            if (j == ncap) {
                vx = bx;
                vy = by;
            } else {
                vx = cc * ux - ss * uy;
                vy = ss * ux + cc * uy;
            }
            edge_mom(R, ux - ox, uy - oy, vx - ox, vy - oy);
            ux = vx;
            uy = vy;
        }
        nseg += (1 << 16) + ncap;
    }
}

// Rows g1, g2 of the inverse edge matrix of E' (vertices Vl): beta1 = g1 . z,
// beta2 = g2 . z for z about vertex 0.
__device__ __forceinline__ void inv_edges(const double *Vl, double (&g)[4])
{
    const double e1x = Vl[2] - Vl[0], e1y = Vl[3] - Vl[1], e2x = Vl[4] - Vl[0], e2y = Vl[5] - Vl[1];
    const double id = 1.0 / (e1x * e2y - e1y * e2x);
    g[0] = e2y * id;
    g[1] = -e2x * id;
    g[2] = -e1y * id;
    g[3] = e1x * id;
}

// S0 = int 1, S1_b = int beta_b, S2 = int beta_b beta_b' (upper 00,01,02,11,12,22)
// over the region from its boundary sums; beta0 = 1 - beta1 - beta2 with g
// from inv_edges.
__device__ __forceinline__ void region_sums_g(const RegionMom &R, const double (&g)[4], double &s0, double (&s1)[3],
                                              double (&s2)[6])
{
    const double g11 = g[0], g12 = g[1], g21 = g[2], g22 = g[3];
    const double A = 0.5 * R.c;
    const double mx = R.mx * (1.0 / 6.0), my = R.my * (1.0 / 6.0);
    const double Qxx = R.qxx * (1.0 / 12.0), Qyy = R.qyy * (1.0 / 12.0), Qxy = R.qxy * (1.0 / 24.0);
    const double I1 = g11 * mx + g12 * my, I2 = g21 * mx + g22 * my;
    const double Q11 = g11 * (g11 * Qxx + g12 * Qxy) + g12 * (g11 * Qxy + g12 * Qyy);
    const double Q22 = g21 * (g21 * Qxx + g22 * Qxy) + g22 * (g21 * Qxy + g22 * Qyy);
    const double Q12 = g11 * (g21 * Qxx + g22 * Qxy) + g12 * (g21 * Qxy + g22 * Qyy);
    s0 = A;
    s1[0] = A - I1 - I2;
    s1[1] = I1;
    s1[2] = I2;
    s2[0] = A - 2.0 * (I1 + I2) + Q11 + 2.0 * Q12 + Q22;
    s2[1] = I1 - Q11 - Q12;
    s2[2] = I2 - Q12 - Q22;
    s2[3] = Q11;
    s2[4] = Q12;
    s2[5] = Q22;
}

__device__ __forceinline__ void region_sums(const RegionMom &R, const double *Vl, double &s0, double (&s1)[3],
                                            double (&s2)[6])
{
    double g[4];
    inv_edges(Vl, g);
    region_sums_g(R, g, s0, s1, s2);
}
