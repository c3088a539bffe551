/*
 * nlo.c - plain FP64 CPU oracle for the P1 nonlocal stiffness assembly of
 * D'Elia, Gunzburger, Vollmann, arXiv:2005.10775.
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the test-suite, the smoke check and the
 * CPU-baseline leg of the benchmark, never by the product library.
 *
 * What it computes, with the passages it follows:
 *   - the D-form (Eq. (bform0)) discretised with P1 elements and assembled over
 *     every ordered element pair (k, k') of Omega u Omega_I, as in Eq.
 *     (bformhj) with the approximate ball of Sec. 4 in place of the exact one
 *     (Eqs. (bform3h), (bformjqqh)); the (A-B-C) recipe of Sec. 7.2 is the
 *     split of the full matrix D into A = D[free,free] and the right-hand side
 *     b = G - D[free, Dirichlet] g (Eqs. (appr), (intcon), (lfunchj));
 *   - balls: barycenter (Eq. (baryball)) and the intersection ball of
 *     Sec. 4.2.1 (inscribed polygon, "nocaps") with caps either replaced by
 *     triangles over equal arcs (Sec. 4.2.2) or integrated by the one-point
 *     centroid rule of Sec. 5.2 (the cap weight is the cap area of
 *     Eq. (areacap); the factor 1/4 printed next to the centroid formula is
 *     read as 1/2, which is what Eq. (areacap) gives); the overlap ball (Eq.
 *     (overlap): whole elements meeting B_delta(x)); the shifted ball of
 *     Sec. 4.3 (the intersection ball about b_k for every point of E_k); and the
 *     barycenter ball with its outer support resolved (Sec. 6, case 2: the outer
 *     rule over the nocaps / approxcaps region of E_k n B_delta(b_k'), the inner
 *     integral over the whole E_k'); the last three for the constant kernel;
 *   - the geometric tasks 1-6 of Sec. 7.1 (vertex test, edge-circle quadratic,
 *     counter-clockwise ordering and fan triangulation from the first point);
 *   - composite inner rules of Eq. (cqr1), outer rule of Sec. 6 (optionally
 *     switched per pair as in Sec. 8: rule 2 for |b_k - b_k'| < switch_dist).
 * Every +,-,* is rounded separately (built with -ffp-contract=off), the
 * barycenter is ((v0+v1)+v2)/3 and an outer point ((l0 v0 + l1 v1) + l2 v2),
 * so the pair list is reproducible by any IEEE implementation of the same
 * expressions.
 *
 * Parity pins: see tests/test_oracle_pins.py (rule moments, kernel
 * normalisation, closed-form whole pairs, exact ball area/second moment with
 * analytic caps, brute-force region moments, matrix invariants, load vector,
 * the paper's printed L2 errors of Sec. 8 for the nocaps, approxcaps, overlap,
 * shifted and barycenter-support balls, the x <-> y identity between the
 * shifted and barycenter-support matrices, grid (b)'s printed element sizes,
 * the one-point centroid caps of Sec. 5.2 against the exact intersection's
 * area and first moments, which a centroid rule integrates exactly).
 * Parity unpinned: the printed barycenter column of Sec. 8.1 and the grid (b)
 * columns are not reproduced (lattice ties; the unstated diagonal direction).
 */
#include "nlo.h"
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif


static const double NLO_PI = 3.14159265358979323846;

/* ------------------------------------------------------------------ mesh */
static void tri_vertices(const nlo_mesh *m, int k, double V[6])
{
    for (int a = 0; a < 3; a++) {
        int j = m->tri[3 * k + a];
        V[2 * a] = m->xy[2 * j];
        V[2 * a + 1] = m->xy[2 * j + 1];
    }
}

/* task 1 of Sec. 7.1: the barycenter is the vertex average */
static void barycenter(const double V[6], double b[2])
{
    b[0] = ((V[0] + V[2]) + V[4]) / 3.0;
    b[1] = ((V[1] + V[3]) + V[5]) / 3.0;
}

static void map_point(const double V[6], const double lam[3], double x[2])
{
    x[0] = (lam[0] * V[0] + lam[1] * V[2]) + lam[2] * V[4];
    x[1] = (lam[0] * V[1] + lam[1] * V[3]) + lam[2] * V[5];
}

static double twice_area(const double V[6])
{
    return fabs((V[2] - V[0]) * (V[5] - V[1]) - (V[3] - V[1]) * (V[4] - V[0]));
}

static double max_vertex_dist(const double V[6], const double b[2])
{
    double r = 0.0;
    for (int a = 0; a < 3; a++) {
        double dx = V[2 * a] - b[0], dy = V[2 * a + 1] - b[1];
        double d = sqrt(dx * dx + dy * dy);
        if (d > r) r = d;
    }
    return r;
}

/* P1 basis of element V at point y: barycentric coordinates */
static void basis_at(const double V[6], const double y[2], double beta[3])
{
    double det = (V[2] - V[0]) * (V[5] - V[1]) - (V[3] - V[1]) * (V[4] - V[0]);
    double b1 = ((y[0] - V[0]) * (V[5] - V[1]) - (y[1] - V[1]) * (V[4] - V[0])) / det;
    double b2 = ((V[2] - V[0]) * (y[1] - V[1]) - (V[3] - V[1]) * (y[0] - V[0])) / det;
    beta[0] = 1.0 - b1 - b2;
    beta[1] = b1;
    beta[2] = b2;
}

/* ------------------------------------------------------------ kernel psi */
static double kernel_psi(const nlo_problem *p, const double x[2], const double y[2])
{
    if (p->kernel == 0) return p->kc;
    double dx = x[0] - y[0], dy = x[1] - y[1];
    double r = sqrt(dx * dx + dy * dy);
    return p->kc * pow(r, -(2.0 + 2.0 * p->ks));
}

/* ------------------------------------------------------ ball predicates */
/* barycenter ball, Eq. (baryball): E_k' belongs to B(x) iff |x - b_k'| <= delta */
static int bary_in(const double x[2], const double b[2], double dd)
{
    double dx = x[0] - b[0], dy = x[1] - b[1];
    return dx * dx + dy * dy <= dd;
}

/* closed ball B_delta(x) meets the triangle V (tasks 2-4 of Sec. 7.1):
 * a vertex within delta, or x inside the triangle, or an edge whose interior
 * comes within delta (projection strictly inside the edge, squared distance
 * c^2/L <= delta^2 written without division). */
static int ball_meets_triangle(const double x[2], const double V[6], double dd)
{
    for (int a = 0; a < 3; a++) {
        double dx = V[2 * a] - x[0], dy = V[2 * a + 1] - x[1];
        if (dx * dx + dy * dy <= dd) return 1;
    }
    int inside = 1;
    for (int a = 0; a < 3; a++) {
        int b = (a + 1) % 3;
        double ex = V[2 * b] - V[2 * a], ey = V[2 * b + 1] - V[2 * a + 1];
        double px = x[0] - V[2 * a], py = x[1] - V[2 * a + 1];
        double o = ex * py - ey * px;
        if (o < 0.0) inside = 0;
    }
    if (inside) return 1;
    for (int a = 0; a < 3; a++) {
        int b = (a + 1) % 3;
        double ex = V[2 * b] - V[2 * a], ey = V[2 * b + 1] - V[2 * a + 1];
        double px = x[0] - V[2 * a], py = x[1] - V[2 * a + 1];
        double t = ex * px + ey * py;
        double L = ex * ex + ey * ey;
        if (t > 0.0 && t < L) {
            double c = ex * py - ey * px;
            if (c * c <= dd * L) return 1;
        }
    }
    return 0;
}

/* which outer rule a pair uses (Sec. 8 switch; one rule when n_out2 == 0) */
static void pair_rule(const nlo_problem *p, const double bk[2], const double bkp[2],
                      int *nq, const double **lam, const double **w)
{
    *nq = p->n_out;
    *lam = p->out_lam;
    *w = p->out_w;
    /* |b_k - b_k'| < switch_dist, compared in squares: never when switch_dist <= 0 */
    if (p->n_out2 > 0 && p->switch_dist > 0.0) {
        double dx = bk[0] - bkp[0], dy = bk[1] - bkp[1];
        if (dx * dx + dy * dy < p->switch_dist * p->switch_dist) {
            *nq = p->n_out2;
            *lam = p->out2_lam;
            *w = p->out2_w;
        }
    }
}

static int pair_interacts(const nlo_problem *p, const double Vk[6], const double bk[2],
                          const double Vkp[6], const double bkp[2])
{
    double dd = p->delta * p->delta;
    /* shifted (Sec. 4.3): every point of E_k uses the ball about b_k */
    if (p->ball == 3) return ball_meets_triangle(bk, Vkp, dd);
    /* barycenter, outer support (Sec. 6, case 2): some x in E_k has b_k' in
     * B_delta(x), i.e. E_k meets the ball about b_k' */
    if (p->ball == 4) return ball_meets_triangle(bkp, Vk, dd);
    int nq;
    const double *lam, *w;
    pair_rule(p, bk, bkp, &nq, &lam, &w);
    for (int q = 0; q < nq; q++) {
        double x[2];
        map_point(Vk, lam + 3 * q, x);
        if (p->ball == 0) {
            if (bary_in(x, bkp, dd)) return 1;
        } else {
            /* intersection and overlap balls: E_k' meets B_delta(x) */
            if (ball_meets_triangle(x, Vkp, dd)) return 1;
        }
    }
    return 0;
}

/* cheap conservative reject: a point of E_k' within delta of a point of E_k
 * needs |b_k - b_k'| <= delta + r_k + r_k' (barycenter ball: delta + r_k). */
static int maybe_pair(const nlo_problem *p, const double bk[2], double rk,
                      const double bkp[2], double rkp)
{
    double reach = p->delta + rk + (p->ball == 0 ? 0.0 : rkp);
    reach = reach * (1.0 + 1e-9) + 1e-14;
    double dx = bk[0] - bkp[0], dy = bk[1] - bkp[1];
    return dx * dx + dy * dy <= reach * reach;
}

/* ------------------------------------------------ intersection ball region */
typedef struct { double x, y; int type; } rpoint;   /* type 0 vertex, 1 entry, 2 exit */

/* tasks 3-6 of Sec. 7.1: walk the edges v0->v1->v2->v0, keep vertices inside
 * the closed ball, and the roots lambda in (0,1) of |v_i + lambda e - x|^2 =
 * delta^2 in increasing order (smaller root = entry, larger = exit). */
static int build_polygon(const double x[2], const double V[6], double dd, rpoint *P)
{
    int n = 0;
    for (int a = 0; a < 3; a++) {
        int b = (a + 1) % 3;
        double px = V[2 * a] - x[0], py = V[2 * a + 1] - x[1];
        if (px * px + py * py <= dd) {
            P[n].x = V[2 * a];
            P[n].y = V[2 * a + 1];
            P[n].type = 0;
            n++;
        }
        double ex = V[2 * b] - V[2 * a], ey = V[2 * b + 1] - V[2 * a + 1];
        double L = ex * ex + ey * ey;
        double B = ex * px + ey * py;
        double C = (px * px + py * py) - dd;
        double disc = B * B - L * C;
        if (disc > 0.0) {
            double s = sqrt(disc);
            double l1 = (-B - s) / L, l2 = (-B + s) / L;
            if (l1 > 0.0 && l1 < 1.0) {
                P[n].x = V[2 * a] + l1 * ex;
                P[n].y = V[2 * a + 1] + l1 * ey;
                P[n].type = 1;
                n++;
            }
            if (l2 > 0.0 && l2 < 1.0) {
                P[n].x = V[2 * a] + l2 * ex;
                P[n].y = V[2 * a + 1] + l2 * ey;
                P[n].type = 2;
                n++;
            }
        }
    }
    return n;
}

static void put_tri(double *sub, int *ns, double ax, double ay, double bx, double by,
                    double cx, double cy)
{
    double *t = sub + 6 * (*ns);
    t[0] = ax; t[1] = ay; t[2] = bx; t[3] = by; t[4] = cx; t[5] = cy;
    (*ns)++;
}

/* The region E_k' n B_{delta,h}(x) of the intersection ball as a list of
 * triangles (polygon fan + cap triangles) and, for exact caps, a list of
 * one-point cap rules (point, weight).  Returns the number of triangles, or
 * -1 when the ball lies inside the triangle without reaching any edge. */
int nlo_region(const nlo_problem *p, const double x[2], const double V[6],
               double *sub, int32_t cap, double *cap_pts, double *cap_w, int32_t *n_cap)
{
    double dd = p->delta * p->delta;
    rpoint P[12];
    int n = build_polygon(x, V, dd, P);
    int ns = 0;
    *n_cap = 0;
    if (n == 0) {
        /* no vertex inside and no crossing: empty, unless x is inside E (ball inside triangle) */
        int inside = 1;
        for (int a = 0; a < 3; a++) {
            int b = (a + 1) % 3;
            double ex = V[2 * b] - V[2 * a], ey = V[2 * b + 1] - V[2 * a + 1];
            double o = ex * (x[1] - V[2 * a + 1]) - ey * (x[0] - V[2 * a]);
            if (o < 0.0) inside = 0;
        }
        return inside ? -1 : 0;
    }
    for (int i = 1; i + 1 < n; i++) {
        if (ns >= cap) return -2;
        put_tri(sub, &ns, P[0].x, P[0].y, P[i].x, P[i].y, P[i + 1].x, P[i + 1].y);
    }
    for (int i = 0; i < n; i++) {
        const rpoint *X = &P[i], *N = &P[(i + 1) % n];
        if (X->type != 2 || N->type != 1) continue;
        double tx = atan2(X->y - x[1], X->x - x[0]);
        double tn = atan2(N->y - x[1], N->x - x[0]);
        double D = tn - tx;
        if (D < 0.0) D += 2.0 * NLO_PI;             /* counter-clockwise span from X to N */
        /* a cap inside a triangle of diameter <= delta spans less than pi; a
         * larger span only arises from rounding when X and N coincide */
        if (!(D > 0.0) || D > NLO_PI) continue;
        if (p->cap_mode == 2) {
            /* analytic caps: the chord ends and the span, integrated in closed form by the caller */
            cap_pts[4 * (*n_cap)] = X->x;
            cap_pts[4 * (*n_cap) + 1] = X->y;
            cap_pts[4 * (*n_cap) + 2] = N->x;
            cap_pts[4 * (*n_cap) + 3] = N->y;
            cap_w[*n_cap] = D;
            (*n_cap)++;
        } else if (p->cap_mode == 1) {
            double th = 0.5 * D;
            double seg = 2.0 * th - sin(2.0 * th);
            if (th < 1e-2) {                        /* series of 2t - sin 2t, cancellation-free */
                double u = 2.0 * th, u2 = u * u;
                seg = u * u2 / 6.0 * (1.0 - u2 / 20.0 * (1.0 - u2 / 42.0 * (1.0 - u2 / 72.0)));
            }
            if (!(seg > 0.0)) continue;
            double s3 = sin(th);
            double dist = 4.0 * p->delta * s3 * s3 * s3 / (3.0 * seg);
            double ang = tx + th;
            cap_pts[2 * (*n_cap)] = x[0] + dist * cos(ang);
            cap_pts[2 * (*n_cap) + 1] = x[1] + dist * sin(ang);
            cap_w[*n_cap] = 0.5 * dd * seg;
            (*n_cap)++;
        } else if (p->cap_edges >= 2) {
            double mx = 0.5 * (X->x + N->x), my = 0.5 * (X->y + N->y);
            double px = X->x, py = X->y;
            for (int j = 1; j <= p->cap_edges; j++) {
                double cx, cy;
                if (j == p->cap_edges) {
                    cx = N->x;
                    cy = N->y;
                } else {
                    double ang = tx + D * (double)j / (double)p->cap_edges;
                    cx = x[0] + p->delta * cos(ang);
                    cy = x[1] + p->delta * sin(ang);
                }
                if (ns >= cap) return -2;
                put_tri(sub, &ns, mx, my, px, py, cx, cy);
                px = cx;
                py = cy;
            }
        }
    }
    return ns;
}

/* t - sin t, by its series where the difference cancels */
static double t_minus_sin(double t)
{
    if (t < 1e-1) {
        double t2 = t * t;
        return t * t2 / 6.0 * (1.0 - t2 / 20.0 * (1.0 - t2 / 42.0 * (1.0 - t2 / 72.0 * (1.0 - t2 / 110.0))));
    }
    return t - sin(t);
}

/* t/8 - sin(t)/6 + sin(2t)/48 = sum_{k>=2} (-1)^k t^(2k+1) (2^(2k+1) - 8) / (48 (2k+1)!),
 * by the series where the direct form cancels (it is t^5/240 + O(t^7)) */
static double cap_v2_factor(double t)
{
    if (t < 0.5) {
        double sum = 0.0, pw = t, fact = 1.0, two = 2.0;
        for (int k = 1; k <= 13; k++) {
            pw *= t * t;
            fact *= (2.0 * k) * (2.0 * k + 1.0);
            two *= 4.0;
            if (k >= 2) sum += ((k & 1) ? -1.0 : 1.0) * pw / fact * (two - 8.0) / 48.0;
        }
        return sum;
    }
    return t / 8.0 - sin(t) / 6.0 + sin(2.0 * t) / 48.0;
}

/* Area, first and second moments about the centre x of the circular segment
 * of the ball B_delta(x) cut off by the chord X N, the arc running
 * counter-clockwise from X to N over the span D < pi (the caps of Sec. 4.2.2
 * taken exactly; cf. Eq. (areacap)).  In the frame of the span's bisector
 * (u along it, v across) with t = D:
 *   A = delta^2 (t - sin t) / 2,  int u = 2/3 delta^3 sin^3(t/2),  int v = 0,
 *   int u^2 = delta^4 (2t - sin 2t) / 16,
 *   int v^2 = delta^4 (t/8 - sin(t)/6 + sin(2t)/48),  int uv = 0
 * (sector minus triangle); rotated to the axes: M1 = (int y - x),
 * M2 = (int (y-x)_1^2, int (y-x)_1 (y-x)_2, int (y-x)_2^2). */
static void cap_segment_moments(double delta, const double x[2], const double X[2], double D,
                                double *A, double M1[2], double M2[3])
{
    double d2 = delta * delta, d4 = d2 * d2;
    double phi = atan2(X[1] - x[1], X[0] - x[0]) + 0.5 * D;
    double c = cos(phi), sn = sin(phi);
    double s3 = sin(0.5 * D);
    double iu = 2.0 / 3.0 * delta * d2 * s3 * s3 * s3;
    double iuu = d4 * t_minus_sin(2.0 * D) / 16.0;
    double ivv = d4 * cap_v2_factor(D);
    *A = 0.5 * d2 * t_minus_sin(D);
    M1[0] = iu * c;
    M1[1] = iu * sn;
    M2[0] = iuu * c * c + ivv * sn * sn;
    M2[1] = (iuu - ivv) * c * sn;
    M2[2] = iuu * sn * sn + ivv * c * c;
}

/* composite inner rule (Eq. (cqr1)) of psi, psi*beta_b, psi*beta_b*beta_b'
 * over the region of (x, E_k').  Returns 0, or a negative status. */
int nlo_inner_sums(const nlo_problem *p, const double x[2], const double V[6],
                   double s0[1], double s1[3], double s2[9])
{
    static const double whole_lam[3] = {0, 0, 0};
    (void)whole_lam;
    s0[0] = 0.0;
    for (int b = 0; b < 3; b++) s1[b] = 0.0;
    for (int b = 0; b < 9; b++) s2[b] = 0.0;
    double dd = p->delta * p->delta;
    double sub[6 * NLO_MAXSUB];
    double cpt[4 * 8], cw[8];
    int ns = 0, nc = 0;
    int use_mlp = 0;
    if (p->ball == 0) {
        double b[2];
        barycenter(V, b);
        if (!bary_in(x, b, dd)) return 0;
        memcpy(sub, V, 6 * sizeof(double));
        ns = 1;
    } else if (p->ball == 2) {
        /* overlap ball, Eq. (overlap): the whole element when it meets B_delta(x) */
        if (!ball_meets_triangle(x, V, dd)) return 0;
        memcpy(sub, V, 6 * sizeof(double));
        ns = 1;
    } else if (p->ball == 4) {
        /* barycenter ball with the outer support resolved: x lies in the
         * support, so the whole inner element */
        memcpy(sub, V, 6 * sizeof(double));
        ns = 1;
    } else {
        if (p->learned) {
            /* a partial item (some vertex outside the ball, at least one cap)
             * far from tangency takes the polygon and the learned caps */
            int nin = 0;
            for (int a = 0; a < 3; a++) {
                double dx = V[2 * a] - x[0], dy = V[2 * a + 1] - x[1];
                nin += dx * dx + dy * dy <= dd;
            }
            if (nin < 3 && nlo_routed(p->delta, p->band, x, V) && nlo_in_domain(p->mlp_domain, x, V, p->delta)) {
                double mm[3];
                int ncap = nlo_cap_moments(p, x, V, mm);
                if (ncap < 0) return ncap;
                use_mlp = ncap > 0;
            }
        }
        nlo_problem p0 = *p;
        if (use_mlp) {
            p0.cap_edges = 0;
            p0.cap_mode = 0;
        }
        ns = nlo_region(&p0, x, V, sub, NLO_MAXSUB, cpt, cw, &nc);
        if (ns < 0) return ns;
    }
    for (int t = 0; t < ns; t++) {
        const double *T = sub + 6 * t;
        double a2 = twice_area(T);
        for (int q = 0; q < p->n_in; q++) {
            double y[2], beta[3];
            map_point(T, p->in_lam + 3 * q, y);
            double wq = p->in_w[q] * a2 * kernel_psi(p, x, y);
            basis_at(V, y, beta);
            s0[0] += wq;
            for (int b = 0; b < 3; b++) {
                s1[b] += wq * beta[b];
                for (int c = 0; c < 3; c++) s2[3 * b + c] += wq * beta[b] * beta[c];
            }
        }
    }
    if (p->ball != 0 && p->cap_mode == 2 && !use_mlp) {
        /* analytic caps (constant kernel): beta_b(y) = a_b + g_b . (y - x) is
         * affine, so its integrals over a segment follow from the segment's
         * moments: int beta_b = a_b A + g_b . M1,
         * int beta_b beta_c = a_b a_c A + a_b g_c . M1 + a_c g_b . M1 + g_b^T M2 g_c */
        double a[3], g[3][2];
        double det = (V[2] - V[0]) * (V[5] - V[1]) - (V[3] - V[1]) * (V[4] - V[0]);
        basis_at(V, x, a);
        g[1][0] = (V[5] - V[1]) / det;
        g[1][1] = -(V[4] - V[0]) / det;
        g[2][0] = -(V[3] - V[1]) / det;
        g[2][1] = (V[2] - V[0]) / det;
        g[0][0] = -g[1][0] - g[2][0];
        g[0][1] = -g[1][1] - g[2][1];
        double psi = kernel_psi(p, x, x);
        for (int c = 0; c < nc; c++) {
            double A, M1[2], M2[3];
            cap_segment_moments(p->delta, x, cpt + 4 * c, cw[c], &A, M1, M2);
            s0[0] += psi * A;
            for (int b = 0; b < 3; b++) {
                double gm_b = g[b][0] * M1[0] + g[b][1] * M1[1];
                s1[b] += psi * (a[b] * A + gm_b);
                for (int e = 0; e < 3; e++) {
                    double gm_e = g[e][0] * M1[0] + g[e][1] * M1[1];
                    double q = g[b][0] * (M2[0] * g[e][0] + M2[1] * g[e][1]) +
                               g[b][1] * (M2[1] * g[e][0] + M2[2] * g[e][1]);
                    s2[3 * b + e] += psi * (a[b] * a[e] * A + a[b] * gm_e + a[e] * gm_b + q);
                }
            }
        }
        nc = 0;
    }
    for (int c = 0; c < nc; c++) {
        double y[2] = {cpt[2 * c], cpt[2 * c + 1]}, beta[3];
        double wq = cw[c] * kernel_psi(p, x, y);
        basis_at(V, y, beta);
        s0[0] += wq;
        for (int b = 0; b < 3; b++) {
            s1[b] += wq * beta[b];
            for (int e = 0; e < 3; e++) s2[3 * b + e] += wq * beta[b] * beta[e];
        }
    }
    if (use_mlp) return nlo_learned_caps(p, x, V, s0, s1, s2);
    return 0;
}

/* ------------------------------------------------ near-diagonal pairs */
static int shares_vertex(const nlo_mesh *m, int k, int kp)
{
    for (int a = 0; a < 3; a++)
        for (int b = 0; b < 3; b++)
            if (m->tri[3 * k + a] == m->tri[3 * kp + b]) return 1;
    return 0;
}

int nlo_duffy_block(const nlo_mesh *m, const nlo_problem *p, int k, int kp, double blk[36]);

/* ------------------------------------------------ local pair block */
/* The 6x6 local block of pair (k, k') in slot order (a0,a1,a2,b0,b1,b2):
 *   [[Mxx, -Mxy], [-Mxy^T, Myy]],
 *   Mxx_aa' = sum_q W_q alpha_a alpha_a' S0_q,  Mxy_ab = sum_q W_q alpha_a S1_qb,
 *   Myy_bb' = sum_q W_q S2_qbb',  W_q = 2|E_k| w_q, alpha = outer barycentrics;
 * the expansion of (phi_j(x)-phi_j(y))(phi_j'(x)-phi_j'(y)) of Eq. (bformhj)
 * over the nodes of E_k (x) and E_k' (y).  D[g(i), g(j)] += blk[i][j]. */
int nlo_pair_block(const nlo_mesh *m, const nlo_problem *p, int32_t k, int32_t kp,
                   double mxy[9], double myy[9], double s0q[64], double blk[36])
{
    double Vk[6], Vkp[6], bk[2], bkp[2];
    tri_vertices(m, k, Vk);
    tri_vertices(m, kp, Vkp);
    barycenter(Vk, bk);
    barycenter(Vkp, bkp);
    for (int i = 0; i < 9; i++) { mxy[i] = 0.0; myy[i] = 0.0; }
    for (int i = 0; i < 36; i++) blk[i] = 0.0;
    if (p->kernel == 1 && shares_vertex(m, k, kp)) {
        /* The joint integrand (phi_n(x) - phi_n(y))(phi_m(x) - phi_m(y)) psi over
         * {x in E_k, y in E_k', |x - y| <= delta} is symmetric under x <-> y, so
         * the node-level block of (k', k) is that of (k, k').  It is computed for
         * k <= k' (or when (k', k) is not an interacting pair) and relabelled. */
        if (k > kp && pair_interacts(p, Vkp, bkp, Vk, bk)) {
            double bt[36];
            int st = nlo_duffy_block(m, p, kp, k, bt);
            if (st < 0) return st;
            int sl[6], slt[6];          /* slot of node n in (k, k') and in (k', k) order */
            for (int i = 0; i < 6; i++) {
                int n = i < 3 ? m->tri[3 * k + i] : m->tri[3 * kp + i - 3];
                sl[i] = -1;
                for (int a = 0; a < 3; a++)
                    if (m->tri[3 * kp + a] == n) sl[i] = a;
                if (sl[i] < 0)
                    for (int a = 0; a < 3; a++)
                        if (m->tri[3 * k + a] == n) sl[i] = 3 + a;
                /* merged slot of (k, k'): a node of E_k' that is also in E_k */
                slt[i] = i >= 3 && (m->tri[3 * k] == n || m->tri[3 * k + 1] == n || m->tri[3 * k + 2] == n);
            }
            for (int i = 0; i < 6; i++)
                for (int j = 0; j < 6; j++)
                    blk[6 * i + j] = (slt[i] || slt[j]) ? 0.0 : bt[6 * sl[i] + sl[j]];
            return 0;
        }
        return nlo_duffy_block(m, p, k, kp, blk);
    }
    int nq;
    const double *lam, *w;
    pair_rule(p, bk, bkp, &nq, &lam, &w);
    double ak2 = twice_area(Vk);
    double mxx[9] = {0};
    if (p->ball == 4) {
        /* Sec. 6, case 2 for the barycenter ball: the outer integrand vanishes
         * outside S = E_k n B_delta(b_k'), so the outer rule is applied to the
         * triangles of S's nocaps / approxcaps region (and exact caps by their
         * one-point centroid rule); at each such x the inner integral runs over
         * the whole E_k'. */
        double sub[6 * NLO_MAXSUB], cpt[4 * 8], cw[8];
        int nc = 0;
        nlo_problem pr = *p;
        pr.ball = 1;
        int ns = nlo_region(&pr, bkp, Vk, sub, NLO_MAXSUB, cpt, cw, &nc);
        if (ns < 0) return ns;
        for (int q = 0; q < 64; q++) s0q[q] = 0.0;
        for (int t = 0; t < ns + nc; t++) {
            int npt = t < ns ? nq : 1;
            for (int q = 0; q < npt; q++) {
                double x[2], al[3], Wq, S0, S1[3], S2[9];
                if (t < ns) {
                    map_point(sub + 6 * t, lam + 3 * q, x);
                    Wq = w[q] * twice_area(sub + 6 * t);
                } else {
                    x[0] = cpt[2 * (t - ns)];
                    x[1] = cpt[2 * (t - ns) + 1];
                    Wq = cw[t - ns];
                }
                basis_at(Vk, x, al);
                int st = nlo_inner_sums(p, x, Vkp, &S0, S1, S2);
                if (st < 0) return st;
                for (int a = 0; a < 3; a++) {
                    for (int c = 0; c < 3; c++) mxx[3 * a + c] += Wq * al[a] * al[c] * S0;
                    for (int b = 0; b < 3; b++) mxy[3 * a + b] += Wq * al[a] * S1[b];
                }
                for (int i = 0; i < 9; i++) myy[i] += Wq * S2[i];
            }
        }
        nq = 0;
    }
    for (int q = 0; q < nq; q++) {
        double x[2], S0, S1[3], S2[9];
        map_point(Vk, lam + 3 * q, x);
        int st;
        if (p->ball == 3) {
            /* shifted ball (Sec. 4.3): the inner region is E_k' n B_delta(b_k)
             * for every outer point (constant kernel) */
            nlo_problem pr = *p;
            pr.ball = 1;
            st = nlo_inner_sums(&pr, bk, Vkp, &S0, S1, S2);
        } else {
            st = nlo_inner_sums(p, x, Vkp, &S0, S1, S2);
        }
        if (st < 0) return st;
        double Wq = w[q] * ak2;
        const double *al = lam + 3 * q;
        if (q < 64) s0q[q] = S0;
        for (int a = 0; a < 3; a++) {
            for (int c = 0; c < 3; c++) mxx[3 * a + c] += Wq * al[a] * al[c] * S0;
            for (int b = 0; b < 3; b++) mxy[3 * a + b] += Wq * al[a] * S1[b];
        }
        for (int i = 0; i < 9; i++) myy[i] += Wq * S2[i];
    }
    for (int a = 0; a < 3; a++)
        for (int c = 0; c < 3; c++) {
            blk[6 * a + c] = mxx[3 * a + c];
            blk[6 * a + 3 + c] = -mxy[3 * a + c];
            blk[6 * (3 + c) + a] = -mxy[3 * a + c];
            blk[6 * (3 + a) + 3 + c] = myy[3 * a + c];
        }
    return 0;
}

/* ------------------------------------------------ pair lists */
typedef struct { double *b; double *r; double *V; } elemdata;

static elemdata elem_precompute(const nlo_mesh *m)
{
    elemdata e;
    e.b = (double *)malloc(sizeof(double) * 2 * m->nt);
    e.r = (double *)malloc(sizeof(double) * m->nt);
    e.V = (double *)malloc(sizeof(double) * 6 * m->nt);
    for (int k = 0; k < m->nt; k++) {
        tri_vertices(m, k, e.V + 6 * k);
        barycenter(e.V + 6 * k, e.b + 2 * k);
        e.r[k] = max_vertex_dist(e.V + 6 * k, e.b + 2 * k);
    }
    return e;
}

static void elem_free(elemdata *e) { free(e->b); free(e->r); free(e->V); }

static int pairs_of(const nlo_mesh *m, const nlo_problem *p, const elemdata *e, int k,
                    int32_t *kp, int32_t cap)
{
    int n = 0;
    for (int j = 0; j < m->nt; j++) {
        if (p->skip_ixi && !m->tri_in_omega[k] && !m->tri_in_omega[j]) continue;
        if (!maybe_pair(p, e->b + 2 * k, e->r[k], e->b + 2 * j, e->r[j])) continue;
        if (!pair_interacts(p, e->V + 6 * k, e->b + 2 * k, e->V + 6 * j, e->b + 2 * j)) continue;
        if (n < cap) kp[n] = j;
        n++;
    }
    return n;
}

/* all k' interacting with outer element k, ascending (task 2 of Sec. 7.1 done
 * as an all-elements loop) */
int nlo_pairs_of(const nlo_mesh *m, const nlo_problem *p, int32_t k, int32_t *kp, int32_t cap)
{
    elemdata e = elem_precompute(m);
    int n = pairs_of(m, p, &e, k, kp, cap);
    elem_free(&e);
    return n;
}

/* ------------------------------------------------ assembly */
struct nlo_result {
    int64_t n_pairs, nnz;
    int32_t status, nv, nt;
    int64_t *pair_ptr;
    int32_t *pair_kp;
    int64_t *rowptr;
    int32_t *col;
    double *val;
};

static int64_t find_col(const int64_t *rowptr, const int32_t *col, int r, int c)
{
    int64_t lo = rowptr[r], hi = rowptr[r + 1] - 1;
    while (lo <= hi) {
        int64_t mid = (lo + hi) / 2;
        if (col[mid] == c) return mid;
        if (col[mid] < c) lo = mid + 1; else hi = mid - 1;
    }
    return -1;
}

/* Neumaier's compensated summation step */
static void neumaier_add(double *s, double *c, double v)
{
    double t = *s + v;
    if (fabs(*s) >= fabs(v)) *c += (*s - t) + v;
    else *c += (v - t) + *s;
    *s = t;
}

nlo_result *nlo_assemble(const nlo_mesh *m, const nlo_problem *p, int32_t nthreads)
{
    nlo_result *r = (nlo_result *)calloc(1, sizeof(nlo_result));
    r->nv = m->nv;
    r->nt = m->nt;
    int K = m->nt, J = m->nv;
    elemdata e = elem_precompute(m);
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
    /* pass 1: pair counts, then the canonical (k asc, k' asc) list */
    int32_t *cnt = (int32_t *)calloc(K, sizeof(int32_t));
#pragma omp parallel for schedule(dynamic, 16)
    for (int k = 0; k < K; k++) cnt[k] = pairs_of(m, p, &e, k, NULL, 0);
    r->pair_ptr = (int64_t *)malloc(sizeof(int64_t) * (K + 1));
    r->pair_ptr[0] = 0;
    for (int k = 0; k < K; k++) r->pair_ptr[k + 1] = r->pair_ptr[k] + cnt[k];
    r->n_pairs = r->pair_ptr[K];
    r->pair_kp = (int32_t *)malloc(sizeof(int32_t) * (r->n_pairs > 0 ? r->n_pairs : 1));
#pragma omp parallel for schedule(dynamic, 16)
    for (int k = 0; k < K; k++) pairs_of(m, p, &e, k, r->pair_kp + r->pair_ptr[k], cnt[k]);
    free(cnt);
    /* pattern: every node pair of E_k x E_k' in both orders (a dense bitmap of
     * the J x J index set, then CSR) */
    int64_t words = ((int64_t)J * J + 63) / 64;
    uint64_t *bits = (uint64_t *)calloc(words, sizeof(uint64_t));
    for (int k = 0; k < K; k++)
        for (int64_t t = r->pair_ptr[k]; t < r->pair_ptr[k + 1]; t++) {
            int kp = r->pair_kp[t];
            int g[6];
            for (int a = 0; a < 3; a++) { g[a] = m->tri[3 * k + a]; g[3 + a] = m->tri[3 * kp + a]; }
            for (int i = 0; i < 6; i++)
                for (int j = 0; j < 6; j++) {
                    int64_t bit = (int64_t)g[i] * J + g[j];
                    bits[bit >> 6] |= (uint64_t)1 << (bit & 63);
                }
        }
    r->rowptr = (int64_t *)calloc(J + 1, sizeof(int64_t));
    int64_t nnz = 0;
    for (int i = 0; i < J; i++) {
        for (int j = 0; j < J; j++) {
            int64_t bit = (int64_t)i * J + j;
            if (bits[bit >> 6] >> (bit & 63) & 1) nnz++;
        }
        r->rowptr[i + 1] = nnz;
    }
    r->nnz = nnz;
    r->col = (int32_t *)malloc(sizeof(int32_t) * (nnz > 0 ? nnz : 1));
    nnz = 0;
    for (int i = 0; i < J; i++)
        for (int j = 0; j < J; j++) {
            int64_t bit = (int64_t)i * J + j;
            if (bits[bit >> 6] >> (bit & 63) & 1) r->col[nnz++] = j;
        }
    free(bits);
    /* values: blocks computed in parallel chunks of outer elements, then added
     * serially in (k, k', i, j) order with Neumaier compensation */
    double *sum = (double *)calloc(nnz > 0 ? nnz : 1, sizeof(double));
    double *cmp = (double *)calloc(nnz > 0 ? nnz : 1, sizeof(double));
    const int CH = 256;
    int status = 0;
    for (int k0 = 0; k0 < K; k0 += CH) {
        int k1 = k0 + CH < K ? k0 + CH : K;
        int64_t base = r->pair_ptr[k0], np = r->pair_ptr[k1] - base;
        double *blks = (double *)malloc(sizeof(double) * 36 * (np > 0 ? np : 1));
#pragma omp parallel for schedule(dynamic, 1)
        for (int k = k0; k < k1; k++)
            for (int64_t t = r->pair_ptr[k]; t < r->pair_ptr[k + 1]; t++) {
                double mxy[9], myy[9], s0q[64];
                int st = nlo_pair_block(m, p, k, r->pair_kp[t], mxy, myy, s0q, blks + 36 * (t - base));
                if (st < 0) {
#pragma omp critical
                    status = st;
                }
            }
        for (int k = k0; k < k1; k++)
            for (int64_t t = r->pair_ptr[k]; t < r->pair_ptr[k + 1]; t++) {
                int kp = r->pair_kp[t];
                int g[6];
                for (int a = 0; a < 3; a++) { g[a] = m->tri[3 * k + a]; g[3 + a] = m->tri[3 * kp + a]; }
                const double *B = blks + 36 * (t - base);
                for (int i = 0; i < 6; i++)
                    for (int j = 0; j < 6; j++) {
                        int64_t at = find_col(r->rowptr, r->col, g[i], g[j]);
                        neumaier_add(&sum[at], &cmp[at], B[6 * i + j]);
                    }
            }
        free(blks);
    }
    r->val = (double *)malloc(sizeof(double) * (nnz > 0 ? nnz : 1));
    for (int64_t i = 0; i < nnz; i++) r->val[i] = sum[i] + cmp[i];
    free(sum);
    free(cmp);
    elem_free(&e);
    r->status = status;
    return r;
}

void nlo_result_sizes(const nlo_result *r, int64_t *n_pairs, int64_t *nnz, int32_t *status)
{
    *n_pairs = r->n_pairs;
    *nnz = r->nnz;
    *status = r->status;
}

void nlo_result_copy(const nlo_result *r, int64_t *pair_ptr, int32_t *pair_kp,
                     int64_t *rowptr, int32_t *col, double *val)
{
    if (pair_ptr) memcpy(pair_ptr, r->pair_ptr, sizeof(int64_t) * (r->nt + 1));
    if (pair_kp) memcpy(pair_kp, r->pair_kp, sizeof(int32_t) * r->n_pairs);
    if (rowptr) memcpy(rowptr, r->rowptr, sizeof(int64_t) * (r->nv + 1));
    if (col) memcpy(col, r->col, sizeof(int32_t) * r->nnz);
    if (val) memcpy(val, r->val, sizeof(double) * r->nnz);
}

void nlo_result_free(nlo_result *r)
{
    if (!r) return;
    free(r->pair_ptr); free(r->pair_kp); free(r->rowptr); free(r->col); free(r->val);
    free(r);
}

/* one row D[j, :] of the full matrix, from every pair with node j in E_k or
 * E_k'; columns ascending.  Returns the number of columns or a negative status. */
int nlo_row(const nlo_mesh *m, const nlo_problem *p, int32_t j, int32_t *cols, double *vals,
            int32_t cap)
{
    int K = m->nt, J = m->nv;
    elemdata e = elem_precompute(m);
    double *sum = (double *)calloc(J, sizeof(double));
    double *cmp = (double *)calloc(J, sizeof(double));
    uint8_t *hit = (uint8_t *)calloc(J, 1);
    int32_t *kp = (int32_t *)malloc(sizeof(int32_t) * K);
    /* the elements with node j, ascending (listed once: the same order as a scan) */
    int32_t *jel = (int32_t *)malloc(sizeof(int32_t) * K);
    int nj = 0;
    for (int kk = 0; kk < K; kk++)
        for (int a = 0; a < 3; a++)
            if (m->tri[3 * kk + a] == j) { jel[nj++] = kk; break; }
    int status = 0;
    for (int k = 0; k < K && status == 0; k++) {
        int kin = 0;
        for (int a = 0; a < 3; a++) kin |= m->tri[3 * k + a] == j;
        if (!kin) {
            /* pairs (k, k') with j a node of E_k' only */
            for (int ij = 0; ij < nj; ij++) {
                const int kk = jel[ij];
                if (p->skip_ixi && !m->tri_in_omega[k] && !m->tri_in_omega[kk]) continue;
                if (!maybe_pair(p, e.b + 2 * k, e.r[k], e.b + 2 * kk, e.r[kk])) continue;
                if (!pair_interacts(p, e.V + 6 * k, e.b + 2 * k, e.V + 6 * kk, e.b + 2 * kk)) continue;
                double mxy[9], myy[9], s0q[64], B[36];
                int st = nlo_pair_block(m, p, k, kk, mxy, myy, s0q, B);
                if (st < 0) { status = st; break; }
                int g[6];
                for (int a = 0; a < 3; a++) { g[a] = m->tri[3 * k + a]; g[3 + a] = m->tri[3 * kk + a]; }
                for (int i = 3; i < 6; i++) {
                    if (g[i] != j) continue;
                    for (int c = 0; c < 6; c++) { neumaier_add(&sum[g[c]], &cmp[g[c]], B[6 * i + c]); hit[g[c]] = 1; }
                }
            }
            continue;
        }
        int n = pairs_of(m, p, &e, k, kp, K);
        for (int t = 0; t < n; t++) {
            double mxy[9], myy[9], s0q[64], B[36];
            int st = nlo_pair_block(m, p, k, kp[t], mxy, myy, s0q, B);
            if (st < 0) { status = st; break; }
            int g[6];
            for (int a = 0; a < 3; a++) { g[a] = m->tri[3 * k + a]; g[3 + a] = m->tri[3 * kp[t] + a]; }
            for (int i = 0; i < 6; i++) {
                if (g[i] != j) continue;
                for (int c = 0; c < 6; c++) { neumaier_add(&sum[g[c]], &cmp[g[c]], B[6 * i + c]); hit[g[c]] = 1; }
            }
        }
    }
    int nc = 0;
    for (int c = 0; c < J; c++)
        if (hit[c]) {
            if (nc < cap) { cols[nc] = c; vals[nc] = sum[c] + cmp[c]; }
            nc++;
        }
    free(sum); free(cmp); free(hit); free(kp); free(jel);
    elem_free(&e);
    return status < 0 ? status : nc;
}

/* G_j = sum over elements of Omega of sum_q W_q phi_j(x_q) f(x_q) (Eq. (lfunchj)),
 * f given at the outer points of the main outer rule, f_outer[k][q]. */
void nlo_load(const nlo_mesh *m, const nlo_problem *p, const double *f_outer, double *G)
{
    for (int j = 0; j < m->nv; j++) G[j] = 0.0;
    for (int k = 0; k < m->nt; k++) {
        if (!m->tri_in_omega[k]) continue;
        double V[6];
        tri_vertices(m, k, V);
        double a2 = twice_area(V);
        for (int q = 0; q < p->n_out; q++) {
            const double *al = p->out_lam + 3 * q;
            double Wq = p->out_w[q] * a2;
            for (int a = 0; a < 3; a++) G[m->tri[3 * k + a]] += Wq * al[a] * f_outer[(int64_t)k * p->n_out + q];
        }
    }
}

void nlo_outer_points(const nlo_mesh *m, const nlo_problem *p, double *xq)
{
    for (int k = 0; k < m->nt; k++) {
        double V[6];
        tri_vertices(m, k, V);
        for (int q = 0; q < p->n_out; q++) map_point(V, p->out_lam + 3 * q, xq + 2 * ((int64_t)k * p->n_out + q));
    }
}

/* Work census over outer elements [k0, k1): counts of
 * out[0] pairs, [1] whole items, [2] partial items, [3] empty items,
 * [4] polygon (fan) triangles, [5] caps, [6] cap triangles, [7] inner points. */
int64_t nlo_flops_census(const nlo_mesh *m, const nlo_problem *p, int32_t k0, int32_t k1, int64_t out[8])
{
    for (int i = 0; i < 8; i++) out[i] = 0;
    elemdata e = elem_precompute(m);
    int32_t *kp = (int32_t *)malloc(sizeof(int32_t) * m->nt);
    double dd = p->delta * p->delta;
    for (int k = k0; k < k1; k++) {
        int n = pairs_of(m, p, &e, k, kp, m->nt);
        out[0] += n;
        if (p->ball >= 2) continue;     /* item counts for the barycenter and intersection balls only */
        for (int t = 0; t < n; t++) {
            const double *Vk = e.V + 6 * k, *Vj = e.V + 6 * kp[t];
            for (int q = 0; q < p->n_out; q++) {
                double x[2];
                map_point(Vk, p->out_lam + 3 * q, x);
                if (p->ball == 0) {
                    if (bary_in(x, e.b + 2 * kp[t], dd)) { out[1]++; out[4]++; out[7] += p->n_in; }
                    else out[3]++;
                    continue;
                }
                int nin = 0;
                for (int a = 0; a < 3; a++) {
                    double dx = Vj[2 * a] - x[0], dy = Vj[2 * a + 1] - x[1];
                    nin += dx * dx + dy * dy <= dd;
                }
                if (nin == 3) { out[1]++; out[4]++; out[7] += p->n_in; continue; }
                rpoint P[12];
                int np_ = build_polygon(x, Vj, dd, P);
                if (np_ == 0) { out[3]++; continue; }
                out[2]++;
                if (np_ >= 3) { out[4] += np_ - 2; out[7] += (int64_t)(np_ - 2) * p->n_in; }
                for (int i = 0; i < np_; i++)
                    if (P[i].type == 2 && P[(i + 1) % np_].type == 1) {
                        out[5]++;
                        out[6] += p->cap_edges;
                        out[7] += (int64_t)p->cap_edges * p->n_in;
                    }
            }
        }
    }
    free(kp);
    elem_free(&e);
    return out[0];
}

/* Pair lists and local blocks of the outer elements [k0, k1), threads over
 * k; returns the number of pairs and a checksum of the blocks.  Used to time
 * the oracle on a bounded sample of a workload. */
int64_t nlo_blocks_range(const nlo_mesh *m, const nlo_problem *p, int32_t k0, int32_t k1, int32_t nthreads,
                         double *checksum)
{
    elemdata e = elem_precompute(m);
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
    int64_t total = 0;
    double cs = 0.0;
#pragma omp parallel for schedule(dynamic, 1) reduction(+ : total, cs)
    for (int k = k0; k < k1; k++) {
        int32_t *kp = (int32_t *)malloc(sizeof(int32_t) * m->nt);
        int n = pairs_of(m, p, &e, k, kp, m->nt);
        for (int t = 0; t < n; t++) {
            double mxy[9], myy[9], s0q[64], blk[36];
            nlo_pair_block(m, p, k, kp[t], mxy, myy, s0q, blk);
            cs += blk[0] + blk[9];
        }
        total += n;
        free(kp);
    }
    elem_free(&e);
    *checksum = cs;
    return total;
}
