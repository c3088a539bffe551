/*
 * nlo_mlp.c - oracle for the learned cap corrector.  TEST INFRASTRUCTURE ONLY.
 *
 * The paper integrates the circular caps left over by the inscribed polygon
 * either with triangles over equal arcs (Sec. 4.2.2) or with a one-point
 * centroid rule (Sec. 5.2, Eq. (cqr3)).  The learned corrector replaces the
 * former for items far from tangency by a small network that predicts the
 * three basis-weighted cap integrals
 *     m_b = (1/delta^2) int_{caps in E_k'} beta_b(y) dy,    b = 0, 1, 2,
 * from the inner-triangle vertices relative to the outer point, scaled by
 * 1/delta.  The second moments follow from the one-point centroid closure of
 * Sec. 5.2: all cap mass at the point where beta = m / sum(m), i.e.
 *     S0 += kc sum(m),  S1_b += kc m_b,  S2_bc += kc m_b m_c / sum(m)
 * (times delta^2), which keeps each item's contribution positive semidefinite.
 *
 * Network input: the vertices in a frame centred at x and rotated so that the
 * triangle's centroid lies on the positive first axis (the cap integrals do
 * not change under that rotation), shifted by the horizon and magnified by 8
 * (the element size of the h = delta/8 family):
 *     f_a = 8 (R(-phi) (v_a - x)/delta - (1, 0)),  phi = angle of the centroid.
 * Network (FP64 here): 6 -> 128 -> 128 -> 3 with the tanh form of GELU,
 *     g(z) = z/2 (1 + tanh(sqrt(2/pi) (z + 0.044715 z^3))),
 * weights in one flat array: W1[128][6], b1[128], W2[128][128], b2[128],
 * W3[3][128], b3[3] (row = output unit).
 *
 * Labels: the cap pieces of the region of Sec. 4.2.2 (the triangles that the
 * arc subdivision adds to the fan of the inscribed polygon), integrated
 * exactly (a linear function over a triangle is its centroid value times the
 * area).
 *
 * Parity pins: tests/test_oracle_mlp.py (finite differences of the forward
 * pass against the backward pass; the saturated-GELU affine special case
 * against a matrix product; the tanh-GELU against the erf-GELU within the
 * approximation's error; cap labels against the shoelace area and centroid of
 * the 8-arc cap polygon; routing band; the closure against the centroid
 * rule at the shoelace centroid of the 8-arc cap polygons).
 */
#include "nlo.h"
#include <math.h>
#include <string.h>

#define HID NLO_MLP_HIDDEN
#define OFF_W1 0
#define OFF_B1 (OFF_W1 + HID * 6)
#define OFF_W2 (OFF_B1 + HID)
#define OFF_B2 (OFF_W2 + HID * HID)
#define OFF_W3 (OFF_B2 + HID)
#define OFF_B3 (OFF_W3 + 3 * HID)

static const double GC = 0.79788456080286535588;   /* sqrt(2/pi) */
static const double GA = 0.044715;

double nlo_gelu(double z)
{
    return 0.5 * z * (1.0 + tanh(GC * (z + GA * z * z * z)));
}

static double gelu_d(double z)
{
    double t = tanh(GC * (z + GA * z * z * z));
    return 0.5 * (1.0 + t) + 0.5 * z * (1.0 - t * t) * GC * (1.0 + 3.0 * GA * z * z);
}

static void forward1(const double *w, const double *f, double z1[HID], double h1[HID], double z2[HID],
                     double h2[HID], double y[3])
{
    for (int i = 0; i < HID; i++) {
        double s = w[OFF_B1 + i];
        for (int c = 0; c < 6; c++) s += w[OFF_W1 + 6 * i + c] * f[c];
        z1[i] = s;
        h1[i] = nlo_gelu(s);
    }
    for (int i = 0; i < HID; i++) {
        double s = w[OFF_B2 + i];
        for (int j = 0; j < HID; j++) s += w[OFF_W2 + HID * i + j] * h1[j];
        z2[i] = s;
        h2[i] = nlo_gelu(s);
    }
    for (int o = 0; o < 3; o++) {
        double s = w[OFF_B3 + o];
        for (int j = 0; j < HID; j++) s += w[OFF_W3 + HID * o + j] * h2[j];
        y[o] = s;
    }
}

void nlo_mlp_forward(const double *w, const double *feat, int64_t n, double *out)
{
    double z1[HID], h1[HID], z2[HID], h2[HID];
    for (int64_t s = 0; s < n; s++) forward1(w, feat + 6 * s, z1, h1, z2, h2, out + 3 * s);
}

/* gradient of sum_s sum_o dout[s][o] y[s][o] with respect to every weight */
void nlo_mlp_backward(const double *w, const double *feat, const double *dout, int64_t n, double *dw)
{
    memset(dw, 0, sizeof(double) * NLO_MLP_NW);
    double z1[HID], h1[HID], z2[HID], h2[HID], y[3], dz2[HID], dz1[HID];
    for (int64_t s = 0; s < n; s++) {
        const double *f = feat + 6 * s, *dy = dout + 3 * s;
        forward1(w, f, z1, h1, z2, h2, y);
        for (int o = 0; o < 3; o++) {
            dw[OFF_B3 + o] += dy[o];
            for (int j = 0; j < HID; j++) dw[OFF_W3 + HID * o + j] += dy[o] * h2[j];
        }
        for (int j = 0; j < HID; j++) {
            double g = 0.0;
            for (int o = 0; o < 3; o++) g += w[OFF_W3 + HID * o + j] * dy[o];
            dz2[j] = g * gelu_d(z2[j]);
        }
        for (int i = 0; i < HID; i++) {
            dw[OFF_B2 + i] += dz2[i];
            for (int j = 0; j < HID; j++) dw[OFF_W2 + HID * i + j] += dz2[i] * h1[j];
        }
        for (int j = 0; j < HID; j++) {
            double g = 0.0;
            for (int i = 0; i < HID; i++) g += w[OFF_W2 + HID * i + j] * dz2[i];
            dz1[j] = g * gelu_d(z1[j]);
        }
        for (int i = 0; i < HID; i++) {
            dw[OFF_B1 + i] += dz1[i];
            for (int c = 0; c < 6; c++) dw[OFF_W1 + 6 * i + c] += dz1[i] * f[c];
        }
    }
}

/* int over the cap pieces of beta_b (E_k' basis), b = 0..2; returns the number
 * of cap triangles, or a negative status from the region builder */
int nlo_cap_moments(const nlo_problem *p, const double x[2], const double V[6], double m[3])
{
    double sub[6 * NLO_MAXSUB], cpt[16], cw[8];
    int nc = 0;
    m[0] = m[1] = m[2] = 0.0;
    nlo_problem p0 = *p;
    p0.cap_mode = 0;
    p0.cap_edges = 0;
    int npoly = nlo_region(&p0, x, V, sub, NLO_MAXSUB, cpt, cw, &nc);
    if (npoly < 0) return npoly;
    nlo_problem p1 = *p;
    p1.cap_mode = 0;
    int ns = nlo_region(&p1, x, V, sub, NLO_MAXSUB, cpt, cw, &nc);
    if (ns < 0) return ns;
    /* the region lists the polygon fan first, then the cap triangles */
    const double det = (V[2] - V[0]) * (V[5] - V[1]) - (V[3] - V[1]) * (V[4] - V[0]);
    for (int t = npoly; t < ns; t++) {
        const double *T = sub + 6 * t;
        double a = 0.5 * fabs((T[2] - T[0]) * (T[5] - T[1]) - (T[3] - T[1]) * (T[4] - T[0]));
        double cx = (T[0] + T[2] + T[4]) / 3.0, cy = (T[1] + T[3] + T[5]) / 3.0;
        double b1 = ((cx - V[0]) * (V[5] - V[1]) - (cy - V[1]) * (V[4] - V[0])) / det;
        double b2 = ((V[2] - V[0]) * (cy - V[1]) - (V[3] - V[1]) * (cx - V[0])) / det;
        m[0] += a * (1.0 - b1 - b2);
        m[1] += a * b1;
        m[2] += a * b2;
    }
    return ns - npoly;
}

/* the network input of (x, E_k') */
void nlo_mlp_features(const double x[2], const double V[6], double delta, double f[6])
{
    double cx = ((V[0] + V[2]) + V[4]) / 3.0 - x[0], cy = ((V[1] + V[3]) + V[5]) / 3.0 - x[1];
    double r = sqrt(cx * cx + cy * cy);
    double c = r > 0.0 ? cx / r : 1.0, s = r > 0.0 ? cy / r : 0.0;
    for (int a = 0; a < 3; a++) {
        double dx = (V[2 * a] - x[0]) / delta, dy = (V[2 * a + 1] - x[1]) / delta;
        f[2 * a] = 8.0 * ((dx * c + dy * s) - 1.0);
        f[2 * a + 1] = 8.0 * (dy * c - dx * s);
    }
}

/* learned routing: far enough from tangency, | |v_a - x| - delta | >= band delta
 * for every vertex, i.e. |v_a - x|^2 >= (delta (1 + band))^2 or
 * |v_a - x|^2 <= (delta (1 - band))^2 (no square root) */
int nlo_routed(double delta, double band, const double x[2], const double V[6])
{
    double hi = delta * (1.0 + band), lo = band < 1.0 ? delta * (1.0 - band) : 0.0;
    double hi2 = hi * hi, lo2 = lo * lo;
    for (int a = 0; a < 3; a++) {
        double dx = V[2 * a] - x[0], dy = V[2 * a + 1] - x[1];
        double d2 = dx * dx + dy * dy;
        if (!(d2 >= hi2 || d2 <= lo2)) return 0;
    }
    return 1;
}

/* the item inside the network's training domain {rlo, rhi, elo, ehi}: every
 * squared vertex distance |v_a - x|^2 within [rlo, rhi] delta^2 and every
 * squared edge length within [elo, ehi] delta^2; dom = NULL is unbounded */
int nlo_in_domain(const double *dom, const double x[2], const double V[6], double delta)
{
    if (!dom) return 1;
    double dd = delta * delta;
    double rlo = dom[0] * dd, rhi = dom[1] * dd, elo = dom[2] * dd, ehi = dom[3] * dd;
    for (int a = 0; a < 3; a++) {
        int b = (a + 1) % 3;
        double dx = V[2 * a] - x[0], dy = V[2 * a + 1] - x[1];
        double d2 = dx * dx + dy * dy;
        double ex = V[2 * b] - V[2 * a], ey = V[2 * b + 1] - V[2 * a + 1];
        double e2 = ex * ex + ey * ey;
        if (!(d2 >= rlo && d2 <= rhi && e2 >= elo && e2 <= ehi)) return 0;
    }
    return 1;
}

/* the learned cap contribution of a routed partial item (constant kernel) */
int nlo_learned_caps(const nlo_problem *p, const double x[2], const double V[6], double s0[1], double s1[3],
                     double s2[9])
{
    if (p->kernel != 0 || !p->mlp_w) return -4;
    double f[6], y[3];
    nlo_mlp_features(x, V, p->delta, f);
    nlo_mlp_forward(p->mlp_w, f, 1, y);
    double m[3], sm = 0.0;
    for (int b = 0; b < 3; b++) {
        m[b] = (y[b] > 0.0 ? y[b] : 0.0) * p->mlp_scale * p->delta * p->delta;
        sm += m[b];
    }
    s0[0] += p->kc * sm;
    for (int b = 0; b < 3; b++) {
        s1[b] += p->kc * m[b];
        if (sm > 0.0)
            for (int c = 0; c < 3; c++) s2[3 * b + c] += p->kc * m[b] * m[c] / sm;
    }
    return 0;
}

/* One training candidate from ten uniforms, in units of delta around x = 0:
 * a right triangle of legs L = h/delta from one of the four halves of a grid
 * cell (both diagonals), the cell centre at distance 1 + (2 u1 - 1) sqrt(2) L
 * in direction 2 pi u2, every vertex jittered by jitter*L*(2u - 1) per
 * coordinate, vertex order rotated cyclically by floor(3 u9).  Valid when the
 * ball cuts the triangle (at least one cap) and the item is routed.  Returns
 * 1 (valid) or 0; verts = the vertices, feat = the network input, label = the
 * cap moments (delta = 1). */
int nlo_cap_candidate(const double u[10], double L, double jitter, double band, int32_t cap_edges,
                      double verts[6], double feat[6], double label[3])
{
    static const double shapes[4][6] = {{0, 0, 1, 0, 1, 1}, {0, 0, 1, 1, 0, 1}, {0, 0, 1, 0, 0, 1},
                                        {1, 0, 1, 1, 0, 1}};
    int s = (int)(4.0 * u[0]);
    if (s > 3) s = 3;
    double r = 1.0 + (2.0 * u[1] - 1.0) * sqrt(2.0) * L;
    double ph = 2.0 * 3.14159265358979323846 * u[2];
    double ox = r * cos(ph) - 0.5 * L, oy = r * sin(ph) - 0.5 * L;
    double V[6];
    for (int a = 0; a < 3; a++) {
        V[2 * a] = ox + L * shapes[s][2 * a] + jitter * L * (2.0 * u[3 + 2 * a] - 1.0);
        V[2 * a + 1] = oy + L * shapes[s][2 * a + 1] + jitter * L * (2.0 * u[4 + 2 * a] - 1.0);
    }
    int rot = (int)(3.0 * u[9]);
    if (rot > 2) rot = 2;
    for (int a = 0; a < 3; a++) {
        int b = (a + rot) % 3;
        verts[2 * a] = V[2 * b];
        verts[2 * a + 1] = V[2 * b + 1];
    }
    const double x0[2] = {0.0, 0.0};
    nlo_mlp_features(x0, verts, 1.0, feat);
    nlo_problem p;
    memset(&p, 0, sizeof p);
    p.delta = 1.0;
    p.kc = 1.0;
    p.ball = 1;
    p.cap_edges = cap_edges;
    int nc = nlo_cap_moments(&p, x0, verts, label);
    if (nc <= 0) return 0;
    return nlo_routed(1.0, band, x0, verts);
}
