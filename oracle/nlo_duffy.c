/*
 * nlo_duffy.c - oracle for element pairs that share a vertex under the
 * singular kernel psi = kc |x-y|^-(2+2s).  TEST INFRASTRUCTURE ONLY.
 *
 * The paper restricts itself to integrable kernels and leaves singular
 * quadrature to the literature (Sec. 3, remark on singular kernels); this is
 * the reading used here.  For a pair (k, k') sharing one, two or three
 * vertices, the split of the integrand into S0, S1, S2 is not finite for
 * k = k', so the local block is formed from the merged differences
 *   d_i(x,y) = phi_g(i)(x) - phi_g(i)(y)       (slot a of E_k, node also in E_k' or not)
 *   d_i(x,y) = -beta_b(y)                      (slot b of E_k' whose node is not in E_k)
 *   d_i = 0                                    (slot b of E_k' whose node is in E_k: merged)
 * and blk_ij = int_{E_k} int_{E_k' n B_delta(x)} d_i d_j psi dy dx, which
 * scatters into D exactly like the regular block (the node-level sums are
 * the same), but every entry is finite.
 *
 * Quadrature (a radial, Duffy-type substitution):
 *   outer: E_k collapsed at vertex c (the shared vertex for one shared
 *     vertex, the unshared vertex for a shared edge, vertex 0 for k = k'):
 *     x = v_c + s((1-w)(v_c1 - v_c) + w(v_c2 - v_c)), weight 2|E_k| s, tensor
 *     Gauss-Legendre of order n in s and w;
 *   inner: polar coordinates y = x + r (cos t, sin t) around x; the angle
 *     range covered by E_k' is cut at the directions of its vertices, each
 *     piece gets Gauss-Legendre of order n in u with t = u^2 (3 - 2u) mapped
 *     onto the piece (points clustered at its ends); along a ray d_i = c_i + e_i r,
 *     so d_i d_j psi r = kc (c_i c_j r^(-1-2s) + (c_i e_j + e_i c_j) r^(-2s)
 *     + e_i e_j r^(1-2s)) is integrated in closed form between the entry and
 *     exit radii of the ray (the exit radius capped at delta: the exact ball).
 */
#include "nlo.h"
#include <math.h>
#include <string.h>

static const double DPI = 3.14159265358979323846;

static void verts(const nlo_mesh *m, int k, double V[6])
{
    for (int a = 0; a < 3; a++) {
        int j = m->tri[3 * k + a];
        V[2 * a] = m->xy[2 * j];
        V[2 * a + 1] = m->xy[2 * j + 1];
    }
}

/* barycentric coordinates and their gradient for triangle V at point y */
static void bary(const double V[6], const double y[2], double b[3], double gx[3], double gy[3])
{
    double det = (V[2] - V[0]) * (V[5] - V[1]) - (V[3] - V[1]) * (V[4] - V[0]);
    b[1] = ((y[0] - V[0]) * (V[5] - V[1]) - (y[1] - V[1]) * (V[4] - V[0])) / det;
    b[2] = ((V[2] - V[0]) * (y[1] - V[1]) - (V[3] - V[1]) * (y[0] - V[0])) / det;
    b[0] = 1.0 - b[1] - b[2];
    gx[1] = (V[5] - V[1]) / det;
    gy[1] = -(V[4] - V[0]) / det;
    gx[2] = -(V[3] - V[1]) / det;
    gy[2] = (V[2] - V[0]) / det;
    gx[0] = -gx[1] - gx[2];
    gy[0] = -gy[1] - gy[2];
}

/* int_{r0}^{r1} kc r^(m - 1 - 2s) dr */
static double radial(double kc, double s, int m, double r0, double r1)
{
    double p = (double)m - 2.0 * s;
    if (fabs(p) < 1e-14) return kc * log(r1 / r0);
    return kc * (pow(r1, p) - pow(r0, p)) / p;
}

int nlo_duffy_block(const nlo_mesh *m, const nlo_problem *p, int k, int kp, double blk[36])
{
    const int n = p->duffy_n;
    if (n < 1 || !p->gl_x || !p->gl_w) return -3;
    double Vk[6], Vp[6];
    verts(m, k, Vk);
    verts(m, kp, Vp);
    int sb[3], bshared[3] = {0, 0, 0}, nshared = 0;
    for (int a = 0; a < 3; a++) {
        sb[a] = -1;
        for (int b = 0; b < 3; b++)
            if (m->tri[3 * k + a] == m->tri[3 * kp + b]) {
                sb[a] = b;
                bshared[b] = 1;
                nshared++;
            }
    }
    const int identical = nshared == 3;
    int c = 0;
    if (nshared == 1) {
        for (int a = 0; a < 3; a++)
            if (sb[a] >= 0) c = a;
    } else if (nshared == 2) {
        for (int a = 0; a < 3; a++)
            if (sb[a] < 0) c = a;
    }
    const int c1 = (c + 1) % 3, c2 = (c + 2) % 3;
    const double a2k = fabs((Vk[2] - Vk[0]) * (Vk[5] - Vk[1]) - (Vk[3] - Vk[1]) * (Vk[4] - Vk[0]));
    const double dd = p->delta;
    for (int i = 0; i < 36; i++) blk[i] = 0.0;
    for (int is = 0; is < n; is++)
        for (int iw = 0; iw < n; iw++) {
            const double sv = p->gl_x[is], wv = p->gl_x[iw];
            const double Wx = p->gl_w[is] * p->gl_w[iw] * a2k * sv;
            double x[2];
            for (int d = 0; d < 2; d++)
                x[d] = Vk[2 * c + d] + sv * ((1.0 - wv) * (Vk[2 * c1 + d] - Vk[2 * c + d]) +
                                             wv * (Vk[2 * c2 + d] - Vk[2 * c + d]));
            double al[3], agx[3], agy[3], be[3], bgx[3], bgy[3];
            bary(Vk, x, al, agx, agy);
            bary(Vp, x, be, bgx, bgy);   /* affine extension of E_k' basis at x */
            /* vertex directions of E_k' from x and the angular pieces */
            double ang[3];
            for (int b = 0; b < 3; b++) ang[b] = atan2(Vp[2 * b + 1] - x[1], Vp[2 * b] - x[0]);
            for (int i = 0; i < 2; i++)          /* sort three values */
                for (int j = 0; j < 2 - i; j++)
                    if (ang[j] > ang[j + 1]) { double t = ang[j]; ang[j] = ang[j + 1]; ang[j + 1] = t; }
            double lo[3], hi[3];
            int npc = 0;
            if (identical) {
                lo[0] = ang[0]; hi[0] = ang[1];
                lo[1] = ang[1]; hi[1] = ang[2];
                lo[2] = ang[2]; hi[2] = ang[0] + 2.0 * DPI;
                npc = 3;
            } else {
                double g0 = ang[1] - ang[0], g1 = ang[2] - ang[1], g2 = ang[0] + 2.0 * DPI - ang[2];
                if (g2 >= g0 && g2 >= g1) {
                    lo[0] = ang[0]; hi[0] = ang[1]; lo[1] = ang[1]; hi[1] = ang[2];
                } else if (g0 >= g1) {
                    lo[0] = ang[1]; hi[0] = ang[2]; lo[1] = ang[2]; hi[1] = ang[0] + 2.0 * DPI;
                } else {
                    lo[0] = ang[2]; hi[0] = ang[0] + 2.0 * DPI; lo[1] = ang[0] + 2.0 * DPI; hi[1] = ang[1] + 2.0 * DPI;
                }
                npc = 2;
            }
            /* constant parts c_i of the merged differences at y = x */
            double c0[6], gxs[6], gys[6];
            for (int a = 0; a < 3; a++) {
                if (sb[a] >= 0) {
                    c0[a] = identical ? 0.0 : al[a] - be[sb[a]];
                    gxs[a] = -bgx[sb[a]];
                    gys[a] = -bgy[sb[a]];
                } else {
                    c0[a] = al[a];
                    gxs[a] = 0.0;
                    gys[a] = 0.0;
                }
            }
            for (int b = 0; b < 3; b++) {
                if (bshared[b]) {
                    c0[3 + b] = 0.0; gxs[3 + b] = 0.0; gys[3 + b] = 0.0;
                } else {
                    c0[3 + b] = -be[b]; gxs[3 + b] = -bgx[b]; gys[3 + b] = -bgy[b];
                }
            }
            for (int pc = 0; pc < npc; pc++)
                for (int it = 0; it < n; it++) {
                    /* angle clustered at both piece ends (where the entry or exit
                     * radius varies fastest): t = u^2 (3 - 2u), dt = 6u(1-u) du */
                    const double u = p->gl_x[it];
                    const double th = lo[pc] + (hi[pc] - lo[pc]) * (u * u * (3.0 - 2.0 * u));
                    const double wt = (hi[pc] - lo[pc]) * p->gl_w[it] * 6.0 * u * (1.0 - u);
                    const double ex = cos(th), ey = sin(th);
                    double rin = 0.0, rout = 1e300;
                    int empty = 0;
                    for (int a = 0; a < 3; a++) {
                        const int b = (a + 1) % 3;
                        const double nx = Vp[2 * b + 1] - Vp[2 * a + 1], ny = -(Vp[2 * b] - Vp[2 * a]);
                        const double f0 = nx * (x[0] - Vp[2 * a]) + ny * (x[1] - Vp[2 * a + 1]);
                        const double f1 = nx * ex + ny * ey;
                        if (f1 > 0.0) { double r = -f0 / f1; if (r < rout) rout = r; }
                        else if (f1 < 0.0) { double r = -f0 / f1; if (r > rin) rin = r; }
                        else if (f0 > 0.0) empty = 1;
                    }
                    if (rout > dd) rout = dd;
                    if (empty || !(rout > rin)) continue;
                    double J0 = 0.0, J1, J2;
                    if (rin > 0.0) J0 = radial(p->kc, p->ks, 0, rin, rout);
                    J1 = rin > 0.0 || 1.0 - 2.0 * p->ks > 0.0 ? radial(p->kc, p->ks, 1, rin, rout) : 0.0;
                    J2 = radial(p->kc, p->ks, 2, rin, rout);
                    double e[6];
                    for (int i = 0; i < 6; i++) e[i] = gxs[i] * ex + gys[i] * ey;
                    const double W = Wx * wt;
                    for (int i = 0; i < 6; i++)
                        for (int j = 0; j < 6; j++)
                            blk[6 * i + j] += W * (c0[i] * c0[j] * J0 + (c0[i] * e[j] + e[i] * c0[j]) * J1 +
                                                   e[i] * e[j] * J2);
                }
        }
    return 0;
}
