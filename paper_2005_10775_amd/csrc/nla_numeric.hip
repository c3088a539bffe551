// Numeric phase of libnlasm: pair quadrature, deterministic segmented sum
// into the CSR values of D, extraction of A = D[free,free] and the load vector.
#include "nla_internal.hpp"
#include <cmath>

static inline unsigned grid_for(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

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

// E' n B_delta(x) retriangulated (Sec. 4.2.1-4.2.2 and Sec. 7.1 tasks 3-6),
// written as one generator loop so that a single copy of the subtriangle
// quadrature is inlined.  The edges are walked v0->v1->v2: vertices inside
// the closed ball and the roots lambda in (0,1) of |v_a + lambda e - x|^2 =
// delta^2 (smaller root entry, larger exit) arrive in order; every new point
// closes the fan triangle (first, previous, new), and every exit followed by
// an entry (cyclically) opens a cap: the arc from exit X counter-clockwise to
// entry N split into ncap equal arcs fanned from the chord midpoint.  A cap
// span not in (0, pi] only arises from rounding when X and N coincide and is
// dropped (cross product <= 0).  POW2: ncap is a power of two and the
// rotation comes from half-angle steps instead of atan2/sincos.  Vl: E' in absolute coordinates (6 values); coordinates below are
// relative to the outer point.
template <bool SYM, bool POW2>
__device__ void partial_item(double xx, double xy, const double *Vl, double dd, int ncap, const RuleMom &M,
                             Acc &A, int &nsub)
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
    int ev = 0, cnt = 0, ft = 0, pt = 0, ea = 0, eb = 0;
    double f[5] = {0, 0, 0, 0, 0}, q[5] = {0, 0, 0, 0, 0};
    double epx = 0, epy = 0, eex = 0, eey = 0, el1 = 2.0, el2 = 2.0;
    int cj = 0;
    bool wrapped = false;
    double Mc[5] = {0, 0, 0, 0, 0}, u[5] = {0, 0, 0, 0, 0}, N[5] = {0, 0, 0, 0, 0};
    double cc = 1.0, ss = 0.0;
    auto start_cap = [&](const double (&X)[5], const double (&Y)[5]) {
        const double cr = X[0] * Y[1] - X[1] * Y[0], dt = X[0] * Y[0] + X[1] * Y[1];
        if (!(cr > 0.0) || ncap < 2) return;      // span in (0, pi): counter-clockwise from X to N
        if (POW2) {
            // rotation by D/ncap from cos D, sin D by repeated half angles:
            // cos(t/2) = sqrt((1 + cos t)/2), sin(t/2) = sin t / (2 cos(t/2))
            const double r = 1.0 / sqrt((X[0] * X[0] + X[1] * X[1]) * (Y[0] * Y[0] + Y[1] * Y[1]));
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
            Mc[i] = 0.5 * (X[i] + Y[i]);
            u[i] = X[i];
            N[i] = Y[i];
        }
        cj = 1;
        nsub += 1 << 16;
    };
    while (true) {
        double t[3][5];
        if (cj > 0) {
            double v[5];
            if (cj == ncap) {
#pragma unroll
                for (int i = 0; i < 5; i++) v[i] = N[i];
                cj = 0;
            } else {
                v[0] = cc * u[0] - ss * u[1];
                v[1] = ss * u[0] + cc * u[1];
                basis_at(B, v[0], v[1], v[2], v[3], v[4]);
                cj++;
            }
#pragma unroll
            for (int i = 0; i < 5; i++) {
                t[0][i] = Mc[i];
                t[1][i] = u[i];
                t[2][i] = v[i];
                u[i] = v[i];
            }
        } else {
            bool got = false;
            double n[5];
            int nt = 0;
            while (ev < 9 && !got) {
                const int a = ev / 3, kind = ev - 3 * (ev / 3);
                ev++;
                if (kind == 0) {
                    const int b = a == 2 ? 0 : a + 1;
                    const double ax = Vl[2 * a], ay = Vl[2 * a + 1];
                    epx = ax - xx;
                    epy = ay - xy;
                    eex = Vl[2 * b] - ax;
                    eey = Vl[2 * b + 1] - ay;
                    ea = a;
                    eb = b;
                    const double r2 = epx * epx + epy * epy;
                    const double L = eex * eex + eey * eey;
                    const double Bq = eex * epx + eey * epy;
                    const double disc = Bq * Bq - L * (r2 - dd);
                    el1 = 2.0;
                    el2 = 2.0;
                    if (disc > 0.0) {
                        const double sq = sqrt(disc);
                        const double l1 = (-Bq - sq) / L, l2 = (-Bq + sq) / L;
                        if (l1 > 0.0 && l1 < 1.0) el1 = l1;
                        if (l2 > 0.0 && l2 < 1.0) el2 = l2;
                    }
                    if (r2 <= dd) {
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
                if (!wrapped && cnt >= 2 && pt == 2 && ft == 1) {
                    wrapped = true;
                    start_cap(q, f);
                    continue;
                }
                break;
            }
            const bool fan = cnt >= 2;
            if (fan) {
#pragma unroll
                for (int i = 0; i < 5; i++) {
                    t[0][i] = f[i];
                    t[1][i] = q[i];
                    t[2][i] = n[i];
                }
            }
            if (cnt >= 1 && pt == 2 && nt == 1) start_cap(q, n);
            if (cnt == 0) {
#pragma unroll
                for (int i = 0; i < 5; i++) f[i] = n[i];
                ft = nt;
            }
#pragma unroll
            for (int i = 0; i < 5; i++) q[i] = n[i];
            pt = nt;
            cnt++;
            if (!fan) continue;
        }
        tri_accum<SYM>(t, M, A);
        nsub++;
    }
}

__device__ __forceinline__ bool meets_edges(double xx, double xy, const double (&V)[6], double dd)
{
    bool inside = true;
#pragma unroll
    for (int a = 0; a < 3; a++) {
        const int b = (a + 1) % 3;
        double ex = V[2 * b] - V[2 * a], ey = V[2 * b + 1] - V[2 * a + 1];
        double px = xx - V[2 * a], py = xy - V[2 * a + 1];
        if (ex * py - ey * px < 0.0) inside = false;
    }
    if (inside) return true;
#pragma unroll
    for (int a = 0; a < 3; a++) {
        const int b = (a + 1) % 3;
        double ex = V[2 * b] - V[2 * a], ey = V[2 * b + 1] - V[2 * a + 1];
        double px = xx - V[2 * a], py = xy - V[2 * a + 1];
        double t = ex * px + ey * py, L = ex * ex + ey * ey;
        if (t > 0.0 && t < L) {
            double c = ex * py - ey * px;
            if (c * c <= dd * L) return true;
        }
    }
    return false;
}

// One wavefront per outer element k (Eq. (bformhj) restricted to the pairs
// of k).  Phase 1: every lane takes one pair (k, k'), classifies its items
// (x_{k,q}, E_k') as whole / partial / empty; whole items (all of E_k' in the
// ball, or the barycenter inside for the barycenter ball) only add their
// outer weights, since with constant psi their inner sums are rule
// constants times |E_k'|.  Partial items are queued in LDS.  Phase 2: the
// wave takes queued items 64 at a time (dense, regardless of owner),
// retriangulates them, and each owner adds its items' sums in q order.
// Outputs: per pair Myy (6); per element Mxx (6) from the fixed-order lane
// reduction of sum_k' S0(x_q), and the row block R_k[a][c] = sum of -Mxy_ab
// over the pairs whose inner slot b is node C_k[c], reduced in LDS column by
// column in pair order (each column owned by one lane).
template <int NQ, bool SYM, bool POW2>
__global__ __launch_bounds__(64, 2) void k_pairs_const_fp64(const int64_t *__restrict__ pair_ptr,
                                                         const int32_t *__restrict__ pair_kp, ElemSoA E,
                                                         const double *__restrict__ xq, const RuleSet *__restrict__ R,
                                                         double dd, double psi, int ball, int ncap,
                                                         const int64_t *__restrict__ col_off,
                                                         const int32_t *__restrict__ colent_ptr,
                                                         const uint16_t *__restrict__ colent, double *__restrict__ Rout,
                                                         double *__restrict__ Cyy, double *__restrict__ Cxx,
                                                         int max_cols, unsigned long long *__restrict__ counters)
{
    extern __shared__ double dyn[];
    __shared__ double sW[NQ][4];
    __shared__ double sX[NQ][2];
    __shared__ double sV[64][7];
    __shared__ unsigned short queue[64 * NQ];
    // item results of a phase-2 round, later the chunk's -Mxy (never live together)
    __shared__ double res[64][10];
    double (*mxy_l)[10] = res;
    const int k = blockIdx.x, lane = threadIdx.x;
    const int nq = R->n_out;
    const double a2k = E.a2[k];
    if (lane < nq) {
        double W = R->out_w[lane] * a2k;
        sW[lane][0] = W;
        sW[lane][1] = W * R->out_lam[lane][0];
        sW[lane][2] = W * R->out_lam[lane][1];
        sW[lane][3] = W * R->out_lam[lane][2];
        sX[lane][0] = xq[2 * ((int64_t)k * nq + lane)];
        sX[lane][1] = xq[2 * ((int64_t)k * nq + lane) + 1];
    }
    __syncthreads();
    const RuleMom M = load_moments(R);
    const int64_t coff = col_off[k];
    const int nC = (int)(col_off[k + 1] - coff);
    double *R_l = dyn;                                  // [3][nC]
    int *cur_l = (int *)(dyn + 3 * (size_t)max_cols);   // [nC]
    for (int c = lane; c < nC; c += 64) {
        R_l[c] = 0.0;
        R_l[nC + c] = 0.0;
        R_l[2 * nC + c] = 0.0;
        cur_l[c] = colent_ptr[coff + c];
    }
    double m0[NQ];
#pragma unroll
    for (int q = 0; q < NQ; q++) m0[q] = 0.0;
    unsigned long long c_whole = 0, c_part = 0, c_empty = 0, c_sub = 0, c_cap = 0;
    const int64_t p0 = pair_ptr[k], p1 = pair_ptr[k + 1];
    for (int64_t base = p0; base < p1; base += 64) {
        const int64_t p = base + lane;
        const bool act = p < p1;
        double V[6] = {0, 0, 0, 0, 0, 0};
        double a2p = 0.0, bxp = 0.0, byp = 0.0;
        if (act) {
            int kp = pair_kp[p];
            V[0] = E.vx0[kp]; V[1] = E.vy0[kp]; V[2] = E.vx1[kp]; V[3] = E.vy1[kp]; V[4] = E.vx2[kp]; V[5] = E.vy2[kp];
            a2p = E.a2[kp];
            bxp = E.bx[kp];
            byp = E.by[kp];
        }
#pragma unroll
        for (int i = 0; i < 6; i++) sV[lane][i] = V[i];
        double ws = 0.0, aw[3] = {0.0, 0.0, 0.0};
        unsigned pmask = 0;
        if (act) {
#pragma unroll
            for (int q = 0; q < NQ; q++) {
                if (q >= nq) break;
                const double xx = sX[q][0], xy = sX[q][1];
                bool whole = false, part = false;
                if (ball == NLA_BALL_BARYCENTER) {
                    double dx = xx - bxp, dy = xy - byp;
                    whole = dx * dx + dy * dy <= dd;
                } else {
                    int nin = 0;
#pragma unroll
                    for (int a = 0; a < 3; a++) {
                        double dx = V[2 * a] - xx, dy = V[2 * a + 1] - xy;
                        nin += dx * dx + dy * dy <= dd;
                    }
                    whole = nin == 3;
                    part = !whole && (nin > 0 || meets_edges(xx, xy, V, dd));
                }
                if (whole) {
                    ws += sW[q][0];
                    aw[0] += sW[q][1];
                    aw[1] += sW[q][2];
                    aw[2] += sW[q][3];
                    m0[q] += a2p * M.wsum;
                    c_whole++;
                } else if (part) {
                    pmask |= 1u << q;
                    c_part++;
                } else {
                    c_empty++;
                }
            }
        }
        double axy[3][3], ayy[6];
#pragma unroll
        for (int a = 0; a < 3; a++)
#pragma unroll
            for (int b = 0; b < 3; b++) axy[a][b] = aw[a] * a2p * M.m1[b];
        {
            const int jj[6] = {0, 0, 0, 1, 1, 2}, ll[6] = {0, 1, 2, 1, 2, 2};
#pragma unroll
            for (int t = 0; t < 6; t++) ayy[t] = ws * a2p * M.m2[jj[t]][ll[t]];
        }
        // queue the partial items: exclusive prefix over lanes of popcounts
        const int cnt = __popc(pmask);
        int pre = cnt;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            int v = __shfl_up(pre, off, 64);
            if (lane >= off) pre += v;
        }
        const int total = __shfl(pre, 63, 64);
        pre -= cnt;
        {
            int o = pre;
            unsigned mm = pmask;
            while (mm) {
                int q = __ffs(mm) - 1;
                mm &= mm - 1;
                queue[o++] = (unsigned short)((lane << 8) | q);
            }
        }
        __syncthreads();
        for (int ib = 0; ib < total; ib += 64) {
            const int i = ib + lane;
            if (i < total) {
                const int e = queue[i], owner = e >> 8, q = e & 0xff;
                Acc A;
                A.a2 = 0.0;
#pragma unroll
                for (int t = 0; t < 3; t++) A.s1[t] = 0.0;
#pragma unroll
                for (int t = 0; t < 6; t++) A.s2[t] = 0.0;
                int ns = 0;
                partial_item<SYM, POW2>(sX[q][0], sX[q][1], &sV[owner][0], dd, ncap, M, A, ns);
                c_sub += ns & 0xffff;
                c_cap += ns >> 16;
                res[lane][0] = A.a2 * M.wsum;
#pragma unroll
                for (int t = 0; t < 3; t++) res[lane][1 + t] = SYM ? A.s1[t] * M.m1c : A.s1[t];
#pragma unroll
                for (int t = 0; t < 6; t++) res[lane][4 + t] = A.s2[t];
            }
            __syncthreads();
            const int j0 = pre > ib ? pre : ib;
            const int j1 = (pre + cnt) < (ib + 64) ? (pre + cnt) : (ib + 64);
            for (int j = j0; j < j1; j++) {
                const int q = queue[j] & 0xff;
                const double *r = res[j - ib];
#pragma unroll
                for (int qq = 0; qq < NQ; qq++)
                    if (qq == q) m0[qq] += r[0];
                const double W = sW[q][0];
#pragma unroll
                for (int a = 0; a < 3; a++)
#pragma unroll
                    for (int b = 0; b < 3; b++) axy[a][b] += sW[q][1 + a] * r[1 + b];
#pragma unroll
                for (int t = 0; t < 6; t++) ayy[t] += W * r[4 + t];
            }
            __syncthreads();
        }
        if (act) {
#pragma unroll
            for (int a = 0; a < 3; a++)
#pragma unroll
                for (int b = 0; b < 3; b++) mxy_l[lane][3 * a + b] = -psi * axy[a][b];
#pragma unroll
            for (int t = 0; t < 6; t++) Cyy[6 * p + t] = psi * ayy[t];
        }
        __syncthreads();
        {
            const int lo = (int)(base - p0), hi = lo + 64;
            for (int c = lane; c < nC; c += 64) {
                int cur = cur_l[c];
                const int end = colent_ptr[coff + c + 1];
                double r0 = R_l[c], r1 = R_l[nC + c], r2 = R_l[2 * nC + c];
                while (cur < end) {
                    const int e = colent[cur];
                    const int pl = e >> 2;
                    if (pl >= hi) break;
                    const int b = e & 3;
                    const double *mm = mxy_l[pl - lo];
                    r0 += mm[b];
                    r1 += mm[3 + b];
                    r2 += mm[6 + b];
                    cur++;
                }
                R_l[c] = r0;
                R_l[nC + c] = r1;
                R_l[2 * nC + c] = r2;
                cur_l[c] = cur;
            }
        }
        __syncthreads();
    }
    for (int i = lane; i < 3 * nC; i += 64) Rout[3 * coff + i] = R_l[i];
    // Mxx(k) = sum_q W_q alpha alpha^T psi sum_k' S0: a fixed butterfly over the
    // lanes, then lane 0's sum is broadcast
#pragma unroll
    for (int q = 0; q < NQ; q++) {
        double x = m0[q];
        for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
        m0[q] = __shfl(x, 0, 64);
    }
    if (lane < 6) {
        const int aa[6] = {0, 0, 0, 1, 1, 2}, cc[6] = {0, 1, 2, 1, 2, 2};
        const int a = aa[lane], c = cc[lane];
        double s = 0.0;
#pragma unroll
        for (int q = 0; q < NQ; q++)
            if (q < nq) s += sW[q][1 + a] * R->out_lam[q][c] * m0[q];
        Cxx[6 * (int64_t)k + lane] = psi * s;
    }
    // work counters
    unsigned long long v[5] = {c_whole, c_part, c_empty, c_sub, c_cap};
#pragma unroll
    for (int i = 0; i < 5; i++) {
        unsigned long long x = v[i];
        for (int off = 32; off > 0; off >>= 1) x += __shfl_down(x, off, 64);
        v[i] = x;
    }
    if (lane == 0) {
        atomicAdd(&counters[0], v[0]);
        atomicAdd(&counters[1], v[1]);
        atomicAdd(&counters[2], v[2]);
        atomicAdd(&counters[4], v[3]);
        atomicAdd(&counters[5], v[4]);
    }
}

// Element blocks E(k') = Mxx(k') + sum_k Myy(k, k'): one wavefront per k'
// over its pairs in the transposed order (k ascending); lane l takes every
// 64th pair from l, lanes are combined by a fixed butterfly.
template <class T>
__global__ __launch_bounds__(64) void k_elem_blocks(int K, const int64_t *__restrict__ tptr,
                                                    const int32_t *__restrict__ tperm, const T *__restrict__ Cyy,
                                                    const T *__restrict__ Cxx, T *__restrict__ Ce)
{
    const int k = blockIdx.x, lane = threadIdx.x;
    double y[6] = {0, 0, 0, 0, 0, 0};
    for (int64_t t = tptr[k] + lane; t < tptr[k + 1]; t += 64) {
        const int64_t p = tperm[t];
#pragma unroll
        for (int i = 0; i < 6; i++) y[i] += (double)Cyy[6 * p + i];
    }
#pragma unroll
    for (int i = 0; i < 6; i++) {
        double v = y[i];
        for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
        y[i] = v;
    }
    if (lane < 6) {
        double v = 0.0;
#pragma unroll
        for (int i = 0; i < 6; i++)
            if (i == lane) v = y[i];
        Ce[6 * (int64_t)k + lane] = (T)(v + (double)Cxx[6 * (int64_t)k + lane]);
    }
}

// Deterministic COO->CSR sum: every upper-triangle entry adds its
// contributions in the fixed order of its code list and writes the sum to
// both mirrored positions, so D is bitwise symmetric and run-to-run identical.
__global__ void k_segsum_f64(int64_t n_up, const int64_t *__restrict__ up_ptr, const int32_t *__restrict__ codes,
                             const int64_t *__restrict__ up_dst, const int64_t *__restrict__ mirror,
                             const double *__restrict__ C, double *__restrict__ val)
{
    int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (u >= n_up) return;
    double s = 0.0;
    for (int64_t t = up_ptr[u]; t < up_ptr[u + 1]; t++) s += C[codes[t]];
    int64_t d = up_dst[u];
    val[d] = s;
    val[mirror[d]] = s;
}

template <class T>
__global__ void k_extract(int64_t n, const int64_t *__restrict__ src, const T *__restrict__ val, T *__restrict__ out)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = val[src[i]];
}

// G restricted to one element of Omega: sum_q W_q alpha_a(q) f(x_q) (Eq. (lfunchj))
__global__ void k_load_elem(int K, const uint8_t *__restrict__ tin, const double *__restrict__ a2,
                            const RuleSet *__restrict__ R, const double *__restrict__ f, double *__restrict__ Gk)
{
    int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= K) return;
    double g[3] = {0.0, 0.0, 0.0};
    if (tin[k]) {
        const int nq = R->n_out;
        for (int q = 0; q < nq; q++) {
            double Wf = R->out_w[q] * a2[k] * f[(int64_t)k * nq + q];
            for (int a = 0; a < 3; a++) g[a] += Wf * R->out_lam[q][a];
        }
    }
    for (int a = 0; a < 3; a++) Gk[3 * (int64_t)k + a] = g[a];
}

// b_i = G_j - sum_{Dirichlet nodes l} D[j,l] g_l for free node j (Eqs. (appr), (intcon)):
// one wavefront per free row, lanes stride the row, fixed butterfly reduction
template <class T>
__global__ __launch_bounds__(256) void k_load_rhs(int n_free, const int32_t *__restrict__ free_nodes,
                                                  const int32_t *__restrict__ n2e_ptr, const int32_t *__restrict__ n2e,
                                                  const double *__restrict__ Gk, const int64_t *__restrict__ rowptr,
                                                  const int32_t *__restrict__ col, const T *__restrict__ val,
                                                  const int32_t *__restrict__ n2f, const double *__restrict__ g,
                                                  double *__restrict__ b)
{
    const int i = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
    if (i >= n_free) return;
    const int j = free_nodes[i];
    double s = 0.0;
    for (int e = n2e_ptr[j] + lane; e < n2e_ptr[j + 1]; e += 64) s += Gk[n2e[e]];
    for (int64_t t = rowptr[j] + lane; t < rowptr[j + 1]; t += 64) {
        const int c = col[t];
        if (n2f[c] < 0) s -= (double)val[t] * g[c];
    }
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
    if (lane == 0) b[i] = s;
}

int nla_numeric(nla_plan *P, const double *f_outer, const double *g_node, hipStream_t s)
{
    const nla_problem &pr = P->prob;
    if (pr.kernel != NLA_KERNEL_CONSTANT || pr.precision != NLA_FP64) {
        nla_set_error("this build assembles the constant kernel in FP64 only");
        return NLA_E_UNSUPPORTED;
    }
    const int64_t NP = P->n_pairs;
    const int K = P->K;
    if (!P->contrib) {
        P->n_contrib = 6 * NP + 12 * (int64_t)K + 3 * P->n_cols;
        NLA_TRY(P->arena.alloc(&P->contrib, sizeof(double) * P->n_contrib));
        NLA_TRY(P->arena.alloc(&P->val, sizeof(double) * P->nnz));
        NLA_TRY(P->arena.alloc(&P->a_val, sizeof(double) * (P->nnz_free > 0 ? P->nnz_free : 1)));
        NLA_TRY(P->arena.get(&P->Gk, 3 * (size_t)K));
        NLA_TRY(P->arena.get(&P->b, P->n_free > 0 ? P->n_free : 1));
    }
    double *Cyy = (double *)P->contrib;
    double *Cxx = Cyy + 6 * NP;
    double *V = Cxx + 6 * (int64_t)K;          // [R (3 n_cols) | E (6K)]: the values the codes index
    double *Ce = V + 3 * P->n_cols;
    const bool timed = P->timing_count < P->timing_slots;
    hipEvent_t *ev = timed ? &P->ev[(size_t)P->timing_count * (NLA_NPHASE + 1)] : nullptr;
    auto mark = [&](int i) -> int {
        if (timed) NLA_HIP(hipEventRecord(ev[i], s));
        return NLA_OK;
    };
    for (int i = 0; i < NLA_NPHASE; i++) P->ran[i] = false;
    NLA_HIP(hipMemsetAsync(P->counters, 0, sizeof(unsigned long long) * 6, s));
    NLA_TRY(mark(NLA_PHASE_PAIRS));
    const size_t lds = (size_t)P->max_cols * (3 * sizeof(double) + sizeof(int));
    const int ncap = pr.ball == NLA_BALL_RETRI ? pr.cap_edges : 0;
#define NLA_LAUNCH_PAIRS(NQ, SYM, POW2)                                                                            \
    k_pairs_const_fp64<NQ, SYM, POW2><<<K, 64, lds, s>>>(P->pair_ptr, P->pair_kp, P->E, P->xq, P->d_rules,          \
                                                         pr.delta * pr.delta, pr.kernel_c, pr.ball, ncap, P->col_off, \
                                                         P->colent_ptr, P->colent, V, Cyy, Cxx, P->max_cols,          \
                                                         P->counters)
    const bool sym = P->rules.in_sym != 0;
    const bool pow2 = (ncap & (ncap - 1)) == 0;     // 0 (no caps) counts as a power of two
    if (P->rules.n_out <= 8 && sym && pow2) NLA_LAUNCH_PAIRS(8, true, true);
    else if (P->rules.n_out <= 8 && sym) NLA_LAUNCH_PAIRS(8, true, false);
    else if (P->rules.n_out <= 8) NLA_LAUNCH_PAIRS(8, false, false);
    else NLA_LAUNCH_PAIRS(16, false, false);
#undef NLA_LAUNCH_PAIRS
    NLA_HIP(hipGetLastError());
    P->ran[NLA_PHASE_PAIRS] = true;
    NLA_TRY(mark(NLA_PHASE_NEAR));
    NLA_TRY(mark(NLA_PHASE_SEGSUM));
    k_elem_blocks<double><<<K, 64, 0, s>>>(K, P->tptr, P->tperm, Cyy, Cxx, Ce);
    if (P->n_up > 0)
        k_segsum_f64<<<grid_for(P->n_up, 256), 256, 0, s>>>(P->n_up, P->up_ptr, P->codes, P->up_dst, P->mirror, V,
                                                           (double *)P->val);
    P->ran[NLA_PHASE_SEGSUM] = true;
    NLA_TRY(mark(NLA_PHASE_EXTRACT));
    if (P->nnz_free > 0)
        k_extract<double><<<grid_for(P->nnz_free, 256), 256, 0, s>>>(P->nnz_free, P->a_src, (const double *)P->val,
                                                                    (double *)P->a_val);
    P->ran[NLA_PHASE_EXTRACT] = true;
    NLA_TRY(mark(NLA_PHASE_LOAD));
    P->have_load = false;
    if (f_outer && g_node) {
        k_load_elem<<<grid_for(K, 256), 256, 0, s>>>(K, P->tin, P->E.a2, P->d_rules, f_outer, P->Gk);
        if (P->n_free > 0)
            k_load_rhs<double><<<grid_for(P->n_free, 4), 256, 0, s>>>(
                P->n_free, P->free_nodes, P->n2e_ptr, P->n2e, P->Gk, P->rowptr, P->col, (const double *)P->val,
                P->node_to_free, g_node, P->b);
        P->have_load = true;
        P->ran[NLA_PHASE_LOAD] = true;
    }
    NLA_TRY(mark(NLA_NPHASE));
    if (timed) P->timing_count++;
    NLA_HIP(hipGetLastError());
    P->val_dtype = NLA_DTYPE_F64;
    P->assembled = true;
    return NLA_OK;
}
