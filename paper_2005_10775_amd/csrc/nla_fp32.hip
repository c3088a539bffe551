// FP32 numeric path (precision NLA_FP32): geometry of the retriangulated ball
// stays FP64, the kernel psi and the quadrature sums are FP32, and every
// accumulation across subtriangles, items, pairs and CSR contributions is
// Kahan-compensated.  Vertex-sharing pairs of the singular kernel are
// integrated in FP64 by a radial (Duffy-type) rule.
#include "nla_device.hpp"
#include <cmath>

static inline unsigned grid_for(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

// Kahan's compensated summation
struct KahanF {
    float s, c;
    __device__ __forceinline__ void zero() { s = 0.f; c = 0.f; }
    __device__ __forceinline__ void add(float v)
    {
        const float y = v - c;
        const float t = s + y;
        c = (t - s) - y;
        s = t;
    }
};

// item sums (S0, S1[3], S2[6]) in FP32, compensated over subtriangles
struct AccF {
    KahanF s0, s1[3], s2[6];
    __device__ __forceinline__ void zero()
    {
        s0.zero();
#pragma unroll
        for (int i = 0; i < 3; i++) s1[i].zero();
#pragma unroll
        for (int i = 0; i < 6; i++) s2[i].zero();
    }
};

// Inner rule on one subtriangle t (vertices relative to x, basis values at the
// vertices).  FRAC: psi = kc r^(2*ex) evaluated at every rule point y in FP32
// (r^2 = |y - x|^2); otherwise psi = kc and the rule is applied through its
// moments (sym form, as in the FP64 kernel).
template <bool FRAC>
struct TriF32 {
    const RuleSet *R;
    float kc, ex, m1c, o, dm;
    AccF *A;
    __device__ __forceinline__ void operator()(const double (&t)[3][5]) const
    {
        const double a2d = fabs((t[1][0] - t[0][0]) * (t[2][1] - t[0][1]) - (t[1][1] - t[0][1]) * (t[2][0] - t[0][0]));
        const float a2 = (float)a2d;
        float tb[3][3];
#pragma unroll
        for (int i = 0; i < 3; i++)
#pragma unroll
            for (int l = 0; l < 3; l++) tb[i][l] = (float)t[i][2 + l];
        const int jj[6] = {0, 0, 0, 1, 1, 2}, ll[6] = {0, 1, 2, 1, 2, 2};
        if (FRAC) {
            const float tx[3] = {(float)t[0][0], (float)t[1][0], (float)t[2][0]};
            const float ty[3] = {(float)t[0][1], (float)t[1][1], (float)t[2][1]};
            float q0 = 0.f, q1[3] = {0.f, 0.f, 0.f}, q2[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
            const int n = R->n_in;
            for (int q = 0; q < n; q++) {
                const float m0 = R->in_lamf[q][0], m1 = R->in_lamf[q][1], m2 = R->in_lamf[q][2];
                const float yx = m0 * tx[0] + m1 * tx[1] + m2 * tx[2];
                const float yy = m0 * ty[0] + m1 * ty[1] + m2 * ty[2];
                float b[3];
#pragma unroll
                for (int l = 0; l < 3; l++) b[l] = m0 * tb[0][l] + m1 * tb[1][l] + m2 * tb[2][l];
                const float r2 = yx * yx + yy * yy;
                // hardware log2 / exp2 (v_log_f32, v_exp_f32): r^(2 ex) = 2^(ex log2 r^2)
                const float wp = R->in_wf[q] * kc * __builtin_amdgcn_exp2f(ex * __builtin_amdgcn_logf(r2));
                q0 += wp;
#pragma unroll
                for (int l = 0; l < 3; l++) q1[l] += wp * b[l];
#pragma unroll
                for (int e = 0; e < 6; e++) q2[e] += wp * b[jj[e]] * b[ll[e]];
            }
            A->s0.add(a2 * q0);
#pragma unroll
            for (int l = 0; l < 3; l++) A->s1[l].add(a2 * q1[l]);
#pragma unroll
            for (int e = 0; e < 6; e++) A->s2[e].add(a2 * q2[e]);
        } else {
            float cs[3];
#pragma unroll
            for (int l = 0; l < 3; l++) cs[l] = tb[0][l] + tb[1][l] + tb[2][l];
            A->s0.add(a2 * (0.5f * kc));
#pragma unroll
            for (int l = 0; l < 3; l++) A->s1[l].add(a2 * kc * m1c * cs[l]);
            const float w = a2 * kc * o, v = a2 * kc * dm;
#pragma unroll
            for (int e = 0; e < 6; e++) {
                const int j = jj[e], l = ll[e];
                const float qq = tb[0][j] * tb[0][l] + tb[1][j] * tb[1][l] + tb[2][j] * tb[2][l];
                A->s2[e].add(w * (cs[j] * cs[l]) + v * qq);
            }
        }
    }
};

// One wavefront per outer element k, FP32 sums (structure as the FP64 kernel):
// phase 1 classifies the items of each lane's pair and integrates whole items
// in the lane, phase 2 retriangulates the queued partial items densely; the
// results are added per pair in q order (compensated), -Mxy is reduced into
// the row block R_k in LDS per column in pair order (compensated), Myy per
// pair and Mxx per element are written.  Pairs flagged near (vertex-sharing,
// singular kernel) are skipped here.
template <int NQ, bool FRAC, bool POW2>
__global__ __launch_bounds__(64, 2) void k_pairs_fp32(const int64_t *__restrict__ pair_ptr,
                                                     const int32_t *__restrict__ pair_kp, ElemSoA E,
                                                     const double *__restrict__ xq, const RuleSet *__restrict__ R,
                                                     double dd, float kc, float ex, int ball, int ncap,
                                                     const uint8_t *__restrict__ near_flag,
                                                     const int64_t *__restrict__ col_off,
                                                     const int32_t *__restrict__ colent_ptr,
                                                     const uint16_t *__restrict__ colent, float *__restrict__ Rout,
                                                     float *__restrict__ Cyy, float *__restrict__ Cxx, int max_cols,
                                                     unsigned long long *__restrict__ counters)
{
    extern __shared__ double dyn[];
    __shared__ double sX[NQ][2];
    __shared__ float sW[NQ][4];
    __shared__ double sV[64][7];
    __shared__ unsigned short queue[64 * NQ];
    __shared__ float res[64][10];
    float(*mxy_l)[10] = res;
    const int k = blockIdx.x, lane = threadIdx.x;
    const int nq = R->n_out;
    const double a2k = E.a2[k];
    if (lane < nq) {
        const double W = R->out_w[lane] * a2k;
        sW[lane][0] = (float)W;
        sW[lane][1] = (float)(W * R->out_lam[lane][0]);
        sW[lane][2] = (float)(W * R->out_lam[lane][1]);
        sW[lane][3] = (float)(W * R->out_lam[lane][2]);
        sX[lane][0] = xq[2 * ((int64_t)k * nq + lane)];
        sX[lane][1] = xq[2 * ((int64_t)k * nq + lane) + 1];
    }
    const int64_t coff = col_off[k];
    const int nC = (int)(col_off[k + 1] - coff);
    float *R_s = (float *)dyn;                                // [3][nC] sums
    float *R_c = R_s + 3 * (size_t)max_cols;                 // [3][nC] compensations
    int *cur_l = (int *)(R_c + 3 * (size_t)max_cols);        // [nC]
    for (int c = lane; c < nC; c += 64) {
#pragma unroll
        for (int a = 0; a < 3; a++) {
            R_s[a * nC + c] = 0.f;
            R_c[a * nC + c] = 0.f;
        }
        cur_l[c] = colent_ptr[coff + c];
    }
    __syncthreads();
    const float m1c = (float)R->in_m1[0], o = (float)R->in_m2[0][1], dm = (float)(R->in_m2[0][0] - R->in_m2[0][1]);
    KahanF m0[NQ];
#pragma unroll
    for (int q = 0; q < NQ; q++) m0[q].zero();
    unsigned long long c_whole = 0, c_part = 0, c_empty = 0, c_sub = 0, c_cap = 0;
    const int64_t p0 = pair_ptr[k], p1 = pair_ptr[k + 1];
    for (int64_t base = p0; base < p1; base += 64) {
        const int64_t p = base + lane;
        const bool act = p < p1 && !(near_flag && near_flag[p]);
        double V[6] = {0, 0, 0, 0, 0, 0};
        double bxp = 0.0, byp = 0.0, a2p = 0.0;
        if (act) {
            const int kp = pair_kp[p];
            V[0] = E.vx0[kp]; V[1] = E.vy0[kp]; V[2] = E.vx1[kp]; V[3] = E.vy1[kp]; V[4] = E.vx2[kp]; V[5] = E.vy2[kp];
            bxp = E.bx[kp];
            byp = E.by[kp];
            a2p = E.a2[kp];
        }
#pragma unroll
        for (int i = 0; i < 6; i++) sV[lane][i] = V[i];
        KahanF axy[9], ayy[6];
#pragma unroll
        for (int i = 0; i < 9; i++) axy[i].zero();
#pragma unroll
        for (int i = 0; i < 6; i++) ayy[i].zero();
        float ws = 0.f, aw[3] = {0.f, 0.f, 0.f};
        unsigned pmask = 0;
        if (act) {
#pragma unroll
            for (int q = 0; q < NQ; q++) {
                if (q >= nq) break;
                const double xx = sX[q][0], xy = sX[q][1];
                bool whole = false, part = false;
                if (ball == NLA_BALL_BARYCENTER) {
                    const double dx = xx - bxp, dy = xy - byp;
                    whole = dx * dx + dy * dy <= dd;
                } else {
                    int nin = 0;
#pragma unroll
                    for (int a = 0; a < 3; a++) {
                        const double dx = V[2 * a] - xx, dy = V[2 * a + 1] - xy;
                        nin += dx * dx + dy * dy <= dd;
                    }
                    whole = nin == 3;
                    part = !whole && (nin > 0 || meets_edges(xx, xy, V, dd));
                }
                if (whole) {
                    c_whole++;
                    if (FRAC) {
                        // psi varies: the inner rule over all of E_k'
                        AccF A;
                        A.zero();
                        TriF32<true> tri{R, kc, ex, m1c, o, dm, &A};
                        double t[3][5];
                        set5(t[0], V[0] - xx, V[1] - xy, 1.0, 0.0, 0.0);
                        set5(t[1], V[2] - xx, V[3] - xy, 0.0, 1.0, 0.0);
                        set5(t[2], V[4] - xx, V[5] - xy, 0.0, 0.0, 1.0);
                        tri(t);
                        m0[q].add(A.s0.s);
#pragma unroll
                        for (int a = 0; a < 3; a++)
#pragma unroll
                            for (int b = 0; b < 3; b++) axy[3 * a + b].add(sW[q][1 + a] * A.s1[b].s);
#pragma unroll
                        for (int e = 0; e < 6; e++) ayy[e].add(sW[q][0] * A.s2[e].s);
                    } else {
                        ws += sW[q][0];
                        aw[0] += sW[q][1];
                        aw[1] += sW[q][2];
                        aw[2] += sW[q][3];
                        m0[q].add((float)(a2p * R->in_wsum) * kc);
                    }
                } else if (part) {
                    pmask |= 1u << q;
                    c_part++;
                } else {
                    c_empty++;
                }
            }
        }
        if (!FRAC) {
            const float ka = kc * (float)a2p;
            const int jj[6] = {0, 0, 0, 1, 1, 2}, ll[6] = {0, 1, 2, 1, 2, 2};
#pragma unroll
            for (int a = 0; a < 3; a++)
#pragma unroll
                for (int b = 0; b < 3; b++) axy[3 * a + b].add(aw[a] * ka * m1c);
#pragma unroll
            for (int e = 0; e < 6; e++) ayy[e].add(ws * ka * (o + (jj[e] == ll[e] ? dm : 0.f)));
        }
        const int cnt = __popc(pmask);
        int pre = cnt;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const int v = __shfl_up(pre, off, 64);
            if (lane >= off) pre += v;
        }
        const int total = __shfl(pre, 63, 64);
        pre -= cnt;
        {
            int oo = pre;
            unsigned mm = pmask;
            while (mm) {
                const int q = __ffs(mm) - 1;
                mm &= mm - 1;
                queue[oo++] = (unsigned short)((lane << 8) | q);
            }
        }
        __syncthreads();
        for (int ib = 0; ib < total; ib += 64) {
            const int i = ib + lane;
            if (i < total) {
                const int e = queue[i], owner = e >> 8, q = e & 0xff;
                AccF A;
                A.zero();
                TriF32<FRAC> tri{R, kc, ex, m1c, o, dm, &A};
                int ns = 0;
                partial_item<POW2>(sX[q][0], sX[q][1], &sV[owner][0], dd, ncap, tri, ns);
                c_sub += ns & 0xffff;
                c_cap += ns >> 16;
                res[lane][0] = A.s0.s;
#pragma unroll
                for (int t = 0; t < 3; t++) res[lane][1 + t] = A.s1[t].s;
#pragma unroll
                for (int t = 0; t < 6; t++) res[lane][4 + t] = A.s2[t].s;
            }
            __syncthreads();
            const int j0 = pre > ib ? pre : ib;
            const int j1 = (pre + cnt) < (ib + 64) ? (pre + cnt) : (ib + 64);
            for (int j = j0; j < j1; j++) {
                const int q = queue[j] & 0xff;
                const float *r = res[j - ib];
#pragma unroll
                for (int qq = 0; qq < NQ; qq++)
                    if (qq == q) m0[qq].add(r[0]);
#pragma unroll
                for (int a = 0; a < 3; a++)
#pragma unroll
                    for (int b = 0; b < 3; b++) axy[3 * a + b].add(sW[q][1 + a] * r[1 + b]);
#pragma unroll
                for (int t = 0; t < 6; t++) ayy[t].add(sW[q][0] * r[4 + t]);
            }
            __syncthreads();
        }
        if (p < p1) {
#pragma unroll
            for (int i = 0; i < 9; i++) mxy_l[lane][i] = -axy[i].s;
#pragma unroll
            for (int t = 0; t < 6; t++) Cyy[6 * p + t] = ayy[t].s;
        }
        __syncthreads();
        {
            const int lo = (int)(base - p0), hi = lo + 64;
            for (int c = lane; c < nC; c += 64) {
                int cur = cur_l[c];
                const int end = colent_ptr[coff + c + 1];
                KahanF r[3];
#pragma unroll
                for (int a = 0; a < 3; a++) {
                    r[a].s = R_s[a * nC + c];
                    r[a].c = R_c[a * nC + c];
                }
                while (cur < end) {
                    const int e = colent[cur];
                    const int pl = e >> 2;
                    if (pl >= hi) break;
                    const int b = e & 3;
                    const float *mm = mxy_l[pl - lo];
                    r[0].add(mm[b]);
                    r[1].add(mm[3 + b]);
                    r[2].add(mm[6 + b]);
                    cur++;
                }
#pragma unroll
                for (int a = 0; a < 3; a++) {
                    R_s[a * nC + c] = r[a].s;
                    R_c[a * nC + c] = r[a].c;
                }
                cur_l[c] = cur;
            }
        }
        __syncthreads();
    }
    for (int i = lane; i < 3 * nC; i += 64) Rout[3 * coff + i] = R_s[i];
    // Mxx(k) from the per-lane S0 sums, fixed butterfly, lane 0's value broadcast
    float msum[NQ];
#pragma unroll
    for (int q = 0; q < NQ; q++) {
        float x = m0[q].s;
        for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
        msum[q] = __shfl(x, 0, 64);
    }
    if (lane < 6) {
        const int aa[6] = {0, 0, 0, 1, 1, 2}, cc[6] = {0, 1, 2, 1, 2, 2};
        const int a = aa[lane], c = cc[lane];
        KahanF s;
        s.zero();
#pragma unroll
        for (int q = 0; q < NQ; q++)
            if (q < nq) s.add(sW[q][1 + a] * (float)R->out_lam[q][c] * msum[q]);
        Cxx[6 * (int64_t)k + lane] = s.s;
    }
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

// ---------------------------------------------------------------- near pairs
// Merged 6x6 block of a vertex-sharing pair under psi = kc |x-y|^-(2+2s), FP64:
// outer points of a tensor Gauss rule on E_k collapsed at vertex c (shared
// vertex / vertex opposite a shared edge / vertex 0 for k = k'); around each
// outer point x the angle range of E_k' is cut at its vertex directions, each
// piece gets Gauss points clustered at its ends (t = u^2 (3 - 2u)); along a
// ray the merged differences are affine in r and the radial integral of
// r^(m-1-2s), m = 0,1,2, is exact between the entry and exit radii (exit
// capped at delta).  Per outer point the ray sums reduce to six angular
// moments, then to the 21 upper entries of the block.  One wavefront per pair.
template <class T>
__global__ __launch_bounds__(64) void k_near(int64_t n_near, const int64_t *__restrict__ near_pair,
                                             const int32_t *__restrict__ pk, const int32_t *__restrict__ pkp,
                                             const int32_t *__restrict__ tri, ElemSoA E, const RuleSet *__restrict__ R,
                                             double delta, double kc, double ks, T *__restrict__ out)
{
    const int64_t i = blockIdx.x;
    const int lane = threadIdx.x;
    if (i >= n_near) return;
    const int64_t p = near_pair[i];
    const int k = pk[p], kp = pkp[p];
    const double Vk[6] = {E.vx0[k], E.vy0[k], E.vx1[k], E.vy1[k], E.vx2[k], E.vy2[k]};
    const double Vp[6] = {E.vx0[kp], E.vy0[kp], E.vx1[kp], E.vy1[kp], E.vx2[kp], E.vy2[kp]};
    int sb[3], nshared = 0;
    bool bsh[3] = {false, false, false};
    for (int a = 0; a < 3; a++) {
        sb[a] = -1;
        for (int b = 0; b < 3; b++)
            if (tri[3 * k + a] == tri[3 * kp + b]) {
                sb[a] = b;
                bsh[b] = true;
                nshared++;
            }
    }
    const bool identical = nshared == 3;
    int c = 0;
    if (nshared == 1) {
        for (int a = 0; a < 3; a++)
            if (sb[a] >= 0) c = a;
    } else if (nshared == 2) {
        for (int a = 0; a < 3; a++)
            if (sb[a] < 0) c = a;
    }
    const int c1 = c == 2 ? 0 : c + 1, c2 = c == 0 ? 2 : c - 1;
    const double a2k = E.a2[k];
    // gradients of the two bases (constant)
    double agx[3], agy[3], bgx[3], bgy[3];
    auto grads = [](const double (&V)[6], double (&gx)[3], double (&gy)[3]) {
        const double det = (V[2] - V[0]) * (V[5] - V[1]) - (V[3] - V[1]) * (V[4] - V[0]);
        gx[1] = (V[5] - V[1]) / det;
        gy[1] = -(V[4] - V[0]) / det;
        gx[2] = -(V[3] - V[1]) / det;
        gy[2] = (V[2] - V[0]) / det;
        gx[0] = -gx[1] - gx[2];
        gy[0] = -gy[1] - gy[2];
    };
    grads(Vk, agx, agy);
    grads(Vp, bgx, bgy);
    double gxs[6], gys[6];
    for (int a = 0; a < 3; a++) {
        gxs[a] = sb[a] >= 0 ? -bgx[sb[a]] : 0.0;
        gys[a] = sb[a] >= 0 ? -bgy[sb[a]] : 0.0;
        gxs[3 + a] = bsh[a] ? 0.0 : -bgx[a];
        gys[3 + a] = bsh[a] ? 0.0 : -bgy[a];
    }
    const int n = R->duffy_n;
    const double pi2 = 6.283185307179586476925286766559;
    const double e0 = -2.0 * ks;                    // exponent of r^(m-2s) at m = 0
    double L[21];
#pragma unroll
    for (int t = 0; t < 21; t++) L[t] = 0.0;
    for (int oi = lane; oi < n * n; oi += 64) {
        const double sv = R->duffy_x[oi / n], wv = R->duffy_x[oi % n];
        const double Wx = R->duffy_w[oi / n] * R->duffy_w[oi % n] * a2k * sv;
        double x[2];
        for (int d = 0; d < 2; d++)
            x[d] = Vk[2 * c + d] + sv * ((1.0 - wv) * (Vk[2 * c1 + d] - Vk[2 * c + d]) + wv * (Vk[2 * c2 + d] - Vk[2 * c + d]));
        // basis values at x (E_k) and the affine extension of E_k' basis at x
        double al[3], be[3];
        {
            const double dx = x[0] - Vk[0], dy = x[1] - Vk[1];
            al[1] = dx * agx[1] + dy * agy[1];
            al[2] = dx * agx[2] + dy * agy[2];
            al[0] = 1.0 - al[1] - al[2];
            const double ex_ = x[0] - Vp[0], ey_ = x[1] - Vp[1];
            be[1] = ex_ * bgx[1] + ey_ * bgy[1];
            be[2] = ex_ * bgx[2] + ey_ * bgy[2];
            be[0] = 1.0 - be[1] - be[2];
        }
        double c0[6];
        for (int a = 0; a < 3; a++) {
            c0[a] = sb[a] >= 0 ? (identical ? 0.0 : al[a] - be[sb[a]]) : al[a];
            c0[3 + a] = bsh[a] ? 0.0 : -be[a];
        }
        double ang[3];
        for (int b = 0; b < 3; b++) ang[b] = atan2(Vp[2 * b + 1] - x[1], Vp[2 * b] - x[0]);
        if (ang[0] > ang[1]) { double t = ang[0]; ang[0] = ang[1]; ang[1] = t; }
        if (ang[1] > ang[2]) { double t = ang[1]; ang[1] = ang[2]; ang[2] = t; }
        if (ang[0] > ang[1]) { double t = ang[0]; ang[0] = ang[1]; ang[1] = t; }
        double lo[3], hi[3];
        int npc;
        if (identical) {
            lo[0] = ang[0]; hi[0] = ang[1]; lo[1] = ang[1]; hi[1] = ang[2]; lo[2] = ang[2]; hi[2] = ang[0] + pi2;
            npc = 3;
        } else {
            const double g0 = ang[1] - ang[0], g1 = ang[2] - ang[1], g2 = ang[0] + pi2 - ang[2];
            if (g2 >= g0 && g2 >= g1) {
                lo[0] = ang[0]; hi[0] = ang[1]; lo[1] = ang[1]; hi[1] = ang[2];
            } else if (g0 >= g1) {
                lo[0] = ang[1]; hi[0] = ang[2]; lo[1] = ang[2]; hi[1] = ang[0] + pi2;
            } else {
                lo[0] = ang[2]; hi[0] = ang[0] + pi2; lo[1] = ang[0] + pi2; hi[1] = ang[1] + pi2;
            }
            lo[2] = hi[2] = 0.0;
            npc = 2;
        }
        // angular moments: A0 = sum w J0, A1 = sum w J1 e, A2 = sum w J2 e e^T
        double A0 = 0, A1x = 0, A1y = 0, Axx = 0, Axy = 0, Ayy = 0;
        for (int pc = 0; pc < npc; pc++)
            for (int it = 0; it < n; it++) {
                const double u = R->duffy_x[it];
                const double th = lo[pc] + (hi[pc] - lo[pc]) * (u * u * (3.0 - 2.0 * u));
                const double wt = (hi[pc] - lo[pc]) * R->duffy_w[it] * 6.0 * u * (1.0 - u);
                double sn, cs;
                sincos(th, &sn, &cs);
                double rin = 0.0, rout = 1e300;
                bool empty = false;
                for (int a = 0; a < 3; a++) {
                    const int b = a == 2 ? 0 : a + 1;
                    const double nx = Vp[2 * b + 1] - Vp[2 * a + 1], ny = -(Vp[2 * b] - Vp[2 * a]);
                    const double f0 = nx * (x[0] - Vp[2 * a]) + ny * (x[1] - Vp[2 * a + 1]);
                    const double f1 = nx * cs + ny * sn;
                    if (f1 > 0.0) rout = fmin(rout, -f0 / f1);
                    else if (f1 < 0.0) rin = fmax(rin, -f0 / f1);
                    else if (f0 > 0.0) empty = true;
                }
                rout = fmin(rout, delta);
                if (empty || !(rout > rin)) continue;
                // J_m = kc (rout^(m+e0) - rin^(m+e0)) / (m + e0)
                double J[3];
                const double po = exp2(e0 * log2(rout)), pi = rin > 0.0 ? exp2(e0 * log2(rin)) : 0.0;
                double ro = 1.0, ri = 1.0;
                for (int m = 0; m < 3; m++) {
                    const double ex = m + e0;
                    if (fabs(ex) < 1e-14) J[m] = rin > 0.0 ? kc * log(rout / rin) : 0.0;
                    else if (rin > 0.0) J[m] = kc * (ro * po - ri * pi) / ex;
                    else J[m] = ex > 0.0 ? kc * ro * po / ex : 0.0;
                    ro *= rout;
                    ri *= rin;
                }
                A0 += wt * J[0];
                A1x += wt * J[1] * cs;
                A1y += wt * J[1] * sn;
                Axx += wt * J[2] * cs * cs;
                Axy += wt * J[2] * cs * sn;
                Ayy += wt * J[2] * sn * sn;
            }
        int t = 0;
        for (int ii = 0; ii < 6; ii++) {
            const double gi1 = gxs[ii] * A1x + gys[ii] * A1y;
            for (int jj = ii; jj < 6; jj++, t++) {
                const double gj1 = gxs[jj] * A1x + gys[jj] * A1y;
                const double g2 = gxs[ii] * (Axx * gxs[jj] + Axy * gys[jj]) + gys[ii] * (Axy * gxs[jj] + Ayy * gys[jj]);
                L[t] += Wx * (c0[ii] * c0[jj] * A0 + c0[ii] * gj1 + gi1 * c0[jj] + g2);
            }
        }
    }
#pragma unroll
    for (int t = 0; t < 21; t++) {
        double v = L[t];
        for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
        L[t] = v;
    }
    if (lane < 21) {
        double v = 0.0;
#pragma unroll
        for (int t = 0; t < 21; t++)
            if (t == lane) v = L[t];
        out[21 * i + lane] = (T)v;
    }
}

// E(k') = Mxx(k') + sum_k Myy(k, k') in FP32 with compensation (lane-strided
// partial sums, then lane 0 adds the 64 partials in lane order)
__global__ __launch_bounds__(64) void k_elem_blocks_f32(int K, const int64_t *__restrict__ tptr,
                                                        const int32_t *__restrict__ tperm, const float *__restrict__ Cyy,
                                                        const float *__restrict__ Cxx, float *__restrict__ Ce)
{
    __shared__ float part[64][6];
    const int k = blockIdx.x, lane = threadIdx.x;
    KahanF y[6];
#pragma unroll
    for (int i = 0; i < 6; i++) y[i].zero();
    for (int64_t t = tptr[k] + lane; t < tptr[k + 1]; t += 64) {
        const int64_t p = tperm[t];
#pragma unroll
        for (int i = 0; i < 6; i++) y[i].add(Cyy[6 * p + i]);
    }
#pragma unroll
    for (int i = 0; i < 6; i++) part[lane][i] = y[i].s;
    __syncthreads();
    if (lane < 6) {
        KahanF s;
        s.zero();
        s.add(Cxx[6 * (int64_t)k + lane]);
        for (int l = 0; l < 64; l++) s.add(part[l][lane]);
        Ce[6 * (int64_t)k + lane] = s.s;
    }
}

// compensated FP32 sum of every upper entry: its [R | E] codes, then its
// near-pair block codes; both mirrored positions written
__global__ void k_segsum_f32(int64_t n_up, const int64_t *__restrict__ up_ptr, const int32_t *__restrict__ codes,
                             const int64_t *__restrict__ nup_ptr, const int32_t *__restrict__ ncodes,
                             const int64_t *__restrict__ up_dst, const int64_t *__restrict__ mirror,
                             const float *__restrict__ V, const float *__restrict__ N, float *__restrict__ val)
{
    const int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (u >= n_up) return;
    KahanF s;
    s.zero();
    for (int64_t t = up_ptr[u]; t < up_ptr[u + 1]; t++) s.add(V[codes[t]]);
    if (nup_ptr)
        for (int64_t t = nup_ptr[u]; t < nup_ptr[u + 1]; t++) s.add(N[ncodes[t]]);
    const int64_t d = up_dst[u];
    val[d] = s.s;
    val[mirror[d]] = s.s;
}

template <class T>
__global__ void k_extract_t(int64_t n, const int64_t *__restrict__ src, const T *__restrict__ val, T *__restrict__ out)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = val[src[i]];
}

int nla_numeric_fp32(nla_plan *P, hipStream_t s, void (*mark)(nla_plan *, int, hipStream_t))
{
    const nla_problem &pr = P->prob;
    const int64_t NP = P->n_pairs;
    const int K = P->K;
    float *Cyy = (float *)P->contrib;
    float *Cxx = Cyy + 6 * NP;
    float *V = Cxx + 6 * (int64_t)K;
    float *Ce = V + 3 * P->n_cols;
    const bool frac = pr.kernel == NLA_KERNEL_FRACTIONAL;
    const float kc = (float)pr.kernel_c;
    const float ex = frac ? (float)(-(1.0 + pr.kernel_s)) : 0.f;
    const int ncap = pr.ball == NLA_BALL_RETRI ? pr.cap_edges : 0;
    const bool pow2 = (ncap & (ncap - 1)) == 0;
    const size_t lds = (size_t)P->max_cols * (6 * sizeof(float) + sizeof(int));
    mark(P, NLA_PHASE_PAIRS, s);
#define NLA_LAUNCH32(NQ, FR, P2)                                                                                     \
    k_pairs_fp32<NQ, FR, P2><<<K, 64, lds, s>>>(P->pair_ptr, P->pair_kp, P->E, P->xq, P->d_rules, pr.delta * pr.delta, \
                                                kc, ex, pr.ball, ncap, P->near_flag, P->col_off, P->colent_ptr,         \
                                                P->colent, V, Cyy, Cxx, P->max_cols, P->counters)
    if (P->rules.n_out > 8) {
        nla_set_error("the FP32 path supports outer rules of at most 8 points");
        return NLA_E_UNSUPPORTED;
    }
    if (!frac && !P->rules.in_sym) {
        nla_set_error("the FP32 constant-kernel path needs a symmetric inner rule");
        return NLA_E_UNSUPPORTED;
    }
    if (frac && pow2) NLA_LAUNCH32(8, true, true);
    else if (frac) NLA_LAUNCH32(8, true, false);
    else if (pow2) NLA_LAUNCH32(8, false, true);
    else NLA_LAUNCH32(8, false, false);
#undef NLA_LAUNCH32
    NLA_HIP(hipGetLastError());
    P->ran[NLA_PHASE_PAIRS] = true;
    mark(P, NLA_PHASE_NEAR, s);
    if (P->n_near > 0) {
        k_near<float><<<(unsigned)P->n_near, 64, 0, s>>>(P->n_near, P->near_pair, P->pair_k, P->pair_kp, P->tri, P->E,
                                                         P->d_rules, pr.delta, pr.kernel_c, pr.kernel_s,
                                                         (float *)P->near_blk);
        NLA_HIP(hipGetLastError());
        P->ran[NLA_PHASE_NEAR] = true;
    }
    mark(P, NLA_PHASE_SEGSUM, s);
    k_elem_blocks_f32<<<K, 64, 0, s>>>(K, P->tptr, P->tperm, Cyy, Cxx, Ce);
    if (P->n_up > 0)
        k_segsum_f32<<<grid_for(P->n_up, 256), 256, 0, s>>>(P->n_up, P->up_ptr, P->codes,
                                                           P->n_near > 0 ? P->nup_ptr : nullptr, P->ncodes, P->up_dst,
                                                           P->mirror, V, (const float *)P->near_blk, (float *)P->val);
    P->ran[NLA_PHASE_SEGSUM] = true;
    mark(P, NLA_PHASE_EXTRACT, s);
    if (P->nnz_free > 0)
        k_extract_t<float><<<grid_for(P->nnz_free, 256), 256, 0, s>>>(P->nnz_free, P->a_src, (const float *)P->val,
                                                                      (float *)P->a_val);
    P->ran[NLA_PHASE_EXTRACT] = true;
    NLA_HIP(hipGetLastError());
    return NLA_OK;
}
