// Numeric phase of libnlasm: pair quadrature, deterministic segmented sum
// into the CSR values of D, extraction of A = D[free,free] and the load vector.
#include "nla_internal.hpp"
#include <cmath>

// workgroups per CU of the FP64 pair kernels (see lds_for_occupancy)
#define NLA_PAIRS_WG_PER_CU 0
#define NLA_SUPPORT_WG_PER_CU 0

static inline unsigned grid_for(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

#include "nla_device.hpp"

// the fold's 15-bit entry offsets (3 per pair) and 16-bit pair indices, and the
// 16-bit (pair << 2 | slot) entries, hold for every element the plan admits
static_assert(3 * NLA_MAX_PAIRS_PER_K + 4 <= 0x7fff && NLA_MAX_PAIRS_PER_K + 64 < 0xffff &&
                  NLA_MAX_PAIRS_PER_K <= (1 << 14),
              "fold cursors and column entries are 16-bit");

// One column's walk for fold_row_block: e holds the entries at the column's
// cursor and r the column's sums so far, both already loaded; further groups
// of four entries are loaded as needed.
__device__ __forceinline__ void fold_column(double *__restrict__ Rg, unsigned *cn_l, int nC, int c, unsigned w,
                                            int end, int cbase, const int (&e0)[4], const double (&r)[3],
                                            const uint16_t *__restrict__ colent, const double (*mxy_l)[12], int lo,
                                            int hi)
{
    int cur = cbase + (int)(w & 0x7fffu);
    double r0 = r[0], r1 = r[1], r2 = r[2];
    int e[4];
#pragma unroll
    for (int j = 0; j < 4; j++) e[j] = e0[j];
    int pl = 0;
    bool more = true;
    while (more) {
        more = false;
#pragma unroll
        for (int j = 0; j < 4; j++) {
            if (cur == end) {
                pl = 0xffff;
                break;
            }
            pl = e[j] >> 2;
            if (pl >= hi) break;
            const int b = e[j] & 3;
            const double *mm = mxy_l[pl - lo];
            r0 += mm[b];
            r1 += mm[3 + b];
            r2 += mm[6 + b];
            cur++;
            more = j == 3;
        }
        if (more) {
#pragma unroll
            for (int j = 0; j < 4; j++) e[j] = colent[cur + j];
        }
    }
    Rg[c] = r0;
    Rg[nC + c] = r1;
    Rg[2 * nC + c] = r2;
    cn_l[c] = ((unsigned)pl << 16) | 0x8000u | (unsigned)(cur - cbase);
}

// Adds a chunk's -Mxy (pairs lo..lo+63 of element k, one row of 9 per pair in
// mxy_l) into the row block R_k[a][c] (Rg: this element's [3][nC] block of the
// output, which only this wavefront touches), column by column: each column is
// owned by one lane, which takes its contributions in pair order (colent: pair
// index << 2 | inner slot, sorted by pair, from cbase on for this element;
// padded by four entries) and carries the column's three sums from one chunk
// to the next through Rg.  cn_l packs per column the offset of its next entry
// (low 15 bits: at most 3 * 4096 entries per element), whether the column has
// sums in Rg yet (bit 15) and its next entry's pair index (high 16 bits,
// 0xffff when done).  The columns with an entry in this chunk (at most 3 * 64)
// are first listed densely, entry i at alist[(i / 4) * arow + i % 4], so that
// the walks spread over all lanes; a lane then takes its listed columns two at
// a time and loads both columns' sums, end and next four entries before
// walking either, so a column pair costs one memory round trip.
__device__ __forceinline__ void fold_row_block(double *__restrict__ Rg, unsigned *cn_l, int nC,
                                               const int32_t *__restrict__ cptr, int cbase,
                                               const uint16_t *__restrict__ colent, const double (*mxy_l)[12], int lo,
                                               int lane, unsigned short *alist, int arow, int hi_max = 0x7fffffff)
{
    // pairs lo .. hi-1 (hi_max: the chunk's pairs beyond it take no part)
    const int hi = lo + 64 < hi_max ? lo + 64 : hi_max;
    int nact = 0;
    auto put = [&](int i, int c) { alist[(i >> 2) * arow + (i & 3)] = (unsigned short)c; };
    // the cursors are read four columns at a time, so one LDS round trip serves four ballots
    for (int c0 = 0; c0 < nC; c0 += 256) {
        unsigned w[4];
#pragma unroll
        for (int j = 0; j < 4; j++) {
            const int c = c0 + 64 * j + lane;
            w[j] = c < nC ? cn_l[c] : 0xffff0000u;
        }
#pragma unroll
        for (int j = 0; j < 4; j++) {
            const bool a = (int)(w[j] >> 16) < hi;
            const unsigned long long m = __ballot(a);
            if (a) put(nact + __popcll(m & ((1ull << lane) - 1ull)), c0 + 64 * j + lane);
            nact += __popcll(m);
        }
    }
    __syncthreads();
    for (int i = lane; i < nact; i += 128) {
        const bool two = i + 64 < nact;
        const int c = alist[(i >> 2) * arow + (i & 3)];
        const int c2 = two ? alist[((i + 64) >> 2) * arow + (i & 3)] : 0;
        const unsigned w0 = cn_l[c];
        const unsigned w1 = two ? cn_l[c2] : 0u;
        int e0[4], e1[4], end1 = 0;
        double r0[3] = {0.0, 0.0, 0.0}, r1[3] = {0.0, 0.0, 0.0};
        {
            const int cur = cbase + (int)(w0 & 0x7fffu);
#pragma unroll
            for (int j = 0; j < 4; j++) e0[j] = colent[cur + j];
            if (w0 & 0x8000u) {
#pragma unroll
                for (int a = 0; a < 3; a++) r0[a] = Rg[a * nC + c];
            }
        }
        const int end0 = cptr[c + 1];
        if (two) {
            const int cur = cbase + (int)(w1 & 0x7fffu);
#pragma unroll
            for (int j = 0; j < 4; j++) e1[j] = colent[cur + j];
            if (w1 & 0x8000u) {
#pragma unroll
                for (int a = 0; a < 3; a++) r1[a] = Rg[a * nC + c2];
            }
            end1 = cptr[c2 + 1];
        }
        fold_column(Rg, cn_l, nC, c, w0, end0, cbase, e0, r0, colent, mxy_l, lo, hi);
        if (two) fold_column(Rg, cn_l, nC, c2, w1, end1, cbase, e1, r1, colent, mxy_l, lo, hi);
    }
}

// Fold cursors of one element in LDS [nC] (see fold_row_block); every column
// starts unvisited at its first entry (a column without entries, which the
// plan does not make, gets zero sums here).
__device__ __forceinline__ unsigned *init_row_block(unsigned *dyn, double *__restrict__ Rg, int nC,
                                                    const int32_t *__restrict__ cptr, int cbase,
                                                    const uint16_t *__restrict__ colent, int lane)
{
    // four columns per lane at a time, so that their loads share the round trips
    for (int c0 = lane; c0 < nC; c0 += 256) {
        int e0[4], e1[4], nx[4];
#pragma unroll
        for (int j = 0; j < 4; j++) {
            const int c = c0 + 64 * j;
            e0[j] = c < nC ? cptr[c] : 0;
            e1[j] = c < nC ? cptr[c + 1] : 0;
        }
#pragma unroll
        for (int j = 0; j < 4; j++) nx[j] = e0[j] < e1[j] ? (int)(colent[e0[j]] >> 2) : 0xffff;
#pragma unroll
        for (int j = 0; j < 4; j++) {
            const int c = c0 + 64 * j;
            if (c >= nC) continue;
            dyn[c] = ((unsigned)nx[j] << 16) | (unsigned)(e0[j] - cbase);
            if (e0[j] >= e1[j]) Rg[c] = Rg[nC + c] = Rg[2 * nC + c] = 0.0;
        }
    }
    return dyn;
}

// The deep pairs' part of the row block: each column's remaining entries
// (after the band chunks they are all deep) name deep partners k' holding the
// column's node; the column adds cf_a times the sum of their areas |E_k'|.
// NC columns per lane at a time: their ends, first four entries and sums so
// far are loaded together, so the walks share their round trips.  TAB: the
// deep pairs' areas are in LDS (dtab, by pair index from nb on), so an entry's
// area costs one LDS read instead of two dependent memory loads.
template <bool TAB, int NC = 4>
__device__ __forceinline__ void deep_row_block(double *__restrict__ Rg, const unsigned *cn_l, int nC,
                                               const int32_t *__restrict__ cptr, int cbase,
                                               const uint16_t *__restrict__ colent,
                                               const int32_t *__restrict__ proc_kp, int64_t p0,
                                               const double *__restrict__ a2, const double (&cf)[3], int lane,
                                               const double *dtab = nullptr, int nb = 0)
{
    auto area = [&](int e) -> double { return TAB ? dtab[(e >> 2) - nb] : a2[proc_kp[p0 + (e >> 2)]]; };
    for (int c0 = lane; c0 < nC; c0 += 64 * NC) {
        unsigned w[NC];
        int cur[NC], end[NC], e[NC][4];
        double r[NC][3], S[NC];
#pragma unroll
        for (int j = 0; j < NC; j++) w[j] = c0 + 64 * j < nC ? cn_l[c0 + 64 * j] : 0xffff0000u;
#pragma unroll
        for (int j = 0; j < NC; j++) {
            const int c = c0 + 64 * j;
            const bool live = (w[j] >> 16) != 0xffffu;
            cur[j] = cbase + (int)(w[j] & 0x7fffu);
            end[j] = live ? cptr[c + 1] : cur[j];
#pragma unroll
            for (int i = 0; i < 4; i++) e[j][i] = live ? colent[cur[j] + i] : 0;   // padded by four
#pragma unroll
            for (int a = 0; a < 3; a++) r[j][a] = (live && (w[j] & 0x8000u)) ? Rg[a * nC + c] : 0.0;
            S[j] = 0.0;
        }
#pragma unroll
        for (int j = 0; j < NC; j++) {
            double av[4];
#pragma unroll
            for (int i = 0; i < 4; i++) av[i] = cur[j] + i < end[j] ? area(e[j][i]) : 0.0;
#pragma unroll
            for (int i = 0; i < 4; i++)
                if (cur[j] + i < end[j]) S[j] += av[i];
            cur[j] += 4;
        }
#pragma unroll
        for (int j = 0; j < NC; j++) {
            // columns with more than four deep entries
            while (cur[j] < end[j]) {
                int ee[4];
                double av[4];
#pragma unroll
                for (int i = 0; i < 4; i++) ee[i] = colent[cur[j] + i];
#pragma unroll
                for (int i = 0; i < 4; i++) av[i] = cur[j] + i < end[j] ? area(ee[i]) : 0.0;
#pragma unroll
                for (int i = 0; i < 4; i++)
                    if (cur[j] + i < end[j]) S[j] += av[i];
                cur[j] += 4;
            }
            if ((w[j] >> 16) != 0xffffu) {
#pragma unroll
                for (int a = 0; a < 3; a++) Rg[a * nC + c0 + 64 * j] = r[j][a] + cf[a] * S[j];
            }
        }
    }
}

// One wavefront per outer element k (Eq. (bformhj) restricted to the pairs
// of k).  Phase 1: every lane takes one pair (k, k'), classifies its items
// (x_{k,q}, E_k') as whole / partial / empty; whole items (all of E_k' in the
// ball, or the barycenter inside for the barycenter ball) only add their
// outer weights, since with constant psi their inner sums are rule
// constants times |E_k'|.  Partial items are queued in LDS.  Phase 2: the
// wave takes queued items 64 at a time (dense, regardless of owner),
// retriangulates them, and each owner adds its items' sums in q order.
// With the plan's processing order (nband), the chunks take the band pairs
// only; deep pairs (every item whole) are summed afterwards from their inner
// elements' areas (SYM), and their Myy reaches the element blocks through
// Dk(k).  Outputs: Myy (6) per band pair; per element Mxx (6) from the
// fixed-order lane reduction of sum_k' S0(x_q), Dk, and the row block
// R_k[a][c] = sum of -Mxy_ab over the pairs whose inner slot b is node
// C_k[c], reduced column by column in pair order (each column owned by one
// lane per chunk, its running sums kept in this element's block of Rout).
template <int NQ, bool SYM, bool POW2, bool BND, bool SW>
__global__ __launch_bounds__(64, (SYM && POW2 && BND && !SW) ? 3 : 2) void k_pairs_const_fp64(const int64_t *__restrict__ pair_ptr,
                                                         const int32_t *__restrict__ pair_kp, ElemSoA E,
                                                         const double *__restrict__ xq, const RuleSet *__restrict__ R,
                                                         double dd, double psi, int ball, int ncap, int centroid,
                                                         double delta, const double *__restrict__ xq2,
                                                         const uint8_t *__restrict__ pair_r2,
                                                         const int64_t *__restrict__ col_off,
                                                         const int32_t *__restrict__ colent_ptr,
                                                         const uint16_t *__restrict__ colent, double *__restrict__ Rout,
                                                         double *__restrict__ Cyy, double *__restrict__ Cxx,
                                                         const int32_t *__restrict__ proc_p,
                                                         const int32_t *__restrict__ proc_kp,
                                                         const int32_t *__restrict__ nband, double *__restrict__ Dk,
                                                         unsigned long long *__restrict__ counters,
                                                         const int32_t *__restrict__ korder)
{
    extern __shared__ unsigned dyn[];
    __shared__ double sW[NQ][4];
    __shared__ double sX[NQ][2];
    // SW: the second outer rule's weights and points (pairs with pair_r2 set); this
    // variant also integrates exact caps (centroid rule or closed form) when asked
    __shared__ double sW2[SW ? NQ : 1][4];
    __shared__ double sX2[SW ? NQ : 1][2];
    // each lane's inner element for phase 2: its vertices (re-read from memory
    // except in the SW variant, bound by its registers) and, for the boundary
    // form, the rows of its inverse edge matrix, formed once per pair
    __shared__ int skp[64];
    __shared__ double sV[SW ? 64 : 1][7];
    __shared__ double sG[BND ? 64 : 1][4];
    // the phase-2 queue, later the fold's list of active columns (at most 3 * 64)
    __shared__ unsigned short queue[64 * NQ];
    static_assert(NQ >= 3, "the queue holds the fold's column list");
    // item results of a phase-2 round, later the chunk's -Mxy (never live together)
    __shared__ double res[64][12];
    double (*mxy_l)[12] = res;
    const int k = korder[blockIdx.x], lane = threadIdx.x;
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
    const int nq2 = SW ? R->n_out2 : 0;
    if (SW && lane < nq2) {
        double W = R->out2_w[lane] * a2k;
        sW2[lane][0] = W;
        sW2[lane][1] = W * R->out2_lam[lane][0];
        sW2[lane][2] = W * R->out2_lam[lane][1];
        sW2[lane][3] = W * R->out2_lam[lane][2];
        sX2[lane][0] = xq2[2 * ((int64_t)k * nq2 + lane)];
        sX2[lane][1] = xq2[2 * ((int64_t)k * nq2 + lane) + 1];
    }
    __syncthreads();
    const RuleMom M = load_moments(R);
    const int64_t coff = col_off[k];
    const int nC = (int)(col_off[k + 1] - coff);
    double *Rg = Rout + 3 * coff;                       // [3][nC], this element's row block
    const int cbase = colent_ptr[coff];
    unsigned *cn_l = init_row_block(dyn, Rg, nC, colent_ptr + coff, cbase, colent, lane);
    double m0[NQ], m0b[SW ? NQ : 1];
#pragma unroll
    for (int q = 0; q < NQ; q++) m0[q] = 0.0;
#pragma unroll
    for (int q = 0; q < (SW ? NQ : 1); q++) m0b[q] = 0.0;
    unsigned long long c_whole = 0, c_part = 0, c_empty = 0, c_sub = 0, c_cap = 0;
    const int64_t p0 = pair_ptr[k], p1 = pair_ptr[k + 1];
    // pairs are visited in the plan's processing order when it has one: those
    // that can have partial items first, then the deep ones, whose items are
    // all whole (chunks of deep pairs skip the classification)
    const int64_t nb = nband ? (int64_t)nband[k] : p1 - p0;
    // deep pairs leave no Myy record: their inner elements are this element's
    // deep partners (the deep test is symmetric), so E(k) takes their Myy
    // from Dk(k) = psi sum_w sum_deep |E_k'| (sum_w: the outer weights' sum)
    double dsum = 0.0;
    // With a symmetric inner rule a deep pair reduces to its inner element's
    // area: Mxy_ab = psi AW_a m1c |E_k'| (AW_a = sum_q W_q alpha_a(x_q)) and S0 =
    // wsum |E_k'| at every outer point, and both outer rules integrate these
    // polynomials exactly; so the chunks take the band pairs only and the deep
    // ones are summed after them.
    const bool collapse = SYM && nband != nullptr;
    const int64_t pend = collapse ? p0 + nb : p1;
    // each chunk's inner-element indices are loaded one chunk ahead, so that a
    // chunk starts with one round trip to memory (its elements' records)
    const int32_t *kp_src = proc_kp ? proc_kp : pair_kp;
    int kp_next = p0 + lane < pend ? kp_src[p0 + lane] : 0;
    for (int64_t base = p0; base < pend; base += 64) {
        const int64_t pi = base + lane;                                   // processing slot
        const bool act = pi < pend;
        const int kp = kp_next;
        kp_next = pi + 64 < pend ? kp_src[pi + 64] : 0;
        const int64_t p = (proc_p && act) ? (int64_t)proc_p[pi] : pi;    // the pair's canonical index
        const bool deep = act && pi - p0 >= nb;
        double V[6] = {0, 0, 0, 0, 0, 0};
        double a2p = 0.0, bxp = 0.0, byp = 0.0;
        if (act && !deep) {
            // the inner element's record in five 16-byte loads
            const double2 *rec = (const double2 *)(E.pk + 16 * (int64_t)kp);
            const double2 r0 = rec[0], r1 = rec[1], r2v = rec[2], r3 = rec[3], r4 = rec[4];
            V[0] = r0.x; V[1] = r0.y; V[2] = r1.x; V[3] = r1.y; V[4] = r2v.x; V[5] = r2v.y;
            bxp = r3.x;
            byp = r3.y;
            a2p = r4.x;
        } else if (act) {
            // a deep pair needs only the inner element's area
            a2p = E.a2[kp];
        }
        if (deep) dsum += a2p;
        skp[lane] = kp;
        if (SW) {
#pragma unroll
            for (int i = 0; i < 6; i++) sV[SW ? lane : 0][i] = V[i];
        }
        if (BND && act && !deep) {
            double g[4];
            inv_edges(V, g);
#pragma unroll
            for (int i = 0; i < 4; i++) sG[BND ? lane : 0][i] = g[i];
        }

        double ws = 0.0, aw[3] = {0.0, 0.0, 0.0};
        unsigned pmask = 0;
        const bool r2 = SW && nq2 > 0 && act && pair_r2[p];
        const int nqp = r2 ? nq2 : nq;
        if (act) {
#pragma unroll
            for (int q = 0; q < NQ; q++) {
                if (q >= nqp) break;
                const double xx = r2 ? sX2[q][0] : sX[q][0], xy = r2 ? sX2[q][1] : sX[q][1];
                bool whole = false, part = false;
                if (deep) {
                    whole = true;
                } else if (ball == NLA_BALL_BARYCENTER) {
                    whole = bary_in(xx, xy, bxp, byp, dd);
                } else {
                    // overlap ball: every element meeting the ball counts whole
                    const int cls = item_class(xx, xy, V, dd);
                    whole = cls == 1 || (ball == NLA_BALL_OVERLAP && cls == 2);
                    part = cls == 2 && ball != NLA_BALL_OVERLAP;
                }
                if (whole) {
                    const double *w4 = r2 ? sW2[q] : sW[q];
                    ws += w4[0];
                    aw[0] += w4[1];
                    aw[1] += w4[2];
                    aw[2] += w4[3];
                    if (r2) m0b[q] += a2p * M.wsum;
                    else m0[q] += a2p * M.wsum;
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
        // queue the partial items outer point by outer point (point 0 of every
        // lane in lane order, then point 1, ...), so that a round of 64 queued
        // items holds at most a few of any one lane: its owner then collects
        // them in a short loop.  A lane's items keep their q order.
        const unsigned long long lt = (1ull << lane) - 1ull;
        int total = 0;
#pragma unroll
        for (int q = 0; q < NQ; q++) {
            const bool mine = (pmask >> q) & 1u;
            const unsigned long long bq = __ballot(mine);
            if (mine) queue[total + __popcll(bq & lt)] = (unsigned short)((lane << 8) | (r2 ? 0x80 : 0) | q);
            total += __popcll(bq);
        }
        __syncthreads();
        for (int ib = 0; ib < total; ib += 64) {
            const int i = ib + lane;
            if (i < total) {
                const int e = queue[i], owner = e >> 8, q = e & 0x0f;
                const bool rr = SW && (e & 0x80);
                const double qx = rr ? sX2[q][0] : sX[q][0], qy = rr ? sX2[q][1] : sX[q][1];
                double Vo[6], iLo[3] = {0.0, 0.0, 0.0};
                if (SW) {
#pragma unroll
                    for (int i = 0; i < 6; i++) Vo[i] = sV[SW ? owner : 0][i];
                } else {
                    const double2 *rec = (const double2 *)(E.pk + 16 * (int64_t)skp[owner]);
                    const double2 r0 = rec[0], r1 = rec[1], r2v = rec[2], r5 = rec[5], r6 = rec[6];
                    Vo[0] = r0.x; Vo[1] = r0.y; Vo[2] = r1.x; Vo[3] = r1.y; Vo[4] = r2v.x; Vo[5] = r2v.y;
                    iLo[0] = r5.x; iLo[1] = r5.y; iLo[2] = r6.x;
                }
                Acc A;
                A.a2 = 0.0;
#pragma unroll
                for (int t = 0; t < 3; t++) A.s1[t] = 0.0;
#pragma unroll
                for (int t = 0; t < 6; t++) A.s2[t] = 0.0;
                int ns = 0;
                if (BND) {
                    // the rule is exact for quadratics: the region's moments from its boundary
                    RegionMom Rm = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
                    partial_boundary<POW2, SW>(qx, qy, Vo, dd, ncap, Rm, ns, &res[lane][0], centroid, delta,
                                               SW ? nullptr : iLo);
                    double s0, s1[3], s2[6], g[4];
#pragma unroll
                    for (int i = 0; i < 4; i++) g[i] = sG[BND ? owner : 0][i];
                    region_sums_g(Rm, g, s0, s1, s2);
                    res[lane][0] = s0;
#pragma unroll
                    for (int t = 0; t < 3; t++) res[lane][1 + t] = s1[t];
#pragma unroll
                    for (int t = 0; t < 6; t++) res[lane][4 + t] = s2[t];
                } else {
                    auto tri = [&](const double (&t)[3][5]) { tri_accum<SYM>(t, M, A); };
                    // the cap endpoints live in this lane's row of res until the sums are written
                    partial_item<POW2>(qx, qy, Vo, dd, ncap, tri, ns, &res[lane][0]);
                    res[lane][0] = A.a2 * M.wsum;
#pragma unroll
                    for (int t = 0; t < 3; t++) res[lane][1 + t] = SYM ? A.s1[t] * M.m1c : A.s1[t];
#pragma unroll
                    for (int t = 0; t < 6; t++) res[lane][4 + t] = A.s2[t];
                }
                c_sub += ns & 0xffff;
                c_cap += ns >> 16;
            }
            __syncthreads();
            // each owner adds its items of this round in q order; the outer
            // points with none in the round are skipped by the whole wave
            int qbase = 0;
#pragma unroll
            for (int q = 0; q < NQ; q++) {
                const bool mine = (pmask >> q) & 1u;
                const unsigned long long bq = __ballot(mine);
                const int qb = qbase, nqi = __popcll(bq);
                qbase += nqi;
                if (qb + nqi <= ib || qb >= ib + 64) continue;      // point q's items lie outside the round
                const int pos = qb + __popcll(bq & lt);
                const bool inr = mine && pos >= ib && pos < ib + 64;
                if (inr) {
                    const double *r = res[pos - ib];
                    if (r2) m0b[SW ? q : 0] += r[0];
                    else m0[q] += r[0];
                    const double *w4 = r2 ? sW2[SW ? q : 0] : sW[q];
                    const double W = w4[0];
#pragma unroll
                    for (int a = 0; a < 3; a++)
#pragma unroll
                        for (int b = 0; b < 3; b++) axy[a][b] += w4[1 + a] * r[1 + b];
#pragma unroll
                    for (int t = 0; t < 6; t++) ayy[t] += W * r[4 + t];
                }
            }
            __syncthreads();
        }
        if (act) {
#pragma unroll
            for (int a = 0; a < 3; a++)
#pragma unroll
                for (int b = 0; b < 3; b++) mxy_l[lane][3 * a + b] = -psi * axy[a][b];
            if (!deep) {
#pragma unroll
                for (int t = 0; t < 6; t++) Cyy[6 * p + t] = psi * ayy[t];
            }
        }
        __syncthreads();
        fold_row_block(Rg, cn_l, nC, colent_ptr + coff, cbase, colent, mxy_l, (int)(base - p0), lane, queue, 4,
                       (int)(pend - p0));
        __syncthreads();
    }
    if (collapse) {
        // the deep pairs: their areas, each item counted whole; four pairs per
        // lane at a time: their indices, then their areas, then the sums in the
        // lane's pair order
        // (the areas are kept in LDS, in res, free after the chunks, when they fit)
        double *dtab = &res[0][0];
        const bool tab = p1 - pend <= 64 * 12;
        for (int64_t pi0 = pend + lane; pi0 < p1; pi0 += 256) {
            int kq[4];
#pragma unroll
            for (int j = 0; j < 4; j++) kq[j] = pi0 + 64 * j < p1 ? proc_kp[pi0 + 64 * j] : -1;
            double av[4];
#pragma unroll
            for (int j = 0; j < 4; j++) av[j] = kq[j] >= 0 ? E.a2[kq[j]] : 0.0;
#pragma unroll
            for (int j = 0; j < 4; j++) {
                if (kq[j] < 0) continue;
                const int64_t pi = pi0 + 64 * j;
                dsum += av[j];
                if (tab) dtab[pi - pend] = av[j];
                c_whole += (SW && nq2 > 0 && pair_r2[proc_p[pi]]) ? nq2 : nq;
            }
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < NQ; q++)
            if (q < nq) m0[q] += dsum * M.wsum;
        // row block: R_k[a][c] += -psi m1c AW_a S(c), S(c) the areas of the deep
        // partners with node c, from each column's remaining entries (all deep)
        double cf[3] = {0.0, 0.0, 0.0};
        for (int q = 0; q < nq; q++) {
#pragma unroll
            for (int a = 0; a < 3; a++) cf[a] += sW[q][1 + a];
        }
#pragma unroll
        for (int a = 0; a < 3; a++) cf[a] *= -psi * M.m1c;
        if (tab)
            deep_row_block<true, 5>(Rg, cn_l, nC, colent_ptr + coff, cbase, colent, proc_kp, p0, E.a2, cf, lane,
                                    dtab, (int)nb);
        else
            deep_row_block<false>(Rg, cn_l, nC, colent_ptr + coff, cbase, colent, proc_kp, p0, E.a2, cf, lane);
    }
    // Mxx(k) = sum_q W_q alpha alpha^T psi sum_k' S0: a fixed butterfly over the
    // lanes, then lane 0's sum is broadcast
#pragma unroll
    for (int q = 0; q < NQ; q++) {
        double x = m0[q];
        for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
        m0[q] = __shfl(x, 0, 64);
    }
#pragma unroll
    for (int q = 0; q < (SW ? NQ : 0); q++) {
        double x = m0b[q];
        for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
        m0b[q] = __shfl(x, 0, 64);
    }
    if (lane < 6) {
        const int aa[6] = {0, 0, 0, 1, 1, 2}, cc[6] = {0, 1, 2, 1, 2, 2};
        const int a = aa[lane], c = cc[lane];
        double s = 0.0;
#pragma unroll
        for (int q = 0; q < NQ; q++)
            if (q < nq) s += sW[q][1 + a] * R->out_lam[q][c] * m0[q];
#pragma unroll
        for (int q = 0; q < (SW ? NQ : 0); q++)
            if (q < nq2) s += sW2[q][1 + a] * R->out2_lam[q][c] * m0b[q];
        Cxx[6 * (int64_t)k + lane] = psi * s;
    }
    if (Dk) {
        double x = dsum;
        for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
        if (lane == 0) {
            double wsum = 0.0;
            for (int q = 0; q < nq; q++) wsum += R->out_w[q];
            Dk[k] = psi * wsum * x;
        }
    }
    // work counters
    unsigned long long v[5] = {c_whole, c_part, c_empty, c_sub, c_cap};
#pragma unroll
    for (int i = 0; i < 5; i++) {
        unsigned long long x = v[i];
        for (int off = 32; off > 0; off >>= 1) x += __shfl_down(x, off, 64);
        v[i] = x;
    }
    if (counters && lane == 0) {
        atomicAdd(&counters[0], v[0]);
        atomicAdd(&counters[1], v[1]);
        atomicAdd(&counters[2], v[2]);
        atomicAdd(&counters[4], v[3]);
        atomicAdd(&counters[5], v[4]);
    }
}

// The shifted ball (Sec. 4.3) and the barycenter ball with its outer support
// resolved (Sec. 6, case 2) integrate one region per pair instead of one per
// (pair, outer point).  One wavefront per outer element k, one lane per pair:
//  * shifted: R = E_k' n B_delta,h(b_k) serves every x in E_k; its inner sums
//    S0, S1_b, S2_bb' (moments through the boundary, the inner rule being exact
//    for quadratics) meet the outer rule over the whole E_k:
//    Mxx = (sum_q W_q alpha alpha^T) S0, Mxy_ab = (sum_q W_q alpha_a) S1_b,
//    Myy = (sum_q W_q) S2;
//  * barycenter support: the inner integrand is non-zero for x in
//    S = E_k n B_delta,h(b_k'), where it runs over the whole E_k' (rule
//    constants T0, T1_b, T2_bb'); the outer rule over the triangles of S is
//    exact for alpha alpha^T, so S's moments a0, a1_a, a2_aa' give
//    Mxx = a2 T0, Mxy_ab = a1_a T1_b, Myy = a0 T2.
// A region is whole (every vertex in the ball), empty, or cut (moments from
// its boundary, caps over ncap equal arcs).  Outputs as k_pairs_const_fp64.
template <bool POW2>
__global__ __launch_bounds__(64) void k_pairs_support_fp64(const int64_t *__restrict__ pair_ptr,
                                                        const int32_t *__restrict__ pair_kp, ElemSoA E,
                                                        const RuleSet *__restrict__ R, double dd, double psi,
                                                        int ball, int ncap, const int64_t *__restrict__ col_off,
                                                        const int32_t *__restrict__ colent_ptr,
                                                        const uint16_t *__restrict__ colent, double *__restrict__ Rout,
                                                        double *__restrict__ Cyy, double *__restrict__ Cxx,
                                                        const int32_t *__restrict__ proc_p,
                                                        const int32_t *__restrict__ proc_kp,
                                                        const int32_t *__restrict__ nband, double *__restrict__ Dk,
                                                        unsigned long long *__restrict__ counters,
                                                        const int32_t *__restrict__ korder)
{
    extern __shared__ unsigned dyn[];
    __shared__ double sQ[10];           // the outer rule over E_k: sum W, sum W alpha_a, sum W alpha_a alpha_c
    // a lane's cap endpoints, then its pair's -Mxy (entries 0..8), with the fold's
    // list of active columns in entries 9..11 of the first 48 rows
    __shared__ double res[64][12];
    const int k = korder[blockIdx.x], lane = threadIdx.x;
    const double a2k = E.a2[k];
    const int jj[6] = {0, 0, 0, 1, 1, 2}, ll[6] = {0, 1, 2, 1, 2, 2};
    if (lane < 10) {
        double v = 0.0;
        for (int q = 0; q < R->n_out; q++) {
            const double W = R->out_w[q] * a2k;
            if (lane == 0) v += W;
            else if (lane < 4) v += W * R->out_lam[q][lane - 1];
            else v += W * R->out_lam[q][jj[lane - 4]] * R->out_lam[q][ll[lane - 4]];
        }
        sQ[lane] = v;
    }
    __syncthreads();
    const RuleMom M = load_moments(R);
    const double bkx = E.bx[k], bky = E.by[k];
    const double Vk[6] = {E.vx0[k], E.vy0[k], E.vx1[k], E.vy1[k], E.vx2[k], E.vy2[k]};
    const int64_t coff = col_off[k];
    const int nC = (int)(col_off[k + 1] - coff);
    double *Rg = Rout + 3 * coff;                       // [3][nC], this element's row block
    const int cbase = colent_ptr[coff];
    unsigned *cn_l = init_row_block(dyn, Rg, nC, colent_ptr + coff, cbase, colent, lane);
    double s0sum = 0.0, mxx[6] = {0, 0, 0, 0, 0, 0};
    unsigned long long c_whole = 0, c_part = 0, c_empty = 0, c_sub = 0, c_cap = 0;
    const int64_t p0 = pair_ptr[k], p1 = pair_ptr[k + 1];
    // with the plan's processing order (symmetric inner rule) the chunks take the
    // band pairs only; a deep pair's region is whole, so its blocks follow from
    // |E_k'| and it is summed after the chunks (as in k_pairs_const_fp64)
    const int64_t pend = nband ? p0 + nband[k] : p1;
    for (int64_t base = p0; base < pend; base += 64) {
        const int64_t pi = base + lane;                                   // processing slot
        const bool act = pi < pend;
        const int64_t p = (proc_p && act) ? (int64_t)proc_p[pi] : pi;    // the pair's canonical index
        double mxy[9], myy[6];
#pragma unroll
        for (int i = 0; i < 9; i++) mxy[i] = 0.0;
#pragma unroll
        for (int i = 0; i < 6; i++) myy[i] = 0.0;
        if (act) {
            const int kp = proc_kp ? proc_kp[pi] : pair_kp[p];
            const double V[6] = {E.vx0[kp], E.vy0[kp], E.vx1[kp], E.vy1[kp], E.vx2[kp], E.vy2[kp]};
            const double a2p = E.a2[kp];
            const bool shifted = ball == NLA_BALL_SHIFTED;
            // the cut element (selected by value, so that both stay in registers)
            // and the centre of the ball that cuts it
            const double cx = shifted ? bkx : E.bx[kp], cy = shifted ? bky : E.by[kp];
            double Vc[6];
#pragma unroll
            for (int i = 0; i < 6; i++) Vc[i] = shifted ? V[i] : Vk[i];
            const double ac = shifted ? a2p : a2k;
            const int cls = item_class(cx, cy, Vc, dd);
            double g0 = 0.0, g1[3] = {0, 0, 0}, g2[6] = {0, 0, 0, 0, 0, 0};   // the region's moments
            if (cls == 1) {
                // whole element: the rule's constants (inner rule on E_k', or the outer rule on E_k)
                if (shifted) {
                    g0 = ac * M.wsum;
#pragma unroll
                    for (int b = 0; b < 3; b++) g1[b] = ac * M.m1[b];
#pragma unroll
                    for (int t = 0; t < 6; t++) g2[t] = ac * M.m2[jj[t]][ll[t]];
                } else {
                    g0 = sQ[0];
#pragma unroll
                    for (int b = 0; b < 3; b++) g1[b] = sQ[1 + b];
#pragma unroll
                    for (int t = 0; t < 6; t++) g2[t] = sQ[4 + t];
                }
                c_whole++;
            } else if (cls == 2) {
                RegionMom Rm = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
                int ns = 0;
                partial_boundary<POW2>(cx, cy, Vc, dd, ncap, Rm, ns, &res[lane][0]);
                region_sums(Rm, Vc, g0, g1, g2);
                c_sub += ns & 0xffff;
                c_cap += ns >> 16;
                c_part++;
            } else {
                c_empty++;
            }
            if (shifted) {
                s0sum += g0;
#pragma unroll
                for (int a = 0; a < 3; a++)
#pragma unroll
                    for (int b = 0; b < 3; b++) mxy[3 * a + b] = sQ[1 + a] * g1[b];
#pragma unroll
                for (int t = 0; t < 6; t++) myy[t] = sQ[0] * g2[t];
            } else {
                const double t0 = a2p * M.wsum;
#pragma unroll
                for (int t = 0; t < 6; t++) mxx[t] += g2[t] * t0;
#pragma unroll
                for (int a = 0; a < 3; a++)
#pragma unroll
                    for (int b = 0; b < 3; b++) mxy[3 * a + b] = g1[a] * (a2p * M.m1[b]);
#pragma unroll
                for (int t = 0; t < 6; t++) myy[t] = g0 * (a2p * M.m2[jj[t]][ll[t]]);
            }
        }
        if (act) {
#pragma unroll
            for (int i = 0; i < 9; i++) res[lane][i] = -psi * mxy[i];
#pragma unroll
            for (int t = 0; t < 6; t++) Cyy[6 * p + t] = psi * myy[t];
        }
        __syncthreads();
        fold_row_block(Rg, cn_l, nC, colent_ptr + coff, cbase, colent, res, (int)(base - p0), lane,
                       (unsigned short *)&res[0][9], 48, (int)(pend - p0));
        __syncthreads();
    }
    if (nband) {
        // deep pairs: S0 sums wsum |E_k'|, -Mxy_ab = -psi m1 sQ_a |E_k'| per column
        // through its deep partners, Myy per element through Dk
        double dsum = 0.0;
        for (int64_t pi = pend + lane; pi < p1; pi += 64) {
            dsum += E.a2[proc_kp[pi]];
            c_whole++;
        }
        if (ball == NLA_BALL_SHIFTED) {
            s0sum += dsum * M.wsum;
        } else {
#pragma unroll
            for (int t = 0; t < 6; t++) mxx[t] += sQ[4 + t] * (dsum * M.wsum);
        }
        const double cf[3] = {-psi * M.m1c * sQ[1], -psi * M.m1c * sQ[2], -psi * M.m1c * sQ[3]};
        deep_row_block<false>(Rg, cn_l, nC, colent_ptr + coff, cbase, colent, proc_kp, p0, E.a2, cf, lane);
        double x = dsum;
        for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
        if (lane == 0) {
            double wsum = 0.0;
            for (int q = 0; q < R->n_out; q++) wsum += R->out_w[q];
            Dk[k] = psi * wsum * x;
        }
    }
    // Mxx(k): a fixed butterfly over the lanes, lane 0's sum broadcast
    {
        double x = s0sum;
        for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
        s0sum = __shfl(x, 0, 64);
    }
#pragma unroll
    for (int t = 0; t < 6; t++) {
        double x = mxx[t];
        for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
        mxx[t] = __shfl(x, 0, 64);
    }
    if (lane < 6) {
        double v = 0.0;
#pragma unroll
        for (int t = 0; t < 6; t++)
            if (t == lane) v = ball == NLA_BALL_SHIFTED ? sQ[4 + t] * s0sum : mxx[t];
        Cxx[6 * (int64_t)k + lane] = psi * v;
    }
    unsigned long long v[5] = {c_whole, c_part, c_empty, c_sub, c_cap};
#pragma unroll
    for (int i = 0; i < 5; i++) {
        unsigned long long x = v[i];
        for (int off = 32; off > 0; off >>= 1) x += __shfl_down(x, off, 64);
        v[i] = x;
    }
    if (counters && lane == 0) {
        atomicAdd(&counters[0], v[0]);
        atomicAdd(&counters[1], v[1]);
        atomicAdd(&counters[2], v[2]);
        atomicAdd(&counters[4], v[3]);
        atomicAdd(&counters[5], v[4]);
    }
}

// Element blocks E(k') = Mxx(k') + sum_k Myy(k, k'): one wavefront per k'
// over its pairs in the transposed order (k ascending); lane l takes every
// 64th pair from l, lanes are combined by a fixed butterfly.  With Dk, the
// transposed order lists band pairs only and the deep pairs' Myy, all of the
// form psi sum_w |E_k| |E_k'| m2 (every item whole), come as Dk(k') |E_k'| m2.
template <class T>
__global__ __launch_bounds__(64) void k_elem_blocks(int K, const int64_t *__restrict__ tptr,
                                                    const int32_t *__restrict__ tperm, const T *__restrict__ Cyy,
                                                    const T *__restrict__ Cxx, T *__restrict__ Ce,
                                                    const double *__restrict__ Dk, const double *__restrict__ a2,
                                                    const RuleSet *__restrict__ R)
{
    const int64_t kb = xcd_block(blockIdx.x, gridDim.x);
    if (kb >= K) return;
    const int k = (int)kb, lane = threadIdx.x;
    double y[6] = {0, 0, 0, 0, 0, 0};
    // two pairs' loads in flight per step (the additions keep the lane's order)
    const int64_t te = tptr[k + 1];
    int64_t t = tptr[k] + lane;
    for (; t + 64 < te; t += 128) {
        const int64_t pa = tperm[t], pb = tperm[t + 64];
        T a[6], b[6];
#pragma unroll
        for (int i = 0; i < 6; i++) {
            a[i] = Cyy[6 * pa + i];
            b[i] = Cyy[6 * pb + i];
        }
#pragma unroll
        for (int i = 0; i < 6; i++) {
            y[i] += (double)a[i];
            y[i] += (double)b[i];
        }
    }
    if (t < te) {
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
        double x = (double)Cxx[6 * (int64_t)k + lane];
        if (Dk) {
            const int jj[6] = {0, 0, 0, 1, 1, 2}, ll[6] = {0, 1, 2, 1, 2, 2};
            x += Dk[k] * a2[k] * R->in_m2[jj[lane]][ll[lane]];
        }
        Ce[6 * (int64_t)k + lane] = (T)(v + x);
    }
}

// Deterministic COO->CSR sum: every upper-triangle entry adds its
// contributions in the fixed order of its code list and writes the sum to
// both mirrored positions, so D is bitwise symmetric and run-to-run identical.
__global__ void k_segsum_f64(int64_t n_up, const int64_t *__restrict__ up_ptr, const int32_t *__restrict__ codes,
                             const int64_t *__restrict__ up_dst, const int64_t *__restrict__ mirror,
                             const double *__restrict__ C, double *__restrict__ val)
{
    int64_t u = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
    if (u >= n_up) return;
    double s = 0.0;
    // four codes' loads in flight per step (the additions keep the code order)
    const int64_t te = up_ptr[u + 1];
    int64_t t = up_ptr[u];
    for (; t + 4 <= te; t += 4) {
        const int c0 = codes[t], c1 = codes[t + 1], c2 = codes[t + 2], c3 = codes[t + 3];
        const double v0 = C[c0], v1 = C[c1], v2 = C[c2], v3 = C[c3];
        s += v0;
        s += v1;
        s += v2;
        s += v3;
    }
    for (; t < te; t++) s += C[codes[t]];
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

// Dynamic LDS for a launch of fn (64 threads per workgroup): `need` bytes,
// raised when more than wg_per_cu workgroups would otherwise share a CU, so
// that at most wg_per_cu do (0: no cap).  The FP64 pair kernels run uncapped:
// on c2 a cap of 8, 10 or 12 workgroups per CU is as fast or slower than none.
static size_t lds_for_occupancy(const void *fn, size_t need, int wg_per_cu)
{
    int n = 0;
    if (wg_per_cu <= 0 || hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, fn, 64, need) != hipSuccess ||
        n <= wg_per_cu)
        return need;
    size_t lo = need, hi = 64 * 1024;           // lo gives too many workgroups per CU
    int nh = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nh, fn, 64, hi) != hipSuccess || nh > wg_per_cu) return need;
    while (hi - lo > 256) {
        const size_t mid = (lo + hi) / 2;
        int nm = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nm, fn, 64, mid) != hipSuccess) return need;
        if (nm > wg_per_cu) lo = mid;
        else hi = mid;
    }
    return hi;
}

static void nla_mark(nla_plan *P, int i, hipStream_t s)
{
    if (P->cur_ev) (void)hipEventRecord(P->cur_ev[i], s);
}

int nla_numeric(nla_plan *P, const double *f_outer, const double *g_node, hipStream_t s)
{
    const nla_problem &pr = P->prob;
    const bool fp64 = pr.precision == NLA_FP64;
    if (fp64 && pr.kernel != NLA_KERNEL_CONSTANT) {
        nla_set_error("the FP64 path assembles the constant kernel; use NLA_FP32 for the fractional kernel");
        return NLA_E_UNSUPPORTED;
    }
    const int64_t NP = P->n_pairs;
    const int K = P->K;
    const size_t es = fp64 ? sizeof(double) : sizeof(float);
    if (!P->contrib) {
        P->n_contrib = 6 * NP + 13 * (int64_t)K + 3 * P->n_cols;   // ... | Ce (6K) | Dk (K)
        NLA_TRY(P->arena.alloc(&P->contrib, es * P->n_contrib));
        NLA_TRY(P->arena.alloc(&P->val, es * P->nnz));
        NLA_TRY(P->arena.alloc(&P->a_val, es * (P->nnz_free > 0 ? P->nnz_free : 1)));
        NLA_TRY(P->arena.alloc(&P->near_blk, es * (P->n_near > 0 ? 21 * P->n_near : 1)));
        NLA_TRY(P->arena.get(&P->Gk, 3 * (size_t)K));
        NLA_TRY(P->arena.get(&P->b, P->n_free > 0 ? P->n_free : 1));
    }
    const bool timed = P->timing_count < P->timing_slots;
    P->cur_ev = timed ? &P->ev[(size_t)P->timing_count * (NLA_NPHASE + 1)] : nullptr;
    for (int i = 0; i < NLA_NPHASE; i++) P->ran[i] = false;
    // the item counters depend on the geometry only: the first assembly counts,
    // later ones pass no counters (and launch no clearing of them)
    unsigned long long *ctr = P->counted ? nullptr : P->counters;
    if (ctr) NLA_HIP(hipMemsetAsync(ctr, 0, sizeof(unsigned long long) * 6, s));
    if (fp64) {
        double *Cyy = (double *)P->contrib;
        double *Cxx = Cyy + 6 * NP;
        double *V = Cxx + 6 * (int64_t)K;          // [R (3 n_cols) | E (6K)]: the values the codes index
        double *Ce = V + 3 * P->n_cols;
        double *Dk = P->nband ? Ce + 6 * (int64_t)K : nullptr;   // deep pairs' Myy per element
        nla_mark(P, NLA_PHASE_MLP, s);
        nla_mark(P, NLA_PHASE_PAIRS, s);
        const size_t lds = (size_t)P->max_cols * sizeof(unsigned);
        const bool cuts = pr.ball == NLA_BALL_RETRI || pr.ball == NLA_BALL_SHIFTED || pr.ball == NLA_BALL_BARYSUPPORT;
        const int ncap = cuts ? pr.cap_edges : 0;
#define NLA_LAUNCH_PAIRS(NQ, SYM, POW2, BND, SW)                                                                   \
    do {                                                                                                           \
        if (P->pairs_lds == 0) {                                                                                   \
            const void *fn = (const void *)k_pairs_const_fp64<NQ, SYM, POW2, BND, SW>;                             \
            P->pairs_lds = lds_for_occupancy(fn, lds, NLA_PAIRS_WG_PER_CU);                                        \
        }                                                                                                          \
        k_pairs_const_fp64<NQ, SYM, POW2, BND, SW><<<K, 64, P->pairs_lds, s>>>(                                    \
            P->pair_ptr, P->pair_kp, P->E, P->xq, P->d_rules, pr.delta * pr.delta, pr.kernel_c, pr.ball, ncap,       \
            pr.cap_mode, pr.delta, P->xq2, P->pair_r2, P->col_off, P->colent_ptr, P->colent, V, Cyy, Cxx,            \
            P->proc_p, P->proc_kp, P->nband, Dk, ctr, P->korder);                                                  \
    } while (0)
        const bool sym = P->rules.in_sym != 0;
        const bool pow2 = (ncap & (ncap - 1)) == 0;     // 0 (no caps) counts as a power of two
        const bool bnd = P->rules.in_q2exact != 0 && pr.ball == NLA_BALL_RETRI;
        // the variant with the second outer rule also carries the exact caps
        const bool sw = P->rules.n_out2 > 0 || pr.cap_mode != NLA_CAPS_ARCS;
        if (sw && !(sym && pow2 && P->rules.n_out <= 8)) {
            nla_set_error("a second outer rule needs outer rules of at most 8 points, a symmetric inner rule and "
                          "2^m arcs per cap");
            return NLA_E_UNSUPPORTED;
        }
        if (pr.ball == NLA_BALL_SHIFTED || pr.ball == NLA_BALL_BARYSUPPORT) {
            if (P->pairs_lds == 0)
                P->pairs_lds = lds_for_occupancy(pow2 ? (const void *)k_pairs_support_fp64<true>
                                                      : (const void *)k_pairs_support_fp64<false>,
                                                 lds, NLA_SUPPORT_WG_PER_CU);
            if (pow2)
                k_pairs_support_fp64<true><<<K, 64, P->pairs_lds, s>>>(P->pair_ptr, P->pair_kp, P->E, P->d_rules,
                                                               pr.delta * pr.delta, pr.kernel_c, pr.ball, ncap,
                                                               P->col_off, P->colent_ptr, P->colent, V, Cyy, Cxx,
                                                               P->proc_p, P->proc_kp, P->nband, Dk, ctr, P->korder);
            else
                k_pairs_support_fp64<false><<<K, 64, P->pairs_lds, s>>>(P->pair_ptr, P->pair_kp, P->E, P->d_rules,
                                                                pr.delta * pr.delta, pr.kernel_c, pr.ball, ncap,
                                                                P->col_off, P->colent_ptr, P->colent, V, Cyy, Cxx,
                                                                P->proc_p, P->proc_kp, P->nband, Dk, ctr, P->korder);
        } else if (sw && bnd) NLA_LAUNCH_PAIRS(8, true, true, true, true);
        else if (sw) NLA_LAUNCH_PAIRS(8, true, true, false, true);
        else if (P->rules.n_out <= 8 && bnd && pow2) NLA_LAUNCH_PAIRS(8, true, true, true, false);
        else if (P->rules.n_out <= 8 && bnd) NLA_LAUNCH_PAIRS(8, true, false, true, false);
        else if (P->rules.n_out <= 8 && sym && pow2) NLA_LAUNCH_PAIRS(8, true, true, false, false);
        else if (P->rules.n_out <= 8 && sym) NLA_LAUNCH_PAIRS(8, true, false, false, false);
        else if (P->rules.n_out <= 8) NLA_LAUNCH_PAIRS(8, false, false, false, false);
        else if (bnd) NLA_LAUNCH_PAIRS(16, false, false, true, false);
        else NLA_LAUNCH_PAIRS(16, false, false, false, false);
#undef NLA_LAUNCH_PAIRS
        NLA_HIP(hipGetLastError());
        P->ran[NLA_PHASE_PAIRS] = true;
        nla_mark(P, NLA_PHASE_NEAR, s);
        nla_mark(P, NLA_PHASE_SEGSUM, s);
        k_elem_blocks<double><<<(unsigned)xcd_grid(K), 64, 0, s>>>(K, P->tptr, P->tperm, Cyy, Cxx, Ce, Dk, P->E.a2,
                                                                   P->d_rules);
        if (P->n_up > 0)
            k_segsum_f64<<<(unsigned)xcd_grid(grid_for(P->n_up, 256)), 256, 0, s>>>(P->n_up, P->up_ptr, P->codes,
                                                                                   P->up_dst, P->mirror, V,
                                                                                   (double *)P->val);
        P->ran[NLA_PHASE_SEGSUM] = true;
        nla_mark(P, NLA_PHASE_EXTRACT, s);
        if (P->nnz_free > 0)
            k_extract<double><<<grid_for(P->nnz_free, 256), 256, 0, s>>>(P->nnz_free, P->a_src,
                                                                        (const double *)P->val, (double *)P->a_val);
        P->ran[NLA_PHASE_EXTRACT] = true;
    } else {
        NLA_TRY(nla_numeric_fp32(P, s, nla_mark));
    }
    nla_mark(P, NLA_PHASE_LOAD, s);
    P->have_load = false;
    if (f_outer && g_node) {
        k_load_elem<<<grid_for(K, 256), 256, 0, s>>>(K, P->tin, P->E.a2, P->d_rules, f_outer, P->Gk);
        if (P->n_free > 0) {
            if (fp64)
                k_load_rhs<double><<<grid_for(P->n_free, 4), 256, 0, s>>>(
                    P->n_free, P->free_nodes, P->n2e_ptr, P->n2e, P->Gk, P->rowptr, P->col, (const double *)P->val,
                    P->node_to_free, g_node, P->b);
            else
                k_load_rhs<float><<<grid_for(P->n_free, 4), 256, 0, s>>>(
                    P->n_free, P->free_nodes, P->n2e_ptr, P->n2e, P->Gk, P->rowptr, P->col, (const float *)P->val,
                    P->node_to_free, g_node, P->b);
        }
        P->have_load = true;
        P->ran[NLA_PHASE_LOAD] = true;
    }
    nla_mark(P, NLA_NPHASE, s);
    if (timed) P->timing_count++;
    P->cur_ev = nullptr;
    NLA_HIP(hipGetLastError());
    P->val_dtype = fp64 ? NLA_DTYPE_F64 : NLA_DTYPE_F32;
    P->assembled = true;
    P->counted = true;
    return NLA_OK;
}
