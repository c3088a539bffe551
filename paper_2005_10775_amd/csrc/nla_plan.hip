// Plan phase of libnlasm: host validation, element data, binning, the
// canonical pair list and the CSR pattern of D with its contribution map.
//
// Built with -ffp-contract=off: every +,-,* of the pair predicate is rounded
// separately so that the pair list is bitwise the one any IEEE evaluation of
// the same expressions produces (barycenter ((v0+v1)+v2)/3, outer point
// ((l0 v0 + l1 v1) + l2 v2), squared distances without sqrt or division).
#include "nla_internal.hpp"
#include <cstring>
#include <cmath>
#include <cstdlib>
#include <algorithm>
#include <string>
#include <rocprim/device/device_radix_sort.hpp>
#include <rocprim/device/device_select.hpp>

// ------------------------------------------------------------------ errors
static thread_local char g_err[1024] = "";

void nla_set_error(const char *fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
}

extern "C" const char *nla_last_error(void) { return g_err; }

// ------------------------------------------------------------------ arena
static size_t device_byte_cap()
{
    const char *e = getenv("NLA_MAX_DEVICE_BYTES");
    if (!e) return (size_t)-1;
    return (size_t)strtoull(e, nullptr, 10);
}

DeviceArena::~DeviceArena()
{
    for (void *p : ptrs) (void)hipFree(p);
}

int DeviceArena::alloc(void **p, size_t n)
{
    *p = nullptr;
    if (n == 0) n = 8;
    if (bytes + n > device_byte_cap()) {
        nla_set_error("device allocation of %zu bytes exceeds NLA_MAX_DEVICE_BYTES", n);
        return NLA_E_NOMEM;
    }
    hipError_t e = hipMalloc(p, n);
    if (e != hipSuccess) {
        nla_set_error("hipMalloc(%zu) failed: %s", n, hipGetErrorString(e));
        return NLA_E_NOMEM;
    }
    ptrs.push_back(*p);
    bytes += n;
    return NLA_OK;
}

// temporary buffers for one build step
struct Scratch {
    std::vector<void *> ptrs;
    size_t bytes = 0;
    ~Scratch()
    {
        for (void *p : ptrs) (void)hipFree(p);
    }
    template <class T> int get(T **p, size_t count)
    {
        size_t n = count * sizeof(T);
        if (n == 0) n = 8;
        if (n > device_byte_cap()) {
            nla_set_error("scratch allocation of %zu bytes exceeds NLA_MAX_DEVICE_BYTES", n);
            return NLA_E_NOMEM;
        }
        hipError_t e = hipMalloc((void **)p, n);
        if (e != hipSuccess) {
            nla_set_error("hipMalloc(%zu) failed: %s", n, hipGetErrorString(e));
            return NLA_E_NOMEM;
        }
        ptrs.push_back((void *)*p);
        return NLA_OK;
    }
};

static inline unsigned grid_for(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

// ------------------------------------------------------------- validation

// the rule integrates quadratics exactly on the reference triangle (weights
// summing to 1/2, first moments 1/6, second moments 1/12 and 1/24)
static bool rule_q2exact(const nla_rule &r)
{
    if (r.n < 1 || !r.lambda || !r.w) return false;
    double ws = 0, m1[3] = {0, 0, 0}, m2[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
    for (int q = 0; q < r.n; q++) {
        const double *l = r.lambda + 3 * q;
        ws += r.w[q];
        for (int a = 0; a < 3; a++) {
            m1[a] += r.w[q] * l[a];
            for (int b = 0; b < 3; b++) m2[a][b] += r.w[q] * l[a] * l[b];
        }
    }
    bool ok = std::fabs(ws - 0.5) <= 1e-14;
    for (int a = 0; a < 3; a++) {
        ok = ok && std::fabs(m1[a] - 1.0 / 6.0) <= 1e-14;
        for (int b = 0; b < 3; b++) ok = ok && std::fabs(m2[a][b] - (a == b ? 1.0 / 12.0 : 1.0 / 24.0)) <= 1e-14;
    }
    return ok;
}

static int validate(const nla_mesh *m, const nla_problem *p)
{
    if (!m || !p) { nla_set_error("null mesh or problem"); return NLA_E_INVALID; }
    if (m->n_vertices < 3 || m->n_triangles < 1 || !m->xy || !m->tri || !m->tri_in_omega || !m->node_free) {
        nla_set_error("mesh arrays missing or empty");
        return NLA_E_MESH;
    }
    if (!(p->delta > 0.0) || !std::isfinite(p->delta)) { nla_set_error("delta must be > 0"); return NLA_E_INVALID; }
    if (p->kernel != NLA_KERNEL_CONSTANT && p->kernel != NLA_KERNEL_FRACTIONAL) {
        nla_set_error("unknown kernel %d", p->kernel);
        return NLA_E_INVALID;
    }
    if (!std::isfinite(p->kernel_c) || p->kernel_c <= 0.0) { nla_set_error("kernel_c must be > 0"); return NLA_E_INVALID; }
    if (p->ball < NLA_BALL_BARYCENTER || p->ball > NLA_BALL_BARYSUPPORT) {
        nla_set_error("unknown ball %d", p->ball);
        return NLA_E_INVALID;
    }
    if (p->ball >= NLA_BALL_OVERLAP && (p->kernel != NLA_KERNEL_CONSTANT || p->precision != NLA_FP64)) {
        nla_set_error("the overlap, shifted and barycenter-support balls are assembled for the constant kernel in "
                      "NLA_FP64");
        return NLA_E_UNSUPPORTED;
    }
    if (p->cap_edges < 0 || p->cap_edges == 1 || p->cap_edges > NLA_MAX_CAP) {
        nla_set_error("cap_edges must be 0 or 2..%d", NLA_MAX_CAP);
        return NLA_E_INVALID;
    }
    if (p->precision != NLA_FP64 && p->precision != NLA_FP32 && p->precision != NLA_FP32_LEARNED) {
        nla_set_error("unknown precision %d", p->precision);
        return NLA_E_INVALID;
    }
    if (p->precision == NLA_FP32_LEARNED) {
        if (!p->mlp) { nla_set_error("learned caps need a network (nla_problem.mlp)"); return NLA_E_INVALID; }
        if (!(p->fallback_band >= 0.0) || !std::isfinite(p->fallback_band)) {
            nla_set_error("fallback_band must be finite and >= 0");
            return NLA_E_INVALID;
        }
        if (p->kernel != NLA_KERNEL_CONSTANT || p->ball != NLA_BALL_RETRI || p->cap_edges < 2) {
            nla_set_error("learned caps replace the arc-subdivided caps of the intersection ball under the constant "
                          "kernel (kernel 0, ball 1, cap_edges >= 2)");
            return NLA_E_UNSUPPORTED;
        }
    }
    if (p->kernel == NLA_KERNEL_FRACTIONAL && p->precision == NLA_FP64) {
        nla_set_error("the fractional kernel is assembled in NLA_FP32 (FP64 geometry and near pairs)");
        return NLA_E_UNSUPPORTED;
    }
    if (p->kernel == NLA_KERNEL_FRACTIONAL) {
        if (p->duffy_n < 1 || p->duffy_n > NLA_MAX_DUFFY || !p->duffy_x || !p->duffy_w) {
            nla_set_error("duffy_n must be 1..%d with nodes and weights", NLA_MAX_DUFFY);
            return NLA_E_INVALID;
        }
        if (!(p->kernel_s > -1.0 && p->kernel_s < 1.0)) { nla_set_error("kernel_s must be in (-1,1)"); return NLA_E_INVALID; }
    }
    const nla_rule *rs[2] = {&p->outer, &p->inner};
    const int mx[2] = {NLA_MAX_OUTER, NLA_MAX_INNER};
    for (int r = 0; r < 2; r++) {
        if (rs[r]->n < 1 || rs[r]->n > mx[r] || !rs[r]->lambda || !rs[r]->w) {
            nla_set_error("%s rule must have 1..%d points", r ? "inner" : "outer", mx[r]);
            return NLA_E_INVALID;
        }
        double ws = 0;
        for (int q = 0; q < rs[r]->n; q++) {
            const double *l = rs[r]->lambda + 3 * q;
            if (!(l[0] >= 0 && l[1] >= 0 && l[2] >= 0) || std::fabs(l[0] + l[1] + l[2] - 1.0) > 1e-12) {
                nla_set_error("%s rule point %d is not barycentric", r ? "inner" : "outer", q);
                return NLA_E_INVALID;
            }
            ws += rs[r]->w[q];
        }
        if (std::fabs(ws - 0.5) > 1e-12) { nla_set_error("rule weights must sum to 1/2"); return NLA_E_INVALID; }
    }
    if (p->flags & ~(uint32_t)NLA_SKIP_IXI) { nla_set_error("unknown flags"); return NLA_E_INVALID; }
    if (p->outer2.n != 0) {
        if (p->outer2.n < 0 || p->outer2.n > NLA_MAX_OUTER || !p->outer2.lambda || !p->outer2.w) {
            nla_set_error("second outer rule must have 1..%d points", NLA_MAX_OUTER);
            return NLA_E_INVALID;
        }
        double ws = 0;
        for (int q = 0; q < p->outer2.n; q++) {
            const double *l = p->outer2.lambda + 3 * q;
            if (!(l[0] >= 0 && l[1] >= 0 && l[2] >= 0) || std::fabs(l[0] + l[1] + l[2] - 1.0) > 1e-12) {
                nla_set_error("second outer rule point %d is not barycentric", q);
                return NLA_E_INVALID;
            }
            ws += p->outer2.w[q];
        }
        if (std::fabs(ws - 0.5) > 1e-12) { nla_set_error("rule weights must sum to 1/2"); return NLA_E_INVALID; }
        if (!(p->switch_dist >= 0.0) || !std::isfinite(p->switch_dist)) {
            nla_set_error("switch_dist must be finite and >= 0");
            return NLA_E_INVALID;
        }
        if (p->precision != NLA_FP64) {
            nla_set_error("the second outer rule is supported in NLA_FP64");
            return NLA_E_UNSUPPORTED;
        }
    }
    if (p->cap_mode != NLA_CAPS_ARCS && p->cap_mode != NLA_CAPS_CENTROID && p->cap_mode != NLA_CAPS_ANALYTIC) {
        nla_set_error("unknown cap_mode %d", p->cap_mode);
        return NLA_E_INVALID;
    }
    if ((p->ball == NLA_BALL_SHIFTED || p->ball == NLA_BALL_BARYSUPPORT) &&
        (p->outer2.n != 0 || p->cap_mode != NLA_CAPS_ARCS)) {
        nla_set_error("the shifted and barycenter-support balls take one outer rule and arc caps");
        return NLA_E_UNSUPPORTED;
    }
    if (p->ball == NLA_BALL_SHIFTED && !rule_q2exact(p->inner)) {
        nla_set_error("the shifted ball needs an inner rule exact for quadratics");
        return NLA_E_UNSUPPORTED;
    }
    if (p->ball == NLA_BALL_BARYSUPPORT && !rule_q2exact(p->outer)) {
        nla_set_error("the barycenter-support ball needs an outer rule exact for quadratics");
        return NLA_E_UNSUPPORTED;
    }
    if (p->cap_mode != NLA_CAPS_ARCS) {
        // exact caps (centroid rule or closed form) ride on the boundary-moment integration
        const bool q2 = rule_q2exact(p->inner);
        if (p->ball != NLA_BALL_RETRI || p->kernel != NLA_KERNEL_CONSTANT || p->precision != NLA_FP64 || !q2) {
            nla_set_error("exact caps need the intersection ball, the constant kernel, NLA_FP64 and an inner rule "
                          "exact for quadratics");
            return NLA_E_UNSUPPORTED;
        }
    }
    // mesh rules of Sec. 3.1
    const int J = m->n_vertices, K = m->n_triangles;
    for (int i = 0; i < 2 * J; i++)
        if (!std::isfinite(m->xy[i])) { nla_set_error("vertex %d not finite", i / 2); return NLA_E_MESH; }
    double dmax = 0.0, inr = 0.0;
    for (int k = 0; k < K; k++) {
        const int32_t *t = m->tri + 3 * k;
        for (int a = 0; a < 3; a++)
            if (t[a] < 0 || t[a] >= J) { nla_set_error("triangle %d has vertex index %d out of range", k, t[a]); return NLA_E_MESH; }
        if (t[0] == t[1] || t[1] == t[2] || t[0] == t[2]) { nla_set_error("triangle %d repeats a vertex", k); return NLA_E_MESH; }
        const double *A = m->xy + 2 * t[0], *B = m->xy + 2 * t[1], *Cc = m->xy + 2 * t[2];
        double cr = (B[0] - A[0]) * (Cc[1] - A[1]) - (B[1] - A[1]) * (Cc[0] - A[0]);
        if (!(cr > 0.0)) { nla_set_error("triangle %d is not counter-clockwise", k); return NLA_E_MESH; }
        if (m->tri_in_omega[k] > 1) { nla_set_error("tri_in_omega[%d] not 0/1", k); return NLA_E_MESH; }
        const double *V[3] = {A, B, Cc};
        double per = 0.0;
        for (int a = 0; a < 3; a++) {
            double dx = V[a][0] - V[(a + 1) % 3][0], dy = V[a][1] - V[(a + 1) % 3][1];
            const double l = std::sqrt(dx * dx + dy * dy);
            dmax = std::max(dmax, l);
            per += l;
        }
        inr = std::max(inr, cr / per);      // inradius = area / semi-perimeter
    }
    for (int j = 0; j < J; j++)
        if (m->node_free[j] > 1) { nla_set_error("node_free[%d] not 0/1", j); return NLA_E_MESH; }
    // a free node must not touch an element of Omega_I (Sec. 3.1: nodes on the boundary belong to Omega_I)
    for (int k = 0; k < K; k++)
        if (!m->tri_in_omega[k])
            for (int a = 0; a < 3; a++)
                if (m->node_free[m->tri[3 * k + a]]) {
                    nla_set_error("free node %d belongs to Omega_I element %d", m->tri[3 * k + a], k);
                    return NLA_E_MESH;
                }
    // a ball inside an element is not seen by the region walk, and a cap of a
    // half circle or more is not a cap; an element holding neither has inradius
    // < delta/2 (a half disk of radius delta has inradius delta/2)
    const bool cuts = p->ball == NLA_BALL_RETRI || p->ball == NLA_BALL_SHIFTED || p->ball == NLA_BALL_BARYSUPPORT;
    if (cuts && p->kernel == NLA_KERNEL_FRACTIONAL && dmax > p->delta) {
        nla_set_error("the fractional kernel with the retriangulated ball needs element diameter (%g) <= delta (%g)",
                      dmax, p->delta);
        return NLA_E_UNSUPPORTED;
    }
    if (cuts && !(inr < 0.5 * p->delta)) {
        nla_set_error("the ball needs every element inradius (largest %g) < delta/2 (%g)", inr, 0.5 * p->delta);
        return NLA_E_UNSUPPORTED;
    }
    return NLA_OK;
}

// ---------------------------------------------------------------- kernels
__global__ void k_elem(int K, const double *__restrict__ xy, const int32_t *__restrict__ tri, ElemSoA E,
                       const RuleSet *__restrict__ R, double *__restrict__ xq, double *__restrict__ xq2)
{
    int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= K) return;
    int i0 = tri[3 * k], i1 = tri[3 * k + 1], i2 = tri[3 * k + 2];
    double x0 = xy[2 * i0], y0 = xy[2 * i0 + 1];
    double x1 = xy[2 * i1], y1 = xy[2 * i1 + 1];
    double x2 = xy[2 * i2], y2 = xy[2 * i2 + 1];
    E.vx0[k] = x0; E.vy0[k] = y0; E.vx1[k] = x1; E.vy1[k] = y1; E.vx2[k] = x2; E.vy2[k] = y2;
    double bx = ((x0 + x1) + x2) / 3.0;
    double by = ((y0 + y1) + y2) / 3.0;
    E.bx[k] = bx;
    E.by[k] = by;
    E.a2[k] = fabs((x1 - x0) * (y2 - y0) - (y1 - y0) * (x2 - x0));
    double r = 0.0;
    double px[3] = {x0, x1, x2}, py[3] = {y0, y1, y2};
#pragma unroll
    for (int a = 0; a < 3; a++) {
        double dx = px[a] - bx, dy = py[a] - by;
        r = fmax(r, sqrt(dx * dx + dy * dy));
    }
    E.r[k] = r;
    double2 *rec = (double2 *)(E.pk + 16 * (int64_t)k);
    rec[0] = make_double2(x0, y0);
    rec[1] = make_double2(x1, y1);
    rec[2] = make_double2(x2, y2);
    rec[3] = make_double2(bx, by);
    rec[4] = make_double2(E.a2[k], r);
    // reciprocal squared edge lengths (v0->v1, v1->v2, v2->v0), rounded as the
    // pair kernels' edge roots form them
    const double l0 = (x1 - x0) * (x1 - x0) + (y1 - y0) * (y1 - y0);
    const double l1 = (x2 - x1) * (x2 - x1) + (y2 - y1) * (y2 - y1);
    const double l2 = (x0 - x2) * (x0 - x2) + (y0 - y2) * (y0 - y2);
    rec[5] = make_double2(1.0 / l0, 1.0 / l1);
    rec[6] = make_double2(1.0 / l2, 0.0);
    rec[7] = make_double2(0.0, 0.0);
    const int nq = R->n_out;
    for (int q = 0; q < nq; q++) {
        const double l0 = R->out_lam[q][0], l1 = R->out_lam[q][1], l2 = R->out_lam[q][2];
        xq[2 * ((int64_t)k * nq + q)] = (l0 * x0 + l1 * x1) + l2 * x2;
        xq[2 * ((int64_t)k * nq + q) + 1] = (l0 * y0 + l1 * y1) + l2 * y2;
    }
    const int nq2 = R->n_out2;
    for (int q = 0; q < nq2; q++) {
        const double l0 = R->out2_lam[q][0], l1 = R->out2_lam[q][1], l2 = R->out2_lam[q][2];
        xq2[2 * ((int64_t)k * nq2 + q)] = (l0 * x0 + l1 * x1) + l2 * x2;
        xq2[2 * ((int64_t)k * nq2 + q) + 1] = (l0 * y0 + l1 * y1) + l2 * y2;
    }
}

// the pair takes the second outer rule when |b_k - b_k'| < switch_dist
__device__ __forceinline__ bool use_rule2(double bkx, double bky, double bpx, double bpy, double sd)
{
    const double dx = bkx - bpx, dy = bky - bpy;
    return dx * dx + dy * dy < sd * sd;
}

__global__ void k_pair_rule2(int64_t P, const int32_t *__restrict__ pk, const int32_t *__restrict__ pkp, ElemSoA E,
                             double sd, uint8_t *__restrict__ r2)
{
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= P) return;
    const int k = pk[p], kp = pkp[p];
    r2[p] = use_rule2(E.bx[k], E.by[k], E.bx[kp], E.by[kp], sd) ? 1 : 0;
}

struct Grid {
    double x0, y0, inv_cs;
    int nx, ny;
};

__device__ __forceinline__ int cell_of(const Grid &g, double bx, double by, int *cx, int *cy)
{
    int ix = (int)floor((bx - g.x0) * g.inv_cs);
    int iy = (int)floor((by - g.y0) * g.inv_cs);
    ix = ix < 0 ? 0 : (ix >= g.nx ? g.nx - 1 : ix);
    iy = iy < 0 ? 0 : (iy >= g.ny ? g.ny - 1 : iy);
    *cx = ix;
    *cy = iy;
    return iy * g.nx + ix;
}

__global__ void k_bin_count(int K, ElemSoA E, Grid g, int32_t *__restrict__ cellof, int32_t *__restrict__ cnt)
{
    int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= K) return;
    int cx, cy;
    int c = cell_of(g, E.bx[k], E.by[k], &cx, &cy);
    cellof[k] = c;
    atomicAdd(&cnt[c], 1);
}

__global__ void k_bin_scatter(int K, const int32_t *__restrict__ cellof, const int32_t *__restrict__ start,
                              int32_t *__restrict__ cursor, int32_t *__restrict__ elems)
{
    int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= K) return;
    int c = cellof[k];
    int slot = atomicAdd(&cursor[c], 1);
    elems[start[c] + slot] = k;
}

// ---- the pair predicate (Eq. (baryball); tasks 2-4 of Sec. 7.1)
__device__ __forceinline__ bool bary_in(double xx, double xy, double bx, double by, double dd)
{
    double dx = xx - bx, dy = xy - by;
    return dx * dx + dy * dy <= dd;
}

__device__ __forceinline__ bool ball_meets(double xx, double xy, const double (&V)[6], double dd)
{
#pragma unroll
    for (int a = 0; a < 3; a++) {
        double dx = V[2 * a] - xx, dy = V[2 * a + 1] - xy;
        if (dx * dx + dy * dy <= dd) return true;
    }
    bool inside = true;
#pragma unroll
    for (int a = 0; a < 3; a++) {
        const int b = (a + 1) % 3;
        double ex = V[2 * b] - V[2 * a], ey = V[2 * b + 1] - V[2 * a + 1];
        double px = xx - V[2 * a], py = xy - V[2 * a + 1];
        double o = ex * py - ey * px;
        if (o < 0.0) inside = false;
    }
    if (inside) return true;
#pragma unroll
    for (int a = 0; a < 3; a++) {
        const int b = (a + 1) % 3;
        double ex = V[2 * b] - V[2 * a], ey = V[2 * b + 1] - V[2 * a + 1];
        double px = xx - V[2 * a], py = xy - V[2 * a + 1];
        double t = ex * px + ey * py;
        double L = ex * ex + ey * ey;
        if (t > 0.0 && t < L) {
            double c = ex * py - ey * px;
            if (c * c <= dd * L) return true;
        }
    }
    return false;
}

struct PairQuery {
    Grid g;
    const int32_t *cell_start;   // [ncell+1]
    const int32_t *cell_elems;
    const uint8_t *tin;
    const double *xq, *xq2;     // outer points of the first and the second rule
    double delta, dd, sd;       // sd: switch distance of the second rule
    int nq, nq2, ball, skip_ixi;
};

// candidate ranges of the 3x3 cells around element k
__device__ __forceinline__ int gather_ranges(const PairQuery &Q, double bx, double by, int (&lo)[9], int (&n)[9])
{
    int cx, cy;
    cell_of(Q.g, bx, by, &cx, &cy);
    int tot = 0, i = 0;
    for (int dy = -1; dy <= 1; dy++)
        for (int dx = -1; dx <= 1; dx++, i++) {
            int x = cx + dx, y = cy + dy;
            if (x < 0 || y < 0 || x >= Q.g.nx || y >= Q.g.ny) {
                lo[i] = 0;
                n[i] = 0;
                continue;
            }
            int c = y * Q.g.nx + x;
            lo[i] = Q.cell_start[c];
            n[i] = Q.cell_start[c + 1] - lo[i];
            tot += n[i];
        }
    return tot;
}

__device__ __forceinline__ int candidate_at(const PairQuery &Q, const int (&lo)[9], const int (&n)[9], int i)
{
    int c = 0;
    while (i >= n[c]) {
        i -= n[c];
        c++;
    }
    return Q.cell_elems[lo[c] + i];
}

__device__ __forceinline__ bool pair_test(const PairQuery &Q, const ElemSoA &E, int k, int kp, double bk_x, double bk_y,
                                          double rk, const double *xs, const double *xs2)
{
    if (Q.skip_ixi && !Q.tin[k] && !Q.tin[kp]) return false;
    double bx = E.bx[kp], by = E.by[kp];
    double reach = Q.delta + rk + (Q.ball == NLA_BALL_BARYCENTER ? 0.0 : E.r[kp]);
    reach = reach * (1.0 + 1e-9) + 1e-14;
    double ddx = bk_x - bx, ddy = bk_y - by;
    if (!(ddx * ddx + ddy * ddy <= reach * reach)) return false;
    if (Q.ball == NLA_BALL_SHIFTED) {
        // every point of E_k uses the ball about b_k (Sec. 4.3)
        const double V[6] = {E.vx0[kp], E.vy0[kp], E.vx1[kp], E.vy1[kp], E.vx2[kp], E.vy2[kp]};
        return ball_meets(bk_x, bk_y, V, Q.dd);
    }
    if (Q.ball == NLA_BALL_BARYSUPPORT) {
        // some x in E_k has b_k' in its ball: E_k meets the ball about b_k'
        const double V[6] = {E.vx0[k], E.vy0[k], E.vx1[k], E.vy1[k], E.vx2[k], E.vy2[k]};
        return ball_meets(bx, by, V, Q.dd);
    }
    // the outer points of the pair's rule
    const bool r2 = Q.nq2 > 0 && use_rule2(bk_x, bk_y, bx, by, Q.sd);
    const double *pts = r2 ? xs2 : xs;
    const int nq = r2 ? Q.nq2 : Q.nq;
    if (Q.ball == NLA_BALL_BARYCENTER) {
        for (int q = 0; q < nq; q++)
            if (bary_in(pts[2 * q], pts[2 * q + 1], bx, by, Q.dd)) return true;
        return false;
    }
    double V[6] = {E.vx0[kp], E.vy0[kp], E.vx1[kp], E.vy1[kp], E.vx2[kp], E.vy2[kp]};
    for (int q = 0; q < nq; q++)
        if (ball_meets(pts[2 * q], pts[2 * q + 1], V, Q.dd)) return true;
    return false;
}

__global__ __launch_bounds__(256) void k_pair_count(int K, PairQuery Q, ElemSoA E, int32_t *__restrict__ cnt)
{
    __shared__ double xs[2 * NLA_MAX_OUTER], xs2[2 * NLA_MAX_OUTER];
    __shared__ int red[256 / 64];
    const int k = blockIdx.x, tid = threadIdx.x;
    if (tid < 2 * Q.nq) xs[tid] = Q.xq[2 * (int64_t)k * Q.nq + tid];
    if (tid < 2 * Q.nq2) xs2[tid] = Q.xq2[2 * (int64_t)k * Q.nq2 + tid];
    __syncthreads();
    const double bx = E.bx[k], by = E.by[k], rk = E.r[k];
    int lo[9], n[9];
    const int tot = gather_ranges(Q, bx, by, lo, n);
    int c = 0;
    for (int i = tid; i < tot; i += blockDim.x) {
        int kp = candidate_at(Q, lo, n, i);
        c += pair_test(Q, E, k, kp, bx, by, rk, xs, xs2) ? 1 : 0;
    }
    for (int off = 32; off > 0; off >>= 1) c += __shfl_down(c, off, 64);
    if ((tid & 63) == 0) red[tid >> 6] = c;
    __syncthreads();
    if (tid == 0) {
        int s = 0;
        for (int w = 0; w < (int)(blockDim.x >> 6); w++) s += red[w];
        cnt[k] = s;
    }
}

// Emits the pairs of k: candidates are tested by the whole workgroup, hits
// are compacted into LDS with a wavefront ballot and prefix popcount, and
// then written in ascending k' order (each hit's rank = number of smaller hits).
__global__ __launch_bounds__(256) void k_pair_emit(int K, PairQuery Q, ElemSoA E, const int64_t *__restrict__ ptr,
                                                   int32_t *__restrict__ out)
{
    __shared__ double xs[2 * NLA_MAX_OUTER], xs2[2 * NLA_MAX_OUTER];
    __shared__ int hits[NLA_MAX_PAIRS_PER_K];
    __shared__ int nh;
    const int k = blockIdx.x, tid = threadIdx.x, lane = tid & 63;
    if (tid < 2 * Q.nq) xs[tid] = Q.xq[2 * (int64_t)k * Q.nq + tid];
    if (tid < 2 * Q.nq2) xs2[tid] = Q.xq2[2 * (int64_t)k * Q.nq2 + tid];
    if (tid == 0) nh = 0;
    __syncthreads();
    const double bx = E.bx[k], by = E.by[k], rk = E.r[k];
    int lo[9], n[9];
    const int tot = gather_ranges(Q, bx, by, lo, n);
    const int rounds = (tot + (int)blockDim.x - 1) / (int)blockDim.x;
    for (int r = 0; r < rounds; r++) {
        int i = r * blockDim.x + tid;
        int kp = -1;
        bool hit = false;
        if (i < tot) {
            kp = candidate_at(Q, lo, n, i);
            hit = pair_test(Q, E, k, kp, bx, by, rk, xs, xs2);
        }
        unsigned long long mask = __ballot(hit);
        int wcnt = __popcll(mask);
        int before = __popcll(mask & ((1ull << lane) - 1ull));
        int base = 0;
        if (lane == 0 && wcnt) base = atomicAdd(&nh, wcnt);
        base = __shfl(base, 0, 64);
        if (hit && base + before < NLA_MAX_PAIRS_PER_K) hits[base + before] = kp;
    }
    __syncthreads();
    const int m = nh < NLA_MAX_PAIRS_PER_K ? nh : NLA_MAX_PAIRS_PER_K;
    const int64_t o = ptr[k];
    for (int i = tid; i < m; i += blockDim.x) {
        int v = hits[i], rank = 0;
        for (int j = 0; j < m; j++) rank += hits[j] < v;
        out[o + rank] = v;
    }
}

// ------------------------------------------------------ pattern kernels
__global__ void k_pair_k(int K, const int64_t *__restrict__ ptr, int32_t *__restrict__ pk)
{
    int k = blockIdx.x;
    for (int64_t p = ptr[k] + threadIdx.x; p < ptr[k + 1]; p += blockDim.x) pk[p] = k;
}

__global__ void k_appears(int64_t P, const int32_t *__restrict__ pk, const int32_t *__restrict__ pkp, uint8_t *app)
{
    int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= P) return;
    app[pk[p]] = 1;
    app[pkp[p]] = 1;
}

__global__ void k_keys_pairs(int64_t P, int J, const int32_t *__restrict__ tri, const int32_t *__restrict__ pk,
                             const int32_t *__restrict__ pkp, uint64_t *__restrict__ keys)
{
    int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= P) return;
    int k = pk[p], kp = pkp[p];
    uint64_t g[3], h[3];
    for (int a = 0; a < 3; a++) {
        g[a] = (uint64_t)tri[3 * k + a];
        h[a] = (uint64_t)tri[3 * kp + a];
    }
    uint64_t *o = keys + 18 * p;
    for (int a = 0; a < 3; a++)
        for (int b = 0; b < 3; b++) {
            o[2 * (3 * a + b)] = g[a] * (uint64_t)J + h[b];
            o[2 * (3 * a + b) + 1] = h[b] * (uint64_t)J + g[a];
        }
}

__global__ void k_keys_elems(int K, int J, const int32_t *__restrict__ tri, const uint8_t *__restrict__ app,
                             uint64_t sentinel, uint64_t *__restrict__ keys)
{
    int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= K) return;
    for (int a = 0; a < 3; a++)
        for (int c = 0; c < 3; c++)
            keys[9 * (int64_t)k + 3 * a + c] =
                app[k] ? (uint64_t)tri[3 * k + a] * (uint64_t)J + (uint64_t)tri[3 * k + c] : sentinel;
}

__device__ __forceinline__ int64_t lower_bound_u64(const uint64_t *a, int64_t n, uint64_t v)
{
    int64_t lo = 0, hi = n;
    while (lo < hi) {
        int64_t mid = (lo + hi) >> 1;
        if (a[mid] < v) lo = mid + 1; else hi = mid;
    }
    return lo;
}

__device__ __forceinline__ int64_t lower_bound_u32(const uint32_t *a, int64_t n, uint32_t v)
{
    int64_t lo = 0, hi = n;
    while (lo < hi) {
        int64_t mid = (lo + hi) >> 1;
        if (a[mid] < v) lo = mid + 1; else hi = mid;
    }
    return lo;
}

__global__ void k_rowptr(int J, const uint64_t *__restrict__ uk, int64_t nnz, int64_t *__restrict__ rowptr)
{
    int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r > J) return;
    rowptr[r] = lower_bound_u64(uk, nnz, (uint64_t)r * (uint64_t)J);
}

__global__ void k_cols(int64_t nnz, int J, const uint64_t *__restrict__ uk, int32_t *__restrict__ col,
                       int64_t *__restrict__ mirror, uint8_t *__restrict__ upflag)
{
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nnz) return;
    uint64_t key = uk[t];
    uint64_t r = key / (uint64_t)J, c = key % (uint64_t)J;
    col[t] = (int32_t)c;
    mirror[t] = lower_bound_u64(uk, nnz, c * (uint64_t)J + r);
    upflag[t] = r <= c;
}

__global__ void k_up_index(int64_t nnz, const uint8_t *__restrict__ upflag, const int64_t *__restrict__ upscan,
                           int64_t *__restrict__ up_dst, int64_t *__restrict__ up_of)
{
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nnz) return;
    if (upflag[t]) {
        int64_t u = upscan[t];
        up_dst[u] = t;
        up_of[t] = u;
    } else {
        up_of[t] = -1;
    }
}

__device__ __forceinline__ uint32_t upper_of(const uint64_t *uk, int64_t nnz, const int64_t *up_of, int J, int r, int c)
{
    int lo = r < c ? r : c, hi = r < c ? c : r;
    int64_t t = lower_bound_u64(uk, nnz, (uint64_t)lo * (uint64_t)J + (uint64_t)hi);
    return (uint32_t)up_of[t];
}

// ---- column sets and contribution lists of the -Mxy reduction
__global__ void k_colkeys(int64_t P, const int32_t *__restrict__ tri, const int32_t *__restrict__ pk,
                          const int32_t *__restrict__ pkp, uint64_t *__restrict__ keys)
{
    int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= P) return;
    const uint64_t k = (uint64_t)pk[p];
    for (int b = 0; b < 3; b++) keys[3 * p + b] = (k << 32) | (uint64_t)tri[3 * pkp[p] + b];
}

__global__ void k_col_off(int K, const uint64_t *__restrict__ U, int64_t nu, int64_t *__restrict__ off)
{
    int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k > K) return;
    off[k] = lower_bound_u64(U, nu, (uint64_t)k << 32);
}

__global__ void k_colset(int64_t nu, const uint64_t *__restrict__ U, int32_t *__restrict__ colset)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < nu) colset[i] = (int32_t)(U[i] & 0xffffffffull);
}

// slot key (global column slot) and value (p_local << 2 | b) of every (pair, b)
// A pair is deep when every point of E_k is within delta of every point of
// E_k' with room to spare (pair_deep).  Key 2 k + deep orders each
// element's pairs band first, deep after.
__global__ void k_deep_keys(int64_t P, const int32_t *__restrict__ pk, const int32_t *__restrict__ pkp, ElemSoA E,
                            double delta, uint32_t *__restrict__ key, int32_t *__restrict__ val)
{
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= P) return;
    const int k = pk[p];
    key[p] = 2u * (uint32_t)k + (pair_deep(E, k, pkp[p], delta) ? 1u : 0u);
    val[p] = (int32_t)p;
}

// Keys of the transposed order: k' for band pairs, K (past every element) for deep ones.
__global__ void k_tkeys(int64_t P, const int32_t *__restrict__ pk, const int32_t *__restrict__ pkp, ElemSoA E,
                        double delta, int K, uint32_t *__restrict__ key)
{
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= P) return;
    const int kp = pkp[p];
    key[p] = pair_deep(E, pk[p], kp, delta) ? (uint32_t)K : (uint32_t)kp;
}

__global__ void k_proc_kp(int64_t P, const int32_t *__restrict__ proc_p, const int32_t *__restrict__ pkp,
                          int32_t *__restrict__ proc_kp)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= P) return;
    proc_kp[i] = pkp[proc_p[i]];
}

__global__ void k_nband(int K, const int64_t *__restrict__ ptr, const uint32_t *__restrict__ skey,
                        int32_t *__restrict__ nband)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= K) return;
    const int64_t lo = ptr[k];
    nband[k] = (int32_t)lower_bound_u32(skey + lo, ptr[k + 1] - lo, 2u * (uint32_t)k + 1u);
}

// Column entries in processing order (slot i of pair proc_p[i], or the pairs
// themselves when proc_p is null), so that the stable sort by column keeps each
// column's entries in the order the pair kernel visits them.
__global__ void k_colent_keys(int64_t P, const int32_t *__restrict__ tri, const int32_t *__restrict__ pk,
                              const int32_t *__restrict__ pkp, const int64_t *__restrict__ pair_ptr,
                              const int32_t *__restrict__ proc_p, const uint64_t *__restrict__ U, int64_t nu,
                              uint32_t *__restrict__ key, uint16_t *__restrict__ val)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= P) return;
    const int64_t p = proc_p ? (int64_t)proc_p[i] : i;
    const uint64_t k = (uint64_t)pk[p];
    const int pl = (int)(i - pair_ptr[k]);
    for (int b = 0; b < 3; b++) {
        int64_t slot = lower_bound_u64(U, nu, (k << 32) | (uint64_t)tri[3 * pkp[p] + b]);
        key[3 * i + b] = (uint32_t)slot;
        val[3 * i + b] = (uint16_t)((pl << 2) | b);
    }
}

__global__ void k_slot_ptr(int64_t nu, const uint32_t *__restrict__ sk, int64_t n, int32_t *__restrict__ ptr)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i > nu) return;
    ptr[i] = (int32_t)lower_bound_u32(sk, n, (uint32_t)i);
}

__device__ __forceinline__ int find_col(const int32_t *cs, int n, int node)
{
    int lo = 0, hi = n;
    while (lo < hi) {
        int mid = (lo + hi) >> 1;
        if (cs[mid] < node) lo = mid + 1; else hi = mid;
    }
    return (lo < n && cs[lo] == node) ? lo : -1;
}

// Codes of one upper entry (j, c), j <= c, in the value array [R | E]:
//   F[j,c]: for every element k with node j (slot a), R_k[a][c] if c in C_k;
//   F[c,j]: for every element k with node c (slot a), R_k[a][j] if j in C_k;
//   E: for every element containing both nodes, its element block entry.
// With fill == 0 only the count is written.
__global__ void k_entry_codes(int64_t n_up, int J, const int64_t *__restrict__ up_dst, const int64_t *__restrict__ rowptr_unused,
                              const uint64_t *__restrict__ uk, const int32_t *__restrict__ tri,
                              const int32_t *__restrict__ n2e_ptr, const int32_t *__restrict__ n2e,
                              const int64_t *__restrict__ col_off, const int32_t *__restrict__ colset, int64_t e_base,
                              int fill, int32_t *__restrict__ cnt, const int64_t *__restrict__ up_ptr,
                              int32_t *__restrict__ codes)
{
    int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (u >= n_up) return;
    const uint64_t key = uk[up_dst[u]];
    const int j = (int)(key / (uint64_t)J), c = (int)(key % (uint64_t)J);
    int n = 0;
    int64_t o = fill ? up_ptr[u] : 0;
    for (int pass = 0; pass < 2; pass++) {
        const int r = pass ? c : j, t = pass ? j : c;
        for (int e = n2e_ptr[r]; e < n2e_ptr[r + 1]; e++) {
            const int k = n2e[e] / 3, a = n2e[e] % 3;
            const int64_t off = col_off[k];
            const int nc = (int)(col_off[k + 1] - off);
            const int lc = find_col(colset + off, nc, t);
            if (lc < 0) continue;
            if (fill) codes[o + n] = (int32_t)(3 * off + (int64_t)a * nc + lc);
            n++;
        }
    }
    const int idx[3][3] = {{0, 1, 2}, {1, 3, 4}, {2, 4, 5}};
    for (int e = n2e_ptr[j]; e < n2e_ptr[j + 1]; e++) {
        const int k = n2e[e] / 3, a = n2e[e] % 3;
        int ac = -1;
        for (int b = 0; b < 3; b++)
            if (tri[3 * k + b] == c) ac = b;
        if (ac < 0) continue;
        if (fill) codes[o + n] = (int32_t)(e_base + 6 * (int64_t)k + idx[a][ac]);
        n++;
    }
    if (!fill) cnt[u] = n;
}

// ---- vertex-sharing pairs under the singular kernel
__global__ void k_near_flag(int64_t P, const int32_t *__restrict__ tri, const int32_t *__restrict__ pk,
                            const int32_t *__restrict__ pkp, uint8_t *__restrict__ flag)
{
    int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= P) return;
    const int k = pk[p], kp = pkp[p];
    bool sh = false;
    for (int a = 0; a < 3; a++)
        for (int b = 0; b < 3; b++) sh |= tri[3 * k + a] == tri[3 * kp + b];
    flag[p] = sh ? 1 : 0;
}

__device__ __forceinline__ int upper_slot(int i, int j)
{
    // index of (min, max) in the row-major upper triangle of a 6x6 matrix
    const int a = i < j ? i : j, b = i < j ? j : i;
    return a * 6 - (a * (a - 1)) / 2 + (b - a);
}

// Mirror partner of a vertex-sharing pair (k, k') with k > k': the near index
// of (k', k) when that pair interacts (its block is the same node-level
// matrix: the joint integrand is symmetric under x <-> y), else -1 (computed).
__global__ void k_near_partner(int64_t n_near, const int64_t *__restrict__ near_pair,
                               const int32_t *__restrict__ pk, const int32_t *__restrict__ pkp,
                               const int64_t *__restrict__ pair_ptr, int64_t *__restrict__ partner)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_near) return;
    const int64_t p = near_pair[i];
    const int k = pk[p], kp = pkp[p];
    int64_t res = -1;
    if (k > kp) {
        int64_t lo = pair_ptr[kp], hi = pair_ptr[kp + 1];     // k' row, k'' ascending
        while (lo < hi) {
            const int64_t mid = (lo + hi) >> 1;
            if (pkp[mid] < k) lo = mid + 1;
            else hi = mid;
        }
        if (lo < pair_ptr[kp + 1] && pkp[lo] == k) {
            int64_t a = 0, b = n_near;                      // near_pair is ascending
            while (a < b) {
                const int64_t mid = (a + b) >> 1;
                if (near_pair[mid] < lo) a = mid + 1;
                else b = mid;
            }
            if (a < n_near && near_pair[a] == lo) res = a;
        }
    }
    partner[i] = res;
}

// 36 slots per near pair: ordered slot pairs (I, J) whose nodes satisfy
// node(I) <= node(J) (the mirror goes to the lower triangle), merged-away
// slots (a node of E_k' that is also a node of E_k) excluded
__global__ void k_near_codes(int64_t n_near, int J, const int64_t *__restrict__ near_pair,
                             const int32_t *__restrict__ tri, const int32_t *__restrict__ pk,
                             const int32_t *__restrict__ pkp, const uint64_t *__restrict__ uk, int64_t nnz,
                             const int64_t *__restrict__ up_of, uint32_t sentinel, const int64_t *__restrict__ partner,
                             uint32_t *__restrict__ key, int32_t *__restrict__ code)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_near) return;
    const int64_t p = near_pair[i];
    const int k = pk[p], kp = pkp[p];
    // a mirrored pair reads its partner's block: slot of each node in (k', k) order
    const int64_t src = partner[i] >= 0 ? partner[i] : i;
    int ps[6];
    int g[6];
    bool valid[6];
    for (int a = 0; a < 3; a++) {
        g[a] = tri[3 * k + a];
        g[3 + a] = tri[3 * kp + a];
        valid[a] = true;
    }
    for (int b = 0; b < 3; b++) {
        valid[3 + b] = true;
        for (int a = 0; a < 3; a++)
            if (g[3 + b] == g[a]) valid[3 + b] = false;
    }
    for (int I = 0; I < 6; I++) {
        ps[I] = I;
        if (src != i) {
            ps[I] = -1;
            for (int a = 0; a < 3; a++)
                if (tri[3 * kp + a] == g[I]) ps[I] = a;
            if (ps[I] < 0)
                for (int a = 0; a < 3; a++)
                    if (tri[3 * k + a] == g[I]) ps[I] = 3 + a;
        }
    }
    for (int I = 0; I < 6; I++)
        for (int Jj = 0; Jj < 6; Jj++) {
            const int64_t s = 36 * i + 6 * I + Jj;
            if (valid[I] && valid[Jj] && g[I] <= g[Jj] && (g[I] < g[Jj] || I == Jj)) {
                key[s] = upper_of(uk, nnz, up_of, J, g[I], g[Jj]);
                code[s] = (int32_t)(21 * src + upper_slot(ps[I], ps[Jj]));
            } else {
                key[s] = sentinel;
                code[s] = -1;
            }
        }
}

__global__ void k_iota(int64_t n, int32_t *__restrict__ v)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) v[i] = (int32_t)i;
}

__global__ void k_tptr(int K, const uint32_t *__restrict__ skp, int64_t P, int64_t *__restrict__ tptr)
{
    int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k > K) return;
    tptr[k] = lower_bound_u32(skp, P, (uint32_t)k);
}

__global__ void k_up_ptr(int64_t n_up, const uint32_t *__restrict__ skeys, int64_t n, int64_t *__restrict__ up_ptr)
{
    int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (u > n_up) return;
    up_ptr[u] = lower_bound_u32(skeys, n, (uint32_t)u);
}

__global__ void k_a_count(int n_free, const int32_t *__restrict__ free_nodes, const int64_t *__restrict__ rowptr,
                          const int32_t *__restrict__ col, const int32_t *__restrict__ n2f, int64_t *__restrict__ cnt)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_free) return;
    int r = free_nodes[i];
    int64_t c = 0;
    for (int64_t t = rowptr[r]; t < rowptr[r + 1]; t++) c += n2f[col[t]] >= 0;
    cnt[i] = c;
}

__global__ void k_a_fill(int n_free, const int32_t *__restrict__ free_nodes, const int64_t *__restrict__ rowptr,
                         const int32_t *__restrict__ col, const int32_t *__restrict__ n2f,
                         const int64_t *__restrict__ a_rowptr, int32_t *__restrict__ a_col, int64_t *__restrict__ a_src)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_free) return;
    int r = free_nodes[i];
    int64_t o = a_rowptr[i];
    for (int64_t t = rowptr[r]; t < rowptr[r + 1]; t++) {
        int f = n2f[col[t]];
        if (f >= 0) {
            a_col[o] = f;
            a_src[o] = t;
            o++;
        }
    }
}

// ------------------------------------------------------------ build steps
static int bits_for(uint64_t v)
{
    int b = 0;
    while (b < 64 && (v >> b) != 0) b++;
    return b < 1 ? 1 : b;
}

int nla_build_pairs(nla_plan *P, hipStream_t s)
{
    const int K = P->K;
    const nla_problem &pr = P->prob;
    // grid of barycenters with cells no smaller than the largest reach
    std::vector<double> hx(2 * (size_t)P->J);
    NLA_HIP(hipMemcpyAsync(hx.data(), P->xy, sizeof(double) * 2 * P->J, hipMemcpyDeviceToHost, s));
    std::vector<double> hr(K);
    NLA_HIP(hipMemcpyAsync(hr.data(), P->E.r, sizeof(double) * K, hipMemcpyDeviceToHost, s));
    NLA_HIP(hipStreamSynchronize(s));
    double xmin = hx[0], xmax = hx[0], ymin = hx[1], ymax = hx[1];
    for (int j = 0; j < P->J; j++) {
        xmin = std::min(xmin, hx[2 * j]); xmax = std::max(xmax, hx[2 * j]);
        ymin = std::min(ymin, hx[2 * j + 1]); ymax = std::max(ymax, hx[2 * j + 1]);
    }
    double rmax = 0;
    for (double r : hr) rmax = std::max(rmax, r);
    double reach = pr.delta + rmax + (pr.ball == NLA_BALL_BARYCENTER ? 0.0 : rmax);
    double cs = reach * (1.0 + 1e-6) + 1e-12;
    Grid g;
    g.x0 = xmin;
    g.y0 = ymin;
    g.inv_cs = 1.0 / cs;
    g.nx = (int)std::floor((xmax - xmin) / cs) + 1;
    g.ny = (int)std::floor((ymax - ymin) / cs) + 1;
    if ((int64_t)g.nx * g.ny > (1 << 24)) { nla_set_error("binning grid too large"); return NLA_E_UNSUPPORTED; }
    const int ncell = g.nx * g.ny;
    Scratch S;
    int32_t *cellof, *cnt, *start, *cursor, *elems, *pcnt;
    NLA_TRY(S.get(&cellof, K));
    NLA_TRY(S.get(&cnt, ncell));
    NLA_TRY(S.get(&start, ncell + 1));
    NLA_TRY(S.get(&cursor, ncell));
    NLA_TRY(S.get(&elems, K));
    NLA_TRY(S.get(&pcnt, K));
    NLA_HIP(hipMemsetAsync(cnt, 0, sizeof(int32_t) * ncell, s));
    NLA_HIP(hipMemsetAsync(cursor, 0, sizeof(int32_t) * ncell, s));
    k_bin_count<<<grid_for(K, 256), 256, 0, s>>>(K, P->E, g, cellof, cnt);
    std::vector<int32_t> hc(ncell), hs(ncell + 1);
    NLA_HIP(hipMemcpyAsync(hc.data(), cnt, sizeof(int32_t) * ncell, hipMemcpyDeviceToHost, s));
    NLA_HIP(hipStreamSynchronize(s));
    hs[0] = 0;
    for (int c = 0; c < ncell; c++) hs[c + 1] = hs[c] + hc[c];
    NLA_HIP(hipMemcpyAsync(start, hs.data(), sizeof(int32_t) * (ncell + 1), hipMemcpyHostToDevice, s));
    k_bin_scatter<<<grid_for(K, 256), 256, 0, s>>>(K, cellof, start, cursor, elems);
    PairQuery Q;
    Q.g = g;
    Q.cell_start = start;
    Q.cell_elems = elems;
    Q.tin = P->tin;
    Q.xq = P->xq;
    Q.xq2 = P->xq2;
    Q.delta = pr.delta;
    Q.dd = pr.delta * pr.delta;
    Q.sd = P->rules.switch_dist;
    Q.nq = P->rules.n_out;
    Q.nq2 = P->rules.n_out2;
    Q.ball = pr.ball;
    Q.skip_ixi = (pr.flags & NLA_SKIP_IXI) ? 1 : 0;
    k_pair_count<<<K, 256, 0, s>>>(K, Q, P->E, pcnt);
    std::vector<int32_t> hp(K);
    NLA_HIP(hipMemcpyAsync(hp.data(), pcnt, sizeof(int32_t) * K, hipMemcpyDeviceToHost, s));
    NLA_HIP(hipStreamSynchronize(s));
    std::vector<int64_t> hptr(K + 1);
    hptr[0] = 0;
    int maxc = 0;
    for (int k = 0; k < K; k++) {
        hptr[k + 1] = hptr[k] + hp[k];
        maxc = std::max(maxc, hp[k]);
    }
    if (maxc > NLA_MAX_PAIRS_PER_K) {
        nla_set_error("an element has %d interacting elements (limit %d)", maxc, NLA_MAX_PAIRS_PER_K);
        return NLA_E_UNSUPPORTED;
    }
    P->n_pairs = hptr[K];
    if (3 * P->n_pairs >= (int64_t)INT32_MAX) {
        nla_set_error("too many pairs (%lld) for 32-bit contribution indices", (long long)P->n_pairs);
        return NLA_E_UNSUPPORTED;
    }
    NLA_TRY(P->arena.get(&P->pair_ptr, K + 1));
    NLA_TRY(P->arena.get(&P->pair_kp, P->n_pairs));
    NLA_TRY(P->arena.get(&P->pair_k, P->n_pairs));
    NLA_HIP(hipMemcpyAsync(P->pair_ptr, hptr.data(), sizeof(int64_t) * (K + 1), hipMemcpyHostToDevice, s));
    k_pair_emit<<<K, 256, 0, s>>>(K, Q, P->E, P->pair_ptr, P->pair_kp);
    k_pair_k<<<K, 256, 0, s>>>(K, P->pair_ptr, P->pair_k);
    if (P->rules.n_out2 > 0 && P->n_pairs > 0) {
        NLA_TRY(P->arena.get(&P->pair_r2, P->n_pairs));
        k_pair_rule2<<<grid_for(P->n_pairs, 256), 256, 0, s>>>(P->n_pairs, P->pair_k, P->pair_kp, P->E,
                                                              P->rules.switch_dist, P->pair_r2);
    }
    // processing order of the constant-kernel pair kernels: band pairs first,
    // then the deep ones (a stable sort of the keys 2 k + deep); under the
    // intersection, overlap and barycenter balls every item of a deep pair is
    // whole (for the barycenter ball: |x_q - b_k'| <= r_k + |b_k - b_k'| <= delta)
    // and under the shifted and barycenter-support balls every region of a deep
    // pair is whole; their kernel sums deep pairs with a symmetric inner rule
    const bool ordered = pr.kernel == NLA_KERNEL_CONSTANT &&
                         (pr.ball == NLA_BALL_RETRI || pr.ball == NLA_BALL_OVERLAP ||
                          pr.ball == NLA_BALL_BARYCENTER ||
                          ((pr.ball == NLA_BALL_SHIFTED || pr.ball == NLA_BALL_BARYSUPPORT) && P->rules.in_sym)) &&
                         P->n_pairs > 0 && 2 * (int64_t)K < (int64_t)UINT32_MAX;
    if (ordered) {
        const int64_t NP = P->n_pairs;
        Scratch S;
        uint32_t *key, *skey;
        int32_t *val;
        NLA_TRY(S.get(&key, NP));
        NLA_TRY(S.get(&skey, NP));
        NLA_TRY(S.get(&val, NP));
        NLA_TRY(P->arena.get(&P->proc_p, NP));
        NLA_TRY(P->arena.get(&P->proc_kp, NP));
        NLA_TRY(P->arena.get(&P->nband, K));
        k_deep_keys<<<grid_for(NP, 256), 256, 0, s>>>(NP, P->pair_k, P->pair_kp, P->E, pr.delta, key, val);
        const int kb = bits_for(2 * (uint64_t)K);
        size_t tb = 0;
        NLA_HIP(rocprim::radix_sort_pairs(nullptr, tb, key, skey, val, P->proc_p, (size_t)NP, 0, kb, s));
        void *tmp;
        NLA_TRY(S.get((char **)&tmp, tb));
        NLA_HIP(rocprim::radix_sort_pairs(tmp, tb, key, skey, val, P->proc_p, (size_t)NP, 0, kb, s));
        k_proc_kp<<<grid_for(NP, 256), 256, 0, s>>>(NP, P->proc_p, P->pair_kp, P->proc_kp);
        k_nband<<<grid_for(K, 256), 256, 0, s>>>(K, P->pair_ptr, skey, P->nband);
        NLA_HIP(hipGetLastError());
        std::vector<int32_t> nb((size_t)K);
        std::vector<int64_t> pp((size_t)K + 1);
        NLA_HIP(hipMemcpyAsync(nb.data(), P->nband, sizeof(int32_t) * K, hipMemcpyDeviceToHost, s));
        NLA_HIP(hipMemcpyAsync(pp.data(), P->pair_ptr, sizeof(int64_t) * (K + 1), hipMemcpyDeviceToHost, s));
        NLA_HIP(hipStreamSynchronize(s));
        for (int k = 0; k < K; k++) P->n_deep += pp[k + 1] - pp[k] - nb[k];
    }
    // launch order of the pair kernels: outer elements by decreasing work (their
    // band pairs when deep pairs are collapsed, else all their pairs), so that
    // the heaviest start first and the light ones fill the end of the launch
    // instead of a few heavy ones trailing it; the work is counted in groups of
    // 16 pairs and a group keeps index order, so that neighbouring elements,
    // which share their partners' records, still run side by side
    NLA_TRY(P->arena.get(&P->korder, K > 0 ? K : 1));
    if (K > 0) {
        std::vector<int64_t> pp((size_t)K + 1);
        std::vector<int32_t> nb(P->nband ? (size_t)K : 0), ord((size_t)K);
        NLA_HIP(hipMemcpyAsync(pp.data(), P->pair_ptr, sizeof(int64_t) * (K + 1), hipMemcpyDeviceToHost, s));
        if (P->nband) NLA_HIP(hipMemcpyAsync(nb.data(), P->nband, sizeof(int32_t) * K, hipMemcpyDeviceToHost, s));
        NLA_HIP(hipStreamSynchronize(s));
        for (int k = 0; k < K; k++) ord[k] = k;
        auto work = [&](int k) { return (P->nband ? (int64_t)nb[k] : pp[k + 1] - pp[k]) >> 4; };
        std::stable_sort(ord.begin(), ord.end(), [&](int a, int b) { return work(a) > work(b); });
        NLA_HIP(hipMemcpyAsync(P->korder, ord.data(), sizeof(int32_t) * K, hipMemcpyHostToDevice, s));
    }
    NLA_HIP(hipGetLastError());
    NLA_HIP(hipStreamSynchronize(s));
    return NLA_OK;
}

int nla_build_pattern(nla_plan *P, hipStream_t s)
{
    const int K = P->K, J = P->J;
    const int64_t NP = P->n_pairs;
    Scratch S;
    uint8_t *app;
    NLA_TRY(S.get(&app, K));
    NLA_HIP(hipMemsetAsync(app, 0, K, s));
    if (NP > 0) k_appears<<<grid_for(NP, 256), 256, 0, s>>>(NP, P->pair_k, P->pair_kp, app);
    const int64_t nkeys = 18 * NP + 9 * (int64_t)K;
    const uint64_t sentinel = (uint64_t)J * (uint64_t)J;
    uint64_t *keys, *skeys, *ukeys;
    NLA_TRY(S.get(&keys, nkeys));
    NLA_TRY(S.get(&skeys, nkeys));
    if (NP > 0) k_keys_pairs<<<grid_for(NP, 256), 256, 0, s>>>(NP, J, P->tri, P->pair_k, P->pair_kp, keys);
    k_keys_elems<<<grid_for(K, 256), 256, 0, s>>>(K, J, P->tri, app, sentinel, keys + 18 * NP);
    const int kbits = bits_for(sentinel);
    size_t tb = 0;
    NLA_HIP(rocprim::radix_sort_keys(nullptr, tb, keys, skeys, (size_t)nkeys, 0, kbits, s));
    void *tmp;
    NLA_TRY(S.get((char **)&tmp, tb));
    NLA_HIP(rocprim::radix_sort_keys(tmp, tb, keys, skeys, (size_t)nkeys, 0, kbits, s));
    // unique keys -> pattern (reuse `keys` as output)
    ukeys = keys;
    int64_t *nuniq;
    NLA_TRY(S.get(&nuniq, 1));
    size_t tb2 = 0;
    NLA_HIP(rocprim::unique(nullptr, tb2, skeys, ukeys, nuniq, (size_t)nkeys, rocprim::equal_to<uint64_t>(), s));
    void *tmp2;
    NLA_TRY(S.get((char **)&tmp2, tb2));
    NLA_HIP(rocprim::unique(tmp2, tb2, skeys, ukeys, nuniq, (size_t)nkeys, rocprim::equal_to<uint64_t>(), s));
    int64_t hu = 0;
    NLA_HIP(hipMemcpyAsync(&hu, nuniq, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    NLA_HIP(hipStreamSynchronize(s));
    uint64_t last = 0;
    NLA_HIP(hipMemcpy(&last, ukeys + hu - 1, sizeof(uint64_t), hipMemcpyDeviceToHost));
    const int64_t nnz = (last == sentinel) ? hu - 1 : hu;
    P->nnz = nnz;
    NLA_TRY(P->arena.get(&P->rowptr, J + 1));
    NLA_TRY(P->arena.get(&P->col, nnz));
    NLA_TRY(P->arena.get(&P->mirror, nnz));
    uint8_t *upflag;
    int64_t *upscan, *up_of;
    NLA_TRY(S.get(&upflag, nnz));
    NLA_TRY(S.get(&upscan, nnz));
    NLA_TRY(S.get(&up_of, nnz));
    k_rowptr<<<grid_for(J + 1, 256), 256, 0, s>>>(J, ukeys, nnz, P->rowptr);
    k_cols<<<grid_for(nnz, 256), 256, 0, s>>>(nnz, J, ukeys, P->col, P->mirror, upflag);
    // exclusive scan of the upper-triangle flags (host; one-time, nnz bytes)
    std::vector<uint8_t> hf(nnz);
    NLA_HIP(hipMemcpyAsync(hf.data(), upflag, nnz, hipMemcpyDeviceToHost, s));
    NLA_HIP(hipStreamSynchronize(s));
    std::vector<int64_t> hsc(nnz);
    int64_t acc = 0;
    for (int64_t t = 0; t < nnz; t++) {
        hsc[t] = acc;
        acc += hf[t];
    }
    P->n_up = acc;
    NLA_HIP(hipMemcpyAsync(upscan, hsc.data(), sizeof(int64_t) * nnz, hipMemcpyHostToDevice, s));
    NLA_TRY(P->arena.get(&P->up_dst, P->n_up));
    k_up_index<<<grid_for(nnz, 256), 256, 0, s>>>(nnz, upflag, upscan, P->up_dst, up_of);
    // column sets C_k (sorted unique nodes of the inner elements of k)
    const int64_t n3 = 3 * NP;
    uint64_t *ck64, *sck64, *U;
    int64_t *nu_d;
    NLA_TRY(S.get(&ck64, n3));
    NLA_TRY(S.get(&sck64, n3));
    NLA_TRY(S.get(&U, n3));
    NLA_TRY(S.get(&nu_d, 1));
    int64_t nu = 0;
    if (NP > 0) {
        k_colkeys<<<grid_for(NP, 256), 256, 0, s>>>(NP, P->tri, P->pair_k, P->pair_kp, ck64);
        const int b64 = 32 + bits_for((uint64_t)K);
        size_t t1 = 0;
        NLA_HIP(rocprim::radix_sort_keys(nullptr, t1, ck64, sck64, (size_t)n3, 0, b64, s));
        void *tm1;
        NLA_TRY(S.get((char **)&tm1, t1));
        NLA_HIP(rocprim::radix_sort_keys(tm1, t1, ck64, sck64, (size_t)n3, 0, b64, s));
        size_t t2 = 0;
        NLA_HIP(rocprim::unique(nullptr, t2, sck64, U, nu_d, (size_t)n3, rocprim::equal_to<uint64_t>(), s));
        void *tm2;
        NLA_TRY(S.get((char **)&tm2, t2));
        NLA_HIP(rocprim::unique(tm2, t2, sck64, U, nu_d, (size_t)n3, rocprim::equal_to<uint64_t>(), s));
        NLA_HIP(hipMemcpyAsync(&nu, nu_d, sizeof(int64_t), hipMemcpyDeviceToHost, s));
        NLA_HIP(hipStreamSynchronize(s));
    }
    P->n_cols = nu;
    if (3 * nu + 12 * (int64_t)K + 6 * NP >= (int64_t)INT32_MAX) {
        nla_set_error("value array too large for 32-bit codes");
        return NLA_E_UNSUPPORTED;
    }
    NLA_TRY(P->arena.get(&P->col_off, K + 1));
    NLA_TRY(P->arena.get(&P->colset, nu));
    NLA_TRY(P->arena.get(&P->colent_ptr, nu + 1));
    // four entries of padding: the fold reads a column's next four entries at once
    NLA_TRY(P->arena.get(&P->colent, n3 + 4));
    NLA_HIP(hipMemsetAsync(P->colent + n3, 0, 4 * sizeof(uint16_t), s));
    k_col_off<<<grid_for(K + 1, 256), 256, 0, s>>>(K, U, nu, P->col_off);
    if (nu > 0) k_colset<<<grid_for(nu, 256), 256, 0, s>>>(nu, U, P->colset);
    {
        std::vector<int64_t> hoff(K + 1);
        NLA_HIP(hipMemcpyAsync(hoff.data(), P->col_off, sizeof(int64_t) * (K + 1), hipMemcpyDeviceToHost, s));
        NLA_HIP(hipStreamSynchronize(s));
        int64_t mc = 0;
        for (int k = 0; k < K; k++) mc = std::max(mc, hoff[k + 1] - hoff[k]);
        P->max_cols = (int32_t)mc;
        if (mc > 1536) {
            nla_set_error("an element reaches %lld nodes (limit 1536)", (long long)mc);
            return NLA_E_UNSUPPORTED;
        }
    }
    // per column slot: contributions (p_local, b) in pair order (stable sort by slot)
    if (NP > 0) {
        uint32_t *sk, *skk;
        uint16_t *sv;
        NLA_TRY(S.get(&sk, n3));
        NLA_TRY(S.get(&skk, n3));
        NLA_TRY(S.get(&sv, n3));
        k_colent_keys<<<grid_for(NP, 256), 256, 0, s>>>(NP, P->tri, P->pair_k, P->pair_kp, P->pair_ptr, P->proc_p,
                                                        U, nu, sk, sv);
        const int sb = bits_for((uint64_t)nu);
        size_t t3 = 0;
        NLA_HIP(rocprim::radix_sort_pairs(nullptr, t3, sk, skk, sv, P->colent, (size_t)n3, 0, sb, s));
        void *tm3;
        NLA_TRY(S.get((char **)&tm3, t3));
        NLA_HIP(rocprim::radix_sort_pairs(tm3, t3, sk, skk, sv, P->colent, (size_t)n3, 0, sb, s));
        k_slot_ptr<<<grid_for(nu + 1, 256), 256, 0, s>>>(nu, skk, n3, P->colent_ptr);
    } else {
        NLA_HIP(hipMemsetAsync(P->colent_ptr, 0, sizeof(int32_t), s));
    }
    // codes of every upper entry into the value array [R (3 n_cols) | E (6K)]
    const int64_t e_base = 3 * nu;
    int32_t *ecnt;
    NLA_TRY(S.get(&ecnt, P->n_up));
    NLA_TRY(P->arena.get(&P->up_ptr, P->n_up + 1));
    k_entry_codes<<<grid_for(P->n_up, 256), 256, 0, s>>>(P->n_up, J, P->up_dst, nullptr, ukeys, P->tri, P->n2e_all_ptr,
                                                        P->n2e_all, P->col_off, P->colset, e_base, 0, ecnt, nullptr,
                                                        nullptr);
    {
        std::vector<int32_t> hc(P->n_up);
        std::vector<int64_t> hp(P->n_up + 1);
        NLA_HIP(hipMemcpyAsync(hc.data(), ecnt, sizeof(int32_t) * P->n_up, hipMemcpyDeviceToHost, s));
        NLA_HIP(hipStreamSynchronize(s));
        hp[0] = 0;
        for (int64_t u = 0; u < P->n_up; u++) hp[u + 1] = hp[u] + hc[u];
        P->n_codes = hp[P->n_up];
        NLA_HIP(hipMemcpyAsync(P->up_ptr, hp.data(), sizeof(int64_t) * (P->n_up + 1), hipMemcpyHostToDevice, s));
    }
    NLA_TRY(P->arena.get(&P->codes, P->n_codes));
    k_entry_codes<<<grid_for(P->n_up, 256), 256, 0, s>>>(P->n_up, J, P->up_dst, nullptr, ukeys, P->tri, P->n2e_all_ptr,
                                                        P->n2e_all, P->col_off, P->colset, e_base, 1, nullptr,
                                                        P->up_ptr, P->codes);
    // vertex-sharing pairs of the singular kernel and the codes of their blocks
    P->n_near = 0;
    if (P->prob.kernel == NLA_KERNEL_FRACTIONAL && NP > 0) {
        NLA_TRY(P->arena.get(&P->near_flag, NP));
        k_near_flag<<<grid_for(NP, 256), 256, 0, s>>>(NP, P->tri, P->pair_k, P->pair_kp, P->near_flag);
        std::vector<uint8_t> hf(NP);
        NLA_HIP(hipMemcpyAsync(hf.data(), P->near_flag, NP, hipMemcpyDeviceToHost, s));
        NLA_HIP(hipStreamSynchronize(s));
        std::vector<int64_t> nl;
        for (int64_t p = 0; p < NP; p++)
            if (hf[p]) nl.push_back(p);
        P->n_near = (int64_t)nl.size();
        NLA_TRY(P->arena.get(&P->near_pair, nl.size()));
        NLA_HIP(hipMemcpyAsync(P->near_pair, nl.data(), sizeof(int64_t) * nl.size(), hipMemcpyHostToDevice, s));
        const int64_t ns = 36 * P->n_near;
        if (21 * P->n_near >= (int64_t)INT32_MAX) { nla_set_error("too many near pairs"); return NLA_E_UNSUPPORTED; }
        uint32_t *nk, *snk;
        int32_t *nv, *snv;
        NLA_TRY(S.get(&nk, ns));
        NLA_TRY(S.get(&snk, ns));
        NLA_TRY(S.get(&nv, ns));
        NLA_TRY(S.get(&snv, ns));
        const uint32_t nsent = (uint32_t)P->n_up;
        int64_t *partner;
        NLA_TRY(P->arena.get(&partner, P->n_near));
        P->near_partner = partner;
        k_near_partner<<<grid_for(P->n_near, 256), 256, 0, s>>>(P->n_near, P->near_pair, P->pair_k, P->pair_kp,
                                                               P->pair_ptr, partner);
        {
            // the blocks computed: near pairs without a mirror partner
            std::vector<int64_t> hp(P->n_near), cl;
            NLA_HIP(hipMemcpyAsync(hp.data(), partner, sizeof(int64_t) * P->n_near, hipMemcpyDeviceToHost, s));
            NLA_HIP(hipStreamSynchronize(s));
            for (int64_t i = 0; i < P->n_near; i++)
                if (hp[i] < 0) cl.push_back(i);
            P->n_near_comp = (int64_t)cl.size();
            NLA_TRY(P->arena.get(&P->near_comp, cl.size() > 0 ? cl.size() : 1));
            if (!cl.empty())
                NLA_HIP(hipMemcpyAsync(P->near_comp, cl.data(), sizeof(int64_t) * cl.size(), hipMemcpyHostToDevice, s));
            NLA_HIP(hipStreamSynchronize(s));
        }
        k_near_codes<<<grid_for(P->n_near, 256), 256, 0, s>>>(P->n_near, J, P->near_pair, P->tri, P->pair_k, P->pair_kp,
                                                             ukeys, nnz, up_of, nsent, partner, nk, nv);
        size_t t5 = 0;
        const int nb = bits_for((uint64_t)nsent);
        NLA_HIP(rocprim::radix_sort_pairs(nullptr, t5, nk, snk, nv, snv, (size_t)ns, 0, nb, s));
        void *tm5;
        NLA_TRY(S.get((char **)&tm5, t5));
        NLA_HIP(rocprim::radix_sort_pairs(tm5, t5, nk, snk, nv, snv, (size_t)ns, 0, nb, s));
        NLA_TRY(P->arena.get(&P->nup_ptr, P->n_up + 1));
        k_up_ptr<<<grid_for(P->n_up + 1, 256), 256, 0, s>>>(P->n_up, snk, ns, P->nup_ptr);
        int64_t nn = 0;
        NLA_HIP(hipMemcpyAsync(&nn, P->nup_ptr + P->n_up, sizeof(int64_t), hipMemcpyDeviceToHost, s));
        NLA_HIP(hipStreamSynchronize(s));
        P->n_ncodes = nn;
        NLA_TRY(P->arena.get(&P->ncodes, nn));
        NLA_HIP(hipMemcpyAsync(P->ncodes, snv, sizeof(int32_t) * nn, hipMemcpyDeviceToDevice, s));
    }
    // transposed pair order (k' major, k ascending within: stable radix sort of
    // k'); with the processing order on, the deep pairs sort past the last
    // element (key K) and so drop out: their Myy reaches E(k') as one sum per
    // element (the pair kernel adds it to Mxx(k'))
    NLA_TRY(P->arena.get(&P->tptr, K + 1));
    NLA_TRY(P->arena.get(&P->tperm, NP));
    if (NP > 0) {
        uint32_t *skp;
        int32_t *iota;
        NLA_TRY(S.get(&skp, NP));
        NLA_TRY(S.get(&iota, NP));
        k_iota<<<grid_for(NP, 256), 256, 0, s>>>(NP, iota);
        const uint32_t *tkey = (const uint32_t *)P->pair_kp;
        if (P->nband) {
            uint32_t *kk;
            NLA_TRY(S.get(&kk, NP));
            k_tkeys<<<grid_for(NP, 256), 256, 0, s>>>(NP, P->pair_k, P->pair_kp, P->E, P->prob.delta, K, kk);
            tkey = kk;
        }
        size_t tb4 = 0;
        const int kb = bits_for((uint64_t)K + 1);
        NLA_HIP(rocprim::radix_sort_pairs(nullptr, tb4, tkey, skp, iota, P->tperm, (size_t)NP, 0, kb, s));
        void *tmp4;
        NLA_TRY(S.get((char **)&tmp4, tb4));
        NLA_HIP(rocprim::radix_sort_pairs(tmp4, tb4, tkey, skp, iota, P->tperm, (size_t)NP, 0, kb, s));
        k_tptr<<<grid_for(K + 1, 256), 256, 0, s>>>(K, skp, NP, P->tptr);
    } else {
        NLA_HIP(hipMemsetAsync(P->tptr, 0, sizeof(int64_t) * (K + 1), s));
    }
    // A = D[free, free]
    const int nf = P->n_free;
    if (nf > 0) {
        int64_t *acnt;
        NLA_TRY(S.get(&acnt, nf));
        k_a_count<<<grid_for(nf, 256), 256, 0, s>>>(nf, P->free_nodes, P->rowptr, P->col, P->node_to_free, acnt);
        std::vector<int64_t> hac(nf), har(nf + 1);
        NLA_HIP(hipMemcpyAsync(hac.data(), acnt, sizeof(int64_t) * nf, hipMemcpyDeviceToHost, s));
        NLA_HIP(hipStreamSynchronize(s));
        har[0] = 0;
        for (int i = 0; i < nf; i++) har[i + 1] = har[i] + hac[i];
        P->nnz_free = har[nf];
        NLA_TRY(P->arena.get(&P->a_rowptr, nf + 1));
        NLA_TRY(P->arena.get(&P->a_col, P->nnz_free));
        NLA_TRY(P->arena.get(&P->a_src, P->nnz_free));
        NLA_HIP(hipMemcpyAsync(P->a_rowptr, har.data(), sizeof(int64_t) * (nf + 1), hipMemcpyHostToDevice, s));
        k_a_fill<<<grid_for(nf, 256), 256, 0, s>>>(nf, P->free_nodes, P->rowptr, P->col, P->node_to_free, P->a_rowptr,
                                                    P->a_col, P->a_src);
    }
    NLA_HIP(hipGetLastError());
    NLA_HIP(hipStreamSynchronize(s));
    return NLA_OK;
}

// ------------------------------------------------------------------- API
static void fill_rules(const nla_problem *p, RuleSet *R)
{
    memset(R, 0, sizeof(*R));
    R->n_out = p->outer.n;
    R->n_in = p->inner.n;
    for (int q = 0; q < p->outer.n; q++) {
        for (int a = 0; a < 3; a++) R->out_lam[q][a] = p->outer.lambda[3 * q + a];
        R->out_w[q] = p->outer.w[q];
    }
    R->n_out2 = p->outer2.n > 0 ? p->outer2.n : 0;
    for (int q = 0; q < R->n_out2; q++) {
        for (int a = 0; a < 3; a++) R->out2_lam[q][a] = p->outer2.lambda[3 * q + a];
        R->out2_w[q] = p->outer2.w[q];
    }
    R->switch_dist = R->n_out2 > 0 ? p->switch_dist : 0.0;
    for (int q = 0; q < p->inner.n; q++) {
        for (int a = 0; a < 3; a++) {
            R->in_lam[q][a] = p->inner.lambda[3 * q + a];
            R->in_lamf[q][a] = (float)p->inner.lambda[3 * q + a];
        }
        R->in_w[q] = p->inner.w[q];
        R->in_wf[q] = (float)p->inner.w[q];
        R->in_wsum += p->inner.w[q];
        for (int i = 0; i < 3; i++) {
            R->in_m1[i] += p->inner.w[q] * p->inner.lambda[3 * q + i];
            for (int j = 0; j < 3; j++)
                R->in_m2[i][j] += p->inner.w[q] * p->inner.lambda[3 * q + i] * p->inner.lambda[3 * q + j];
        }
    }
    {
        const double tol = 1e-15;
        bool sym = std::fabs(R->in_m1[1] - R->in_m1[0]) <= tol && std::fabs(R->in_m1[2] - R->in_m1[0]) <= tol;
        for (int i = 0; i < 3; i++)
            for (int j = 0; j < 3; j++)
                sym = sym && std::fabs(R->in_m2[i][j] - (i == j ? R->in_m2[0][0] : R->in_m2[0][1])) <= tol;
        R->in_sym = sym ? 1 : 0;
        // exact for quadratics on the reference triangle (weights summing to 1/2):
        // sum w lambda_i = 1/6, sum w lambda_i lambda_j = (1 + [i == j]) / 24
        bool q2 = std::fabs(R->in_wsum - 0.5) <= 1e-14;
        for (int i = 0; i < 3; i++) {
            q2 = q2 && std::fabs(R->in_m1[i] - 1.0 / 6.0) <= 1e-14;
            for (int j = 0; j < 3; j++) q2 = q2 && std::fabs(R->in_m2[i][j] - (i == j ? 1.0 / 12.0 : 1.0 / 24.0)) <= 1e-14;
        }
        R->in_q2exact = q2 ? 1 : 0;
    }
    if (p->kernel == NLA_KERNEL_FRACTIONAL) {
        R->duffy_n = p->duffy_n;
        for (int i = 0; i < p->duffy_n; i++) {
            R->duffy_x[i] = p->duffy_x[i];
            R->duffy_w[i] = p->duffy_w[i];
        }
    }
}

static int plan_create(const nla_mesh *m, const nla_problem *p, hipStream_t s, nla_plan *P)
{
    NLA_HIP(hipGetDevice(&P->device));
    P->K = m->n_triangles;
    P->J = m->n_vertices;
    P->prob = *p;
    P->prob.duffy_x = nullptr;
    P->prob.duffy_w = nullptr;
    P->prob.outer.lambda = P->prob.outer.w = nullptr;
    P->prob.outer2.lambda = P->prob.outer2.w = nullptr;
    P->prob.inner.lambda = P->prob.inner.w = nullptr;
    fill_rules(p, &P->rules);
    const int K = P->K, J = P->J;
    NLA_TRY(P->arena.get(&P->d_rules, 1));
    NLA_TRY(P->arena.get(&P->xy, 2 * (size_t)J));
    NLA_TRY(P->arena.get(&P->tri, 3 * (size_t)K));
    NLA_TRY(P->arena.get(&P->tin, K));
    NLA_TRY(P->arena.get(&P->nfree, J));
    double *eb;
    NLA_TRY(P->arena.get(&eb, 10 * (size_t)K));
    double **f[10] = {&P->E.vx0, &P->E.vy0, &P->E.vx1, &P->E.vy1, &P->E.vx2, &P->E.vy2,
                      &P->E.bx, &P->E.by, &P->E.a2, &P->E.r};
    for (int i = 0; i < 10; i++) *f[i] = eb + (size_t)i * K;
    NLA_TRY(P->arena.get(&P->E.pk, 16 * (size_t)K));
    NLA_TRY(P->arena.get(&P->xq, 2 * (size_t)K * P->rules.n_out));
    if (P->rules.n_out2 > 0) NLA_TRY(P->arena.get(&P->xq2, 2 * (size_t)K * P->rules.n_out2));
    NLA_HIP(hipMemcpyAsync(P->d_rules, &P->rules, sizeof(RuleSet), hipMemcpyHostToDevice, s));
    NLA_HIP(hipMemcpyAsync(P->xy, m->xy, sizeof(double) * 2 * J, hipMemcpyHostToDevice, s));
    NLA_HIP(hipMemcpyAsync(P->tri, m->tri, sizeof(int32_t) * 3 * K, hipMemcpyHostToDevice, s));
    NLA_HIP(hipMemcpyAsync(P->tin, m->tri_in_omega, K, hipMemcpyHostToDevice, s));
    NLA_HIP(hipMemcpyAsync(P->nfree, m->node_free, J, hipMemcpyHostToDevice, s));
    // free nodes, node -> free index, node -> Omega element adjacency (host, mesh only)
    std::vector<int32_t> fn, n2f(J, -1);
    for (int j = 0; j < J; j++)
        if (m->node_free[j]) {
            n2f[j] = (int32_t)fn.size();
            fn.push_back(j);
        }
    P->n_free = (int32_t)fn.size();
    std::vector<int32_t> n2e_ptr(J + 1, 0), n2e;
    for (int k = 0; k < K; k++)
        if (m->tri_in_omega[k])
            for (int a = 0; a < 3; a++) n2e_ptr[m->tri[3 * k + a] + 1]++;
    for (int j = 0; j < J; j++) n2e_ptr[j + 1] += n2e_ptr[j];
    n2e.resize(n2e_ptr[J]);
    std::vector<int32_t> fill(n2e_ptr.begin(), n2e_ptr.end() - 1);
    for (int k = 0; k < K; k++)
        if (m->tri_in_omega[k])
            for (int a = 0; a < 3; a++) n2e[fill[m->tri[3 * k + a]]++] = 3 * k + a;
    std::vector<int32_t> na_ptr(J + 1, 0), na;
    for (int k = 0; k < K; k++)
        for (int a = 0; a < 3; a++) na_ptr[m->tri[3 * k + a] + 1]++;
    for (int j = 0; j < J; j++) na_ptr[j + 1] += na_ptr[j];
    na.resize(na_ptr[J]);
    {
        std::vector<int32_t> f2(na_ptr.begin(), na_ptr.end() - 1);
        for (int k = 0; k < K; k++)
            for (int a = 0; a < 3; a++) na[f2[m->tri[3 * k + a]]++] = 3 * k + a;
    }
    NLA_TRY(P->arena.get(&P->n2e_all_ptr, J + 1));
    NLA_TRY(P->arena.get(&P->n2e_all, na.size()));
    NLA_HIP(hipMemcpyAsync(P->n2e_all_ptr, na_ptr.data(), sizeof(int32_t) * (J + 1), hipMemcpyHostToDevice, s));
    NLA_HIP(hipMemcpyAsync(P->n2e_all, na.data(), sizeof(int32_t) * na.size(), hipMemcpyHostToDevice, s));
    NLA_TRY(P->arena.get(&P->free_nodes, fn.size()));
    NLA_TRY(P->arena.get(&P->node_to_free, J));
    NLA_TRY(P->arena.get(&P->n2e_ptr, J + 1));
    NLA_TRY(P->arena.get(&P->n2e, n2e.size()));
    if (!fn.empty()) NLA_HIP(hipMemcpyAsync(P->free_nodes, fn.data(), sizeof(int32_t) * fn.size(), hipMemcpyHostToDevice, s));
    NLA_HIP(hipMemcpyAsync(P->node_to_free, n2f.data(), sizeof(int32_t) * J, hipMemcpyHostToDevice, s));
    NLA_HIP(hipMemcpyAsync(P->n2e_ptr, n2e_ptr.data(), sizeof(int32_t) * (J + 1), hipMemcpyHostToDevice, s));
    if (!n2e.empty()) NLA_HIP(hipMemcpyAsync(P->n2e, n2e.data(), sizeof(int32_t) * n2e.size(), hipMemcpyHostToDevice, s));
    k_elem<<<grid_for(K, 128), 128, 0, s>>>(K, P->xy, P->tri, P->E, P->d_rules, P->xq, P->xq2);
    NLA_HIP(hipGetLastError());
    NLA_TRY(nla_build_pairs(P, s));
    NLA_TRY(nla_build_pattern(P, s));
    NLA_TRY(P->arena.get(&P->counters, 6));
    if (p->precision == NLA_FP32_LEARNED) {
        P->mlp = (const nla_mlp *)p->mlp;
        P->mlp_dom = nla_mlp_domain_of(P->mlp);
        NLA_TRY(nla_build_routes(P, s));
    }
    return NLA_OK;
}

extern "C" int nla_plan_create(const nla_mesh *mesh, const nla_problem *prob, void *stream, nla_plan **out)
{
    if (!out) { nla_set_error("out is null"); return NLA_E_INVALID; }
    *out = nullptr;
    int st = validate(mesh, prob);
    if (st != NLA_OK) return st;
    nla_plan *P = new (std::nothrow) nla_plan();
    if (!P) { nla_set_error("host allocation failed"); return NLA_E_NOMEM; }
    try {
        st = plan_create(mesh, prob, (hipStream_t)stream, P);
    } catch (...) {
        nla_set_error("unexpected exception in plan creation");
        st = NLA_E_DEVICE;
    }
    if (st != NLA_OK) {
        delete P;
        return st;
    }
    *out = P;
    return NLA_OK;
}

extern "C" int nla_plan_info(const nla_plan *P, nla_info *info)
{
    if (!P || !info) { nla_set_error("null argument"); return NLA_E_INVALID; }
    info->n_pairs = P->n_pairs;
    info->nnz_full = P->nnz;
    info->nnz_free = P->nnz_free;
    info->n_free = P->n_free;
    info->n_outer = P->rules.n_out;
    info->n_codes = P->n_codes;
    info->n_near = P->n_near;
    info->n_deep = P->n_deep;
    unsigned long long c[6] = {0, 0, 0, 0, 0, 0};
    if (P->assembled) NLA_HIP(hipMemcpy(c, P->counters, sizeof(c), hipMemcpyDeviceToHost));
    for (int i = 0; i < 4; i++) info->items[i] = (int64_t)c[i];
    info->subtriangles = (int64_t)c[4];
    info->caps = (int64_t)c[5];
    return NLA_OK;
}

extern "C" int nla_pairs_view(const nla_plan *P, const int64_t **pair_ptr, const int32_t **pair_kp)
{
    if (!P || !pair_ptr || !pair_kp) { nla_set_error("null argument"); return NLA_E_INVALID; }
    *pair_ptr = P->pair_ptr;
    *pair_kp = P->pair_kp;
    return NLA_OK;
}

extern "C" int nla_outer_points(const nla_plan *P, double *xq, void *stream)
{
    if (!P || !xq) { nla_set_error("null argument"); return NLA_E_INVALID; }
    NLA_HIP(hipMemcpyAsync(xq, P->xq, sizeof(double) * 2 * (size_t)P->K * P->rules.n_out, hipMemcpyDeviceToDevice,
                           (hipStream_t)stream));
    return NLA_OK;
}

extern "C" int nla_csr_view(const nla_plan *P, int32_t which, const int64_t **rowptr, const int32_t **col,
                            const void **val, int32_t *val_dtype)
{
    if (!P || !rowptr || !col || !val || !val_dtype) { nla_set_error("null argument"); return NLA_E_INVALID; }
    if (which != 0 && which != 1) { nla_set_error("which must be 0 or 1"); return NLA_E_INVALID; }
    if (!P->assembled) { nla_set_error("nla_assemble has not run"); return NLA_E_STATE; }
    *rowptr = which ? P->a_rowptr : P->rowptr;
    *col = which ? P->a_col : P->col;
    *val = which ? P->a_val : P->val;
    *val_dtype = P->val_dtype;
    return NLA_OK;
}

extern "C" int nla_load_view(const nla_plan *P, const double **b)
{
    if (!P || !b) { nla_set_error("null argument"); return NLA_E_INVALID; }
    if (!P->have_load) { nla_set_error("no load vector assembled"); return NLA_E_STATE; }
    *b = P->b;
    return NLA_OK;
}

extern "C" int nla_free_nodes_view(const nla_plan *P, const int32_t **free_nodes)
{
    if (!P || !free_nodes) { nla_set_error("null argument"); return NLA_E_INVALID; }
    *free_nodes = P->free_nodes;
    return NLA_OK;
}

// Myy of the deep pairs, which the FP64 assembly folds into one sum per inner
// element instead of storing: every item whole, so Myy = psi W(k) |E_k'| m2
// with W(k) the sum of the pair's outer weights over E_k.
template <class T>
__global__ void k_deep_myy(int64_t P, const int32_t *__restrict__ pk, const int32_t *__restrict__ pkp, ElemSoA E,
                           double delta, double psi, const RuleSet *__restrict__ R, const uint8_t *__restrict__ r2,
                           T *__restrict__ myy)
{
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= P) return;
    const int k = pk[p], kp = pkp[p];
    if (!pair_deep(E, k, kp, delta)) return;
    const bool second = r2 && r2[p] && R->n_out2 > 0;
    double ws = 0.0;
    if (second)
        for (int q = 0; q < R->n_out2; q++) ws += R->out2_w[q] * E.a2[k];
    else
        for (int q = 0; q < R->n_out; q++) ws += R->out_w[q] * E.a2[k];
    const int jj[6] = {0, 0, 0, 1, 1, 2}, ll[6] = {0, 1, 2, 1, 2, 2};
    for (int t = 0; t < 6; t++) myy[6 * p + t] = (T)(psi * (ws * E.a2[kp] * R->in_m2[jj[t]][ll[t]]));
}

extern "C" int nla_blocks_view(const nla_plan *P, const void **myy, const void **mxx, const void **elem,
                               const void **rows, const int64_t **col_off, const int32_t **colset, int32_t *dtype)
{
    if (!P || !myy || !mxx || !elem || !rows || !col_off || !colset || !dtype) {
        nla_set_error("null argument");
        return NLA_E_INVALID;
    }
    if (!P->assembled) { nla_set_error("nla_assemble has not run"); return NLA_E_STATE; }
    if (P->nband && P->n_pairs > 0) {
        // the deep pairs' records, formed here on request (after the assembly has finished)
        NLA_HIP(hipDeviceSynchronize());
        if (P->val_dtype == NLA_DTYPE_F64)
            k_deep_myy<double><<<grid_for(P->n_pairs, 256), 256, 0, 0>>>(
                P->n_pairs, P->pair_k, P->pair_kp, P->E, P->prob.delta, P->prob.kernel_c, P->d_rules, P->pair_r2,
                (double *)P->contrib);
        else
            k_deep_myy<float><<<grid_for(P->n_pairs, 256), 256, 0, 0>>>(
                P->n_pairs, P->pair_k, P->pair_kp, P->E, P->prob.delta, P->prob.kernel_c, P->d_rules, P->pair_r2,
                (float *)P->contrib);
        NLA_HIP(hipGetLastError());
        NLA_HIP(hipDeviceSynchronize());
    }
    const size_t es = P->val_dtype == NLA_DTYPE_F64 ? 8 : 4;
    const char *c = (const char *)P->contrib;
    *myy = c;
    *mxx = c + es * 6 * P->n_pairs;
    *rows = c + es * (6 * P->n_pairs + 6 * (int64_t)P->K);
    *elem = c + es * (6 * P->n_pairs + 6 * (int64_t)P->K + 3 * P->n_cols);
    *col_off = P->col_off;
    *colset = P->colset;
    *dtype = P->val_dtype;
    return NLA_OK;
}

// the blocks of mirrored near pairs, relabelled from their partners' (view only;
// the assembly reads the partner's block through the codes)
template <class T>
__global__ void k_near_mirror_fill(int64_t n_near, const int64_t *__restrict__ near_pair,
                                   const int32_t *__restrict__ tri, const int32_t *__restrict__ pk,
                                   const int32_t *__restrict__ pkp, const int64_t *__restrict__ partner,
                                   T *__restrict__ blk)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_near || partner[i] < 0) return;
    const int64_t j = partner[i], p = near_pair[i];
    const int k = pk[p], kp = pkp[p];
    int ps[6];
    bool merged[6];
    for (int I = 0; I < 6; I++) {
        const int g = I < 3 ? tri[3 * k + I] : tri[3 * kp + I - 3];
        ps[I] = -1;
        for (int a = 0; a < 3; a++)
            if (tri[3 * kp + a] == g) ps[I] = a;
        if (ps[I] < 0)
            for (int a = 0; a < 3; a++)
                if (tri[3 * k + a] == g) ps[I] = 3 + a;
        merged[I] = I >= 3 && (tri[3 * k] == g || tri[3 * k + 1] == g || tri[3 * k + 2] == g);
    }
    for (int I = 0; I < 6; I++)
        for (int Jj = I; Jj < 6; Jj++)
            blk[21 * i + upper_slot(I, Jj)] = (merged[I] || merged[Jj]) ? (T)0 : blk[21 * j + upper_slot(ps[I], ps[Jj])];
}

extern "C" int nla_near_view(const nla_plan *P, int64_t *n_near, const int64_t **near_pair, const void **blocks,
                             int32_t *dtype)
{
    if (!P || !n_near || !near_pair || !blocks || !dtype) { nla_set_error("null argument"); return NLA_E_INVALID; }
    if (!P->assembled) { nla_set_error("nla_assemble has not run"); return NLA_E_STATE; }
    if (P->n_near > 0 && P->n_near_comp < P->n_near) {
        NLA_HIP(hipDeviceSynchronize());
        if (P->val_dtype == NLA_DTYPE_F32)
            k_near_mirror_fill<float><<<grid_for(P->n_near, 256), 256>>>(P->n_near, P->near_pair, P->tri, P->pair_k,
                                                                        P->pair_kp, P->near_partner, (float *)P->near_blk);
        else
            k_near_mirror_fill<double><<<grid_for(P->n_near, 256), 256>>>(P->n_near, P->near_pair, P->tri, P->pair_k,
                                                                         P->pair_kp, P->near_partner, (double *)P->near_blk);
        NLA_HIP(hipGetLastError());
        NLA_HIP(hipDeviceSynchronize());
    }
    *n_near = P->n_near;
    *near_pair = P->near_pair;
    *blocks = P->near_blk;
    *dtype = P->val_dtype;
    return NLA_OK;
}

extern "C" int nla_cg(const nla_plan *P, const double *b, double *u, double rtol, int32_t maxit, int32_t *iters,
                      double *relres, void *stream)
{
    if (!P || !b || !u || !iters || !relres) { nla_set_error("null argument"); return NLA_E_INVALID; }
    if (!P->assembled) { nla_set_error("nla_assemble has not run"); return NLA_E_STATE; }
    if (maxit < 1 || !(rtol > 0)) { nla_set_error("maxit >= 1 and rtol > 0 required"); return NLA_E_INVALID; }
    return nla_cg_run(P, b, u, rtol, maxit, iters, relres, (hipStream_t)stream);
}

extern "C" int nla_assemble(nla_plan *P, const double *f_outer, const double *g_node, void *stream)
{
    if (!P) { nla_set_error("null plan"); return NLA_E_INVALID; }
    if ((f_outer == nullptr) != (g_node == nullptr)) { nla_set_error("pass both f_outer and g_node, or neither"); return NLA_E_INVALID; }
    return nla_numeric(P, f_outer, g_node, (hipStream_t)stream);
}

extern "C" int nla_set_timing(nla_plan *P, int32_t n)
{
    if (!P || n < 0) { nla_set_error("null plan or negative count"); return NLA_E_INVALID; }
    for (auto &e : P->ev)
        if (e) NLA_HIP(hipEventDestroy(e));
    P->ev.clear();
    P->timing_slots = n;
    P->timing_count = 0;
    if (n > 0) {
        P->ev.assign((size_t)n * (NLA_NPHASE + 1), nullptr);
        for (auto &e : P->ev) NLA_HIP(hipEventCreate(&e));
    }
    return NLA_OK;
}

extern "C" int nla_timings(const nla_plan *P, double *ms, int32_t *count)
{
    if (!P || !ms || !count) { nla_set_error("null argument"); return NLA_E_INVALID; }
    const int n = P->timing_count;
    *count = n;
    for (int i = 0; i < NLA_NPHASE; i++) ms[i] = 0.0;
    if (n == 0) return NLA_OK;
    NLA_HIP(hipEventSynchronize(P->ev[(size_t)(n - 1) * (NLA_NPHASE + 1) + NLA_NPHASE]));
    for (int c = 0; c < n; c++) {
        const hipEvent_t *e = &P->ev[(size_t)c * (NLA_NPHASE + 1)];
        for (int i = 0; i < NLA_NPHASE; i++) {
            if (!P->ran[i]) continue;
            float t = 0.f;
            NLA_HIP(hipEventElapsedTime(&t, e[i], e[i + 1]));
            ms[i] += t / n;
        }
    }
    return NLA_OK;
}

extern "C" void nla_plan_destroy(nla_plan *P) { delete P; }
