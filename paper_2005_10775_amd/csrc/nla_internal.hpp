// Internal declarations shared by the translation units of libnlasm.so.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>
#include <cstdio>
#include <cstdarg>
#include <vector>
#include "../../include/nlasm.h"

#define NLA_MAX_OUTER 16
#define NLA_MAX_INNER 32
#define NLA_MAX_CAP 64
#define NLA_MAX_PAIRS_PER_K 4096
#define NLA_MAX_DUFFY 24

void nla_set_error(const char *fmt, ...);

#define NLA_HIP(call)                                                                   \
    do {                                                                                \
        hipError_t e_ = (call);                                                         \
        if (e_ != hipSuccess) {                                                         \
            nla_set_error("%s failed: %s (%s:%d)", #call, hipGetErrorString(e_),        \
                          __FILE__, __LINE__);                                          \
            return NLA_E_DEVICE;                                                        \
        }                                                                               \
    } while (0)

#define NLA_TRY(expr)                                                                   \
    do {                                                                                \
        int s_ = (expr);                                                                \
        if (s_ != NLA_OK) return s_;                                                    \
    } while (0)

// Quadrature data as the kernels read it: outer/inner points plus the inner
// rule's own first and second barycentric moments (sum w mu_i, sum w mu_i mu_j),
// which let a constant-psi inner integral over a subtriangle be evaluated
// from the values of the P1 basis at its three vertices (the rule applied
// with its sums reordered, not a different rule).
struct RuleSet {
    int32_t n_out, n_in, duffy_n, in_sym;   // in_sym: inner rule symmetric under vertex permutations
    int32_t in_q2exact, pad_;               // inner rule integrates quadratics exactly
    double out_lam[NLA_MAX_OUTER][3];
    double out_w[NLA_MAX_OUTER];
    int32_t n_out2, pad2_;                  // second outer rule (0: none) for pairs closer than switch_dist
    double out2_lam[NLA_MAX_OUTER][3];
    double out2_w[NLA_MAX_OUTER];
    double switch_dist;
    double in_lam[NLA_MAX_INNER][3];
    double in_w[NLA_MAX_INNER];
    double in_wsum;
    double in_m1[3];
    double in_m2[3][3];
    double duffy_x[NLA_MAX_DUFFY];
    double duffy_w[NLA_MAX_DUFFY];
    float in_lamf[NLA_MAX_INNER][3];   // FP32 copies for the FP32 point quadrature
    float in_wf[NLA_MAX_INNER];
};

// Element data, structure of arrays, K entries each.
struct ElemSoA {
    double *vx0, *vy0, *vx1, *vy1, *vx2, *vy2; // vertices
    double *bx, *by;                           // barycenter ((v0+v1)+v2)/3
    double *a2;                                // twice the area
    double *r;                                 // max vertex distance from the barycenter
    // the same per element as one 128-byte record (one cache line): v0x, v0y,
    // v1x, v1y, v2x, v2y, bx, by, a2, r, the reciprocal squared lengths of the
    // edges v0->v1, v1->v2, v2->v0, then padding; kernels that gather an inner
    // element's data by index read it in 16-byte loads
    double *pk;                                // [K][16]
};

// Training domain of a learned cap network: an item goes to the network only
// when each squared vertex distance |v_a - x|^2 lies in [rlo, rhi] delta^2
// and each squared edge length |v_b - v_a|^2 in [elo, ehi] delta^2 (the
// shape and place of the triangle relative to the ball, whatever its
// rotation), tested in FP64 with every operation rounded on its own;
// otherwise it takes the exact caps.  Training sets the ranges to those of
// its samples; they are unbounded (infinite limits) for weights set from
// outside.
struct MlpDomain {
    double rlo, rhi, elo, ehi;
};

struct DeviceArena {
    std::vector<void *> ptrs;
    size_t bytes = 0;
    ~DeviceArena();
    int alloc(void **p, size_t n);
    template <class T> int get(T **p, size_t count) { return alloc((void **)p, count * sizeof(T)); }
};

struct nla_plan {
    int device = 0;
    int32_t K = 0, J = 0, n_free = 0;
    nla_problem prob{};
    RuleSet rules{};
    RuleSet *d_rules = nullptr;
    DeviceArena arena;         // plan-lifetime allocations
    // mesh
    double *xy = nullptr;
    int32_t *tri = nullptr;
    uint8_t *tin = nullptr, *nfree = nullptr;
    ElemSoA E{};
    double *xq = nullptr;      // [K][n_out][2]
    double *xq2 = nullptr;     // [K][n_out2][2] (second outer rule)
    uint8_t *pair_r2 = nullptr;// [n_pairs] 1: the pair takes the second outer rule
    // pairs
    int64_t n_pairs = 0;
    int64_t *pair_ptr = nullptr;
    int32_t *pair_kp = nullptr;
    int32_t *pair_k = nullptr;
    // processing order of the FP64 constant-kernel pair kernel (nullptr: canonical):
    // within each element the pairs that can have partial items first, then the
    // deep pairs (every item whole), each in canonical order
    int32_t *proc_p = nullptr;  // [n_pairs] canonical pair index of processing slot i
    int32_t *proc_kp = nullptr; // [n_pairs] k' of processing slot i
    int32_t *nband = nullptr;   // [K] pairs of k before its deep ones
    int32_t *korder = nullptr;  // [K] launch order of the pair kernels: outer elements by decreasing work
    int64_t n_deep = 0;         // deep pairs in all (with nband)
    // launch shape of the FP64 pair kernel, chosen at its first launch
    size_t pairs_lds = 0;       // dynamic LDS per workgroup (0: not chosen yet)
    // pattern of D
    int64_t nnz = 0;
    int64_t *rowptr = nullptr;
    int32_t *col = nullptr;
    int64_t *mirror = nullptr;  // index of (col,row) for every entry
    // segmented sum: upper-triangle entries and their contribution codes
    int64_t n_up = 0, n_codes = 0;
    int64_t *up_dst = nullptr;  // [n_up] entry index of the upper entry
    int64_t *up_ptr = nullptr;  // [n_up+1]
    int32_t *codes = nullptr;   // [n_codes] indices into the contribution array
    // column sets: for outer element k the sorted nodes C_k of all its inner
    // elements; the pair kernel reduces -Mxy into R_k[a][c] (3 x |C_k|)
    int64_t n_cols = 0;         // sum_k |C_k|
    int32_t max_cols = 0;       // max_k |C_k|
    int64_t *col_off = nullptr; // [K+1]
    int32_t *colset = nullptr;  // [n_cols] node ids
    int32_t *colent_ptr = nullptr; // [n_cols+1] per column slot: contributions (p_local << 2 | b), p ascending
    uint16_t *colent = nullptr;    // [3 n_pairs]
    int32_t *n2e_all_ptr = nullptr; // [J+1] node -> (3k+a) over all elements
    int32_t *n2e_all = nullptr;
    // transposed pair order: pairs (k, k') grouped by k', k ascending within
    int64_t *tptr = nullptr;    // [K+1]
    int32_t *tperm = nullptr;   // [n_pairs]
    // near-diagonal pairs (singular kernel): pairs sharing a vertex, their 6x6
    // merged blocks (upper triangle, 21 values) and codes of the upper entries
    int64_t n_near = 0;
    int64_t *near_pair = nullptr;   // [n_near] pair indices, ascending
    uint8_t *near_flag = nullptr;   // [n_pairs]
    int64_t n_ncodes = 0;
    int64_t *nup_ptr = nullptr;     // [n_up+1]
    int32_t *ncodes = nullptr;      // [n_ncodes] indices into the near-block array
    int64_t n_near_comp = 0;        // near pairs whose block is computed (the others mirror a partner)
    int64_t *near_comp = nullptr;   // [n_near_comp] their near indices
    int64_t *near_partner = nullptr;// [n_near] near index of the mirror partner, or -1
    void *near_blk = nullptr;       // [n_near][21]
    // contributions and values
    int64_t n_contrib = 0;      // 6P (Myy) + 6K (Mxx) + 6K (element blocks) + 3 n_cols (R) + 21 n_near
    void *contrib = nullptr;    // f64 or f32 [n_contrib]
    void *val = nullptr;        // [nnz]
    // A = D[free, free]
    int64_t nnz_free = 0;
    int32_t *free_nodes = nullptr;
    int32_t *node_to_free = nullptr;
    int64_t *a_rowptr = nullptr;
    int32_t *a_col = nullptr;
    int64_t *a_src = nullptr;
    void *a_val = nullptr;
    // load vector
    int32_t *n2e_ptr = nullptr; // [J+1] node -> (element*3+slot) of Omega elements
    int32_t *n2e = nullptr;
    double *Gk = nullptr;       // [K][3]
    double *b = nullptr;        // [n_free]
    // learned caps: routed items per outer element, their features and outputs
    const nla_mlp *mlp = nullptr;
    MlpDomain mlp_dom{};            // the network's training domain when the plan was made
    int64_t *route_off = nullptr;   // [K+1]
    uint8_t *route_mask = nullptr;  // [n_pairs] by processing slot: outer points routed to the network
    int64_t n_routed = 0;
    float *route_feat = nullptr;    // [n_routed][6]
    float *route_y = nullptr;       // [n_routed][3]
    // counters: whole, partial, empty, learned, subtriangles, caps
    unsigned long long *counters = nullptr;
    // phase timing: (NLA_NPHASE + 1) events per timed assembly
    int timing_slots = 0, timing_count = 0;
    std::vector<hipEvent_t> ev;
    hipEvent_t *cur_ev = nullptr;   // events of the assembly being timed, or null
    bool ran[8] = {};
    // second stream (default priority) on which the FP32 singular pairs overlap
    // the regular pairs, with its fork and join events; made at first use
    hipStream_t aux = nullptr;
    hipEvent_t fork = nullptr, join = nullptr;
    ~nla_plan()
    {
        for (auto &e : ev)
            if (e) (void)hipEventDestroy(e);
        if (fork) (void)hipEventDestroy(fork);
        if (join) (void)hipEventDestroy(join);
        if (aux) (void)hipStreamDestroy(aux);
    }
    bool assembled = false;
    bool counted = false;       // the item counters hold the first assembly's counts (geometry only)
    bool have_load = false;
    int val_dtype = NLA_DTYPE_F64;
};


// arguments of the FP32 pair kernel for one instance (plan)
struct PairArgs {
    const int64_t *pair_ptr;
    const int32_t *pair_kp;
    ElemSoA E;
    const double *xq;
    const RuleSet *R;
    double dd;
    float kc, ex;
    int ball, ncap, frac, max_cols;
    int bnd;                    // constant kernel, rule exact for quadratics: partial items by boundary moments
    const uint8_t *near_flag;
    const int64_t *col_off;
    const int32_t *colent_ptr;
    const uint16_t *colent;
    float *Rout, *Cyy, *Cxx;
    unsigned long long *counters;
    // learned caps: routed partial items take the network's cap moments
    double delta, band;
    const int64_t *route_off;   // [K+1] first routed item of each outer element
    uint8_t *route_mask;        // [n_pairs] by processing slot: routed outer points (the routing pass's)
    int64_t n_routed;
    const float *mlp_y;         // [n_routed][3] network outputs
    float mlp_k;                // kc delta^2 scale
    MlpDomain dom;              // the network's training domain, taken at plan creation
    // processing order (constant kernel): band pairs first, deep ones after
    const int32_t *proc_p, *proc_kp, *nband;
    const int32_t *korder;      // [K] launch order: outer elements by decreasing work
    float *Dk;                  // [K] the deep pairs' Myy factor of each element
};
PairArgs nla_pair_args(const nla_plan *P);

// Workgroups are dealt round-robin to the 8 XCDs, each with its own L2: the
// work index of workgroup b (of nb) such that each XCD takes one contiguous
// range, so neighbouring work items (sharing cache lines) meet in one L2.
__device__ __forceinline__ int64_t xcd_block(int64_t b, int64_t nb)
{
    const int64_t chunk = (nb + 7) / 8;
    return (b % 8) * chunk + b / 8;
}
inline int64_t xcd_grid(int64_t nb) { return (nb + 7) / 8 * 8; }

// A deep pair: every point of E_k within delta of every point of E_k' with
// room to spare.  The largest distance between two triangles is attained at a
// pair of vertices, so max |v - w| over the nine vertex pairs <= delta (1 - 1e-9)
// makes every item whole under the intersection, overlap and barycenter balls
// (outer points lie in E_k, b_k' in E_k'; the relative margin covers the
// rounding of these distances and of the outer points).  The squared distances
// are formed without contraction, and their maximum is the same set's for
// (k, k') and (k', k), so the test gives the same bits both ways: each
// element's deep partners are the deep pairs it owns.
__device__ __forceinline__ bool pair_deep(const ElemSoA &E, int k, int kp, double delta)
{
#pragma clang fp contract(off)
    const double vx[3] = {E.vx0[k], E.vx1[k], E.vx2[k]}, vy[3] = {E.vy0[k], E.vy1[k], E.vy2[k]};
    const double wx[3] = {E.vx0[kp], E.vx1[kp], E.vx2[kp]}, wy[3] = {E.vy0[kp], E.vy1[kp], E.vy2[kp]};
    double m = 0.0;
#pragma unroll
    for (int i = 0; i < 3; i++)
#pragma unroll
        for (int j = 0; j < 3; j++) {
            const double dx = vx[i] - wx[j], dy = vy[i] - wy[j];
            const double d2 = dx * dx + dy * dy;
            m = d2 > m ? d2 : m;
        }
    const double lim = delta * (1.0 - 1e-9);
    return m <= lim * lim;
}

// learned cap corrector (nla_mlp.hip)
struct nla_mlp;
int nla_mlp_infer_launch(const nla_mlp *M, const float *feat, int64_t n, float *out, hipStream_t s);
float nla_mlp_scale(const nla_mlp *M);
MlpDomain nla_mlp_domain_of(const nla_mlp *M);
int nla_build_routes(nla_plan *P, hipStream_t s);

// translation-unit entry points
int nla_build_pairs(nla_plan *P, hipStream_t s);
int nla_build_pattern(nla_plan *P, hipStream_t s);
int nla_numeric(nla_plan *P, const double *f_outer, const double *g_node, hipStream_t s);
int nla_numeric_fp32(nla_plan *P, hipStream_t s, void (*mark)(nla_plan *, int, hipStream_t));
int nla_cg_run(const nla_plan *P, const double *b, double *u, double rtol, int32_t maxit, int32_t *iters,
               double *relres, hipStream_t s);
