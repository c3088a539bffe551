/*
 * nlasm.h - C ABI of libnlasm.so, the MI355X (gfx950) assembler for the P1
 * finite element discretisation of the 2D nonlocal diffusion problem of
 * D'Elia, Gunzburger, Vollmann, "A cookbook for finite element methods for
 * nonlocal problems, including quadrature rules and approximate Euclidean
 * balls" (arXiv:2005.10775).
 *
 * Problem (Sec. 2.1, Eqs. (prob), (oper), (inter)): -L u = f on Omega,
 * u = g on the interaction layer Omega_I, with
 *     L u(x) = 2 int (u(y) - u(x)) gamma(x,y) dy,
 *     gamma(x,y) = psi(x,y) chi_{B_delta(x)}(y).
 * The library assembles the full matrix D of the D-form (Eq. (bform0)) over
 * every ordered pair of elements (k, k') of Omega u Omega_I (Eq. (bformhj)),
 * with the Euclidean ball replaced by an approximate ball B_{delta,h}(x)
 * (Sec. 4: the barycenter ball of Eq. (baryball), or the retriangulated
 * intersection ball of Secs. 4.2.1-4.2.2 with caps filled by triangles over
 * equal arcs) and both integrals replaced by quadrature (Eqs. (cqr1),
 * (bformjqqh)).  The stiffness matrix is A = D[free, free] and the load
 * vector b = G - D[free, Dirichlet] g, with g interpolated at the nodes of
 * Omega_I (Eqs. (appr), (intcon), (lfunchj); the (A-B-C) recipe of Sec. 7.2).
 *
 * Conventions for every call:
 *  - Status: 0 (NLA_OK) or a negative NLA_E_* code; nla_last_error() returns
 *    a message for the calling thread's last failure.  No C++ exception
 *    crosses this boundary.
 *  - Memory: arguments documented "host" are read during the call only and
 *    may be freed afterwards (create calls copy them).  Arguments documented
 *    "device" are caller-owned device allocations on the plan's GPU.  Views
 *    returned by *_view calls are owned by the plan and stay valid until the
 *    next nla_assemble on that plan or nla_plan_destroy.
 *  - Streams: every call that touches the GPU is ordered on the HIP stream
 *    passed in (hipStream_t cast to void*; NULL = default stream).  A plan
 *    must not be used from two threads at once.
 *  - Determinism: pair lists and CSR patterns are bitwise reproducible, and
 *    all reductions run in a fixed order, so repeated calls give bitwise
 *    identical values; D is bitwise symmetric.
 *  - Validation: all mesh and problem checks run on the host before any GPU
 *    work, so invalid input is reported without touching the device.
 */
#ifndef NLASM_H
#define NLASM_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    NLA_OK = 0,
    NLA_E_INVALID = -1,        /* bad argument (null pointer, out-of-range value) */
    NLA_E_MESH = -2,           /* mesh violates the rules of Sec. 3.1 (orientation, labels, indices) */
    NLA_E_NOMEM = -3,          /* device allocation failed or exceeds NLA_MAX_DEVICE_BYTES */
    NLA_E_DEVICE = -4,         /* a HIP runtime call failed */
    NLA_E_UNSUPPORTED = -5,    /* valid but outside what the kernels handle (see each field) */
    NLA_E_NOT_CONVERGED = -6,  /* CG reached maxit before rtol */
    NLA_E_STATE = -7           /* call out of order (e.g. a view before nla_assemble) */
};

enum { NLA_KERNEL_CONSTANT = 0, NLA_KERNEL_FRACTIONAL = 1 };
/* balls (Sec. 4): barycenter (Eq. (baryball)); intersection ball, retriangulated
 * (Sec. 4.2); overlap (Eq. (overlap): every element meeting B_delta(x), whole);
 * shifted (Sec. 4.3: the intersection ball about b_k for every point of E_k);
 * barycenter ball with the outer integral restricted to its support
 * E_k n B_delta(b_k') (Sec. 6, case 2), approximated by the intersection-ball
 * region of that set.  The last three: constant kernel, NLA_FP64. */
enum { NLA_BALL_BARYCENTER = 0, NLA_BALL_RETRI = 1, NLA_BALL_OVERLAP = 2, NLA_BALL_SHIFTED = 3,
       NLA_BALL_BARYSUPPORT = 4 };
enum { NLA_FP64 = 0, NLA_FP32 = 1, NLA_FP32_LEARNED = 2 };
enum { NLA_DTYPE_F64 = 0, NLA_DTYPE_F32 = 1 };
enum { NLA_SKIP_IXI = 1u };     /* flags: drop Omega_I x Omega_I pairs (A and b unchanged) */

/* Mesh of Omega u Omega_I (Sec. 3.1): matching triangulations of the two
 * parts, all host arrays. */
typedef struct {
    int32_t n_vertices;          /* J */
    int32_t n_triangles;         /* K */
    const double *xy;            /* [J][2] vertex coordinates */
    const int32_t *tri;          /* [K][3] vertex indices, counter-clockwise */
    const uint8_t *tri_in_omega; /* [K] 1 = element of Omega, 0 = element of Omega_I */
    const uint8_t *node_free;    /* [J] 1 = node in the open Omega, 0 = node of Omega_I
                                    (boundary nodes of Omega count as Omega_I, Sec. 3.1) */
} nla_mesh;

/* Triangle quadrature rule in barycentric form (host arrays).  Weights sum
 * to 1/2, the area of the reference triangle (as in Sec. 6's 7-point rule). */
typedef struct {
    int32_t n;                   /* points, 1..16 for outer rules, 1..32 for inner rules */
    const double *lambda;        /* [n][3] barycentric coordinates */
    const double *w;             /* [n] weights */
} nla_rule;

typedef struct {
    double delta;                /* horizon, > 0 */
    int32_t kernel;              /* NLA_KERNEL_CONSTANT: psi = kernel_c;
                                    NLA_KERNEL_FRACTIONAL: psi = kernel_c |x-y|^-(2+2 kernel_s)
                                    (truncated to the approximate ball) */
    double kernel_c, kernel_s;
    nla_rule outer;              /* outer rule on every E_k (Sec. 6) */
    nla_rule inner;              /* inner rule on every subtriangle (Sec. 5.3) */
    int32_t duffy_n;             /* fractional kernel: Gauss-Legendre order on [0,1] for
                                    element pairs sharing a vertex (0 = not used) */
    const double *duffy_x;       /* [duffy_n] host, nodes on [0,1] */
    const double *duffy_w;       /* [duffy_n] host, weights summing to 1 */
    int32_t ball;                /* NLA_BALL_* */
    int32_t cap_edges;           /* retri, shifted, barysupport: equal arcs per cap, 0 (= inscribed
                                    polygon) or 2..64 */
    int32_t precision;           /* NLA_FP64 | NLA_FP32 (compensated) | NLA_FP32_LEARNED */
    const void *mlp;             /* NLA_FP32_LEARNED: an nla_mlp* ; else NULL */
    double fallback_band;        /* learned caps: exact path when min_a | |v_a - x| - delta | <
                                    fallback_band * delta, or outside the network's training
                                    domain (nla_mlp_set_domain) */
    uint32_t flags;              /* NLA_SKIP_IXI */
    nla_rule outer2;             /* optional second outer rule (n = 0: none), used for the pairs
                                    with |b_k - b_k'| < switch_dist (Sec. 8: a lower-order rule
                                    for pairs well inside each other's ball), decided in FP64 with
                                    every operation rounded on its own */
    double switch_dist;
    int32_t cap_mode;            /* retri caps: NLA_CAPS_ARCS (cap_edges equal arcs, Sec. 4.2.2),
                                    NLA_CAPS_CENTROID (exact caps, one-point rule at the cap
                                    centroid with the cap area as weight, Sec. 5.2) or
                                    NLA_CAPS_ANALYTIC (exact caps integrated in closed form from the
                                    circular segment's area and first and second moments: the exact
                                    ball, no geometric error, the route Sec. 9 points to); the last
                                    two: FP64, constant kernel, inner rule exact for quadratics */
} nla_problem;

enum { NLA_CAPS_ARCS = 0, NLA_CAPS_CENTROID = 1, NLA_CAPS_ANALYTIC = 2 };

typedef struct nla_plan nla_plan;

typedef struct {
    int64_t n_pairs;             /* interacting ordered element pairs */
    int64_t nnz_full;            /* nonzeros of D (J x J) */
    int64_t nnz_free;            /* nonzeros of A = D[free, free] */
    int32_t n_free;              /* J_Omega */
    int32_t n_outer;             /* outer points per element */
    int64_t n_codes;             /* contributions summed by the segmented sum */
    int64_t n_near;              /* vertex-sharing pairs handled by the singular rule */
    int64_t items[4];            /* after nla_assemble: (k,q,k') items whole, partial, empty, learned */
    int64_t subtriangles;        /* after nla_assemble: polygon + cap triangles integrated */
    int64_t caps;                /* after nla_assemble: caps filled with triangles */
    int64_t n_deep;              /* pairs whose items are all whole, summed from element areas
                                    instead of item by item (constant kernel; 0 otherwise) */
} nla_info;

/* phases timed by nla_timings, in launch order (MLP: routing pass and network
 * inference of the learned caps) */
enum { NLA_PHASE_MLP = 0, NLA_PHASE_PAIRS = 1, NLA_PHASE_NEAR = 2, NLA_PHASE_SEGSUM = 3, NLA_PHASE_EXTRACT = 4,
       NLA_PHASE_LOAD = 5, NLA_NPHASE = 6 };

const char *nla_last_error(void);

/* Builds the plan: element data, the canonical pair list (k ascending, k'
 * ascending within k) of pairs with at least one outer point x_{k,q} whose
 * approximate ball reaches E_k' (Sec. 7.1 tasks 1-4; barycenter ball:
 * |x - b_k'| <= delta; retri and overlap: the closed ball meets E_k'; shifted:
 * the closed ball about b_k meets E_k'; barysupport: the closed ball about b_k'
 * meets E_k), and the CSR pattern of D.  The balls that cut elements (retri,
 * shifted, barysupport) need every element's inradius < delta/2 (the fractional
 * kernel: every diameter <= delta), so that no ball lies inside an element and
 * every cap spans less than a half circle; NLA_E_UNSUPPORTED otherwise.
 * Shifted needs an inner rule exact for quadratics, barysupport an outer rule
 * exact for quadratics (their regions are integrated through their moments).
 * *out receives a new plan; destroy it with nla_plan_destroy. */
int nla_plan_create(const nla_mesh *mesh, const nla_problem *prob, void *stream, nla_plan **out);
int nla_plan_info(const nla_plan *plan, nla_info *info);

/* Device views of the pair list: pair_ptr [K+1] (int64), pair_kp [n_pairs] (int32). */
int nla_pairs_view(const nla_plan *plan, const int64_t **pair_ptr, const int32_t **pair_kp);

/* Writes the outer quadrature points x_{k,q} = l0 v0 + l1 v1 + l2 v2 to
 * xq [K][n_outer][2] (device, f64), so a caller can sample f there. */
int nla_outer_points(const nla_plan *plan, double *xq, void *stream);

/* Numeric assembly: D (CSR), A = D[free,free] and b = G - D[free,Dir] g.
 * f_outer [K][n_outer] device f64: f at the outer points (rows of Omega_I
 * elements are ignored).  g_node [J] device f64: g at the nodes (read at
 * Omega_I nodes).  Either may be NULL to skip the load vector. */
int nla_assemble(nla_plan *plan, const double *f_outer, const double *g_node, void *stream);

/* which = 0: full D (J x J); which = 1: A (n_free x n_free, rows/cols in
 * increasing node order of the free nodes).  val_dtype = NLA_DTYPE_F64 or
 * NLA_DTYPE_F32 (FP32 modes).  All pointers are device views. */
int nla_csr_view(const nla_plan *plan, int32_t which, const int64_t **rowptr, const int32_t **col,
                 const void **val, int32_t *val_dtype);

/* b [n_free] (device f64) after nla_assemble with f_outer and g_node. */
int nla_load_view(const nla_plan *plan, const double **b);

/* Free-node indices [n_free] (device int32, increasing). */
int nla_free_nodes_view(const nla_plan *plan, const int32_t **free_nodes);

/* Intermediate blocks (test hook), device views valid as for the CSR views:
 *   myy  [n_pairs][6]  Myy of each pair (b<=b': 00,01,02,11,12,22); the FP64
 *                      assembly of the intersection and overlap balls keeps no
 *                      record for pairs whose items are all whole (it adds
 *                      their Myy per element), and this call forms those
 *                      records in place, after a device synchronization;
 *   mxx  [K][6]        Mxx of each outer element (same order);
 *   elem [K][6]        element block E(k) = Mxx(k) + sum_k' Myy(k', k);
 *   rows               for outer element k, the row block R_k [3][|C_k|] at
 *                      offset 3*col_off[k]: R_k[a][c] = -sum over pairs (k,k') and
 *                      slots b with node(k',b) = colset[col_off[k]+c] of Mxy_ab;
 *   col_off [K+1] (int64) and colset [sum |C_k|] (int32, nodes ascending per k).
 * dtype as in nla_csr_view. */
int nla_blocks_view(const nla_plan *plan, const void **myy, const void **mxx, const void **elem, const void **rows,
                    const int64_t **col_off, const int32_t **colset, int32_t *dtype);

/* Vertex-sharing pairs under the singular kernel (test hook): n_near, their
 * pair indices near_pair [n_near] (int64, ascending) and merged 6x6 blocks
 * blocks [n_near][21] (upper triangle, row-major over the slots a0,a1,a2,b0,b1,b2;
 * a slot of E_k' whose node is also a node of E_k is merged into E_k's slot and
 * holds zeros), dtype as in nla_csr_view; device views.  The joint integrand
 * of such a pair is symmetric under x <-> y, so a pair (k, k') with k > k'
 * whose mirror (k', k) interacts is not integrated: the assembly reads the
 * mirror's block with the nodes relabelled.  This call writes those relabelled
 * blocks into the view (it synchronises the device). */
int nla_near_view(const nla_plan *plan, int64_t *n_near, const int64_t **near_pair, const void **blocks,
                  int32_t *dtype);

/* Conjugate gradients on A (after nla_assemble): b [n_free] device, u [n_free]
 * device (in: x0, out: solution), FP64 residuals and fixed-order dot
 * products.  Returns NLA_E_NOT_CONVERGED (with u holding the last iterate)
 * if ||r|| > rtol ||b|| after maxit iterations. */
int nla_cg(const nla_plan *plan, const double *b, double *u, double rtol, int32_t maxit,
           int32_t *iters, double *relres, void *stream);

/* nla_cg for callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * iteration and kernels, bitwise the same results, with its scratch (r, p, Ap
 * and the dot products' partial sums) in a device array of the library that
 * every device it runs on holds from the module's load until the process ends
 * (24 MiB), instead of memory allocated per call.  Calls no hipMalloc or
 * hipFree.  n_free at most NLA_CG_NOALLOC_MAX_FREE, else NLA_E_INVALID; the
 * plan's device must be current (NLA_E_DEVICE otherwise).  Every call on a
 * device shares that device's scratch, so calls that overlap on one device
 * (two streams, two threads) race: serialise them.  No scratch value is read
 * before the call writes it.  Other arguments and errors as nla_cg. */
#define NLA_CG_NOALLOC_MAX_FREE 1048576
int nla_cg_noalloc(const nla_plan *plan, const double *b, double *u, double rtol, int32_t maxit,
                   int32_t *iters, double *relres, void *stream);

/* Timing: nla_set_timing(plan, n) with n > 0 makes the next n calls of
 * nla_assemble record HIP events on their stream around each phase (n = 0
 * turns it off).  nla_timings waits for the last recorded event and writes
 * the mean elapsed milliseconds per phase over those calls (ms[NLA_NPHASE],
 * host; 0 for phases that did not run) and how many calls were timed. */
int nla_set_timing(nla_plan *plan, int32_t n);
int nla_timings(const nla_plan *plan, double *ms, int32_t *count);

void nla_plan_destroy(nla_plan *plan);

/* ------------------------------------------------------------------ batches
 * Many independent problems (meshes, horizons, kernels, balls) assembled
 * together.  All instances must use NLA_FP32, outer rules of at most 8
 * points and cap counts that are 0 or powers of two (NLA_E_UNSUPPORTED
 * otherwise).  mode 1 replays a hipGraph, captured once on a private stream
 * (ordered after and before the caller's stream with events), of either one
 * persistent launch of the pair kernel (a fixed grid taking (instance, outer
 * element) work items, heaviest first, from a device cursor) followed by
 * instance-batched near-pair (on a second stream beside the pair kernel),
 * element-block, segmented-sum, extraction and load kernels, or (chunk 0,
 * when the autotuner times it faster) every instance's own launches; mode 0
 * assembles the instances one after the other with their own launches.  All
 * give bitwise identical values. */
typedef struct nla_batch nla_batch;
typedef struct {
    int32_t n;                   /* instances */
    int64_t total_pairs, total_elements, total_near;   /* total_near: singular-pair blocks integrated */
    int32_t chunk;               /* work items taken per cursor fetch (0: the graph of each instance's launches) */
    int32_t grid;                /* wavefronts of the persistent launch */
} nla_batch_summary;

/* meshes [n], probs [n] (host); the plans are owned by the batch. */
int nla_batch_create(int32_t n, const nla_mesh *meshes, const nla_problem *probs, void *stream, nla_batch **out);
/* f_outer, g_node: host arrays of n device pointers (as in nla_assemble), or both NULL. */
int nla_batch_assemble(nla_batch *batch, int32_t mode, const double *const *f_outer, const double *const *g_node,
                       void *stream);
/* the plan of instance i (owned by the batch; use the nla_*_view calls on it) */
int nla_batch_plan(const nla_batch *batch, int32_t i, nla_plan **plan);
int nla_batch_info(const nla_batch *batch, nla_batch_summary *info);
/* picks (chunk, grid) by timing graph replays of every candidate on this
 * batch; cache_path (may be NULL) is a text file of earlier choices keyed by
 * the batch shape, read first and appended to. */
int nla_batch_autotune(nla_batch *batch, const char *cache_path, void *stream);
void nla_batch_destroy(nla_batch *batch);

/* ------------------------------------------------------------------------
 * Learned cap corrector.  The caps that the inscribed polygon of the
 * intersection ball leaves out (Sec. 4.2.1) are filled with triangles over
 * equal arcs in Sec. 4.2.2; for partial items far from tangency
 * (min_a | |v_a - x| - delta | >= fallback_band delta, FP64 test) the
 * NLA_FP32_LEARNED path replaces them by a network that predicts
 *     m_b = (1/delta^2) int_{caps in E_k'} phi_b dy,   b = 0, 1, 2,
 * from the vertices of E_k' (mesh order) in a frame centred at x and rotated
 * so that the triangle's centroid lies on the positive first axis (the cap
 * integrals are invariant under it), shifted by the horizon and magnified by
 * 8 (the element size of the h = delta/8 family):
 *     f_a = 8 (R(-phi) (v_a - x)/delta - (1, 0)),  phi = angle of the centroid;
 * the item then adds S0 += kc delta^2 sum m,
 * S1_b += kc delta^2 m_b and the one-point centroid closure of Sec. 5.2,
 * S2_bc += kc delta^2 m_b m_c / sum m (network outputs clamped at 0).
 * Network: 6 -> 128 -> 128 -> 3 with g(z) = z/2 (1 + tanh(sqrt(2/pi)(z +
 * 0.044715 z^3))); weights in one flat float array W1[128][6], b1[128],
 * W2[128][128], b2[128], W3[3][128], b3[3] (row = output unit), 17795 floats;
 * W2 and W3 are used rounded to bfloat16 (matrix cores, FP32 accumulation),
 * W1 and the biases in FP32.  Outputs are in units of `scale` (m = scale *
 * output).  An nla_mlp must outlive every plan that uses it; calls are
 * stream-ordered on the caller's stream, and an nla_mlp is not thread-safe.
 *
 * Training domain (out-of-distribution fallback): an item goes to the network
 * only when it is also inside the network's training domain, 4 doubles
 * dom = {rlo, rhi, elo, ehi}: every squared vertex distance |v_a - x|^2 within
 * [rlo delta^2, rhi delta^2] and every squared edge length |v_b - v_a|^2
 * within [elo delta^2, ehi delta^2] (the triangle's size and place relative
 * to the ball, whatever its rotation), tested in FP64 with every product and
 * sum rounded on its own (the limits times delta^2 included).  Other items
 * take the exact caps.  nla_mlp_train sets the domain to the range of its
 * samples, read back from their inputs (|v_a|^2 = (f_a0/8 + 1)^2 +
 * (f_a1/8)^2, |v_b - v_a|^2 = |f_b - f_a|^2 / 64 with delta = 1), joined with
 * earlier training calls' ranges; nla_mlp_create and nla_mlp_set_weights
 * leave it unbounded.  A plan takes the network's domain when it is created.
 * ------------------------------------------------------------------------ */
#define NLA_MLP_WEIGHTS 17795
typedef struct nla_mlp nla_mlp;

/* A network with seeded uniform initial weights (bound sqrt(6/fan_in), W3
 * sqrt(1/fan_in), zero biases) and scale 0 (set by the first training call
 * to the root mean square of its labels). */
int nla_mlp_create(uint64_t seed, nla_mlp **out);
/* Host weights in the flat layout (copied), output scale > 0; resets Adam. */
int nla_mlp_set_weights(nla_mlp *mlp, const float *w, float scale);
/* Master FP32 weights to host w[NLA_MLP_WEIGHTS], and the scale. */
int nla_mlp_get_weights(const nla_mlp *mlp, float *w, float *scale);
/* Training candidates first .. first+n_cand-1 in units of delta around x = 0,
 * each from ten SplitMix64 outputs 10c .. 10c+9 of `seed`: a right triangle of
 * legs L (= h/delta) from one of the four halves of a grid cell, its cell
 * centre at distance 1 + (2u1 - 1) sqrt(2) L in direction 2 pi u2, each vertex
 * coordinate jittered by jitter L (2u - 1) (u3..u8), vertex order rotated by
 * floor(3 u9).  Kept when the ball cuts the triangle (at least one cap) and
 * every vertex is at least `band` from the circle.  Writes the kept samples in
 * candidate order to feat (device, [n_cand][6] floats of room: the network
 * input above, with x = 0 and delta = 1) and label
 * (device, [n_cand][3]: cap moments from the FP64 arc subdivision with
 * cap_edges arcs) and their number to *n_valid (host; synchronises). */
int nla_mlp_samples(int64_t n_cand, uint64_t seed, int64_t first, double L, double jitter, double band,
                    int32_t cap_edges, float *feat, float *label, int64_t *n_valid, void *stream);
/* Adam (beta 0.9, 0.999, eps 1e-8) on the mean squared error of the outputs
 * against label/scale, cosine learning-rate decay from lr over the call,
 * `epochs` passes over n device samples in seeded affine-permutation order,
 * batch a multiple of 64 with n >= batch.  loss_log (host, may be NULL)
 * receives the mean loss of each epoch.  Records the samples' range as the
 * training domain (see above).  Synchronises once per epoch. */
int nla_mlp_train(nla_mlp *mlp, const float *feat, const float *label, int64_t n, int32_t epochs, int32_t batch,
                  float lr, uint64_t seed, float *loss_log, void *stream);
/* Network outputs (before scale) of n device samples into out [n][3]. */
int nla_mlp_forward(const nla_mlp *mlp, const float *feat, int64_t n, float *out, void *stream);
/* Gradient of sum_i sum_o dout[i][o] y[i][o] with respect to every weight
 * (device dw[NLA_MLP_WEIGHTS], flat layout), on the weights as used. */
int nla_mlp_backward(nla_mlp *mlp, const float *feat, const float *dout, int64_t n, float *dw, void *stream);
/* The training domain (host dom[4], layout above).  set: dom = NULL makes it
 * unbounded; NLA_E_INVALID for a NaN limit or lo > hi.  Plans made earlier
 * keep the domain they took. */
int nla_mlp_set_domain(nla_mlp *mlp, const double *dom);
int nla_mlp_get_domain(const nla_mlp *mlp, double *dom);
/* Checkpoint (weights, scale, Adam state, training domain) to / from a file;
 * a checkpoint written without a domain loads with an unbounded one. */
int nla_mlp_save(const nla_mlp *mlp, const char *path);
int nla_mlp_load(const char *path, nla_mlp **out);
void nla_mlp_destroy(nla_mlp *mlp);

#ifdef __cplusplus
}
#endif
#endif
