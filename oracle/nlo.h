/*
 * nlo.h - plain FP64 CPU oracle for the P1 nonlocal stiffness assembly of
 * D'Elia, Gunzburger, Vollmann, "A cookbook for finite element methods for
 * nonlocal problems, including quadrature rules and approximate Euclidean
 * balls" (arXiv:2005.10775).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load this library.  It is slow on
 * purpose: an all-pairs loop, no binning, literal quadrature.
 *
 * Parity-pinned functions are listed in the file that implements them.
 */
#ifndef NLO_H
#define NLO_H
#include <stdint.h>

typedef struct {
    int32_t nv, nt;
    const double *xy;            /* [nv][2] */
    const int32_t *tri;          /* [nt][3] counter-clockwise */
    const uint8_t *tri_in_omega; /* [nt] */
    const uint8_t *node_free;    /* [nv] */
} nlo_mesh;

typedef struct {
    double delta;
    int32_t kernel;              /* 0: psi = kc ; 1: psi = kc |x-y|^-(2+2 ks) */
    double kc, ks;
    int32_t ball;                /* 0: barycenter ; 1: intersection (retriangulated) ball ;
                                  * 2: overlap ; 3: shifted (intersection ball about b_k) ;
                                  * 4: barycenter with the outer integral over E_k n B(b_k') */
    int32_t cap_mode;            /* 0: caps by cap_edges equal arcs ; 1: exact caps, 1-pt centroid rule ;
                                  * 2: exact caps integrated in closed form (constant kernel) */
    int32_t cap_edges;           /* 0 = inscribed polygon only */
    int32_t n_out; const double *out_lam; const double *out_w;
    int32_t n_in;  const double *in_lam;  const double *in_w;
    int32_t n_out2; const double *out2_lam; const double *out2_w; double switch_dist;
    int32_t duffy_n; const double *gl_x; const double *gl_w;   /* Gauss-Legendre on [0,1] */
    int32_t skip_ixi;
    /* learned caps (constant kernel, intersection ball): partial items with
     * min_a | |v_a - x| - delta | >= band delta take the polygon plus the
     * network's cap moments; the others keep the arc-subdivided caps */
    int32_t learned; double band; const double *mlp_w; double mlp_scale;
    /* the network's training domain {rlo, rhi, elo, ehi}, or NULL
     * (unbounded): a routed item outside it keeps the arc-subdivided caps */
    const double *mlp_domain;
} nlo_problem;

#define NLO_MLP_HIDDEN 128
#define NLO_MLP_NW (128 * 6 + 128 + 128 * 128 + 128 + 3 * 128 + 3)
#define NLO_MAXCAP 256
#define NLO_MAXSUB (4 + 3 * NLO_MAXCAP + 8)

typedef struct nlo_result nlo_result;

#ifdef __cplusplus
extern "C" {
#endif
int nlo_pairs_of(const nlo_mesh *m, const nlo_problem *p, int32_t k, int32_t *kp, int32_t cap);
int nlo_pair_block(const nlo_mesh *m, const nlo_problem *p, int32_t k, int32_t kp,
                   double mxy[9], double myy[9], double s0q[64], double blk[36]);
int nlo_region(const nlo_problem *p, const double x[2], const double tri[6],
               double *sub, int32_t cap, double *cap_pts, double *cap_w, int32_t *n_cap);
int nlo_inner_sums(const nlo_problem *p, const double x[2], const double tri[6],
                   double s0[1], double s1[3], double s2[9]);
nlo_result *nlo_assemble(const nlo_mesh *m, const nlo_problem *p, int32_t nthreads);
void nlo_result_sizes(const nlo_result *r, int64_t *n_pairs, int64_t *nnz, int32_t *status);
void nlo_result_copy(const nlo_result *r, int64_t *pair_ptr, int32_t *pair_kp,
                     int64_t *rowptr, int32_t *col, double *val);
void nlo_result_free(nlo_result *r);
int nlo_row(const nlo_mesh *m, const nlo_problem *p, int32_t j, int32_t *cols, double *vals, int32_t cap);
void nlo_load(const nlo_mesh *m, const nlo_problem *p, const double *f_outer, double *G);
void nlo_outer_points(const nlo_mesh *m, const nlo_problem *p, double *xq);
int64_t nlo_blocks_range(const nlo_mesh *m, const nlo_problem *p, int32_t k0, int32_t k1, int32_t nthreads,
                         double *checksum);
double nlo_gelu(double z);
void nlo_mlp_forward(const double *w, const double *feat, int64_t n, double *out);
void nlo_mlp_backward(const double *w, const double *feat, const double *dout, int64_t n, double *dw);
int nlo_cap_moments(const nlo_problem *p, const double x[2], const double V[6], double m[3]);
int nlo_routed(double delta, double band, const double x[2], const double V[6]);
int nlo_in_domain(const double *dom, const double x[2], const double V[6], double delta);
int nlo_learned_caps(const nlo_problem *p, const double x[2], const double V[6], double s0[1], double s1[3],
                     double s2[9]);
void nlo_mlp_features(const double x[2], const double V[6], double delta, double f[6]);
int nlo_cap_candidate(const double u[10], double L, double jitter, double band, int32_t cap_edges,
                      double verts[6], double feat[6], double label[3]);
int64_t nlo_flops_census(const nlo_mesh *m, const nlo_problem *p, int32_t k0, int32_t k1, int64_t out[8]);
#ifdef __cplusplus
}
#endif
#endif
