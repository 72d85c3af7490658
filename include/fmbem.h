/*
 * fmbem: fast-multipole Nystrom operator and BEM solver for 3-D Helmholtz
 * scattering on one gfx950 GPU.  C ABI.
 *
 * The operator follows the electric field integral equation of the paper
 * (Sec. 2.1, eq. 2.5) discretised by the Nystrom rule (eq. 2.8) at the nodes
 * of a planar triangle mesh.  For one wavenumber k the library computes, for
 * complex 3-vector densities a and b given at the n nodes,
 *
 *   y_alpha = sum_{beta : t(beta) != t(alpha)} w_beta [ n_beta (grad'g . a_beta)
 *               - (n_beta . grad'g) a_beta - grad'g (n_beta . a_beta) + g b_beta ]
 *           + sum over the nodes beta of alpha's own triangle of the
 *             analytically integrated self-triangle blocks (Appendix B),
 *
 * g = exp(i k R)/(4 pi R) (eq. 2.4), grad'g its gradient at the source node
 * s_beta, R = |s_beta - s_alpha|, t(.) the triangle of a node.  The far part
 * of the sum uses the fast multipole method of Sec. 2.2 (expansions of
 * eqs. 2.14-2.17, collect / upward / downward / distribute steps of eqs.
 * 2.18-2.23 on the octree of Appendix C); near pairs are summed directly.
 *
 * Conventions for every entry point:
 *  - every call returns an int status: FMB_OK (0) or one of the codes below;
 *    on error fmb_last_error() returns a thread-local message.  Nothing is
 *    thrown across the ABI.
 *  - "host" pointers are CPU memory read during the call only; "device"
 *    pointers are GPU memory owned by the caller.  Complex arrays are
 *    interleaved (re, im) pairs: c128 = two doubles, c64 = two floats.
 *  - `stream` is a hipStream_t (NULL = the null stream).  Matvec work is
 *    enqueued on it asynchronously; plan and solve calls synchronise it.
 *  - a plan owns its device workspace: at most one matvec per plan may be in
 *    flight at a time.  Input and output buffers must not alias.
 */
#ifndef FMBEM_H
#define FMBEM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    FMB_OK = 0,
    FMB_EINVAL = 1,      /* bad argument (sizes, non-finite input, bad normals, ...) */
    FMB_ENOMEM = 2,      /* device allocation failed */
    FMB_EDEVICE = 3,     /* a HIP runtime call failed */
    FMB_ENOCONV = 4,     /* iterative solve hit its iteration limit */
    FMB_EBREAKDOWN = 5,  /* solver breakdown it could not recover from */
    FMB_ENONFINITE = 6,  /* NaN/Inf met in a solve */
    FMB_ENOTIMPL = 7     /* entry point present, feature not implemented */
};

enum { FMB_FP64 = 0, FMB_FP32 = 1 };
enum { FMB_CORR_NONE = 0, FMB_CORR_MEAN = 1, FMB_CORR_LINEAR = 2 };

typedef struct fmb_plan_s *fmb_plan_t;
typedef struct fmb_problem_s *fmb_problem_t;

typedef struct {
    int32_t depth;              /* octree depth below the root cube, 1..10 (0: pick one)     */
    int32_t precision;          /* FMB_FP64 or FMB_FP32 (expansions, translations, near sum)  */
    int32_t nrhs_max;           /* largest nrhs a matvec on this plan will pass (>= 1)       */
    int32_t corr_mode;          /* FMB_CORR_*: how the self-triangle integrals are shared     */
    const int32_t *point_tri;   /* host i32[n]: triangle of each node (NULL: own triangle)    */
    const double *tri_vertices; /* host f64[ntri][3][3]: triangle corners (corr_mode > 0)     */
    int64_t ntri;               /* number of triangles                                        */
    int32_t leaf_target;        /* depth 0 only: aim for about this many nodes per leaf (0=32)*/
    int32_t translate_mode;     /* FP32 plans: FMB_TRANSLATE_FP32 (default) or FMB_TRANSLATE_BF16X3 */
    int32_t reserved0;
    double tol;                 /* order <= 0 only: target relative accuracy (0: 1e-6 FP64, 1e-4 FP32) */
    double far_cutoff;          /* lossy k: drop interactions damped below this factor (0: default) */
} fmb_plan_opts;

/*
 * Translation arithmetic of FP32 plans.  FMB_TRANSLATE_BF16X3 splits operator
 * and coefficients into BF16 high and low parts and forms hi*hi + hi*lo +
 * lo*hi on the BF16 matrix cores with FP32 accumulation (about 1e-5 relative
 * per product); it applies to orders p <= 9 and falls back to FP32 otherwise.
 */
enum { FMB_TRANSLATE_DEFAULT = 0, FMB_TRANSLATE_FP32 = 1, FMB_TRANSLATE_BF16X3 = 2 };

typedef struct {
    int32_t depth;
    int32_t order;              /* p: expansions keep degrees n <= p-1 (eq. 2.17 truncation) */
    int32_t precision;
    int32_t nrhs_max;
    int64_t n;
    int64_t nbox[16];           /* boxes per level 0..depth                                   */
    int64_t m2l_pairs[16];      /* far-field (S|R) pairs per level                             */
    int64_t p2p_pairs;          /* near (target, source) pairs incl. excluded same-triangle  */
    int64_t corr_blocks;        /* self-triangle blocks                                       */
    int64_t device_bytes;       /* device memory the plan holds                               */
    int32_t order_level[16];    /* truncation order of each level (0: no far field there)      */
    int32_t far_lmin;           /* first level with far-field translations (depth+1: none)    */
    int32_t reserved;
} fmb_plan_info;

/* Fill opts with defaults: depth 0, FP64, nrhs_max 1, LINEAR corrections. */
int fmb_plan_opts_default(fmb_plan_opts *opts);

/*
 * fmm_plan: build the octree (Appendix C), the per-level translation
 * operators S|S, S|R, R|R (eqs. 2.20-2.21) and the self-triangle correction
 * blocks (Appendix B) for one wavenumber k = k_re + i k_im (k_im >= 0).
 *   points   host f64[n][3]   node positions s_beta
 *   normals  host f64[n][3]   unit normals (|n| within 1e-6 of 1), outward
 *   weights  host f64[n]      Nystrom weights w_beta > 0 (eq. 2.8)
 *   order    p >= 1: degrees 0..p-1 kept at every level (eq. 2.17 cut), translations
 *            as dense per-offset operators (p <= 24);
 *            p <= 0: an order per level chosen for opts->tol (default 1e-6 FP64,
 *            1e-4 FP32): p_l = max(2.8 d0, k d + 1.8 d0^(2/3) (k d)^(1/3)) with
 *            d0 = -log10 tol and d the level's box diameter, so that boxes many
 *            wavelengths across keep p_l ~ k d; translations by rotation, coaxial
 *            shift and rotation back (O(p^3) each).  Refused when the leaf level
 *            needs p > 40 or any level p > 400.
 * Lossy wavenumbers (Im k > 0, Sec. 2.1: g decays as exp(-Im k R)): the
 * far field of level l is dropped when exp(-Im k h_l) < far_cutoff, h_l being
 * the level's box side, the shortest distance between two boxes of its
 * far-field lists (Appendix C).  When every level is dropped the plan is
 * local only: no expansions are built or used, and near pairs farther apart
 * than R_c = ln(1/far_cutoff)/Im k are dropped too.  far_cutoff = 0 selects
 * 1e-16 for FP64 plans and 1e-8 for FP32 plans; a negative value keeps every
 * interaction.  Real k is never cut.
 * Errors: FMB_EINVAL for n < 2, non-finite input, bad normal, w <= 0,
 * k_im < 0, depth out of range, order out of range (1..24), two nodes at
 * the same position, corr_mode > 0 without triangles or with a triangle not
 * holding exactly 1 or 3 nodes.  The plan deep-copies its inputs.
 */
int fmm_plan(const double *points, const double *normals, const double *weights, int64_t n,
             double k_re, double k_im, int32_t order, const fmb_plan_opts *opts, void *stream,
             fmb_plan_t *out);

/*
 * fmm_matvec: y = Op_k(a, b) as defined at the top of this header.
 *   a, b  device [nrhs][n][3] complex (c128 for an FP64 plan, c64 for FP32), user node order
 *   y     device [nrhs][n][3] complex, written (not accumulated)
 *   1 <= nrhs <= nrhs_max.  Asynchronous on `stream`.
 */
int fmm_matvec(fmb_plan_t plan, const void *a, const void *b, void *y, int32_t nrhs, void *stream);

/*
 * fmm_matvec_adjoint: (a_bar, b_bar) = Op_k^H y, the conjugate transpose of
 * the operator fmm_matvec applies (eq. 2.12 with the point rule of eq. 2.8,
 * plus the self-triangle terms of App. B), so that
 *   sum conj(y) . Op_k(a, b) = sum conj(a_bar) . a + sum conj(b_bar) . b.
 * Per node beta, with F_c = sum_alpha g(s_beta, s_alpha) conj(y_alpha,c) and H_ic = d_i F_c,
 *   a_bar = conj(w (H n - H^T n - n tr H) + ...),  b_bar = conj(w F + ...)
 * (the dots being the transposed self-triangle blocks).  It runs the same
 * fast multipole method with monopole sources and value-and-gradient
 * evaluation.  y, a_bar, b_bar: device [nrhs][n][3] complex of the plan's
 * precision, user node order; none may alias.  Asynchronous on `stream`.
 * The first call allocates a workspace of nrhs_max * n * 12 complex.
 * FMB_EINVAL for FP64 plans of order above 23.
 */
int fmm_matvec_adjoint(fmb_plan_t plan, const void *y, void *a_bar, void *b_bar, int32_t nrhs,
                       void *stream);

int fmm_plan_info(fmb_plan_t plan, fmb_plan_info *info);

/*
 * fmm_plan_export_tree: copy the octree of App. C (levels, boxes, Neighbor and
 * far-field lists FF(l, q) = Children(Neighbor(Parent)) minus Neighbor) to
 * host memory for inspection.
 *   codes  host u64[n]   Morton code of every node (user order)
 *   perm   host i32[n]   perm[i] = user index of the i-th node in Morton order
 * and for one level l (0..depth), sized by fmm_plan_info.nbox[l] = B:
 *   keys   host u64[B]        box keys (code >> 3(21-l)), ascending
 *   parent host i32[B]        parent box index at level l-1 (-1 at level 0)
 *   start  host i32[B+1]      node range of each box in Morton order
 *   nbr    host i32[B][27]    neighbour box indices (-1 where absent), slot
 *                             (dz+1)*9 + (dy+1)*3 + (dx+1)
 *   ff_ofs host i32[B+1], ff_idx host i32[ff_ofs[B]]: far-field list (l >= 2)
 * Any pointer may be NULL to skip it; ff_idx needs ff_ofs from a first call.
 */
int fmm_plan_export_tree(fmb_plan_t plan, int32_t level, uint64_t *codes, int32_t *perm,
                         uint64_t *keys, int32_t *parent, int32_t *start, int32_t *nbr,
                         int32_t *ff_ofs, int32_t *ff_idx);

int fmm_plan_destroy(fmb_plan_t plan);

/*
 * Stage timers.  fmm_plan_profile(plan, mask) makes every later matvec on the
 * plan record HIP events around the stages whose bit (1 << stage) is set in
 * mask, on the matvec's stream; mask = 0 turns timing off and FMB_PROFILE_ALL
 * (or 1, kept for callers that pass a boolean) times every stage;
 * fmm_plan_profile_read synchronises on them and returns, per stage, the
 * summed time in milliseconds and the number of kernel launches timed since
 * the last read with reset = 1 (the S|R launches of all levels run back to
 * back and share one pair of events).  Stage order (FMB_NSTAGES = 11): gather, P2M,
 * M2M (S|S translation kernel), M2L (S|R translation kernel), L2L (R|R), L2P,
 * P2P, corrections (with the return to user order, plans with corrections),
 * scatter (the return to user order, plans without corrections), sums (the
 * per-target sums of the S|S and S|R translation slots), and the finest level's
 * S|R launch alone (plans with an order per level; its launch is also counted
 * in M2L).  ms and launches: host arrays of FMB_NSTAGES entries (either may be
 * NULL).
 */
#define FMB_NSTAGES 11
#define FMB_PROFILE_ALL 0x7ff
int fmm_plan_profile(fmb_plan_t plan, int32_t mask);
int fmm_plan_profile_read(fmb_plan_t plan, double *ms, int64_t *launches, int32_t reset);

/* ---------------- BEM system and solver (Secs. 2.2 and 3.1) ---------------- */

typedef struct {
    double tol;          /* stop when |b - A x| <= tol |b| (relative, 2-norm)               */
    int32_t restart;     /* Krylov basis size m                                              */
    int32_t maxit;       /* total iteration cap (nested mode: outer plus inner steps, checked */
                         /*    between outer steps, so one inner cycle may run past it)      */
    int32_t precond;     /* 0 none; 1 block A_self (6x6 per node, 3x3 for ibc), each block    */
                         /*    inverted exactly; 2 the paper's form (Sec. 3.1): an inner     */
                         /*    GMRES on the same block-diagonal A_self, at most 10 steps, to */
                         /*    a relative residual of 1e-2 per right-hand side (it keeps     */
                         /*    M = A_self and rebuilds it from the stored inverses at the    */
                         /*    first such solve: n nu^2 more complex entries per precision)  */
    int32_t x0_given;    /* 1: x holds the initial guess on entry                            */
    int32_t mixed;       /* 1: FP32 inner solves refined by FP64 residuals (needs FP32 plans);*/
                         /* 2: nested: FP64 fGMRES preconditioned by one FP32 fGMRES cycle   */
                         /*    of up to min(restart, inner_maxit) steps to inner_tol per     */
                         /*    outer step (for systems whose conditioning stops refinement)  */
    double inner_tol;    /* relative tolerance of each inner FP32 solve (mixed mode)         */
    int32_t inner_maxit; /* iteration cap of each inner solve                                */
    int32_t serial;      /* 1: the k0 and k1 FMM products of each application run one after  */
                         /*    the other on the caller's stream (0, the default: concurrently */
                         /*    on the caller's stream and the problem's second stream)        */
    int32_t adjoint;     /* 1: solve the adjoint system A^H x = rhs, right-preconditioned by */
                         /*    M^{-H} (info->residual is then |rhs - A^H x| / |rhs|)          */
    int32_t inner_reorth;/* mixed mode: 1 = the DGKS-triggered second Gram-Schmidt pass in   */
                         /*    the inner FP32 solves too; 0 (default) = one classical pass    */
                         /*    there (FP64 solves always use the DGKS test)                   */
    int32_t reserved[2];
} fmb_gmres_opts;

typedef struct {
    int32_t iterations;      /* Krylov iterations (all inner iterations in mixed mode; outer  */
                             /*    plus inner in nested mode)                                 */
    int32_t refinements;     /* outer FP64 refinement steps (mixed mode), outer FP64 fGMRES  */
                             /*    steps (nested mode)                                        */
    int32_t matvecs64;       /* BEM applies with the FP64 plans                               */
    int32_t matvecs32;       /* BEM applies with the FP32 plans                               */
    int32_t fp64_fallback;   /* mixed mode: 1 if a refinement step cut the FP64 residual by    */
                             /*    less than 2x, or by less than 1/20 of the reduction its     */
                             /*    inner tolerance asked for, and the solve went on in nested  */
                             /*    mode from the current iterate (inner cycles <= 100 steps)   */
    int32_t reserved;
    double residual;         /* final true relative residual |b - A x| / |b| (FP64 operator) */
    double history[256];     /* residual estimate per iteration (first 256)                  */
} fmb_gmres_info;

int fmb_gmres_opts_default(fmb_gmres_opts *opts);

/*
 * bem_problem_create: the 6N system of one scatterer in vacuum (eqs. 2.9-2.13),
 * unknowns per node (Phi, Psi) = (E_0, n x curl E_0):
 *   rows 0..2: 1/2 Phi + Op_{k0}(Phi, -Psi)
 *   rows 3..5: 1/2 T Phi - Op_{k1}(T Phi, -gamma Psi),  T = I + (1 - eps)/eps n n,
 * with p0 a plan at k0 and p1 a plan at k1 = k0 sqrt(eps mu) over the same
 * nodes (same order), gamma = mu.  p0_32/p1_32 are optional FP32 plans of the
 * same nodes for mixed-precision solves (NULL if unused).  The problem keeps
 * references to the plans (the caller destroys them after the problem).
 *   eps, mu  host c128 (2 doubles each)
 */
int bem_problem_create(fmb_plan_t p0, fmb_plan_t p1, fmb_plan_t p0_32, fmb_plan_t p1_32,
                       const double *eps, const double *mu, void *stream, fmb_problem_t *out);

/*
 * bem_problem_create_multi: J scatterers in vacuum (Sec. 2.1, Fig. 1).  Node
 * alpha belongs to scatterer region[alpha] (host i32[n], values 0..J-1), with
 * permittivity eps[j] and permeability mu[j] (host c128[J] each).  The host
 * rows use p0, a plan at k0 over all n nodes; the interior rows of scatterer j
 * use pj[j], a plan at k_j = k0 sqrt(eps_j mu_j) over that scatterer's nodes
 * in their global order (the nodes with region j, ascending):
 *   rows 0..2: 1/2 Phi + Op_{k0}(Phi, -Psi)                          (all nodes)
 *   rows 3..5: 1/2 T_j Phi - Op_{kj}(T_j Phi, -gamma_j Psi)          (scatterer j's plan)
 * p0_32 and pj_32 (J FP32 plans) are optional, together.  J <= 8.  J = 1 with
 * region all 0 is bem_problem_create.  All other entry points accept the
 * problem (the interior field of bem_field needs J = 1); the products of the
 * scatterers' plans run one after the other beside the host product.
 */
int bem_problem_create_multi(fmb_plan_t p0, const fmb_plan_t *pj, int32_t J, const int32_t *region,
                             const double *eps, const double *mu, fmb_plan_t p0_32, const fmb_plan_t *pj_32,
                             void *stream, fmb_problem_t *out);

/*
 * bem_problem_create_ibc: the impedance-boundary-condition system of eq. 2.25
 * for a good conductor: with n x E = Z n x (n x H) (eq. 2.24) the unknowns
 * are Phi = E_0 alone (three per node), and
 *   (A Phi) = 1/2 Phi + Op_{k0}(Phi, c n x (n x Phi)),   c = i k0 / Z,
 * right-preconditioned by the 3x3 self blocks 1/2 I + K(dV) + c dG (n n^T - I).
 * p0: FP64 plan at k0 with self-triangle corrections; p0_32: optional FP32
 * plan of the same nodes and wavenumber (mixed solves); Z: host c128 surface
 * impedance relative to vacuum (Z = sqrt(mu/eps) of the conductor).  On such
 * a problem bem_apply, bem_apply_adjoint, bem_precond_apply,
 * bem_rhs_planewave and gmres_solve(_group) take [nrhs][n][3] vectors.
 */
int bem_problem_create_ibc(fmb_plan_t p0, fmb_plan_t p0_32, const double *Z, void *stream, fmb_problem_t *out);

/*
 * bem_problem_use_graphs: enable (1) or disable (0, the default) the replay of
 * the two FMM products of each application from a captured HIP graph.  The
 * graph is captured on first use per precision and rhs count, on a stream the
 * problem owns, ordered after and before the caller's stream by events; plans
 * with stage timers on always run eagerly.  Results are identical either way.
 * Eager launches alternate between the two products' streams; on MI355X they
 * measured faster than the replay.
 */
int bem_problem_use_graphs(fmb_problem_t pb, int32_t enable);

/* bem_apply: r = A x, x and r device c128 [nrhs][n][6]. */
int bem_apply(fmb_problem_t pb, const void *x, void *r, int32_t nrhs, void *stream);

/*
 * bem_apply32: r = A x with the problem's FP32 plans, the operator the inner solves of the
 * mixed modes apply (eqs. 2.9-2.13; FP32 products, FP64 self-triangle blocks rounded to FP32
 * in the return to user order).  x and r device c64 [nrhs][n][nu] (nu = 6, or 3 for
 * impedance problems), not aliased.  When both FP32 plans share their nodes and octree, k0
 * is real and the interior plan is local only (strongly lossy k1), the two near fields run as
 * one launch.  FMB_EINVAL without FP32 plans or for nrhs
 * out of range.  Asynchronous on `stream`.
 */
int bem_apply32(fmb_problem_t pb, const void *x, void *r, int32_t nrhs, void *stream);

/*
 * bem_apply_adjoint: r = A^H x, the conjugate transpose of bem_apply's
 * operator, x and r device c128 [nrhs][n][6].  With (a_j, b_j) = Op_kj^H x_j
 * (fmm_matvec_adjoint) for x_0 = x[0:3], x_1 = x[3:6]:
 *   r[0:3] = 1/2 x_0 + a_0 + T^H (1/2 x_1 - a_1),   r[3:6] = conj(gamma) b_1 - b_0.
 * The first call allocates the plans' adjoint workspaces.
 */
int bem_apply_adjoint(fmb_problem_t pb, const void *x, void *r, int32_t nrhs, void *stream);

/* bem_precond_apply: z = M^{-1} v with M = A_self (6x6 per node, eq. 3.2). c128 [nrhs][n][6]. */
int bem_precond_apply(fmb_problem_t pb, const void *v, void *z, int32_t nrhs, void *stream);

/*
 * bem_rhs_planewave: the right-hand side Phi^inc of eqs. 2.9-2.12 for incident
 * plane waves E^inc(s) = p_q exp(i k0 d_q . s) in the host medium (no incident
 * field inside the scatterers, Sec. 2.1):
 *   rhs[q][alpha] = (p_q exp(i k0 d_q . s_alpha), 0, 0, 0)    (6 unknowns per node)
 *   rhs[q][alpha] = p_q exp(i k0 d_q . s_alpha)                (impedance problems)
 *   dirs  host f64[nrhs][3]   propagation directions (used as given)
 *   pols  host c128[nrhs][3]  complex polarisations (linear, circular or
 *                             elliptic; interleaved re, im), used as given
 *   rhs   device c128[nrhs][n][nu], user node order, written
 * Synchronises `stream` before returning (dirs and pols may be freed).
 * FMB_EINVAL for a null pointer or nrhs < 1.
 */
int bem_rhs_planewave(fmb_problem_t pb, const double *dirs, const double *pols, void *rhs,
                      int32_t nrhs, void *stream);

/*
 * gmres_solve: right-preconditioned flexible GMRES (Sec. 3.1, eq. 3.1) on
 * A x = rhs (or A^H x = rhs with o->adjoint) for each of nrhs right-hand
 * sides.  rhs, x device c128 [nrhs][n][nu] (nu = 6, or 3 for an impedance
 * problem).  o->mixed selects the precision path: 0 FP64 throughout; 1 FP32
 * inner solves inside FP64 iterative refinement, which switches to nested
 * mode when a step stops contracting; 2 nested (FP64 fGMRES whose
 * preconditioner is one FP32 fGMRES cycle).  The residual that stops the
 * solve is always the FP64 one.  Synchronous.  Returns FMB_ENOCONV (x holds
 * the last iterate, info filled) when maxit is reached.  info may be NULL;
 * with nrhs > 1 it describes the slowest right-hand side.
 */
int gmres_solve(fmb_problem_t pb, const void *rhs, void *x, int32_t nrhs, const fmb_gmres_opts *o,
                fmb_gmres_info *info, void *stream);

/*
 * gmres_solve_group: the solves of `count` independent problems (meshes of
 * any sizes, each with its own plans, wavenumbers and permittivity) run
 * together on the current device: problem i solves A_i x[i] = rhs[i] for
 * nrhs[i] right-hand sides exactly as gmres_solve would (same options o for
 * all, results bit-identical to separate calls), each on its own host thread
 * and its own stream, so that the GPU overlaps the problems' launches.  The
 * batched multi-mesh workload of the fGMRES loop (Sec. 3.1) thus runs as one
 * call.  Problems and their plans must be distinct.  rhs[i], x[i]: device
 * c128 [nrhs[i]][n_i][6].  info: NULL or `count` entries.  The work starts
 * after the work queued on `stream` so far; synchronous.  Returns the first
 * failing problem's error, else FMB_ENOCONV if any problem reached maxit.
 */
int gmres_solve_group(const fmb_problem_t *pbs, int32_t count, const void *const *rhs, void *const *x,
                      const int32_t *nrhs, const fmb_gmres_opts *o, fmb_gmres_info *info, void *stream);

/*
 * bem_field: fields away from the surface from a solution x (device c128
 * [nrhs][n][nu], nu = 6, or 3 for an impedance problem).  Eq. 2.5 at points off
 * the boundary carries the jump term 1 instead of 1/2, so with the rows of
 * bem_apply:
 *   region 0, far 0: the scattered field at host points, E_sca(r) = -Op_k0(Phi, -Psi)(r)
 *                    (b = c n x (n x Phi) in place of -Psi for an impedance problem);
 *   region 1, far 0: the field inside the scatterer, E_1(r) = Op_k1(T Phi, -gamma Psi)(r)
 *                    (dielectric problems);
 *   region 0, far 1: the far-field amplitude F(rhat), E_sca ~ e^{i k0 r} / r F(rhat), for unit
 *                    directions rhat;
 *   region 0, far 2: curl E_sca at host points (the scattered magnetic field is
 *                    curl E_sca / (i k0) in units with eps0 = mu0 = 1), the curl in r of the
 *                    same sum: -sum w [ Hess(g) (a x n) + k0^2 g (a x n) + grad g x b ].
 * points: host f64[nt][3] target points (off the surface: a target that
 * coincides with a node skips that node) or unit directions; E: device c128
 * [nrhs][nt][3].  Direct FP64 sums over all nodes (cost nt * n per right-hand
 * side); synchronous.  far outside 0..2, or far != 0 with region 1, is
 * FMB_EINVAL.
 */
int bem_field(fmb_problem_t pb, const void *x, int32_t nrhs, const double *points, int64_t nt, int32_t region,
              int32_t far, void *E, void *stream);

/*
 * bem_field_noalloc: bem_field for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  Same arguments, results and errors as bem_field; it calls no
 * hipMalloc or hipFree.  The target points are staged in a fixed array that the
 * library holds on every GPU it runs on until the process ends, so nt is at most
 * FMB_FIELD_NOALLOC_MAX_TARGETS (more is FMB_EINVAL).  All calls on one GPU share
 * that array: calls that overlap on one GPU (other threads or streams) race;
 * calls in sequence do not, since each returns after its stream is idle.
 */
#define FMB_FIELD_NOALLOC_MAX_TARGETS 65536
int bem_field_noalloc(fmb_problem_t pb, const void *x, int32_t nrhs, const double *points, int64_t nt,
                      int32_t region, int32_t far, void *E, void *stream);

/*
 * bem_far_field_adjoint: the conjugate transpose of the far-field map of
 * bem_field (region 0, far 1: the far-zone limit of eq. 2.5, whose power
 * gives C_sca of eq. 4.2), x -> F: given samples G at nd unit directions it
 * returns xbar = L^H G, so that sum conj(G) . (L x) = sum conj(xbar) . x for
 * every x.  This is the backward pass of a functional of the far field (e.g.
 * C_sca = oint |F|^2 dOmega) with respect to the unknowns.  G: device c128
 * [nrhs][nd][3]; dirs: host f64[nd][3] unit vectors; xbar: device c128
 * [nrhs][n][nu] (every entry written).  Direct FP64 sums (cost n * nd);
 * synchronous.
 */
int bem_far_field_adjoint(fmb_problem_t pb, const void *G, int32_t nrhs, const double *dirs, int64_t nd, void *xbar,
                          void *stream);

/*
 * bem_field_fmm: the field of bem_field's kind 0 (eq. 2.5 off the surface;
 * region 0: E_sca at host points; region 1: the interior field) by the fast
 * multipole method of eqs. 2.17-2.23 instead of
 * direct sums, for many targets.  A temporary FP64 plan of the given order is
 * built over the nodes followed by the nt targets (the targets carry zero
 * density, so only the nodes radiate); one product of it gives the sum at every
 * target.  Cost O((n + nt) log) per call plus the plan build, against n * nt for
 * bem_field; the result agrees with bem_field to the FMM tolerance of the order
 * (measured p = 16: 7e-7 relative on plane grids around a sphere and a torus,
 * 3.5e-6 for a lone target far outside; p = 22: about 2e-8).
 * points: host f64[nt][3], off the surface and distinct from every node and
 * from each other (a coincident point is FMB_EINVAL); E: device c128
 * [nrhs][nt][3].  Allocates device memory for the plan and three
 * [nrhs][n + nt][3] work arrays; synchronous.
 */
int bem_field_fmm(fmb_problem_t pb, const void *x, int32_t nrhs, const double *points, int64_t nt, int32_t region,
                  int32_t order, void *E, void *stream);

/*
 * bem_shape_pairs: derivatives of one wavenumber's point sum with respect to
 * the nodes, the part of a shape gradient (eq. 4.2 differentiated through the
 * system of eqs. 2.8 and 2.12) that couples distinct triangles.  For fixed
 * densities (a, b) and adjoint weights lam, the bilinear form
 *   B = sum_alpha conj(lam_alpha) . PS_k(a, b)_alpha
 * of the point sum PS_k (fmm_matvec's operator without the self-triangle
 * blocks, pairs inside one triangle excluded) is differentiated with respect
 * to every node's position, normal and weight; a node's position derivative
 * sums its source and target roles.  With u = conj(lam_alpha), d = s_beta - s_alpha,
 * g of eq. 2.4, grad'g = f d, f = (ikR - 1) g / R^2, f'/R = (3 - 3ikR - k^2 R^2) g / R^4,
 * c = (u . n_beta) a_beta - (u . a_beta) n_beta - (n_beta . a_beta) u, e = u . b_beta:
 *   ds[beta]  = sum_alpha w_beta [ f c + ((f'/R)(d . c) + f e) d ] - sum_gamma (the same with beta as target)
 *   dn[beta]  = sum_alpha w_beta f [ (d . a_beta) u - (u . a_beta) d - (d . u) a_beta ]
 *   dw[beta]  = sum_alpha [ f (d . c) + g e ]
 * (holomorphic derivatives of the complex B; a real functional takes Re).
 *   points, normals  device f64[n][3];  weights device f64[n];  point_tri device i32[n]
 *                    (triangle of each node; values are compared, not indexed)
 *   lam, a, b        device c128[n][3], user node order
 *   ds, dn           device c128[n][3], written;  dw device c128[n], written
 * Direct FP64 sums, two passes of n^2 pairs, each split over chunks of the
 * other side whose partial sums (a temporary device buffer of at most
 * 64 n x 10 complex) are added in a fixed order; synchronous.  A pair of nodes
 * of different triangles at the same position contributes nothing.
 * FMB_EINVAL for n < 1, a NULL pointer, k_im < 0 or an output aliasing an input.
 */
int bem_shape_pairs(const double *points, const double *normals, const double *weights, const int32_t *point_tri,
                    int64_t n, double k_re, double k_im, const void *lam, const void *a, const void *b, void *ds,
                    void *dn, void *dw, void *stream);

/*
 * bem_self_blocks: the self-triangle correction blocks of Appendix B for a
 * given geometry, as fmm_plan builds them (mode FMB_CORR_MEAN or
 * FMB_CORR_LINEAR), without a plan: the local part of a shape gradient
 * differentiates them numerically.  Node alpha's row gets, for the j-th node
 * beta of its triangle (the triangle's nodes in ascending index order),
 *   y_alpha += n_beta (dV . a_beta) - (n_beta . dV) a_beta - dV (n_beta . a_beta) + dG b_beta,
 *   dV = dv[alpha][j] (c128[3]),  dG = dg[alpha][j].
 *   points, normals  host f64[n][3] (unit normals);  point_tri host i32[n] in [0, ntri)
 *   tri_vertices     host f64[ntri][3][3];  every triangle holds n / ntri in {1, 3} nodes
 *   dv               device c128[n][m][3], dg device c128[n][m], m = n / ntri, written
 * Allocates temporary device memory; synchronous.  FMB_EINVAL for bad sizes,
 * non-finite input, non-unit normals, out-of-range point_tri, a triangle not
 * holding exactly m nodes, or LINEAR with m = 1.
 */
int bem_self_blocks(const double *points, const double *normals, const int32_t *point_tri, const double *tri_vertices,
                    int64_t n, int64_t ntri, int32_t mode, double k_re, double k_im, void *dv, void *dg,
                    void *stream);

int bem_problem_destroy(fmb_problem_t pb);

/* Thread-local message for the last non-zero status returned on this thread. */
const char *fmb_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* FMBEM_H */
