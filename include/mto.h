/*
 * mto.h: C ABI of the MI355X (gfx950) library for the finite element analysis
 * and sensitivity step of dp-adaptive multiresolution topology optimization
 * (Gupta, van Keulen, Langelaar, arXiv 1811.09821).
 *
 * What one solve computes, for every design instance and load case:
 *   - the modified SIMP modulus of every density cell (Sec. 2.2):
 *       E(rho) = Emin + rho^q (E0 - Emin);
 *   - the element stiffness of Sec. 2.2 in the composite per-density-cell
 *     form of Appendix B: K_e = sum_s E(rho_{e,s}) K_s, with K_s the exact
 *     integral of B^T D0 B (plane stress) over density cell s;
 *   - the displacement u solving K u = f (Eq. eq_comp_1) with supported DOFs
 *     eliminated, by matrix-free preconditioned conjugate gradients (K is
 *     never assembled); the preconditioner is chosen per plan
 *     (mto_params.precond): a multigrid V-cycle with element-block Schwarz
 *     smoothing, the same V-cycle with l1-Jacobi smoothing, or Jacobi.  The
 *     paper names no solver; any SPD preconditioner reaches the same u to
 *     the tolerance;
 *   - the compliance c = f^T u (the objective z^T u with z = f, Sec. 4.1);
 *   - the sensitivity dc/drho_{e,s} = -E'(rho_{e,s}) u_e^T K_s u_e.  The paper
 *     names the sensitivity analysis (Sec. 1, Sec. 2.1) without printing it;
 *     compliance is self-adjoint (adjoint = -u), so no second solve is needed.
 *
 * Discretisation (readings of points the paper leaves open):
 *   - structured mesh of unit-square elements, element e = ey*nelx + ex, origin
 *     bottom-left, y up; vertex (vx, vy) with 0 <= vx <= nelx, 0 <= vy <= nely;
 *   - each element has its own order p (1..MTO_MAX_P) and its own d x d grid of
 *     density cells (d in 1..MTO_MAX_D), cell s = sy*d + sx (Sec. 2.1 background
 *     mesh; the paper's "number of design points" is d*d here);
 *   - hierarchic basis: (1 -/+ xi)/2 and integrated Legendre polynomials
 *     int_{-1}^{xi} P_{k-1}, k = 2..p;
 *   - mixed orders are made compatible by the conforming "minimum rule": a
 *     shared edge carries the edge modes 2..min(p_left, p_right) (the
 *     conforming continuous piecewise-Q_p space; the paper requires a compatible
 *     mixed-p field, Sec. 3, without spelling out the construction).
 *
 * Layouts (all arrays FP64, contiguous, device memory unless stated):
 *   - densities rho and sensitivities g: per instance, element-major cells
 *     (instance i starts at its cell offset, mto_instance_info); g has one
 *     block of n_cells per load case: [L_i][n_cells_i];
 *   - displacements u: per instance [L_i][n_dof_i], scalar function id k has
 *     DOFs 2k (x) and 2k+1 (y).  Ids: vertices vy*(nelx+1)+vx; then horizontal
 *     edges (index vy*nelx+ex) each with modes 2..deg; then vertical edges
 *     (index ey*(nelx+1)+vx); then element interiors (i, j >= 2, i fastest).
 *     Supported DOFs hold 0;
 *   - compliances c: per instance [L_i].
 *   Instances are concatenated in the order they were given.
 *
 * Conventions: every function returns MTO_OK (0) or a negative error code and
 * never throws; mto_last_error() gives a thread-local message.  Device work is
 * enqueued on the HIP stream passed as `stream` (NULL: the null stream).
 * A plan owns its device buffers and may be used by one stream at a time.
 */
#ifndef MTO_H
#define MTO_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MTO_MAX_P 4
#define MTO_MAX_D 8

enum {
  MTO_OK = 0,
  MTO_EINVAL = -1,      /* bad argument: shape, range, NULL pointer, load on a support */
  MTO_ESINGULAR = -2,   /* supports leave a rigid-body mode free */
  MTO_ENOCONV = -3,     /* the true residual misses rtol: PCG hit max_iter, or the residual
                           stalled above rtol after the restarts (outputs still written) */
  MTO_EBREAKDOWN = -4,  /* p^T K p <= 0 or non-finite value in PCG */
  MTO_EHIP = -5,        /* HIP runtime error */
  MTO_ENOMEM = -6       /* device allocation failed */
};

enum { /* support kinds */
  MTO_SUP_VERTEX = 0,      /* vertex (a, b) */
  MTO_SUP_EDGE_LEFT = 1,   /* whole boundary x = 0: its vertices and edge modes */
  MTO_SUP_EDGE_RIGHT = 2,  /* x = nelx */
  MTO_SUP_EDGE_BOTTOM = 3, /* y = 0 */
  MTO_SUP_EDGE_TOP = 4     /* y = nely */
};

enum { /* element contraction kernels */
  MTO_PATH_MFMA = 0,  /* per-(p,d) group, FP64 MFMA tiles (default) */
  MTO_PATH_PLAIN = 1  /* one thread per element column, FP64 VALU (comparison path) */
};

enum { /* PCG preconditioners (the caller sets one in mto_params; the Python
          binding's default is MTO_PRECOND_MG_ASM, the fastest on every
          workload measured) */
  MTO_PRECOND_JACOBI = 0, /* diagonal of K */
  MTO_PRECOND_MG = 1,     /* one multigrid V-cycle: hierarchic-order injection to the bilinear
                             vertex grid, then geometric coarsening with Galerkin operators,
                             l1-Jacobi smoothing, dense coarsest solve */
  MTO_PRECOND_MG_ASM = 2  /* the same V-cycle with an element-block additive Schwarz smoother on
                             the hierarchic level: exact inverses of the assembled operator
                             restricted to each element's DOFs, formed once per design */
};

typedef struct {
  int32_t nelx, nely;
  const int8_t* p; /* host [nelx*nely], order per element */
  const int8_t* d; /* host [nelx*nely], density cells per side per element */
} mto_mesh;

typedef struct {
  int32_t kind;      /* MTO_SUP_* */
  int32_t a, b;      /* vertex coordinates for MTO_SUP_VERTEX, else ignored */
  int32_t comp_mask; /* bit 0: fix x, bit 1: fix y */
} mto_support;

typedef struct {
  int32_t vx, vy;    /* loaded vertex */
  double fx, fy;     /* force components */
  int32_t load_case; /* 0 .. n_load_cases-1 */
} mto_point_load;

typedef struct {
  double E0;      /* solid Young's modulus (Sec. 2.2) */
  double Emin;    /* void modulus, typically 1e-9 E0 (Sec. 2.2) */
  double nu;      /* Poisson ratio */
  double q;       /* SIMP penalisation power */
  double rtol;    /* PCG stop: ||r||_2 <= rtol ||f||_2 */
  int32_t max_iter;         /* PCG iteration cap per system (<= 0: 20 * n_free) */
  int32_t kernel_path;      /* MTO_PATH_* */
  int32_t iters_per_launch; /* PCG iterations per captured graph launch (<= 0: 32 with Jacobi,
                               8 with a multigrid preconditioner) */
  int32_t max_restarts;     /* refinement restarts from the true residual when it misses rtol (< 0: 3) */
  int32_t precond;          /* MTO_PRECOND_* */
  double mg_omega;          /* level-0 smoother weight.  MTO_PRECOND_MG: damped Jacobi with this
                               factor if > 0, else l1-Jacobi.  MTO_PRECOND_MG_ASM: Schwarz
                               damping if > 0, else 2 / (9 * 1.05), below the bound 2 / 9 that
                               the nine-colouring of element blocks guarantees */
  int32_t mg_coarse_max;    /* multigrid: coarsen until the largest instance's grid has at most this
                               many DOFs, solved exactly (<= 0: 3000, the most allowed) */
  int32_t stored_matrices;  /* 1: mto_autotune may give a group of order p >= 3 stored element
                               matrices (mto_set_tile ks = -2) when they are faster than its
                               contraction; 0: it chooses among contraction shapes only */
} mto_params;

/* A linear spring from one vertex DOF to ground, stiffness k > 0: adds k to
 * that diagonal entry of K.  The force inverter of Sec. 4.1 has one at its
 * input (k_in) and one at its output (k_out).  Springs enter the operator of
 * the solve and its true residual, not the preconditioner (a rank-n_springs
 * change costs PCG at most n_springs extra iterations).  A spring on a
 * supported DOF is MTO_EINVAL. */
typedef struct {
  int32_t vx, vy; /* vertex */
  int32_t comp;   /* 0: x, 1: y */
  double k;
} mto_spring;

typedef struct {
  mto_mesh mesh;
  const mto_support* supports; /* host [n_supports] */
  int32_t n_supports;
  const mto_point_load* loads; /* host [n_loads] */
  int32_t n_loads;
  int32_t n_load_cases;        /* >= 1 */
  const mto_spring* springs;   /* host [n_springs] or NULL */
  int32_t n_springs;           /* >= 0 */
} mto_problem;

typedef struct {
  int32_t status;            /* MTO_OK, MTO_ENOCONV or MTO_EBREAKDOWN */
  int32_t n_systems;         /* instances x load cases */
  int32_t max_iterations;    /* over systems */
  int32_t restarts;          /* restarts taken */
  int32_t* iterations;       /* host [n_systems] or NULL: PCG iterations per system */
  double* true_rel_residual; /* host [n_systems] or NULL: ||f - K u|| / ||f|| at exit, with
                                f - K u evaluated in extended precision (see mto_solve) */
  double solve_ms;           /* host wall time of the call */
} mto_solve_stats;

typedef struct {
  int32_t n_instances;
  int32_t n_systems;     /* sum of load cases */
  int32_t n_groups;      /* distinct (p, d) pairs */
  int32_t reserved;
  int64_t n_cells;       /* length of rho */
  int64_t n_u;           /* length of u */
  int64_t n_g;           /* length of g */
  int64_t n_free_total;  /* sum over systems of free DOFs */
  int64_t n_elements;
  double flops_per_matvec; /* algorithmic contraction flops, all systems: sum 2 S n_e^2 */
} mto_plan_info_t;

typedef struct mto_plan mto_plan;

/* Thread-local description of the last error (empty string if none). */
const char* mto_last_error(void);

/* Library version string. */
const char* mto_version(void);

/* Builds a plan for one design (Sec. 2.2 problem, Eq. eq_comp_1): checks the
 * mesh, numbers the conforming space, groups elements by (p, d), uploads the
 * K_s tables and the gather/scatter descriptors.  Host inputs are copied.
 * Uses the current HIP device.  Errors: MTO_EINVAL (p or d out of range, a
 * support or load outside the mesh, a load on a supported DOF, no free DOF),
 * MTO_ESINGULAR (supports do not remove all three rigid-body modes),
 * MTO_ENOMEM, MTO_EHIP.  *out receives the plan (caller destroys it). */
int mto_plan_create(const mto_problem* prob, const mto_params* params, mto_plan** out);

/* Same for n_instances independent designs (each with its own mesh, p, d,
 * supports and load cases), solved together: all (p, d) groups of all
 * instances share each kernel launch. */
int mto_batch_plan_create(const mto_problem* probs, int32_t n_instances, const mto_params* params,
                          mto_plan** out);

/* Sizes of the plan's arrays (host struct filled). */
int mto_plan_info(const mto_plan* plan, mto_plan_info_t* info);

/* Offsets of instance `inst` in rho/g (cells), u and c, its sizes and free DOFs.
 * Any output pointer may be NULL. */
int mto_instance_info(const mto_plan* plan, int32_t inst, int64_t* cell_off, int64_t* n_cells,
                      int64_t* u_off, int64_t* n_dof, int64_t* g_off, int64_t* c_off,
                      int64_t* n_free, int32_t* n_load_cases);

/* One FEA + sensitivity step (Sec. 2.2: the state equation K u = f of
 * Eq. eq_comp_1 with the SIMP stiffness, the objective c = f^T u of Sec. 4.1,
 * and its design sensitivities, Sec. 1 and 2.1; the sensitivity formula is
 * the adjoint result for the self-adjoint compliance, derived, since the
 * paper does not print it).
 *   rho  device [n_cells]: densities, each finite and in [0, 1] (Eq. eq_comp_1
 *        constrains 0 <= rho <= 1); otherwise MTO_EINVAL (outputs undefined)
 *   u    device [n_u] out; c device [total load cases] out
 *   g    device [n_g] out (dc/drho per load case) or NULL to skip it
 *   u0   device [n_u] initial guess or NULL (zero)
 *   stats host, may be NULL: iteration counts and true residuals
 * Stop test: ||f - K u||_2 <= rtol ||f||_2 per system, with u kept in
 * double-double and f - K u evaluated in extended precision (compensated
 * per-cell dot products, double-double over the cells) at the end of each
 * PCG cycle.  Inside a cycle, a system whose recursive residual nears the
 * rounding floor of its FP64 recurrence has its correction folded into u and
 * its residual replaced by that accurate one, PCG continuing with the same
 * search direction (at most 8 times per cycle); restarts from the final
 * residual (at most max_restarts) continue while it misses rtol and still
 * improves.
 * Returns MTO_OK, MTO_ENOCONV (the residual of some system misses rtol) or
 * MTO_EBREAKDOWN (outputs are written in these three cases), MTO_EINVAL, or
 * a HIP error.
 * The call blocks the calling thread until the convergence of every system
 * is known.  Convergence is decided on the device, per system, and the host
 * decides how many captured chunks of iterations to launch: it keeps two
 * chunks queued past the last progress report it has read (a 16-byte copy
 * to pinned memory per chunk), so the GPU never waits for the host; only the
 * host thread waits.  Returning before convergence would need either a
 * fixed, over-provisioned number of chunks (each costs its launches even
 * when every system has stopped) or device-side control of the loop.  The
 * work is enqueued on `stream`, so other streams keep running meanwhile. */
int mto_solve(mto_plan* plan, const double* rho, double* u, double* c, double* g, const double* u0,
              void* stream, mto_solve_stats* stats);

/* Binds device buffers (rho in; u, c, g out; g may be NULL) and records the
 * setup, one block of PCG iterations and the finishing steps as HIP graphs. */
int mto_batch_capture(mto_plan* plan, const double* rho, double* u, double* c, double* g,
                      void* stream);

/* Replays the graphs bound by mto_batch_capture with the current contents of
 * the bound rho: same results and return codes as mto_solve. */
int mto_batch_replay(mto_plan* plan, void* stream, mto_solve_stats* stats);

/* y = K x for every system of the plan (x, y device arrays in the u layout),
 * with K assembled from the element matrices of Sec. 2.2 in the composite
 * per-cell form of Appendix B; the product of each PCG iteration.
 * Supported DOFs of x are ignored and those of y are set to 0, i.e.
 * y = K_ff x_f.  rho is not checked (mto_solve checks it).  Asynchronous on
 * stream. */
int mto_apply_stiffness(mto_plan* plan, const double* rho, const double* x, double* y, void* stream);

/* Size of the device scratch array of mto_apply_stiffness_noalloc (per GPU,
 * held from the library's first use on that GPU until the process ends). */
#define MTO_NOALLOC_SCRATCH_BYTES (32 * 1024 * 1024)

/* mto_apply_stiffness for callers that cannot allocate device memory: code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc.  Same arguments and result (y = K x, u layout, supported DOFs
 * of y set to 0); it calls no hipMalloc/hipFree.  Its scratch (cell moduli,
 * gathered x, element slots: 8 (2 n_cells + n_free_total + slots) bytes,
 * slots being 4 per free vertex DOF, 2 per free edge DOF and 1 per free
 * interior DOF of every system) lives in one static device array of
 * MTO_NOALLOC_SCRATCH_BYTES per GPU, shared by every call on that GPU: calls
 * that overlap on one GPU (other streams, other threads, other plans) race
 * and must be serialised by the caller.  The current device must be the
 * plan's device.  The first call on a device looks the array's address up
 * (no allocation).  MTO_EINVAL if the plan needs more scratch than the
 * array holds, or on NULL arguments.  Asynchronous on stream. */
int mto_apply_stiffness_noalloc(mto_plan* plan, const double* rho, const double* x, double* y, void* stream);

/* g = -E'(rho) u_e^T K_s u_e for given displacements u (device, u layout)
 * into g (device, g layout): the compliance sensitivity (Sec. 1 and 2.1 name
 * the sensitivity analysis; the formula is the adjoint result for the
 * self-adjoint compliance, lambda = -u).  Asynchronous on stream. */
int mto_sensitivity(mto_plan* plan, const double* rho, const double* u, double* g, void* stream);

/* Adjoint sensitivity of a linear objective J = z^T u (Eq. (1)): for every
 * system l, g_l[cell] = -E'(rho) lam_{l,e}^T K_s u_{l,e}, with u and lam
 * device arrays in the u layout (lam_l the adjoint state of system l, i.e.
 * the solution of K lam = z for J = z^T u_l) and g in the g layout.  With
 * lam = u this is mto_sensitivity.  For the force inverter of Sec. 4.1,
 * solve with load case 0 = f_in and load case 1 = the unit load at the
 * output DOF and pass lam = u with the two cases swapped: g_0 = dJ/drho.
 * Overwrites the plan's moduli and PCG work vectors. */
int mto_adjoint_sensitivity(mto_plan* plan, const double* rho, const double* u, const double* lam, double* g,
                            void* stream);

/* Backward of the map densities -> compliances: out[cell] = sum over the
 * load cases l of the cell's instance of w[l] g_l[cell], with g as written by
 * mto_solve (layout [L_i][n_cells_i] per instance) and w [total load cases]
 * in the c layout; out [n_cells] in the rho layout.  Compliance is
 * self-adjoint, so g_l = dc_l/drho already is the adjoint product. */
int mto_weighted_sensitivity(mto_plan* plan, const double* g, const double* w, double* out, void* stream);

/* Jacobi preconditioner diagonal: diag(K) per instance in the u layout of its
 * first load case (length sum_i n_dof_i); supported DOFs get 0. */
int mto_jacobi_diagonal(mto_plan* plan, const double* rho, double* diag, void* stream);

/* Times the element contraction of every (p, d) group of the plan for each
 * tile shape (ncol x ks, see mto_set_tile) and keeps the fastest per group.  rho is a
 * representative density field.  cache_path (host string, may be NULL): a
 * text file of tile shapes keyed by (GPU architecture, p, d, floor(log2 of
 * the group's element columns)); a group found there takes the cached
 * shape without timing, and the shapes timed in this call are added to the
 * file (a missing file is created; MTO_EINVAL if it cannot be parsed).
 * report (host, may be NULL) receives a text summary of at most report_len
 * bytes.  With mto_params.stored_matrices = 1 the stored element matrices
 * (mto_set_tile ks = -2) are a candidate for the groups of p >= 3.  Blocks
 * until the timing is done. */
int mto_autotune(mto_plan* plan, const double* rho, const char* cache_path, void* stream, char* report,
                 int32_t report_len);

/* Sets the tile shape of the element contraction for the group with order p
 * and cell grid d (all groups if p <= 0): ncol blocks of 16 element columns
 * per tile (1, 2 or 4) and ks waves per tile splitting the density cells
 * (1..8, clamped to d*d); or, with ks = 0 (p >= 3 only, ncol 1 or 2), the
 * LDS-staged contraction: 4 waves of 16 ncol columns each share the cell
 * tables, staged in LDS one cell ahead (with p <= 0 the groups of p < 3 keep
 * their shape).  ks = -1 (p, d, ncol ignored): the product of every group in
 * one launch (the LDS-staged contraction of 64-column tiles from all groups,
 * the long ones first); any other call returns to one launch per group.
 * mto_autotune picks between the two by timing.  ks = -2 (ncol ignored):
 * stored element matrices for the group(s): K_e = sum_s E_s K_s (the
 * operator of Eq. (2) with the composite integration of Appendix B, per
 * element) is assembled once per solve set-up and mto_apply_stiffness call,
 * its packed upper triangle kept on the device (n_e (n_e + 1) / 2 doubles per
 * element, allocated on first use), and each product reads it instead of
 * contracting the cell tables; every load case of an instance shares one
 * read.  The product is HBM-bound instead of MFMA-bound; it is not part of
 * the one-launch product.  MTO_EINVAL if the shape needs more LDS than the
 * kernel takes (64 KB; 160 KB for ks = 0) or no group matches (ks = -2).
 * Invalidates captured graphs. */
int mto_set_tile(mto_plan* plan, int32_t p, int32_t d, int32_t ncol, int32_t ks);

/* Average time (ms, from HIP events on `stream`) of one PCG search-direction
 * product K p, i.e. the element contraction kernels of all (p, d) groups.
 * in_loop = 0: `reps` back-to-back launches of the first iteration's product
 * after 3 warm-ups, between two stream events.  in_loop = 1: `reps` PCG
 * iterations run eagerly from x = 0 (the kernels of a captured chunk, in
 * order), each product kernel launched with start/end events on its own
 * dispatch (hipExtLaunchKernel), summed over groups and averaged over
 * iterations; reps should not exceed the iteration count of a solve,
 * since the products of a converged system return at once.  Both run the
 * solve setup for rho first and overwrite the plan's PCG state.  MTO_EINVAL
 * for reps < 1 or in_loop outside {0, 1}. */
int mto_time_contraction(mto_plan* plan, const double* rho, int32_t reps, int32_t in_loop, void* stream,
                         double* ms_per_matvec);

/* Frees the plan and its device buffers (NULL is a no-op). */
void mto_plan_destroy(mto_plan* plan);

/* QR-error indicator of Sec. 3.2.3 (Eq. (9)) for every element and load case:
 * eps = 1 - J^(p) / J^(p+1), with J^(p) = u_e^T K^(p) u_e / 2 the element's
 * strain energy at order p (K^(p) = sum_s E(rho_s) K_s^(p)) and J^(p+1) that
 * of the element-level problem at order p + 1, K^(p+1) u' = f', under the
 * element's own load f^(p) = K^(p) u_e kept on the (hierarchic) order-p
 * functions and zero on the new ones, with 3 DOFs (vertex (0,0) x and y,
 * vertex (1,0) y) taken from u_e; eps = 0 where J^(p+1) = 0.  The energies do
 * not depend on the choice or the values of the 3 DOFs (the load is
 * self-equilibrated), so the rigid motion they carry is removed first.
 *   rho  device, n_cells doubles (the densities u was computed for)
 *   u    device, u layout (as written by mto_solve)
 *   eps  device, sum over instances of L_i nel_i doubles: instance-major,
 *        then load case, then element e = ey*nelx + ex
 * Overwrites the plan's moduli and PCG work vectors (like mto_sensitivity).
 * The order-(p+1) cell tables are built on the host and uploaded at the
 * first call (p + 1 <= MTO_MAX_P + 1), which therefore allocates: do not
 * make the first call inside stream capture.  MTO_EINVAL, MTO_ENOMEM. */
int mto_qr_error(mto_plan* plan, const double* rho, const double* u, double* eps, void* stream);

/* ---- refinement indicators and the dp update (Sec. 3.2-3.3) -------------- */

/* Analysis indicator of Sec. 3.2.1 (Kelly): Gamma^a of an element = sum over
 * its interior edges F of c_F * integral_F |[du/dn]|^2 ds, [.] the jump of
 * the normal derivative of both displacement components across F, c_F =
 * h_F / (2 p_F), h_F = sqrt(2) (the element diagonal in element edge
 * lengths), p_F the larger order of the two elements.  Boundary edges carry
 * no jump.  u: device, u layout; gamma: device, the QR-error layout
 * (instance-major, then load case, then element).  Overwrites the plan's
 * PCG work vectors; the first call allocates lookup tables. */
int mto_kelly_indicator(mto_plan* plan, const double* u, double* gamma, void* stream);

/* Density indicator of Sec. 3.2.2 for adaptive cycle `cycle` (>= 1): per
 * element, over its cells rho, the refinement contributions (rho - r_l)/n
 * for r_l <= rho <= rho_avg and (r_u - rho)/n for rho_avg < rho <= r_u and
 * the coarsening contributions -(c_l - rho)/n for rho <= c_l and
 * -(rho - c_u)/n for rho >= c_u, with rho_avg = (rho_min + rho_max)/2,
 * s = rho_avg exp(-beta (cycle - 1)), r_l = rho_min + (1 - alpha) s,
 * r_u = rho_max - (1 - alpha) s, c_l = rho_min + alpha s, c_u = rho_max - alpha s
 * (the paper's alpha = 0.2, beta = 0.8; rho_min = 0, rho_max = 1).  rho: device,
 * rho layout; gamma: device, one value per element, instances concatenated. */
int mto_density_indicator(mto_plan* plan, const double* rho, int32_t cycle, double alpha, double beta,
                          double rho_min, double rho_max, double* gamma, void* stream);

/* Parameters of the dp update (Sec. 3.3): the analysis indicator refines
 * the top frac_a_refine and coarsens the bottom frac_a_coarsen of the
 * elements (the paper: 0.10, 0.05); the density indicator refines
 * frac_d_refine of the elements with Gamma^d > 0 and coarsens frac_d_coarsen of
 * those with Gamma^d < 0 (the paper: 1.0, 1.0); orders stay in [1, p_max];
 * an element's design points are capped at d_max (the paper: 64). */
typedef struct {
  double frac_a_refine, frac_a_coarsen, frac_d_refine, frac_d_coarsen;
  int32_t p_max, d_max;
} mto_dp_params;

/* Steps 2 and 3 of the dp update (Sec. 3.3) on one nelx x nely mesh, all
 * arrays on the host, one entry per element (e = ey*nelx + ex):
 *   ranking by ascending Gamma (ties by element index); step 2 sets the
 *   flag theta = -1 / +1 on the bottom / top fractions of Gamma^a and moves p
 *   by theta; step 3 lowers p of the density-coarsened elements whose theta
 *   is 0 (theta = -2 where p is already 1) and raises p of the
 *   density-refined elements whose theta is 0 or -1; then neighbouring orders
 *   are brought within 2 of each other by (p_max - p_min - 2) passes over the
 *   rows from the bottom, each element against its right and upper
 *   neighbour, raising the lower; design points = 1 where theta = -2, else
 *   min(2 (p+1)^2 - 3, d_max) (element DOFs minus the 3 rigid modes); the
 *   background grid gets the smallest perfect square of cells per element
 *   not below the largest number of design points.
 * Outputs: p_out, theta_out, design_points [nel], cells_per_element [1].
 * MTO_EINVAL on bad arguments. */
int mto_dp_update(int32_t nelx, int32_t nely, const int8_t* p, const double* gamma_a, const double* gamma_d,
                  const mto_dp_params* params, int8_t* p_out, int8_t* theta_out, int32_t* design_points,
                  int32_t* cells_per_element);

/* Step 4 of the dp update (Sec. 3.3): p_out = min(p + 1, p_max) where the
 * QR error (mto_qr_error, computed on the mesh after steps 2-3) exceeds
 * alpha_qr (the paper: 0.9), else p.  Host arrays [nel]. */
int mto_qr_update(int32_t nel, const int8_t* p, const double* eps, double alpha_qr, int32_t p_max, int8_t* p_out);

/* ---- density filter (Sec. 2.2, Eqs. (4)-(5)) ------------------------------
 * The step that precedes the analysis: filtered densities
 *   rho~_i = sum_j H_ij rho_j / sum_j H_ij,   H_ij = R - |c_i - c_j|  (> 0),
 * over the density cells j of the same instance whose centres c_j lie closer
 * than R to the centre c_i of cell i (composite integration: one point per
 * cell).  Lengths are in element edge lengths; cell s = sy*d + sx of element
 * e = ey*nelx + ex has its centre at (ex + (sx + 1/2)/d, ey + (sy + 1/2)/d).
 * The chain rule is the transpose: dJ/drho_j = sum_i dJ/drho~_i H_ij / sum_k H_ik.
 * Cell arrays use the plan layout (instances concatenated, element-major). */
typedef struct mto_filter mto_filter;

/* Builds H (symmetric, so one pattern serves W and W^T) and the row scales
 * 1 / sum_j H_ij on the host from the meshes of probs[0..n_inst) (only
 * mesh.nelx, mesh.nely and mesh.d are read; the same array a batch plan
 * takes) and uploads them to the current device, on which the filter must
 * then be used.  Host work and memory grow with n_cells * (R d)^2.  R > 0 and
 * finite.  MTO_EINVAL on bad arguments, MTO_ENOMEM (host or device). */
int mto_filter_create(const mto_problem* probs, int32_t n_inst, double R, mto_filter** out);

/* rho_tilde = W rho.  Device arrays of n_cells doubles, distinct (MTO_EINVAL
 * in place); asynchronous on stream. */
int mto_filter_apply(const mto_filter* filter, const double* rho, double* rho_tilde, void* stream);

/* g = W^T g_tilde (the chain rule).  Device arrays of n_cells doubles,
 * distinct (MTO_EINVAL in place); asynchronous on stream. */
int mto_filter_grad(const mto_filter* filter, const double* g_tilde, double* g, void* stream);

/* Number of cells and of nonzero H_ij (host outputs, may be NULL). */
int mto_filter_info(const mto_filter* filter, int64_t* n_cells, int64_t* nnz);

/* Frees the filter (NULL is a no-op). */
void mto_filter_destroy(mto_filter* filter);

#ifdef __cplusplus
}
#endif

#endif /* MTO_H */
