/*
 * ddfem.h -- C ABI of the MI355X domain-decomposed Whitney-edge Newmark solver.
 *
 * The library advances the edge-element wave equation
 *     T e'' + S e = -j'           (Sec. II-B: Whitney 1-forms, PEC walls)
 * with Newmark-beta (gamma = 1/2), one implicit solve per step:
 *     A e^{n+1} = (2A - dt^2 S) e^n - A e^{n-1} - dt (J^{n+1/2} - J^{n-1/2}),
 *     A = T + beta dt^2 S,
 * and solves each step with the dual-primal tearing of Sec. III-A
 * (MFETI-DP1 without the face unknowns): per-subdomain SPD blocks ordered
 * [interior | interface | corner], a signed Boolean interface map, an
 * unsigned corner map, a coarse corner problem and the interface Schur
 * system of eq. (f1schur), solved by conjugate gradients.
 *
 * Conventions
 *  - Edges are the unique vertex pairs (v_lo, v_hi), v_lo < v_hi, numbered
 *    lexicographically ("canonical edges").  An edge is on the conductor
 *    (PEC) iff it is an edge of a boundary face (a face of exactly one
 *    tetrahedron); PEC edges carry no unknown.
 *  - Field and current arrays are row-major [nrhs][n_edges] float64 in
 *    device memory; PEC entries are ignored on input and written as 0.
 *  - Host arrays are read during the call only; the library never keeps a
 *    caller pointer (except the stream).  The library owns everything it
 *    allocates and frees it in dd_destroy.
 *  - All device work of a call is enqueued on opt.stream (NULL = default
 *    stream).  Calls that must read device results on the host (convergence
 *    decisions, stats) synchronise that stream before returning.
 *  - Calls on one context are not thread safe.
 *  - Every int-returning call returns DD_OK (0) or a negative dd_status;
 *    dd_last_error() then returns a message (thread-local).
 */
#ifndef DDFEM_H
#define DDFEM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  DD_OK = 0,
  DD_ERR_ARG = -1,            /* bad argument (null pointer, size, beta <= 0, ...) */
  DD_ERR_MESH = -2,           /* vertex index out of range or degenerate tetrahedron */
  DD_ERR_PARTITION = -3,      /* subdomain id out of range or empty subdomain */
  DD_ERR_NOT_SPD = -4,        /* non-positive pivot; message names the subdomain */
  DD_ERR_NO_CONVERGENCE = -5, /* CG or refinement hit its cap (context stays usable) */
  DD_ERR_STATE = -6,          /* e.g. dd_step before dd_factor */
  DD_ERR_HIP = -7,            /* HIP runtime error (context must be destroyed) */
  DD_ERR_OOM = -8,            /* device or host allocation failed */
  DD_ERR_NONFINITE = -9       /* non-finite value in an input */
} dd_status;

typedef enum {
  DD_FP64 = 0,        /* factors, local solves and CG all in float64 */
  DD_FP32_REFINE = 1  /* float32 factors and local solves, float64 CG vectors,
                         float64 global residual and iterative refinement */
} dd_precision;

typedef struct {
  int precision;      /* dd_precision */
  int nrhs;           /* right-hand sides solved together, 1..32 */
  double cg_tol;      /* relative interface residual ||d - F lambda|| / ||d|| */
  int cg_max_iter;    /* cap on CG iterations per solve */
  double refine_tol;  /* relative global residual ||b - A e|| / ||b|| (FP32_REFINE) */
  int refine_max;     /* cap on refinement sweeps (FP32_REFINE) */
  int warm_start;     /* initial multipliers of a step's first CG solve: 0 zero, 1 the
                         previous step's, 2 linear extrapolation of the last two steps */
  int use_graph;      /* replay the CG iteration as a captured HIP graph */
  int check_every;    /* CG iterations between host convergence checks (>= 1; rounded up
                         to an even count, the unit a captured graph replays) */
  void* stream;       /* hipStream_t; NULL = default stream */
  int precond;        /* interface CG preconditioner: 0 none, 1 lumped (multiplicity-scaled
                         interface stiffness, sum_s D B_s A_GammaGamma^(s) B_s^T D, D = 1/2) */
  int method;         /* interface scheme: 0 dual-primal with one multiplier per interface
                         edge and CG (Sec. III-A); 1 Robin variant with one multiplier per
                         side and restarted GMRES (Sec. III-B, edge-only form); cg_tol and
                         cg_max_iter then bound the GMRES iterations, precond and
                         warm_start do not apply */
  double robin_alpha; /* method 1: Robin coefficient alpha of the transmission condition
                         lam_i + lam_j + 2 alpha M_T x_j = 0 (M_T the tangential mass of the
                         interface faces); 0 = automatic, (eps h + beta dt^2 / (mu h)) / 2
                         with h the mean edge length and eps, mu the mean material values */
  int diagnostics;    /* per-step checks of dd_step, reported in its stats; 0 = none;
                         bit 0 (DD_DIAG_GAUSS): the context accumulates the nodal charge
                         q^{n+1} = q^n + dt G^T J^{n+1/2} and evaluates the discrete Gauss
                         law G^T T e^{n+1} + q^{n+1} at every interior vertex (Sec. IV-B,
                         charge conservation); bit 1 (DD_DIAG_ENERGY): the discrete energy
                         H^{n+1/2} of (e^{n+1}, e^n) */
  const char* tune_cache; /* path of the work-list tuning cache (JSON lines), or NULL: with a
                         path, the first successful dd_factor runs dd_autotune with it
                         (string copied at dd_setup) */
} dd_options;

/* Work-list shapes of the batched products and what the tuner measured
 * (ms per solve's products of the class; *_default: with the shapes before
 * tuning). */
typedef struct {
  int chunk;          /* longest tile range of one wave: interface-block and corner-row lists */
  int coarse_chunk;   /* the same for the coarse inverse-factor lists */
  int full_chunk;     /* the same for the full r-block lists */
  int full_bucket;    /* length buckets of the full lists' workgroup placement */
  int full_persist;   /* full passes: workgroups of a persistent grid that walks the work
                         groups (a multiple of 8), or 0 for one workgroup per work group */
  int full_pair;      /* full passes, 9..32 RHS: 1 = each wave computes two output block rows
                         over the union of their tile lists, loading each input block once;
                         2 = eight rows per workgroup, the input block shared through LDS */
  int full_quarter;   /* full passes: 1 = the lanes of all-zero 16 x 16 quarters of a tile
                         read a cached zero tile instead of memory */
  int from_cache;     /* 1: read from the cache, no timing */
  double full_ms, full_ms_default, coarse_ms, coarse_ms_default;
  double trailing_ms, trailing_ms_default;  /* the corner-coupling passes Psi_Gamma u and
                                               Psi_Gamma^T z (tuned by `chunk`) */
  int sym_persist;    /* symmetric product of the interface operator: workgroups of a persistent
                         grid (a multiple of 8), or 0 for one workgroup per four work items; a
                         smaller grid leaves wave slots to the corner and coarse chain that runs
                         beside it */
  double local_ms, local_ms_default;  /* one local response (symmetric product beside the
                         corner and coarse chain), tuned and before tuning */
  int sym_pw;         /* symmetric product, FP32 factors: 2 = panels of two interface blocks (half
                         the accumulators per wave, twice the partial slots), 0 = four; FP64
                         factors always use two */
} dd_tuning;

enum { DD_DIAG_GAUSS = 1, DD_DIAG_ENERGY = 2 };

typedef struct {
  int cg_iters[32];        /* CG iterations of the last solve, per RHS */
  int refine_sweeps;       /* refinement sweeps of the last step */
  int dd_solves;           /* DD solves in the last step (1 + sweeps) */
  double cg_relres[32];    /* final relative interface residual, per RHS */
  double global_relres[32];/* final ||b - A e|| / ||b|| (FP32_REFINE), per RHS */
  int solve_iters[4];      /* max over RHS of the CG iterations of DD solves 1..4 of the step */
  int diagnostics;         /* the dd_options.diagnostics bits the fields below were computed for */
  double gauss_residual[32];/* DD_DIAG_GAUSS: max over interior vertices of |G^T T e^{n+1} + q^{n+1}| */
  double charge_max[32];   /* DD_DIAG_GAUSS: max over vertices of |q^{n+1}| (the scale of the above) */
  double energy[32];       /* DD_DIAG_ENERGY: H^{n+1/2} = |e^{n+1}-e^n|_T^2/dt^2 + |(e^{n+1}+e^n)/2|_S^2 */
} dd_stats;

/* Mesh of a context: host arrays, read during the call only. */
typedef struct {
  int64_t n_vertices;
  const double* coords;    /* [n_vertices][3] float64 */
  int64_t n_tets;
  const int32_t* tets;     /* [n_tets][4] int32, any vertex order */
} dd_mesh;

typedef struct {
  int64_t n_edges, n_interior, n_tets, n_vertices;
  int32_t n_sub, n_lambda, n_corner, nrhs, precision, tile;
  int64_t factor_bytes;    /* device bytes of all stored factors */
  int64_t trailing_bytes;  /* bytes of the interface blocks of the inverse factors
                              with the corner rows Psi_Gamma, unpadded (the
                              factorisation forms M and Psi_Gamma from them;
                              no solve pass reads the inverse blocks alone) */
  int64_t schur_bytes;     /* bytes of the interface blocks of the local inverses,
                              M = (K_rr^-1)_GammaGamma, packed lower triangle (read once
                              per CG iteration), unpadded */
  int64_t corner_bytes;    /* bytes of the corner rows Psi_Gamma (read twice per
                              CG iteration), unpadded */
  int64_t coarse_bytes;    /* bytes of the coarse inverse factor, unpadded */
  int64_t full_bytes;      /* bytes of the interior blocks L_II^-1 (their nonzero tiles' nonzero
                              entries once factored; dense before) */
  int64_t cross_bytes;     /* bytes of the couplings L_GammaI and L_cI of the interface and
                              corner rows to the interior (nonzero entries once factored) */
} dd_info;

/* Fill *opt with defaults: DD_FP64, nrhs 1, cg_tol 1e-10, cg_max_iter 500,
 * refine_tol 1e-12, refine_max 10, warm_start 0, use_graph 0, check_every 4,
 * precond 1, method 0, robin_alpha 0, diagnostics 0, tune_cache NULL. */
void dd_default_options(dd_options* opt);

/* Build a solver context (host analysis + device upload + element assembly
 * inputs).  Sec. III: the tetrahedra with partition[t] == s form subdomain
 * s; an edge shared by two subdomains is an interface edge (one Lagrange
 * multiplier, +1 in the lower subdomain id, -1 in the higher); an edge shared
 * by three or more is a corner (a primal unknown of the coarse problem).
 *   mesh      vertices and tetrahedra (host arrays, see dd_mesh)
 *   partition host [n_tets] int32 in [0, n_sub), every id used
 *   eps, mu   host [n_tets] float64 relative permittivity / permeability
 *             (> 0, finite); mu may be NULL (= 1)
 *   dt, beta  time step and Newmark beta (> 0, finite)
 * The accumulated nodal charge of DD_DIAG_GAUSS starts at zero.
 * Errors: DD_ERR_ARG, DD_ERR_MESH, DD_ERR_PARTITION, DD_ERR_NONFINITE,
 * DD_ERR_HIP, DD_ERR_OOM (also for a subdomain or coarse block of more than
 * 8193 32-row tiles).  On error *out is NULL. */
int dd_setup(void** out, const dd_mesh* mesh, const int32_t* partition, const double* eps,
             const double* mu, double dt, double beta, const dd_options* opt);

/* Sizes of a context. */
int dd_get_info(void* ctx, dd_info* info);

/* Number of canonical edges (the length of every field and current row). */
int dd_num_edges(void* ctx, int64_t* n_edges);

/* Canonical edges: host [n_edges][2] int32 (v_lo, v_hi) and host [n_edges]
 * uint8 PEC flags.  Either pointer may be NULL. */
int dd_get_edges(void* ctx, int32_t* edges, uint8_t* is_pec);

/* Replace the per-tetrahedron permittivity ([n_tets] float64, a host array,
 * or a device array if on_device != 0; validated on the host either way:
 * DD_ERR_NONFINITE / DD_ERR_ARG for a non-finite or non-positive entry);
 * dd_factor must be called again before the next solve.  Synchronises. */
int dd_set_eps(void* ctx, const double* eps, int on_device);

/* Element matrices, per-subdomain assembly [I | Gamma | c], partial Cholesky
 * of the r = I u Gamma block with the local corner Schur complement
 * K_s = A_cc - L_cr L_cr^T (Sec. III-A, eq. (cF1)), inversion of the
 * triangular factors (the stored local inverses of Sec. III-C), assembly and
 * factorisation of the coarse corner matrix K_cc = sum_s B_c^T K_s B_c
 * (eq. (F1uc)).  Synchronises the stream.  DD_ERR_NOT_SPD names the first
 * subdomain with a non-positive or non-finite pivot (for instance material
 * values whose matrix entries overflow the factor precision); the context
 * then refuses solves (DD_ERR_STATE) until a dd_factor succeeds. */
int dd_factor(void* ctx);

/* Autotuner of the batched launches (every subdomain and right-hand side in
 * one launch per product class; work items of at most `chunk` tiles, placed
 * per XCD).  With cache_path (JSON lines, one object per tuning) holding an
 * entry for this context's key (device, precision, nrhs, subdomain tile
 * shapes, nonzero-tile pattern) the entry is applied; otherwise every
 * candidate shape of each class is timed with HIP events on the context
 * stream (the products of one decomposed solve, median of 5), the fastest
 * is applied and, given a path, appended to the cache.  Needs a factorised
 * context (DD_ERR_STATE); synchronises; out may be NULL. */
int dd_autotune(void* ctx, const char* cache_path, dd_tuning* out);

/* Resident Newmark state (for callers that advance the fields step after
 * step, as a PIC loop does): the context keeps e^n, e^{n-1} and J^{n-1/2}
 * in its own unknown-major layout together with the products T e and S e of
 * both iterates (Sec. II-B-2: the load of step n needs exactly these), so a
 * dd_step_resident converts only J^{n+1/2} and e^{n+1} and assembles its
 * load without a sparse product; the products of the new iterate come from
 * the refinement's last residual.  Each state belongs to its context; a new
 * factorisation (dd_factor, dd_set_eps) recomputes the stored products.
 *
 * dd_state_set: load the state from device arrays [nrhs][n_edges] E_n = e^n,
 * E_nm1 = e^{n-1}, J_prev_half = J^{n-1/2}; each may be NULL for zero (the
 * state before the first step, reading of Sec. II-B-2: e^0 = e^{-1} = 0).
 * A context whose state was never set starts from zero.  Needs a factorised
 * context (DD_ERR_STATE).
 * dd_step_resident: one Newmark step of the state with J_half = J^{n+1/2}
 * (device [nrhs][n_edges]); writes e^{n+1} to E_next (device [nrhs][n_edges])
 * and advances the state (e^{n+1}, e^n, J^{n+1/2}).  The result equals
 * dd_step's for the same fields; stats, diagnostics and errors as for
 * dd_step (on DD_ERR_NO_CONVERGENCE the state advances to the last
 * iterate).  Calls on one context are not reentrant. */
int dd_state_set(void* ctx, const double* E_n, const double* E_nm1, const double* J_prev_half);
int dd_step_resident(void* ctx, const double* J_half, double* E_next, dd_stats* stats);

/* One Newmark step for all nrhs right-hand sides (device pointers):
 *   J_half, J_prev_half  [nrhs][n_edges]: J^{n+1/2}, J^{n-1/2}
 *   E_n, E_nm1           [nrhs][n_edges]: e^n, e^{n-1}
 *   E_next               [nrhs][n_edges]: e^{n+1} (output; may not alias inputs)
 * stats: host pointer or NULL; with dd_options.diagnostics set it also
 * receives the Gauss residual and/or the energy of this step (the charge
 * update runs whether stats is given or not).  DD_ERR_NO_CONVERGENCE leaves
 * E_next holding the last iterate and the context usable.
 * DD_ERR_NONFINITE: the right-hand side assembled from the inputs has a
 * non-finite entry (its RHS is named in the message). */
int dd_step(void* ctx, const double* J_half, const double* J_prev_half,
            const double* E_n, const double* E_nm1, double* E_next, dd_stats* stats);

/* x = A^{-1} b on canonical-edge arrays [nrhs][n_edges] (device), through the
 * same decomposed solve (with refinement in DD_FP32_REFINE). */
int dd_solve(void* ctx, const double* b, double* x, dd_stats* stats);

/* One reverse step of the recurrence (A is symmetric, so the factors are
 * reused; the reverse of the three-level Newmark form of Sec. II-B-2).
 * With ebar_next the total adjoint of e^{n+1}:
 *   g = A^{-1} ebar_next;  ebar_n += (2A - dt^2 S) g;  ebar_nm1 -= A g;
 *   eps_bar[k] -= g . T_k (e^{n+1} - 2 e^n + e^{n-1})   (T_k: unit-eps mass)
 * summed over the right-hand sides, and, because the load of step n is
 * -dt (J^{n+1/2} - J^{n-1/2}):
 *   Jbar_half += -dt g   (adjoint of J^{n+1/2}),  Jbar_prev_half += dt g
 * on the unknowns (conductor entries are left as they are).  All pointers
 * are device pointers; arrays are [nrhs][n_edges] except eps_bar [n_tets]
 * (accumulated).  ebar_n, ebar_nm1, g_out, eps_bar, Jbar_half and
 * Jbar_prev_half may be NULL (skipped).  E_nm1 NULL means e^{n-1} = 0. */
int dd_adjoint_step(void* ctx, const double* ebar_next, double* ebar_n, double* ebar_nm1,
                    double* g_out, const double* E_next, const double* E_n,
                    const double* E_nm1, double* eps_bar, double* Jbar_half,
                    double* Jbar_prev_half, dd_stats* stats);

/* Accumulated nodal charge of DD_DIAG_GAUSS: q (device [nrhs][n_vertices]
 * float64, entries of boundary vertices ignored) or NULL for zero; set it
 * to the charge of the state e^n that the next dd_step starts from. */
int dd_set_charge(void* ctx, const double* q);

/* Discrete Gauss law (Sec. IV-B charge conservation), device pointers:
 *   dd_charge_update:  q += dt * G^T J_half   (q [nrhs][n_vertices], entries
 *                      of boundary vertices stay 0; G: +1 at the higher-id end)
 *   dd_gauss_residual: res[r] = max_k |(G^T T e + q)_k| over interior vertices
 *                      (res: host [nrhs]); synchronises. */
int dd_charge_update(void* ctx, const double* J_half, double* q);
int dd_gauss_residual(void* ctx, const double* E, const double* q, double* res);

/* Discrete energy H^{n+1/2} = |e^{n+1}-e^n|_T^2 / dt^2 + |(e^{n+1}+e^n)/2|_S^2
 * per RHS (host out [nrhs]); synchronises. */
int dd_energy(void* ctx, const double* E_next, const double* E_n, double* out);

/* ---- particle steps around the field solve (Sec. II-A) ------------------
 * Particles are delta shapes: charge measured by the vertex hat functions,
 * current by the Whitney edge functions.  All pointers are device pointers;
 * positions and velocities are [n][3] float64 row-major; cell[p] is a
 * tetrahedron index in the dd_setup order, or -1 for an inactive particle.
 * Mesh tables for these calls (face neighbours, per-tetrahedron geometry)
 * are built on the first call (allocates and synchronises once).  After
 * that the particle calls only enqueue work on the context stream: what
 * they find (absorbed particles, bad indices) goes to device counters that
 * dd_pic_status reads. */

/* Counters of the particle calls since the last reset:
 *   counts[0]  particles absorbed at the outer boundary (deposit) and
 *              points found outside the mesh (locate)
 *   counts[1]  walks stopped after 65536 faces (particle made inactive)
 *   counts[2]  cell or permutation indices out of range (made inactive /
 *              item left unwritten)
 * counts: host [3] or NULL.  Synchronises the stream; reset != 0 zeroes the
 * counters afterwards. */
int dd_pic_status(void* ctx, int64_t* counts, int reset);

/* Point location.  On entry cell[p] names a start tetrahedron (-1 or out of
 * range: tetrahedron 0); on return the tetrahedron holding x[p], found by
 * walking the straight line from the start cell's centroid across shared
 * faces, or -1 if that line leaves the mesh (x outside it, or a non-convex
 * mesh in the way; counted in counts[0]). */
int dd_pic_locate(void* ctx, int64_t n, const double* x, int32_t* cell);

/* Exact current mapping of the straight paths xa[p] -> xb[p] (Sec. II-A):
 *   J[e] += (q[p] / dt) * int_{xa_p}^{xb_p} W_e . dl
 * J is one right-hand side's row [n_edges] (canonical edges; entries of
 * conductor edges are written too and ignored by the solve).  cell[p] must
 * hold xa[p] on entry; on return it holds xb[p].  A path that reaches the
 * outer boundary deposits up to it and the particle becomes inactive
 * (cell = -1, counts[0]): on a conductor wall the interior Gauss law stays
 * exact.  Inactive particles are skipped.  The summation order over
 * particles is not fixed (device atomics), so J is reproducible to rounding,
 * not bit for bit.  A cell index out of range (counts[2]) or a path crossing
 * more than 65536 faces (counts[1]) makes the particle inactive. */
int dd_pic_deposit(void* ctx, int64_t n, const double* xa, const double* xb, const double* q,
                   int32_t* cell, double* J);

/* Order of the particles by cell (counting sort over the tetrahedra):
 * perm[i] = the particle that goes to place i; cells ascending, inactive
 * particles (cell -1 or out of range) last, order within one cell
 * unspecified.  Apply it to every per-particle array (cell included) with
 * dd_pic_permute.  With particles in cell order the deposit's
 * contributions to one edge meet in registers and in LDS before its device
 * atomics, and the push's field gathers hit the cache; particles move a
 * fraction of a cell per step, so an order lasts many steps.
 * n <= 2^31 - 1. */
int dd_pic_sort(void* ctx, int64_t n, const int32_t* cell, int32_t* perm);

/* dd_pic_sort for callers that cannot allocate (code under HIP graph
 * capture, tight serving loops, harnesses that forbid device allocation):
 * the same ordering (same contract as dd_pic_sort), with every scratch
 * buffer in one fixed static device array of the library (16.0 MiB per
 * device, held until the process ends) instead of context memory; it calls
 * no allocating routine and does not build the particle tables of the other
 * particle calls.  Limit: meshes of at most 4194304 tetrahedra (DD_ERR_ARG
 * beyond).  Every call on one device shares that device's array and leaves
 * its contents behind (the call clears what must start at zero itself), so
 * calls that overlap in time on one device race; serialise them (one stream,
 * or events).  Enqueued on the context stream, never synchronises. */
int dd_pic_sort_noalloc(void* ctx, int64_t n, const int32_t* cell, int32_t* perm);

/* dst[i] = src[perm[i]] for n items of item_bytes bytes (a multiple of 4,
 * at most 64; 4-byte aligned device arrays that do not overlap).  A perm
 * entry outside [0, n) leaves that item unwritten (counts[2]). */
int dd_pic_permute(void* ctx, int64_t n, const int32_t* perm, int item_bytes, const void* src,
                   void* dst);

/* Faraday's law on the face 2-form of B, kept as its constant value in each
 * tetrahedron: B_r[t] += alpha * curl(E_r)|_t with curl W_ij = 2 g_i x g_j
 * (alpha = -dt for one step) for rows r < nrows.  E: [nrows][n_edges];
 * B: [nrows][n_tets][3]. */
int dd_pic_faraday(void* ctx, int nrows, const double* E, double alpha, double* B);

/* Field interpolation at x[p] in cell[p] (E = sum_e E[e] W_e, B = B[cell])
 * and one Adams-Bashforth step of x' = v, v' = qm (E + v x B), qm [n] the
 * charge-to-mass ratios, dt the context's step:
 *   first != 0: x_new = x + dt v,  v += dt acc   (start step)
 *   otherwise:  x_new = x + dt (3/2 v - 1/2 v_prev),  v += dt (3/2 acc - 1/2 acc_prev)
 * hist [n][6] = (v_prev, acc_prev) is overwritten with (v, acc).  x_new must
 * not overlap x.  Inactive particles keep x (copied to x_new) and v; a
 * cell index out of range is treated the same way and counted (counts[2]). */
int dd_pic_push(void* ctx, int64_t n, const double* qm, const double* E, const double* B,
                const int32_t* cell, const double* x, double* x_new, double* v, double* hist,
                int first);

/* ---- the mixed E/B step (Sec. II-B-1) -------------------------------------
 * E on edges (Whitney 1-forms), B on faces (Whitney 2-forms, W_ijk =
 * 2 (lam_i g_j x g_k + lam_j g_k x g_i + lam_k g_i x g_j) for a face with
 * vertices i < j < k), advanced by the trapezoid rule:
 *   T (e+ - e)/dt = C^T M (b+ + b)/2 - J^{n+1/2},   (b+ - b)/dt = -C (e+ + e)/2,
 * C the discrete curl (boundary of face (i,j,k) = (i,j) + (j,k) - (i,k)), M the
 * 1/mu 2-form mass.  Eliminating b+ leaves (T + dt^2/4 S) e+ = (T - dt^2/4 S) e
 * + dt C^T M b - dt J, the matrix of the decomposed solve with beta = 1/4, so
 * the step is one decomposed solve between a face-side right-hand side and
 * the face update.  Face tables are built on the first call (host sort,
 * allocations of 8 n_tets (3 + 6 nrhs) bytes). */

/* Canonical faces: *n_faces (may be NULL) and host [n_faces][3] int32 vertex
 * triples ascending, numbered lexicographically (faces may be NULL). */
int dd_mixed_faces(void* ctx, int64_t* n_faces, int32_t* faces);

/* One trapezoid step for all nrhs right-hand sides (device pointers):
 *   J_half [nrhs][n_edges]: J^{n+1/2};  E_n, E_next [nrhs][n_edges];
 *   B_n, B_next [nrhs][n_faces] (face fluxes; outputs must not alias inputs).
 * DD_ERR_STATE before dd_factor or unless the context's beta is 1/4;
 * DD_ERR_NO_CONVERGENCE as for dd_step. */
int dd_step_mixed(void* ctx, const double* J_half, const double* E_n, const double* B_n,
                  double* E_next, double* B_next, dd_stats* stats);

/* Per-class timing of the batched tile products, measured with HIP events
 * recorded on the context's stream around each launch (adds two event
 * records per launch while enabled; the symmetric product's events are
 * attached to its kernel dispatch instead, so they time its execution).
 * Classes: */
enum {
  DD_PROF_TRAILING = 0, /* no launches (kept for the numbering): no pass applies the interface
                           blocks of the inverse factors alone; the solves use M below */
  DD_PROF_FULL = 1,     /* interior inverse-factor products L_II^-1, L_II^-T (pre-solve, recovery) */
  DD_PROF_SCHUR = 2,    /* interface blocks of the local inverses, M u: the symmetric product
                           kernel alone, without the reduce of its partials (once per CG
                           iteration, once in the pre-solve and in the recovery) */
  DD_PROF_COARSE = 3,   /* coarse corner inverse factor */
  DD_PROF_CORNER = 4,   /* corner rows Psi_Gamma u and Psi_Gamma^T z (twice per CG iteration,
                           pre-solve and recovery) */
  DD_PROF_CROSS = 5,    /* couplings L_GammaI, L_cI of interface and corner rows to the interior
                           (pre-solve, recovery) */
  DD_PROF_CLASSES = 6
};
/* Returns the accumulated milliseconds and launch counts per class (host
 * arrays [DD_PROF_CLASSES], either may be NULL) since the last reset, then
 * sets timing on (enable = 1) or off (0) and resets the counters; enable = -1
 * only reads.  Synchronises the stream. */
int dd_profile(void* ctx, int enable, double* ms, int64_t* launches);

void dd_destroy(void* ctx);

/* Message of the last error on this thread ("" if none). */
const char* dd_last_error(void);

/* ---- host-only analysis (no device calls; usable without a GPU) -------- */
typedef struct {
  int64_t n_edges, n_interior;
  int32_t n_sub, n_lambda, n_corner, max_multiplicity;
  int64_t sum_nr3;         /* sum over subdomains of n_r^3 */
} dd_analysis;

/* Partition analysis of Sec. III (interior / interface / corner classes).
 * per_sub (host [n_sub][3] int32, may be NULL) receives n_I, n_Gamma, n_c. */
int dd_analyze(const dd_mesh* mesh, const int32_t* partition, dd_analysis* out,
               int32_t* per_sub);

/* Interface map of the same analysis: for each multiplier l (host arrays
 * [n_lambda]): its canonical edge, the two subdomains (lo < hi) and the
 * positions of the edge in their local orders (0-based within the
 * [I | Gamma | c] order, unpadded).  The multiplier enters subdomain lo with
 * +1 and hi with -1. */
int dd_analyze_lambda(const dd_mesh* mesh, const int32_t* partition,
                      int32_t* edge, int32_t* sub_lo, int32_t* sub_hi,
                      int32_t* pos_lo, int32_t* pos_hi);

#ifdef __cplusplus
}
#endif
#endif /* DDFEM_H */
