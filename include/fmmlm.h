/*
 * fmmlm.h -- C ABI of the MI355X (gfx950) fast multipole method for the 3-D
 * Laplace equation in layered media (Wang, Zhang & Cai, arXiv:1908.10863).
 *
 * Problem (Sec. 3.1): a stack of L interfaces z = d_0 > d_1 > ... > d_{L-1}
 * separates L+1 layers; layer l is d_l < z < d_{l-1} (layer 0 on top, layer L
 * at the bottom) with permittivity eps_l.  Charges Q_j sit at r_j inside layer
 * layer_id[j].  fmm_layered_eval returns, for every charge i in layer l,
 *
 *   Phi_i = sum_{j != i, layer j = l} Q_j / (4 pi |r_i - r_j|)           (free)
 *         + sum_{all j, incl. j = i} Q_j u^r_{l, layer j}(r_i, r_j)     (reaction)
 *
 * (eqs. potential1 / totalinteraction), where the reaction Green's function is
 * the sum of the four reaction components of eq. reactioncomponent, each a
 * Sommerfeld integral of eq. generalcomponents with the densities of App. A
 * (interface conditions: u and eps du/dz continuous).  The 1/(4 pi) factor is
 * included in both parts.
 *
 * Conventions shared by every call:
 *  - All functions return FMMLM_OK (0) or a negative error code; nothing is
 *    thrown across the ABI.  fmm_layered_strerror turns a code into text; the
 *    last HIP error message is kept per thread and appended.
 *  - "host" pointers are ordinary CPU memory; "device" pointers are HIP device
 *    memory of the current device (e.g. torch tensors' data_ptr()).
 *  - hip_stream is a hipStream_t passed as void* (NULL = the default stream).
 *    Plan-time work is synchronised before fmm_layered_plan returns;
 *    fmm_layered_eval is asynchronous on hip_stream.
 */
#ifndef FMMLM_H
#define FMMLM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- error codes ---------------------------------------------------------- */
#define FMMLM_OK 0
#define FMMLM_EINVAL (-1)        /* null pointer, n < 1, nrhs out of range, p out of range, bad option */
#define FMMLM_EINTERFACES (-2)   /* interfaces not strictly decreasing or not finite */
#define FMMLM_EEPS (-3)          /* a permittivity is <= 0 or not finite */
#define FMMLM_ELAYER (-4)        /* layer_id out of range or a point outside its layer */
#define FMMLM_EONINTERFACE (-5)  /* a point lies on an interface (Sommerfeld integrals diverge) */
#define FMMLM_EDEVICE (-6)       /* a HIP call failed */
#define FMMLM_ENOMEM (-7)        /* host or device allocation failed, or a list exceeds its limit */
#define FMMLM_EUNSUPPORTED (-8)  /* option combination not built */
#define FMMLM_EBUSY (-9)         /* the plan is in use: another call is enqueuing work on it, or its
                                    last evaluation, enqueued on another stream, has not finished */

/* ---- options --------------------------------------------------------------- */
#define FMMLM_PMAX 16            /* largest truncation order p (n = 0..p) */
#define FMMLM_MAX_INTERFACES 12  /* largest L */

#define FMMLM_FP64 0             /* every kernel in FP64 */
#define FMMLM_FP32_COMPENSATED 1 /* P2P and M2L in FP32 with compensated sums (see fmmlm_opts) */

#define FMMLM_FREE 1u            /* parts bit: free-space component */
#define FMMLM_REACTION 2u        /* parts bit: reaction components */

typedef struct fmmlm_plan_s* fmmlm_plan_t;
typedef struct fmmlm_surrogate_s* fmmlm_surrogate_t;

typedef struct {
  int32_t leaf_cap;        /* a box is split while it holds more points (default 64) */
  int32_t precision;       /* FMMLM_FP64 (default) or FMMLM_FP32_COMPENSATED */
  int32_t fp64_top_levels; /* tree levels 0..k-1 whose M2L runs in the sparse FP64 kernel
                              (default 3); the FP32 form keeps these levels in FP64 */
  int32_t max_rhs;         /* largest nrhs accepted by eval (default 1).  Above 1 the plan
                              holds expansions for G = min(max_rhs, 64) charge vectors and
                              evaluates them together (batched M2L on the matrix cores in
                              the FP32 form, one 1/r per pair for all vectors in P2P);
                              device memory grows by about G times the single-vector
                              expansion and point arrays */
  int32_t mac_d2;          /* multipole acceptance: two same-level boxes exchange expansions
                              only if their centres are at least sqrt(mac_d2) box sizes apart
                              (and not adjacent); 4 is the classic one-box separation.
                              Range 4..12, default 6 */
  int32_t graph;           /* 1: fmm_layered_eval captures its kernel launches into a HIP graph
                              on the first call and replays the graph while nrhs, q, ldq, phi,
                              ldphi, parts and the stream stay the same (a change captures
                              anew).  Needs a stream other than the null stream (on the null
                              stream evaluations launch directly).  Not used while profiling.
                              Default 0 */
  int32_t reserved[2];     /* must be 0 */
  fmmlm_surrogate_t surrogate; /* learned form (default NULL = quadrature): a trained network
                              for this medium serves the reaction Sommerfeld initial values
                              and near-field kernels inside its domain, the quadrature the
                              rest (see fmm_layered_surrogate_train).  The plan does not
                              keep the handle after it returns */
} fmmlm_opts;

/* Fills *opts with the defaults listed above. */
void fmmlm_default_opts(fmmlm_opts* opts);

/* ---- plan ------------------------------------------------------------------ */
/*
 * Builds an immutable plan for one geometry (Algorithm 2's set-up: trees,
 * interaction lists, M2L operators with the Sommerfeld recurrence of
 * eq. recurrence, near-field reaction kernels).
 *
 *  n_interfaces   L >= 1 (<= FMMLM_MAX_INTERFACES)
 *  z_interfaces   [L] host or device, strictly decreasing, finite
 *  eps            [L+1] host or device, > 0, top to bottom
 *  n              number of charges, 1 <= n < 2^31
 *  x, y, z        [n] host or device, SoA coordinates (FP64)
 *  layer_id       [n] host or device, 0..L, with d_l < z < d_{l-1}
 *  p              truncation order, 1..FMMLM_PMAX (expansions hold (p+1)^2 terms)
 *  opts           NULL for defaults
 *  hip_stream     stream for plan-time kernels
 *  out            receives the plan; the caller owns it and frees it with
 *                 fmm_layered_destroy.  Geometry is deep-copied: the caller may
 *                 free its arrays after return.
 *
 * Errors: FMMLM_EINVAL, FMMLM_EINTERFACES, FMMLM_EEPS, FMMLM_ELAYER,
 * FMMLM_EONINTERFACE (|z - d| below 1e-12 of the root box size),
 * FMMLM_EDEVICE, FMMLM_ENOMEM.  On error *out is NULL.
 */
int fmm_layered_plan(int32_t n_interfaces, const double* z_interfaces, const double* eps,
                     int64_t n, const double* x, const double* y, const double* z,
                     const int32_t* layer_id, int32_t p, const fmmlm_opts* opts,
                     void* hip_stream, fmmlm_plan_t* out);

/* ---- evaluation ------------------------------------------------------------- */
/*
 * One matrix-vector product per charge vector: phi = G q (eq. totalinteraction).
 *
 *  nrhs           1..opts.max_rhs charge vectors, evaluated together in passes of
 *                 G = min(max_rhs, 64)
 *  q              device, q[r * ldq + j] for r < nrhs, j < n (user order, FP64)
 *  ldq            >= n
 *  phi            device, phi[r * ldphi + i], overwritten (FP64)
 *  ldphi          >= n; phi must not overlap q
 *  parts          FMMLM_FREE | FMMLM_REACTION (both = total potential)
 *  hip_stream     all work is enqueued here; nothing is synchronised
 *
 * The plan owns one workspace: evaluations of one plan must not overlap in
 * time (enqueue them on one stream).  An evaluation is refused with
 * FMMLM_EBUSY while another host thread is inside fmm_layered_eval or
 * fmm_layered_solve on the plan, or when the plan's last evaluation was
 * enqueued on another stream and has not finished (the check uses an event
 * recorded after each evaluation; it is skipped while hip_stream is being
 * captured into a graph).  Errors: FMMLM_EINVAL (null plan, q or phi; nrhs
 * outside 1..max_rhs; ldq or ldphi below n; parts empty or with unknown bits),
 * FMMLM_EBUSY, FMMLM_EDEVICE.
 */
int fmm_layered_eval(fmmlm_plan_t plan, int32_t nrhs, const double* q, int64_t ldq,
                     double* phi, int64_t ldphi, uint32_t parts, void* hip_stream);

/* Frees the plan and its device memory (NULL is a no-op).  Synchronises the
 * device first so that in-flight evaluations finish. */
int fmm_layered_destroy(fmmlm_plan_t plan);

/*
 * A plan for the general interface conditions of App. A (eq.
 * generalinterfacecond):
 *
 *   a_{l-1} u_{l-1} = a_l u_l,   b_{l-1} du_{l-1}/dz = b_l du_l/dz   at z = d_{l-1},
 *
 * for l = 1..L, with the same decay at z -> +-infinity; the classic
 * transmission conditions are a_l = 1, b_l = eps_l.  Only the reaction
 * densities change.  With v = a u in every layer the conditions become the
 * classic ones for v with permittivities b / a and a source of strength a in
 * the source layer, so each density is a_{l'} / a_l times the classic density
 * for eps = b / a (target layer l, source layer l'), and every kernel of the
 * classic plan serves unchanged.
 *
 *  a, b   host or device, n_interfaces + 1 coefficients each (top to bottom),
 *         finite and > 0 (FMMLM_EEPS otherwise)
 *  the other arguments are those of fmm_layered_plan; evaluation, solve and
 *  destruction are the same calls.  opts.surrogate must be NULL (the learned
 *  form is built for the classic conditions): FMMLM_EUNSUPPORTED otherwise.
 */
int fmm_layered_plan_general(int32_t n_interfaces, const double* z_interfaces, const double* a, const double* b,
                             int64_t n, const double* x, const double* y, const double* z,
                             const int32_t* layer_id, int32_t p, const fmmlm_opts* opts, void* hip_stream,
                             fmmlm_plan_t* out);

/* ---- iterative solve around the matvec ------------------------------------------ */
/*
 * The paper's motivating application (Sec. 1): a dense system whose product is
 * the layered-media potential, solved by GMRES with the FMM as the matvec.
 * fmm_layered_solve solves the second-kind system
 *
 *   (diag(diag) + G) x = b,      G x = fmm_layered_eval(x) (both parts),
 *
 * by restarted GMRES (Saad & Schultz, SIAM J. Sci. Stat. Comput. 7 (1986)):
 * Arnoldi with classical Gram-Schmidt applied twice, Givens rotations for the
 * least-squares problem, the true residual recomputed at each restart.  All
 * vector work runs on the device in FP64 with fixed-order reductions (the
 * result is reproducible for a given plan); the small Hessenberg problem is
 * solved on the host, which reads k + 2 values per Arnoldi step.
 *
 *  diag       device, n values in user order, or NULL for a zero diagonal
 *             (e.g. the self term of a collocation panel)
 *  b          device, n values (user order)
 *  x          device, n values: the initial guess on entry (ignored when
 *             opts.zero_guess), the solution on return; must not overlap b
 *  opts       NULL for the defaults (restart 30, max_iters 300, tol 1e-6,
 *             zero_guess 0)
 *  hip_stream all device work is enqueued here; the call returns after it has
 *             finished (it synchronises hip_stream once per Arnoldi step)
 *  info       host, filled on FMMLM_OK (also when not converged)
 *
 * The reachable tolerance is bounded by the plan's matvec accuracy (about
 * 1e-5 relative for the FP32 form at p = 10) times the system's conditioning.
 * Workspace: (restart + 1) n doubles plus small buffers, allocated and freed
 * by the call.  Evaluations of the plan must not overlap the call.
 * Errors: FMMLM_EINVAL (null plan, b, x or info; restart outside 1..256;
 * max_iters < 1; tol not in (0, 1); x overlapping b), FMMLM_EBUSY (as for
 * fmm_layered_eval), FMMLM_ENOMEM, FMMLM_EDEVICE.  With the plan's graph option every step captures anew (the
 * vectors change from step to step): leave it off for solves.
 */
typedef struct {
  int32_t restart;     /* Krylov vectors per cycle, 1..256 (default 30) */
  int32_t max_iters;   /* Arnoldi steps in all, >= 1 (default 300) */
  double tol;          /* stop when ||b - (diag + G) x|| <= tol ||b|| (default 1e-6) */
  int32_t zero_guess;  /* 1: start from x = 0 (no matvec for the first residual) */
  int32_t reserved;
} fmmlm_solve_opts;

typedef struct {
  int32_t iters;       /* Arnoldi steps (one matvec each) */
  int32_t matvecs;     /* evaluations in all (Arnoldi steps + true residuals) */
  int32_t cycles;      /* restart cycles run */
  int32_t converged;   /* 1 when the final true residual meets tol */
  double relres;       /* final true ||b - (diag + G) x|| / ||b|| */
  double relres_est;   /* the GMRES estimate at the last Arnoldi step */
  double seconds;      /* wall time of the call */
} fmmlm_solve_info;

int fmm_layered_solve(fmmlm_plan_t plan, const double* diag, const double* b, double* x,
                      const fmmlm_solve_opts* opts, void* hip_stream, fmmlm_solve_info* info);

/* Static text for an error code, followed by the calling thread's last HIP
 * error message when there is one.  Never NULL. */
const char* fmm_layered_strerror(int code);

/* ---- introspection (tests, benchmarks) --------------------------------------- */
typedef struct {
  int64_t n_points;            /* n */
  int64_t n_tree_points;       /* points over all interface-anchored trees */
  int32_t n_trees;             /* 2L anchored trees */
  int32_t p;
  int32_t max_level;           /* deepest box level */
  int32_t precision;
  int64_t n_boxes;
  int64_t n_leaves;
  int64_t m2l_free_pairs;      /* source box -> target box free-space translations */
  int64_t m2l_reaction_pairs;  /* reaction-component translations */
  int64_t p2p_free_pairs;      /* particle pairs in the free-space near field */
  int64_t p2p_reaction_pairs;  /* particle pairs in the reaction near field */
  int64_t n_free_ops;          /* distinct free-space M2L operators */
  int64_t n_reaction_ops;      /* distinct reaction M2L operators */
  int64_t n_sommerfeld_tasks;  /* distinct (component, level, rho, z) integral sets */
  double root_side;            /* common root box side W */
  double x0, y0;               /* common xy origin */
  double plan_seconds;         /* wall time of fmm_layered_plan */
  int64_t device_bytes;        /* device memory held by the plan */
  double tree_seconds;         /* plan phases: anchored trees, Morton keys and sort */
  double lists_seconds;        /*   boxes, interaction lists, M2L tiles, P2P lists */
  double ops_seconds;          /*   M2L operators (free and reaction, incl. table_seconds) */
  double table_seconds;        /*   Sommerfeld initial values + recurrence of the reaction M2L */
  double nearfield_seconds;    /*   reaction near-field kernel values */
  int64_t surrogate_tasks;     /* learned form: Sommerfeld tasks served by the network ... */
  int64_t surrogate_pairs;     /*   ... and near-field pairs (the rest took the quadrature) */
  double surrogate_check;      /*   learned (or table) form against the quadrature on up to
                                    256 sampled tasks: the largest R1 max_{N,M} 0.87^N
                                    |difference of S^N I_{N,M}|, R1 = |(rho, z + zinf)| (the error
                                    relative to the interaction 1/R1 that the operator carries).
                                    Above 1e-5 the plan rejects the form (surrogate_rejected) */
  int64_t m2l_steps;           /* M2L GEMM steps (one operator applied to one chunk's sources) ... */
  int32_t m2l_tile_cols;       /*   ... of this many target columns: the fill of the steps is
                                    (m2l_free_pairs + m2l_reaction_pairs - m2l_top_pairs)
                                    / (steps * cols) */
  int32_t m2l_variant;         /* FP32 form: M2L tile shape picked by the plan's autotuner (see m2l_eval_ms) */
  int64_t m2l_top_pairs;       /* M2L pairs on the top levels (fp64_top_levels), run by the
                                    sparse FP64 kernel in the "M2L top" stage */
  double m2l_variant_ms[6];    /* autotuner: time of one M2L launch alone in each tile shape (outputs
                                  per wave, rows x columns, operator columns per LDS slice; 0: 16
                                  waves of 32 x 32, slices of 32; 1: 8 of 32 x 64; 2: 8 of 64 x 32;
                                  3: 16 of 32 x 32; 4: 16 of 64 x 16; 5: 16 of 64 x 16, slices of
                                  32; slices of 16 otherwise, and where the padded column count is
                                  not a multiple of 32; (p+1)^2 <= 128 only, else unused) */
  int32_t batch_variant;       /* batched FP32 form: M2L variant picked by the autotuner ... */
  int32_t surrogate_rejected;  /* 1 when the plan's surrogate (network or tables) missed
                                    surrogate_check <= 1e-5 on the plan's sampled tasks and the
                                    quadrature served the whole plan instead */
  double batch_variant_ms[10]; /*   ... and one launch's time in each: variant v has the tile shape
                                  v % 5 (outputs per wave over operator rows x 64 vectors; 0: 4 waves
                                  of 64 x 32, 1: 8 of 32 x 32, 2: 8 of 64 x 16, 3: 16 of 32 x 16,
                                  4: 16 of 16 x 32) as one block per target box (v < 5) or as a
                                  persistent XCD-aware grid (v >= 5); (p+1)^2 <= 128 only */
  double m2l_eval_ms[6];       /* FP32 form: time of a whole unprofiled evaluation (near field and
                                  sparse top levels on their streams beside the main M2L) with
                                  each tile shape; m2l_variant is the fastest of these */
  double p2p_split_ms[5];      /* FP32 form: the same time with 100, 75, 50, 25 and 0 percent of
                                  the free P2P leaves launched at the fork and the rest after the
                                  main M2L launch ... */
  int32_t p2p_split_pct;       /*   ... and the percentage kept (the fastest) */
  int32_t batch_min_rhs;       /* batched passes narrower than this run vector by vector
                                  (timed at plan time: one batched pass of max_rhs vectors
                                  against one single-vector evaluation) */
  int32_t p2p_lds_reserve;     /* FP32 form: bytes of LDS each free P2P block reserves beyond its
                                  own use when it runs beside the far field (unprofiled
                                  evaluations): the fastest of the candidates timed in
                                  p2p_reserve_ms; it bounds the P2P blocks a CU holds and leaves
                                  room for far-field blocks beside them */
  double p2p_reserve_ms[3];    /*   ... whole-evaluation times with 28672, 40960 and 0 bytes */
  int64_t m2l_chunks;          /* M2L chunks below the top levels: each holds up to m2l_tile_cols
                                  targets and one step per operator of its group (up to 4
                                  operators that reach the same targets), and stores one partial
                                  sum per target for all its steps */
} fmmlm_stats;

int fmm_layered_plan_stats(fmmlm_plan_t plan, fmmlm_stats* out);

/* Overrides the autotuner's choices (tests, benchmarks): m2l_variant selects the
 * FP32 M2L tile shape (0..5, see m2l_variant_ms), batch_variant the batched FP32
 * M2L variant (0..9, see batch_variant_ms), batch_min_rhs the narrowest pass that
 * runs batched (2..65, see fmmlm_stats.batch_min_rhs; 65 runs every vector on its
 * own); -1 leaves a choice unchanged.  FMMLM_EINVAL for a value out of range or a
 * variant the plan does not have ((p+1)^2 > 128 has one shape: 0, or 0 and 1 for
 * the batched M2L). */
int fmm_layered_plan_set_variants(fmmlm_plan_t plan, int32_t m2l_variant, int32_t batch_variant,
                                  int32_t batch_min_rhs);

/*
 * Tree t (0 <= t < n_trees) of a plan.  Trees are ordered by layer, then side
 * (1: heights above the layer's bottom interface d_l; 2: depths below its top
 * interface d_{l-1}).  Outputs are host arrays; pass keys = perm = NULL to
 * query *n only.  keys[i] is the 63-bit Morton key of the i-th point in tree
 * order, perm[i] its user index.  Errors: FMMLM_EINVAL.
 */
int fmm_layered_plan_tree(fmmlm_plan_t plan, int32_t t, int32_t* layer, int32_t* side,
                          int64_t* n, uint64_t* keys, int64_t* perm);

/*
 * The plan's interaction lists (Algorithm 1's interaction lists, checked by tests).
 * Points are numbered in global tree order: the trees of fmm_layered_plan_tree
 * concatenated in their order.  which selects the table; *count receives its
 * rows; out (host, may be NULL to query the count) receives them:
 *   0  boxes   [count][4]: first point, points, parent box (-1 for a root), level
 *   1  M2L     [count][3]: target box, source box, 1 for a free-space entry (same
 *              tree) or 0 for a reaction entry (the source tree's expansion,
 *              mirrored, for the component of the target tree and source tree)
 *   2  P2P free     [count][3]: target leaf box, first source point, source points
 *   3  P2P reaction [count][3]: the same for the reaction near field
 * A source's multipole expansion reaches a target through M2L between any
 * ancestor-or-self of the source's leaf and any ancestor-or-self of the
 * target's leaf.  Errors: FMMLM_EINVAL, FMMLM_EDEVICE.
 */
int fmm_layered_plan_lists(fmmlm_plan_t plan, int32_t which, int64_t* count, int32_t* out);

/*
 * The scaled Sommerfeld-type integrals S^N I^{ab}_{N,M}(rho, z) of
 * eq. scaledsommerfeldint for 0 <= M <= N <= nmax, computed on the GPU the
 * way plans compute them: 4 nmax + 1 initial values (M = 0, 1), the rest by
 * eq. recurrence.  An initial value is the leading term sinf e^{-k zinf} of the
 * density (fmm_layered_density_asymptotic) integrated in closed form, plus the
 * remainder by quadrature (real axis, or the K_M contour form of
 * eq. contourchange when rho exceeds z + zinf + 2 dmin, the remainder's decay
 * length).
 *
 *  medium         n_interfaces, z_interfaces [L], eps [L+1] (host); n_interfaces = 0
 *                 selects sigma == 1
 *  lt, ls, a, b   target layer, source layer, component indices (1 or 2)
 *  S              scale factor (box size)
 *  npts, rho, z   host arrays [npts]: rho >= 0 (the recurrence needs rho = 0 or
 *                 rho >= S * 2 nmax / a_{2 nmax}), z > 0
 *  nmax           <= 2 * FMMLM_PMAX
 *  out            host [npts][(nmax+1)(nmax+2)/2], entry N(N+1)/2 + M
 */
int fmm_layered_sommerfeld(int32_t n_interfaces, const double* z_interfaces, const double* eps,
                           int32_t lt, int32_t ls, int32_t a, int32_t b, double S, int64_t npts,
                           const double* rho, const double* z, int32_t nmax, double* out,
                           void* hip_stream);

/*
 * Allocation-free form of fmm_layered_sommerfeld, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  It computes the same values with the same
 * kernels, but rho, z and out are device arrays and the call allocates
 * nothing: the component and one task per point are staged in a file-scope
 * device array of FMMLM_NOALLOC_MAX_POINTS * 32 + 256 bytes (about 2 MiB),
 * which each device the library runs on holds until the process ends.  Its
 * device address is looked up (and the quadrature's node table written to
 * constant memory) on the first call on each device; later calls only launch
 * kernels on hip_stream and return without synchronising.
 *
 *  medium, lt, ls, a, b, S, nmax   as for fmm_layered_sommerfeld (host scalars and arrays)
 *  npts           1..FMMLM_NOALLOC_MAX_POINTS
 *  rho, z         device [npts]; a point with rho < 0, z <= 0 or a non-finite
 *                 value gets NaN in all of its outputs
 *  out            device [npts][(nmax+1)(nmax+2)/2], entry N(N+1)/2 + M
 *
 * Every call on a device shares that device's staging array: calls that
 * overlap in time on one device (other streams, other host threads) race and
 * must be ordered by the caller.  Errors: FMMLM_EINVAL (npts above the limit
 * or below 1, bad component, S or nmax, null pointer), medium errors,
 * FMMLM_EDEVICE.
 */
#define FMMLM_NOALLOC_MAX_POINTS 65536
int fmm_layered_sommerfeld_noalloc(int32_t n_interfaces, const double* z_interfaces, const double* eps,
                                   int32_t lt, int32_t ls, int32_t a, int32_t b, double S, int64_t npts,
                                   const double* rho, const double* z, int32_t nmax, double* out,
                                   void* hip_stream);

/* ---- learned form: image ladder + MLP surrogate of the reaction Sommerfeld integrals
 *
 * Reaction component (lt, ls, a, b) of the medium, density sigma(k) with
 * leading term sinf e^{-k zinf} (eq. densityasymptotic).  The 4p+1 initial
 * values S^n I_{n,0}, S^n I_{n,1} of eq. scaledsommerfeldint (p = the
 * surrogate's order) are served as the sum of three parts:
 *   1. the leading term, integrated in closed form (an image at zeta + zinf);
 *   2. a ladder of kLadder = 8 rungs c_j e^{-k (zinf + j delta)}, delta = 2 dmin
 *      (dmin the thinnest finite layer), also closed-form images; c_j is a
 *      weighted least-squares fit of sigma(k) e^{k zinf} - sinf, made once per
 *      component when the surrogate is created (densities from the GPU);
 *   3. the network (4 layers of width 128, tanh, FP32): output j, times
 *      yscale S^n / (0.7^n R2^{n+1}), R2 = |(rho, zeta + zinf + 2 dmin)|, is
 *      what parts 1 and 2 leave (degree n_j, order m_j: outputs 0..2p are
 *      (n, 0), outputs 2p+1..4p are (n - 2p, 1)).
 * Orders M >= 2 follow by eq. recurrence in FP64, as without the network.
 * Outside the trained (rho, zeta) box the quadrature is used (fallback); the
 * quadrature also judges the learned form: plans report the largest
 * deviation on sampled tasks (fmmlm_stats.surrogate_check).
 * Network inputs: the component (one-hot) and
 * (2 rho/rho_max - 1, 2 zeta/zeta_max - 1, 2 Z2/R2 - 1, 4 dmin/R2 - 1).
 * Components are numbered over the medium's 2L sides (layer, side) in order
 * (layer 0 side 1, layer 1 side 1, layer 1 side 2, ...): c = t * 2L + s for
 * target side t and source side s.  Needs at least two interfaces (with one,
 * the density is its leading term and the quadrature is not used at all).
 */
typedef struct {
  int64_t nsamples;        /* samples generated by the quadrature (default 2097152);
                              1/32 of them are held out for validation */
  int32_t steps;           /* Adam steps (default 6000) */
  int32_t batch;           /* minibatch, a multiple of 64 (default 8192) */
  double lr;               /* peak learning rate (default 2e-3): 2% linear warm-up,
                              then cosine decay to lr/100 */
  uint64_t seed;           /* initialisation, samples, minibatches (default 1) */
  int32_t reserved[4];     /* must be 0 */
} fmmlm_train_opts;

typedef struct {
  int64_t n_train, n_val, n_params;
  int32_t n_components, n_outputs;
  double sample_seconds;   /* generating the samples (quadrature on the GPU) */
  double train_seconds;    /* the Adam steps */
  double loss_first;       /* mean minibatch loss over the first and ...             */
  double loss_last;        /* ... last 2% of the steps (normalised outputs y)        */
  double val_rms, val_max; /* held-out error of y (network output units)             */
  double yscale;           /* the output unit: rms of the targets in physical units  */
  double ladder_fit;       /* largest relative weighted residual of the ladder fits  */
} fmmlm_train_report;

void fmmlm_default_train_opts(fmmlm_train_opts* opts);

/*
 * A new, untrained network (Glorot-uniform weights from seed) for the medium
 * (host arrays as in fmm_layered_plan), order p (outputs 4p+1) and the
 * (rho, zeta) box [0, rho_max] x (0, zeta_max].  Errors: FMMLM_EINVAL
 * (p out of range, non-positive box), FMMLM_EUNSUPPORTED (fewer than two
 * interfaces), medium errors, FMMLM_EDEVICE.
 */
int fmm_layered_surrogate_create(int32_t n_interfaces, const double* z_interfaces, const double* eps,
                                 int32_t p, double rho_max, double zeta_max, uint64_t seed,
                                 fmmlm_surrogate_t* out);

/* The same for a plan's medium and p, with the box covering every (rho, zeta)
 * the plan's trees can produce: rho_max = sqrt(2) W, zeta_max = 2 W, W the
 * common root box side. */
int fmm_layered_surrogate_create_for_plan(fmmlm_plan_t plan, uint64_t seed, fmmlm_surrogate_t* out);

/* Generates opts->nsamples samples with the quadrature and trains the network
 * in place with its own forward/backward/Adam kernels on hip_stream
 * (synchronised on return).  opts NULL = defaults; rep may be NULL. */
int fmm_layered_surrogate_train(fmmlm_surrogate_t s, const fmmlm_train_opts* opts, void* hip_stream,
                                fmmlm_train_report* rep);

int fmm_layered_surrogate_destroy(fmmlm_surrogate_t s);

/* Parameters as one host float vector (layout in the network description
 * above: E [ncomp][128], A [4][128], b1, W2 [128][128], b2, W3, b3, W4 [128][nout],
 * b4, W[k][j] mapping input k to output j).  *n receives the count; get or set
 * may be NULL (get copies out, then set copies in). */
int fmm_layered_surrogate_params(fmmlm_surrogate_t s, float* get, const float* set, int64_t* n);

/* One forward and backward pass on the GPU over n samples (host arrays:
 * comp [n] component index, feat [n][4] features, target [n][nout]): the
 * mean squared error into *loss and its gradient into grad [nparams] (host).
 * For checking the training kernels. */
int fmm_layered_surrogate_grad(fmmlm_surrogate_t s, int64_t n, const int32_t* comp, const float* feat,
                               const float* target, double* loss, float* grad, void* hip_stream);

/* The network's outputs (the remainder of the initial values in output units,
 * before the closed-form parts are added) for n samples: host arrays comp [n],
 * feat [n][4] as for fmm_layered_surrogate_grad, out [n][nout].  The same forward
 * kernel as the plans' learned form.  Errors: FMMLM_EINVAL, FMMLM_ENOMEM,
 * FMMLM_EDEVICE. */
int fmm_layered_surrogate_forward(fmmlm_surrogate_t s, int64_t n, const int32_t* comp, const float* feat,
                                  float* out, void* hip_stream);

/* nsteps (1..64) steps of the training's Adam update (Kingma & Ba 2015, Algorithm 1:
 * beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected moments) applied in place to the
 * network's parameters, starting from zero moments at t = 1: step t uses the
 * gradient grads [t-1][nparams] and the learning rate lr [t-1] (host arrays).
 * The parameters after each step go to params_out [nsteps][nparams] (host, may be
 * NULL).  For checking the training kernel.  Errors: FMMLM_EINVAL (lr not finite
 * and positive), FMMLM_ENOMEM, FMMLM_EDEVICE. */
int fmm_layered_surrogate_adam(fmmlm_surrogate_t s, int32_t nsteps, const float* grads, const double* lr,
                               float* params_out, void* hip_stream);

/* The training samples fmm_layered_surrogate_train draws for seed: n samples
 * into host arrays comp [n], rho [n], zeta [n], feat [n][4], target [n][nout]
 * (target = what the leading term and the ladder leave of the quadrature's
 * initial values, times 0.7^n R2^{n+1} / yscale: the network's output units). */
int fmm_layered_surrogate_samples(fmmlm_surrogate_t s, int64_t n, uint64_t seed, int32_t* comp, double* rho,
                                  double* zeta, float* feat, float* target, void* hip_stream);

/* S^N I_{N,M}(rho, z) for 0 <= M <= N <= nmax (nmax <= 2p of the surrogate)
 * through the learned form, with the same layout as fmm_layered_sommerfeld; used[i]
 * (may be NULL) is 1 where the network served point i, 0 where the quadrature
 * did.  Host arrays. */
int fmm_layered_surrogate_eval(fmmlm_surrogate_t s, int32_t lt, int32_t ls, int32_t a, int32_t b, double S,
                               int64_t npts, const double* rho, const double* z, int32_t nmax, double* out,
                               int32_t* used, void* hip_stream);

/* ---- pre-computed tables for the initial values (the Remark after Table 3.1)
 *
 * The table form serves the same 4p+1 initial values S^n I_{n,0}, S^n I_{n,1}
 * (and the near-field kernels I_00) as the learned form, with the network's
 * part 3 replaced by 2-D tables: per component, what the leading term and the
 * ladder leave, times 0.7^n R2^{n+1} (output units as for the network, with
 * yscale 1), is tabulated at the kTabK = 12 Chebyshev points of the first kind
 * x_k = cos((2k + 1) pi / 24), k = 0..11, of each of npr x npz equal panels
 * over [0, rho_max] x [0, zeta_max] (node (a, b) of panel (i, j) at
 * rho = (i + (1 + x_a) / 2) rho_max / npr, zeta = (j + (1 + x_b) / 2) zeta_max / npz),
 * filled by the GPU quadrature when the form is created, and interpolated by
 * the barycentric formula (tensor product of degree 11 in each variable).
 * Panels are no wider than the thinnest finite layer (4..48 per direction).
 * The handle is a fmmlm_surrogate_t: a plan takes it through opts.surrogate,
 * fmm_layered_surrogate_eval and _destroy accept it, the network calls
 * (train, params, grad, forward, adam, samples) return FMMLM_EUNSUPPORTED.
 * Needs at least two interfaces.  Errors as for fmm_layered_surrogate_create,
 * FMMLM_ENOMEM for the tables' device memory.
 */
int fmm_layered_tables_create(int32_t n_interfaces, const double* z_interfaces, const double* eps, int32_t p,
                              double rho_max, double zeta_max, void* hip_stream, fmmlm_surrogate_t* out);

/* The same over a plan's medium, p and (rho, zeta) domain (as for
 * fmm_layered_surrogate_create_for_plan). */
int fmm_layered_tables_create_for_plan(fmmlm_plan_t plan, void* hip_stream, fmmlm_surrogate_t* out);

/* Grid of a table form (panels per direction), the tables' device bytes and the
 * seconds it took to create them (ladder fit and quadrature at the nodes); any
 * output may be NULL.  FMMLM_EINVAL for a network handle. */
int fmm_layered_tables_info(fmmlm_surrogate_t s, int32_t* npr, int32_t* npz, int64_t* bytes, double* seconds);

/* The table form's interpolation alone, on given node values (tests): nodes
 * (host) [npr * npz][nout][12 * 12] in the layout above (panel i * npz + j,
 * node a * 12 + b), points rho, zeta (host [npts], inside the box), out (host)
 * [npts][nout].  Exact for polynomials of degree <= 11 in each variable on each
 * panel.  Errors: FMMLM_EINVAL, FMMLM_ENOMEM, FMMLM_EDEVICE. */
int fmm_layered_interp2d(int32_t npr, int32_t npz, double rho_max, double zeta_max, int32_t nout,
                         const double* nodes, int64_t npts, const double* rho, const double* zeta, double* out,
                         void* hip_stream);

/*
 * Leading term of a reaction density as k -> infinity (eq. densityasymptotic):
 * sigma^{ab}_{lt,ls}(k) = sinf e^{-k zinf} (1 + O(e^{-2 k dmin})), dmin the
 * thinnest finite layer.  zinf is the shortest ray path from the source's exit
 * interface to the target's entry interface, sinf the product of the local
 * reflection/transmission coefficients along it.  Host computation (no GPU).
 *
 *  sinf, zinf     host scalars, written on success
 *  errors         FMMLM_EINVAL (null pointer, invalid component), medium errors
 */
int fmm_layered_density_asymptotic(int32_t n_interfaces, const double* z_interfaces,
                                   const double* eps, int32_t lt, int32_t ls, int32_t a, int32_t b,
                                   double* sinf, double* zinf);

/*
 * Reaction densities sigma^{ab}_{lt,ls}(k) of App. A at complex k (Re k >= 0),
 * computed on the GPU by the plan's own routine.  Host arrays [nk].
 */
int fmm_layered_density(int32_t n_interfaces, const double* z_interfaces, const double* eps,
                        int32_t lt, int32_t ls, int32_t a, int32_t b, int64_t nk,
                        const double* k_re, const double* k_im, double* out_re, double* out_im,
                        void* hip_stream);

/*
 * Live per-stage timing of evaluations (benchmarks).  profile_begin makes the
 * next max_evals evaluations of the plan record a HIP event on their stream
 * before the first stage and after every stage (FMMLM_NSTAGES stages, in the
 * order gather, P2M, M2M, M2L top, M2L, M2L reduce, L2L, L2P, P2P free,
 * P2P reaction, combine).  "M2L" is one kernel launch: the operator-major M2L
 * chunks of the levels below the top ones (FP32 matrix cores in the FP32 form,
 * FP64 matrix cores in the FP64 form); "M2L top" clears the local expansions,
 * runs the top levels (sparse FP64 kernel) and, in the FP32 form, converts the
 * multipole expansions to FP32; "M2L reduce" adds each target's chunk
 * products.
 * profile_end synchronises the device, writes the summed milliseconds of each
 * stage over the recorded evaluations to stage_ms[FMMLM_NSTAGES] (host), the
 * number of recorded evaluations to *n_evals, and stops recording.
 * Errors: FMMLM_EINVAL, FMMLM_EDEVICE, FMMLM_ENOMEM.
 */
#define FMMLM_NSTAGES 11
int fmm_layered_profile_begin(fmmlm_plan_t plan, int32_t max_evals);
int fmm_layered_profile_end(fmmlm_plan_t plan, double* stage_ms, int64_t* n_evals);

#ifdef __cplusplus
}
#endif

#endif /* FMMLM_H */
