/*
 * chert.h -- C ABI of the MI355X (gfx950) CHERT hot path.
 *
 * CHERT (Cached Hamiltonian-Enhanced Ray Tracing) separates two stages
 * (Method overview; Algorithm 2):
 *   1. a directional cache C(m, k, theta) of ray velocity, attenuation, Q and
 *      ray direction per wave mode m, cache class k and sampled ray
 *      direction theta, filled by solving the g*-Hamiltonian homogeneity
 *      problem (eqs 2-14, 26);
 *   2. first-arrival shortest-path traveltimes whose edge costs come from
 *      cache lookups (eqs 18-19, 22-34): propagation tau_R, attenuation
 *      tau_I, predecessors, raypaths, and t* along the propagation raypath.
 *
 * Conventions shared by every call:
 *   - Plain C; every call returns an int status (chert_status).  On failure
 *     chert_last_error() gives a message (thread-local, valid until the next
 *     failing call on the same thread).
 *   - Units are SI: metres, seconds, density-normalised moduli in m^2/s^2,
 *     angles in radians.
 *   - 2D frame: x to the right, z down (depth).  Angles are measured from +z
 *     towards +x; the unit vector at angle a is (sin a, cos a) in (x, z).
 *     A class's symmetry axis is tilted from +z towards +x by `tilt` (eq 36).
 *   - Node index = ix + nx * iz (x fastest).
 *   - Pointers named *_dev are device memory, *_host host memory.  The
 *     library never allocates device memory: outputs and scratch
 *     ("workspace") are owned by the caller; sizes come from the *_bytes()
 *     queries.
 *   - `stream` is a hipStream_t passed as void*.  Kernels are enqueued on it.
 *     Argument validation happens before anything is enqueued; a validation
 *     failure leaves every output untouched.  The one check that needs the
 *     device -- class ids of a class map in range -- runs as the first
 *     kernel of a trace; a failing map makes every later kernel of the call
 *     leave at once, so the outputs stay untouched there too, and the call
 *     (or chert_trace_graph_finish) returns INVALID_ARG.
 */
#ifndef CHERT_H
#define CHERT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  CHERT_OK = 0,
  CHERT_ERR_INVALID_ARG = 1,   /* bad sizes, NaN/negative parameters, ... */
  CHERT_ERR_UNSUPPORTED = 2,   /* valid but not implemented (e.g. dim 3)  */
  CHERT_ERR_HIP = 3,           /* a HIP runtime call failed               */
  CHERT_ERR_NO_CONVERGENCE = 4,/* relaxation round cap reached            */
  CHERT_ERR_CAPACITY = 5,      /* output buffer too small                 */
  CHERT_ERR_UNREACHABLE = 6,   /* receiver has no predecessor             */
  CHERT_ERR_CYCLE = 7,         /* predecessor chain longer than the grid  */
  CHERT_ERR_ABORTED = 8        /* the caller's abort word was raised      */
} chert_status;

/* wave modes of the sagittal-plane problem */
typedef enum { CHERT_QP = 0, CHERT_QSV = 1, CHERT_QSH = 2 } chert_mode;

/* Energy-velocity kernel.  MEV (eqs 13-14) is read as the p-gradient of the
 * g*-Hamiltonian with the eigenvector and its conjugate held fixed:
 *   v_m = a_mjkl p_l Re(g_j conj(g_k)) / (g^H g).
 * OEV is eq 12: v_m = a_mjkl p_l g_j g_k / (g^T g). */
typedef enum { CHERT_KERNEL_MEV = 0, CHERT_KERNEL_OEV = 1 } chert_kernel;

/* Per-entry status bits of the cache. */
enum {
  CHERT_ST_OK = 0,
  CHERT_ST_NO_BRACKET = 1, /* no slowness angle reaches the ray direction   */
  CHERT_ST_ILL = 2,        /* chosen root where |dpsi/dtheta_R| < 1e-2       */
  CHERT_ST_FLUID = 4,      /* shear mode in a class without shear stiffness */
  CHERT_ST_NONPHYS = 8,    /* negative attenuation or non-finite velocity   */
  CHERT_ST_NOCONV = 16     /* the chosen root's residual (CHERT_F_RES) is
                              above the descriptor's resid_tol             */
};
/* Entries with NO_BRACKET, FLUID, NONPHYS or NOCONV are unusable: an edge
 * that reads one is impassable (w = +inf). */

/* Counters of one cache build (device memory, written by the build calls
 * when chert_cache_desc.stats_dev is set).  Entries are stored columns
 * (modes in mode_mask x classes x columns, centrosymmetric copies
 * included). */
typedef struct chert_cache_stats {
  int64_t n_entries;    /* stored entries of the built modes                */
  int64_t n_converged;  /* status OK or ILL only: a root within resid_tol   */
  int64_t n_fallback;   /* entries the surrogate-started build sent back
                           to the plain solver: whole 2D jobs, single 3D
                           directions (0 for plain builds)                  */
  int64_t n_noconv;     /* CHERT_ST_NOCONV set                               */
  int64_t n_illcond;    /* CHERT_ST_ILL set                                  */
  int64_t n_nobracket;  /* CHERT_ST_NO_BRACKET set                           */
  int64_t n_unusable;   /* FLUID or NONPHYS set                              */
  double max_resid;     /* largest residual over entries with a root        */
} chert_cache_stats;

/* One cache class: the stored medium of eq 26 (c_ijkl(k), Q_ijkl(k), rho(k))
 * for a transversely isotropic medium.  Complex moduli follow eq 2:
 * a_pq = a_pq (1 - i / q_pq); q = INFINITY means elastic. */
typedef struct chert_class {
  double a11, a13, a33, a44, a66; /* real density-normalised moduli [m^2/s^2] */
  double q11, q13, q33, q44, q66; /* quality factors per component          */
  double rho;                     /* density [kg/m^3]; stored, not used     */
  double tilt;                    /* symmetry-axis tilt theta_0 (eq 36)      */
  double azimuth;                 /* phi_0 (eq 35); must be 0 in 2D          */
} chert_class;

/* Thomsen parameters -> class (exact relations of Thomsen 1986 for the real
 * moduli; Qp on a11/a13/a33, Qs on a44/a66).  Host, synchronous.
 * INVALID_ARG on NaN, vp0 <= 0, vs0 < 0, vs0 >= vp0, Q <= 0 or a negative
 * radicand in the a13 relation (1 + 2 delta < vs0^2/vp0^2). */
int chert_class_from_thomsen(double vp0, double vs0, double rho, double eps,
                             double delta, double gamma, double tilt,
                             double azimuth, double qp, double qs,
                             chert_class *out);

/* Device batch of chert_class_from_thomsen for per-node media (one class per
 * node).  params_dev: [n][10] doubles (vp0, vs0, rho, eps, delta, gamma,
 * tilt, azimuth, qp, qs); out_dev: [n] classes.  A row the host function
 * would reject becomes a class with NaN moduli, whose cache entries get
 * CHERT_ST_NONPHYS.  Asynchronous on `stream`. */
int chert_classes_from_thomsen(const double *params_dev, int64_t n,
                               chert_class *out_dev, void *stream);

/* ------------------------------------------------------------------------
 * Stage 1: the directional cache (eq 26; Algorithm 2, cache construction).
 * Entry (m, k, d) holds the homogeneous solution (eq 9) whose ray direction
 * is exactly d * 2 pi / n_dirs (global frame).  The slowness-angle pair
 * (theta_R, theta_I) is searched as follows: theta_I is the root of the
 * homogeneity residual nearest 0 in [-30, 30] deg; theta_R is bracketed on a
 * sweep of n_sweep samples over [0, 2 pi) and refined to the target ray
 * direction; among several roots (triplications) the largest ray velocity
 * wins.  Entries d >= n_dirs/2 are the centrosymmetric copies of d - n_dirs/2.
 * ------------------------------------------------------------------------ */
/* 3D caches (dim 3; eqs 6, 35): column i is the Fibonacci ray direction
 *   f_i = (r cos phi_i, r sin phi_i, z_i), z_i = 1 - (2i+1)/n_dirs,
 *   r = sqrt(1 - z_i^2), phi_i = i pi (3 - sqrt 5)   (global x, y, z; z down),
 * n_dirs = 41253 giving about one direction per square degree.  For a TI
 * class the ray direction f_i is reached with the slowness in the plane of
 * the symmetry axis e_z' (eq 35: (sin t0 cos p0, sin t0 sin p0, cos t0) with
 * t0 = tilt, p0 = azimuth) and f_i, imaginary azimuth 0; entry i is that
 * sagittal-plane solve at the local polar angle arccos(f_i . e_z') with the
 * same root search as in 2D.  Every column is solved (no centrosymmetric
 * copies, no subsets); RX and RZ hold the x and z components of f_i. */
typedef struct chert_cache_desc {
  int32_t dim;        /* 2, or 3 (Fibonacci directions, see above)          */
  int32_t n_dirs;     /* 2D: even, >= 4; 360 = 1 degree.  3D: 2..2^20      */
  uint32_t mode_mask; /* bit (1 << chert_mode) per mode to build            */
  int32_t kernel;     /* chert_kernel                                       */
  int32_t n_sweep;    /* theta_R sweep samples, >= 16 (1440 = 0.25 degree)  */
  int32_t n_subset;   /* 0: every direction; else the number of columns     */
  const int32_t *subset_host; /* n_subset direction indices, ascending,
                         closed under d -> d + n_dirs/2 (mod n_dirs), at
                         most 512; only these columns are stored and built
                         (per-node caches need only the star's bins).  Read
                         during the call only.                              */
  double resid_tol;   /* homogeneity / direction residual above which an
                         entry gets CHERT_ST_NOCONV; finite, >= 0 (0 = 1e-9) */
  int32_t max_iter;   /* cap on the refinement steps of each theta_R bracket
                         (Newton steps, then the halvings of the bisection
                         fallback); >= 0 (0 = 12 Newton steps and 200
                         halvings)                                          */
  int32_t sampling;   /* CHERT_SAMPLE_RAY (0): column d holds the solution
                         whose ray direction is d 2pi/n_dirs (above);
                         CHERT_SAMPLE_SLOWNESS (1): column s holds the
                         solution at real slowness angle s 2pi/n_dirs in the
                         class's symmetry-axis frame (eq 26 read literally;
                         2D class caches only, no subset), and an edge reads,
                         at each endpoint, the column whose stored ray
                         direction is closest to the edge (see below)      */
  chert_cache_stats *stats_dev; /* nullable device struct: the build calls
                         overwrite it with their counters (after the
                         entries, on the same stream)                       */
} chert_cache_desc;
/* The trace calls read dim, n_dirs, mode_mask, sampling and the subset of
 * a descriptor; the solver fields (kernel, n_sweep, resid_tol, max_iter,
 * stats_dev) matter only to the build calls. */
enum { CHERT_SAMPLE_RAY = 0, CHERT_SAMPLE_SLOWNESS = 1 };
/* Slowness-sampled caches: column s of (mode, class) is the homogeneous
 * solution at theta_R = s 2 pi / n_dirs (symmetry-axis frame): theta_I is
 * the homogeneity root nearest 0 in [-30, 30] deg (NO_BRACKET if none),
 * the ray quantities follow (eqs 10-11), RX/RZ hold the ray direction in
 * the global frame and RES the homogeneity residual.  n_sweep is not used.
 * In a trace, the edge i -> j with offset o reads column b_k(o) of each
 * endpoint's class k: the column whose stored ray direction has the largest
 * dot product with the edge's unit vector o / |o| (lowest column on ties;
 * columns with NO_BRACKET or FLUID are not candidates), then eqs 28-30
 * with the two columns:
 *   w_R = L_o / (0.5 (V[k_i][b_ki(o)] + V[k_j][b_kj(o)]))
 * (unusable entries make the edge impassable, as above). */

/* Field order of the cache arrays. */
enum {
  CHERT_F_V = 0,   /* ray velocity V^Ray (eq 11) [m/s]                   */
  CHERT_F_A = 1,   /* ray attenuation A^Ray (eq 11) [s/m]                */
  CHERT_F_Q = 2,   /* ray quality factor Q^Ray (eq 11)                   */
  CHERT_F_RX = 3,  /* ray direction r_hat, global x                      */
  CHERT_F_RZ = 4,  /* ray direction r_hat, global z                      */
  CHERT_F_THR = 5, /* real slowness angle theta_R, local frame [0, 2 pi) */
  CHERT_F_THI = 6, /* imaginary slowness angle theta_I                   */
  CHERT_F_RES = 7, /* max(|sin angle(v^R, v^I)|, |ray-direction miss|)   */
  CHERT_NF = 8
};

/* Device layout of a cache blob (all offsets in bytes from its start), with
 * n_cols = n_subset if a subset is given, else n_dirs:
 *   [0, 256)            header: uint32 magic 'CHRT' (0x54524843), uint32
 *                       version (1), int32 dim, n_dirs, mode_mask, kernel,
 *                       n_sweep, n_subset, int64 n_classes, int32
 *                       sampling; rest zero.
 *   fields_offset       double fields[CHERT_NF][3][n_classes][n_cols]
 *   status_offset       int32 status[3][n_classes][n_cols]
 * Slots of modes outside mode_mask are left as they were.  The blob is
 * position-independent, so it may be copied to disk and back. */
typedef struct chert_cache_layout {
  size_t fields_offset;
  size_t status_offset;
  size_t total_bytes;
} chert_cache_layout;

/* Layout of a cache for n_classes classes.  INVALID_ARG on a bad desc. */
int chert_cache_layout_of(const chert_cache_desc *d, int64_t n_classes,
                          chert_cache_layout *out);

/* Scratch needed by chert_build_cache (the theta_R sweep tables). */
size_t chert_build_cache_workspace_bytes(const chert_cache_desc *d,
                                         int64_t n_classes);

/* Build the cache for n_classes classes (device array classes_dev) into
 * cache_dev (layout above).  Asynchronous on `stream`.  Per-entry failures
 * are reported through the status array, not the return value. */
int chert_build_cache(const chert_cache_desc *d, const chert_class *classes_dev,
                      int64_t n_classes, void *cache_dev, void *workspace_dev,
                      size_t workspace_bytes, void *stream);

/* chert_build_cache for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same kernels and results, with the theta_R sweep tables
 * in a file-scope device array of chert_build_cache_noalloc_max_bytes()
 * (16 MiB) instead of a caller's workspace.  The call allocates nothing and
 * enqueues kernels only (no memset, no host copy), asynchronously on
 * `stream`.  Each GPU holds its own copy of the array until the process
 * ends; its device address is resolved on the first call on that device.
 * Every call on one GPU shares that GPU's array: calls that overlap on one
 * GPU (concurrent streams, or host threads) race and must be serialised by
 * the caller.  Nothing in the array needs to start at zero: each call
 * writes every sweep entry before reading it.  CAPACITY when the build's
 * sweep tables (chert_build_cache_workspace_bytes) exceed the array; other
 * errors as chert_build_cache. */
size_t chert_build_cache_noalloc_max_bytes(void);
int chert_build_cache_noalloc(const chert_cache_desc *d, const chert_class *classes_dev,
                              int64_t n_classes, void *cache_dev, void *stream);

/* ------------------------------------------------------------------------
 * Stage 2: traveltime fields (eqs 22, 24, 27-34; Algorithm 2, tracing).
 * Graph: every node connects to the nodes at the forward-star offsets o with
 * max(|ox|, |oz|) <= radius and gcd(|ox|, |oz|) = 1, ordered by (oz, ox)
 * ascending; offsets leaving the grid are dropped.  The edge i -> j with
 * offset o uses the bin b(o) = round(atan2(ox hx, oz hz) n_dirs / 2 pi) mod
 * n_dirs and the classes k_i, k_j:
 *   w_R = L_o / (0.5 (V[k_i][b] + V[k_j][b]))     (eqs 28-29)
 *   w_I = L_o * (0.5 (A[k_i][b] + A[k_j][b]))     (eqs 28, 30)
 * with L_o = sqrt((ox hx)^2 + (oz hz)^2) (eq 27); an entry whose status has
 * NO_BRACKET, FLUID or NONPHYS makes the edge impassable (w = +inf).
 * tau_R and tau_I are independent first-arrival problems (eqs 24, 31): each
 * node gets the minimum over paths of the left-to-right FP64 sum of edge
 * weights (unreachable: +inf).  Predecessors (eq 33) are deterministic: among
 * the neighbours i with tau_i + w_ij == tau_j the one with the smallest BFS
 * hop count over such edges, then the smallest offset index, wins.  t* is the
 * attenuation folded along the propagation raypath: t*_src = 0,
 * t*_j = t*_pred_p(j) + w_I(pred_p(j) -> j).
 * ------------------------------------------------------------------------ */
/* 3D grids (dim 3): node index ix + nx (iy + ny iz); the star holds the
 * offsets with max(|ox|, |oy|, |oz|) <= radius (1..4) and gcd 1, ordered by
 * (oy, oz, ox) ascending, L_o = sqrt((ox hx)^2 + (oz hz)^2 + (oy hy)^2), and
 * the bin of o is the Fibonacci direction with the largest dot product with
 * o / L_o (lowest index on ties).  3D traces (with a class map and a 3D
 * cache) give every output of the 2D path by the same rules; the relaxation
 * runs on 3D tiles or on a node frontier with near/far buckets (see
 * chert_trace_opts.launch) to the same fixed point; predecessors come from
 * BFS layers over tight edges. */
typedef struct chert_grid {
  int32_t dim;                 /* 2 or 3                                   */
  int32_t radius;              /* forward-star radius R, 1..8 (3D: 1..4)   */
  int64_t nx, nz, ny;          /* nodes per axis; ny must be 1 in 2D       */
  double hx, hz, hy;           /* node spacing [m]                         */
  const int32_t *class_id_dev; /* [n_nodes] class of each node, in range   */
} chert_grid;

/* output selection bits */
enum {
  CHERT_OUT_TAU_R = 1,
  CHERT_OUT_TAU_I = 2,
  CHERT_OUT_TSTAR = 4,
  CHERT_OUT_PRED_P = 8,
  CHERT_OUT_PRED_A = 16
};

/* Work counters of one trace call, per phase.  Tile runs (2D): 0 =
 * traveltimes, 1 = the predecessor tree (hop counts, predecessors and t*
 * in one relaxation over the tight edges), slot 2 unused (0).  3D tile
 * runs fill slot 0 and rounds[1] = BFS layers.  Frontier runs fill
 * rounds[0] = iterations, rounds[1] = BFS layers, tile_visits[0] =
 * iterations that had work and edge_relaxations[0] = (frontier node,
 * offset) pairs examined. */
typedef struct chert_trace_stats {
  int32_t rounds[3];           /* relaxation rounds until no tile changed   */
  int32_t reserved;
  int64_t tile_visits[3];      /* (problem, tile) workgroup visits           */
  int64_t edge_relaxations[3]; /* raw edges examined (pulls + pushes)        */
  int64_t levels_sum[3];       /* push levels summed over visits             */
  int32_t levels_max[3];       /* most push levels in one visit              */
  int32_t reserved2;
} chert_trace_stats;

/* How the relaxation rounds are launched (the fields are the same either
 * way: the fixed point does not depend on the schedule):
 *   PER_ROUND   one launch per round over every tile; the host checks for
 *               termination after 16, then every 32, then every 64 rounds
 *               (launches past convergence find no active tile);
 *   PERSISTENT  one launch per phase: an occupancy-sized grid walks each
 *               round's active tiles, rounds separated by a device-wide
 *               barrier (bounded wait: a stalled barrier fails the call with
 *               CHERT_ERR_HIP instead of hanging); the host waits only at
 *               the end, and the launch sequence can be captured into a
 *               graph (chert_trace_graph_create);
 *   FRONTIER    no tiles: the node-frontier label-correcting iteration of
 *               the 3D path (one thread per (frontier node, offset), 64-bit
 *               atomicMin on the head, optional near/far buckets), one launch
 *               per iteration, the host checking the frontier sizes every 8
 *               iterations; predecessors from BFS layers over tight edges.
 * 3D batches: CHERT_LAUNCH_FRONTIER runs the node frontier;
 * CHERT_LAUNCH_PER_ROUND runs the traveltimes on 3D tiles of tile_x x
 * tile_x x tile_z nodes (default 8 x 8 x 8; at least radius per side, at
 * most 1024 nodes; the same per-round scheme, 26 neighbour tiles) and the
 * predecessors and t* with the frontier's BFS layers; _PERSISTENT runs
 * the same 3D tiles in one launch (an occupancy-sized grid, rounds
 * separated by the bounded device-wide barrier, the abort word polled by
 * the kernel) and the same BFS layers.
 * In per-node mode (no class map) the relaxation may read an edge's weight
 * from either endpoint's row; both hold the same value because a cache
 * stores direction d + n_dirs/2 as the exact copy of d. */
enum { CHERT_LAUNCH_PER_ROUND = 0, CHERT_LAUNCH_PERSISTENT = 1, CHERT_LAUNCH_FRONTIER = 2 };

typedef struct chert_trace_opts {
  uint32_t outputs;   /* CHERT_OUT_* bits.  TSTAR needs TAU_R and PRED_P;
                         PRED_P needs TAU_R; PRED_A needs TAU_I.           */
  int32_t tile_x;     /* relaxation tile width in nodes (0 = default 32)   */
  int32_t tile_z;     /* relaxation tile height in nodes (0 = default 32)  */
  int32_t max_rounds; /* cap on relaxation rounds per phase (0 = default)  */
  int32_t push_group; /* star offsets per push work item: 1, 2, 4, or 8 on
                         2D tiles (0 = 2)                                  */
  int32_t launch;     /* CHERT_LAUNCH_PER_ROUND (0), _PERSISTENT (1) or
                         _FRONTIER (2)                                     */
  double bucket_width;/* ordering width in units of the batch's smallest
                         positive edge weight of the field (0 = none; must
                         be >= 0).  Frontier iteration: near/far buckets,
                         an improvement at or above the problem's far
                         minimum + width waits.  Tiles: a tile woken with
                         key k (smallest changed border value: tau, t*, or
                         the hop count with the width in hops) is visited
                         only once k <= its problem's smallest pending key
                         + width; otherwise it stays active for a later
                         round (2D tiles; the 3D tiles have no
                         ordering).  The fields do not depend on it.      */
  chert_trace_stats *stats_host; /* nullable: filled when the call returns */
  const volatile int32_t *abort_flag_host; /* nullable caller-owned word in
                         pinned host memory (hipHostMalloc).  While it is
                         non-zero the relaxation stops at its next round
                         boundary: the host checks it between launches, the
                         persistent and graph-replayed kernels poll it at
                         every round, and every kernel still exits normally.
                         The call then returns CHERT_ERR_ABORTED; tau_R and
                         tau_I hold upper bounds of the fixed point (each
                         value +inf or the length of some path), predecessor
                         and t* outputs are unspecified.                    */
} chert_trace_opts;

/* Scratch needed by chert_trace_field for these arguments. */
size_t chert_trace_workspace_bytes(const chert_cache_desc *d, int64_t n_classes,
                                   const chert_grid *g, int32_t n_src,
                                   const chert_trace_opts *o);

/* Trace n_src sources (host array of node indices) for one mode, reading
 * edge costs from `cache_dev` (built by chert_build_cache or imported with
 * the documented layout).  Outputs are device arrays [n_src][n_nodes]; the
 * ones not selected in o->outputs may be NULL.  Enqueues on `stream` and
 * returns after the relaxation has converged (the call synchronises the
 * stream to test for termination).  NO_CONVERGENCE if a phase reaches
 * max_rounds (outputs then hold a valid upper bound). */
int chert_trace_field(const chert_cache_desc *d, const void *cache_dev,
                      int64_t n_classes, const chert_grid *g, int32_t mode,
                      const int64_t *src_nodes_host, int32_t n_src,
                      const chert_trace_opts *o, double *tau_r_dev,
                      double *tau_i_dev, double *tstar_dev,
                      int32_t *pred_p_dev, int32_t *pred_a_dev,
                      void *workspace_dev, size_t workspace_bytes,
                      void *stream);

/* One job of a batched trace: a grid, the cache (and mode) its edge costs
 * come from, its sources and its outputs ([n_src][nx*nz] device arrays, the
 * ones not selected in the options may be NULL). */
typedef struct chert_trace_job {
  const chert_cache_desc *d;
  const void *cache_dev;
  int64_t n_classes;
  const chert_grid *g;
  int32_t mode;
  int32_t n_src;
  const int64_t *src_nodes_host;
  double *tau_r_dev;
  double *tau_i_dev;
  double *tstar_dev;
  int32_t *pred_p_dev;
  int32_t *pred_a_dev;
} chert_trace_job;

/* Scratch needed by chert_trace_batch (0 on invalid arguments). */
size_t chert_trace_batch_workspace_bytes(const chert_trace_job *jobs, int32_t n_jobs,
                                         const chert_trace_opts *o);

/* Many shots on grids of uneven size (Algorithm 2's loops over sources and
 * modes, run together): every (job, source, field) problem of the batch
 * advances in the same relaxation launches, so the rounds of all problems
 * overlap.  Semantics per job are those of chert_trace_field; all jobs must
 * share one forward-star radius.  At most 65535 problems per batch. */
int chert_trace_batch(const chert_trace_job *jobs, int32_t n_jobs,
                      const chert_trace_opts *o, void *workspace_dev,
                      size_t workspace_bytes, void *stream);

/* Autotuner of the relaxation's launch parameters for a given batch.  The
 * fixed point does not depend on them (every candidate gives the same
 * fields); only the time does.  Candidates: in 3D the frontier iteration
 * with bucket widths 0 (one bucket), 4, 16, 32, 64, 128, 256 (units of the
 * smallest edge weight) and the 3D tiles 8x8x8, 8x8x16, 16x16x4, 4x4x16
 * with push groups 1, 2, 4, per-round and persistent launch; in 2D the
 * frontier with widths 16 and 64 and the tiles 32x32, 64x16, 16x64, 32x16,
 * 16x32, 128x8, 16x16 with push groups 1, 2, 4, 8, per-round and
 * persistent launch, then, if tiles win, their ordering width 16, 64 or 256
 * on the fastest shape.  Each is timed (HIP events,
 * second of two runs) on a probe batch made of the first source of every
 * job; when some job has more than one source, the three fastest are timed
 * the same way on the whole batch.  The fastest is written into o->tile_x,
 * tile_z, push_group, launch and bucket_width (other fields are kept) and
 * its time (on the whole batch when it was timed there, else on the probe)
 * into *best_ms (nullable).  The runs write the jobs' outputs (the probe
 * the first source's rows).  The workspace must hold
 * chert_trace_autotune_workspace_bytes (which also covers the full batch
 * under any candidate).  Synchronous. */
size_t chert_trace_autotune_workspace_bytes(const chert_trace_job *jobs, int32_t n_jobs,
                                            const chert_trace_opts *o);
int chert_trace_autotune(const chert_trace_job *jobs, int32_t n_jobs,
                         chert_trace_opts *o, void *workspace_dev,
                         size_t workspace_bytes, void *stream, double *best_ms);

/* The whole of a chert_trace_batch call as one replayable HIP graph:
 * create plans the batch, uploads its tables into workspace_dev
 * (synchronously on `stream`, which must not be NULL) and captures every
 * kernel -- edge weights, field initialisation, the traveltime phase,
 * the tight-edge masks and the tree phase (predecessors and t*) -- from
 * stream capture of `stream`.  The
 * phases are either the persistent launches (CHERT_LAUNCH_PERSISTENT) or,
 * with CHERT_LAUNCH_PER_ROUND and a round budget max_rounds > 0, exactly
 * max_rounds per-round launches each (rounds after convergence find no
 * active tile and leave at once; a budget too short makes finish return
 * NO_CONVERGENCE -- take it from an eager run's stats with a margin).  The
 * node-frontier launch cannot be captured (INVALID_ARG).  launch enqueues
 * one replay (asynchronous, no host work); finish waits on `stream` and
 * reports that replay's errors and counters like chert_trace_batch; destroy
 * releases the graph.  Outputs, caches and
 * the workspace named at create time must stay allocated while the graph
 * exists; their contents may change between replays (e.g. a rebuilt cache).
 * One replay at a time per workspace. */
typedef struct chert_trace_graph chert_trace_graph;
int chert_trace_graph_create(const chert_trace_job *jobs, int32_t n_jobs,
                             const chert_trace_opts *o, void *workspace_dev,
                             size_t workspace_bytes, void *stream,
                             chert_trace_graph **out);
int chert_trace_graph_launch(chert_trace_graph *g, void *stream);
int chert_trace_graph_finish(chert_trace_graph *g, void *stream,
                             chert_trace_stats *stats_host);
int chert_trace_graph_destroy(chert_trace_graph *g);

/* ------------------------------------------------------------------------
 * The cell network (grid and nodal ray-network section; eqs 23-24, 27-32).
 * The medium is cut into ncx x ncz rectangular cells whose sides hold
 * cell_n intervals of hx (along x) or hz (along z).  The nodes are the
 * points of the NX x NZ lattice (NX = ncx cell_n + 1, NZ = ncz cell_n + 1)
 * that lie on a cell edge (ix % cell_n == 0 or iz % cell_n == 0), indexed
 * ix + NX iz; points inside a cell are not nodes.  Every pair of nodes on the
 * boundary of one cell is joined by the straight segment between them
 * (eq 27); its weight is eqs 28-30 with the classes of its two end nodes:
 * a ray-direction cache is read at the tabulated direction nearest to the
 * segment (the forward star's rule, non-primitive offsets included), a
 * slowness-sampled cache at each end class's closest stored ray direction.
 * Each traveltime field is the network's shortest-path field, relaxed in
 * both directions of each segment (eq 31) cell by cell; with
 * o->bucket_width > 0 the cells are taken in order of their block
 * traveltime (eqs 23-24, 32) within that width (units of the smallest
 * positive segment weight of the field), else every woken cell each round.
 * Predecessors: BFS hop counts over tight segments (tau_i + w_ij == tau_j),
 * pred_j = the tight neighbour with the smallest (hop, node index); t* folds
 * the attenuation weights along the propagation tree.
 * ---------------------------------------------------------------------- */
typedef struct chert_cell_grid {
  int32_t ncx, ncz;   /* cells along x and z (>= 1)                       */
  int32_t cell_n;     /* intervals per cell side, 1..16 (4 cell_n <= 64)  */
  int32_t reserved;   /* 0                                               */
  double hx, hz;      /* lattice spacing along x and z [m]               */
  const int32_t *class_id_dev; /* [NZ][NX] class of every lattice point
                         (read at nodes only; required)                   */
} chert_cell_grid;

/* Workspace of chert_trace_cells (0 on invalid arguments). */
size_t chert_trace_cells_workspace_bytes(const chert_cache_desc *d, int64_t n_classes,
                                         const chert_cell_grid *g, int32_t n_src,
                                         const chert_trace_opts *o);

/* Trace n_src sources (lattice indices of nodes) of one mode on the cell
 * network of g with a 2D class cache (ray-direction or slowness-sampled,
 * any subset holding every segment bin).  Outputs are device arrays
 * [n_src][NX NZ] under the same output-mask rules as chert_trace_field;
 * lattice points inside cells get +inf (tau, t*) and -1 (pred).  Options
 * read: outputs, max_rounds, bucket_width, stats_host (rounds[0] =
 * traveltime rounds, rounds[1] = BFS levels of the deepest tree, tile_visits[0] = cell
 * visits, edge_relaxations[0] = pair relaxations, levels_sum[0] = passes
 * over the pairs of the visited cells), abort_flag_host; the tile fields and
 * launch are ignored.  INVALID_ARG on a source inside a cell, a class id out
 * of range (checked on the device before any output is written) or a
 * workspace that is too small or not 256-byte aligned.  Synchronous with
 * respect to `stream` (the host checks the rounds); NO_CONVERGENCE when the
 * round cap is reached. */
int chert_trace_cells(const chert_cache_desc *d, const void *cache_dev, int64_t n_classes,
                      const chert_cell_grid *g, int32_t mode, const int64_t *src_nodes_host,
                      int32_t n_src, const chert_trace_opts *o, double *tau_r_dev,
                      double *tau_i_dev, double *tstar_dev, int32_t *pred_p_dev,
                      int32_t *pred_a_dev, void *workspace_dev, size_t workspace_bytes,
                      void *stream);

/* MSPM baseline (Algorithm 1; Table A-1) on the same cell network, with no
 * cache: each round's visited cells regenerate their local tables, i.e.
 * every corner of every visited cell is solved afresh (theta_R sweep of
 * n_sweep samples, then one root search per canonical segment direction:
 * the exact direction of the segment's offset or its reverse, whichever has
 * angle in [0, pi)) with the corner's class and the chosen kernel (MEV or
 * OEV).  A node between two corners of its edge takes V and A reconstructed
 * linearly from those corners at its fraction t of the edge,
 * x = x1 + t (x2 - x1) (the paper leaves the rule open); weights then follow
 * eqs 28-30.  classes_dev: [n_classes] device classes; the class map of g
 * indexes them.  Outputs, options and errors as chert_trace_cells; the
 * predecessors, t* and the ordering scale read a per-class table solved
 * once per call with the same kernel code (the same values).  stats_host
 * also gets edge_relaxations[1] = corner solves of the rounds. */
size_t chert_trace_mspm_workspace_bytes(int64_t n_classes, const chert_cell_grid *g,
                                        int32_t n_src, const chert_trace_opts *o);
int chert_trace_mspm(const chert_class *classes_dev, int64_t n_classes,
                     const chert_cell_grid *g, int32_t mode, int32_t kernel, int32_t n_sweep,
                     const int64_t *src_nodes_host, int32_t n_src, const chert_trace_opts *o,
                     double *tau_r_dev, double *tau_i_dev, double *tstar_dev,
                     int32_t *pred_p_dev, int32_t *pred_a_dev, void *workspace_dev,
                     size_t workspace_bytes, void *stream);

/* ------------------------------------------------------------------------
 * The block network: the cell network in 3D (the discretisation section
 * names cells in 2D and blocks in 3D; eqs 27-31 with the 3D cache of
 * eq 35).  The medium is cut into ncx x ncy x ncz boxes whose edges hold
 * block_n intervals of hx, hy or hz.  The nodes are the points of the
 * NX x NY x NZ lattice (N? = nc? block_n + 1) that lie on a block face (any
 * coordinate a multiple of block_n), indexed ix + NX (iy + NY iz); every
 * pair of face points of one block is joined by the straight segment
 * between them, whose weight is eqs 28-30 with the classes of its two end
 * nodes, both read at the cache's Fibonacci direction closest to the
 * segment (largest dot product with its unit vector, the lowest index among
 * equals: the 3D forward star's rule).  Traveltimes, predecessors and t*
 * follow the same rules as chert_trace_cells.
 * ---------------------------------------------------------------------- */
typedef struct chert_block_grid {
  int32_t ncx, ncy, ncz; /* blocks along x, y and z (>= 1)                 */
  int32_t block_n;       /* intervals per block edge, 1..3 (at most 56
                            face nodes per block, one lane each)           */
  double hx, hy, hz;     /* lattice spacing along x, y and z [m]           */
  const int32_t *class_id_dev; /* [NZ][NY][NX] class of every lattice
                            point (read at nodes only; required)            */
} chert_block_grid;

/* Workspace of chert_trace_blocks (0 on invalid arguments). */
size_t chert_trace_blocks_workspace_bytes(const chert_cache_desc *d, int64_t n_classes,
                                          const chert_block_grid *g, int32_t n_src,
                                          const chert_trace_opts *o);

/* Trace n_src sources (lattice indices of nodes) of one mode on the block
 * network of g with a 3D class cache (d->dim == 3, n_dirs Fibonacci
 * directions).  Outputs are device arrays [n_src][NX NY NZ]; lattice points
 * inside blocks get +inf (tau, t*) and -1 (pred).  Options, statistics
 * (cell visits count block visits) and errors as chert_trace_cells;
 * INVALID_ARG on a 2D cache or a source inside a block.  Synchronous with
 * respect to `stream`. */
int chert_trace_blocks(const chert_cache_desc *d, const void *cache_dev, int64_t n_classes,
                       const chert_block_grid *g, int32_t mode, const int64_t *src_nodes_host,
                       int32_t n_src, const chert_trace_opts *o, double *tau_r_dev,
                       double *tau_i_dev, double *tstar_dev, int32_t *pred_p_dev,
                       int32_t *pred_a_dev, void *workspace_dev, size_t workspace_bytes,
                       void *stream);

/* Raypath (eqs 25, 33-34): follow pred from rcv back to src and write the
 * node sequence src ... rcv into path_out.  Host, synchronous.
 * *path_len receives the length (also on CAPACITY, so the caller can retry).
 * UNREACHABLE if a node on the way has pred -1; CYCLE if the chain is longer
 * than n_nodes; INVALID_ARG on out-of-range indices. */
int chert_extract_raypath(const int32_t *pred_host, int64_t n_nodes,
                          int64_t src, int64_t rcv, int64_t *path_out,
                          int64_t capacity, int64_t *path_len);

/* Forward-star offsets, lengths and bins as used by chert_trace_field
 * (host, synchronous).  Returns the number of offsets, or -1 on bad args;
 * arrays may be NULL to count only. */
int chert_star_2d(int32_t radius, double hx, double hz, int32_t n_dirs,
                  int32_t *ox, int32_t *oz, double *len, int32_t *bin);

/* The 3D star of a grid (see chert_grid) with the bins of an n_dirs
 * Fibonacci cache (host, synchronous; returns the count or -1). */
int chert_star_3d(int32_t radius, double hx, double hy, double hz, int32_t n_dirs,
                  int32_t *ox, int32_t *oy, int32_t *oz, double *len, int32_t *bin);

/* ------------------------------------------------------------------------
 * Learned surrogate of the cache solve (an addition to the paper's method,
 * which finds coarse property classes too crude for structurally complex
 * media and per-node caches too costly to solve; see its application to a
 * Marmousi-type model and its conclusions).  An MLP maps
 *   inputs  (16): a11/a33 - 1, a13/a33, a44/a33, a66/a33, 1/q11, 1/q13,
 *                 1/q33, 1/q44, 1/q66 (0 when elastic), mode one-hot (3),
 *                 cos psi, sin psi, cos 2 psi, sin 2 psi, psi = target ray
 *                 angle in the symmetry-axis frame (eq 36);
 *   outputs (4):  theta_R - psi (wrapped to (-pi, pi]), theta_I,
 *                 log(V / sqrt(a33)), A sqrt(a33)   (eqs 9-11)
 * through three tanh layers of 128 (linear output), standardised inputs and
 * outputs.  Products run on BF16 operands with FP32 accumulation; master
 * weights and Adam moments are FP32.  Parameter order (FP32): W1[16][128],
 * b1[128], W2[128][128], b2, W3[128][128], b3, W4[128][4], b4[4]; a layer
 * maps x -> x W + b.
 *
 * The surrogate lives in one caller-allocated device blob of total_bytes
 * (256-byte aligned).  Layout (byte offsets from chert_surrogate_layout_of):
 *   [0, 256)        header: uint32 magic 'CHSG' (0x47534843), version 1,
 *                   n_in, n_hidden, n_out, n_params, int32 last Adam step
 *   norm_offset     float in_mean[16], in_inv_std[16], out_mean[4],
 *                   out_std[4]
 *   params_offset   float params[n_params] (master weights)
 *   adam_m_offset   float m[n_params];  adam_v_offset float v[n_params]
 *   then BF16 operand copies of the weights (internal).
 * Training data comes from solved caches (chert_surrogate_dataset); the
 * cache builder then uses the surrogate as the starting point of its
 * Newton polish (chert_build_cache_surrogate).
 * ------------------------------------------------------------------------ */
typedef struct chert_surrogate_layout {
  size_t total_bytes;
  size_t norm_offset;
  size_t params_offset;
  size_t adam_m_offset;
  size_t adam_v_offset;
  int32_t n_params; /* 35716 */
  int32_t n_in;     /* 16 */
  int32_t n_hidden; /* 128 */
  int32_t n_out;    /* 4 */
} chert_surrogate_layout;

int chert_surrogate_layout_of(chert_surrogate_layout *out);

/* Initialise a blob: master weights from params_dev (device, n_params
 * floats, e.g. a seeded random draw), zero Adam moments, identity
 * standardisation.  Asynchronous on `stream`. */
int chert_surrogate_init(void *blob_dev, const float *params_dev, void *stream);

/* Training samples of every (mode in d->mode_mask ascending, class, column)
 * entry of a cache built with desc d, in that order (column fastest):
 * x_dev [n][16] inputs, y_dev [n][4] targets, ok_dev [n] 1 where the entry's
 * status is CHERT_ST_OK (others hold NaN or are unusable).  n = modes *
 * n_classes * columns. */
int chert_surrogate_dataset(const chert_cache_desc *d, const void *cache_dev,
                            const chert_class *classes_dev, int64_t n_classes,
                            float *x_dev, float *y_dev, int32_t *ok_dev,
                            void *stream);

/* Set the blob's standardisation to the mean and standard deviation
 * (population; 1 where zero) of every input and target column over the n
 * samples with ok_dev != 0. */
int chert_surrogate_fit_norm(void *blob_dev, const float *x_dev,
                             const float *y_dev, const int32_t *ok_dev,
                             int64_t n, void *stream);

/* Gradient of the mean squared error of the standardised outputs over the
 * batch idx_dev[0..batch) (indices into x_dev / y_dev):
 *   loss = sum over samples and outputs of (out - y_std)^2 / (4 batch).
 * grad_dev: n_params floats (parameter order above); loss_dev: one float,
 * nullable.  The sum over samples is taken per 32-sample tile and then over
 * tiles in order, so the result does not depend on scheduling. */
size_t chert_surrogate_grad_workspace_bytes(int32_t batch);
int chert_surrogate_grad(const void *blob_dev, const float *x_dev,
                         const float *y_dev, const int32_t *idx_dev,
                         int32_t batch, float *grad_dev, float *loss_dev,
                         void *workspace_dev, size_t workspace_bytes,
                         void *stream);

/* One Adam step (Kingma and Ba 2015; beta1 0.9, beta2 0.999, eps 1e-8,
 * bias-corrected, step counted from 1) on the master weights with gradient
 * grad_dev; refreshes the BF16 copies. */
int chert_surrogate_adam(void *blob_dev, const float *grad_dev, int32_t step,
                         float lr, void *stream);

/* Outputs (de-standardised, [n][4]) for inputs x_dev [n][16]. */
int chert_surrogate_infer(const void *blob_dev, const float *x_dev, int64_t n,
                          float *y_dev, void *stream);

/* Counters of a surrogate-started build (device int64[10]):
 * [0] (mode, class) jobs, [1] jobs sent to the full plain solver,
 * [2] directions, [3] of them near a fold of the ray-angle map (solved by
 * the windowed plain search), [4] Newton not converged, [5] slope of the
 * ray-angle map too small, [6] theta_I not the root nearest 0, [7] residual
 * or entry rejected, [8] sweep samples evaluated by windowed searches,
 * [9] jobs whose windowed search failed its guard, needed more than 512
 * sweep samples or found no room for its brackets (those jobs are redone by
 * the plain path). */
enum { CHERT_WARM_NSTATS = 10 };

/* Scratch needed by chert_build_cache_surrogate. */
size_t chert_build_cache_surrogate_workspace_bytes(const chert_cache_desc *d,
                                                   int64_t n_classes);

/* Build the same cache as chert_build_cache, starting every direction's
 * root search from the surrogate instead of a theta_R sweep:
 *   1. the MLP predicts (theta_R, theta_I) for every solved direction;
 *   2. an FP64 Newton iteration on (homogeneity residual, ray-direction
 *      miss) (eq 9, eq 26's target direction) polishes it;
 *   3. the root is accepted only if it is the one the plain search selects:
 *      the elastic ray-angle map of the class has no fold (triplication)
 *      within 2 degrees of the direction, the map's slope at the root is
 *      at least 0.05, theta_I is the root of the residual nearest 0, and
 *      the residual is at most resid_tol (0 = 1e-11);
 *   4. directions near a fold are solved by the plain sweep-and-bracket
 *      search restricted to the sweep samples whose theta_R the elastic map
 *      sends within 2 degrees of the target (the rest of the sweep cannot
 *      bracket it while the viscoelastic map stays within that margin of
 *      the elastic one, which is checked on every evaluated sample);
 *   5. every (mode, class) job with any other rejected direction, or a
 *      failed check in 4, is solved again by the full plain path, so each
 *      entry equals the plain solver's to the Newton tolerance.
 * stats_dev: nullable device int64[CHERT_WARM_NSTATS], overwritten.
 * UNSUPPORTED above 512 stored directions (n_dirs or n_subset) in 2D.
 * 3D caches (dim 3): every (mode, class, Fibonacci direction) is polished
 * on its own from its prediction under the checks of step 3 (the fold test
 * against the elastic map of its class); a direction near a fold or failing
 * a check is solved by the plain sweep-and-bracket search from its (mode,
 * class) sweep table, so again each entry equals the plain solver's.  The
 * counters then hold [0] (mode, class) jobs, [1] directions sent to the
 * plain search, [2]..[7] as in 2D; [8], [9] stay 0. */
int chert_build_cache_surrogate(const chert_cache_desc *d,
                                const chert_class *classes_dev,
                                int64_t n_classes, const void *blob_dev,
                                double resid_tol, void *cache_dev,
                                int64_t *stats_dev, void *workspace_dev,
                                size_t workspace_bytes, void *stream);

/* Measurement support.  While enabled, every kernel launch the library
 * makes (or, if `only` is non-NULL, every launch of the kernel of that name)
 * is bracketed by HIP events on its stream; chert_prof_read() synchronises
 * those events and returns per-kernel launch counts and summed durations.
 * Enabling clears the totals.  Host, not thread-safe. */
typedef struct chert_prof_entry {
  char name[40];
  int64_t launches;
  double total_ms;
} chert_prof_entry;
int chert_prof_enable(int32_t on, const char *only);
int chert_prof_read(chert_prof_entry *out, int32_t capacity, int32_t *n_out);

const char *chert_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* CHERT_H */
