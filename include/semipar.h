/*
 * semipar.h -- C ABI of libsemipar, an MI355X (gfx950) evolver for one globally
 * hyperbolic spacetime region of a cosmic-string network.
 *
 * Paper: J. J. Blanco-Pillado, K. D. Olum, B. Shlaer, "A new parallel simulation
 * technique" (arXiv:1011.4046).
 *
 *  - Section "Introduction": the spacetime 4-volume is cut into regions that take in
 *    information only through initial surfaces and pass it on only through final
 *    surfaces, so each region is a task that can run alone given its predecessors'
 *    output.
 *  - Section "Geometry", subsection "Initial conditions": a region with no
 *    predecessors generates initial conditions inside itself, evolves them and writes
 *    out its four final surfaces.
 *  - Subsection "Boundary conditions": one surface file per (region, final surface).
 *  - Section "Semi-parallel cosmic string simulation": the region's work is to build
 *    all world-sheet diamonds (flat space, or first-order expansion per diamond in a
 *    flat Robertson-Walker universe in comoving coordinates and conformal time), look
 *    for intersections between different pieces of string and exchange partners.
 *    A region whose initial surfaces hold no string is only noted, never simulated.
 *  - Section "Conclusion": a failed region is simply run again from its initial
 *    surfaces.
 *
 * All calls return 0 on success or a negative SEMIPAR_E_* code; no exception or
 * C++ type crosses the boundary. Every GPU buffer the library needs is allocated by
 * the library (hipMalloc) and freed by region_destroy. Caller buffers are never
 * retained after a call returns.
 */
#ifndef SEMIPAR_H
#define SEMIPAR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- error codes ---------------------------------------------------------------- */
#define SEMIPAR_OK 0
#define SEMIPAR_E_ARG (-1)      /* bad argument (NULL pointer, negative size, bad enum) */
#define SEMIPAR_E_SURFACE (-2)  /* inconsistent surface: duplicate id, dangling link in a
                                   whole-volume region, broken next/prev pairing, or
                                   records on different lattice slices */
#define SEMIPAR_E_OOM (-3)      /* device or host allocation failed */
#define SEMIPAR_E_HIP (-4)      /* a HIP runtime call failed */
#define SEMIPAR_E_OVERFLOW (-5) /* a per-step buffer could not grow further (beyond 2^29
                                   entries); the region is then unusable: destroy it and
                                   re-run from the initial surfaces */
#define SEMIPAR_E_STATE (-6)    /* call out of order (e.g. evolve after an overflow) */

/* ---- enums --------------------------------------------------------------------- */
enum { SEMIPAR_FLAT = 0, SEMIPAR_MATTER = 1, SEMIPAR_RADIATION = 2 };
enum { SEMIPAR_MEM_HOST = 0, SEMIPAR_MEM_DEVICE = 1 };
enum { SEMIPAR_SCREEN_F64 = 0, SEMIPAR_SCREEN_F32 = 1 };

/* ---- data records ---------------------------------------------------------------- */

/* One string point on a surface (160 bytes, little-endian, no padding).
 *   id       stable point id (never changes, never reused)
 *   next_id  id of the right neighbour along the string, -1 when absent
 *   prev_id  id of the left neighbour, -1 when absent
 *   step     lattice slice index of x; x_prev is slice step-1
 *   flags    SEMIPAR_FLAG_* bits below. Input records: 0. Output records: FROZEN (with
 *            the exit face in bits 8..15), HAS_R, ACTIVE or REMOVED
 *   x        world-sheet vertex (x, y, z, t) of this point on slice `step`
 *   x_prev   the same point on slice step-1
 *   r, r_prev output records with HAS_R: the right neighbour's vertices on slices step
 *            and step-1 (the other inputs of this point's next diamond); else zero.
 *            Ignored on input
 * Positions are unwrapped along each point's own trajectory in the periodic box. */
typedef struct semipar_point_rec {
  int64_t id, next_id, prev_id;
  int32_t step, flags;
  double x[4], x_prev[4], r[4], r_prev[4];
} semipar_point_rec;

/* One logged crossing, 56 bytes.
 *   step    lattice step n whose band (slice n to n+1) held the crossing
 *   kind    0 = intercommutation (exchange of partners); 1 = the strings passed through
 *           each other (intercommutation probability p < 1: the crossing's draw was
 *           >= p, see semipar_evolve_params.p)
 *   id_a < id_b  ids of the two points whose elements (strip to the right neighbour)
 *           crossed; after the event next(a) and next(b) are exchanged
 *   t_star, x_star  meeting point, in the periodic image of element a */
typedef struct semipar_event {
  int32_t step, kind;
  int64_t id_a, id_b;
  double t_star, x_star[3];
} semipar_event;

/* A surface handed to region_init_from_surfaces. `recs` points to n records in host
 * memory (mem = SEMIPAR_MEM_HOST) or device memory (mem = SEMIPAR_MEM_DEVICE, e.g. a
 * torch tensor's data pointer). face: 0..3 for a predecessor face, -1 for generated
 * initial conditions. The library copies the records during the call. */
typedef struct semipar_surface {
  const semipar_point_rec* recs;
  int64_t n;
  int32_t face;
  int32_t mem;
} semipar_surface;

/* Record flags (field `flags` of semipar_point_rec). */
#define SEMIPAR_FLAG_HAS_R 1  /* r, r_prev hold the right neighbour's vertices on slices
                                 step and step-1 (captured when the point stopped) */
#define SEMIPAR_FLAG_FROZEN 2 /* the point stopped in this region; bits 8..15 hold
                                 face + 1 (0: no owning face, e.g. a cut string end) */
#define SEMIPAR_FLAG_ACTIVE 4 /* the point was still advancing when evolution stopped */
#define SEMIPAR_FLAG_REMOVED 8 /* the point belongs to a loop that was recorded and
                                  removed (semipar_evolve_params.loop_every); x, x_prev
                                  are its vertices at the removal step */

/* Region description.
 *   cosmology  SEMIPAR_FLAT, SEMIPAR_MATTER (a ∝ eta^2, H = 2/eta) or
 *              SEMIPAR_RADIATION (a ∝ eta, H = 1/eta); conformal time eta = t
 *   box        side L of the periodic cube (> 0)
 *   capacity   maximum number of points (0 = number of input records)
 *   bounded    0: the whole periodic volume, every point advances every step.
 *              1: one 4-cube of the spacetime tiling (Section "Geometry"): generators
 *              g/2 (1,1,1,1), g/2 (1,-1,-1,1), g/2 (-1,1,-1,1), g/2 (-1,-1,1,1) in
 *              (x, y, z, tau), tau = sqrt(3) t; generator coordinates
 *              c = H^T (P - origin) / (2 g); the region is floor(c) == idx. Point k
 *              advances at step n only while the earliest point of its next diamond,
 *              X[n-1][next k], lies in the region and its neighbours' inputs exist;
 *              otherwise it stops and is emitted on the face its diamond leaves by.
 *              Links may dangle (next_id/prev_id = -1).
 *   idx, origin, inv2g  region index, lattice origin (x, y, z, tau) and 1/(2 g)
 *   n_sub, sub  a batch: with bounded = 1 and n_sub > 0, surface i of the init call
 *              holds the points of sub-region i, whose geometry is sub[i]. The
 *              sub-regions evolve together, step for step, in one set of launches; they
 *              must not overlap in space (they never interact) and their point ids
 *              must be distinct. Results equal those of separate runs.
 *   stream     hipStream_t to run on. NULL: the library creates its own blocking
 *              stream of default priority (ordered against the null stream), since
 *              the null stream cannot be captured into a graph. All work of the
 *              region is ordered on this stream. */
/* Geometry of one 4-cube region: index, lattice origin (x, y, z, tau), 1/(2 g). */
typedef struct semipar_region_geom {
  int32_t idx[4];
  double origin[4];
  double inv2g;
} semipar_region_geom;

typedef struct semipar_region_desc {
  int32_t cosmology;
  int32_t bounded;
  double box;
  int64_t capacity;
  void* stream;
  int32_t idx[4];
  double origin[4];
  double inv2g;
  int32_t n_sub;                   /* > 0: a batch of n_sub independent bounded regions */
  int32_t reserved;
  const semipar_region_geom* sub;  /* n_sub geometries (host memory, copied) */
} semipar_region_desc;

/* Evolution parameters.
 *   max_steps     lattice steps to take at most in this call (>= 0)
 *   t_end         stop before a step when the smallest t on the current slice is
 *                 >= t_end (use +inf for a step count only)
 *   screen        SEMIPAR_SCREEN_F64 or SEMIPAR_SCREEN_F32: precision of the
 *                 bounding-box screen; every candidate is confirmed in FP64 and the
 *                 event list does not depend on this choice
 *   intercommute  1: search crossings and exchange partners each step; 0: evolution only
 *   cell_size     spatial hash cell (0 = automatic). Any value is correct: elements
 *                 larger than a cell are tested against all others
 *   steps_per_sync  steps issued between host checks of the stop rule (0 = 32)
 *   use_graph     1: issue each block of steps as one captured hipGraph
 *   cand_per_point, events_per_point  per-step buffer sizes as multiples of the point
 *                 count (+64); 0 = defaults 4*n + 65536 and n/2 + 65536. A step that
 *                 overflows either buffer is not taken: the buffer is doubled and the
 *                 step is taken again from the same state, so results never depend on
 *                 these sizes.
 *   loop_every    loop record and removal (Section "Semi-parallel cosmic string
 *                 simulation": loops that cannot intersect again are logged and taken
 *                 out of the simulation). 0: off. P > 0: before every step n with
 *                 n - n0 a positive multiple of P (n0 the slice of the initial
 *                 surfaces), every closed chain of still-advancing points is tested;
 *                 a chain of L points is recorded (semipar_loop) and its points stop
 *                 (flag REMOVED, no owning face) when no logged event (either kind)
 *                 touched any of its elements in steps n - L .. n - 1 (one period of a flat-space
 *                 loop of L points) and every point lies within a quarter of the box,
 *                 per axis, of the chain's lowest slot (a string winding the box never
 *                 does). Events are tracked from init, whatever this field was in
 *                 earlier calls. */
typedef struct semipar_evolve_params {
  int64_t max_steps;
  double t_end;
  int32_t screen;
  int32_t intercommute;
  double cell_size;
  int32_t steps_per_sync;
  int32_t use_graph;
  double cand_per_point;
  double events_per_point;
  int32_t timed_kernel;   /* -1: none; else one of SEMIPAR_K_*: HIP events are recorded
                             around every launch of that kernel and the summed device
                             time is returned in the stats (measurement only; a timed
                             call issues its steps without graphs) */
  int32_t screen_split;   /* screen variant: 1 or 5 threads share the 5 neighbour-
                             pencil lookups of one element; 2: the bucket sort writes
                             each element's 5 pencil ranges next to its sorted entry and
                             the screen reads them (64 more bytes per element each way,
                             two dependent loads fewer). Any other value = 5.
                             Performance only */
  int32_t loop_every;     /* loop record and removal period P in steps (0: off) */
  int32_t persistent;     /* 1: a batch (n_sub > 0) whose sub-regions all hold at most
                             SEMIPAR_PERSISTENT_MAX points, evolved to its regions' own
                             stop (t_end = +inf, loop_every = 0, intercommute = 1, no
                             timed kernel), runs in one launch of persistent workgroups:
                             each takes the next sub-region from a device counter and
                             evolves it through all its steps, testing every pair of its
                             elements with the exact FP64 box test; results equal the
                             step kernels'. Stats count those exact-box pairs as
                             candidates. A step with more crossings than a workgroup
                             holds gives SEMIPAR_E_OVERFLOW (the region is then unusable:
                             run it again from its surfaces with persistent = 0).
                             0 or another batch: the step kernels */
  double p;               /* intercommutation probability in (0, 1]; 0 means 1 (Section
                             "Semi-parallel cosmic string simulation": crossing strings
                             exchange partners with probability p, 1 for field-theory
                             strings, down to 1e-3 for superstrings). Each confirmed
                             crossing (id_a < id_b) of step n draws u = (w >> 11) 2^-53,
                             w the first word of Philox4x64-10 (Salmon et al., SC 2011)
                             under key (seed, 0) of counter (id_a, id_b, n, 0); u >= p:
                             the strings pass through (logged with kind 1, neither element
                             claimed), else the crossing enters the greedy matching.
                             Results depend on (p, seed) only, never on batching or launch
                             order. Outside [0, 1] or NaN: SEMIPAR_E_ARG */
  uint64_t seed;          /* key of the crossings' draws (used when p < 1) */
  double cell_factor;     /* edge of the next step's cells in units of this step's
                             largest element extent (cell_size = 0 only); 0: the default,
                             1.15. Any value in [1, 4] gives the same events; smaller
                             cells hold fewer entries, and elements that outgrow the
                             previous step's largest are screened apart (each walks the
                             cells its box reaches). Else SEMIPAR_E_ARG. Performance
                             only */
} semipar_evolve_params;

/* most points of a sub-region evolved by persistent workgroups, and most crossings of
 * one of its steps that a workgroup holds */
#define SEMIPAR_PERSISTENT_MAX 512
#define SEMIPAR_PERSISTENT_EVENTS 160

/* kernels that can be timed through semipar_evolve_params.timed_kernel */
enum {
  SEMIPAR_K_EVOLVE = 0,  /* diamond tops + element box + hash count */
  SEMIPAR_K_SCAN = 1,    /* bucket scan (tiles and totals) */
  SEMIPAR_K_SCATTER = 2, /* bucket lists */
  SEMIPAR_K_SCREEN = 3,  /* bounding-box screen */
  SEMIPAR_K_CONFIRM = 4, /* FP64 triangle-pair confirmation */
  SEMIPAR_K_RESOLVE = 5  /* matching, partner exchange, log */
};

/* Statistics of one region_evolve call (counts over that call). */
typedef struct semipar_evolve_stats {
  int64_t steps;          /* lattice steps taken */
  int64_t point_steps;    /* diamond tops computed (one per active point per step) */
  int64_t candidates;     /* pairs passing the bounding-box screen */
  int64_t confirmed;      /* pairs whose FP64 triangle test found a crossing */
  int64_t accepted;       /* intercommutations applied and logged */
  int64_t large_elements; /* element-steps handled outside the spatial hash */
  int32_t final_step;     /* slice index of the current slice after the call */
  int32_t done;           /* 1 when the stop rule (t_end or max_steps) ended the call */
  double elapsed_ms;      /* device time of the call's step loop (HIP events) */
  double timed_kernel_ms; /* summed device time of the timed kernel (HIP events) */
  int64_t timed_kernel_launches; /* launches of the timed kernel that did work */
  int64_t loops;          /* loops recorded and removed */
  int64_t loop_points;    /* points they held */
  int64_t resolve_rounds; /* rounds of the event matching (iterated local minima),
                             summed over the steps taken */
  int64_t passed;         /* crossings that passed through (p < 1), logged with kind 1 */
} semipar_evolve_stats;

/* A loop recorded and removed (48 bytes).
 *   step      slice n at which it was removed (the check before step n)
 *   n_points  its number of points L
 *   rep_id    id of its point in the lowest slot (input record order)
 *   energy    sum over its points k, j = next(k), of |X[n][k] - X[n-1][j]| +
 *             |X[n][j] - X[n-1][j]| (spatial parts, the first to the nearest periodic
 *             image): the string length of its last band, the invariant energy of a
 *             flat-space loop
 *   centre    mean spatial position of its points on slice n, each taken at the
 *             periodic image nearest the lowest slot's point
 * Energy and centre are FP64 sums in an unspecified order (not bitwise
 * reproducible); step, n_points and rep_id are exact. */
typedef struct semipar_loop {
  int32_t step, n_points;
  int64_t rep_id;
  double energy, centre[3];
} semipar_loop;

typedef struct semipar_region semipar_region;

/* Build a region from its initial surfaces (paper: a region is a task given only the
 * initial-surface information of its predecessors).
 *   d, in[0..n_in)  description and surfaces; all records must sit on one slice
 *   out             receives the new region (owned by the caller until
 *                   region_destroy)
 * In a whole-volume region every point must have both neighbours among the records.
 * Errors: SEMIPAR_E_ARG,
 * SEMIPAR_E_SURFACE, SEMIPAR_E_OOM, SEMIPAR_E_HIP; *out is NULL on error. An empty
 * input (n_in = 0 or all n = 0) gives a valid empty region. */
int region_init_from_surfaces(const semipar_region_desc* d, const semipar_surface* in, int n_in,
                              semipar_region** out);

/* Advance the region (paper: construct the diamonds, look for intersections between
 * different pieces of string, reconnect). Each step n: diamond tops X[n+1] of every
 * point from X[n] and X[n-1]; world-sheet elements of the band n..n+1; bounding-box
 * screen through a spatial hash; FP64 triangle-pair confirmation; one event per
 * element in (t*, id_a, id_b) order; partner exchange. Stops after max_steps steps or
 * when the current slice's smallest t reaches t_end. st may be NULL.
 * Errors: SEMIPAR_E_ARG, SEMIPAR_E_OVERFLOW, SEMIPAR_E_HIP, SEMIPAR_E_STATE. */
int region_evolve(semipar_region* r, const semipar_evolve_params* p, semipar_evolve_stats* st);

/* Write the region's output surfaces (paper: pass on what lies on each final
 * surface). A whole-volume region has one output surface, the current slice: every
 * point goes to out[0] (x = current slice, x_prev = previous slice); n[1..3] = 0.
 * A bounded region writes each stopped point to out[f], f its face (flags FROZEN,
 * HAS_R when r holds the right neighbour's inputs); points without an owning face and
 * points still active (ACTIVE, when max_steps ended the call) go to out[0]. Points of
 * a removed loop (flag REMOVED, either kind of region) go to out[0] with their
 * vertices at the removal step.
 * Two-call pattern: with out[f] == NULL the counts are returned in n[f]. cap[f] is
 * the capacity of out[f] in records; a short buffer gives SEMIPAR_E_ARG. mem says
 * whether the out pointers are host or device memory. Records are in slot order. */
int region_emit_final_surfaces(semipar_region* r, semipar_point_rec* out[4],
                               const int64_t cap[4], int64_t n[4], int32_t mem);

/* Copy the loop log (every loop recorded and removed since init) into host memory,
 * sorted by (step, rep_id). buf == NULL returns the count in *n only; otherwise at
 * most cap loops are written and *n is the number written. Errors: SEMIPAR_E_ARG,
 * SEMIPAR_E_HIP. */
int region_loops(const semipar_region* r, semipar_loop* buf, int64_t cap, int64_t* n);

/* Copy the event log (all intercommutations since init) into host memory, sorted by
 * (step, t_star, id_a, id_b). buf == NULL returns the count in *n only; otherwise at
 * most cap events are written and *n is the number written. */
int region_events(const semipar_region* r, semipar_event* buf, int64_t cap, int64_t* n);

/* Diagnostics of the screen (C ABI for tests): the pairs of elements that passed the
 * bounding-box screen in the last step the region took, as (smaller id, larger id) of
 * the two points whose elements they are, sorted, into ids[2 i], ids[2 i + 1]. Both
 * screens report what they passed, so the FP32 screen's pairs of a step can be checked
 * to contain the FP64 screen's. ids == NULL returns the count in *n; otherwise at most
 * cap pairs are written and *n is the number written. A region that has taken no step
 * with intercommutation reports 0. Errors: SEMIPAR_E_ARG, SEMIPAR_E_OOM, SEMIPAR_E_HIP. */
int region_candidates(const semipar_region* r, int64_t* ids, int64_t cap, int64_t* n);

/* Release all device and host memory of the region. NULL is accepted. */
void region_destroy(semipar_region* r);

/* Static description of an error code. */
const char* semipar_strerror(int code);

/* Text of the last failed HIP call of this thread ("" if none): which call, where,
 * and the HIP error string. For diagnostics after SEMIPAR_E_HIP. */
const char* semipar_last_error(void);

/* Library build string (compiler, target). */
const char* semipar_version(void);


/* ---- many regions: the tiling and the scheduler ---------------------------------- */

/* A set of regions to run (paper, Section "Implementation": a manager keeps the
 * regions whose predecessors have all finished and hands them to idle workers).
 *   n_regions  number of regions (>= 0)
 *   cosmology, box  as in semipar_region_desc, shared by all regions
 *   surfaces   n_regions initial surfaces, surfaces[r] the points of region r (n = 0:
 *              an empty region, which is only noted, never launched). Point ids must
 *              be distinct over the whole tiling. Host or device memory per surface.
 *   geoms      n_regions region geometries (host)
 *   n_pred     NULL: the regions are independent. Else, per region, the number of
 *              predecessors that must finish before it may start; succ_off (n_regions
 *              + 1 offsets) and succ list each region's successors. A region becomes
 *              ready when its count reaches zero. BATCHED keeps these counts, the
 *              successor lists and the ring of ready regions on the device; a finished
 *              batch releases its regions' successors at once (a region with no string
 *              is done as soon as it is ready), and ready regions are packed into the
 *              next batches. This orders the work only: a successor's input is its own
 *              surface, not its predecessors' output.
 *   stream     hipStream_t for all work (NULL: each region creates its own stream). */
typedef struct semipar_tiling {
  int32_t n_regions;
  int32_t cosmology;
  double box;
  const semipar_surface* surfaces;
  const semipar_region_geom* geoms;
  const int32_t* n_pred;
  const int32_t* succ_off;
  const int32_t* succ;
  void* stream;
} semipar_tiling;

enum {
  SEMIPAR_PACK_POINTS = 0, /* batches of at most batch_points points */
  SEMIPAR_PACK_WORK = 1    /* batches of equal predicted work (needs cost) */
};

enum {
  SEMIPAR_SCHED_PLAIN = 0,  /* one region at a time, each its own launch sequence */
  SEMIPAR_SCHED_BATCHED = 1 /* ready regions packed into batches (one set of launches
                               per batch over the points of all its regions) */
};

/* Scheduler parameters.
 *   policy        SEMIPAR_SCHED_PLAIN or SEMIPAR_SCHED_BATCHED
 *   batch_points  BATCHED: at most this many points per batch (a larger region gets a
 *                 batch of its own); 0 = all ready regions in one batch
 *   cost          BATCHED: host array of n_regions predicted costs (lattice steps,
 *                 e.g. exp of the cost model's output); the ready regions are ordered
 *                 by decreasing cost and cut into batches in that order. NULL: the
 *                 point-count heuristic (decreasing number of points). Ordering only:
 *                 results never depend on it.
 *   evolve        parameters of every region_evolve call (max_steps, t_end, screen,
 *                 graphs, ...). Each region runs until all its points have stopped
 *                 unless max_steps or t_end ends it first.
 *   out, out_mem  output records (host or device), capacity = total input records;
 *                 region r owns out[out_off[4r] .. out_off[4r+4]) with its face-f
 *                 records at out_off[4r+f] .. out_off[4r+f+1] (same content and order
 *                 as region_emit_final_surfaces of that region run alone). NULL: not
 *                 written.
 *   out_off       host, 4 n_regions + 1 entries, or NULL
 *   events, events_cap, events_off  host event buffer, its capacity and n_regions + 1
 *                 offsets: region r's events (listing order) at events_off[r] ..
 *                 events_off[r+1]. Offsets count every event; entries past events_cap
 *                 are not written (stats.events is the total). NULL: not returned.
 *   lanes         BATCHED: concurrent lanes (see the field)
 *   region_steps, region_point_steps, region_batch, region_ms  optional host arrays
 *                 (n_regions) receiving per-region logs: slices advanced by the
 *                 region's furthest point, its point-steps, the batch that ran it (-1:
 *                 empty) and the device time of that batch's evolve call. These are
 *                 the costs the cost model is trained on. */
typedef struct semipar_sched_params {
  int32_t policy;
  int32_t out_mem;
  int64_t batch_points;
  const float* cost;
  semipar_evolve_params evolve;
  semipar_point_rec* out;
  int64_t* out_off;
  semipar_event* events;
  int64_t events_cap;
  int64_t* events_off;
  int32_t* region_steps;
  int64_t* region_point_steps;
  int32_t* region_batch;
  double* region_ms;
  int32_t lanes;     /* BATCHED: batches evolved concurrently, each lane a host thread
                        with a stream of its own (0 or 1: one lane). Waiting batches go
                        to idle lanes longest predicted first. */
  int32_t pack;      /* BATCHED: SEMIPAR_PACK_POINTS, or SEMIPAR_PACK_WORK: with a cost
                        vector, the ready regions (in decreasing cost order) are cut into
                        B = max(lanes, ceil(points / batch_points)) batches holding about
                        equal shares of the predicted point-steps (points x cost), so that
                        the regions needing the most steps share a smaller batch. Without
                        a cost vector it acts as SEMIPAR_PACK_POINTS. Ordering only. */
  semipar_loop* loops;  /* host loop buffer (evolve.loop_every > 0), capacity loops_cap,
                           and n_regions + 1 offsets loops_off: region r's loops, sorted
                           by (step, rep_id), at loops_off[r] .. loops_off[r+1]. Offsets
                           count every loop; entries past loops_cap are not written
                           (stats.loops is the total). NULL: not returned. */
  int64_t loops_cap;
  int64_t* loops_off;
  double lane_sleep_ms;  /* BATCHED: 0: every lane is held for the whole call. > 0: the
                            paper's variable-size worker pool (Section "Implementation"):
                            a lane with nothing to do sleeps, is woken by new batches, and
                            exits once it has slept this long; */
  double lane_submit_ms; /* when batches have waited this long for lanes, the manager
                            starts lanes again, up to `lanes` (the pool's job submission).
                            Results do not depend on either; stats report the lanes'
                            summed lifetimes (lane_held_ms) */
} semipar_sched_params;

typedef struct semipar_sched_stats {
  int64_t regions;       /* regions finished */
  int64_t empty_regions; /* of which empty (no launch) */
  int64_t batches;       /* launch batches (PLAIN: one per non-empty region) */
  int64_t point_steps;   /* over all regions */
  int64_t steps;         /* lattice steps summed over batches */
  int64_t events;        /* logged crossings over all regions (with p < 1 also those of
                            kind 1, which passed through) */
  double makespan_ms;    /* host wall time of the call, from the first upload to the
                            last result */
  double evolve_ms;      /* summed device time of the evolve calls */
  double timed_kernel_ms;        /* with evolve.timed_kernel set: summed device time of
                                    that kernel over all calls (HIP events) */
  int64_t timed_kernel_launches; /* and the number of its launches that did work */
  int64_t loops;                 /* loops recorded and removed over all regions */
  int64_t passed;                /* crossings that passed through (p < 1) */
  double lane_held_ms;   /* BATCHED: summed lifetimes of the lanes (from start to exit):
                            the paper's "total real time" (Table 1) */
  double lane_busy_ms;   /* summed wall time lanes spent on batches (build, evolve,
                            results): its "total CPU time" */
  int64_t lanes_started; /* lanes started, the first `lanes` included */
} semipar_sched_stats;

/* Run every region of the tiling on this GPU, in dependency order (paper: manager and
 * workers; empty regions only noted). Per region the result is exactly that of
 * region_init_from_surfaces + region_evolve + region_emit_final_surfaces on that
 * region alone. st may be NULL.
 * Errors: SEMIPAR_E_ARG (bad tiling, or predecessor counts that leave regions never
 * ready), SEMIPAR_E_SURFACE, SEMIPAR_E_OOM, SEMIPAR_E_HIP, SEMIPAR_E_OVERFLOW. */
int schedule_regions(const semipar_tiling* t, const semipar_sched_params* p,
                     semipar_sched_stats* st);

/* ---- a tiling run with hand-off between regions ------------------------------------ */

/* A periodic spacetime tiling run region by region, each region taking its input from
 * its predecessors' output (Section "Geometry" and its subsections "Initial conditions"
 * and "Boundary conditions"; Section "Semi-parallel cosmic string simulation": a diamond
 * is built by the region that holds its earliest point, and a region passes on what
 * overlaps its final surfaces; one GPU holds the whole world sheet in its memory, so
 * "passing on" is a region writing vertices that later regions read).
 *   n_regions, geoms  the regions (host). All share origin and inv2g; the box must hold
 *              a whole number of region steps: K = 4 box inv2g a multiple of 4. A
 *              region is named by its layer S = idx0 + idx1 + idx2 + idx3 and its past
 *              vertex p = idx0 (1,1,1) + idx1 (1,-1,-1) + idx2 (-1,1,-1) + idx3 (-1,-1,1)
 *              taken mod K (the names repeat with the box); two regions may not share a
 *              name, and vertices whose region has no entry are outside the run.
 *   n_pred, succ_off, succ  dependency lists as in semipar_tiling (required; each
 *              successor must lie in a later layer). Regions run layer by layer: a
 *              region reads and is told only what earlier layers or it itself built, and
 *              the regions of one layer never exchange anything
 *   ic, n_points, ic_mem  the initial surface of the whole volume (host or device):
 *              records on one slice s0 >= 1 (x on s0, x_prev on s0 - 1), ids distinct,
 *              every next_id and prev_id among the records and paired
 *   hist, hist_slices  device memory for hist_slices x n_points x 4 doubles, the world
 *              sheet: the vertex (x, y, z, t) of the point in record slot q on slice
 *              s0 - 1 + s is at hist[4 (s n_points + q)]. The call fills it with
 *              t = NaN (not built) and the two initial slices; on return it holds every
 *              vertex a region of the tiling built. Too few slices: SEMIPAR_E_OVERFLOW.
 *   stream     hipStream_t for all work (NULL: the library's own) */
typedef struct semipar_handoff {
  int32_t n_regions;
  int32_t cosmology;
  double box;
  const semipar_region_geom* geoms;
  const int32_t* n_pred;
  const int32_t* succ_off;
  const int32_t* succ;
  const semipar_point_rec* ic;
  int64_t n_points;
  int32_t ic_mem;
  int32_t reserved;
  double* hist;
  int64_t hist_slices;
  void* stream;
} semipar_handoff;

/* Run every region of the tiling in dependency order with hand-off. Region R builds
 * every diamond whose bottom lies in R, from inputs that R itself, its predecessors or
 * the initial surface built. Point q's diamonds in R begin when its right neighbour's
 * world line enters R -- the region that builds that entry vertex tells R (a start
 * token) -- and end when that world line leaves R. Crossings between elements of one
 * region are searched, confirmed and logged as in region_evolve, and pass through
 * (kind 1; links never change), so every vertex equals that of one whole-volume run
 * with intercommutation probability 0; crossings between elements of different regions
 * are not searched.
 *   p  used: lanes (0 or 1; more is refused with SEMIPAR_E_ARG), batch_points (at most
 *      this many points per batch; 0: a layer's regions in one batch), cost (ordering
 *      only: longest
 *      predicted first, else most start tokens first), evolve (screen, intercommute,
 *      use_graph, steps_per_sync, screen_split, cell_size, cell_factor, cand_per_point,
 *      events_per_point, seed; max_steps caps the steps of each batch; loop_every must be
 *      0; p is ignored), events / events_cap / events_off, region_steps,
 *      region_point_steps, region_batch, region_ms. out must be NULL (the world sheet is
 *      the output); policy, pack and the lane_* fields are ignored. Results never depend
 *      on batch_points or cost.
 *   st regions, empty_regions, batches, point_steps, steps, events, passed, makespan_ms,
 *      evolve_ms.
 * Errors: SEMIPAR_E_ARG, SEMIPAR_E_SURFACE (initial surface), SEMIPAR_E_OOM,
 * SEMIPAR_E_HIP, SEMIPAR_E_OVERFLOW (hist_slices too few), SEMIPAR_E_STATE (a region
 * received work after it had run, or a diamond lacked an input: the tiling's dependency
 * lists or geometry do not match; semipar_last_error says which). */
int schedule_handoff(const semipar_handoff* h, const semipar_sched_params* p,
                     semipar_sched_stats* st);

/* ---- the learned cost model --------------------------------------------------------- */
#define SEMIPAR_MLP_IN 12
#define SEMIPAR_MLP_HIDDEN 64
#define SEMIPAR_MLP_PARAMS 5057 /* 64*12 + 64 + 64*64 + 64 + 64 + 1 */

/* Cost-model features of each region's initial surface, computed on the GPU
 * (host output, 12 floats per region, zeros for an empty region):
 *   0 log1p(points)   1 log1p(open string pieces: points without a left neighbour)
 *   2 RMS transverse speed of the first diamonds
 *   3..10 occupancy histogram: the region's spatial cube of side 2g (g the generator
 *         scale) around its centre (origin + g/2 times the index summed along the
 *         generators' spatial parts) in 16^3 cells; the fraction of points in cells whose count, relative
 *         to the mean over all cells, has floor(log2) + 4 = b (clamped to 0..7)
 *   11 log1p(mean distance to the right neighbour / region size)
 * Surfaces all in device memory are read in place (only an id table for the right
 * neighbours is built); otherwise the regions are loaded as one batch first. Both give
 * the same features. Errors: SEMIPAR_E_ARG, SEMIPAR_E_SURFACE (a duplicate id),
 * SEMIPAR_E_OOM, SEMIPAR_E_HIP; feat holds no valid features then. */
int semipar_region_features(const semipar_tiling* t, float* feat);

/* The cost model is a 12 -> 64 -> 64 -> 1 perceptron with ReLU, FP32. Parameters
 * (SEMIPAR_MLP_PARAMS floats, row-major): W1[64][12], b1[64], W2[64][64], b2[64],
 * w3[64], b3. Optional normalisation norm[24] (NULL: none): inputs become
 * (x - norm[0..11]) * norm[12..23]. All array arguments below are device pointers
 * unless marked host; x holds n rows of 12 features. The calls synchronise `stream`
 * before returning. Errors: SEMIPAR_E_ARG, SEMIPAR_E_OOM, SEMIPAR_E_HIP. */

/* y[s] = model(x[s]) for s < n. */
int semipar_mlp_forward(const float* params, const float* norm, const float* x, int64_t n,
                        float* y, void* stream);

/* loss = mean over s of (model(x[s]) - target[s])^2 and grad = d loss / d params
 * (loss may be NULL). Summation is in a fixed order (deterministic). */
int semipar_mlp_loss_grad(const float* params, const float* norm, const float* x,
                          const float* target, int64_t n, float* grad, float* loss,
                          void* stream);

/* The same loss and gradient without allocating anything, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc). The per-block partial gradients live in a fixed array of
 * device memory that the library holds on each GPU it runs on until the process ends
 * (about 5 MB). Every call on one GPU uses that same array, so calls that overlap on
 * one GPU (different streams or threads) race and give wrong results: issue them one
 * after another. Results equal semipar_mlp_loss_grad's. n above
 * SEMIPAR_MLP_NOALLOC_MAX gives SEMIPAR_E_ARG (semipar_last_error says why), nothing
 * launched. Errors otherwise as semipar_mlp_loss_grad. */
#define SEMIPAR_MLP_NOALLOC_MAX 8192
int semipar_mlp_loss_grad_noalloc(const float* params, const float* norm, const float* x,
                                  const float* target, int64_t n, float* grad, float* loss,
                                  void* stream);

/* One Adam update (Kingma and Ba) at 1-based step number `step`:
 * m = b1 m + (1-b1) g; v = b2 v + (1-b2) g^2;
 * params -= lr (m / (1 - b1^step)) / (sqrt(v / (1 - b2^step)) + eps). */
int semipar_mlp_adam_step(float* params, float* m, float* v, const float* grad, int64_t step,
                          float lr, float beta1, float beta2, float eps, void* stream);

/* iters full-batch Adam steps (b1 0.9, b2 0.999, eps 1e-8) on the mean squared error,
 * numbered step0 + 1 .. step0 + iters. loss_host (host, iters + 1 floats, or NULL):
 * the loss before each step and, last, at the final parameters. */
int semipar_mlp_train(float* params, float* m, float* v, const float* norm, const float* x,
                      const float* target, int64_t n, int32_t iters, int64_t step0, float lr,
                      float* loss_host, void* stream);

/* Host helper: per-feature mean and inverse standard deviation of n host rows, into
 * norm[24] (host). A feature with standard deviation below 1e-6 gets scale 1. */
int semipar_mlp_norm(const float* x, int64_t n, float* norm);

#ifdef __cplusplus
}
#endif
#endif /* SEMIPAR_H */
