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
 *   flags    0 (reserved)
 *   x        world-sheet vertex (x, y, z, t) of this point on slice `step`
 *   x_prev   the same point on slice step-1
 *   r, r_prev reserved (right neighbour's vertices for bounded regions), zero here
 * Positions are unwrapped along each point's own trajectory in the periodic box. */
typedef struct semipar_point_rec {
  int64_t id, next_id, prev_id;
  int32_t step, flags;
  double x[4], x_prev[4], r[4], r_prev[4];
} semipar_point_rec;

/* One intercommutation (exchange of partners), 56 bytes.
 *   step    lattice step n whose band (slice n to n+1) held the crossing
 *   kind    0 = intercommutation
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
 *                 these sizes. */
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
  int32_t screen_split;   /* threads sharing the 14 cell lookups of one element in the
                             screen: 1, 2, 7 or 14 (0 = 7). Performance only */
} semipar_evolve_params;

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
} semipar_evolve_stats;

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
 * points still active (ACTIVE, when max_steps ended the call) go to out[0].
 * Two-call pattern: with out[f] == NULL the counts are returned in n[f]. cap[f] is
 * the capacity of out[f] in records; a short buffer gives SEMIPAR_E_ARG. mem says
 * whether the out pointers are host or device memory. Records are in slot order. */
int region_emit_final_surfaces(semipar_region* r, semipar_point_rec* out[4],
                               const int64_t cap[4], int64_t n[4], int32_t mem);

/* Copy the event log (all intercommutations since init) into host memory, sorted by
 * (step, t_star, id_a, id_b). buf == NULL returns the count in *n only; otherwise at
 * most cap events are written and *n is the number written. */
int region_events(const semipar_region* r, semipar_event* buf, int64_t cap, int64_t* n);

/* Release all device and host memory of the region. NULL is accepted. */
void region_destroy(semipar_region* r);

/* Static description of an error code. */
const char* semipar_strerror(int code);

/* Text of the last failed HIP call of this thread ("" if none): which call, where,
 * and the HIP error string. For diagnostics after SEMIPAR_E_HIP. */
const char* semipar_last_error(void);

/* Library build string (compiler, target). */
const char* semipar_version(void);

#ifdef __cplusplus
}
#endif
#endif /* SEMIPAR_H */
